/*
 * adot_oracle.c -- plain, slow CPU FP64 oracle for the A-DOT scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (Carraro, Valiani, Caleffi, "Efficient analytical
 * implementation of the DOT Riemann solver for the de Saint Venant-Exner
 * morphodynamic model"):
 *   - the flux matrix A(W) of the quasi-linear dSVE system   (Sec. 2, Eq. W&A_definition)
 *   - bed-load closures and their derivatives: Grass (Eq. Grass), Grass with a threshold
 *     (Eq. GrassThr), the power law of Sec. 5.1, Meyer-Peter & Mueller (Eqs. MPM, Shields),
 *     Van Rijn (Eqs. vanRijn, u_star)                         (Sec. 2; Sec. 3.3 step 1)
 *   - the Strickler friction slope and its point source       (Sec. 2; Sec. 3, Eq. scheme)
 *   - the closed-form eigenvalues (trigonometric Cardano)     (Sec. 3.3, Eqs. charPol, lambda,
 *                                                              parameters, parameters_bis)
 *   - right / left eigenvectors                               (Sec. 3.3, Eqs. RR, RR-1, circPerm)
 *   - |A| = R |Lambda| R^-1 as an explicit triple product     (Sec. 3.1 Eq. asbA; Sec. 3.3 Eq. ExAbsA)
 *   - the DOT fluctuations by G-point Gauss quadrature along
 *     the segment path                                        (Sec. 3.1, Eqs. path, DOTjump, DOTjumpN)
 *   - the first-order path-conservative cell update, with the friction source as a
 *     point source (S = 0 when no Strickler coefficient is given, as in Sec. 4) (Sec. 3, Eq. scheme)
 *   - the CFL time step  dt = CFL dx / max_i max_m |lambda_m(W_i)|  (reading: the paper names
 *     the CFL condition but does not print the rule)
 *
 * Style: every step is written in the order and notation of the paper, in
 * plain loops, FP64, compiled with -O2 -ffp-contract=off and no fast-math,
 * with glibc acos/cos/sqrt.  Threads only split independent loops (edges,
 * cells, channels); the results are bitwise independent of the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_NONFINITE (-3)
#define OR_E_NONHYPERBOLIC (-4)

#define OR_BC_TRANSMISSIVE 0
#define OR_BC_PERIODIC 1
#define OR_BC_INFLOW_Q 2
#define OR_BC_FIXED_DEPTH 3
#define OR_BC_INFLOW_QH 4
#define OR_BC_DIRICHLET 5

#define OR_LAW_GRASS 0
#define OR_LAW_GRASS_THR 1
#define OR_LAW_POWER 2
#define OR_LAW_MPM 3
#define OR_LAW_VANRIJN 4

/* Tolerance on the arccos argument before it is declared outside [-1, 1]
 * (reading: rounding may push a real-root argument marginally past 1). */
#define OR_ACOS_TOL 1e-12

static const double OR_PI = 3.14159265358979323846264338327950288;

/* Physical parameters of one channel.
 *   law  OR_LAW_*; par[] depends on it:
 *        GRASS      q_s = A_g u^3                               (no par)
 *        GRASS_THR  q_s = A_g (u - u_cr)^3                      par[0] = u_cr
 *        POWER      q_s = A_g u^beta  (A_g is the coefficient)  par[0] = beta
 *        MPM        Meyer-Peter & Mueller                       par[0] = d50, par[1] = S_g
 *        VANRIJN    Van Rijn                                    par[0] = d50, par[1] = S_g,
 *                                                               par[2] = nu, par[3] = theta_cr
 *   ks   Strickler coefficient K_s of the friction slope (0: no friction; MPM and Van Rijn
 *        need it, their Shields stress and shear velocity come from s_f). */
typedef struct {
    double g;  /* gravitational acceleration */
    double xi; /* 1 / (1 - porosity), Sec. 2 */
    double Ag; /* coefficient of the Grass-type laws */
    int law;
    double par[4];
    double ks;
} or_phys;

/* One channel of the scheme. */
typedef struct {
    int64_t n_cells;
    double g, xi, Ag;
    int n_gauss;
    double cfl, dx;
    int bc_left, bc_right;
    double q_in;  /* discharge imposed by an inflow-q boundary */
    double h_out; /* depth imposed by a fixed-depth boundary */
    double h_in;  /* depth imposed with q_in by an inflow-(q, h) boundary */
    double dir_l[4], dir_r[4]; /* Dirichlet ghost (h, q, z at t = 0, dz/dt) of each end */
    int law;
    double par[4];
    double ks;
} or_channel;

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule on [0, 1] (Sec. 3.1, Eq. DOTjumpN: nodes s_k, weights w_Gk).
 * Roots of the Legendre polynomial P_G by Newton's method from the classical
 * initial guesses x ~ cos(pi (i + 3/4) / (G + 1/2)); weights 2 / ((1-x^2) P_G'(x)^2)
 * on [-1, 1]; mapped to [0, 1] by s = (x+1)/2, w = w/2, so the weights sum to 1
 * (the path derivative dPsi/ds = W+ - W- has been taken out of the integral).
 * Nodes are returned in increasing order of s. */
int or_gauss(int G, double *s, double *w)
{
    if (G < 1 || G > 64) return OR_E_ARG;
    for (int i = 0; i < G; ++i) {
        double x = cos(OR_PI * (i + 0.75) / (G + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            /* P_G(x) and P_G'(x) by the three-term recurrence */
            double p0 = 1.0, p1 = x;
            for (int n = 2; n <= G; ++n) {
                double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            /* here p1 = P_G, p0 = P_{G-1} */
            dp = G * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) {
                /* one more evaluation of the derivative at the converged root */
                p0 = 1.0; p1 = x;
                for (int n = 2; n <= G; ++n) {
                    double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
                    p0 = p1;
                    p1 = p2;
                }
                dp = G * (x * p1 - p0) / (x * x - 1.0);
                break;
            }
        }
        double wi = 2.0 / ((1.0 - x * x) * dp * dp);
        /* x runs from near +1 downwards as i grows; store ascending in s */
        s[G - 1 - i] = 0.5 * (x + 1.0);
        w[G - 1 - i] = 0.5 * wi;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Step 1 of the A-DOT procedure (Sec. 3.3): derivatives of the Grass law
 * q_s = A_g (q/h)^3 (Eq. Grass):  dq_s/dh = -3 q_s / h,  dq_s/dq = 3 q_s / q.
 * The q-derivative is evaluated as 3 A_g u^2 / h, equal to 3 q_s / q for q != 0
 * and defined at q = 0 (reading: the printed form is 0/0 there). */
static void grass_derivatives(double h, double q, double Ag, double *dqs_dh, double *dqs_dq)
{
    double u = q / h;
    double qs = Ag * u * u * u;
    *dqs_dh = -3.0 * qs / h;
    *dqs_dq = 3.0 * Ag * u * u / h;
}

static double sign_of(double v) { return (v > 0.0) ? 1.0 : ((v < 0.0) ? -1.0 : 0.0); }

/* A law of the velocity only, q_s = f(u) with u = q/h: by the chain rule
 * dq_s/dq = f'(u) / h and dq_s/dh = -f'(u) u / h. */
static void velocity_law(double h, double q, double dfdu, double *dqs_dh, double *dqs_dq)
{
    double u = q / h;
    *dqs_dq = dfdu / h;
    *dqs_dh = -dfdu * u / h;
}

/* Step 1 for every closure of Sec. 2 (and the power law of Sec. 5.1).
 * Readings: the laws act in the direction of the flow (odd in u or q); Grass with a
 * threshold transports only when |u| > u_cr, q_s = A_g sign(u) (|u| - u_cr)^3; the power
 * law is q_s = A_g sign(u) |u|^beta; in the Shields stress and the shear velocity the
 * friction slope enters through its magnitude s_f = q^2 / (K_s^2 h^(10/3)) (Sec. 2);
 * Van Rijn takes the dimensionless grain size D_* = d50 (g (S_g - 1) / nu^2)^(1/3) and the
 * critical shear velocity from u_*cr^2 = theta_cr g (S_g - 1) d50 (the printed forms are
 * not dimensionless / not the Shields relation). */
static void qs_derivatives(double h, double q, const or_phys *p, double *dqs_dh, double *dqs_dq)
{
    switch (p->law) {
    case OR_LAW_GRASS:
        grass_derivatives(h, q, p->Ag, dqs_dh, dqs_dq);
        return;
    case OR_LAW_GRASS_THR: {
        double u = q / h;
        double ex = fabs(u) - p->par[0];
        double dfdu = (ex > 0.0) ? 3.0 * p->Ag * ex * ex : 0.0;
        velocity_law(h, q, dfdu, dqs_dh, dqs_dq);
        return;
    }
    case OR_LAW_POWER: {
        double u = q / h;
        double beta = p->par[0];
        double dfdu = (u != 0.0) ? p->Ag * beta * pow(fabs(u), beta - 1.0) : 0.0;
        velocity_law(h, q, dfdu, dqs_dh, dqs_dq);
        return;
    }
    case OR_LAW_MPM: {
        /* q_s = Phi(theta) sqrt(g (S_g-1) d50^3), Phi = 8 (theta - 0.047)^(3/2) above 0.047,
         * theta = s_f h / ((S_g - 1) d50)  (Eqs. MPM, Shields) */
        double d50 = p->par[0], Sg = p->par[1];
        double sf = q * q / (p->ks * p->ks * pow(h, 10.0 / 3.0));
        double theta = sf * h / ((Sg - 1.0) * d50);
        if (!(theta > 0.047)) { *dqs_dh = 0.0; *dqs_dq = 0.0; return; }
        double scale = sqrt(p->g * (Sg - 1.0) * d50 * d50 * d50);
        double dqs_dtheta = scale * 12.0 * sqrt(theta - 0.047);   /* d/dtheta of 8 (theta - 0.047)^(3/2) */
        /* theta = q^2 / (K_s^2 (S_g-1) d50 h^(7/3)): dtheta/dq = 2 theta / q, dtheta/dh = -(7/3) theta / h */
        *dqs_dq = dqs_dtheta * 2.0 * theta / fabs(q);
        *dqs_dh = sign_of(q) * dqs_dtheta * (-7.0 / 3.0) * theta / h;
        return;
    }
    case OR_LAW_VANRIJN: {
        /* q_s = 0.053 T^2.1 / D_*^0.3 sqrt(g (S_g-1) d50^3), T = (u_*^2 - u_*cr^2) / u_*cr^2,
         * u_*^2 = g h s_f  (Eqs. vanRijn, u_star) */
        double d50 = p->par[0], Sg = p->par[1], nu = p->par[2], theta_cr = p->par[3];
        double sf = q * q / (p->ks * p->ks * pow(h, 10.0 / 3.0));
        double us2 = p->g * h * sf;
        double uscr2 = theta_cr * p->g * (Sg - 1.0) * d50;
        double T = (us2 - uscr2) / uscr2;
        if (!(T > 0.0)) { *dqs_dh = 0.0; *dqs_dq = 0.0; return; }
        double Dstar = d50 * cbrt(p->g * (Sg - 1.0) / (nu * nu));
        double scale = 0.053 / pow(Dstar, 0.3) * sqrt(p->g * (Sg - 1.0) * d50 * d50 * d50);
        double dqs_dT = scale * 2.1 * pow(T, 1.1);
        /* u_*^2 = g q^2 / (K_s^2 h^(7/3)): dT/dq = 2 (T + 1) / q, dT/dh = -(7/3) (T + 1) / h */
        *dqs_dq = dqs_dT * 2.0 * (T + 1.0) / fabs(q);
        *dqs_dh = sign_of(q) * dqs_dT * (-7.0 / 3.0) * (T + 1.0) / h;
        return;
    }
    default:
        *dqs_dh = NAN;
        *dqs_dq = NAN;
        return;
    }
}

/* Friction slope (Sec. 2) with the sign of the flow, s_f = q |q| / (K_s^2 h^(10/3)), so that
 * the momentum source -c^2 s_f opposes the flow (reading: the printed q^2 is the magnitude). */
static double friction_slope(double h, double q, double ks)
{
    return q * fabs(q) / (ks * ks * pow(h, 10.0 / 3.0));
}

/* Flux matrix of the quasi-linear system (Sec. 2, Eq. W&A_definition):
 *   A = [[0, 1, 0], [c^2 - u^2, 2u, c^2], [xi dq_s/dh, xi dq_s/dq, 0]],
 * u = q/h, c = sqrt(g h).  Row-major 3x3. */
void or_flux_matrix(const double W[3], const or_phys *p, double A[9])
{
    double h = W[0], q = W[1];
    double u = q / h;
    double c2 = p->g * h;
    double dqs_dh, dqs_dq;
    qs_derivatives(h, q, p, &dqs_dh, &dqs_dq);
    A[0] = 0.0;              A[1] = 1.0;               A[2] = 0.0;
    A[3] = c2 - u * u;       A[4] = 2.0 * u;           A[5] = c2;
    A[6] = p->xi * dqs_dh;   A[7] = p->xi * dqs_dq;    A[8] = 0.0;
}

/* Steps 1-4 of the A-DOT procedure (Sec. 3.3).
 *   step 2: k1 = 3 + Fr^2 + 3 xi dq_s/dq                         (Eq. parameters)
 *           k2 = -2 Fr^3 + 18 Fr (1 + xi dq_s/dq) + 27 xi dq_s/dh / c   (Eq. parameters_bis)
 *           phi = arccos(k2 / sqrt(4 k1^3))                       (Eq. parameters)
 *   step 3: lambda_1/c = 2/3 Fr - 2/3 sqrt(k1) cos(phi/3 - pi/3)
 *           lambda_2/c = 2/3 Fr - 2/3 sqrt(k1) cos(phi/3 + pi/3)
 *           lambda_3/c = 2/3 Fr + 2/3 sqrt(k1) cos(phi/3)          (Eq. lambda)
 *           and store them;
 *   step 4: right eigenvectors r_m = [1, lambda_m, (u - lambda_m)^2/c^2 - 1]^T   (Eq. RR)
 *           left eigenvectors  l_i = [c^2 - u^2 + l_j l_k, 2u - l_j - l_k, c^2]
 *                                    / ((l_i - l_j)(l_i - l_k))          (Eq. RR-1)
 *           with (i, j, k) the circular permutation of Eq. circPerm,
 *           all from the stored eigenvalues.
 * R holds r_m as columns, Rinv holds l_i as rows (row-major 3x3).
 * Fr = u/c keeps its sign (reading: the formulas are used for u < 0 too).
 * The arccos argument is clamped to [-1, 1]; if it lies further than 1e-12
 * outside, or k1 <= 0, *nonhyp is set (the roots would not be real; this
 * cannot happen for the Grass law with A_g >= 0).  When R^-1 is asked for and two
 * stored eigenvalues are equal, *nonhyp is set too: the denominators of Eq. RR-1
 * vanish and R^-1 does not exist (the eigenvalues are distinct for a movable bed,
 * Sec. 3.3; with a fixed bed they coalesce at Fr = +-1). */
int or_eigensystem(const double W[3], const or_phys *p, double lam[3], double R[9], double Rinv[9],
                   int *nonhyp)
{
    double h = W[0], q = W[1];
    double u = q / h;
    double c2 = p->g * h;
    double c = sqrt(c2);
    double Fr = u / c;
    /* step 1 */
    double dqs_dh, dqs_dq;
    qs_derivatives(h, q, p, &dqs_dh, &dqs_dq);
    /* step 2 */
    double k1 = 3.0 + Fr * Fr + 3.0 * p->xi * dqs_dq;
    double k2 = -2.0 * Fr * Fr * Fr + 18.0 * Fr * (1.0 + p->xi * dqs_dq) + 27.0 * p->xi * dqs_dh / c;
    double arg = k2 / sqrt(4.0 * k1 * k1 * k1);
    if (nonhyp && isfinite(k1) && isfinite(k2) && (!(k1 > 0.0) || fabs(arg) > 1.0 + OR_ACOS_TOL))
        *nonhyp = 1;
    if (arg > 1.0) arg = 1.0;
    if (arg < -1.0) arg = -1.0;
    double phi = acos(arg);
    /* step 3 */
    lam[0] = c * (2.0 / 3.0 * Fr - 2.0 / 3.0 * sqrt(k1) * cos(phi / 3.0 - OR_PI / 3.0));
    lam[1] = c * (2.0 / 3.0 * Fr - 2.0 / 3.0 * sqrt(k1) * cos(phi / 3.0 + OR_PI / 3.0));
    lam[2] = c * (2.0 / 3.0 * Fr + 2.0 / 3.0 * sqrt(k1) * cos(phi / 3.0));
    /* step 4: right eigenvectors as columns of R */
    if (R) {
        for (int m = 0; m < 3; ++m) {
            R[0 * 3 + m] = 1.0;
            R[1 * 3 + m] = lam[m];
            R[2 * 3 + m] = (u - lam[m]) * (u - lam[m]) / c2 - 1.0;
        }
    }
    /* step 4: left eigenvectors as rows of R^-1, circular permutation (i, j, k) */
    if (Rinv) {
        for (int i = 1; i <= 3; ++i) {
            int j = (i < 3) ? i + 1 : i - 2;
            int k = (i < 2) ? i + 2 : i - 1;
            double li = lam[i - 1], lj = lam[j - 1], lk = lam[k - 1];
            double den = (li - lj) * (li - lk);
            if (nonhyp && den == 0.0) *nonhyp = 1;
            Rinv[(i - 1) * 3 + 0] = (c2 - u * u + lj * lk) / den;
            Rinv[(i - 1) * 3 + 1] = (2.0 * u - lj - lk) / den;
            Rinv[(i - 1) * 3 + 2] = c2 / den;
        }
    }
    return OR_OK;
}

/* Step 5 (Sec. 3.3, Eq. ExAbsA; definition Eq. asbA): |A| = R diag(|lambda|) R^-1
 * evaluated as the explicit product of the three matrices. */
int or_abs_matrix(const double W[3], const or_phys *p, double absA[9], int *nonhyp)
{
    double lam[3], R[9], Rinv[9], RL[9];
    or_eigensystem(W, p, lam, R, Rinv, nonhyp);
    for (int r = 0; r < 3; ++r)
        for (int m = 0; m < 3; ++m) RL[r * 3 + m] = R[r * 3 + m] * fabs(lam[m]);
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) acc += RL[r * 3 + m] * Rinv[m * 3 + cc];
            absA[r * 3 + cc] = acc;
        }
    return OR_OK;
}

/* DOT fluctuations at one edge (Sec. 3.1, Eq. DOTjumpN with the segment path Eq. path):
 *   D^{+-} = 1/2 sum_k w_k (A(Psi(s_k)) +- |A(Psi(s_k))|) (W+ - W-),
 *   Psi(s) = W- + s (W+ - W-).
 * A is the explicit flux matrix (Eq. W&A_definition), |A| the triple product. */
int or_fluct(const double Wm[3], const double Wp[3], const or_phys *p, int G, const double *s,
             const double *w, double Dm[3], double Dp[3], int *nonhyp)
{
    double dW[3], Sm[3] = {0.0, 0.0, 0.0}, Sp[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < 3; ++r) dW[r] = Wp[r] - Wm[r];
    for (int k = 0; k < G; ++k) {
        double Psi[3], A[9], absA[9];
        for (int r = 0; r < 3; ++r) Psi[r] = Wm[r] + s[k] * dW[r];
        or_flux_matrix(Psi, p, A);
        or_abs_matrix(Psi, p, absA, nonhyp);
        for (int r = 0; r < 3; ++r) {
            double am = 0.0, ap = 0.0;
            for (int cc = 0; cc < 3; ++cc) {
                am += (A[r * 3 + cc] - absA[r * 3 + cc]) * dW[cc];
                ap += (A[r * 3 + cc] + absA[r * 3 + cc]) * dW[cc];
            }
            Sm[r] += w[k] * am;
            Sp[r] += w[k] * ap;
        }
    }
    for (int r = 0; r < 3; ++r) {
        Dm[r] = 0.5 * Sm[r];
        Dp[r] = 0.5 * Sp[r];
    }
    return OR_OK;
}

/* Largest characteristic speed of one state, max_m |lambda_m| (used by the CFL rule). */
static double state_speed(const double W[3], const or_phys *p, int *nonhyp)
{
    double lam[3];
    or_eigensystem(W, p, lam, NULL, NULL, nonhyp);
    double a = fabs(lam[0]);
    if (fabs(lam[1]) > a) a = fabs(lam[1]);
    if (fabs(lam[2]) > a) a = fabs(lam[2]);
    return a;
}

/* ------------------------------------------------------------------------- */
/* Threading helpers: split [0, n) into contiguous parts. */
typedef void (*range_fn)(void *ctx, int64_t lo, int64_t hi, int part);

typedef struct {
    range_fn fn;
    void *ctx;
    int64_t lo, hi;
    int part;
} range_job;

static void *range_thread(void *arg)
{
    range_job *j = (range_job *)arg;
    j->fn(j->ctx, j->lo, j->hi, j->part);
    return NULL;
}

static int clamp_threads(int nthreads, int64_t n)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (n < (int64_t)nthreads) nthreads = (int)(n > 0 ? n : 1);
    return nthreads;
}

static void parallel_for(int64_t n, int nthreads, range_fn fn, void *ctx)
{
    nthreads = clamp_threads(nthreads, n);
    if (nthreads == 1) {
        fn(ctx, 0, n, 0);
        return;
    }
    pthread_t th[256];
    range_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn;
        jobs[t].ctx = ctx;
        jobs[t].lo = n * t / nthreads;
        jobs[t].hi = n * (t + 1) / nthreads;
        jobs[t].part = t;
        pthread_create(&th[t], NULL, range_thread, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Batched per-state eigen-decomposition, for the tests: n states (SoA h, q, z).
 * Outputs (any may be NULL): lam[3n] (lam[3i+m]), R[9n], Rinv[9n], A[9n], absA[9n]
 * (each 3x3 row-major per state). Returns OR_E_NONHYPERBOLIC if any state's
 * arccos argument was out of range. */
int or_eig_batch(int64_t n, const double *h, const double *q, const double *z, const or_phys *pp,
                 double *lam, double *R, double *Rinv, double *A, double *absA)
{
    or_phys p = *pp;
    int nonhyp = 0;
    for (int64_t i = 0; i < n; ++i) {
        double W[3] = {h[i], q[i], z[i]};
        double l[3], r[9], ri[9];
        or_eigensystem(W, &p, l, r, ri, &nonhyp);
        if (lam) memcpy(lam + 3 * i, l, sizeof l);
        if (R) memcpy(R + 9 * i, r, sizeof r);
        if (Rinv) memcpy(Rinv + 9 * i, ri, sizeof ri);
        if (A) or_flux_matrix(W, &p, A + 9 * i);
        if (absA) or_abs_matrix(W, &p, absA + 9 * i, NULL);
    }
    return nonhyp ? OR_E_NONHYPERBOLIC : OR_OK;
}

/* Pairwise fluctuations for n independent edges.  Inputs SoA left/right states;
 * outputs Dm, Dp laid out [3][n] (row r of edge e at r*n + e). */
typedef struct {
    const double *hL, *qL, *zL, *hR, *qR, *zR;
    or_phys p;
    int G;
    const double *s, *w;
    int64_t n;
    double *Dm, *Dp;
    int nonhyp[256];
} fluct_batch_ctx;

static void fluct_batch_range(void *vctx, int64_t lo, int64_t hi, int part)
{
    fluct_batch_ctx *c = (fluct_batch_ctx *)vctx;
    for (int64_t e = lo; e < hi; ++e) {
        double Wm[3] = {c->hL[e], c->qL[e], c->zL[e]};
        double Wp[3] = {c->hR[e], c->qR[e], c->zR[e]};
        double dm[3], dp[3];
        or_fluct(Wm, Wp, &c->p, c->G, c->s, c->w, dm, dp, &c->nonhyp[part]);
        for (int r = 0; r < 3; ++r) {
            c->Dm[r * c->n + e] = dm[r];
            c->Dp[r * c->n + e] = dp[r];
        }
    }
}

int or_fluct_batch(int64_t n, const double *hL, const double *qL, const double *zL, const double *hR,
                   const double *qR, const double *zR, const or_phys *pp, int G, double *Dm,
                   double *Dp, int nthreads)
{
    if (n < 0 || G < 1 || G > 64) return OR_E_ARG;
    double s[64], w[64];
    or_gauss(G, s, w);
    fluct_batch_ctx *c = (fluct_batch_ctx *)calloc(1, sizeof(fluct_batch_ctx));
    c->hL = hL; c->qL = qL; c->zL = zL; c->hR = hR; c->qR = qR; c->zR = zR;
    c->p = *pp;
    c->G = G; c->s = s; c->w = w; c->n = n; c->Dm = Dm; c->Dp = Dp;
    parallel_for(n, nthreads, fluct_batch_range, c);
    int nonhyp = 0;
    for (int t = 0; t < 256; ++t) nonhyp |= c->nonhyp[t];
    free(c);
    return nonhyp ? OR_E_NONHYPERBOLIC : OR_OK;
}

/* ------------------------------------------------------------------------- */
/* CFL reduction: amax = max over the real cells i of max_m |lambda_m(W_i)|. */
typedef struct {
    const double *h, *q, *z;
    or_phys p;
    double part_max[256];
    int nonhyp[256];
} amax_ctx;

static void amax_range(void *vctx, int64_t lo, int64_t hi, int part)
{
    amax_ctx *c = (amax_ctx *)vctx;
    double m = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        double W[3] = {c->h[i], c->q[i], c->z[i]};
        double a = state_speed(W, &c->p, &c->nonhyp[part]);
        /* a NaN speed must win the maximum so that it is detected */
        if (a > m || isnan(a)) m = a;
        if (isnan(m)) break;
    }
    c->part_max[part] = m;
}

static double amax_of(int64_t n, const double *h, const double *q, const double *z, const or_phys *p,
                      int nthreads, int *nonhyp)
{
    amax_ctx *c = (amax_ctx *)calloc(1, sizeof(amax_ctx));
    c->h = h; c->q = q; c->z = z; c->p = *p;
    int nt = clamp_threads(nthreads, n);
    parallel_for(n, nt, amax_range, c);
    double m = 0.0;
    for (int t = 0; t < nt; ++t) {
        if (c->part_max[t] > m || isnan(c->part_max[t])) m = c->part_max[t];
        if (isnan(m)) break;
    }
    for (int t = 0; t < 256; ++t) *nonhyp |= c->nonhyp[t];
    free(c);
    return m;
}

int or_cfl_amax(int64_t n, const double *h, const double *q, const double *z, const or_phys *pp,
                double *amax, int nthreads)
{
    or_phys p = *pp;
    int nonhyp = 0;
    *amax = amax_of(n, h, q, z, &p, nthreads, &nonhyp);
    if (nonhyp) return OR_E_NONHYPERBOLIC;
    if (!isfinite(*amax)) return OR_E_NONFINITE;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* One first-order path-conservative step (Sec. 3, Eq. scheme, S = 0) on one
 * channel of N cells with given ghost states and time step:
 *   W_i^{n+1} = W_i^n - dt/dx (D^-_{i+1/2} + D^+_{i-1/2}).
 * Edge e (e = 0..N) lies between cell e-1 and cell e; cell -1 is the left
 * ghost and cell N the right ghost.  The new state is written to hn, qn, zn. */
typedef struct {
    const double *h, *q, *z;
    const double *gl, *gr;
    int64_t N;
    or_phys p;
    int G;
    const double *s, *w;
    double *Dm, *Dp; /* [3][N+1] */
    double *hn, *qn, *zn;
    double dt, dx;
    int nonhyp[256];
} step_ctx;

static void edge_range(void *vctx, int64_t lo, int64_t hi, int part)
{
    step_ctx *c = (step_ctx *)vctx;
    int64_t E = c->N + 1;
    for (int64_t e = lo; e < hi; ++e) {
        double Wm[3], Wp[3], dm[3], dp[3];
        if (e == 0) { Wm[0] = c->gl[0]; Wm[1] = c->gl[1]; Wm[2] = c->gl[2]; }
        else { Wm[0] = c->h[e - 1]; Wm[1] = c->q[e - 1]; Wm[2] = c->z[e - 1]; }
        if (e == c->N) { Wp[0] = c->gr[0]; Wp[1] = c->gr[1]; Wp[2] = c->gr[2]; }
        else { Wp[0] = c->h[e]; Wp[1] = c->q[e]; Wp[2] = c->z[e]; }
        or_fluct(Wm, Wp, &c->p, c->G, c->s, c->w, dm, dp, &c->nonhyp[part]);
        for (int r = 0; r < 3; ++r) {
            c->Dm[r * E + e] = dm[r];
            c->Dp[r * E + e] = dp[r];
        }
    }
}

static void update_range(void *vctx, int64_t lo, int64_t hi, int part)
{
    (void)part;
    step_ctx *c = (step_ctx *)vctx;
    int64_t E = c->N + 1;
    double r = c->dt / c->dx;
    for (int64_t i = lo; i < hi; ++i) {
        /* D^-_{i+1/2} is edge i+1 (right face), D^+_{i-1/2} is edge i (left face) */
        c->hn[i] = c->h[i] - r * (c->Dm[0 * E + i + 1] + c->Dp[0 * E + i]);
        c->qn[i] = c->q[i] - r * (c->Dm[1 * E + i + 1] + c->Dp[1 * E + i]);
        c->zn[i] = c->z[i] - r * (c->Dm[2 * E + i + 1] + c->Dp[2 * E + i]);
        /* point source dt S(W_i^n), S = (0, -c^2 s_f, 0) with c^2 = g h (Sec. 2, Eq. scheme) */
        if (c->p.ks > 0.0)
            c->qn[i] += c->dt * (-c->p.g * c->h[i] * friction_slope(c->h[i], c->q[i], c->p.ks));
    }
}

int or_step(int64_t N, const double *h, const double *q, const double *z, const double ghost_l[3],
            const double ghost_r[3], const or_phys *pp, int G, double dt, double dx,
            double *hn, double *qn, double *zn, int nthreads)
{
    if (N < 1 || G < 1 || G > 64) return OR_E_ARG;
    double s[64], w[64];
    or_gauss(G, s, w);
    step_ctx *c = (step_ctx *)calloc(1, sizeof(step_ctx));
    c->h = h; c->q = q; c->z = z; c->gl = ghost_l; c->gr = ghost_r; c->N = N;
    c->p = *pp; c->G = G; c->s = s; c->w = w;
    c->Dm = (double *)malloc(sizeof(double) * 3 * (N + 1));
    c->Dp = (double *)malloc(sizeof(double) * 3 * (N + 1));
    c->hn = hn; c->qn = qn; c->zn = zn; c->dt = dt; c->dx = dx;
    parallel_for(N + 1, nthreads, edge_range, c);
    parallel_for(N, nthreads, update_range, c);
    int nonhyp = 0;
    for (int t = 0; t < 256; ++t) nonhyp |= c->nonhyp[t];
    free(c->Dm);
    free(c->Dp);
    free(c);
    return nonhyp ? OR_E_NONHYPERBOLIC : OR_OK;
}

/* Ghost states from the boundary conditions (reading: the paper does not spell
 * out the ghost-cell form):  transmissive = copy of the adjacent cell;
 * periodic = the cell at the other end; inflow-q = (h, q_in, z) of the adjacent cell;
 * fixed depth = (h_out, q, z) of the adjacent cell; inflow-(q, h) = (h_in, q_in, z) of the
 * adjacent cell (an imposed solid discharge enters through the depth h_in at which the
 * closure gives that q_s for q_in, Sec. 5.1); Dirichlet = a given state whose bed level moves
 * at a constant rate, (h_d, q_d, z_d + t dz/dt) at the time t of the step's start (the
 * ghost cells of an analytical solution such as Sec. 4.2, Eq. berthon, whose bed falls
 * linearly in time). */
static void ghost_states(const or_channel *ch, const double *h, const double *q, const double *z,
                         double t, double gl[3], double gr[3])
{
    int64_t N = ch->n_cells;
    switch (ch->bc_left) {
    case OR_BC_PERIODIC: gl[0] = h[N - 1]; gl[1] = q[N - 1]; gl[2] = z[N - 1]; break;
    case OR_BC_INFLOW_Q: gl[0] = h[0]; gl[1] = ch->q_in; gl[2] = z[0]; break;
    case OR_BC_FIXED_DEPTH: gl[0] = ch->h_out; gl[1] = q[0]; gl[2] = z[0]; break;
    case OR_BC_INFLOW_QH: gl[0] = ch->h_in; gl[1] = ch->q_in; gl[2] = z[0]; break;
    case OR_BC_DIRICHLET:
        gl[0] = ch->dir_l[0]; gl[1] = ch->dir_l[1]; gl[2] = ch->dir_l[2] + t * ch->dir_l[3];
        break;
    default: gl[0] = h[0]; gl[1] = q[0]; gl[2] = z[0]; break;
    }
    switch (ch->bc_right) {
    case OR_BC_PERIODIC: gr[0] = h[0]; gr[1] = q[0]; gr[2] = z[0]; break;
    case OR_BC_INFLOW_Q: gr[0] = h[N - 1]; gr[1] = ch->q_in; gr[2] = z[N - 1]; break;
    case OR_BC_FIXED_DEPTH: gr[0] = ch->h_out; gr[1] = q[N - 1]; gr[2] = z[N - 1]; break;
    case OR_BC_INFLOW_QH: gr[0] = ch->h_in; gr[1] = ch->q_in; gr[2] = z[N - 1]; break;
    case OR_BC_DIRICHLET:
        gr[0] = ch->dir_r[0]; gr[1] = ch->dir_r[1]; gr[2] = ch->dir_r[2] + t * ch->dir_r[3];
        break;
    default: gr[0] = h[N - 1]; gr[1] = q[N - 1]; gr[2] = z[N - 1]; break;
    }
}

static int check_channel(const or_channel *ch)
{
    if (ch->n_cells < 1) return OR_E_ARG;
    if (ch->n_gauss < 1 || ch->n_gauss > 64) return OR_E_ARG;
    if (!(ch->cfl > 0.0) || !(ch->dx > 0.0) || !(ch->g > 0.0) || !(ch->xi >= 1.0)) return OR_E_ARG;
    if (ch->bc_left < 0 || ch->bc_left > 5 || ch->bc_right < 0 || ch->bc_right > 5) return OR_E_ARG;
    if ((ch->bc_left == OR_BC_PERIODIC) != (ch->bc_right == OR_BC_PERIODIC)) return OR_E_ARG;
    if (ch->law < OR_LAW_GRASS || ch->law > OR_LAW_VANRIJN) return OR_E_ARG;
    if ((ch->law == OR_LAW_MPM || ch->law == OR_LAW_VANRIJN) && !(ch->ks > 0.0)) return OR_E_ARG;
    return OR_OK;
}

/* The time loop for one channel: for each step, ghosts from the BCs, then
 * dt = CFL dx / amax(W^n), then the path-conservative update; t += dt.
 * The state (h, q, z) is advanced in place; *t accumulates the time.
 * dt_log, if not NULL, receives the n_steps time steps. */
int or_run(const or_channel *ch, double *h, double *q, double *z, int n_steps, double *t,
           double *dt_log, int nthreads)
{
    int st = check_channel(ch);
    if (st != OR_OK || n_steps < 0) return OR_E_ARG;
    int64_t N = ch->n_cells;
    or_phys p = {ch->g, ch->xi, ch->Ag, ch->law, {ch->par[0], ch->par[1], ch->par[2], ch->par[3]},
                 ch->ks};
    double *hn = (double *)malloc(sizeof(double) * N);
    double *qn = (double *)malloc(sizeof(double) * N);
    double *zn = (double *)malloc(sizeof(double) * N);
    int status = OR_OK;
    for (int n = 0; n < n_steps; ++n) {
        double gl[3], gr[3];
        ghost_states(ch, h, q, z, *t, gl, gr);
        int nonhyp = 0;
        double amax = amax_of(N, h, q, z, &p, nthreads, &nonhyp);
        if (nonhyp) { status = OR_E_NONHYPERBOLIC; break; }
        if (!isfinite(amax) || !(amax > 0.0)) { status = OR_E_NONFINITE; break; }
        double dt = ch->cfl * ch->dx / amax;
        st = or_step(N, h, q, z, gl, gr, &p, ch->n_gauss, dt, ch->dx, hn, qn, zn, nthreads);
        if (st != OR_OK) { status = st; break; }
        memcpy(h, hn, sizeof(double) * N);
        memcpy(q, qn, sizeof(double) * N);
        memcpy(z, zn, sizeof(double) * N);
        *t += dt;
        if (dt_log) dt_log[n] = dt;
    }
    free(hn);
    free(qn);
    free(zn);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Many independent channels: channel c owns cells [off[c], off[c+1]) of the
 * concatenated arrays, its own parameters, time step and clock t[c].
 * Channels are spread over threads; each channel runs single-threaded. */
typedef struct {
    int64_t n_channels;
    const int64_t *off;
    const or_channel *chs;
    double *h, *q, *z, *t;
    int n_steps;
    int status[256];
} batch_ctx;

static void batch_range(void *vctx, int64_t lo, int64_t hi, int part)
{
    batch_ctx *c = (batch_ctx *)vctx;
    for (int64_t ch = lo; ch < hi; ++ch) {
        int64_t o = c->off[ch];
        int st = or_run(&c->chs[ch], c->h + o, c->q + o, c->z + o, c->n_steps, &c->t[ch], NULL, 1);
        if (st != OR_OK && c->status[part] == OR_OK) c->status[part] = st;
    }
}

int or_run_batched(int64_t n_channels, const int64_t *off, const or_channel *chs, double *h, double *q,
                   double *z, int n_steps, double *t, int nthreads)
{
    if (n_channels < 1) return OR_E_ARG;
    for (int64_t c = 0; c < n_channels; ++c) {
        if (chs[c].n_cells != off[c + 1] - off[c]) return OR_E_ARG;
        if (check_channel(&chs[c]) != OR_OK) return OR_E_ARG;
    }
    batch_ctx *c = (batch_ctx *)calloc(1, sizeof(batch_ctx));
    c->n_channels = n_channels; c->off = off; c->chs = chs;
    c->h = h; c->q = q; c->z = z; c->t = t; c->n_steps = n_steps;
    parallel_for(n_channels, nthreads, batch_range, c);
    int status = OR_OK;
    for (int p = 0; p < 256; ++p)
        if (c->status[p] != OR_OK && status == OR_OK) status = c->status[p];
    free(c);
    return status;
}

/* Sizes of the records, so the caller can check its own struct layouts. */
int or_channel_size(void) { return (int)sizeof(or_channel); }
int or_phys_size(void) { return (int)sizeof(or_phys); }
