// dsve_math.hpp -- per-node and per-edge arithmetic of the A-DOT hot path (device code).
//
// Everything is evaluated in the non-dimensional form the paper uses for the characteristic
// polynomial (Sec. 3.3, Eq. charPol): eigenvalues are mu_m = lambda_m / c and depend on the
// Froude number only.  For one state W = (h, q, z):
//   c = sqrt(g h), Fr = u/c = q / sqrt(g h^3)  (one reciprocal square root gives Fr, c, 1/c);
//   Grass closure (Sec. 2 Eq. Grass; Sec. 3.3 step 1), with u^2/h = g Fr^2:
//     b = xi dq_s/dq = 3 xi A_g g Fr^2 = kqg Fr^2,   xi dq_s/dh = -b u;
//   cubic parameters (Eqs. parameters, parameters_bis), substituting the closure:
//     k1 = 3 + Fr^2 + 3b           = 3 + Fr^2 (1 + 3 kqg)
//     k2 = -2Fr^3 + 18Fr(1+b) - 27bFr = Fr (18 - Fr^2 (2 + 9 kqg)),
//     x = k2 / sqrt(4 k1^3),  phi = arccos(x),  theta = phi/3;
//   eigenvalues (Eq. lambda), m = (2/3) sqrt(k1), f = (2/3) Fr:
//     mu_{1,2} = f - m cos(theta -+ pi/3),  mu_3 = f + m cos(theta),
//   with cos(theta -+ pi/3) = cos(theta)/2 +- (sqrt3/2) sin(theta), so one (cos, sin) pair
//   serves all three roots and the gaps follow without cancellation:
//     mu_2 - mu_1 = sqrt3 m sin(theta),  mu_3 - mu_1 = m (3/2 cos + sqrt3/2 sin),
//     mu_3 - mu_2 = m (3/2 cos - sqrt3/2 sin);
//   right eigenvectors (Eq. RR):  r_m = [1, c mu_m, (Fr - mu_m)^2 - 1];
//   left eigenvectors (Eqs. RR-1, circPerm), the factor c^2 of numerator and denominator
//   cancelling:  l_i . dW = [(1 - Fr^2 + mu_j mu_k) dh + (2Fr - mu_j - mu_k) dq/c + dz]
//                           / ((mu_i - mu_j)(mu_i - mu_k)),
//   where 2Fr - mu_j - mu_k = mu_i (the roots sum to the trace, 2Fr), and the three
//   denominators come from the gap products (one reciprocal for all three).
// Other closures (Sec. 2, Eqs. GrassThr, MPM, vanRijn; Sec. 5.1, Eq. Soni_qs) enter through
// b = xi dq_s/dq, evaluated per state.  Each depends on (h, q) through the velocity u = q/h
// (Grass-type laws) or through q^2 / h^(7/3) (laws of the Shields stress or shear velocity,
// where s_f h and g h s_f carry that combination), and the chain rule then gives
// xi dq_s/dh = -kappa b u with kappa = 1 or 7/6 respectively, so that
//     k1 = 3 + Fr^2 + 3b,   k2 = Fr (18 - 2 Fr^2 + (18 - 27 kappa) b),
//     xi (dq_s/dh dh + dq_s/dq dq) = b c (dq/c - kappa Fr dh);
// the Grass law is kappa = 1 with b = kqg Fr^2.
// The fluctuation (Sec. 3.1, Eq. DOTjumpN) is accumulated as
//   S_A = sum_k w_k A(Psi_k) dW   with the explicit flux matrix (Eq. W&A_definition):
//         A dW = [dq, c^2 ((1 - Fr^2) dh + 2Fr dq/c + dz), b c (dq/c - kappa Fr dh)],
// and, in FP64,
//   D^- = sum_k w_k A^-(Psi_k) dW,  D^+ = S_A - D^-,
// where A^- = (A - |A|)/2 (Eqs. asbA, ExAbsA) is the sum of c mu_m r_m l_m over the negative
// eigenvalues.  The root labelled 3 below is always the middle one, so at most one root differs
// in sign from it, and A^- takes one eigenpair o: A^- dW = c min(mu_o, 0) (l_o . dW) r_o when
// mu_3 >= 0 (o the smallest root), A^- dW = A dW - c max(mu_o, 0) (l_o . dW) r_o when mu_3 < 0
// (o the largest).  So |A| is never formed, and R^-1 dW is needed for one row only.
// The mixed form sums in FP32
//   S_B = sum_k w_k |A(Psi_k)| dW  with |A| dW = sum_m c |mu_m| (l_m . dW) r_m,
//   D^- = (S_A - S_B)/2,  D^+ = (S_A + S_B)/2,
// whose rounding is spread evenly over D^- and D^+ (with one eigenpair, FP32 rounding lands on
// whichever of the two is formed as a difference, and long runs through stagnant flow drift
// further from FP64).
//
// Arithmetic kernels (own implementations of published methods):
//   rcp_h / rsqrt_h: hardware reciprocal / reciprocal-square-root estimate (about 2^-24
//     relative) refined by one Halley step (cubic convergence, about 2^-72).
//   third_angle: cos(theta), sin(theta), theta = arccos(a)/3 for a = |x| in [0, 1], where the
//     function is analytic (its branch point is at a = -1): the cosine C from a degree-7
//     polynomial in 1 - a (FP32) and two Newton steps on the trisection cubic 4C^3 - 3C = a
//     (FP64), the sine from sin(3 theta) = S (4C^2 - 1), i.e. S = sqrt(1 - a^2) / (4C^2 - 1),
//     with 4C^2 - 1 in [2, 3].  The roots at -x are those at x negated, so the eigenvalues are
//     sign(x) {C, -P, -Q} about f, P, Q = C/2 +- (sqrt3/2) S, labelled in that order, not
//     sorted (a sum over the three eigenpairs is symmetric in the labels); since P >= Q >= 0,
//     mu_3 is the middle root, and mu_2 the smallest for x >= 0 and the largest for x < 0.
//   Gap product: (mu_2 - mu_1)(mu_3 - mu_1)(mu_3 - mu_2) = (3 sqrt3 / 4) m^3 sin(3 theta)
//     = (2 sqrt3 / 9) k1^(3/2) sin(phi), so its reciprocal is (3 sqrt3 / 2) k1^(-3/2) / sin(phi),
//     from the k1^(-1/2) and 1/sin(phi) the roots already need.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dsve_internal.hpp"

namespace dsve {

constexpr double kSqrt3Half = 0.86602540378443864676372317075293618;
constexpr double kAcosTol = 1e-12;            // tolerance on |arccos argument| - 1 before flagging
constexpr double kInvGapScale = 2.59807621135331594029116951225880855;   // 3 sqrt3 / 2
constexpr float kMixedFp64Band = 1e-2f;       // mixed form: 1 - |x| below this -> FP64 node

// Unrolling of the quadrature-node loop (independent nodes interleave for ILP when unrolled;
// a rolled loop needs fewer registers).
#ifndef DSVE_NODE_UNROLL
#define DSVE_NODE_UNROLL 8
#endif
#define DSVE_PRAGMA(x) _Pragma(#x)
#define DSVE_UNROLL(n) DSVE_PRAGMA(unroll n)


// 1/x: r (1 + e + e^2), e = 1 - x r
__device__ __forceinline__ double rcp_h(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// 1/sqrt(x): r (1 + e/2 + 3e^2/8), e = 1 - x r^2
__device__ __forceinline__ double rsqrt_h(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * r, r, 1.0);
    return fma(r * e, fma(e, 0.375, 0.5), r);
}

// ---------------------------------------------------------------------------
// Per-channel constants of the closure: kqg = 3 xi A_g g, K1 = 1 + 3 kqg, K2h = 1 + 4.5 kqg for
// the Grass law in closed form; the law and its constants lp0, lp1 for the general form.
struct Closure {
    double kqg, K1, K2h;
    double lp0, lp1;
    int law, ipow;
};
__device__ __forceinline__ Closure closure_of(const ChanInfo &ci)
{
    return Closure{ci.kqg, ci.K1, ci.K2h, ci.lp0, ci.lp1, ci.law, ci.ipow};
}

// FP64 power a^b, a > 0, as 2^(b log2 a): a relative error of about 2 |b log2 a| ulp, a few ulp
// at the laws' speeds, at well under half the cost of the library pow
__device__ __forceinline__ double m_pow(double a, double b) { return exp2(b * log2(a)); }
// FP32 power of the mixed form, a >= 0, b > 0: 2^(b log2 a) from the hardware base-2 logarithm
// and exponential (relative error about 1e-6 for the exponents of the laws; a = 0 gives 0)
__device__ __forceinline__ float m_pow(float a, float b)
{
    return __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(a));
}
// a^n, n in [0, 15], as a product of a, a^2, a^4, a^8
template <typename T>
__device__ __forceinline__ T ipow15(T a, int n)
{
    const T a2 = a * a, a4 = a2 * a2, a8 = a4 * a4;
    T r = (n & 1) ? a : T(1);
    r = (n & 2) ? r * a2 : r;
    r = (n & 4) ? r * a4 : r;
    return (n & 8) ? r * a8 : r;
}
// a^1.1 = a^2 y^9 with y = a^(-1/10), a > 0: y from an FP32 estimate 2^(-log2(a)/10) and two
// Newton steps for y^-10 = a in FP64, y <- y (11 - a y^10) / 10 (each takes a relative error e
// to about 5.5 e^2: 4e-7 -> 1e-12 -> the rounding of y^9, a few ulp); no division
__device__ __forceinline__ double pow_1p1(double a);
__device__ __forceinline__ float pow_1p1(float a) { return m_pow(a, 1.1f); }
// a^(-1/3), a > 0: FP32 estimate 2^(-log2(a)/3) from the hardware base-2 logarithm and
// exponential, then two Newton steps for y^-3 = a, y <- y (4 - a y^3) / 3, in FP64 (each takes a
// relative error e to about 2 e^2: 1e-6 -> 2e-12 -> the rounding of the last step); no division
__device__ __forceinline__ double rcbrt_h(double a)
{
    double y = (double)__builtin_amdgcn_exp2f(-(1.0f / 3.0f) * __builtin_amdgcn_logf((float)a));
#pragma unroll
    for (int it = 0; it < 2; ++it) y = (y * (1.0 / 3.0)) * fma(-a, y * y * y, 4.0);
    return y;
}
__device__ __forceinline__ double m_rcbrt(double a) { return rcbrt_h(a); }
__device__ __forceinline__ float m_rcbrt(float a)
{
    return __builtin_amdgcn_exp2f(-(1.0f / 3.0f) * __builtin_amdgcn_logf(a));
}
__device__ __forceinline__ double m_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float m_sqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double m_abs(double a) { return fabs(a); }
__device__ __forceinline__ float m_abs(float a) { return fabsf(a); }
__device__ __forceinline__ double pow_1p1(double a)
{
    double y = (double)__builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf((float)fmax(a, 1e-30)));
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y2 = y * y, y5 = y2 * y2 * y;
        y = (y * 0.1) * fma(-a, y5 * y5, 11.0);
    }
    const double y2 = y * y, y4 = y2 * y2;
    return (a * a) * (y4 * y4 * y);
}

// b = xi dq_s/dq of the closure CL at the state (h, q), invh = 1/h (constants lp0, lp1 of the
// law as laid out in ChanInfo).  Below a law's threshold, and at rest, b = 0.
template <int CL, typename T>
__device__ __forceinline__ T law_b(const Closure &K, T h, T q, T invh)
{
    const T lp0 = T(K.lp0), lp1 = T(K.lp1);
    const T u = q * invh;
    const T au = m_abs(u);
    if constexpr (CL == CL_GRASS) {
        return lp0 * (u * u) * invh;
    } else if constexpr (CL == CL_GRASS_THR) {
        const T ex = au - lp1;
        return ex > T(0) ? lp0 * (ex * ex) * invh : T(0);
    } else if constexpr (CL == CL_POWER) {
        return au > T(0) ? lp0 * m_pow(au, lp1) * invh : T(0);
    } else if constexpr (CL == CL_POWER_INT) {
        return au > T(0) ? lp0 * ipow15(au, K.ipow) * invh : T(0);
    } else if constexpr (CL == CL_MPM) {
        // b = lp1 sqrt(th - 0.047) th / |q| with the Shields stress th = lp0 u^2 h^(-1/3); since
        // |q| = h |u|, th / |q| = lp0 |u| h^(-1/3) / h, which needs no reciprocal of q
        const T r = m_rcbrt(h);
        const T th = lp0 * (u * u) * r;
        return th > T(0.047) ? lp1 * m_sqrt(th - T(0.047)) * (lp0 * au * r * invh) : T(0);
    } else {
        // b = lp1 T^1.1 (T + 1) / |q| with T + 1 = u_*^2 / u_*cr^2 = lp0 u^2 h^(-1/3), the same way
        const T r = m_rcbrt(h);
        const T tt = lp0 * (u * u) * r - T(1);
        return tt > T(0) ? lp1 * pow_1p1(tt) * (lp0 * au * r * invh) : T(0);
    }
}

// Cubic parameters k1, k2 / 2 (Eqs. parameters, parameters_bis), b and kappa Fr at a state (the
// halved k2 is exact: every term is halved).
template <int CL, typename T>
__device__ __forceinline__ void cubic_params(const Closure &K, T h, T q, T g, T Fr, T inv_c,
                                             T &k1, T &k2h, T &b, T &kFr)
{
    const T Fr2 = Fr * Fr;
    if constexpr (CL == CL_GRASS) {
        b = T(K.kqg) * Fr2;
        k1 = fma(Fr2, T(K.K1), T(3));
        k2h = Fr * fma(-Fr2, T(K.K2h), T(9));
        kFr = Fr;
    } else {
        const T invh = g * (inv_c * inv_c);   // c^2 = g h
        b = law_b<CL, T>(K, h, q, invh);
        constexpr bool stress = CL == CL_MPM || CL == CL_VANRIJN;
        const T kk = stress ? T(-6.75) : T(-4.5);   // (18 - 27 kappa) / 2
        k1 = fma(T(3), b, fma(Fr, Fr, T(3)));
        k2h = Fr * fma(kk, b, fma(-Fr, Fr, T(9)));
        kFr = stress ? T(7.0 / 6.0) * Fr : Fr;
    }
}

// cos(arccos(a) / 3) for a in [0, 1] in FP32: the function is analytic there (its branch point is
// at a = -1); a polynomial of degree 7 in t = 1 - a, interpolated at the Chebyshev nodes of
// [0, 1] in 50-digit arithmetic, meets it to about 1 ulp in FP32.
__device__ __forceinline__ float cos_third_acos(float a)
{
    const float t = 1.0f - a;
    float p = -0.0005426077404990792f;
    p = fmaf(p, t, 0.0008754234877415001f);
    p = fmaf(p, t, -0.0015220807399600744f);
    p = fmaf(p, t, -0.0008192436653189361f);
    p = fmaf(p, t, -0.004411802161484957f);
    p = fmaf(p, t, -0.01644226536154747f);
    p = fmaf(p, t, -0.11111201345920563f);
    return fmaf(p, t, 1.0f);
}
// The same in FP64: C = cos(arccos(a) / 3) is the root in [cos(pi/6), 1] of the trisection cubic
// f(C) = 4C^3 - 3C - a, whose derivative 12C^2 - 3 is at least 6 there.  From the FP32 estimate,
// two Newton steps in FP64 dividing by the derivative taken once in FP32: each takes an error e to
// about e * 1e-7 + e^2 (1e-7 -> 4e-14 -> FP64 rounding).  Its FP32 constants are instruction
// literals, so nothing stays in registers between calls.  r receives the FP32 reciprocal of the
// derivative.
__device__ __forceinline__ double cos_third_acos(double a, double &r)
{
    const float cf = cos_third_acos((float)a);
    r = (double)__builtin_amdgcn_rcpf(fmaf(12.0f * cf, cf, -3.0f));
    double c = (double)cf;
#pragma unroll
    for (int k = 0; k < 2; ++k) c = fma(-fma(c, fma(4.0 * c, c, -3.0), -a), r, c);
    return c;
}
__device__ __forceinline__ double cos_third_acos(double a)
{
    double r;
    return cos_third_acos(a, r);
}

// cos(theta) and sin(theta) for theta = arccos(a) / 3, a in [0, 1] (theta in [0, pi/6]), given
// y = sin(3 theta) = sqrt(1 - a^2).  Since sin(3 theta) = S (3 - 4 S^2) = S (4 C^2 - 1) and
// 4 C^2 - 1 lies in [2, 3], S = y / (4 C^2 - 1) keeps the relative accuracy of y as a -> 1,
// where S -> 0 (no cancellation, unlike sqrt(1 - C^2)).  The reciprocal 1 / (4 C^2 - 1) is three
// times the FP32 reciprocal of the derivative above, refined by one Halley step (e ~ 1e-7 ->
// e^3).
__device__ __forceinline__ void third_angle(double a, double y, double &C, double &S)
{
    double r;
    C = cos_third_acos(a, r);
    const double u = fma(4.0 * C, C, -1.0);
    const double R0 = 3.0 * r;
    const double e = fma(-u, R0, 1.0);
    S = y * fma(R0, fma(e, e, e), R0);
}
// The same in FP32 (the polynomial alone; one rounded reciprocal).
__device__ __forceinline__ void third_angle(float a, float y, float &C, float &S)
{
    C = cos_third_acos(a);
    S = y * __builtin_amdgcn_rcpf(fmaf(4.0f * C, C, -1.0f));
}


// FP64 non-dimensional eigenstructure at one state.
struct Eig64 {
    double Fr, c, inv_c, b, kFr;
    double mu1, mu2, mu3;
    double g21, g31, g32;   // mu_2 - mu_1, mu_3 - mu_1, mu_3 - mu_2
    double inv_gp;          // 1 / (g21 g31 g32)
    double ms;              // sign(x) m: the smallest root is mu_2 when ms >= 0, mu_1 otherwise
};

// Arccos argument x = k2 / sqrt(4 k1^3) of Eq. parameters at a state, with the quantities the
// eigenstructure reuses: 1/sqrt(g h^3), Fr, 1/c, k1, b, kappa Fr and k1^(-1/2).
template <int CL>
struct ArgX {
    double gh, Fr, inv_c, k1, b, kFr, r1, x;
};
template <int CL>
__device__ __forceinline__ ArgX<CL> arg_x(double h, double q, double g, const Closure &K)
{
    ArgX<CL> a;
    a.gh = g * h;
    const double t = rsqrt_h(a.gh * h * h);   // 1 / sqrt(g h^3)
    a.Fr = q * t;
    a.inv_c = h * t;
    double k2h;
    cubic_params<CL, double>(K, h, q, g, a.Fr, a.inv_c, a.k1, k2h, a.b, a.kFr);
    a.r1 = rsqrt_h(a.k1);
    a.x = k2h * (a.r1 * a.r1 * a.r1);
    return a;
}

// Error bits (kFlag*) from the largest |x| over a set of states, held as a bit pattern (a NaN
// orders above every number): a NaN argument (an overflowed or NaN state, which the clamp would
// turn into -1), complex roots (|x| beyond 1 + tol; k1 = 3 + Fr^2 + 3b > 0 for every closure, so
// k1 <= 0 only comes with a NaN), and, with `coal`, an argument of +-1 after the clamp, where two
// roots coalesce to working precision (sin(phi) = 0: the gap product and R^-1 do not exist).
__device__ __forceinline__ unsigned arg_flags(unsigned long long xmax, bool coal)
{
    if (xmax > 0x7FF0000000000000ull) return kFlagNonfinite;
    const double ax = __longlong_as_double((long long)xmax);
    if (ax > 1.0 + kAcosTol) return kFlagComplex;
    return (coal && ax >= 1.0) ? kFlagCoalesce : 0u;
}
__device__ __forceinline__ void track_arg(unsigned long long &xmax, double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(x));
    xmax = b > xmax ? b : xmax;
}

// The largest |x| seen goes to `xmax` (classified by arg_flags).
template <int CL>
__device__ __forceinline__ void eig64(double h, double q, double g, const Closure &K, Eig64 &E,
                                      unsigned long long &xmax)
{
    const ArgX<CL> a = arg_x<CL>(h, q, g, K);
    const double Fr = a.Fr, inv_c = a.inv_c, k1 = a.k1, b = a.b, kFr = a.kFr, r1 = a.r1;
    const double gh = a.gh, r13 = r1 * r1 * r1;
    track_arg(xmax, a.x);
    const double x = fmin(fmax(a.x, -1.0), 1.0);
    const double v = fma(-x, x, 1.0);
    const double inv_y = rsqrt_h(fmax(v, 1e-300));   // 1 / sin(phi), huge but finite at x = +-1
    double C, S;
    third_angle(fabs(x), v * inv_y, C, S);
    // roots about f: sign(x) m {C, -P, -Q}, P, Q = C/2 +- r, labelled 1, 2, 3 in that order
    const double m = (2.0 / 3.0) * (k1 * r1);
    const double ms = copysign(m, x);
    const double f = (2.0 / 3.0) * Fr;
    const double r = kSqrt3Half * S;
    E.Fr = Fr;
    E.c = gh * inv_c;
    E.inv_c = inv_c;
    E.b = b;
    E.kFr = kFr;
    E.mu1 = fma(ms, C, f);
    E.mu2 = fma(-ms, fma(0.5, C, r), f);
    E.mu3 = fma(-ms, fma(0.5, C, -r), f);
    E.g21 = -ms * fma(1.5, C, r);    // mu2 - mu1 = -ms (P + C)
    E.g31 = -ms * fma(1.5, C, -r);   // mu3 - mu1 = -ms (Q + C)
    E.g32 = (2.0 * ms) * r;          // mu3 - mu2 = ms (P - Q)
    E.ms = ms;
    // 1 / (g21 g31 g32): the gap product is sign(x) (3 sqrt3 / 4) m^3 sin(phi)
    E.inv_gp = (copysign(kInvGapScale, x) * r13) * inv_y;
}

// Largest characteristic speed max_m |lambda_m| of a cell state (the CFL quantity).  k1 is even
// and k2 odd in Fr, so the spectrum at -Fr is the negation of the spectrum at Fr, and the largest
// |mu| is the largest root at |Fr|: mu_3 = (2/3)(|Fr| + sqrt(k1) cos(theta')), theta' =
// arccos(x')/3 with x' = x sign(Fr) the arccos argument at |Fr|.  For x' >= 0 (|Fr| below about 3
// under weak transport) the cosine is cos_third_acos(x'); for x' < 0 it follows from the angle
// at -x' (third_angle).
template <int CL>
__device__ __forceinline__ double speed64(double h, double q, double g, const Closure &K, unsigned &bad)
{
    const ArgX<CL> a = arg_x<CL>(h, q, g, K);
    const double Fr = a.Fr, k1 = a.k1, r1 = a.r1, x = a.x;
    unsigned long long xmax = 0ull;
    track_arg(xmax, x);
    bad |= arg_flags(xmax, false);   // no R^-1 here: no coalescence bit
    const double xa = fmin(Fr < 0.0 ? -x : x, 1.0);
    double cth;
    if (xa >= 0.0) {
        cth = cos_third_acos(xa);
    } else {
        // theta' = pi/3 - theta for a = -x': cos(theta') = C/2 + (sqrt3/2) S
        const double na = fmin(-xa, 1.0);
        const double v = fma(-na, na, 1.0);
        double C, S;
        third_angle(na, v * rsqrt_h(fmax(v, 1e-300)), C, S);
        cth = fma(0.5, C, kSqrt3Half * S);
    }
    // a NaN argument falls through both branches' arithmetic as NaN (the state is flagged)
    return (a.gh * a.inv_c) * ((2.0 / 3.0) * fma(k1 * r1, cth, fabs(Fr)));
}

// One quadrature node with all three eigenpairs, for the mixed form's FP64 band nodes:
// SA += w A dW (rows 1, 2; row 0 of A dW is dq at every node, and the weights sum to one, so the
// caller takes sum_k w_k dq = dq), SB += w |A| dW.
__device__ __forceinline__ void node_accumulate64(const Eig64 &E, double w, double dh, double dq,
                                                  double dz, double SA[3], double SB[3])
{
    const double Fr = E.Fr, c = E.c;
    const double mu1 = E.mu1, mu2 = E.mu2, mu3 = E.mu3;
    const double dqn = dq * E.inv_c;
    const double base = fma(-Fr, Fr, 1.0);   // (c^2 - u^2) / c^2
    // explicit A dW (row 0 is dq)
    const double A1n = fma(base, dh, fma(2.0 * Fr, dqn, dz));
    const double A2n = E.b * fma(-E.kFr, dh, dqn);
    // numerators of l_i . dW (non-dimensional)
    const double n1 = fma(fma(mu2, mu3, base), dh, fma(mu1, dqn, dz));
    const double n2 = fma(fma(mu3, mu1, base), dh, fma(mu2, dqn, dz));
    const double n3 = fma(fma(mu1, mu2, base), dh, fma(mu3, dqn, dz));
    // |mu_i| (l_i . dW) up to the common factor 1/P of the denominators 1/d_1 = g32/P,
    // 1/d_2 = -g31/P, 1/d_3 = g21/P, which enters once per row with w and c or c^2
    const double b1 = n1 * (fabs(mu1) * E.g32);
    const double b2 = -n2 * (fabs(mu2) * E.g31);
    const double b3 = n3 * (fabs(mu3) * E.g21);
    const double e1 = Fr - mu1, e2 = Fr - mu2, e3 = Fr - mu3;
    const double B0 = b1 + b2 + b3;
    const double B1 = fma(b1, mu1, fma(b2, mu2, b3 * mu3));
    const double B2 = fma(b1, fma(e1, e1, -1.0), fma(b2, fma(e2, e2, -1.0), b3 * fma(e3, e3, -1.0)));
    const double wc = w * c, wcc = wc * c;
    const double wcP = wc * E.inv_gp, wccP = wcc * E.inv_gp;
    SA[1] = fma(wcc, A1n, SA[1]);
    SA[2] = fma(wc, A2n, SA[2]);
    SB[0] = fma(wcP, B0, SB[0]);
    SB[1] = fma(wccP, B1, SB[1]);
    SB[2] = fma(wcP, B2, SB[2]);
}

// Paths of an FP64 quadrature node through D^-: with every lane's mu_3 >= 0 and ms >= 0 (flow
// towards +x below |Fr| of about 3 under weak transport), o = 2 and A^- dW takes the share
// min(mu_2, 0) of that eigenpair; with every lane's mu_3 < 0 and ms < 0 (the mirror case), o = 2
// and A^- dW = A dW less the share max(mu_2, 0); any other wave picks o per lane (o = 2 exactly
// when the signs of mu_3 and ms agree).
enum { NODE_PER_LANE = 0, NODE_UP = 1, NODE_DOWN = 2 };

// Sums over the nodes of an edge: S1, S2 = w A dW (rows 1, 2) over the nodes with mu_3 >= 0 and
// mu_3 < 0, Wt = sum of w over the latter (row 0 of A dW is dq at every node), SD = twice the
// projection terms of D^-.  Then D^- = (dq Wt, S2) + SD/2 and D^+ = (dq, S1 + S2) - D^-; the
// weights sum to one, so row 0 of S_A is dq.
struct NodeSums {
    double S1[3], S2[3], SD[3];   // rows 0-2 of the state; S1[0] and S2[0] are not used (dq, Wt)
    double Wt;
};

template <int PATH>
__device__ __forceinline__ void node_minus64(const Eig64 &E, double w, double dh, double dq, double dz,
                                             NodeSums &N)
{
    // One body for the three paths, so that a lane's arithmetic does not depend on the path its
    // wave takes: the uniform paths fix `up` and `two`, and their selects fold away.
    const bool up = PATH == NODE_UP ? true : PATH == NODE_DOWN ? false : E.mu3 >= 0.0;
    const bool two = PATH != NODE_PER_LANE ? true : up == (E.ms >= 0.0);
    const double Fr = E.Fr, c = E.c;
    const double dqn = dq * E.inv_c;
    const double base = fma(-Fr, Fr, 1.0);   // (c^2 - u^2) / c^2
    // explicit A dW (row 0 is dq)
    const double A1n = fma(base, dh, fma(2.0 * Fr, dqn, dz));
    const double A2n = E.b * fma(-E.kFr, dh, dqn);
    // eigenpair o, the other root x of the pair {1, 2}, and the numerator of 1/d_o over the
    // common factor 1/P (1/d_1 = g32/P, 1/d_2 = -g31/P)
    const double mo = two ? E.mu2 : E.mu1;
    const double mx = two ? E.mu1 : E.mu2;
    const double gd = two ? -E.g31 : E.g32;
    // twice mu_o's share of D^-: 2 min(mu_o, 0) = mu_o - |mu_o| when mu_3 >= 0, and
    // -2 max(mu_o, 0) = -mu_o - |mu_o| otherwise (exact: a doubling or zero); the sums SD hold
    // twice the projection terms
    const double to = (up ? mo : -mo) - fabs(mo);
    // (l_o . dW) d_o P, non-dimensional: l_o = [1 - Fr^2 + mu_3 mu_x, mu_o, 1] (rows dh, dq/c, dz)
    const double no = fma(fma(E.mu3, mx, base), dh, fma(mo, dqn, dz));
    const double bo = no * (to * gd);
    const double eo = Fr - mo;
    const double wc = w * c, wcc = wc * c;
    // w c to (l_o . dW), the weight of r_o = [1, c mu_o, (Fr - mu_o)^2 - 1] in 2 D^-
    const double pb = (wc * E.inv_gp) * bo;
    N.SD[0] += pb;
    N.SD[1] = fma(pb, c * mo, N.SD[1]);
    N.SD[2] = fma(pb, fma(eo, eo, -1.0), N.SD[2]);
    // w A dW into S1 (mu_3 >= 0) or S2 (mu_3 < 0, with its weight)
    const double a1 = fma(wcc, A1n, up ? N.S1[1] : N.S2[1]);
    const double a2 = fma(wc, A2n, up ? N.S1[2] : N.S2[2]);
    N.S1[1] = up ? a1 : N.S1[1];
    N.S1[2] = up ? a2 : N.S1[2];
    N.S2[1] = up ? N.S2[1] : a1;
    N.S2[2] = up ? N.S2[2] : a2;
    N.Wt = up ? N.Wt : N.Wt + w;
}

// D^- and D^+ of an edge from its node sums (D^- + D^+ = dq in row 0).
__device__ __forceinline__ void node_sums_to_fluct(const NodeSums &N, double dq, double Dm[3],
                                                   double Dp[3])
{
    Dm[0] = fma(0.5, N.SD[0], dq * N.Wt);
    Dp[0] = dq - Dm[0];
#pragma unroll
    for (int r = 1; r < 3; ++r) {
        Dm[r] = fma(0.5, N.SD[r], N.S2[r]);
        Dp[r] = fma(-0.5, N.SD[r], N.S1[r]);
    }
}

// DOT fluctuations of one edge, FP64 throughout.  Each node takes the path its wave allows
// (one branch per node for the whole wave).
template <int G, int CL>
__device__ __forceinline__ void fluct64(double hL, double qL, double zL, double hR, double qR,
                                        double zR, double g, const Closure &K, double Dm[3],
                                        double Dp[3], unsigned &bad)
{
    const double dh = hR - hL, dq = qR - qL, dz = zR - zL;
    NodeSums N = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, 0.0};
    unsigned long long xmax = 0ull;
    DSVE_UNROLL(DSVE_NODE_UNROLL)
    for (int k = 0; k < G; ++k) {
        const double s = Gauss<G>::s[k];
        Eig64 E;
        eig64<CL>(fma(s, dh, hL), fma(s, dq, qL), g, K, E, xmax);
        const double w = Gauss<G>::w[k];
        const unsigned long long act = __builtin_amdgcn_read_exec();
        const unsigned long long m3 = __builtin_amdgcn_ballot_w64(E.mu3 >= 0.0);
        const unsigned long long ms = __builtin_amdgcn_ballot_w64(E.ms >= 0.0);
        if ((m3 & ms) == act)
            node_minus64<NODE_UP>(E, w, dh, dq, dz, N);
        else if ((m3 | ms) == 0ull)
            node_minus64<NODE_DOWN>(E, w, dh, dq, dz, N);
        else
            node_minus64<NODE_PER_LANE>(E, w, dh, dq, dz, N);
    }
    bad |= arg_flags(xmax, true);
    node_sums_to_fluct(N, dq, Dm, Dp);
}

// ---------------------------------------------------------------------------
// Mixed form: FP32 eigenstructure and quadrature; a node whose arccos argument lies within
// kMixedFp64Band of +-1 (coalescing eigenvalues: Fr near +-1 with weak transport) is redone
// in FP64 from the FP64 path state.  The jumps dW and the free-surface jump dh + dz are formed
// in FP64 and rounded once; the h-row of sum_k w_k A dW is dq in FP64, so the water mass the
// update moves between cells telescopes to FP64 rounding.
struct EigF {
    float Fr, c, inv_c, b, kFr;
    float mu1, mu2, mu3;
    float g21, g31, g32;
    float inv_gp;
};

// Returns false when the node must be evaluated in FP64 (the FP32 argument only selects
// the band, a width of 1e-2 far wider than FP32 rounding; it never decides a result there).
template <int CL>
__device__ __forceinline__ bool eigf(float h, float q, float g, const Closure &K, EigF &E)
{
    const float gh = g * h;
    const float t = __builtin_amdgcn_rsqf(gh * h * h);
    const float Fr = q * t;
    const float inv_c = h * t;
    float k1, k2h, b, kFr;
    cubic_params<CL, float>(K, h, q, g, Fr, inv_c, k1, k2h, b, kFr);
    const float r1 = __builtin_amdgcn_rsqf(k1);
    const float r13 = r1 * r1 * r1;
    const float x = k2h * r13;
    if (!(fabsf(x) < 1.0f - kMixedFp64Band)) return false;
    const float v = fmaf(-x, x, 1.0f);
    const float inv_y = __builtin_amdgcn_rsqf(v);
    const float a = fabsf(x);
    float C, S;
    third_angle(a, v * inv_y, C, S);
    // the roots and gaps as in eig64
    const float m = (2.0f / 3.0f) * (k1 * r1);
    const float ms = copysignf(m, x);
    const float f = (2.0f / 3.0f) * Fr;
    const float r = (float)kSqrt3Half * S;
    E.Fr = Fr;
    E.c = gh * inv_c;
    E.inv_c = inv_c;
    E.b = b;
    E.kFr = kFr;
    // Q = C/2 - r = sin(arcsin(a)/3) cancels as a -> 0, where Q ~ a/3: there it comes from its
    // series a/3 + 4a^3/81 + O(a^5) (relative error below 1e-8 for a < 1/64), so that near still
    // water (Fr -> 0) the bed speed keeps its relative accuracy and is exactly 0 at Fr = 0
    const float Q = a < 0.015625f ? a * fmaf(a * a, 4.0f / 81.0f, 1.0f / 3.0f) : fmaf(0.5f, C, -r);
    E.mu1 = fmaf(ms, C, f);
    E.mu2 = fmaf(-ms, fmaf(0.5f, C, r), f);
    E.mu3 = fmaf(-ms, Q, f);
    E.g21 = -ms * fmaf(1.5f, C, r);
    E.g31 = -ms * (C + Q);
    E.g32 = (2.0f * ms) * r;
    E.inv_gp = (copysignf((float)kInvGapScale, x) * r13) * inv_y;
    return true;
}

// One FP32 node: SA += w A dW (rows 1, 2), SB += w |A| dW.  eta = dh + dz (rounded from FP64):
// (1 - Fr^2) dh + dz = eta - Fr^2 dh keeps a still free surface (eta = 0, Fr = 0) exact.
__device__ __forceinline__ void node_accumulatef(const EigF &E, float w, float dh, float dq, float eta,
                                                 float SA[3], float SB[3])
{
    const float Fr = E.Fr, c = E.c;
    const float mu1 = E.mu1, mu2 = E.mu2, mu3 = E.mu3;
    const float dqn = dq * E.inv_c;
    const float nF2 = -Fr * Fr;
    const float A1n = fmaf(nF2, dh, fmaf(2.0f * Fr, dqn, eta));
    const float A2n = E.b * fmaf(-E.kFr, dh, dqn);
    const float n1 = fmaf(fmaf(mu2, mu3, nF2), dh, fmaf(mu1, dqn, eta));
    const float n2 = fmaf(fmaf(mu3, mu1, nF2), dh, fmaf(mu2, dqn, eta));
    const float n3 = fmaf(fmaf(mu1, mu2, nF2), dh, fmaf(mu3, dqn, eta));
    const float b1 = n1 * (fabsf(mu1) * E.g32);
    const float b2 = -n2 * (fabsf(mu2) * E.g31);
    const float b3 = n3 * (fabsf(mu3) * E.g21);
    const float e1 = Fr - mu1, e2 = Fr - mu2, e3 = Fr - mu3;
    const float B0 = b1 + b2 + b3;
    const float B1 = fmaf(b1, mu1, fmaf(b2, mu2, b3 * mu3));
    const float B2 = fmaf(b1, fmaf(e1, e1, -1.0f), fmaf(b2, fmaf(e2, e2, -1.0f), b3 * fmaf(e3, e3, -1.0f)));
    const float wc = w * c, wcc = wc * c;
    const float wcP = wc * E.inv_gp, wccP = wcc * E.inv_gp;
    SA[1] = fmaf(wcc, A1n, SA[1]);
    SA[2] = fmaf(wc, A2n, SA[2]);
    SB[0] = fmaf(wcP, B0, SB[0]);
    SB[1] = fmaf(wccP, B1, SB[1]);
    SB[2] = fmaf(wcP, B2, SB[2]);
}

template <int G, int CL>
__device__ __forceinline__ void fluct_mixed(double hL, double qL, double zL, double hR, double qR,
                                            double zR, double g, const Closure &K, double Dm[3],
                                            double Dp[3], unsigned &bad)
{
    const double dh = hR - hL, dq = qR - qL, dz = zR - zL;
    const float dhf = (float)dh, dqf = (float)dq, etaf = (float)(dh + dz);
    const float hLf = (float)hL, qLf = (float)qL;
    const float gf = (float)g;
    // the node sums in FP32 (row 0 of S_A is dq, in FP64); a node in the band is evaluated in FP64
    // and its terms, which no longer carry the FP32 error near coalescence, are added rounded
    float SA[3] = {0.f, 0.f, 0.f}, SB[3] = {0.f, 0.f, 0.f};
    unsigned long long xmax = 0ull;
    DSVE_UNROLL(DSVE_NODE_UNROLL)
    for (int k = 0; k < G; ++k) {
        const float sf = (float)Gauss<G>::s[k];
        EigF E;
        if (eigf<CL>(fmaf(sf, dhf, hLf), fmaf(sf, dqf, qLf), gf, K, E)) {
            node_accumulatef(E, (float)Gauss<G>::w[k], dhf, dqf, etaf, SA, SB);
        } else {
            const double s = Gauss<G>::s[k];
            Eig64 E64;
            eig64<CL>(fma(s, dh, hL), fma(s, dq, qL), g, K, E64, xmax);
            double NA[3] = {0.0, 0.0, 0.0}, NB[3] = {0.0, 0.0, 0.0};
            node_accumulate64(E64, Gauss<G>::w[k], dh, dq, dz, NA, NB);
            SA[1] += (float)NA[1];
            SA[2] += (float)NA[2];
#pragma unroll
            for (int r = 0; r < 3; ++r) SB[r] += (float)NB[r];
        }
    }
    bad |= arg_flags(xmax, true);
    const double A[3] = {dq, (double)SA[1], (double)SA[2]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double B = (double)SB[r];
        Dm[r] = 0.5 * (A[r] - B);
        Dp[r] = 0.5 * (A[r] + B);
    }
}

// CFL speed in FP32 for the mixed form (the largest root at |Fr|, as speed64); the FP64 speed
// where the FP32 argument at |Fr| is negative, or within kMixedFp64Band of 1 as for the nodes of
// the fluctuation (so that complex roots and non-finite states, which the FP64 path reports, do
// not pass as FP32 rounding).
template <int CL>
__device__ __forceinline__ double speed_mixed(double h, double q, double g, const Closure &K,
                                              unsigned &bad)
{
    const float hf = (float)h, qf = (float)q, gf = (float)g;
    const float gh = gf * hf;
    const float t = __builtin_amdgcn_rsqf(gh * hf * hf);
    const float Fr = qf * t;
    const float inv_c = hf * t;
    float k1, k2h, b, kFr;
    cubic_params<CL, float>(K, hf, qf, gf, Fr, inv_c, k1, k2h, b, kFr);
    const float r1 = __builtin_amdgcn_rsqf(k1);
    const float x = k2h * (r1 * r1 * r1);
    const float xa = Fr < 0.0f ? -x : x;
    if (xa >= 0.0f && xa < 1.0f - kMixedFp64Band)
        return (double)((gh * inv_c) * ((2.0f / 3.0f) * fmaf(k1 * r1, cos_third_acos(xa), fabsf(Fr))));
    return speed64<CL>(h, q, g, K, bad);
}

// Friction source of the momentum equation (Sec. 2): -g h s_f with
// s_f = q |q| / (K_s^2 h^(10/3)), fric = 1 / K_s^2; evaluated in FP64 at the old cell state,
// h^(-7/3) as the seventh power of h^(-1/3).
__device__ __forceinline__ double friction_source(double h, double q, double g, double fric)
{
    const double r = rcbrt_h(h), r2 = r * r;
    return -g * (q * fabs(q)) * fric * ((r2 * r2) * (r2 * r));
}

}  // namespace dsve
