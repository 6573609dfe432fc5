// dsve_dot.hpp -- the original DOT solver (Sec. 3.1) on the GPU: |A| = R |Lambda| R^-1 from a
// generic numerical eigen-decomposition of the 3x3 flux matrix, the route the paper's A-DOT
// replaces with the closed form of Sec. 3.3.  It is the baseline the closed form is measured
// against (same quadrature, same update; only the eigenstructure differs).
//
// Per quadrature node, in FP64 and in registers (every array index is a compile-time constant):
//   1. A(W) of Eq. W&A_definition, the closure's derivatives entering its third row;
//   2. real Schur form A = Q T Q^T: a Givens rotation reduces A to Hessenberg form, then
//      implicit single-shift QR sweeps with the Wilkinson shift (the eigenvalue of the trailing
//      2x2 block closer to its last diagonal entry), deflating when a subdiagonal entry falls
//      below the unit roundoff times its diagonal neighbours; the last 2x2 block is brought to
//      triangular form by one rotation built from its eigenvector;
//   3. eigenvectors of T by back substitution (T - lambda_k) y_k = 0 with y_k[k] = 1, then
//      R = Q Y with columns scaled to unit length;
//   4. R^-1 by LU factorisation with partial pivoting and forward/back substitution of the
//      identity columns;
//   5. |A| = R |Lambda| R^-1 as a 3x3 matrix, then applied to dW.
// A complex eigenvalue pair (negative discriminant of a 2x2 block) or a sweep that has not
// converged after kMaxSweeps raises the non-hyperbolic flag.
#pragma once

#include "dsve_math.hpp"

namespace dsve {

constexpr int kMaxSweeps = 40;
constexpr double kUnitRoundoff = 1.1102230246251565e-16;   // 2^-53

struct Rot {
    double c, s;
};

// (c, s) with [c s; -s c] (x, y)^T = (r, 0)^T
__device__ __forceinline__ Rot givens(double x, double y)
{
    const double r2 = fma(x, x, y * y);
    if (r2 == 0.0) return Rot{1.0, 0.0};
    const double ir = rsqrt_h(r2);
    return Rot{x * ir, y * ir};
}

// H <- G H G^T on rows/columns (I, J); Q <- Q G^T.
template <int I, int J>
__device__ __forceinline__ void rotate(double H[3][3], double Q[3][3], Rot g)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = H[I][k], b = H[J][k];
        H[I][k] = fma(g.c, a, g.s * b);
        H[J][k] = fma(g.c, b, -g.s * a);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = H[k][I], b = H[k][J];
        H[k][I] = fma(g.c, a, g.s * b);
        H[k][J] = fma(g.c, b, -g.s * a);
        const double qa = Q[k][I], qb = Q[k][J];
        Q[k][I] = fma(g.c, qa, g.s * qb);
        Q[k][J] = fma(g.c, qb, -g.s * qa);
    }
}

__device__ __forceinline__ double sign1(double v) { return v < 0.0 ? -1.0 : 1.0; }

// The eigenvalue of [[a, b], [c, d]] closer to d (d itself if the pair is complex).
__device__ __forceinline__ double wilkinson_shift(double a, double b, double c, double d)
{
    const double p = 0.5 * (a - d);
    const double disc = fma(p, p, b * c);
    if (disc < 0.0) return d;
    const double den = p + sign1(p) * sqrt(disc);
    return den == 0.0 ? d : d - b * c / den;
}

// Triangularise the 2x2 diagonal block (P, P+1) of H by one rotation whose first column is an
// eigenvector of the block; false if the block's eigenvalues are complex.
template <int P>
__device__ __forceinline__ bool standardise_2x2(double H[3][3], double Q[3][3])
{
    const double a = H[P][P], b = H[P][P + 1], c = H[P + 1][P], d = H[P + 1][P + 1];
    if (c == 0.0) return true;
    const double p = 0.5 * (a - d);
    const double disc = fma(p, p, b * c);
    if (disc < 0.0) return false;
    const double z = p + sign1(p) * sqrt(disc);   // lambda - d for the eigenvalue put first
    rotate<P, P + 1>(H, Q, givens(z, c));
    H[P + 1][P] = 0.0;
    return true;
}

__device__ __forceinline__ bool negligible(double sub, double d0, double d1)
{
    return fabs(sub) <= kUnitRoundoff * (fabs(d0) + fabs(d1));
}

// Real Schur form A = Q T Q^T (T upper triangular, returned in H); false if an eigenvalue pair
// is complex or the sweeps did not converge.
__device__ __forceinline__ bool schur3(double H[3][3], double Q[3][3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? 1.0 : 0.0;
    // Hessenberg form: zero H[2][0] with a rotation of rows/columns 1, 2
    if (H[2][0] != 0.0) {
        rotate<1, 2>(H, Q, givens(H[1][0], H[2][0]));
        H[2][0] = 0.0;
    }
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        if (negligible(H[2][1], H[1][1], H[2][2])) {
            H[2][1] = 0.0;
            return standardise_2x2<0>(H, Q);
        }
        if (negligible(H[1][0], H[0][0], H[1][1])) {
            H[1][0] = 0.0;
            return standardise_2x2<1>(H, Q);
        }
        double mu = wilkinson_shift(H[1][1], H[1][2], H[2][1], H[2][2]);
        if (sweep == 10 || sweep == 20 || sweep == 30) mu = H[2][2] + 0.75 * fabs(H[2][1]);
        // implicit QR sweep: the first rotation from the first column of H - mu I, the second
        // chases the bulge it creates at (2, 0)
        rotate<0, 1>(H, Q, givens(H[0][0] - mu, H[1][0]));
        rotate<1, 2>(H, Q, givens(H[1][0], H[2][0]));
        H[2][0] = 0.0;
    }
    return false;
}

// x / d with d replaced by a tiny value of its sign when it underflows the scale (the
// perturbation of near-equal eigenvalues in triangular back substitution).
__device__ __forceinline__ double safe_div(double x, double d, double smin)
{
    const double dd = fabs(d) < smin ? (d < 0.0 ? -smin : smin) : d;
    return x / dd;
}

// Eigen-decomposition: eigenvalues lam[k] = T[k][k] and unit right eigenvectors R[:, k].
__device__ __forceinline__ bool eig3_numeric(const double A[3][3], double lam[3], double R[3][3])
{
    double T[3][3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) T[i][j] = A[i][j];
    const bool ok = schur3(T, Q);
    lam[0] = T[0][0];
    lam[1] = T[1][1];
    lam[2] = T[2][2];
    const double smin = kUnitRoundoff * fmax(fmax(fabs(lam[0]), fabs(lam[1])), fmax(fabs(lam[2]), 1e-300));
    // eigenvectors of T: y_k[k] = 1, y_k[j > k] = 0
    double Y[3][3];
    Y[0][0] = 1.0; Y[1][0] = 0.0; Y[2][0] = 0.0;
    Y[1][1] = 1.0; Y[2][1] = 0.0;
    Y[0][1] = safe_div(-T[0][1], T[0][0] - lam[1], smin);
    Y[2][2] = 1.0;
    Y[1][2] = safe_div(-T[1][2], T[1][1] - lam[2], smin);
    Y[0][2] = safe_div(-fma(T[0][1], Y[1][2], T[0][2]), T[0][0] - lam[2], smin);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            v0 = fma(Q[0][m], Y[m][k], v0);
            v1 = fma(Q[1][m], Y[m][k], v1);
            v2 = fma(Q[2][m], Y[m][k], v2);
        }
        const double in = rsqrt_h(fma(v0, v0, fma(v1, v1, v2 * v2)));
        R[0][k] = v0 * in;
        R[1][k] = v1 * in;
        R[2][k] = v2 * in;
    }
    return ok;
}

// Conditional swap of two rows of a 3x3 matrix and of a permutation (selects only).
template <int I, int J>
__device__ __forceinline__ void swap_rows_if(bool c, double M[3][3], int P[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = M[I][k], b = M[J][k];
        M[I][k] = c ? b : a;
        M[J][k] = c ? a : b;
    }
    const int pa = P[I], pb = P[J];
    P[I] = c ? pb : pa;
    P[J] = c ? pa : pb;
}

// Inverse of a 3x3 matrix by LU factorisation with partial pivoting (P R = L U), then
// L U X = P for the columns of the identity.
__device__ __forceinline__ void inverse3_lu(const double R[3][3], double Ri[3][3])
{
    double M[3][3];
    int P[3] = {0, 1, 2};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i][j] = R[i][j];
    // column 0: pivot among rows 0..2
    {
        const double a0 = fabs(M[0][0]), a1 = fabs(M[1][0]), a2 = fabs(M[2][0]);
        const bool s1 = a1 > a0 && a1 >= a2;
        const bool s2 = a2 > a0 && a2 > a1;
        swap_rows_if<0, 1>(s1, M, P);
        swap_rows_if<0, 2>(s2, M, P);
    }
    const double i00 = 1.0 / M[0][0];
    const double l10 = M[1][0] * i00, l20 = M[2][0] * i00;
    M[1][1] = fma(-l10, M[0][1], M[1][1]);
    M[1][2] = fma(-l10, M[0][2], M[1][2]);
    M[2][1] = fma(-l20, M[0][1], M[2][1]);
    M[2][2] = fma(-l20, M[0][2], M[2][2]);
    M[1][0] = l10;
    M[2][0] = l20;
    // column 1: pivot among rows 1..2 (the multipliers of column 0 move with their rows)
    swap_rows_if<1, 2>(fabs(M[2][1]) > fabs(M[1][1]), M, P);
    const double i11 = 1.0 / M[1][1];
    const double l21 = M[2][1] * i11;
    M[2][2] = fma(-l21, M[1][2], M[2][2]);
    const double i22 = 1.0 / M[2][2];
    // solve for each column e_c of the identity: row i of P e_c is (P[i] == c)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double b0 = P[0] == c ? 1.0 : 0.0;
        const double b1 = P[1] == c ? 1.0 : 0.0;
        const double b2 = P[2] == c ? 1.0 : 0.0;
        const double y0 = b0;
        const double y1 = fma(-M[1][0], y0, b1);
        const double y2 = fma(-l21, y1, fma(-M[2][0], y0, b2));
        const double x2 = y2 * i22;
        const double x1 = fma(-M[1][2], x2, y1) * i11;
        const double x0 = fma(-M[0][2], x2, fma(-M[0][1], x1, y0)) * i00;
        Ri[0][c] = x0;
        Ri[1][c] = x1;
        Ri[2][c] = x2;
    }
}

// Flux matrix (Eq. W&A_definition) at (h, q): the closure enters its third row through
// b = xi dq_s/dq and xi dq_s/dh = -kappa b u (the closure forms of dsve_math.hpp).
template <int CL>
__device__ __forceinline__ void flux_matrix(double h, double q, double g, const Closure &K,
                                            double A[3][3])
{
    const double gh = g * h;
    const double t = rsqrt_h(gh * h * h);
    const double Fr = q * t;
    const double inv_c = h * t;
    double k1, k2h, b, kFr;
    cubic_params<CL, double>(K, h, q, g, Fr, inv_c, k1, k2h, b, kFr);
    const double c = gh * inv_c;
    const double u = Fr * c;
    A[0][0] = 0.0; A[0][1] = 1.0; A[0][2] = 0.0;
    A[1][0] = fma(-u, u, gh); A[1][1] = 2.0 * u; A[1][2] = gh;
    A[2][0] = -kFr * c * b; A[2][1] = b; A[2][2] = 0.0;
}

// Largest |lambda| of a state by the numerical route (eigenvalues of the Schur form).
template <int CL>
__device__ __forceinline__ double speed_dot(double h, double q, double g, const Closure &K, unsigned &bad)
{
    double A[3][3], Q[3][3];
    flux_matrix<CL>(h, q, g, K, A);
    bad |= schur3(A, Q) ? 0u : kFlagComplex;
    return fmax(fmax(fabs(A[0][0]), fabs(A[1][1])), fabs(A[2][2]));
}

// DOT fluctuations of one edge with the numerical eigen-decomposition at every node.
template <int G, int CL>
__device__ __forceinline__ void fluct_dot(double hL, double qL, double zL, double hR, double qR,
                                          double zR, double g, const Closure &K, double Dm[3],
                                          double Dp[3], unsigned &bad)
{
    const double dW[3] = {hR - hL, qR - qL, zR - zL};
    double SA[3] = {0.0, 0.0, 0.0}, SB[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < G; ++k) {
        const double s = Gauss<G>::s[k], w = Gauss<G>::w[k];
        double A[3][3], lam[3], R[3][3], Ri[3][3];
        flux_matrix<CL>(fma(s, dW[0], hL), fma(s, dW[1], qL), g, K, A);
        bad |= eig3_numeric(A, lam, R) ? 0u : kFlagComplex;
        inverse3_lu(R, Ri);
        // |A| = R |Lambda| R^-1 (Eq. asbA), then the node's contributions to sum_k w_k (A, |A|) dW
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ad = 0.0, aad = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double absA = 0.0;
#pragma unroll
                for (int m = 0; m < 3; ++m) absA = fma(R[i][m] * fabs(lam[m]), Ri[m][j], absA);
                ad = fma(A[i][j], dW[j], ad);
                aad = fma(absA, dW[j], aad);
            }
            SA[i] = fma(w, ad, SA[i]);
            SB[i] = fma(w, aad, SB[i]);
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Dm[r] = 0.5 * (SA[r] - SB[r]);
        Dp[r] = 0.5 * (SA[r] + SB[r]);
    }
}

}  // namespace dsve
