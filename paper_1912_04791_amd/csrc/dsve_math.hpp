// dsve_math.hpp -- per-node and per-edge arithmetic of the A-DOT hot path (device code).
//
// For one state W = (h, q, z) on the segment path (Sec. 3.1, Eq. path):
//   u = q/h, c^2 = g h, Fr = u/c;
//   Grass closure (Sec. 2 Eq. Grass; Sec. 3.3 step 1):
//     b = xi dq_s/dq = 3 xi A_g u^2/h,  a = xi dq_s/dh = -3 xi A_g u^3/h = -b u
//   cubic parameters (Sec. 3.3, Eqs. parameters, parameters_bis):
//     k1 = 3 + Fr^2 + 3b,  k2 = -2 Fr^3 + 18 Fr (1 + b) + 27 a / c,
//     phi = arccos(k2 / sqrt(4 k1^3))
//   eigenvalues (Eq. lambda), theta = phi/3:
//     lambda_{1,2} = c (2/3 Fr - 2/3 sqrt(k1) cos(theta -+ pi/3)),  lambda_3 = c (2/3 Fr + 2/3 sqrt(k1) cos theta)
//   with cos(theta -+ pi/3) = cos(theta)/2 +- (sqrt(3)/2) sin(theta), so one sine/cosine pair serves
//   all three roots;
//   right eigenvectors r_m = [1, lambda_m, (u - lambda_m)^2/c^2 - 1]       (Eq. RR)
//   left eigenvectors  l_i = [c^2 - u^2 + l_j l_k, 2u - l_j - l_k, c^2] / ((l_i - l_j)(l_i - l_k))
//                      with (i, j, k) cyclic                               (Eqs. RR-1, circPerm)
// The fluctuation (Sec. 3.1, Eq. DOTjumpN) is accumulated as
//   S_A = sum_k w_k A(Psi_k) dW   with the explicit flux matrix (Eq. W&A_definition),
//   S_B = sum_k w_k |A(Psi_k)| dW  with |A| dW = sum_m |lambda_m| (l_m . dW) r_m   (Eqs. asbA, ExAbsA),
//   D^- = (S_A - S_B)/2,  D^+ = (S_A + S_B)/2,
// i.e. |A| is applied to dW as R (|Lambda| (R^-1 dW)) instead of being formed as a 3x3
// matrix: the same product, associated differently (27 multiplies instead of 54 per node).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dsve_internal.hpp"

namespace dsve {

constexpr double kSqrt3Half = 0.86602540378443864676372317075293618;   // sqrt(3)/2
constexpr double kAcosTol = 1e-12;   // tolerance on |arccos argument| - 1 before flagging

// Clamp to [-1, 1] keeping NaN (a NaN argument must stay visible downstream).
__device__ __forceinline__ double clamp_unit(double x)
{
    return (x > 1.0) ? 1.0 : ((x < -1.0) ? -1.0 : x);
}

// ---------------------------------------------------------------------------
// FP64 eigenvalues at one state.  Returns u, c^2, a, b and the three roots.
struct Eig64 {
    double u, c2, inv_c2, a, b;
    double l1, l2, l3;
};

__device__ __forceinline__ void eig64(double h, double q, double g, double kq, Eig64 &E, bool &bad)
{
    const double inv_h = 1.0 / h;
    const double u = q * inv_h;
    const double c2 = g * h;
    const double c = sqrt(c2);
    const double inv_c = 1.0 / c;
    const double Fr = u * inv_c;
    const double b = kq * u * u * inv_h;   // xi dq_s/dq
    const double a = -b * u;               // xi dq_s/dh
    const double k1 = 3.0 + Fr * Fr + 3.0 * b;
    const double k2 = Fr * (18.0 * (1.0 + b) - 2.0 * Fr * Fr) + 27.0 * a * inv_c;
    const double s1 = sqrt(k1);
    double x = k2 / (2.0 * k1 * s1);
    bad |= isfinite(k1) && isfinite(k2) && (!(k1 > 0.0) || fabs(x) > 1.0 + kAcosTol);
    x = clamp_unit(x);
    const double th = acos(x) * (1.0 / 3.0);
    double sn, cs;
    sincos(th, &sn, &cs);
    const double m = (2.0 / 3.0) * s1 * c;
    const double f = (2.0 / 3.0) * u;
    const double p = 0.5 * cs, r = kSqrt3Half * sn;
    E.u = u;
    E.c2 = c2;
    E.inv_c2 = inv_c * inv_c;
    E.a = a;
    E.b = b;
    E.l1 = f - m * (p + r);
    E.l2 = f - m * (p - r);
    E.l3 = f + m * cs;
}

// Largest characteristic speed max_m |lambda_m| of a cell state (the CFL quantity).
__device__ __forceinline__ double speed64(double h, double q, double g, double kq, bool &bad)
{
    Eig64 E;
    eig64(h, q, g, kq, E, bad);
    return fmax(fmax(fabs(E.l1), fabs(E.l2)), fabs(E.l3));
}

// Accumulate one quadrature node: SA += w A dW, SB += w |A| dW.
__device__ __forceinline__ void node_accumulate64(const Eig64 &E, double w, double dh, double dq,
                                                  double dz, double SA[3], double SB[3])
{
    const double u = E.u, c2 = E.c2;
    const double l1 = E.l1, l2 = E.l2, l3 = E.l3;
    // A dW with the explicit flux matrix; row 0 is dq
    const double base = c2 - u * u;
    const double A1 = base * dh + 2.0 * u * dq + c2 * dz;
    const double A2 = E.a * dh + E.b * dq;
    // (R^-1 dW)_i = l_i . dW
    const double tu = 2.0 * u;
    const double c2dz = c2 * dz;
    const double d1 = (l1 - l2) * (l1 - l3);
    const double d2 = (l2 - l3) * (l2 - l1);
    const double d3 = (l3 - l1) * (l3 - l2);
    const double al1 = ((base + l2 * l3) * dh + (tu - l2 - l3) * dq + c2dz) / d1;
    const double al2 = ((base + l3 * l1) * dh + (tu - l3 - l1) * dq + c2dz) / d2;
    const double al3 = ((base + l1 * l2) * dh + (tu - l1 - l2) * dq + c2dz) / d3;
    // R |Lambda| (R^-1 dW)
    const double b1 = fabs(l1) * al1, b2 = fabs(l2) * al2, b3 = fabs(l3) * al3;
    const double e1 = u - l1, e2 = u - l2, e3 = u - l3;
    const double r1 = e1 * e1 * E.inv_c2 - 1.0;
    const double r2 = e2 * e2 * E.inv_c2 - 1.0;
    const double r3 = e3 * e3 * E.inv_c2 - 1.0;
    SA[0] += w * dq;
    SA[1] += w * A1;
    SA[2] += w * A2;
    SB[0] += w * (b1 + b2 + b3);
    SB[1] += w * (b1 * l1 + b2 * l2 + b3 * l3);
    SB[2] += w * (b1 * r1 + b2 * r2 + b3 * r3);
}

// DOT fluctuations of one edge, FP64 throughout.
template <int G>
__device__ __forceinline__ void fluct64(double hL, double qL, double zL, double hR, double qR,
                                        double zR, double g, double kq, const GaussRule &rule,
                                        double Dm[3], double Dp[3], bool &bad)
{
    const double dh = hR - hL, dq = qR - qL, dz = zR - zL;
    double SA[3] = {0.0, 0.0, 0.0}, SB[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const double s = rule.s[k];
        Eig64 E;
        eig64(hL + s * dh, qL + s * dq, g, kq, E, bad);
        node_accumulate64(E, rule.w[k], dh, dq, dz, SA, SB);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Dm[r] = 0.5 * (SA[r] - SB[r]);
        Dp[r] = 0.5 * (SA[r] + SB[r]);
    }
}

}  // namespace dsve
