// dsve_math.hpp -- per-node and per-edge arithmetic of the A-DOT hot path (device code).
//
// For one state W = (h, q, z) on the segment path (Sec. 3.1, Eq. path):
//   u = q/h, c^2 = g h, Fr = u/c;
//   Grass closure (Sec. 2 Eq. Grass; Sec. 3.3 step 1):
//     b = xi dq_s/dq = 3 xi A_g u^2/h,  a = xi dq_s/dh = -3 xi A_g u^3/h = -b u
//   cubic parameters (Sec. 3.3, Eqs. parameters, parameters_bis):
//     k1 = 3 + Fr^2 + 3b,  k2 = -2 Fr^3 + 18 Fr (1 + b) + 27 a / c,  x = k2 / sqrt(4 k1^3),
//     phi = arccos(x)
//   eigenvalues (Eq. lambda), theta = phi/3, m = (2/3) c sqrt(k1), f = (2/3) u:
//     lambda_{1,2} = f - m cos(theta -+ pi/3),  lambda_3 = f + m cos(theta)
//   where cos(theta -+ pi/3) = cos(theta)/2 +- (sqrt 3/2) sin(theta): one (cos, sin) pair
//   serves all three roots, and the gaps follow without cancellation:
//     lambda_2 - lambda_1 = sqrt3 m sin(theta),
//     lambda_3 - lambda_1 = m (3/2 cos(theta) + sqrt3/2 sin(theta)),
//     lambda_3 - lambda_2 = m (3/2 cos(theta) - sqrt3/2 sin(theta));
//   right eigenvectors r_m = [1, lambda_m, (u - lambda_m)^2/c^2 - 1]       (Eq. RR)
//   left eigenvectors  l_i = [c^2 - u^2 + l_j l_k, 2u - l_j - l_k, c^2] / ((l_i - l_j)(l_i - l_k)),
//                      (i, j, k) cyclic                                     (Eqs. RR-1, circPerm)
//   with the three denominators taken from the gap products (one reciprocal for all three).
// The fluctuation (Sec. 3.1, Eq. DOTjumpN) is accumulated as
//   S_A = sum_k w_k A(Psi_k) dW   with the explicit flux matrix (Eq. W&A_definition),
//   S_B = sum_k w_k |A(Psi_k)| dW  with |A| dW = sum_m |lambda_m| (l_m . dW) r_m   (Eqs. asbA, ExAbsA),
//   D^- = (S_A - S_B)/2,  D^+ = (S_A + S_B)/2,
// i.e. |A| is applied to dW as R (|Lambda| (R^-1 dW)) instead of being formed as a 3x3 matrix.
//
// Arithmetic kernels used below (own implementations, published methods):
//   rcp_nr / rsqrt_nr: hardware reciprocal / reciprocal-square-root estimate refined by two
//     Newton-Raphson steps (quadratic convergence).
//   trisect: cos(theta), sin(theta) with theta = arccos(x)/3.  An FP32 estimate of theta
//     (arccos, then sine/cosine) gives a point on the unit circle, renormalised in FP64; the
//     residual angle follows from the complex identity  Im(w conj(z)^3) = sin(phi - 3 theta0),
//     w = x + i sqrt(1-x^2), z = cos(theta0) + i sin(theta0), and a rotation by that residual/3
//     (second-order sine/cosine of a small angle) removes it.  Each correction leaves an
//     error of order (residual)^3.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dsve_internal.hpp"

namespace dsve {

constexpr double kSqrt3 = 1.73205080756887729352744634150587237;
constexpr double kSqrt3Half = 0.86602540378443864676372317075293618;
constexpr double kAcosTol = 1e-12;      // tolerance on |arccos argument| - 1 before flagging
constexpr double kTrisectTwoRounds = 0.984;   // |x| above which the FP32 estimate gets two rounds
constexpr float kMixedFp64Band = 1e-3f;       // mixed form: 1 - |x| below this -> FP64 node

// Clamp to [-1, 1] keeping NaN (a NaN argument must stay visible downstream).
__device__ __forceinline__ double clamp_unit(double x)
{
    return (x > 1.0) ? 1.0 : ((x < -1.0) ? -1.0 : x);
}
__device__ __forceinline__ float clamp_unitf(float x)
{
    return (x > 1.0f) ? 1.0f : ((x < -1.0f) ? -1.0f : x);
}

__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double rsqrt_nr(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    // r <- r (1 + e/2), e = 1 - x r^2
    double e = fma(-x * r, r, 1.0);
    r = fma(0.5 * r, e, r);
    e = fma(-x * r, r, 1.0);
    return fma(0.5 * r, e, r);
}

// One correction of (c, s) ~ (cos theta, sin theta) towards 3 theta = phi, cos(phi) = x,
// sin(phi) = y >= 0; (c, s) must be unit length to rounding.
__device__ __forceinline__ void trisect_correct(double x, double y, double &c, double &s)
{
    const double c2 = c * c, s2 = s * s;
    const double C3 = c * fma(4.0, c2, -3.0);      // cos(3 theta0)
    const double S3 = s * fma(-4.0, s2, 3.0);      // sin(3 theta0)
    const double res = fma(y, C3, -x * S3);        // sin(phi - 3 theta0)
    const double d = res * (1.0 / 3.0);
    const double cd = fma(-0.5 * d, d, 1.0);
    const double cn = fma(c, cd, -s * d);
    const double sn = fma(s, cd, c * d);
    c = cn;
    s = sn;
}

// (cos theta, sin theta), theta = arccos(x) / 3, for x in [-1, 1] (NaN propagates).
__device__ __forceinline__ void trisect(double x, double &c, double &s)
{
    const double v = (1.0 - x) * (1.0 + x);
    const double y = (v > 0.0) ? v * rsqrt_nr(v) : (v == 0.0 ? 0.0 : v);   // sin(phi)
    const float th0 = acosf((float)x) * (1.0f / 3.0f);
    const double c0 = (double)__cosf(th0), s0 = (double)__sinf(th0);
    // renormalise: r = 1 / sqrt(c0^2 + s0^2) to second order in e = c0^2 + s0^2 - 1 (|e| ~ 1e-7)
    const double e = fma(c0, c0, fma(s0, s0, -1.0));
    const double nr = fma(e, fma(e, 0.375, -0.5), 1.0);
    c = c0 * nr;
    s = s0 * nr;
    trisect_correct(x, y, c, s);
    if (fabs(x) > kTrisectTwoRounds) trisect_correct(x, y, c, s);
}

// ---------------------------------------------------------------------------
// FP64 eigenvalues at one state, with what the eigenvectors need.
struct Eig64 {
    double u, c2, inv_c2, a, b;
    double l1, l2, l3;
    double g21, g31, g32;   // lambda_2 - lambda_1, lambda_3 - lambda_1, lambda_3 - lambda_2
};

__device__ __forceinline__ void eig64(double h, double q, double g, double kq, Eig64 &E, bool &bad)
{
    const double inv_h = rcp_nr(h);
    const double u = q * inv_h;
    const double c2 = g * h;
    const double inv_c = rsqrt_nr(c2);
    const double c = c2 * inv_c;
    const double Fr = u * inv_c;
    const double b = kq * u * u * inv_h;   // xi dq_s/dq
    const double a = -b * u;               // xi dq_s/dh
    const double Fr2 = Fr * Fr;
    const double k1 = 3.0 + Fr2 + 3.0 * b;
    const double k2 = Fr * (18.0 * (1.0 + b) - 2.0 * Fr2) + 27.0 * a * inv_c;
    const double r1 = rsqrt_nr(k1);
    const double s1 = k1 * r1;                       // sqrt(k1)
    double x = 0.5 * k2 * (r1 * r1 * r1);            // k2 / sqrt(4 k1^3)
    bad |= isfinite(k1) && isfinite(k2) && (!(k1 > 0.0) || fabs(x) > 1.0 + kAcosTol);
    x = clamp_unit(x);
    double cs, sn;
    trisect(x, cs, sn);
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
    E.g21 = m * (kSqrt3 * sn);
    E.g31 = m * (3.0 * p + r);
    E.g32 = m * (3.0 * p - r);
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
    const double tu = 2.0 * u;
    const double c2dz = c2 * dz;
    const double A1 = base * dh + tu * dq + c2dz;
    const double A2 = E.a * dh + E.b * dq;
    // 1/d_i from the gap products: d1 = g21 g31, d2 = -g21 g32, d3 = g31 g32
    const double invP = rcp_nr(E.g21 * E.g31 * E.g32);
    const double id1 = E.g32 * invP, id2 = -E.g31 * invP, id3 = E.g21 * invP;
    // (R^-1 dW)_i = l_i . dW, scaled by w |lambda_i|
    const double al1 = ((base + l2 * l3) * dh + (tu - l2 - l3) * dq + c2dz) * id1;
    const double al2 = ((base + l3 * l1) * dh + (tu - l3 - l1) * dq + c2dz) * id2;
    const double al3 = ((base + l1 * l2) * dh + (tu - l1 - l2) * dq + c2dz) * id3;
    const double b1 = w * fabs(l1) * al1, b2 = w * fabs(l2) * al2, b3 = w * fabs(l3) * al3;
    const double e1 = u - l1, e2 = u - l2, e3 = u - l3;
    const double r1 = e1 * e1 * E.inv_c2 - 1.0;
    const double r2 = e2 * e2 * E.inv_c2 - 1.0;
    const double r3 = e3 * e3 * E.inv_c2 - 1.0;
    SA[0] += w * dq;
    SA[1] += w * A1;
    SA[2] += w * A2;
    SB[0] += b1 + b2 + b3;
    SB[1] += b1 * l1 + b2 * l2 + b3 * l3;
    SB[2] += b1 * r1 + b2 * r2 + b3 * r3;
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

// ---------------------------------------------------------------------------
// Mixed form: FP32 eigenstructure and quadrature; a node whose arccos argument lies within
// kMixedFp64Band of +-1 (coalescing eigenvalues: Fr near +-1 with weak transport) is redone
// in FP64 from the FP64 path state.  The jumps dW are formed in FP64 and rounded once.
struct EigF {
    float u, c2, inv_c2, a, b;
    float l1, l2, l3;
    float g21, g31, g32;
};

// Returns false when the node must be evaluated in FP64.
__device__ __forceinline__ bool eigf(float h, float q, float g, float kq, EigF &E, bool &bad)
{
    const float inv_h = __builtin_amdgcn_rcpf(h);
    const float u = q * inv_h;
    const float c2 = g * h;
    const float inv_c = __builtin_amdgcn_rsqf(c2);
    const float c = c2 * inv_c;
    const float Fr = u * inv_c;
    const float b = kq * u * u * inv_h;
    const float a = -b * u;
    const float Fr2 = Fr * Fr;
    const float k1 = 3.0f + Fr2 + 3.0f * b;
    const float k2 = Fr * (18.0f * (1.0f + b) - 2.0f * Fr2) + 27.0f * a * inv_c;
    const float r1 = __builtin_amdgcn_rsqf(k1);
    const float s1 = k1 * r1;
    float x = 0.5f * k2 * (r1 * r1 * r1);
    // the FP32 argument decides only whether to switch to FP64 (a band of width 1e-3 around
    // +-1, far wider than FP32 rounding), never the result near the band
    if (!(fabsf(x) < 1.0f - kMixedFp64Band)) return false;
    (void)bad;
    x = clamp_unitf(x);
    const float th = acosf(x) * (1.0f / 3.0f);
    const float cs = __cosf(th), sn = __sinf(th);
    const float m = (2.0f / 3.0f) * s1 * c;
    const float f = (2.0f / 3.0f) * u;
    const float p = 0.5f * cs, r = (float)kSqrt3Half * sn;
    E.u = u;
    E.c2 = c2;
    E.inv_c2 = inv_c * inv_c;
    E.a = a;
    E.b = b;
    E.l1 = f - m * (p + r);
    E.l2 = f - m * (p - r);
    E.l3 = f + m * cs;
    E.g21 = m * ((float)kSqrt3 * sn);
    E.g31 = m * (3.0f * p + r);
    E.g32 = m * (3.0f * p - r);
    return true;
}

__device__ __forceinline__ void node_accumulatef(const EigF &E, float w, float dh, float dq, float dz,
                                                 float SA[3], float SB[3])
{
    const float u = E.u, c2 = E.c2;
    const float l1 = E.l1, l2 = E.l2, l3 = E.l3;
    const float base = c2 - u * u;
    const float tu = 2.0f * u;
    const float c2dz = c2 * dz;
    const float A1 = base * dh + tu * dq + c2dz;
    const float A2 = E.a * dh + E.b * dq;
    const float invP = __builtin_amdgcn_rcpf(E.g21 * E.g31 * E.g32);
    const float id1 = E.g32 * invP, id2 = -E.g31 * invP, id3 = E.g21 * invP;
    const float al1 = ((base + l2 * l3) * dh + (tu - l2 - l3) * dq + c2dz) * id1;
    const float al2 = ((base + l3 * l1) * dh + (tu - l3 - l1) * dq + c2dz) * id2;
    const float al3 = ((base + l1 * l2) * dh + (tu - l1 - l2) * dq + c2dz) * id3;
    const float b1 = w * fabsf(l1) * al1, b2 = w * fabsf(l2) * al2, b3 = w * fabsf(l3) * al3;
    const float e1 = u - l1, e2 = u - l2, e3 = u - l3;
    const float r1 = e1 * e1 * E.inv_c2 - 1.0f;
    const float r2 = e2 * e2 * E.inv_c2 - 1.0f;
    const float r3 = e3 * e3 * E.inv_c2 - 1.0f;
    SA[0] += w * dq;
    SA[1] += w * A1;
    SA[2] += w * A2;
    SB[0] += b1 + b2 + b3;
    SB[1] += b1 * l1 + b2 * l2 + b3 * l3;
    SB[2] += b1 * r1 + b2 * r2 + b3 * r3;
}

template <int G>
__device__ __forceinline__ void fluct_mixed(double hL, double qL, double zL, double hR, double qR,
                                            double zR, double g, double kq, const GaussRule &rule,
                                            double Dm[3], double Dp[3], bool &bad)
{
    const double dh = hR - hL, dq = qR - qL, dz = zR - zL;
    const float dhf = (float)dh, dqf = (float)dq, dzf = (float)dz;
    const float gf = (float)g, kqf = (float)kq;
    float SA[3] = {0.f, 0.f, 0.f}, SB[3] = {0.f, 0.f, 0.f};
    double SA64[3] = {0.0, 0.0, 0.0}, SB64[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const double s = rule.s[k];
        const double h = hL + s * dh, q = qL + s * dq;
        EigF E;
        if (eigf((float)h, (float)q, gf, kqf, E, bad)) {
            node_accumulatef(E, (float)rule.w[k], dhf, dqf, dzf, SA, SB);
        } else {
            Eig64 E64;
            eig64(h, q, g, kq, E64, bad);
            node_accumulate64(E64, rule.w[k], dh, dq, dz, SA64, SB64);
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double A = (double)SA[r] + SA64[r], B = (double)SB[r] + SB64[r];
        Dm[r] = 0.5 * (A - B);
        Dp[r] = 0.5 * (A + B);
    }
}

__device__ __forceinline__ double speed_mixed(double h, double q, double g, double kq, bool &bad)
{
    EigF E;
    if (eigf((float)h, (float)q, (float)g, (float)kq, E, bad))
        return (double)fmaxf(fmaxf(fabsf(E.l1), fabsf(E.l2)), fabsf(E.l3));
    return speed64(h, q, g, kq, bad);
}

}  // namespace dsve
