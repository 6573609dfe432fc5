"""Host model of the mixed form's FP32 node arithmetic (test infrastructure).

Evaluates, with numpy, the FP32 eigenstructure and node accumulation the mixed-form kernels
run at each quadrature node (the closed form of Sec. 3.3 in Froude-number variables, the
matrix-vector |A| dW of Eqs. asbA, ExAbsA), so that the rounding error of FP32 near coalescing
eigenvalues can be studied on the CPU: with every node in FP32 ("band off"), which no kernel
runs, and with the nodes whose arccos argument lies within the FP64 band taken from the FP64
oracle instead.

Rounding model: every FP32 operation rounds once, an FMA is the exact product (a float64
product of two floats is exact) plus the addend rounded to FP32 (two roundings where the device
rounds once, a difference of at most one ulp in rare cases); the reciprocal square root and
reciprocal are rounded correctly, where the device approximates them to about one ulp.  The model's FP32 error therefore slightly understates the device's; the band-on
figures of the tests come from the device itself.
"""
from __future__ import annotations

import os
import re

import numpy as np

f32 = np.float32


def _r(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fmaf(a, b, c):
    return _r(np.float64(1) * a.astype(np.float64) * b.astype(np.float64) + np.asarray(c, dtype=np.float64))


def mul(a, b):
    return _r(np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64))


def add(a, b):
    return _r(np.asarray(a, dtype=np.float64) + np.asarray(b, dtype=np.float64))


def rsq(x):
    return _r(1.0 / np.sqrt(np.asarray(x, dtype=np.float64)))


def rcp(x):
    return _r(1.0 / np.asarray(x, dtype=np.float64))


def _cos_third_acos_coeffs():
    """Horner coefficients (highest degree first) of the kernels' FP32 cos(arccos(a)/3)."""
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_1912_04791_amd", "csrc",
                            "dsve_math.hpp")).read()
    body = src[src.index("float cos_third_acos(float a)"):]
    body = body[:body.index("\n}\n")]
    lit = r"(-?\d+(?:\.\d+)?(?:e-?\d+)?)f?"
    first = float(re.search(r"p = " + lit + ";", body).group(1))
    return [first] + [float(v) for v in re.findall(r"fmaf?\(p, t, " + lit + r"\)", body)]


_CT = _cos_third_acos_coeffs()


def cos_third_acos_f32(a):
    """cos(arccos(a)/3), a in [0, 1]: the degree-7 polynomial in 1 - a, in FP32."""
    t = add(f32(1), -a)
    p = np.full_like(t, f32(_CT[0]))
    for c in _CT[1:]:
        p = fmaf(p, t, f32(c))
    return p


def node_terms(h, q, dh, dq, eta, w, g, kqg, band):
    """One quadrature node of the mixed form (Grass law in closed form, kappa = 1): returns the
    node's contributions w A dW (rows 1, 2) and w |A| dW (rows 0..2) in FP32, and a mask of the
    nodes whose arccos argument lies within `band` of +-1 (band = 0: none)."""
    h, q, dh, dq, eta = (_r(v) for v in (h, q, dh, dq, eta))
    g, w = f32(g), f32(w)
    K1, K2 = f32(1.0 + 3.0 * kqg), f32(2.0 + 9.0 * kqg)
    gh = mul(g, h)
    t = _r(1.0 / np.sqrt(mul(mul(gh, h), h).astype(np.float64)))
    Fr = mul(q, t)
    inv_c = mul(h, t)
    Fr2 = mul(Fr, Fr)
    b = mul(f32(kqg), Fr2)
    k1 = fmaf(Fr2, np.full_like(Fr2, K1), f32(3))
    k2 = mul(Fr, fmaf(-Fr2, np.full_like(Fr2, K2), f32(18)))
    r1 = rsq(k1)
    r13 = mul(mul(r1, r1), r1)
    x = mul(mul(f32(0.5), k2), r13)
    inband = ~(np.abs(x) < f32(1) - f32(band)) if band > 0 else np.zeros(x.shape, dtype=bool)
    xc = np.clip(x, f32(-1), f32(1))
    v = np.maximum(fmaf(-xc, xc, f32(1)), f32(1e-30))
    inv_y = rsq(v)
    C = cos_third_acos_f32(np.abs(xc))
    S = mul(mul(v, inv_y), rcp(fmaf(mul(f32(4), C), C, f32(-1))))
    m = mul(f32(2.0 / 3.0), mul(k1, r1))
    ms = np.copysign(m, xc).astype(np.float32)
    f = mul(f32(2.0 / 3.0), Fr)
    rr = mul(f32(0.86602540378443864676), S)
    c = mul(gh, inv_c)
    # the roots sign(x) m {C, -P, -Q} about f, unsorted (the sums are symmetric in the labels)
    mu1 = fmaf(ms, C, f)
    mu2 = fmaf(-ms, fmaf(np.full_like(C, f32(0.5)), C, rr), f)
    aa = np.abs(xc)
    ser = mul(aa, fmaf(mul(aa, aa), np.full_like(aa, f32(4 / 81)), f32(1 / 3)))
    Q = np.where(aa < f32(1 / 64), ser, fmaf(np.full_like(C, f32(0.5)), C, -rr)).astype(np.float32)
    mu3 = fmaf(-ms, Q, f)
    g21 = mul(-ms, fmaf(np.full_like(C, f32(1.5)), C, rr))
    g31 = mul(-ms, add(C, Q))
    g32 = mul(mul(f32(2), ms), rr)
    inv_gp = mul(mul(np.copysign(f32(2.59807621135331594029), xc).astype(np.float32), r13), inv_y)
    dqn = mul(dq, inv_c)
    nF2 = -Fr2
    A1n = fmaf(nF2, dh, fmaf(mul(f32(2), Fr), dqn, eta))
    A2n = mul(b, fmaf(-Fr, dh, dqn))
    n1 = fmaf(fmaf(mu2, mu3, nF2), dh, fmaf(mu1, dqn, eta))
    n2 = fmaf(fmaf(mu3, mu1, nF2), dh, fmaf(mu2, dqn, eta))
    n3 = fmaf(fmaf(mu1, mu2, nF2), dh, fmaf(mu3, dqn, eta))
    b1 = mul(n1, mul(np.abs(mu1), g32))
    b2 = mul(-n2, mul(np.abs(mu2), g31))
    b3 = mul(n3, mul(np.abs(mu3), g21))
    e1, e2, e3 = add(Fr, -mu1), add(Fr, -mu2), add(Fr, -mu3)
    B0 = add(add(b1, b2), b3)
    B1 = fmaf(b1, mu1, fmaf(b2, mu2, mul(b3, mu3)))
    B2 = fmaf(b1, fmaf(e1, e1, f32(-1)), fmaf(b2, fmaf(e2, e2, f32(-1)), mul(b3, fmaf(e3, e3, f32(-1)))))
    wc = mul(w, c)
    wcc = mul(wc, c)
    wcP, wccP = mul(wc, inv_gp), mul(wcc, inv_gp)
    SA = (mul(wcc, A1n), mul(wc, A2n))
    SB = (mul(wcP, B0), mul(wccP, B1), mul(wcP, B2))
    return SA, SB, inband


def fluct_fp32(WL, WR, g, xi, Ag, G=3, band=0.0):
    """D-, D+ ([3, n], float64) of the mixed form with every node in FP32 (no FP64 band): the
    jumps and the free-surface jump formed in FP64 and rounded once, the h-row of sum w A dW
    taken as dq, the node sums in FP32, D+- formed in FP64.  Also returns, per edge, whether any
    node's arccos argument lies within `band` of +-1."""
    hL, qL, zL = (np.asarray(a, dtype=np.float64) for a in WL)
    hR, qR, zR = (np.asarray(a, dtype=np.float64) for a in WR)
    dh, dq, dz = hR - hL, qR - qL, zR - zL
    eta = dh + dz
    x, wq = np.polynomial.legendre.leggauss(G)
    s, w = (x + 1) / 2, wq / 2
    kqg = 3.0 * xi * Ag * g
    SA = [np.zeros(hL.shape, np.float32) for _ in range(2)]
    SB = [np.zeros(hL.shape, np.float32) for _ in range(3)]
    touched = np.zeros(hL.shape, dtype=bool)
    dhf, dqf = _r(dh), _r(dq)
    for k in range(G):
        sf = f32(s[k])
        hn = fmaf(np.full_like(dhf, sf), dhf, _r(hL))
        qn = fmaf(np.full_like(dqf, sf), dqf, _r(qL))
        sa, sb, inb = node_terms(hn, qn, dhf, dqf, eta, w[k], g, kqg, band)
        touched |= inb
        SA = [add(a, b) for a, b in zip(SA, sa)]
        SB = [add(a, b) for a, b in zip(SB, sb)]
    A = np.stack([dq, SA[0].astype(np.float64), SA[1].astype(np.float64)])
    B = np.stack([v.astype(np.float64) for v in SB])
    return 0.5 * (A - B), 0.5 * (A + B), touched
