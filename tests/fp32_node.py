"""Host model of the mixed form's FP32 node arithmetic (test infrastructure).

Evaluates, with numpy, the FP32 eigenstructure and node accumulation the mixed-form kernels
run at each quadrature node (the closed form of Sec. 3.3 in Froude-number variables, the
matrix-vector |A| dW of Eqs. asbA, ExAbsA), so that the rounding error of FP32 near coalescing
eigenvalues can be studied on the CPU: with every node in FP32 ("band off"), which no kernel
runs, and with the nodes whose arccos argument lies within the FP64 band taken from the FP64
oracle instead.

Rounding model: every FP32 operation rounds once, an FMA is the exact product (a float64
product of two floats is exact) plus the addend rounded to FP32 (two roundings where the device
rounds once, a difference of at most one ulp in rare cases); the reciprocal square root,
reciprocal, cosine and sine are rounded correctly, where the device approximates them to one or
two ulp.  The model's FP32 error therefore slightly understates the device's; the band-on
figures of the tests come from the device itself.
"""
from __future__ import annotations

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


def acos_f32(x):
    """Abramowitz & Stegun 4.4.46 (degree 7), as the mixed form evaluates it."""
    a = np.abs(x)
    cs = [-0.0012624911, 0.0066700901, -0.0170881256, 0.0308918810, -0.0501743046, 0.0889789874,
          -0.2145988016, 1.5707963050]
    p = fmaf(a, np.full_like(a, f32(cs[0])), f32(cs[1]))
    for c in cs[2:]:
        p = fmaf(a, p, f32(c))
    r = mul(p, _r(np.sqrt((f32(1) - a).astype(np.float64))))
    return np.where(x < 0, add(f32(3.14159265358979), -r), r).astype(np.float32)


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
    r1 = _r(1.0 / np.sqrt(k1.astype(np.float64)))
    x = mul(mul(f32(0.5), k2), mul(mul(r1, r1), r1))
    inband = ~(np.abs(x) < f32(1) - f32(band)) if band > 0 else np.zeros(x.shape, dtype=bool)
    xc = np.clip(x, f32(-1), f32(1))
    th = mul(acos_f32(xc), f32(1.0 / 3.0))
    cs, sn = _r(np.cos(th.astype(np.float64))), _r(np.sin(th.astype(np.float64)))
    m = mul(f32(2.0 / 3.0), mul(k1, r1))
    f = mul(f32(2.0 / 3.0), Fr)
    p, rr = mul(f32(0.5), cs), mul(f32(0.86602540378443864676), sn)
    c = mul(gh, inv_c)
    mu1 = fmaf(-m, add(p, rr), f)
    mu2 = fmaf(-m, add(p, -rr), f)
    mu3 = fmaf(m, cs, f)
    g21 = mul(mul(f32(2), m), rr)
    g31 = mul(m, fmaf(np.full_like(p, f32(3)), p, rr))
    g32 = mul(m, fmaf(np.full_like(p, f32(3)), p, -rr))
    dqn = mul(dq, inv_c)
    nF2 = -Fr2
    A1n = fmaf(nF2, dh, fmaf(mul(f32(2), Fr), dqn, eta))
    A2n = mul(b, fmaf(-Fr, dh, dqn))
    n1 = fmaf(fmaf(mu2, mu3, nF2), dh, fmaf(mu1, dqn, eta))
    n2 = fmaf(fmaf(mu3, mu1, nF2), dh, fmaf(mu2, dqn, eta))
    n3 = fmaf(fmaf(mu1, mu2, nF2), dh, fmaf(mu3, dqn, eta))
    wP = mul(w, _r(1.0 / mul(mul(g21, g31), g32).astype(np.float64)))
    b1 = mul(mul(n1, mul(np.abs(mu1), g32)), wP)
    b2 = mul(mul(-n2, mul(np.abs(mu2), g31)), wP)
    b3 = mul(mul(n3, mul(np.abs(mu3), g21)), wP)
    e1, e2, e3 = add(Fr, -mu1), add(Fr, -mu2), add(Fr, -mu3)
    B0 = add(add(b1, b2), b3)
    B1 = fmaf(b1, mu1, fmaf(b2, mu2, mul(b3, mu3)))
    B2 = fmaf(b1, fmaf(e1, e1, f32(-1)), fmaf(b2, fmaf(e2, e2, f32(-1)), mul(b3, fmaf(e3, e3, f32(-1)))))
    wc = mul(w, c)
    SA = (mul(mul(wc, c), A1n), mul(wc, A2n))
    SB = (mul(c, B0), mul(mul(c, c), B1), mul(c, B2))
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
