"""Pins of the oracle's DOT fluctuations (Sec. 3.1, Eqs. jumps, path, DOTjump, DOTjumpN).

* Gauss-Legendre nodes/weights vs numpy's leggauss (mapped to [0, 1]);
* consistency: W- = W+ gives D+- = 0;
* compatibility (Eq. jumps): D- + D+ = sum_k w_k A(Psi_k) dW; row 1 equals dq;
* with dh = 0 the compatibility integrand is a polynomial of degree 2 in s, so a
  2-point rule already gives the exact path integral: row 3 = xi (q_s(W+) - q_s(W-)),
  row 2 = d(q^2/h) + g h dz;
* as G grows the rule converges to the exact path integral: row 3 -> xi dq_s,
  row 2 -> d(g h^2/2 + q^2/h) + g (h- + h+)/2 dz;
* the full DOT integral (Eq. DOTjump) by adaptive quadrature with a numerical
  eigensolver matches the oracle at large G;
* the oracle's G-point fluctuation equals the numerical-eigensolver DOT at G = 3;
* mirror symmetry x -> -x: D+(P W_R, P W_L) = P D-(W_L, W_R), P = diag(1, -1, 1);
* fixed bed, supercritical flow: D- = 0 (pure upwinding); subcritical reverse: D+ = 0.
"""
import numpy as np
import pytest

from oracle import dot_numeric
from paper_1912_04791_amd import inputs

G = 9.81


def qs(h, q, Ag):
    return Ag * (q / h) ** 3


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 24])
def test_gauss_rule_vs_numpy(orc, n):
    s, w = orc.gauss(n)
    x, wl = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(s, 0.5 * (x + 1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, 0.5 * wl, rtol=0, atol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-14


def test_zero_jump_gives_zero_fluctuation(orc):
    WL, _ = inputs.make_random_edges(500, seed=1)
    Dm, Dp = orc.fluct(WL, WL, G, 1.0 / 0.6, 0.01)
    assert np.all(Dm == 0.0) and np.all(Dp == 0.0)


def test_compatibility_condition(orc):
    WL, WR = inputs.make_random_edges(400, seed=2)
    xi, Ag = 1.0 / 0.6, 0.01
    for Gq in (1, 2, 3, 5):
        Dm, Dp = orc.fluct(WL, WR, G, xi, Ag, G=Gq)
        s, w = orc.gauss(Gq)
        WLa, WRa = np.array(WL), np.array(WR)
        dW = WRa - WLa
        ref = np.zeros_like(dW)
        for k in range(Gq):
            Psi = WLa + s[k] * dW
            A = dot_numeric.flux_matrix(Psi[0], Psi[1], G, xi, Ag)
            ref += w[k] * np.einsum("nij,jn->in", A, dW)
        tot = Dm + Dp
        scale = np.abs(ref).max(axis=0) + np.abs(Dp - Dm).max(axis=0)
        assert np.max(np.abs(tot - ref) / scale) < 1e-13
        # row 1: the weights sum to one, so D- + D+ reproduces dq
        np.testing.assert_allclose(tot[0], dW[1], rtol=1e-13, atol=1e-14 * np.abs(dW[1]).max())


def test_polynomial_path_is_integrated_exactly(orc):
    rng = np.random.default_rng(3)
    n = 300
    h = rng.uniform(0.2, 3.0, n)
    qL, qR = rng.uniform(-2, 2, n), rng.uniform(-2, 2, n)
    zL, zR = rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n)
    xi, Ag = 1.0 / 0.65, 0.02
    for Gq in (2, 3, 4):
        Dm, Dp = orc.fluct((h, qL, zL), (h, qR, zR), G, xi, Ag, G=Gq)
        tot = Dm + Dp
        row3 = xi * (qs(h, qR, Ag) - qs(h, qL, Ag))
        row2 = qR ** 2 / h - qL ** 2 / h + G * h * (zR - zL)
        sc = np.abs(Dp - Dm).max(axis=0) + 1.0
        assert np.max(np.abs(tot[2] - row3) / sc) < 1e-13
        assert np.max(np.abs(tot[1] - row2) / sc) < 1e-13


def test_high_order_rule_reaches_path_integral(orc):
    WL, WR = inputs.make_random_edges(200, seed=4, h_range=(0.3, 3.0), u_range=(-2, 2))
    xi, Ag = 1.0 / 0.6, 0.01
    Dm, Dp = orc.fluct(WL, WR, G, xi, Ag, G=24)
    (hL, qL, zL), (hR, qR, zR) = WL, WR
    tot = Dm + Dp
    row3 = xi * (qs(hR, qR, Ag) - qs(hL, qL, Ag))
    row2 = (0.5 * G * hR ** 2 + qR ** 2 / hR) - (0.5 * G * hL ** 2 + qL ** 2 / hL) \
        + G * 0.5 * (hL + hR) * (zR - zL)
    sc = np.abs(Dp - Dm).max(axis=0) + np.abs(row2)
    assert np.max(np.abs(tot[2] - row3) / sc) < 1e-10
    assert np.max(np.abs(tot[1] - row2) / sc) < 1e-10


def test_dot_integral_by_adaptive_quadrature(orc):
    WL, WR = inputs.make_random_edges(12, seed=5, h_range=(0.3, 3.0), u_range=(-2, 2))
    xi, Ag = 1.0 / 0.6, 0.01
    Dm, Dp = orc.fluct(WL, WR, G, xi, Ag, G=32)
    WLa, WRa = np.array(WL), np.array(WR)
    for e in range(WLa.shape[1]):
        rm, rp = dot_numeric.dot_integral(WLa[:, e], WRa[:, e], G, xi, Ag)
        sc = np.abs(rm).max() + np.abs(rp).max()
        # |A(Psi(s))| has kinks where an eigenvalue changes sign; the Gauss rule then
        # converges only algebraically, hence the looser bound.
        assert np.max(np.abs(Dm[:, e] - rm)) < 1e-6 * sc
        assert np.max(np.abs(Dp[:, e] - rp)) < 1e-6 * sc


def test_smooth_path_dot_integral_tight(orc):
    # subcritical edges with no sign change of any eigenvalue along the path:
    # the integrand is analytic and the Gauss rule converges exponentially
    rng = np.random.default_rng(6)
    n = 10
    hL = rng.uniform(0.8, 1.5, n)
    hR = hL * (1 + 0.2 * rng.uniform(-1, 1, n))
    uL = rng.uniform(0.2, 0.6, n)
    uR = uL + 0.1 * rng.uniform(-1, 1, n)
    zL = rng.uniform(-0.2, 0.2, n)
    zR = zL + 0.1 * rng.uniform(-1, 1, n)
    WL, WR = (hL, hL * uL, zL), (hR, hR * uR, zR)
    xi, Ag = 1.0 / 0.6, 0.005
    Dm, Dp = orc.fluct(WL, WR, G, xi, Ag, G=24)
    for e in range(n):
        rm, rp = dot_numeric.dot_integral([hL[e], hL[e] * uL[e], zL[e]],
                                          [hR[e], hR[e] * uR[e], zR[e]], G, xi, Ag)
        sc = np.abs(rm).max() + np.abs(rp).max()
        assert np.max(np.abs(Dm[:, e] - rm)) < 1e-11 * sc
        assert np.max(np.abs(Dp[:, e] - rp)) < 1e-11 * sc


def test_matches_numerical_eigensolver_dot(orc):
    WL, WR = inputs.make_random_edges(2000, seed=7)
    xi, Ag = 1.0 / 0.62, 0.02
    for Gq in (1, 3, 5):
        Dm, Dp = orc.fluct(WL, WR, G, xi, Ag, G=Gq)
        rm, rp = dot_numeric.fluct(np.array(WL), np.array(WR), G, xi, Ag, G=Gq)
        sc = np.abs(rm).max(axis=0) + np.abs(rp).max(axis=0)
        assert np.max(np.abs(Dm - rm) / sc) < 1e-12
        assert np.max(np.abs(Dp - rp) / sc) < 1e-12


def test_mirror_symmetry(orc):
    WL, WR = inputs.make_random_edges(1000, seed=8)
    xi, Ag = 1.0 / 0.6, 0.03
    Dm, Dp = orc.fluct(WL, WR, G, xi, Ag)
    (hL, qL, zL), (hR, qR, zR) = WL, WR
    Em, Ep = orc.fluct((hR, -qR, zR), (hL, -qL, zL), G, xi, Ag)
    P = np.array([1.0, -1.0, 1.0])[:, None]
    sc = np.abs(Dm).max(axis=0) + np.abs(Dp).max(axis=0)
    assert np.max(np.abs(Ep - P * Dm) / sc) < 1e-13
    assert np.max(np.abs(Em - P * Dp) / sc) < 1e-13


def test_upwinding_on_fixed_bed(orc):
    rng = np.random.default_rng(9)
    n = 500
    hL = rng.uniform(0.1, 1.0, n)
    hR = hL * (1 + 0.1 * rng.uniform(-1, 1, n))
    cmax = np.sqrt(G * np.maximum(hL, hR))
    uL = cmax * rng.uniform(1.5, 3.0, n)
    uR = cmax * rng.uniform(1.5, 3.0, n)
    z = rng.uniform(-0.1, 0.1, n)
    xi = 1.0
    Dm, Dp = orc.fluct((hL, hL * uL, z), (hR, hR * uR, z), G, xi, 0.0)
    sc = np.abs(Dp).max(axis=0)
    assert np.max(np.abs(Dm).max(axis=0) / sc) < 1e-13
    # reversed supercritical flow: everything goes left
    Dm, Dp = orc.fluct((hL, -hL * uL, z), (hR, -hR * uR, z), G, xi, 0.0)
    sc = np.abs(Dm).max(axis=0)
    assert np.max(np.abs(Dp).max(axis=0) / sc) < 1e-13
