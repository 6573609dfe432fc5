"""The original DOT solver with a generic numerical eigensolver (Sec. 3.1).

TEST INFRASTRUCTURE ONLY.  A second, independent route to the same numbers as
the closed-form oracle: |A| = R |Lambda| R^-1 (Eq. asbA) is taken from LAPACK's
general eigen-decomposition (``numpy.linalg.eig``) instead of the analytical
eigenstructure of Sec. 3.3.  The paper states that A-DOT and DOT give the same
solution (Secs. 4.3, 5.1); the tests use this module to pin the oracle to that.

Vectorised with numpy over edges and nodes; plain otherwise.
"""
from __future__ import annotations

import numpy as np


def grass_qs(h, q, Ag):
    """Grass bed-load discharge q_s = A_g u^3, u = q/h (Sec. 2, Eq. Grass)."""
    u = q / h
    return Ag * u ** 3


def flux_matrix(h, q, g, xi, Ag):
    """A(W) of Sec. 2, Eq. W&A_definition, for arrays of states -> [..., 3, 3]."""
    h = np.asarray(h, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    u = q / h
    c2 = g * h
    A = np.zeros(h.shape + (3, 3))
    A[..., 0, 1] = 1.0
    A[..., 1, 0] = c2 - u * u
    A[..., 1, 1] = 2.0 * u
    A[..., 1, 2] = c2
    A[..., 2, 0] = xi * (-3.0 * Ag * u ** 3 / h)
    A[..., 2, 1] = xi * (3.0 * Ag * u ** 2 / h)
    return A


def abs_matrix(A):
    """|A| = R |Lambda| R^-1 with R from numpy.linalg.eig (Sec. 3.1, Eq. asbA)."""
    lam, R = np.linalg.eig(A)
    lam = lam.real
    R = R.real
    Rinv = np.linalg.inv(R)
    return R @ (np.abs(lam)[..., :, None] * Rinv)


def gauss01(G):
    x, w = np.polynomial.legendre.leggauss(G)
    return 0.5 * (x + 1.0), 0.5 * w


def fluct(WL, WR, g, xi, Ag, G=3):
    """D^{+-} = 1/2 sum_k w_k (A(Psi_k) +- |A(Psi_k)|) dW (Eq. DOTjumpN) -> ([3,n], [3,n])."""
    WL = np.asarray(WL, dtype=np.float64)  # [3, n]
    WR = np.asarray(WR, dtype=np.float64)
    dW = WR - WL
    s, w = gauss01(G)
    Sm = np.zeros_like(dW)
    Sp = np.zeros_like(dW)
    for k in range(G):
        Psi = WL + s[k] * dW
        A = flux_matrix(Psi[0], Psi[1], g, xi, Ag)
        aA = abs_matrix(A)
        Adw = np.einsum("nij,jn->in", A, dW)
        aAdw = np.einsum("nij,jn->in", aA, dW)
        Sm += w[k] * (Adw - aAdw)
        Sp += w[k] * (Adw + aAdw)
    return 0.5 * Sm, 0.5 * Sp


def dot_integral(Wm, Wp, g, xi, Ag, epsabs=1e-14, epsrel=1e-13):
    """The DOT integral of Eq. DOTjump for one edge by adaptive quadrature (scipy)."""
    from scipy.integrate import quad

    Wm = np.asarray(Wm, dtype=np.float64)
    Wp = np.asarray(Wp, dtype=np.float64)
    dW = Wp - Wm

    def integrand(s, r, sign):
        Psi = Wm + s * dW
        A = flux_matrix(Psi[0], Psi[1], g, xi, Ag)
        aA = abs_matrix(A)
        return 0.5 * ((A + sign * aA) @ dW)[r]

    Dm = np.array([quad(integrand, 0.0, 1.0, args=(r, -1.0), epsabs=epsabs, epsrel=epsrel,
                        limit=200)[0] for r in range(3)])
    Dp = np.array([quad(integrand, 0.0, 1.0, args=(r, +1.0), epsabs=epsabs, epsrel=epsrel,
                        limit=200)[0] for r in range(3)])
    return Dm, Dp


def run(h, q, z, n_steps, dx, g, xi, Ag, G=3, cfl=0.9, periodic=False):
    """First-order path-conservative scheme with numerical-eigensolver DOT (transmissive or periodic)."""
    W = np.stack([np.asarray(h, float), np.asarray(q, float), np.asarray(z, float)]).copy()
    t = 0.0
    for _ in range(n_steps):
        A_cells = flux_matrix(W[0], W[1], g, xi, Ag)
        amax = np.max(np.abs(np.linalg.eigvals(A_cells).real))
        dt = cfl * dx / amax
        if periodic:
            gl, gr = W[:, -1:], W[:, :1]
        else:
            gl, gr = W[:, :1], W[:, -1:]
        Wext = np.concatenate([gl, W, gr], axis=1)
        Dm, Dp = fluct(Wext[:, :-1], Wext[:, 1:], g, xi, Ag, G)
        W = W - dt / dx * (Dm[:, 1:] + Dp[:, :-1])
        t += dt
    return W[0], W[1], W[2], t


# ---------------------------------------------------------------------------
# Closures of Sec. 2 (and the power law of Sec. 5.1) as functions q_s(h, q), written to accept
# complex arguments so that complex-step differentiation gives dq_s/dh and dq_s/dq without
# any hand-derived derivative.  The branch (threshold, direction) is taken on the real part.
# Readings shared with the oracle: the laws act in the direction of the flow; Grass with a
# threshold is A_g sign(u) (|u| - u_cr)^3 above the threshold; the friction slope enters the
# Shields stress and the shear velocity as q^2 / (K_s^2 h^(10/3)); Van Rijn uses
# D_* = d50 (g (S_g - 1) / nu^2)^(1/3) and u_*cr^2 = theta_cr g (S_g - 1) d50.
LAW_GRASS, LAW_GRASS_THR, LAW_POWER, LAW_MPM, LAW_VANRIJN = 0, 1, 2, 3, 4


def _sgn(v):
    return np.sign(np.real(v))


def qs_law(h, q, g, law, Ag=0.0, par=(), ks=0.0):
    par = tuple(par) + (0.0,) * (4 - len(par))
    u = q / h
    if law == LAW_GRASS:
        return Ag * u ** 3
    if law == LAW_GRASS_THR:
        s = _sgn(u)
        ex = s * u - par[0]
        return np.where(np.real(ex) > 0, Ag * s * ex ** 3, 0.0 * ex)
    if law == LAW_POWER:
        s = _sgn(u)
        return Ag * s * (s * u) ** par[0]
    d50, Sg = par[0], par[1]
    sf = q * q / (ks * ks * h ** (10.0 / 3.0))
    if law == LAW_MPM:
        theta = sf * h / ((Sg - 1.0) * d50)
        ex = theta - 0.047
        return np.where(np.real(ex) > 0, _sgn(q) * 8.0 * ex ** 1.5, 0.0 * ex) * \
            np.sqrt(g * (Sg - 1.0) * d50 ** 3)
    if law == LAW_VANRIJN:
        nu, theta_cr = par[2], par[3]
        us2 = g * h * sf
        uscr2 = theta_cr * g * (Sg - 1.0) * d50
        T = (us2 - uscr2) / uscr2
        Dstar = d50 * (g * (Sg - 1.0) / nu ** 2) ** (1.0 / 3.0)
        return np.where(np.real(T) > 0, _sgn(q) * 0.053 * T ** 2.1, 0.0 * T) / Dstar ** 0.3 * \
            np.sqrt(g * (Sg - 1.0) * d50 ** 3)
    raise ValueError(law)


def qs_derivatives_cs(h, q, g, law, Ag=0.0, par=(), ks=0.0, eps=1e-30):
    """(dq_s/dh, dq_s/dq) by complex-step differentiation of qs_law."""
    h = np.asarray(h, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    dh = np.imag(qs_law(h + 1j * eps, q + 0j, g, law, Ag, par, ks)) / eps
    dq = np.imag(qs_law(h + 0j, q + 1j * eps, g, law, Ag, par, ks)) / eps
    return dh, dq


def flux_matrix_law(h, q, g, xi, law, Ag=0.0, par=(), ks=0.0):
    """A(W) of Eq. W&A_definition with the closure's derivatives by complex step."""
    h = np.asarray(h, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    u = q / h
    c2 = g * h
    dh, dq = qs_derivatives_cs(h, q, g, law, Ag, par, ks)
    A = np.zeros(h.shape + (3, 3))
    A[..., 0, 1] = 1.0
    A[..., 1, 0] = c2 - u * u
    A[..., 1, 1] = 2.0 * u
    A[..., 1, 2] = c2
    A[..., 2, 0] = xi * dh
    A[..., 2, 1] = xi * dq
    return A


def fluct_law(WL, WR, g, xi, law, Ag=0.0, par=(), ks=0.0, G=3):
    """Numerical-eigensolver DOT fluctuations for any closure -> ([3,n], [3,n])."""
    WL = np.asarray(WL, dtype=np.float64)
    WR = np.asarray(WR, dtype=np.float64)
    dW = WR - WL
    s, w = gauss01(G)
    Sm = np.zeros_like(dW)
    Sp = np.zeros_like(dW)
    for k in range(G):
        Psi = WL + s[k] * dW
        A = flux_matrix_law(Psi[0], Psi[1], g, xi, law, Ag, par, ks)
        aA = abs_matrix(A)
        Adw = np.einsum("nij,jn->in", A, dW)
        aAdw = np.einsum("nij,jn->in", aA, dW)
        Sm += w[k] * (Adw - aAdw)
        Sp += w[k] * (Adw + aAdw)
    return 0.5 * Sm, 0.5 * Sp
