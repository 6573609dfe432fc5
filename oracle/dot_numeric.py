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
