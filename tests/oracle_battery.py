"""A fast battery of oracle pins, runnable against any build of the oracle C file.

Used by ``test_oracle_mutants.py``: each planted mistake in a copy of the oracle
must make at least one of these checks fail.  Every reference here is
independent of the oracle's own arithmetic (LAPACK eigen-decomposition,
numpy's Gauss-Legendre rule, a complex-step Jacobian, the numerical-eigensolver
DOT scheme, closed-form path integrals).

Run as ``python oracle_battery.py <liboracle.so>``; exit status 0 iff all pass.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import dot_numeric  # noqa: E402
from paper_1912_04791_amd import inputs  # noqa: E402

G = 9.81


def checks(lib):
    out = {}
    rng = np.random.default_rng(0)
    n = 200
    h = rng.uniform(0.1, 4.0, n)
    u = rng.uniform(-2.5, 2.5, n)
    q = h * u
    z = rng.uniform(-1, 1, n)
    xi, Ag = 1.0 / 0.6, 0.02

    e = oracle.eigensystem(h, q, z, G, xi, Ag, lib=lib, check=False)
    A_ind = dot_numeric.flux_matrix(h, q, G, xi, Ag)
    out["flux_matrix"] = np.max(np.abs(e["A"] - A_ind)) <= 1e-13 * np.abs(A_ind).max()
    lam_ref = np.sort(np.linalg.eigvals(A_ind).real, axis=1)
    out["eigenvalues"] = bool(np.all(np.abs(e["lam"] - lam_ref)
                                     <= 1e-12 * np.abs(lam_ref).max(axis=1, keepdims=True)))
    Ar = A_ind @ e["R"]
    lr = e["R"] * e["lam"][:, None, :]
    out["right_vectors"] = bool(np.max(np.abs(Ar - lr)) <= 1e-10 * np.abs(Ar).max())
    lA = e["Rinv"] @ A_ind
    ll = e["Rinv"] * e["lam"][:, :, None]
    out["left_vectors"] = bool(np.max(np.abs(lA - ll)) <= 1e-10 * np.abs(lA).max())
    aref = dot_numeric.abs_matrix(A_ind)
    out["abs_matrix"] = bool(np.max(np.abs(e["absA"] - aref)) <= 1e-11 * np.abs(aref).max())

    s, w = oracle.gauss(3, lib=lib)
    x, wl = np.polynomial.legendre.leggauss(3)
    out["gauss"] = bool(np.allclose(s, 0.5 * (x + 1), atol=1e-15) and
                        np.allclose(w, 0.5 * wl, atol=1e-15))

    WL, WR = inputs.make_random_edges(300, seed=3)
    Dm, Dp = oracle.fluct(WL, WR, G, xi, Ag, G=3, nthreads=2, lib=lib, check=False)
    rm, rp = dot_numeric.fluct(np.array(WL), np.array(WR), G, xi, Ag, G=3)
    sc = np.abs(rm).max() + np.abs(rp).max()
    out["fluct"] = bool(np.max(np.abs(Dm - rm)) <= 1e-11 * sc and
                        np.max(np.abs(Dp - rp)) <= 1e-11 * sc)

    # other closures: third row of A against complex-step derivatives of q_s
    laws = {"closure_grass_thr": (oracle.LAW_GRASS_THR, 0.0024, (0.3,), 0.0),
            "closure_power": (oracle.LAW_POWER, 1.45e-3, (5.0,), 0.0),
            "closure_mpm": (oracle.LAW_MPM, 0.0, (3.2e-4, 2.6), 20.0),
            "closure_vanrijn": (oracle.LAW_VANRIJN, 0.0, (3.2e-4, 2.6, 1e-6, 0.03), 20.0)}
    hh = rng.uniform(0.1, 0.8, 100)
    uu = rng.uniform(0.8, 3.0, 100) * np.where(rng.uniform(size=100) < 0.5, -1.0, 1.0)
    for name, (law, Ag, par, ks) in laws.items():
        e2 = oracle.eigensystem(hh, hh * uu, 0 * hh, G, xi, Ag, lib=lib, check=False, law=law, par=par,
                                ks=ks)
        ref = dot_numeric.flux_matrix_law(hh, hh * uu, G, xi, law, Ag, par, ks)
        out[name] = bool(np.max(np.abs(e2["A"][:, 2, :2] - ref[:, 2, :2]))
                         <= 1e-10 * np.abs(ref[:, 2, :2]).max())

    # friction: uniform flow down a slope whose friction slope equals the bed slope is steady
    ksf, h0, q0, n, dxf = 40.0, 0.3, 0.45, 60, 0.05
    s0 = q0 * q0 / (ksf * ksf * h0 ** (10.0 / 3.0))
    zf = 1.0 - s0 * (np.arange(n) + 0.5) * dxf
    spec = oracle.ChannelSpec(n_cells=n, dx=dxf, Ag=0.005, porosity=0.4, ks=ksf)
    try:
        h1, q1, z1, _ = oracle.run(spec, np.full(n, h0), np.full(n, q0), zf, 8, nthreads=2, lib=lib)
        inner = slice(10, n - 10)
        out["friction_steady"] = bool(np.max(np.abs(q1[inner] - q0)) < 1e-13 and
                                      np.max(np.abs(h1[inner] - h0)) < 1e-13)
    except oracle.OracleError:
        out["friction_steady"] = False

    # fixed-depth ghost: a run of one step equals one step with the ghost given explicitly
    spec = oracle.ChannelSpec(n_cells=32, dx=0.1, Ag=0.01, porosity=0.4,
                              bc_right=oracle.BC_FIXED_DEPTH, h_out=0.9)
    hb = 1.0 + 0.05 * rng.uniform(-1, 1, 32)
    qb = 0.3 + 0.02 * rng.uniform(-1, 1, 32)
    zb = 0.01 * rng.uniform(-1, 1, 32)
    try:
        hr, qr, zr, _ = oracle.run(spec, hb, qb, zb, 1, nthreads=2, lib=lib)
        am = oracle.cfl_amax(hb, qb, zb, G, 1 / 0.6, 0.01, lib=lib)
        hs, qs2, zs = oracle.step(hb, qb, zb, [hb[0], qb[0], zb[0]], [0.9, qb[-1], zb[-1]], G, 1 / 0.6,
                                  0.01, 3, 0.9 * 0.1 / am, 0.1, lib=lib)
        out["fixed_depth"] = bool(np.array_equal(hr, hs) and np.array_equal(qr, qs2))
    except oracle.OracleError:
        out["fixed_depth"] = False
    spec = oracle.ChannelSpec(n_cells=32, dx=0.1, Ag=0.01, porosity=0.4,
                              bc_left=oracle.BC_INFLOW_QH, q_in=0.33, h_in=0.95)
    try:
        hr, qr, zr, _ = oracle.run(spec, hb, qb, zb, 1, nthreads=2, lib=lib)
        hs, qs2, zs = oracle.step(hb, qb, zb, [0.95, 0.33, zb[0]], [hb[-1], qb[-1], zb[-1]], G, 1 / 0.6,
                                  0.01, 3, 0.9 * 0.1 / am, 0.1, lib=lib)
        out["inflow_qh"] = bool(np.array_equal(hr, hs) and np.array_equal(qr, qs2))
    except oracle.OracleError:
        out["inflow_qh"] = False
    # Dirichlet ghosts with a moving bed: after two steps the left ghost's bed has moved
    spec = oracle.ChannelSpec(n_cells=32, dx=0.1, Ag=0.01, porosity=0.4,
                              bc_left=oracle.BC_DIRICHLET, bc_right=oracle.BC_DIRICHLET,
                              dir_left=(0.97, 0.31, 0.02, -0.5), dir_right=(1.02, 0.29, -0.01, 0.0))
    try:
        h1, q1, z1, t1 = oracle.run(spec, hb, qb, zb, 1, nthreads=2, lib=lib)
        hr, qr, zr, t2 = oracle.run(spec, h1, q1, z1, 1, t0=t1, nthreads=2, lib=lib)
        am = oracle.cfl_amax(h1, q1, z1, G, 1 / 0.6, 0.01, lib=lib)
        hs, qs2, zs = oracle.step(h1, q1, z1, [0.97, 0.31, 0.02 - 0.5 * t1], [1.02, 0.29, -0.01], G,
                                  1 / 0.6, 0.01, 3, 0.9 * 0.1 / am, 0.1, lib=lib)
        out["dirichlet"] = bool(np.allclose(hr, hs, rtol=1e-14, atol=0) and
                                np.allclose(zr, zs, rtol=1e-14, atol=1e-16))
    except oracle.OracleError:
        out["dirichlet"] = False

    for name, wl, periodic in (("scheme_c1", inputs.make_c1(n_cells=120, steps=25), False),
                               ("scheme_periodic", inputs.make_c2(n_cells=256, steps=25), True)):
        xi_c = 1.0 / (1.0 - wl.porosity[0])
        spec = oracle.ChannelSpec(n_cells=wl.n_cells, dx=float(wl.dx[0]), Ag=float(wl.Ag[0]),
                                  porosity=float(wl.porosity[0]), bc_left=int(wl.bc_left[0]),
                                  bc_right=int(wl.bc_right[0]))
        try:
            hh, qq, zz, t = oracle.run(spec, wl.h, wl.q, wl.z, wl.steps, nthreads=2, lib=lib)
        except oracle.OracleError:
            out[name] = False
            continue
        hn, qn, zn, tn = dot_numeric.run(wl.h, wl.q, wl.z, wl.steps, wl.dx[0], G, xi_c, wl.Ag[0],
                                         cfl=wl.cfl, periodic=periodic)
        ok = abs(t - tn) <= 1e-12 * tn
        for a, r in ((hh, hn), (qq, qn), (zz, zn)):
            ok = ok and np.abs(a - r).sum() <= 1e-12 * max(np.abs(r).sum(), 1e-3 * np.abs(hn).sum())
        out[name] = bool(ok)
    return out


def main(path):
    lib = oracle._load(path)
    res = checks(lib)
    failed = [k for k, v in res.items() if not v]
    print("failed:", failed if failed else "none")
    return 1 if failed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
