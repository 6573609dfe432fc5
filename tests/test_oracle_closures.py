"""Pins of the oracle's other closures (Sec. 2; Sec. 5.1 power law), the friction source
(Sec. 2; Sec. 3 Eq. scheme) and the fixed-depth boundary.

* the third row of A (xi dq_s/dh, xi dq_s/dq) against complex-step derivatives of the
  closures written independently from the paper's formulas (oracle/dot_numeric.py);
* reductions: Grass with u_cr = 0 and the power law with beta = 3 are the Grass law;
  below the transport threshold the third row vanishes (eigenvalues u-c, 0, u+c);
* eigenvalues against LAPACK; states LAPACK finds complex are flagged non-hyperbolic, the
  others are not;
* fluctuations against the numerical-eigensolver DOT with the complex-step matrix;
* steady uniform flow down a constant slope (friction slope = bed slope) is preserved to
  rounding away from the boundaries (the pressure/bed term and the friction source balance);
* friction-only decay of a uniform flow converges at first order to the exact solution of
  dq/dt = -g q|q| / (K_s^2 h^(7/3));
* the fixed-depth ghost is the state (h_out, q, z) of the adjacent cell.
"""
import numpy as np
import pytest

import oracle
from oracle import dot_numeric as dn

G = 9.81
LAWS = {
    "grass_thr": (oracle.LAW_GRASS_THR, 0.0024, (0.3,), 0.0),
    "power": (oracle.LAW_POWER, 1.45e-3, (5.0,), 0.0),
    "mpm": (oracle.LAW_MPM, 0.0, (3.2e-4, 2.6), 49.4),
    "vanrijn": (oracle.LAW_VANRIJN, 0.0, (3.2e-4, 2.6, 1e-6, 0.03), 62.0),
}


def states_above_threshold(name, n, seed):
    """Random states with transport clearly above the closure's threshold."""
    law, Ag, par, ks = LAWS[name]
    rng = np.random.default_rng(seed)
    out_h, out_q = [], []
    while sum(len(x) for x in out_h) < n:
        h = rng.uniform(0.05, 1.0, 4 * n)
        u = rng.uniform(-3.0, 3.0, 4 * n)
        q = h * u
        keep = np.abs(u) > 0.05
        if law == oracle.LAW_GRASS_THR:
            keep &= np.abs(np.abs(u) - par[0]) > 0.05
        if law == oracle.LAW_MPM:
            theta = q * q / (ks * ks * h ** (10 / 3)) * h / ((par[1] - 1) * par[0])
            keep &= theta > 0.06
        if law == oracle.LAW_VANRIJN:
            us2 = G * q * q / (ks * ks * h ** (7 / 3))
            uscr2 = par[3] * G * (par[1] - 1) * par[0]
            keep &= us2 > 1.1 * uscr2
        out_h.append(h[keep])
        out_q.append(q[keep])
    return np.concatenate(out_h)[:n], np.concatenate(out_q)[:n]


@pytest.mark.parametrize("name", sorted(LAWS))
def test_row3_against_complex_step(orc, name):
    law, Ag, par, ks = LAWS[name]
    h, q = states_above_threshold(name, 500, seed=1)
    xi = 1.0 / 0.6
    e = orc.eigensystem(h, q, np.zeros_like(h), G, xi, Ag, law=law, par=par, ks=ks, check=False)
    ref = dn.flux_matrix_law(h, q, G, xi, law, Ag, par, ks)
    for col in (0, 1):
        got, exp = e["A"][:, 2, col], ref[:, 2, col]
        assert np.max(np.abs(got - exp) / (np.abs(exp) + 1e-300)) < 1e-11


def test_reductions_to_grass(orc):
    rng = np.random.default_rng(2)
    h = rng.uniform(0.1, 2.0, 300)
    q = h * rng.uniform(-2.0, 2.0, 300)
    z = np.zeros_like(h)
    ref = orc.eigensystem(h, q, z, G, 1.5, 0.01)
    thr = orc.eigensystem(h, q, z, G, 1.5, 0.01, law=orc.LAW_GRASS_THR, par=(0.0,))
    pw = orc.eigensystem(h, q, z, G, 1.5, 0.01, law=orc.LAW_POWER, par=(3.0,))
    for other in (thr, pw):
        np.testing.assert_allclose(other["A"], ref["A"], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(other["lam"], ref["lam"], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name", ["grass_thr", "mpm", "vanrijn"])
def test_below_threshold_is_fixed_bed(orc, name):
    law, Ag, par, ks = LAWS[name]
    h = np.array([0.5, 1.0, 2.0])
    q = h * np.array([0.05, -0.1, 0.08])       # slow flow: no transport
    e = orc.eigensystem(h, q, np.zeros_like(h), G, 1.6, Ag, law=law, par=par, ks=ks)
    assert np.all(e["A"][:, 2, :] == 0.0)
    u, c = q / h, np.sqrt(G * h)
    np.testing.assert_allclose(e["lam"], np.sort(np.stack([u - c, 0 * u, u + c], 1), 1),
                               rtol=0, atol=1e-13 * c.max())


@pytest.mark.parametrize("name", sorted(LAWS))
def test_eigenvalues_and_hyperbolicity_against_lapack(orc, name):
    law, Ag, par, ks = LAWS[name]
    rng = np.random.default_rng(3)
    n = 3000
    h = 10 ** rng.uniform(-2, 0.5, n)
    q = h * rng.uniform(-6, 6, n)
    xi = 1.0 / (1.0 - rng.uniform(0.0, 0.5))
    if law in (oracle.LAW_MPM, oracle.LAW_VANRIJN):
        par = (10 ** rng.uniform(-4.5, -2.5),) + tuple(par[1:])
    A = dn.flux_matrix_law(h, q, G, xi, law, Ag, par, ks)
    ev = np.linalg.eigvals(A)
    complex_ = np.abs(ev.imag).max(axis=1) > 1e-6 * np.abs(ev).max(axis=1)
    ok = 0
    for i in range(n):
        e = orc.eigensystem([h[i]], [q[i]], [0.0], G, xi, Ag, law=law, par=par, ks=ks, check=False)
        if complex_[i]:
            assert e["status"] == orc.E_NONHYPERBOLIC, i
        else:
            lam = e["lam"][0]
            ref = np.sort(ev[i].real)
            # near coalescence the roots are ill-conditioned for both methods
            tol = 1e-10 * np.abs(ref).max() / max(np.min(np.diff(ref)) / np.abs(ref).max(), 1e-3)
            assert np.max(np.abs(lam - ref)) <= tol, (i, lam, ref)
            ok += 1
    assert ok > n // 3


@pytest.mark.parametrize("name", sorted(LAWS))
def test_fluct_against_numerical_eigensolver(orc, name):
    law, Ag, par, ks = LAWS[name]
    hL, qL = states_above_threshold(name, 400, seed=4)
    rng = np.random.default_rng(5)
    hR = hL * (1 + 0.05 * rng.uniform(-1, 1, hL.size))
    qR = qL * (1 + 0.05 * rng.uniform(-1, 1, hL.size))
    zL = rng.uniform(-0.1, 0.1, hL.size)
    zR = zL + 0.01 * rng.uniform(-1, 1, hL.size)
    xi = 1.0 / 0.6
    Dm, Dp = orc.fluct((hL, qL, zL), (hR, qR, zR), G, xi, Ag, law=law, par=par, ks=ks)
    rm, rp = dn.fluct_law(np.array([hL, qL, zL]), np.array([hR, qR, zR]), G, xi, law, Ag, par, ks)
    sc = np.abs(rm).max(axis=0) + np.abs(rp).max(axis=0)
    assert np.max(np.abs(Dm - rm) / sc) < 1e-10
    assert np.max(np.abs(Dp - rp) / sc) < 1e-10


@pytest.mark.parametrize("name", ["grass", "power", "mpm"])
def test_uniform_flow_down_a_slope_is_steady(orc, name):
    if name == "grass":
        law, Ag, par = orc.LAW_GRASS, 0.005, ()
    else:
        law, Ag, par, _ = LAWS[name]
    ks, h0, q0 = 40.0, 0.3, 0.45
    s0 = q0 * q0 / (ks * ks * h0 ** (10.0 / 3.0))   # friction slope = bed slope
    n, dx, steps = 200, 0.05, 40
    x = (np.arange(n) + 0.5) * dx
    h = np.full(n, h0)
    q = np.full(n, q0)
    z = 1.0 - s0 * x
    spec = orc.ChannelSpec(n_cells=n, dx=dx, Ag=Ag, porosity=0.4, law=law, par=par, ks=ks)
    h1, q1, z1, _ = orc.run(spec, h, q, z, steps)
    inner = slice(steps + 2, n - steps - 2)
    assert np.max(np.abs(h1[inner] - h0)) < 1e-13
    assert np.max(np.abs(q1[inner] - q0)) < 1e-13
    assert np.max(np.abs(z1[inner] - z[inner])) < 1e-13
    # the boundaries did move something (transmissive ghosts do not continue the slope)
    assert np.max(np.abs(q1 - q0)) > 1e-8


def test_friction_decay_converges_first_order(orc):
    ks, h0, q0, T = 30.0, 0.4, 0.8, 2.0
    kappa = G / (ks * ks * h0 ** (7.0 / 3.0))
    exact = q0 / (1.0 + kappa * q0 * T)   # dq/dt = -kappa q^2 for q > 0
    errs = []
    for dx in (0.4, 0.2, 0.1, 0.05):
        n = 16
        h, q, z = np.full(n, h0), np.full(n, q0), np.zeros(n)
        spec = orc.ChannelSpec(n_cells=n, dx=dx, Ag=0.0, porosity=0.4, ks=ks,
                               bc_left=orc.BC_PERIODIC, bc_right=orc.BC_PERIODIC)
        t = 0.0
        while t < T - 1e-12:
            amax = orc.cfl_amax(h, q, z, G, 1 / 0.6, 0.0)
            dt = min(0.9 * dx / amax, T - t)
            h, q, z = orc.step(h, q, z, [h[-1], q[-1], z[-1]], [h[0], q[0], z[0]], G, 1 / 0.6, 0.0,
                               3, dt, dx, ks=ks)
            t += dt
        assert np.ptp(q) < 1e-14 and np.all(h == h0)
        errs.append(abs(q[0] - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 1.8) & (ratios < 2.2)), (errs, ratios)


def test_fixed_depth_ghost(orc):
    n, dx = 64, 0.1
    rng = np.random.default_rng(6)
    h = 1.0 + 0.05 * rng.uniform(-1, 1, n)
    q = 0.3 + 0.02 * rng.uniform(-1, 1, n)
    z = 0.01 * rng.uniform(-1, 1, n)
    spec = orc.ChannelSpec(n_cells=n, dx=dx, Ag=0.01, porosity=0.4, bc_left=orc.BC_INFLOW_Q,
                           bc_right=orc.BC_FIXED_DEPTH, q_in=0.31, h_out=0.9)
    h1, q1, z1, t = orc.run(spec, h, q, z, 1)
    xi = 1 / 0.6
    amax = orc.cfl_amax(h, q, z, G, xi, 0.01)
    hs, qs, zs = orc.step(h, q, z, [h[0], 0.31, z[0]], [0.9, q[-1], z[-1]], G, xi, 0.01, 3,
                          0.9 * dx / amax, dx)
    assert np.array_equal(h1, hs) and np.array_equal(q1, qs) and np.array_equal(z1, zs)
    assert abs(h1[-1] - h[-1]) > 1e-6   # the imposed depth entered


def test_inflow_qh_ghost(orc):
    # inflow-(q, h) on the left (ghost = (h_in, q_in, z_0)), fixed depth on the right
    n, dx = 48, 0.1
    rng = np.random.default_rng(7)
    h = 0.05 + 0.002 * rng.uniform(-1, 1, n)
    q = 0.02 + 0.001 * rng.uniform(-1, 1, n)
    z = 1.2 - 0.00356 * (np.arange(n) + 0.5) * dx
    law, par = orc.LAW_POWER, (5.0,)
    spec = orc.ChannelSpec(n_cells=n, dx=dx, Ag=1.45e-3, porosity=0.4, law=law, par=par, ks=49.4,
                           bc_left=orc.BC_INFLOW_QH, bc_right=orc.BC_FIXED_DEPTH, q_in=0.02,
                           h_in=0.038, h_out=0.05)
    h1, q1, z1, t = orc.run(spec, h, q, z, 1)
    xi = 1 / 0.6
    amax = orc.cfl_amax(h, q, z, G, xi, 1.45e-3, law=law, par=par, ks=49.4)
    hs, qs, zs = orc.step(h, q, z, [0.038, 0.02, z[0]], [0.05, q[-1], z[-1]], G, xi, 1.45e-3, 3,
                          0.9 * dx / amax, dx, law=law, par=par, ks=49.4)
    assert np.array_equal(h1, hs) and np.array_equal(q1, qs) and np.array_equal(z1, zs)


def test_sediment_overfeeding_aggrades_the_inflow_reach(orc):
    # uniform flow in equilibrium (friction slope = bed slope), then a solid discharge of five
    # times the equilibrium one fed upstream through the inflow depth: a wedge of deposit forms,
    # thickest at the inflow and thinning downstream (Sec. 5.1 set-up)
    n, dx, Ag, beta, q0, h0 = 100, 0.3, 1.45e-3, 5.0, 0.02, 0.05
    x = (np.arange(n) + 0.5) * dx
    z = 1.2 - 0.00356 * x
    u_in = (5.0 * (q0 / h0) ** beta) ** (1.0 / beta)
    spec = orc.ChannelSpec(n_cells=n, dx=dx, Ag=Ag, porosity=0.4, law=orc.LAW_POWER, par=(beta,),
                           ks=49.4, bc_left=orc.BC_INFLOW_QH, bc_right=orc.BC_FIXED_DEPTH,
                           q_in=q0, h_in=q0 / u_in, h_out=h0)
    h1, q1, z1, t = orc.run(spec, np.full(n, h0), np.full(n, q0), z, 1500)
    dz = z1 - z
    assert dz[0] > 1e-3
    assert np.all(np.diff(dz[:12]) < 0)            # the deposit thins downstream ...
    assert np.max(np.abs(dz[25:60])) < 1e-2 * dz[0]  # ... and has not reached mid-channel
    assert np.all(np.isfinite(h1)) and h1.min() > 0


def test_closures_need_a_strickler_coefficient(orc):
    spec = orc.ChannelSpec(n_cells=8, dx=0.1, Ag=0.0, law=orc.LAW_MPM, par=(3e-4, 2.6), ks=0.0)
    with pytest.raises(orc.OracleError) as ei:
        orc.run(spec, np.ones(8), np.ones(8), np.zeros(8), 1)
    assert ei.value.status == orc.E_ARG


@pytest.mark.parametrize("law,h,u,d50,ks,xi", [
    (oracle.LAW_VANRIJN, 0.26, 9.97, 1.76e-4, 74.45, 1.063),
    (oracle.LAW_MPM, 0.25, -9.96, 1.236e-3, 15.33, 1.519),
])
def test_high_froude_strong_transport_is_flagged(orc, law, h, u, d50, ks, xi):
    # supercritical flow (Fr ~ 6) with strong transport: LAPACK finds a complex pair
    par = (d50, 2.6) if law == oracle.LAW_MPM else (d50, 2.6, 1e-6, 0.03)
    A = dn.flux_matrix_law(np.array([h]), np.array([h * u]), G, xi, law, 0.0, par, ks)[0]
    assert np.abs(np.linalg.eigvals(A).imag).max() > 0.1
    e = orc.eigensystem([h], [h * u], [0.0], G, xi, 0.0, law=law, par=par, ks=ks, check=False)
    assert e["status"] == orc.E_NONHYPERBOLIC
