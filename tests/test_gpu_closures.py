"""Other closures, the friction source and the experiment boundary conditions on the HIP path
(MI355X), through the C ABI, against the CPU oracle.

Bars: relative L1 <= 1e-12 per variable in FP64, <= 1e-5 in the mixed form (per channel for
batched runs); pairwise fluctuations and CFL maxima per law at the FP64 bar.  Workloads are the
Sec. 5.1- and Sec. 5.2-shaped runs of ``inputs`` (power law; Meyer-Peter & Mueller, Van Rijn,
Grass with threshold) with Strickler friction, an inflow-(q, h) upstream end and a fixed-depth
downstream end; states LAPACK finds non-hyperbolic are reported as such.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04791_amd import inputs

from common import max_rel_l1, oracle_run, per_channel_rel_l1

pytestmark = pytest.mark.gpu

LAWS = {   # law, A_g, parameters, K_s  (the same values as the oracle's closure pins)
    "grass_thr": (oracle.LAW_GRASS_THR, 0.0024, (0.3,), 0.0),
    "power": (oracle.LAW_POWER, 1.45e-3, (5.0,), 0.0),        # integer beta - 1: product form
    "power_real": (oracle.LAW_POWER, 1.45e-3, (2.5,), 0.0),   # general power
    "power_b2": (oracle.LAW_POWER, 4e-3, (2.0,), 0.0),        # beta - 1 = 1: the lowest bit
    "mpm": (oracle.LAW_MPM, 0.0, (3.2e-4, 2.6), 49.4),
    "vanrijn": (oracle.LAW_VANRIJN, 0.0, (3.2e-4, 2.6, 1e-6, 0.03), 62.0),
}
WORKLOADS = ["soni", "bellal_mpm", "bellal_vanrijn", "bellal_thr"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def dsve():
    from paper_1912_04791_amd import dsve as d
    return d


def single(name, **kw):
    if name == "soni":
        return inputs.make_soni(n_channels=1, **kw)
    return inputs.make_bellal(name.split("_", 1)[1], n_channels=1, **kw)


def batched(name, **kw):
    if name == "soni":
        return inputs.make_soni(**kw)
    return inputs.make_bellal(name.split("_", 1)[1], **kw)


def run_gpu(dsve, wl, steps=None, precision="fp64", launch=None):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    if launch is not None:
        ctx.set_launch(*launch)
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, wl.steps if steps is None else steps, t)
    ctx.sync()
    out = (h.cpu().numpy(), q.cpu().numpy(), z.cpu().numpy(), t.cpu().numpy())
    ctx.close()
    return out


def random_states(name, n, seed):
    """States with transport above the closure's threshold, and small jumps to a right state."""
    law, Ag, par, ks = LAWS[name]
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.05, 1.0, n)
    u = rng.uniform(0.6, 3.0, n) * np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    return h, h * u


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(LAWS))
@pytest.mark.parametrize("G", [1, 3, 5])
def test_pairwise_fluct_per_law(torch_dev, dsve, name, G):
    torch = torch_dev
    law, Ag, par, ks = LAWS[name]
    n = 50_021
    hL, qL = random_states(name, n, seed=7 + G)
    rng = np.random.default_rng(100 + G)
    hR = hL * (1 + 0.1 * rng.uniform(-1, 1, n))
    qR = qL * (1 + 0.1 * rng.uniform(-1, 1, n))
    zL = rng.uniform(-0.2, 0.2, n)
    zR = zL + 0.02 * rng.uniform(-1, 1, n)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=Ag, n_gauss=G, dx=1.0, law=law, law_extra=par,
                              ks=ks)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (hL, qL, zL, hR, qR, zR)]
    Dm = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    Dp = torch.zeros_like(Dm)
    ctx.dot_edge_fluct(*dev, Dm, Dp)
    ctx.sync()
    rm, rp = oracle.fluct((hL, qL, zL), (hR, qR, zR), 9.81, 1.0 / 0.6, Ag, G=G, law=law, par=par,
                          ks=ks)
    sc = np.abs(rm).max(axis=0) + np.abs(rp).max(axis=0)
    for got, ref in ((Dm.cpu().numpy(), rm), (Dp.cpu().numpy(), rp)):
        assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-12
        per = np.abs(got - ref).max(axis=0) / sc
        assert np.quantile(per, 0.999) <= 1e-12 and per.max() <= 1e-9, per.max()
    ctx.close()


@pytest.mark.parametrize("name", sorted(LAWS))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfl_reduce_per_law(torch_dev, dsve, name, precision):
    torch = torch_dev
    law, Ag, par, ks = LAWS[name]
    h, q = random_states(name, 70_001, seed=3)
    z = np.zeros_like(h)
    ctx = dsve.Context.single(h.size, porosity=0.4, A_g=Ag, dx=0.5, law=law, law_extra=par, ks=ks,
                              precision=precision)
    dh, dq, dz = (torch.from_numpy(a).cuda() for a in (h, q, z))
    amax = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cfl_reduce(dh, dq, dz, amax, dt)
    ctx.sync()
    ref = oracle.cfl_amax(h, q, z, 9.81, 1.0 / 0.6, Ag, law=law, par=par, ks=ks)
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert abs(float(amax[0]) - ref) <= tol * ref
    assert abs(float(dt[0]) - 0.9 * 0.5 / ref) <= tol * 0.9 * 0.5 / ref
    ctx.close()


@pytest.mark.parametrize("name", WORKLOADS)
def test_single_channel_run_fp64(torch_dev, dsve, name):
    wl = single(name, steps=400)
    got = run_gpu(dsve, wl)
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= 1e-12
    assert abs(got[3][0] - ref[3][0]) <= 1e-12 * ref[3][0]


@pytest.mark.parametrize("name", WORKLOADS)
def test_single_channel_run_mixed(torch_dev, dsve, name):
    wl = single(name, steps=400)
    got = run_gpu(dsve, wl, precision="mixed")
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= 1e-5


@pytest.mark.parametrize("name", WORKLOADS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batched_ensemble(torch_dev, dsve, name, precision, tol):
    # ragged lengths (several tiles, tails, channels shorter than a tile), per-channel parameters
    wl = batched(name, n_channels=24, len_lo=40, len_hi=700, steps=150, seed=5)
    got = run_gpu(dsve, wl, precision=precision, launch=(128, 2, 60))
    ref = oracle_run(wl)
    per = per_channel_rel_l1(got, ref, wl.offsets)
    assert per.max() <= tol, (per.max(), int(np.argmax(per)))
    np.testing.assert_allclose(got[3], ref[3], rtol=1e-12 if precision == "fp64" else 1e-6)


def test_friction_with_the_grass_law(torch_dev, dsve):
    # the closed-form Grass kernels with the friction source and both new boundaries
    wl = inputs.make_soni(n_channels=1, n_cells=300, steps=300)
    wl.law = inputs.LAW_GRASS
    wl.law_par[:] = 0.0
    wl.Ag[:] = 0.004
    got = run_gpu(dsve, wl)
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= 1e-12


def test_cell_update_applies_friction(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_soni(n_channels=1, n_cells=257)
    rng = np.random.default_rng(9)
    h = wl.h * (1 + 0.05 * rng.uniform(-1, 1, wl.n_cells))
    q = wl.q * (1 + 0.05 * rng.uniform(-1, 1, wl.n_cells))
    z = wl.z.copy()
    ks, par = float(wl.ks[0]), tuple(wl.law_par[0])
    ctx = dsve.Context.from_workload(wl)
    gl = np.array([wl.h_in[0], wl.q_in[0], z[0]])
    gr = np.array([wl.h_out[0], q[-1], z[-1]])
    WL = [np.concatenate([[gl[k]], a]) for k, a in enumerate((h, q, z))]
    WR = [np.concatenate([a, [gr[k]]]) for k, a in enumerate((h, q, z))]
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (*WL, *WR)]
    E = wl.n_cells + 1
    Dm = torch.zeros(3, E, dtype=torch.float64, device="cuda")
    Dp = torch.zeros_like(Dm)
    ctx.dot_edge_fluct(*dev, Dm, Dp)
    dt = 0.01
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    hd, qd, zd = (torch.from_numpy(a.copy()).cuda() for a in (h, q, z))
    ctx.cell_update(Dm, Dp, dtd, hd, qd, zd)
    ctx.sync()
    ho, qo, zo = oracle.step(h, q, z, gl, gr, 9.81, 1.0 / 0.6, float(wl.Ag[0]), 3, dt,
                             float(wl.dx[0]), law=wl.law, par=par, ks=ks)
    for a, r in ((hd, ho), (qd, qo), (zd, zo)):
        np.testing.assert_allclose(a.cpu().numpy(), r, rtol=1e-13, atol=0)
    # the friction source is on: without it the discharge would differ
    assert np.abs(qo - q).max() > 1e-8
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("law,h,u,par,ks,por", [
    (oracle.LAW_MPM, 0.25, -9.96, (1.236e-3, 2.6), 15.33, 1.0 - 1.0 / 1.519),
    (oracle.LAW_VANRIJN, 0.26, 9.97, (1.76e-4, 2.6, 1e-6, 0.03), 74.45, 1.0 - 1.0 / 1.063),
])
def test_non_hyperbolic_state_is_reported(torch_dev, dsve, precision, law, h, u, par, ks, por):
    # strong transport at Fr ~ 6: complex eigenvalues (LAPACK, in the oracle's closure pins)
    torch = torch_dev
    e = oracle.eigensystem([h], [h * u], [0.0], 9.81, 1.0 / (1.0 - por), 0.0, law=law, par=par,
                           ks=ks, check=False)
    assert e["status"] == oracle.E_NONHYPERBOLIC
    n = 40
    ctx = dsve.Context.single(n, porosity=por, A_g=0.0, dx=0.1, law=law, law_extra=par, ks=ks,
                              precision=precision)
    hd = torch.full((n,), h, dtype=torch.float64, device="cuda")
    qd = torch.full((n,), h * u, dtype=torch.float64, device="cuda")
    zd = torch.zeros(n, dtype=torch.float64, device="cuda")
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.adot_step(hd, qd, zd, 1, t)
    assert ctx.sync_status() == dsve.E_NONHYPERBOLIC
    assert "complex" in ctx.last_error()
    ctx.close()
