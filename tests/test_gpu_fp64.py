"""FP64 HIP path vs the CPU oracle, through the C ABI (MI355X).

Bar: relative L1 <= 1e-12 per variable for whole runs (the FP64 tolerance);
pairwise fluctuations and the CFL maximum are held to the same bar per edge set.
Sizes span several tiles and ragged tails; full-size cases (2^20 and 2^24 cells)
run a few steps of the launch configuration the benchmark times.
"""
import numpy as np
import pytest

import oracle
from paper_1912_04791_amd import inputs

from common import max_rel_l1, oracle_run, per_channel_rel_l1, spec_of

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def run_gpu(dsve, torch, wl, steps=None, precision="fp64", launch=None, autotune=False, split=None):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    if launch is not None:
        ctx.set_launch(*launch)
    if split is not None:
        ctx.set_cfl_split(split)
        assert ctx.get_cfl_split() == split
    h, q, z, t = dsve.upload(wl)
    if autotune:   # the launch the benchmark times: tuned on a scratch copy of the state
        ctx.autotune(h, q, z, trial_steps=20)
    ctx.adot_step(h, q, z, wl.steps if steps is None else steps, t)
    ctx.sync()
    out = (h.cpu().numpy(), q.cpu().numpy(), z.cpu().numpy(), t.cpu().numpy())
    ctx.close()
    return out


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("G", [1, 2, 3, 4, 5])
def test_pairwise_fluct_matches_oracle(torch_dev, dsve, G):
    torch = torch_dev
    n = 100_003
    WL, WR = inputs.make_random_edges(n, seed=100 + G)
    xi_p, Ag = 0.4, 0.02
    ctx = dsve.Context.single(16, porosity=xi_p, A_g=Ag, n_gauss=G, dx=1.0)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (*WL, *WR)]
    Dm = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    Dp = torch.zeros_like(Dm)
    ctx.dot_edge_fluct(*dev, Dm, Dp)
    ctx.sync()
    rm, rp = oracle.fluct(WL, WR, 9.81, 1.0 / (1.0 - xi_p), Ag, G=G)
    gm, gp = Dm.cpu().numpy(), Dp.cpu().numpy()
    # per edge, relative to the edge's own fluctuation size: every edge within the FP64 bar (the
    # oracle and an exact-arithmetic evaluation of the kernels' matrix-vector form agree to 3e-14
    # per edge on these inputs)
    sc = np.abs(rm).max(axis=0) + np.abs(rp).max(axis=0)
    for got, ref in ((gm, rm), (gp, rp)):
        l1 = np.abs(got - ref).sum() / np.abs(ref).sum()
        assert l1 <= TOL, l1
        per = np.abs(got - ref).max(axis=0) / sc
        print(f"G={G}: per-edge relative error max {per.max():.3g} (edge {np.argmax(per)}), "
              f"99.9% {np.quantile(per, 0.999):.3g}, L1 {l1:.3g}")
        assert per.max() <= TOL, (per.max(), np.argmax(per))
    ctx.close()


def test_node_paths_do_not_change_bits(torch_dev, dsve):
    # An FP64 node takes a path chosen for its whole wave: flow towards +x in every lane, towards
    # -x in every lane, or otherwise a per-lane choice of the eigenpair that D- is taken from
    # (Sec. 3.1, Eqs. asbA, ExAbsA: one eigenvalue differs in sign from the middle one).  The
    # same edges, laid out once in waves of one kind each and once shuffled (every wave mixed,
    # some lanes past abs(Fr) = 3, where the eigenpair is the other one), must give the same
    # bits edge by edge, and match the oracle.
    torch = torch_dev
    rng = np.random.default_rng(77)
    n = 64 * 600
    h = rng.uniform(0.3, 3.0, n)
    hR = h * (1 + 0.05 * rng.uniform(-1, 1, n))
    kind = np.arange(n) // (n // 3)            # 0: towards +x, 1: towards -x, 2: mixed signs and fast
    fr = np.where(kind == 0, rng.uniform(0.05, 2.5, n),
                  np.where(kind == 1, -rng.uniform(0.05, 2.5, n), rng.uniform(-5.0, 5.0, n)))
    u = fr * np.sqrt(9.81 * h)
    uR = u * (1 + 0.05 * rng.uniform(-1, 1, n))
    z = rng.uniform(-0.2, 0.2, n)
    zR = z + 0.02 * rng.uniform(-1, 1, n)
    WL, WR = (h, h * u, z), (hR, hR * uR, zR)
    perm = rng.permutation(n)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=0.01, dx=1.0)
    outs = []
    for order in (np.arange(n), perm):
        dev = [torch.from_numpy(np.ascontiguousarray(a[order])).cuda() for a in (*WL, *WR)]
        Dm = torch.zeros(3, n, dtype=torch.float64, device="cuda")
        Dp = torch.zeros_like(Dm)
        ctx.dot_edge_fluct(*dev, Dm, Dp)
        ctx.sync()
        gm, gp = np.empty((3, n)), np.empty((3, n))
        gm[:, order], gp[:, order] = Dm.cpu().numpy(), Dp.cpu().numpy()
        outs.append((gm, gp))
    ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    rm, rp = oracle.fluct(WL, WR, 9.81, 1.0 / 0.6, 0.01)
    sc = np.abs(rm).max(axis=0) + np.abs(rp).max(axis=0)
    for got, ref in zip(outs[0], (rm, rp)):
        per = np.abs(got - ref).max(axis=0) / sc
        assert per.max() <= TOL, (per.max(), np.argmax(per))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [0, 1, 63, 65, 257])
def test_pairwise_fluct_small_and_ragged_edge_counts(torch_dev, dsve, n, precision):
    # no edges (nothing launched), one edge, and counts just off whole waves and workgroups
    torch = torch_dev
    WL, WR = inputs.make_random_edges(max(n, 1), seed=300 + n)
    WL, WR = tuple(a[:n] for a in WL), tuple(a[:n] for a in WR)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=0.02, dx=1.0, precision=precision)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (*WL, *WR)]
    # padded outputs: what lies past [3][n] must stay untouched
    Dm = torch.full((3 * n + 64,), 7.0, dtype=torch.float64, device="cuda")
    Dp = torch.full_like(Dm, 7.0)
    ctx.dot_edge_fluct(*dev, Dm[:3 * n], Dp[:3 * n])
    ctx.sync()
    assert torch.all(Dm[3 * n:] == 7.0) and torch.all(Dp[3 * n:] == 7.0)
    if n:
        rm, rp = oracle.fluct(WL, WR, 9.81, 1.0 / 0.6, 0.02)
        tol = TOL if precision == "fp64" else 1e-5
        for got, ref in ((Dm[:3 * n], rm), (Dp[:3 * n], rp)):
            got = got.cpu().numpy().reshape(3, n)
            assert np.abs(got - ref).sum() <= tol * np.abs(ref).sum()
    ctx.close()


def test_cfl_reduce_matches_oracle(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_c3(n_cells=300_001)
    ctx = dsve.Context.from_workload(wl, precision="fp64")
    h, q, z, _ = dsve.upload(wl)
    amax = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.cfl_reduce(h, q, z, amax, dt)
    ctx.sync()
    ref = oracle.cfl_amax(wl.h, wl.q, wl.z, 9.81, 1.0 / (1 - wl.porosity[0]), wl.Ag[0])
    assert abs(float(amax[0]) - ref) <= 1e-14 * ref
    assert abs(float(dt[0]) - wl.cfl * wl.dx[0] / ref) <= 1e-14 * float(dt[0])
    ctx.close()


def test_cell_update_matches_oracle_step(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_c2(n_cells=5000)
    xi = 1.0 / (1.0 - wl.porosity[0])
    N = wl.n_cells
    # edge states with periodic ghosts; fluctuations from the oracle
    hL, qL, zL = (np.concatenate([a[-1:], a]) for a in (wl.h, wl.q, wl.z))
    hR, qR, zR = (np.concatenate([a, a[:1]]) for a in (wl.h, wl.q, wl.z))
    Dm, Dp = oracle.fluct((hL, qL, zL), (hR, qR, zR), 9.81, xi, wl.Ag[0])
    dt = 1.3e-4
    ref = oracle.step(wl.h, wl.q, wl.z, [wl.h[-1], wl.q[-1], wl.z[-1]], [wl.h[0], wl.q[0], wl.z[0]],
                      9.81, xi, wl.Ag[0], 3, dt, wl.dx[0])
    ctx = dsve.Context.from_workload(wl)
    h, q, z, _ = dsve.upload(wl)
    tDm = torch.from_numpy(np.ascontiguousarray(Dm)).cuda()
    tDp = torch.from_numpy(np.ascontiguousarray(Dp)).cuda()
    tdt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ctx.cell_update(tDm, tDp, tdt, h, q, z)
    ctx.sync()
    assert N + 1 == Dm.shape[1]
    # one update is W - r s; allow a few roundings of the operands (FMA contraction on the GPU)
    eps = np.finfo(np.float64).eps
    for got, r, w0 in zip((h, q, z), ref, (wl.h, wl.q, wl.z)):
        g = got.cpu().numpy()
        assert np.all(np.abs(g - r) <= 4 * eps * (np.abs(w0) + np.abs(w0 - r)))
    ctx.close()


# ---------------------------------------------------------------------------
def test_c1_full_run(torch_dev, dsve):
    wl = inputs.make_c1()
    got = run_gpu(dsve, torch_dev, wl)
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= TOL
    assert abs(got[3][0] - ref[3][0]) <= 1e-12 * ref[3][0]


@pytest.mark.parametrize("n_cells,steps", [(1, 7), (2, 6), (254, 13), (255, 12), (256, 61),
                                           (257, 121), (16_385, 100)])
def test_ragged_sizes_and_odd_steps(torch_dev, dsve, n_cells, steps):
    wl = inputs.make_c2(n_cells=max(n_cells, 1), steps=steps, length=1000.0 * n_cells / (1 << 20) + 1e-3,
                        max_mode=min(64, max(1, n_cells // 4)))
    got = run_gpu(dsve, torch_dev, wl)
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= TOL


@pytest.mark.parametrize("bc", ["transmissive", "inflow"])
def test_c3_shape_reduced(torch_dev, dsve, bc):
    wl = inputs.make_c3(n_cells=1 << 14, steps=150)
    if bc == "transmissive":
        wl.bc_left[:] = inputs.BC_TRANSMISSIVE
    got = run_gpu(dsve, torch_dev, wl, precision="fp64")
    ref = oracle_run(wl)
    assert max_rel_l1(got, ref) <= TOL


def test_c4_shape_batched_reduced(torch_dev, dsve):
    wl = inputs.make_c4(n_channels=48, len_lo=64, len_hi=3000, steps=60)
    got = run_gpu(dsve, torch_dev, wl)
    ref = oracle_run(wl)
    per = per_channel_rel_l1(got, ref, wl.offsets)
    assert per.max() <= TOL, (per.max(), per.argmax())
    np.testing.assert_allclose(got[3], ref[3], rtol=1e-12)


def test_c5_shape_batched_reduced_fp64(torch_dev, dsve):
    wl = inputs.make_c5(n_channels=64, len_lo=100, len_hi=700, steps=80)
    got = run_gpu(dsve, torch_dev, wl, precision="fp64")
    ref = oracle_run(wl)
    per = per_channel_rel_l1(got, ref, wl.offsets)
    assert per.max() <= TOL, (per.max(), per.argmax())


def test_single_cell_channels_batched(torch_dev, dsve):
    # channels as short as one cell, mixed with long ones
    base = inputs.make_c4(n_channels=10, len_lo=1, len_hi=600, steps=9)
    got = run_gpu(dsve, torch_dev, base)
    ref = oracle_run(base)
    per = per_channel_rel_l1(got, ref, base.offsets)
    assert per.max() <= TOL


# ---------------------------------------------------------------------------
def test_launch_configuration_does_not_change_bits(torch_dev, dsve):
    wl = inputs.make_c4(n_channels=12, len_lo=100, len_hi=5000, steps=37)
    outs = []
    for launch in [(256, 0, 60), (64, 1, 0), (128, 2, 6), (256, 4, 12), (64, 8, 36), (192, 2, 18), (64, 128, 6)]:
        outs.append(run_gpu(dsve, torch_dev, wl, launch=launch))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_tile_runs_across_many_short_channels(torch_dev, dsve):
    # the per-step kernel (resident runs off) on 300 channels of 1-90 cells: a workgroup's run of
    # tiles crosses many channels, and a tile holds several whole channels; every launch gives the
    # same bits (runs of one tile per workgroup up to runs of hundreds) and matches the oracle
    wl = inputs.make_c4(n_channels=300, len_lo=1, len_hi=90, steps=23)
    outs = []
    for precision in ("fp64", "mixed"):
        runs = []
        for launch in [(64, 1, 0), (64, 3, 6), (256, 1, 0), (128, 7, 12), (64, 128, 6), (192, 2, 0)]:
            ctx = dsve.Context.from_workload(wl, precision=precision)
            ctx.set_resident(0)
            ctx.set_launch(*launch)
            h, q, z, t = dsve.upload(wl)
            ctx.adot_step(h, q, z, wl.steps, t)
            ctx.sync()
            runs.append(tuple(x.cpu().numpy() for x in (h, q, z, t)))
            ctx.close()
        for o in runs[1:]:
            for a, b in zip(o, runs[0]):
                assert np.array_equal(a, b)
        outs.append(runs[0])
    ref = oracle_run(wl)
    for got, tol in zip(outs, (TOL, 1e-5)):
        per = per_channel_rel_l1(got, ref, wl.offsets)
        assert per.max() <= tol, per.max()


def test_cfl_sub_slots_do_not_change_bits(torch_dev, dsve):
    # the per-channel CFL maximum merged into 1, 2 or 4 sub-slots, with one tile per
    # workgroup and with persistent workgroups, single channel and batched
    for wl in (inputs.make_c2(n_cells=150_000, steps=42),
               inputs.make_c4(n_channels=9, len_lo=100, len_hi=20_000, steps=42)):
        outs = []
        for launch in [(256, 64, 6), (128, 2, 0)]:
            for split in (1, 2, 4):
                outs.append(run_gpu(dsve, torch_dev, wl, launch=launch, split=split))
        for o in outs[1:]:
            for a, b in zip(o, outs[0]):
                assert np.array_equal(a, b)


def test_automatic_cfl_sub_slots(torch_dev, dsve):
    # many single-tile workgroups on one channel: 4 sub-slots; persistent workgroups, or
    # few workgroups per channel: 1
    ctx = dsve.Context.from_workload(inputs.make_c2(n_cells=1 << 20, steps=1))
    ctx.set_launch(256, 32, 60)
    assert ctx.get_cfl_split() == 4
    ctx.set_launch(256, 1, 60)
    assert ctx.get_cfl_split() == 1
    ctx.set_cfl_split(2)
    assert ctx.get_cfl_split() == 2
    ctx.close()
    ctx = dsve.Context.from_workload(inputs.make_c4(n_channels=64, len_lo=100, len_hi=400, steps=1))
    ctx.set_launch(256, 32, 60)
    assert ctx.get_cfl_split() == 1
    ctx.close()


def test_repeat_runs_are_bitwise_identical(torch_dev, dsve):
    wl = inputs.make_c2(n_cells=70_000, steps=66)
    a = run_gpu(dsve, torch_dev, wl)
    b = run_gpu(dsve, torch_dev, wl)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_split_run_equals_straight_run(torch_dev, dsve):
    # checkpoint/resume: k steps, copy state to host and back, k more == 2k straight
    torch = torch_dev
    wl = inputs.make_c1(steps=0)
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, 70, t)
    ctx.sync()
    saved = [x.cpu() for x in (h, q, z, t)]
    h2, q2, z2, t2 = (x.cuda() for x in saved)
    ctx.adot_step(h2, q2, z2, 70, t2)
    ctx.sync()
    h1, q1, z1, t1 = dsve.upload(wl)
    ctx.adot_step(h1, q1, z1, 140, t1)
    ctx.sync()
    for a, b in ((h1, h2), (q1, q2), (z1, z2)):
        assert torch.equal(a, b)
    assert abs(float(t1[0]) - float(t2[0])) <= 1e-14 * float(t1[0])
    ctx.close()


def test_zero_steps_is_a_no_op(torch_dev, dsve):
    wl = inputs.make_c1()
    got = run_gpu(dsve, torch_dev, wl, steps=0)
    assert np.array_equal(got[0], wl.h) and np.array_equal(got[2], wl.z) and got[3][0] == 0.0


# ---------------------------------------------------------------------------
def test_full_size_c2_autotuned_launch(torch_dev, dsve):
    # 2^20 cells, 66 steps (one 60-step graph replay and six direct launches) in the
    # launch the autotuner picks, as the benchmark runs it
    wl = inputs.make_c2()
    got = run_gpu(dsve, torch_dev, wl, steps=66, autotune=True)
    ref = oracle_run(wl, steps=66)
    assert max_rel_l1(got, ref) <= TOL


def test_full_size_c3_two_steps_fp64(torch_dev, dsve):
    wl = inputs.make_c3()
    got = run_gpu(dsve, torch_dev, wl, steps=2, precision="fp64", autotune=True)
    ref = oracle_run(wl, steps=2)
    assert max_rel_l1(got, ref) <= TOL


# ---------------------------------------------------------------------------
def test_nonfinite_state_is_reported(torch_dev, dsve):
    wl = inputs.make_c1(n_cells=300, steps=5)
    wl.h[17] = -0.5
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, 5, t)
    assert ctx.sync_status() == dsve.E_NONFINITE
    # sticky until cleared
    assert ctx.sync_status() == dsve.E_NONFINITE
    ctx.clear_error()
    h, q, z, t = dsve.upload(inputs.make_c1(n_cells=300, steps=5))
    ctx.adot_step(h, q, z, 5, t)
    ctx.sync()
    ctx.close()


def test_bad_launch_arguments(torch_dev, dsve):
    wl = inputs.make_c1()
    ctx = dsve.Context.from_workload(wl)
    for bad in [(96, 0, 60), (512, 0, 60), (256, -1, 60), (256, 1025, 60), (256, 0, 7)]:
        with pytest.raises(dsve.DsveError):
            ctx.set_launch(*bad)
        ctx.clear_error()
    for bad in (-1, 3, 8):
        with pytest.raises(dsve.DsveError):
            ctx.set_cfl_split(bad)
        ctx.clear_error()
    ctx.close()


def test_binding_refuses_wrong_sizes_before_launch(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_c1(n_cells=300, steps=5)
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    short = h[:-1].contiguous()
    f64 = dict(dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.adot_step(short, q, z, 5, t)
    with pytest.raises(ValueError):
        ctx.adot_step(h, q, z, 5, torch.zeros(0, **f64))
    with pytest.raises(ValueError):
        ctx.autotune(h, short, z)
    with pytest.raises(ValueError):
        ctx.cfl_reduce(h, q, z, torch.zeros(0, **f64), torch.zeros(1, **f64))
    E = wl.n_cells + 1
    with pytest.raises(ValueError):
        ctx.cell_update(torch.zeros(3, E - 1, **f64), torch.zeros(3, E, **f64),
                        torch.zeros(1, **f64), h, q, z)
    with pytest.raises(ValueError):
        ctx.dot_edge_fluct(*[torch.ones(8, **f64)] * 5, torch.ones(7, **f64),
                           torch.zeros(3, 8, **f64), torch.zeros(3, 8, **f64))
    with pytest.raises(ValueError):
        ctx.dot_edge_fluct(*[torch.ones(8, **f64)] * 6, torch.zeros(3, 7, **f64),
                           torch.zeros(3, 8, **f64))
    # nothing was enqueued; the context still runs
    ctx.adot_step(h, q, z, 5, t)
    ctx.sync()
    ctx.close()


@pytest.mark.parametrize("resident", [0, 1])
def test_runs_write_only_the_callers_arrays(torch_dev, dsve, resident):
    # ragged batched channels, an odd step count (ends with the copy back); the caller's
    # arrays are views into padded buffers whose padding must stay untouched
    torch = torch_dev
    wl = inputs.make_c4(n_channels=5, len_lo=100, len_hi=400, steps=7)
    ctx = dsve.Context.from_workload(wl)
    ctx.set_resident(resident)
    assert ctx.get_resident() == (resident == 0)
    pad = 256
    bufs = []
    for a in (wl.h, wl.q, wl.z, np.zeros(wl.n_channels)):
        b = torch.full((a.size + 2 * pad,), 7.0, dtype=torch.float64, device="cuda")
        b[pad:pad + a.size] = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        bufs.append(b)
    h, q, z, t = (b[pad:-pad] for b in bufs)
    ctx.adot_step(h, q, z, wl.steps, t)
    ctx.sync()
    for b in bufs:
        assert torch.all(b[:pad] == 7.0) and torch.all(b[-pad:] == 7.0)
    got = tuple(x.cpu().numpy() for x in (h, q, z, t))
    ref = oracle_run(wl)
    assert per_channel_rel_l1(got, ref, wl.offsets).max() <= TOL
    np.testing.assert_allclose(got[3], ref[3], rtol=1e-13)
    ctx.close()


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coalescing_roots_are_reported(torch_dev, dsve, precision):
    # a fixed bed at Fr = 1 (g = 4, h = 1, q = 2: every quantity exact, arccos argument 1): two
    # roots coincide and R^-1 does not exist; the oracle reports the same edges (its pins)
    torch = torch_dev
    n = 100
    f64 = dict(dtype=torch.float64, device="cuda")
    ctx = dsve.Context.single(16, g=4.0, porosity=0.0, A_g=0.0, dx=1.0, precision=precision)
    one, two = torch.ones(n, **f64), torch.full((n,), 2.0, **f64)
    Dm, Dp = torch.zeros(3, n, **f64), torch.zeros(3, n, **f64)
    ctx.dot_edge_fluct(one, two, torch.zeros(n, **f64), one, two, torch.full((n,), 0.1, **f64), Dm, Dp)
    assert ctx.sync_status() == dsve.E_NONHYPERBOLIC
    assert "coalescing" in ctx.last_error()
    ctx.close()
    # a movable bed at the same states: no error
    ctx = dsve.Context.single(16, g=4.0, porosity=0.0, A_g=0.01, dx=1.0, precision=precision)
    ctx.dot_edge_fluct(one, two, torch.zeros(n, **f64), one, two, torch.full((n,), 0.1, **f64), Dm, Dp)
    ctx.sync()
    assert torch.all(torch.isfinite(Dm)) and torch.all(torch.isfinite(Dp))
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fixed_bed_next_to_coalescence_is_reported_or_bounded(torch_dev, dsve, precision):
    # Fr = 1 +- 1e-9 over a fixed bed: the roots differ by 1e-9 c, below what the arccos argument
    # resolves; each edge is either reported (roots equal to working precision) or finite and
    # bounded by the size of its jump (|D| <= |A| |dW| ~ c^2 |dz|), never huge numbers
    torch = torch_dev
    n = 64
    f64 = dict(dtype=torch.float64, device="cuda")
    q = torch.tensor([2.0 * (1.0 + (1e-9 if k % 2 else -1e-9)) for k in range(n)], **f64)
    one = torch.ones(n, **f64)
    Dm, Dp = torch.zeros(3, n, **f64), torch.zeros(3, n, **f64)
    ctx = dsve.Context.single(16, g=4.0, porosity=0.0, A_g=0.0, dx=1.0, precision=precision)
    ctx.dot_edge_fluct(one, q, torch.zeros(n, **f64), one, q, torch.full((n,), 0.1, **f64), Dm, Dp)
    st = ctx.sync_status()
    if st == dsve.OK:
        assert torch.all(torch.isfinite(Dm)) and torch.all(torch.isfinite(Dp))
        assert float(torch.max(torch.abs(Dm))) < 10.0 and float(torch.max(torch.abs(Dp))) < 10.0
    else:
        assert st == dsve.E_NONHYPERBOLIC
    ctx.close()


def test_overflowed_state_is_reported_as_nonfinite(torch_dev, dsve):
    # g h^3 overflows: the arccos argument is NaN, which the clamp would otherwise turn into -1
    torch = torch_dev
    n = 64
    f64 = dict(dtype=torch.float64, device="cuda")
    h = torch.full((n,), 1e110, **f64)
    Dm, Dp = torch.zeros(3, n, **f64), torch.zeros(3, n, **f64)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=0.01, dx=1.0)
    ctx.dot_edge_fluct(h, h, torch.zeros(n, **f64), torch.ones(n, **f64), torch.ones(n, **f64),
                       torch.zeros(n, **f64), Dm, Dp)
    assert ctx.sync_status() == dsve.E_NONFINITE
    ctx.close()
