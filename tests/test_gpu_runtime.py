"""Runtime pieces of the HIP path on the MI355X: autotuner and its cache, HIP-graph reuse
and re-capture, streams, full-size batched runs checked on sampled channels.

Channels are independent, so comparing whole channels of a full-size batched run with the
oracle run on just those channels is exact sampling.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1912_04791_amd import inputs

from common import max_rel_l1, oracle_run, per_channel_rel_l1

pytestmark = pytest.mark.gpu


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


def to_np(*ts):
    return tuple(t.cpu().numpy() for t in ts)


def test_autotune_keeps_results_and_writes_cache(torch_dev, dsve, tmp_path):
    wl = inputs.make_c4(n_channels=24, len_lo=200, len_hi=6000, steps=30)
    cache = str(tmp_path / "tune.json")
    ref_ctx = dsve.Context.from_workload(wl)
    h0, q0, z0, t0 = dsve.upload(wl)
    ref_ctx.adot_step(h0, q0, z0, wl.steps, t0)
    ref_ctx.sync()

    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    before = [x.clone() for x in (h, q, z)]
    ctx.autotune(h, q, z, trial_steps=4, cache_path=cache)
    # the caller's arrays are read, never written
    for a, b in zip(before, (h, q, z)):
        assert torch_dev.equal(a, b)
    launch = ctx.get_launch()
    assert launch[0] in (64, 128, 192, 256) and 0 <= launch[1] <= 128
    lines = [json.loads(l) for l in open(cache).read().splitlines() if l.strip()]
    assert len(lines) == 1 and lines[0]["tile"] == launch[0]
    assert lines[0]["blocks_per_cu"] == launch[1]
    assert lines[0]["cfl_split"] in (0, 1, 4)
    ctx.adot_step(h, q, z, wl.steps, t)
    ctx.sync()
    for a, b in zip(to_np(h, q, z, t), to_np(h0, q0, z0, t0)):
        assert np.array_equal(a, b)

    # a second context finds the cached choice without tuning
    ctx2 = dsve.Context.from_workload(wl)
    ctx2.set_launch(64, 1, 12)
    ctx2.autotune(h, q, z, trial_steps=4, cache_path=cache)
    assert ctx2.get_launch()[:2] == launch[:2]
    assert ctx2.get_cfl_split() == ctx.get_cfl_split()
    for c in (ref_ctx, ctx, ctx2):
        c.close()


def test_autotune_reports_pending_error_first(torch_dev, dsve):
    # a run on a state with a negative depth, enqueued and not yet synchronised: the
    # autotuner waits for it and returns its deferred error before any trial
    wl = inputs.make_c1(n_cells=300, steps=5)
    wl.h[17] = -0.5
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    launch = tuple(ctx.get_launch())
    ctx.adot_step(h, q, z, 5, t)
    with pytest.raises(dsve.DsveError) as err:
        ctx.autotune(h, q, z, trial_steps=4)
    assert err.value.status == dsve.E_NONFINITE
    assert tuple(ctx.get_launch()) == launch
    ctx.close()


@pytest.mark.parametrize("resident", [0, 1])
def test_autotune_trials_leave_no_error_behind(torch_dev, dsve, resident):
    # tuned on a state that is not finite: the trial runs meet it, but only the caller's own
    # runs after tuning are reported
    wl = inputs.make_c1(n_cells=300, steps=5)
    ctx = dsve.Context.from_workload(wl)
    ctx.set_resident(resident)
    good = dsve.upload(wl)
    wl.h[17] = -0.5
    bad = dsve.upload(wl)
    ctx.autotune(*bad[:3], trial_steps=4)
    assert ctx.sync_status() == dsve.OK
    ctx.adot_step(*good[:3], 5, good[3])
    ctx.sync()
    ref = oracle_run(inputs.make_c1(n_cells=300, steps=5))
    assert max_rel_l1(to_np(*good), ref) <= 1e-12
    ctx.adot_step(*bad[:3], 5, bad[3])
    assert ctx.sync_status() == dsve.E_NONFINITE
    ctx.close()


def test_graph_recaptured_for_new_buffers(torch_dev, dsve):
    wl = inputs.make_c2(n_cells=40_000, steps=120)
    ctx = dsve.Context.from_workload(wl)
    ctx.set_launch(256, 0, 60)
    a = dsve.upload(wl)
    b = dsve.upload(wl)
    ctx.adot_step(*a[:3], 120, a[3])       # captures a graph for buffers a
    ctx.adot_step(*b[:3], 60, b[3])        # different buffers: a new graph
    ctx.adot_step(*b[:3], 60, b[3])        # reuses it
    ctx.sync()
    for x, y in zip(to_np(*a), to_np(*b)):
        assert np.array_equal(x, y)
    ref = oracle_run(wl, steps=120)
    assert max_rel_l1(to_np(*a), ref) <= 1e-12
    ctx.close()


def test_non_default_stream(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_c1()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = dsve.Context.from_workload(wl, stream=s)
        h, q, z, t = dsve.upload(wl)
        ctx.adot_step(h, q, z, wl.steps, t)
        ctx.sync()
    ref = oracle_run(wl)
    assert max_rel_l1(to_np(h, q, z), ref) <= 1e-12
    ctx.close()


def test_cfl_reduce_mixed(torch_dev, dsve):
    torch = torch_dev
    wl = inputs.make_c3(n_cells=100_003)
    ctx = dsve.Context.from_workload(wl, precision="mixed")
    h, q, z, _ = dsve.upload(wl)
    amax = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros_like(amax)
    ctx.cfl_reduce(h, q, z, amax, dt)
    ctx.sync()
    ref = oracle.cfl_amax(wl.h, wl.q, wl.z, 9.81, 1.0 / (1 - wl.porosity[0]), wl.Ag[0])
    assert abs(float(amax[0]) - ref) <= 1e-6 * ref
    ctx.close()


def _sampled_channels_check(dsve, wl, precision, tol, every, launch=None):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    h, q, z, t = dsve.upload(wl)
    if launch is None:
        ctx.autotune(h, q, z, trial_steps=20)   # the launch the benchmark times
    else:
        ctx.set_launch(*launch)
    ctx.adot_step(h, q, z, wl.steps, t)
    ctx.sync()
    got = to_np(h, q, z, t)
    ctx.close()
    chans = np.arange(0, wl.n_channels, every)
    sub = wl.subset(chans)
    ref = oracle_run(sub)
    lo = wl.offsets[chans]
    hi = wl.offsets[chans + 1]
    sel = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    got_sub = tuple(g[sel] for g in got[:3])
    per = per_channel_rel_l1(got_sub, ref, sub.offsets)
    assert per.max() <= tol, (per.max(), chans[per.argmax()])
    np.testing.assert_allclose(got[3][chans], ref[3], rtol=1e-12 if precision == "fp64" else 1e-5)


def test_full_size_c4_fp64_sampled_channels(torch_dev, dsve):
    # all 4096 channels (4.8e7 cells) for the full 500 steps; 16 channels checked
    wl = inputs.make_c4()
    _sampled_channels_check(dsve, wl, "fp64", 1e-12, every=256)


def test_full_size_c5_mixed_sampled_channels(torch_dev, dsve):
    # all 65536 channels (1.5e8 cells) for the full 5000 steps; 32 channels checked
    wl = inputs.make_c5()
    assert wl.steps == 5000
    _sampled_channels_check(dsve, wl, "mixed", 1e-5, every=2048)


def test_full_size_c5_fp64_sampled_channels(torch_dev, dsve):
    # the same run in FP64; 16 channels checked
    wl = inputs.make_c5()
    _sampled_channels_check(dsve, wl, "fp64", 1e-12, every=4096)


def test_wide_index_path_sampled_channels(torch_dev, dsve):
    # 2^14 channels of 2^15 cells: 2^29 cells and 2^29 + 2^14 edges, past the range of the
    # step kernel's 32-bit indexing, so the 64-bit form runs; 3 steps, 8 channels checked
    wl = inputs.make_c4(n_channels=16384, len_lo=32768, len_hi=32768, steps=3)
    assert wl.n_cells + wl.n_channels >= 2 ** 29
    _sampled_channels_check(dsve, wl, "fp64", 1e-12, every=2048, launch=(256, 32, 0))


def test_pairwise_fluct_past_32_bit_offsets(torch_dev, dsve):
    # 2^30 + 7 edges: row 2 of the fluctuations starts past element 2^31 (byte 2^34), so every
    # offset of that row needs 64-bit arithmetic; about 103 GB of device memory.  The edge states
    # come from a seeded device generator (the recipe of make_random_edges); 4096 sampled edges
    # are checked against the oracle at the FP64 bar.
    torch = torch_dev
    n = (1 << 30) + 7
    f64 = dict(dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(1234)
    def uni(lo, hi):
        return torch.rand(n, generator=gen, **f64) * (hi - lo) + lo
    hL = uni(0.05, 5.0)
    uL = uni(-3.0, 3.0)
    zL = uni(-1.0, 1.0)
    hR = hL * (1.0 + 0.3 * uni(-1.0, 1.0))
    uR = uL + 0.3 * uni(-1.0, 1.0)
    zR = zL + 0.3 * uni(-1.0, 1.0)
    qL = hL * uL
    del uL
    qR = hR * uR
    del uR
    Dm = torch.empty(3, n, **f64)
    Dp = torch.empty(3, n, **f64)
    ctx = dsve.Context.single(16, porosity=0.4, A_g=0.02, dx=1.0)
    ctx.dot_edge_fluct(hL, qL, zL, hR, qR, zR, Dm, Dp)
    ctx.sync()
    ctx.close()
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.integers(0, n, 4000), np.arange(n - 96, n)]))
    ti = torch.from_numpy(idx).cuda()
    WL = tuple(a[ti].cpu().numpy() for a in (hL, qL, zL))
    WR = tuple(a[ti].cpu().numpy() for a in (hR, qR, zR))
    gm, gp = Dm[:, ti].cpu().numpy(), Dp[:, ti].cpu().numpy()
    del hL, qL, zL, hR, qR, zR, Dm, Dp, ti
    torch.cuda.empty_cache()
    rm, rp = oracle.fluct(WL, WR, 9.81, 1.0 / 0.6, 0.02)
    for got, ref in ((gm, rm), (gp, rp)):
        assert np.abs(got - ref).sum() <= 1e-12 * np.abs(ref).sum()


@pytest.mark.parametrize("where", ["middle", "last"])
def test_cfl_reduce_past_32_bit_cell_indices(torch_dev, dsve, where):
    # 2^31 + 3 cells of one state, with one faster cell planted past index 2^31: the maximum is
    # that cell's speed, whatever the kernel's ranges and their 64-bit arithmetic (about 103 GB
    # of device memory with the context's own copy of the state)
    torch = torch_dev
    N = (1 << 31) + 3
    f64 = dict(dtype=torch.float64, device="cuda")
    h = torch.full((N,), 1.0, **f64)
    q = torch.full((N,), 0.5, **f64)
    z = torch.zeros(N, **f64)
    k = (1 << 31) + 1 if where == "middle" else N - 1
    h[k], q[k] = 2.0, 3.0
    ctx = dsve.Context.single(N, porosity=0.4, A_g=0.01, dx=1.0)
    amax, dt = torch.zeros(1, **f64), torch.zeros(1, **f64)
    ctx.cfl_reduce(h, q, z, amax, dt)
    ctx.sync()
    ctx.close()
    del h, q, z
    torch.cuda.empty_cache()
    xi = 1.0 / 0.6
    base = oracle.cfl_amax(np.array([1.0]), np.array([0.5]), np.array([0.0]), 9.81, xi, 0.01)
    fast = oracle.cfl_amax(np.array([2.0]), np.array([3.0]), np.array([0.0]), 9.81, xi, 0.01)
    assert fast > base
    assert abs(float(amax[0]) - fast) <= 1e-14 * fast


@pytest.mark.parametrize("graph_steps,n", [(60, 5), (60, 20), (60, 59), (60, 60), (60, 61),
                                           (60, 125), (6, 20), (6, 7)])
def test_every_step_replays_a_graph(torch_dev, dsve, graph_steps, n):
    # a run of n steps replays n // graph_steps full graphs and one graph of the remaining
    # steps; bitwise the same as launching every step directly
    wl = inputs.make_c4(n_channels=7, len_lo=600, len_hi=3000, steps=n)
    outs = []
    for gs in (graph_steps, 0):
        ctx = dsve.Context.from_workload(wl)
        ctx.set_launch(256, 2, gs)
        h, q, z, t = dsve.upload(wl)
        ctx.adot_step(h, q, z, n, t)
        ctx.sync()
        launches, gsteps, direct = ctx.last_run()
        if gs:
            assert (launches, gsteps, direct) == (n // gs + (1 if n % gs else 0), n, 0)
        else:
            assert (launches, gsteps, direct) == (0, 0, n)
        outs.append(to_np(h, q, z, t))
        ctx.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_prepared_run_replays_without_capture(torch_dev, dsve):
    # graphs captured ahead for a run length are reused by that run; other lengths still run
    wl = inputs.make_c2(n_cells=20_000, steps=23)
    ctx = dsve.Context.from_workload(wl)
    ctx.set_launch(256, 4, 12)
    h, q, z, t = dsve.upload(wl)
    ctx.prepare_run(h, q, z, 23, t)
    ctx.adot_step(h, q, z, 23, t)
    ctx.sync()
    assert ctx.last_run() == (2, 23, 0)
    ctx.adot_step(h, q, z, 5, t)
    ctx.sync()
    assert ctx.last_run() == (1, 5, 0)
    ref = oracle_run(wl, steps=28)
    assert max_rel_l1(to_np(h, q, z, t), ref) <= 1e-12
    ctx.close()
