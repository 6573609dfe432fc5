"""Channel-resident runs on the MI355X: every channel of at most 511 cells held by one
workgroup (256 threads, or 512 past 255 cells) for all steps of a run.  The results must be bitwise those of the per-step kernels
(same arithmetic in the same order), and match the oracle to the FP64 / mixed bars.
"""
import numpy as np
import pytest

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


def run(dsve, wl, precision="fp64", resident=0, steps=None, solver="adot"):
    ctx = dsve.Context.from_workload(wl, precision=precision, solver=solver)
    ctx.set_resident(resident)
    assert ctx.get_resident() == (resident == 0)
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, wl.steps if steps is None else steps, t)
    ctx.sync()
    out = tuple(x.cpu().numpy() for x in (h, q, z, t))
    ctx.close()
    return out


def short(name):
    if name == "c1":
        return inputs.make_c1(steps=200)
    if name == "c1_255":
        return inputs.make_c1(n_cells=255, steps=37)
    if name == "c1_1":
        return inputs.make_c1(n_cells=1, steps=9)
    if name == "c1_256":
        return inputs.make_c1(n_cells=256, steps=41)
    if name == "c1_511":
        return inputs.make_c1(n_cells=511, steps=23)
    if name == "ragged_511":
        return inputs.make_c4(n_channels=30, len_lo=200, len_hi=511, steps=19)
    if name == "periodic":
        return inputs.make_c2(n_cells=255, steps=61)
    if name == "ragged":
        return inputs.make_c4(n_channels=40, len_lo=1, len_hi=255, steps=33)
    if name == "soni":
        return inputs.make_soni(n_channels=12, len_lo=40, len_hi=255, steps=80)
    if name == "bellal_mpm":
        return inputs.make_bellal("mpm", n_channels=12, len_lo=40, len_hi=255, steps=60)
    if name == "bellal_vanrijn":
        return inputs.make_bellal("vanrijn", n_channels=12, len_lo=40, len_hi=255, steps=60)
    if name == "berthon":
        return inputs.make_berthon(200, steps=150)
    raise KeyError(name)


CASES = ["c1", "c1_255", "c1_1", "c1_256", "c1_511", "ragged_511", "periodic", "ragged", "soni", "bellal_mpm",
         "bellal_vanrijn", "berthon"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_resident_equals_per_step_kernels_bitwise(torch_dev, dsve, name, precision):
    wl = short(name)
    a = run(dsve, wl, precision, resident=0)
    b = run(dsve, wl, precision, resident=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["c1", "ragged", "ragged_511", "soni", "berthon"])
def test_resident_matches_oracle(torch_dev, dsve, name):
    wl = short(name)
    ref = oracle_run(wl)
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        got = run(dsve, wl, precision, resident=0)
        per = per_channel_rel_l1(got, ref, wl.offsets)
        assert per.max() <= tol, (precision, per.max())
        np.testing.assert_allclose(got[3], ref[3], rtol=1e-12 if precision == "fp64" else 1e-6)


def test_resident_dot_solver_bitwise(torch_dev, dsve):
    wl = short("ragged")
    a = run(dsve, wl, "fp64", resident=0, solver="dot")
    b = run(dsve, wl, "fp64", resident=1, solver="dot")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert max_rel_l1(a, oracle_run(wl)) <= 1e-12


def test_resident_one_step_and_split_runs(torch_dev, dsve):
    torch = torch_dev
    wl = short("ragged")
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    for n in (1, 4, 28):          # 33 steps in three runs
        ctx.adot_step(h, q, z, n, t)
    ctx.sync()
    h2, q2, z2, t2 = dsve.upload(wl)
    ctx.adot_step(h2, q2, z2, 33, t2)
    ctx.sync()
    for x, y in ((h, h2), (q, q2), (z, z2), (t, t2)):
        assert torch.equal(x, y)
    ctx.close()


def test_resident_eligibility(torch_dev, dsve):
    ctx = dsve.Context.from_workload(inputs.make_c1(n_cells=255))
    assert ctx.get_resident()
    ctx.set_resident(1)
    assert not ctx.get_resident()
    with pytest.raises(dsve.DsveError):
        ctx.set_resident(2)
    ctx.clear_error()
    ctx.close()
    ctx = dsve.Context.from_workload(inputs.make_c1(n_cells=511))
    assert ctx.get_resident()
    ctx.close()
    ctx = dsve.Context.from_workload(inputs.make_c1(n_cells=512))
    assert not ctx.get_resident()
    ctx.close()
    wl = inputs.make_c4(n_channels=8, len_lo=10, len_hi=700, steps=1)
    ctx = dsve.Context.from_workload(wl)
    assert ctx.get_resident() == bool(wl.lengths().max() <= 511)
    ctx.close()


def test_resident_reports_nonfinite(torch_dev, dsve):
    wl = inputs.make_c1(n_cells=200, steps=5)
    wl.h[17] = -0.5
    ctx = dsve.Context.from_workload(wl)
    assert ctx.get_resident()
    h, q, z, t = dsve.upload(wl)
    ctx.adot_step(h, q, z, 5, t)
    assert ctx.sync_status() == dsve.E_NONFINITE
    ctx.close()


def test_autotune_chooses_between_resident_and_per_step(torch_dev, dsve, tmp_path):
    import json
    wl = inputs.make_c4(n_channels=600, len_lo=20, len_hi=255, steps=24)
    ref = run(dsve, wl, "fp64", resident=1)
    ctx = dsve.Context.from_workload(wl)
    h, q, z, t = dsve.upload(wl)
    cache = str(tmp_path / "tune.json")
    ctx.autotune(h, q, z, trial_steps=12, cache_path=cache)
    chosen = ctx.get_resident()
    entry = json.loads(open(cache).read().splitlines()[0])
    assert entry["resident_mode"] == (0 if chosen else 1)
    ctx.adot_step(h, q, z, wl.steps, t)
    ctx.sync()
    for x, y in zip((h, q, z, t), ref):
        assert np.array_equal(x.cpu().numpy(), y)
    # the cached choice is restored without tuning
    ctx2 = dsve.Context.from_workload(wl)
    ctx2.autotune(h, q, z, trial_steps=12, cache_path=cache)
    assert ctx2.get_resident() == chosen
    ctx.close()
    ctx2.close()
