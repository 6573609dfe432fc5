"""Long runs at full size on the HIP path against the CPU oracle (MI355X), in the launch the
autotuner picks, as the benchmark runs them.

* c3 (transcritical flow over a bed bump, 2^24 cells) for 200 steps in both forms, against one
  oracle run of the same 200 steps (about a minute of the oracle on 16 host threads);
* the printed initial states of the paper's Test 1 (Sec. 4.1, Eq. murillo; tests/golden/
  riemann_test1.json) on its five A-DOT grids up to t_end = 1.5 s, in both forms.
"""
import json
import os

import numpy as np
import pytest

from paper_1912_04791_amd import inputs

from common import max_rel_l1, oracle_run, spec_of

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def run_gpu(dsve, wl, steps, precision, autotune=False):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    h, q, z, t = dsve.upload(wl)
    if autotune:
        ctx.autotune(h, q, z, trial_steps=20)
    ctx.adot_step(h, q, z, steps, t)
    ctx.sync()
    out = (h.cpu().numpy(), q.cpu().numpy(), z.cpu().numpy(), t.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.timeout(900)
def test_full_size_c3_200_steps_both_forms(torch_dev, dsve):
    wl = inputs.make_c3()
    steps = 200
    got = {p: run_gpu(dsve, wl, steps, p, autotune=True) for p in ("fp64", "mixed")}
    ref = oracle_run(wl, steps=steps)
    e64, emx = max_rel_l1(got["fp64"], ref), max_rel_l1(got["mixed"], ref)
    print(f"c3 2^24 cells, {steps} steps: relative L1 FP64 {e64:.3g}, mixed {emx:.3g}; "
          f"t {got['fp64'][3][0]:.9g} (oracle {ref[3][0]:.9g})")
    assert e64 <= 1e-12 and emx <= 1e-5
    assert abs(got["fp64"][3][0] - ref[3][0]) <= 1e-12 * ref[3][0]


def paper_test1_workload(n_cells):
    d = json.load(open(os.path.join(HERE, "golden", "riemann_test1.json")))
    L, xj = d["L"], d["x_jump"]
    # xi = 1 / (1 - porosity) = 1 (Sec. 4.1)
    assert d["xi"] == 1.0
    return inputs.make_riemann(n_cells, L, xj, d["left"], d["right"], A_g=d["A_g"], porosity=0.0,
                               steps=0), d["t_end"]


@pytest.mark.parametrize("n_cells", [500, 750, 1000, 1500, 3000])
def test_paper_test1_states_to_t_end(torch_dev, dsve, n_cells):
    import oracle
    wl, t_end = paper_test1_workload(n_cells)
    # the oracle's run fixes the step count: the first step whose end reaches t_end (twice the
    # steps the initial speeds need bound it)
    speed = np.max(np.abs(wl.q / wl.h) + np.sqrt(wl.g * wl.h))
    bound = int(2 * t_end / (wl.cfl * wl.dx[0] / speed)) + 10
    dts = oracle.run(spec_of(wl), wl.h, wl.q, wl.z, bound, return_dt=True)[4]
    assert np.sum(dts) >= t_end
    steps = int(np.searchsorted(np.cumsum(dts), t_end) + 1)
    ref = oracle_run(wl, steps=steps)
    assert ref[3][0] >= t_end and ref[3][0] - dts[steps - 1] < t_end
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        got = run_gpu(dsve, wl, steps, precision)
        err = max_rel_l1(got, ref)
        print(f"Test 1, {n_cells} cells, {steps} steps to t = {ref[3][0]:.6f} s: {precision} "
              f"relative L1 {err:.3g}")
        assert err <= tol
        assert abs(got[3][0] - ref[3][0]) <= (1e-12 if precision == "fp64" else 1e-6) * ref[3][0]
    # the bed moved at the jump and the water left the channel's middle
    assert np.max(np.abs(got[2] - wl.z)) > 1e-3


@pytest.mark.timeout(600)
def test_c2_mixed_error_is_far_below_the_discretisation_error(torch_dev, dsve):
    # "at equal accuracy": c2 (2^20 cells, 1000 steps) in both forms against a proxy of the
    # scheme's own error, the difference between the 2^20-cell solution and the 2^21-cell one
    # (the same initial functions sampled finer, 2000 steps, restricted by averaging cell pairs).
    # The FP64 form equals the oracle to about 2e-15 over these steps (bench.py checks it in
    # every run), so it stands in for the oracle here.  Measured: proxy 1.3e-8, 2.8e-7, 2.4e-9
    # against mixed 2.8e-10, 1.3e-9, 8.9e-11 (h, q, z): the mixed form's error is 27-200 times
    # below the proxy; the bar asks for 10.
    from common import l1_scales, rel_l1
    wl = inputs.make_c2()
    fine = inputs.make_c2(n_cells=2 << 20, steps=2000)
    a = run_gpu(dsve, wl, wl.steps, "fp64")
    m = run_gpu(dsve, wl, wl.steps, "mixed")
    b = run_gpu(dsve, fine, fine.steps, "fp64")
    restricted = [0.5 * (v[0::2] + v[1::2]) for v in b[:3]]
    disc = [rel_l1(r, x, sc) for r, x, sc in zip(restricted, a[:3], l1_scales(a[0]))]
    mixed = [rel_l1(y, x, sc) for y, x, sc in zip(m[:3], a[:3], l1_scales(a[0]))]
    print(f"c2: t {a[3][0]:.6f} s (2^21 cells: {b[3][0]:.6f} s); relative L1 per variable h, q, z: "
          f"discretisation proxy {disc[0]:.3g} {disc[1]:.3g} {disc[2]:.3g}; mixed vs FP64 "
          f"{mixed[0]:.3g} {mixed[1]:.3g} {mixed[2]:.3g}")
    assert max(mixed) <= 1e-5
    assert all(mx <= 0.1 * d for mx, d in zip(mixed, disc))
