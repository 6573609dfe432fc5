"""The allocation-free entry point adot_step_noalloc against adot_step / adot_step_batched,
through the C ABI (MI355X): bit-for-bit equal results on two calls in a row, the second on a
smaller input, for the per-step kernels and the channel-resident ones, in both precisions; the
largest context it accepts, and a larger one refused before any launch."""
import numpy as np
import pytest

from paper_1912_04791_amd import inputs

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


def run(dsve, wl, precision, noalloc):
    ctx = dsve.Context.from_workload(wl, precision=precision)
    h, q, z, t = dsve.upload(wl)
    (ctx.adot_step_noalloc if noalloc else ctx.adot_step)(h, q, z, wl.steps, t)
    ctx.sync()
    out = tuple(a.cpu().numpy() for a in (h, q, z, t))
    resident = ctx.get_resident()
    ctx.close()
    return out, resident


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["per_step", "resident"])
def test_noalloc_equals_adot_step_twice_second_smaller(torch_dev, dsve, precision, kind):
    if kind == "per_step":
        shapes = [dict(n_channels=12, len_lo=600, len_hi=20_000, steps=37),
                  dict(n_channels=5, len_lo=600, len_hi=3000, steps=22)]
    else:
        shapes = [dict(n_channels=300, len_lo=64, len_hi=511, steps=41),
                  dict(n_channels=40, len_lo=16, len_hi=255, steps=16)]
    for k, shp in enumerate(shapes):
        wl = inputs.make_c4(**shp)
        got, res_got = run(dsve, wl, precision, noalloc=True)
        ref, res_ref = run(dsve, wl, precision, noalloc=False)
        assert res_got == res_ref == (kind == "resident")
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (k, shp)


def test_noalloc_largest_context_and_a_larger_one_refused(torch_dev, dsve):
    wl = inputs.make_c2(n_cells=1 << 20, steps=7)
    got, _ = run(dsve, wl, "fp64", noalloc=True)
    ref, _ = run(dsve, wl, "fp64", noalloc=False)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    big = inputs.make_c2(n_cells=(1 << 20) + 1, steps=2)
    ctx = dsve.Context.from_workload(big)
    h, q, z, t = dsve.upload(big)
    with pytest.raises(dsve.DsveError) as ex:
        ctx.adot_step_noalloc(h, q, z, 2, t)
    assert ex.value.status == dsve.E_ARG and "static scratch" in str(ex.value)
    ctx.close()
