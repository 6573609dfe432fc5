"""The seeded synthetic workloads: sizes, determinism, per-channel fields, and the stated values
of the paper's cases in the single-channel forms (Secs. 4.1, 4.2, 5.1, 5.2)."""
import numpy as np
import pytest

from paper_1912_04791_amd import inputs


@pytest.mark.parametrize("name,kw", [
    ("c4", dict(n_channels=40, len_hi=900)),
    ("c5", dict(n_channels=40, len_lo=64, len_hi=300)),
    ("soni", dict(n_channels=30, len_lo=64, len_hi=300)),
    ("bellal_mpm", dict(n_channels=30, len_lo=64, len_hi=300)),
])
def test_batched_workloads_are_seeded_and_consistent(name, kw):
    a = inputs.MAKERS[name](**kw)
    b = inputs.MAKERS[name](**kw)
    for f in ("h", "q", "z", "offsets", *inputs.PER_CHANNEL):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    C = a.n_channels
    assert a.offsets[0] == 0 and np.all(np.diff(a.offsets) > 0) and a.offsets[-1] == a.h.size
    for f in inputs.PER_CHANNEL:
        assert getattr(a, f).shape[0] == C, f
    assert np.all(a.h > 0) and np.all(np.isfinite(a.q)) and np.all(np.isfinite(a.z))


def test_subset_and_channel_keep_every_per_channel_field():
    wl = inputs.make_bellal("vanrijn", n_channels=12, len_lo=50, len_hi=200)
    sub = wl.subset([3, 7, 11])
    for j, c in enumerate([3, 7, 11]):
        for f in inputs.PER_CHANNEL:
            assert np.array_equal(getattr(sub, f)[j], getattr(wl, f)[c]), f
        one = wl.channel(c)
        lo, hi = wl.offsets[c], wl.offsets[c + 1]
        assert np.array_equal(one.h, wl.h[lo:hi]) and one.law == wl.law


def test_soni_single_channel_has_the_stated_values():
    wl = inputs.make_soni(n_channels=1)
    assert wl.n_cells == 100 and abs(wl.dx[0] * 100 - 30.0) < 1e-12
    assert np.allclose(wl.h, 0.05) and np.allclose(wl.q, 0.02)
    x = (np.arange(100) + 0.5) * 0.3
    assert np.allclose(wl.z, 1.2 - 3.56e-3 * x)
    assert wl.law == inputs.LAW_POWER and wl.law_par[0, 0] == 5.0 and wl.Ag[0] == 1.45e-3
    assert wl.ks[0] == 49.4 and wl.porosity[0] == 0.4
    # the power law carries five times the equilibrium solid discharge at the inflow depth
    u0, uin = 0.02 / 0.05, 0.02 / wl.h_in[0]
    assert abs(uin ** 5 / u0 ** 5 - 5.0) < 1e-12
    assert wl.bc_left[0] == inputs.BC_INFLOW_QH and wl.bc_right[0] == inputs.BC_FIXED_DEPTH
    assert wl.h_out[0] == 0.05


def test_bellal_single_channel_has_the_stated_values():
    wl = inputs.make_bellal("mpm", n_channels=1)
    assert wl.n_cells == 200 and abs(wl.dx[0] * 200 - 6.9) < 1e-12
    assert np.allclose(wl.q, 0.024) and wl.h_out[0] == 0.2093 and wl.ks[0] == 62.0
    assert tuple(wl.law_par[0, :2]) == (1.65e-3, 2.6) and wl.porosity[0] == 0.42
    # uniform flow: friction slope equals the bed slope at the initial depth
    sf = 0.024 ** 2 / (62.0 ** 2 * wl.h[0] ** (10.0 / 3.0))
    assert abs(sf - 0.0302) < 1e-12
    thr = inputs.make_bellal("thr", n_channels=1)
    assert thr.Ag[0] == 0.0024 and thr.law_par[0, 0] == 0.3


def test_berthon_initial_state_and_ghosts_are_the_exact_solution():
    wl = inputs.make_berthon(64)
    h, q, z = inputs.berthon_exact(wl.meta["x"], 0.0)
    assert np.array_equal(wl.h, h) and np.array_equal(wl.q, q) and np.array_equal(wl.z, z)
    dx = 7.0 / 64
    gh, gq, gz = inputs.berthon_exact(np.array([-0.5 * dx, 7.0 + 0.5 * dx]), 0.0)
    assert np.allclose(wl.dir_left[0], [gh[0], gq[0], gz[0], -0.005])
    assert np.allclose(wl.dir_right[0], [gh[1], gq[1], gz[1], -0.005])
    # the bed falls at the rate alpha and the flow is steady (Eq. berthon)
    h1, q1, z1 = inputs.berthon_exact(wl.meta["x"], 3.0)
    assert np.array_equal(h1, h) and np.allclose(z1, z - 0.015)
    # subcritical on [0, L] with q0 = 1
    assert np.all(q / h < np.sqrt(9.81 * h))


def test_c1_is_the_stated_riemann_problem():
    wl = inputs.make_c1()
    assert wl.n_cells == 250 and abs(wl.dx[0] * 250 - 10.0) < 1e-12
    left = np.arange(250) < 125
    assert np.allclose(wl.h[left], 2.0) and np.allclose(wl.q[left], 1.0)
    assert np.allclose(wl.h[~left], 1.0) and np.allclose(wl.q[~left], 0.3)
    assert np.allclose(wl.z[left], 0.0) and np.allclose(wl.z[~left], 0.2)
