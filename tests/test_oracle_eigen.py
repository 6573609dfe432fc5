"""Pins of the oracle's eigenstructure (Sec. 3.3) against things other than itself.

* flux matrix vs a complex-step Jacobian of the conservative flux of Eq. SV-Ex
  plus the non-conservative bed term (Eq. quasiLinNC / W&A_definition);
* eigenvalues vs LAPACK (numpy.linalg.eigvals) and vs 50-digit mpmath roots;
* Vieta relations of the characteristic polynomial (Eq. charPol times c^3);
* textbook special cases: fixed bed A_g = 0 gives {u-c, 0, u+c}; still water
  u = 0 gives {-c, 0, c};
* the Grass law makes lambda/c a function of (Fr, xi A_g g) only;
* A r = lambda r, l A = lambda l, R R^-1 = I, R Lambda R^-1 = A;
* |A| vs the numerical-eigensolver |A| of the original DOT; |A|^2 = A^2;
  A|A| = |A|A; |A| = A when all eigenvalues are positive.
"""
import mpmath
import numpy as np
import pytest

from oracle import dot_numeric

G = 9.81


def random_states(n, seed=0, h=(0.05, 5.0), u=(-3.0, 3.0)):
    rng = np.random.default_rng(seed)
    hh = rng.uniform(*h, n)
    uu = rng.uniform(*u, n)
    zz = rng.uniform(-1.0, 1.0, n)
    Ag = 10 ** rng.uniform(-4, -1, n)
    por = rng.uniform(0.0, 0.45, n)
    return hh, hh * uu, zz, Ag, 1.0 / (1.0 - por)


def eig_one(orc, h, q, z, xi, Ag):
    return orc.eigensystem([h], [q], [z], G, xi, Ag)


def conservative_flux(W, xi, Ag):
    """F(W) = (q, g h^2/2 + q^2/h, xi q_s) of Eq. SV-Ex (complex-step friendly)."""
    h, q = W[0], W[1]
    return np.array([q, 0.5 * G * h * h + q * q / h, xi * Ag * (q / h) ** 3])


def test_flux_matrix_is_jacobian_plus_bed_term(orc):
    hh, qq, zz, Ags, xis = random_states(200, seed=1)
    for h, q, z, Ag, xi in zip(hh, qq, zz, Ags, xis):
        A = orc.eigensystem([h], [q], [z], G, xi, Ag)["A"][0]
        J = np.zeros((3, 3))
        eps = 1e-30
        for j in range(3):
            W = np.array([h, q, z], dtype=complex)
            W[j] += 1j * eps
            J[:, j] = conservative_flux(W, xi, Ag).imag / eps
        J[1, 2] += G * h  # non-conservative product g h dz/dx
        np.testing.assert_allclose(A, J, rtol=1e-13, atol=1e-13 * np.abs(J).max())


def test_eigenvalues_vs_lapack(orc):
    hh, qq, zz, Ags, xis = random_states(3000, seed=2)
    worst = 0.0
    for i in range(hh.size):
        e = eig_one(orc, hh[i], qq[i], zz[i], xis[i], Ags[i])
        lam = e["lam"][0]
        ref = np.sort(np.linalg.eigvals(e["A"][0]).real)
        worst = max(worst, np.max(np.abs(lam - ref)) / np.max(np.abs(ref)))
        assert lam[0] <= lam[1] <= lam[2]
    assert worst < 1e-13, worst


def _mp_roots(h, q, xi, Ag):
    mpmath.mp.dps = 50
    h, q = mpmath.mpf(h), mpmath.mpf(q)
    u = q / h
    c2 = mpmath.mpf(G) * h
    dh = -3 * mpmath.mpf(Ag) * u ** 3 / h
    dq = 3 * mpmath.mpf(Ag) * u ** 2 / h
    # det(lambda I - A) for A of Eq. W&A_definition, expanded by hand
    coeffs = [1, -2 * u, -(c2 - u * u) - c2 * xi * dq, -c2 * xi * dh]
    r = mpmath.polyroots(coeffs, maxsteps=200, extraprec=200)
    return sorted(float(mpmath.re(x)) for x in r)


@pytest.mark.parametrize("h,u,Ag,por", [
    (1.0, 0.5, 0.01, 0.4), (0.3, 1.8, 0.001, 0.3), (2.0, -1.2, 0.05, 0.0),
    (0.294, 1.6985, 1e-3, 0.4),   # Fr close to 1, weak transport (near coalescence)
    (0.5, 0.0, 0.01, 0.4), (4.0, 5.0, 0.1, 0.45),
])
def test_eigenvalues_vs_mpmath(orc, h, u, Ag, por):
    xi = 1.0 / (1.0 - por)
    lam = eig_one(orc, h, h * u, 0.0, xi, Ag)["lam"][0]
    ref = np.array(_mp_roots(h, h * u, xi, Ag))
    assert np.max(np.abs(lam - ref)) <= 2e-13 * np.max(np.abs(ref))


def test_vieta_relations(orc):
    hh, qq, zz, Ags, xis = random_states(2000, seed=3)
    for i in range(hh.size):
        h, q, xi, Ag = hh[i], qq[i], xis[i], Ags[i]
        lam = eig_one(orc, h, q, zz[i], xi, Ag)["lam"][0]
        u, c2 = q / h, G * h
        dqs_dh, dqs_dq = -3 * Ag * u ** 3 / h, 3 * Ag * u ** 2 / h
        scale = max(abs(lam).max(), 1e-300)
        assert abs(lam.sum() - 2 * u) <= 1e-13 * scale
        s2 = lam[0] * lam[1] + lam[0] * lam[2] + lam[1] * lam[2]
        assert abs(s2 + (c2 - u * u + c2 * xi * dqs_dq)) <= 1e-13 * scale ** 2
        assert abs(lam.prod() - c2 * xi * dqs_dh) <= 1e-13 * scale ** 3


def test_fixed_bed_reduces_to_shallow_water(orc):
    hh, qq, zz, _, xis = random_states(500, seed=4)
    for h, q, z, xi in zip(hh, qq, zz, xis):
        u, c = q / h, np.sqrt(G * h)
        if abs(abs(u / c) - 1.0) < 1e-6:
            continue
        lam = eig_one(orc, h, q, z, xi, 0.0)["lam"][0]
        ref = np.sort([u - c, 0.0, u + c])
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-13 * (abs(u) + c))


def test_still_water_gives_minus_c_zero_plus_c(orc):
    for h in [0.05, 0.3, 1.0, 4.0]:
        c = np.sqrt(G * h)
        lam = eig_one(orc, h, 0.0, 0.1, 1.0 / 0.6, 0.02)["lam"][0]
        np.testing.assert_allclose(lam, [-c, 0.0, c], rtol=0, atol=1e-14 * c)


def test_grass_scaling_depends_on_froude_only(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        Fr = rng.uniform(-2.5, 2.5)
        xiAg = 10 ** rng.uniform(-4, -1)
        h1, h2 = rng.uniform(0.05, 5.0, 2)
        u1, u2 = Fr * np.sqrt(G * h1), Fr * np.sqrt(G * h2)
        l1 = eig_one(orc, h1, h1 * u1, 0.0, 1.0, xiAg)["lam"][0] / np.sqrt(G * h1)
        l2 = eig_one(orc, h2, h2 * u2, 0.0, 1.0, xiAg)["lam"][0] / np.sqrt(G * h2)
        np.testing.assert_allclose(l1, l2, rtol=0, atol=1e-13 * np.abs(l1).max())


def test_eigenvectors_and_inverse(orc):
    hh, qq, zz, Ags, xis = random_states(1000, seed=6)
    for i in range(hh.size):
        e = eig_one(orc, hh[i], qq[i], zz[i], xis[i], Ags[i])
        A, R, Ri, lam = e["A"][0], e["R"][0], e["Rinv"][0], e["lam"][0]
        for m in range(3):
            r = R[:, m]
            assert np.linalg.norm(A @ r - lam[m] * r) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r)
            l = Ri[m, :]
            assert np.linalg.norm(l @ A - lam[m] * l) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(l)
        cond = np.linalg.cond(R)
        assert np.max(np.abs(R @ Ri - np.eye(3))) <= 1e-15 * cond * 10
        RLR = R @ np.diag(lam) @ Ri
        assert np.max(np.abs(RLR - A)) <= 1e-12 * np.max(np.abs(A))


def test_abs_matrix_vs_numerical_eigensolver(orc):
    hh, qq, zz, Ags, xis = random_states(1000, seed=7)
    for i in range(hh.size):
        e = eig_one(orc, hh[i], qq[i], zz[i], xis[i], Ags[i])
        A, aA = e["A"][0], e["absA"][0]
        ref = dot_numeric.abs_matrix(dot_numeric.flux_matrix(hh[i], qq[i], G, xis[i], Ags[i]))
        assert np.max(np.abs(aA - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.max(np.abs(aA @ aA - A @ A)) <= 1e-12 * np.max(np.abs(A @ A))
        assert np.max(np.abs(A @ aA - aA @ A)) <= 1e-12 * np.max(np.abs(A @ A))


def test_abs_matrix_equals_matrix_when_all_speeds_positive(orc):
    # fixed bed (A_g = 0) and Fr > 1: eigenvalues {0, u-c, u+c}, none negative, so |A| = A.
    # (With A_g > 0 and u > 0 the product of the eigenvalues, c^2 xi dq_s/dh, is negative.)
    for h, u in [(0.3, 3.0), (1.0, 5.0), (0.1, 2.0)]:
        e = eig_one(orc, h, h * u, 0.0, 1.0, 0.0)
        assert np.all(e["lam"][0] >= -1e-15 * np.abs(e["lam"][0]).max())
        np.testing.assert_allclose(e["absA"][0], e["A"][0], rtol=0,
                                   atol=1e-12 * np.abs(e["A"][0]).max())


@pytest.mark.parametrize("h,u,Ag", [(1.0, 2.0, -0.05), (1.0, 1.0, -0.5)])
def test_complex_roots_are_reported(orc, h, u, Ag):
    # a negative A_g lies outside the paper's closure and gives complex roots (checked with
    # LAPACK): arccos argument > 1 in the first case, k1 < 0 in the second
    A = dot_numeric.flux_matrix(h, h * u, G, 1.0, Ag)
    assert np.max(np.abs(np.linalg.eigvals(A).imag)) > 0.1
    e = orc.eigensystem([h], [h * u], [0.0], G, 1.0, Ag, check=False)
    assert e["status"] == orc.E_NONHYPERBOLIC


def test_coalescing_roots_of_a_fixed_bed_are_reported(orc):
    # a fixed bed (A_g = 0) at Fr = 1: the roots u - c and 0 coincide and A is defective (one
    # eigenvector for the double root), so R^-1 of Eq. RR-1 does not exist.  With g = 4, h = 1
    # and q = 2 every quantity is exact: Fr = 1, k1 = 4, k2 = 16, arccos argument 1.
    A = dot_numeric.flux_matrix(1.0, 2.0, 4.0, 1.0, 0.0)
    lam = np.sort(np.linalg.eigvals(A).real)
    assert abs(lam[0]) < 1e-7 and abs(lam[1]) < 1e-7 and abs(lam[2] - 4.0) < 1e-12
    e = orc.eigensystem([1.0], [2.0], [0.0], 4.0, 1.0, 0.0, check=False)
    assert e["status"] == orc.E_NONHYPERBOLIC
    assert e["lam"][0][0] == e["lam"][0][1] and abs(e["lam"][0][0]) < 1e-15
    # the edge whose quadrature nodes all sit there is reported too, not returned as numbers
    Dm, Dp = orc.fluct(([1.0], [2.0], [0.0]), ([1.0], [2.0], [0.1]), 4.0, 1.0, 0.0, check=False)
    with pytest.raises(orc.OracleError) as ex:
        orc.fluct(([1.0], [2.0], [0.0]), ([1.0], [2.0], [0.1]), 4.0, 1.0, 0.0)
    assert ex.value.status == orc.E_NONHYPERBOLIC
    # the CFL speed needs no R^-1: the state's largest speed u + c = 4 is reported
    assert orc.cfl_amax([1.0], [2.0], [0.0], 4.0, 1.0, 0.0) == 4.0
    # a movable bed at the same state keeps its roots apart (Sec. 3.3)
    e = orc.eigensystem([1.0], [2.0], [0.0], 4.0, 1.0, 0.01, check=False)
    assert e["status"] == orc.OK and e["lam"][0][1] - e["lam"][0][0] > 0.1


@pytest.mark.parametrize("dfr", [1e-9, -1e-9])
def test_fixed_bed_next_to_coalescence(orc, dfr):
    # Fr = 1 +- 1e-9 over a fixed bed: the roots are apart by 1e-9 c, below what the arccos
    # argument resolves (1 - x ~ 3e-19), so they coincide in FP64 and the state is reported
    q = 2.0 * (1.0 + dfr)
    e = orc.eigensystem([1.0], [q], [0.0], 4.0, 1.0, 0.0, check=False)
    lam = e["lam"][0]
    if lam[0] == lam[1]:
        assert e["status"] == orc.E_NONHYPERBOLIC
    else:
        assert e["status"] == orc.OK and np.all(np.isfinite(e["Rinv"]))
