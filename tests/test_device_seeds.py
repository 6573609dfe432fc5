"""Host-side checks of the arithmetic kernels in dsve_math.hpp (coefficients read from the
header, evaluated in FP32 or with correctly rounded FMAs as the kernels evaluate them).

The eigenvalues come from cos and sin of theta = arccos(|x|)/3: the cosine from an FP32
polynomial refined by Newton steps in FP64, the sine from sin(3 theta) = S (4 C^2 - 1).  The
roots at -x are those at x negated, so the kernels label the roots sign(x) {C, -P, -Q} without
sorting them.
"""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1912_04791_amd", "csrc", "dsve_math.hpp")


def test_roots_labelled_by_the_sign_of_x_are_the_trisection_roots():
    # sign(x) {C, -P, -Q}, P, Q = C/2 +- (sqrt3/2) S, with (C, S) at arccos(|x|)/3, is the set
    # {cos(phi/3), cos(phi/3 +- 2 pi/3)}, phi = arccos(x); the gaps of the labels and their
    # product sign(x) (3 sqrt3 / 4) sin(phi), whose reciprocal the kernels take
    x = np.concatenate([np.linspace(-1.0, 1.0, 20001), -1 + np.logspace(-12, -1, 200),
                        1 - np.logspace(-12, -1, 200)])
    th = np.arccos(np.abs(x)) / 3
    C, S = np.cos(th), np.sin(th)
    sg = np.copysign(1.0, x)
    r = np.sqrt(3) / 2 * S
    lab = np.stack([sg * C, -sg * (0.5 * C + r), -sg * (0.5 * C - r)])
    ph = np.arccos(x) / 3
    ref = np.stack([np.cos(ph), np.cos(ph + 2 * np.pi / 3), np.cos(ph - 2 * np.pi / 3)])
    np.testing.assert_allclose(np.sort(lab, axis=0), np.sort(ref, axis=0), rtol=0, atol=2e-15)
    g21 = -sg * (1.5 * C + r)
    g31 = -sg * (1.5 * C - r)
    g32 = 2 * sg * r
    np.testing.assert_allclose(g21, lab[1] - lab[0], rtol=0, atol=4e-15)
    np.testing.assert_allclose(g31, lab[2] - lab[0], rtol=0, atol=4e-15)
    np.testing.assert_allclose(g32, lab[2] - lab[1], rtol=0, atol=4e-15)
    np.testing.assert_allclose(g21 * g31 * g32, sg * 3 * np.sqrt(3) / 4 * np.sin(np.arccos(x)),
                               rtol=1e-12, atol=1e-15)


def test_third_angle_fp64():
    # (C, S) in FP64 as the kernels compute them: the FP32 polynomial, the FP32 reciprocal of the
    # cubic's derivative, two Newton steps, then S = y / (4C^2 - 1) with 1 / (4C^2 - 1) = 3r
    # refined by one Halley step, every FMA correctly rounded; y = sqrt(1 - a^2) correctly
    # rounded.  Against 40-digit values: C within 2 ulp, S within 4 ulp relative (also as
    # a -> 1, where S -> 0)
    import mpmath as mp
    mp.mp.dps = 40
    src = open(HDR).read()
    body = src[src.index("void third_angle(double a, double y, double &C, double &S)"):]
    body = body[:body.index("\n}\n")]
    for line in ("const double u = fma(4.0 * C, C, -1.0);", "const double R0 = 3.0 * r;",
                 "const double e = fma(-u, R0, 1.0);", "S = y * fma(R0, fma(e, e, e), R0);"):
        assert line in body, line
    pts = np.concatenate([np.linspace(0.0, 1.0, 601), 1 - np.logspace(-16, -1, 120),
                          np.logspace(-16, -1, 60)])
    cf = _cos_third_acos_f32(pts.astype(np.float32))
    d = (np.float32(12) * cf * cf - np.float32(3)).astype(np.float32)
    rr = (np.float32(1) / d).astype(np.float32)
    worst_c = worst_s = 0.0
    for a, c0, r in zip(pts, cf, rr):
        c, r = float(c0), float(r)
        for _ in range(2):
            c = _fma(-_fma(c, _fma(4.0 * c, c, -3.0), -a), r, c)
        u = _fma(4.0 * c, c, -1.0)
        R0 = 3.0 * r
        e = _fma(-u, R0, 1.0)
        y = float(mp.sqrt(1 - mp.mpf(float(a)) ** 2))
        S = y * _fma(R0, _fma(e, e, e), R0)
        th = mp.acos(mp.mpf(float(a))) / 3
        worst_c = max(worst_c, float(abs((mp.mpf(c) - mp.cos(th)) / mp.cos(th))))
        if a < 1.0:
            worst_s = max(worst_s, float(abs((mp.mpf(S) - mp.sin(th)) / mp.sin(th))))
    assert worst_c < 2 * 2.0 ** -52, worst_c
    assert worst_s < 4 * 2.0 ** -52, worst_s


def test_third_angle_fp32():
    # the mixed form's (C, S): the polynomial and S = y * rcp(4C^2 - 1) in FP32, y correctly
    # rounded to FP32; against FP64 values: C within 4 ulp, S within 6 ulp relative
    a = np.concatenate([np.linspace(0.0, 1.0, 200001), 1 - np.logspace(-7, -1, 2000)]).astype(np.float32)
    C = _cos_third_acos_f32(a)
    y = np.sqrt(1 - a.astype(np.float64) ** 2).astype(np.float32)
    u = (np.float32(4) * C * C - np.float32(1)).astype(np.float32)
    S = (y * (np.float32(1) / u).astype(np.float32)).astype(np.float32)
    th = np.arccos(a.astype(np.float64)) / 3
    assert np.max(np.abs(C - np.cos(th)) / np.cos(th)) < 4 * 2.0 ** -24
    m = a < 1
    assert np.max(np.abs(S[m] - np.sin(th[m])) / np.sin(th[m])) < 6 * 2.0 ** -24


def test_small_root_series_in_fp32():
    # the mixed form's Q = C/2 - r = sin(arcsin(a)/3), which cancels as a -> 0, comes from its
    # series a/3 + 4a^3/81 below a = 1/64: within 1e-8 relative of the function there (FP64
    # evaluation), and within 3 ulp when evaluated in FP32 as the kernel does
    src = open(HDR).read()
    assert "a < 0.015625f ? a * fmaf(a * a, 4.0f / 81.0f, 1.0f / 3.0f) : fmaf(0.5f, C, -r)" in src
    a = np.concatenate([np.linspace(0.0, 1 / 64, 20001), np.logspace(-30, np.log10(1 / 64), 400)])
    ref = np.sin(np.arcsin(a) / 3)
    ser = a * (a * a * 4 / 81 + 1 / 3)
    m = a > 0
    assert np.max(np.abs(ser[m] - ref[m]) / ref[m]) < 1e-8
    a32 = a.astype(np.float32)
    aa = (a32 * a32).astype(np.float32)
    inner = (aa.astype(np.float64) * np.float64(np.float32(4 / 81)) + np.float64(np.float32(1 / 3))).astype(np.float32)
    s32 = (a32 * inner).astype(np.float32)
    ref32 = np.sin(np.arcsin(a32.astype(np.float64)) / 3)
    m = a32 > 0
    assert np.max(np.abs(s32[m] - ref32[m]) / ref32[m]) < 3 * 2.0 ** -24
    assert s32[0] == 0.0


def test_gap_product_identity():
    # (mu2 - mu1)(mu3 - mu1)(mu3 - mu2) = (2 sqrt3 / 9) k1^(3/2) sin(phi) for the roots
    # mu = f - m cos(theta -+ pi/3), f + m cos(theta), m = (2/3) sqrt(k1), 3 theta = phi
    rng = np.random.default_rng(5)
    k1 = rng.uniform(0.1, 20.0, 1000)
    phi = rng.uniform(0.0, np.pi, 1000)
    f = rng.uniform(-2, 2, 1000)
    m = 2.0 / 3.0 * np.sqrt(k1)
    th = phi / 3
    mu1 = f - m * np.cos(th - np.pi / 3)
    mu2 = f - m * np.cos(th + np.pi / 3)
    mu3 = f + m * np.cos(th)
    P = (mu2 - mu1) * (mu3 - mu1) * (mu3 - mu2)
    np.testing.assert_allclose(P, 2 * np.sqrt(3) / 9 * k1 ** 1.5 * np.sin(phi), rtol=1e-9, atol=1e-12)
    src = open(HDR).read()
    val = float(re.search(r"kInvGapScale = ([0-9.]+);", src).group(1))
    assert abs(val - 1.5 * np.sqrt(3)) < 1e-15


def test_tenth_root_newton_reaches_fp64():
    # a^1.1 = a^2 y^9 with y = a^(-1/10): FP32 estimate 2^(-log2(a)/10) (emulated here with
    # numpy's float32 exp2/log2), then two Newton steps y <- y (11 - a y^10) / 10 in FP64, as the
    # Van Rijn closure takes it; also from estimates degraded to a relative error of 1e-6
    a = np.concatenate([np.logspace(-15, 3, 20001), np.linspace(0.5, 2.0, 2001)])
    y0 = np.exp2(np.float32(-0.1) * np.log2(a.astype(np.float32))).astype(np.float64)
    exact = a ** -0.1
    assert np.max(np.abs(y0 / exact - 1)) < 1e-6
    for seed in (y0, exact * (1 + 1e-6), exact * (1 - 1e-6)):
        y = seed
        for _ in range(2):
            y2 = y * y
            y5 = y2 * y2 * y
            y = (y * 0.1) * (11.0 - a * (y5 * y5))
        y4 = (y * y) * (y * y)
        np.testing.assert_allclose(y, exact, rtol=1e-15)
        # y^9 carries nine times y's last-bit rounding: about 6e-15 at worst
        np.testing.assert_allclose((a * a) * (y4 * y4 * y), a ** 1.1, rtol=8e-15)


def test_integer_power_product():
    # |u|^n for n in [0, 15] as the product of u, u^2, u^4, u^8 selected by the bits of n
    u = np.linspace(1e-3, 3.0, 1001)
    for n in range(16):
        u2 = u * u
        u4 = u2 * u2
        u8 = u4 * u4
        r = np.where(n & 1, u, 1.0)
        r = np.where(n & 2, r * u2, r)
        r = np.where(n & 4, r * u4, r)
        r = np.where(n & 8, r * u8, r)
        np.testing.assert_allclose(r, u ** n, rtol=4 * 2.2e-16 * max(n, 1))


def test_reciprocal_cube_root_newton_reaches_fp64():
    # a^(-1/3): FP32 estimate 2^(-log2(a)/3) (numpy's float32 exp2/log2 here), then two Newton
    # steps y <- y (4 - a y^3) / 3 in FP64, as the MPM and Van Rijn closures and the friction
    # source take it; also from estimates degraded to a relative error of 1e-6
    a = np.concatenate([np.logspace(-6, 4, 20001), np.linspace(0.01, 3.0, 2001)])
    y0 = np.exp2(np.float32(-1.0 / 3.0) * np.log2(a.astype(np.float32))).astype(np.float64)
    exact = a ** (-1.0 / 3.0)
    assert np.max(np.abs(y0 / exact - 1)) < 1e-6
    for seed in (y0, exact * (1 + 1e-6), exact * (1 - 1e-6)):
        y = seed
        for _ in range(2):
            y = (y * (1.0 / 3.0)) * (4.0 - a * (y * y * y))
        np.testing.assert_allclose(y, exact, rtol=1e-15)
        r2 = y * y
        np.testing.assert_allclose((r2 * r2) * (r2 * y), a ** (-7.0 / 3.0), rtol=1e-14)


def test_stress_law_derivatives_without_reciprocal_of_q():
    # MPM and Van Rijn: th / |q| with th = lp0 u^2 h^(-1/3) equals lp0 |u| h^(-1/3) / h, since
    # |q| = h |u|; the rewritten b equals the form with the reciprocal of |q|
    rng = np.random.default_rng(7)
    h = rng.uniform(0.01, 3.0, 5000)
    q = rng.uniform(-5.0, 5.0, 5000)
    lp0, lp1 = 40.0, 0.3
    u = q / h
    r = h ** (-1.0 / 3.0)
    th = lp0 * u * u * r
    mpm_q = np.where(th > 0.047, lp1 * np.sqrt(np.maximum(th - 0.047, 0)) * th / np.abs(q), 0)
    mpm_r = np.where(th > 0.047, lp1 * np.sqrt(np.maximum(th - 0.047, 0)) * (lp0 * np.abs(u) * r / h), 0)
    np.testing.assert_allclose(mpm_r, mpm_q, rtol=1e-14)
    tt = th - 1.0
    vr_q = np.where(tt > 0, lp1 * np.maximum(tt, 0) ** 1.1 * th / np.abs(q), 0)
    vr_r = np.where(tt > 0, lp1 * np.maximum(tt, 0) ** 1.1 * (lp0 * np.abs(u) * r / h), 0)
    np.testing.assert_allclose(vr_r, vr_q, rtol=1e-14)
    assert np.count_nonzero(mpm_q) > 1000 and np.count_nonzero(vr_q) > 1000


def test_power_as_exp2_of_log2():
    # a^b = 2^(b log2 a) for the power law with a non-integer exponent (FP64 form): the rounding of
    # log2 a and of the product each leave y = b log2 a an absolute error up to about |y| 2^-53,
    # so the power's relative error is about 2 |y| ln2 2^-53: a few ulp at the speeds of the laws
    # (|y| of a few units), 1e-14 at the far end of this range
    a = np.concatenate([np.logspace(-4, 1.5, 20001), np.linspace(0.5, 2.0, 2001)])
    for b in (1.5, 2.5, 5.5, 9.5):
        y = b * np.log2(a)
        got = np.exp2(y)
        bound = (2 * np.abs(y) * np.log(2) + 4) * 2.0 ** -53
        assert np.all(np.abs(got / a ** b - 1) <= bound), b


def _poly_coeffs(sig):
    """Horner coefficients (highest degree first) of a `p = ...; p = fma(p, t, c); ...` body."""
    src = open(HDR).read()
    body = src[src.index(sig):]
    body = body[:body.index("\n}\n")]
    lit = r"(-?\d+(?:\.\d+)?(?:e-?\d+)?)f?"
    first = float(re.search(r"p = " + lit + ";", body).group(1))
    # every Horner step, the returned last one included
    rest = [float(v) for v in re.findall(r"fmaf?\(p, t, " + lit + r"\)", body)]
    return [first] + rest


def _fma(a, b, c):
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _cos_third_acos_f32(a32):
    cs = _poly_coeffs("float cos_third_acos(float a)")
    t = (np.float32(1) - a32).astype(np.float32)
    p = np.full_like(a32, np.float32(cs[0]))
    for c in cs[1:]:
        p = (p.astype(np.float64) * t.astype(np.float64) + np.float64(np.float32(c))).astype(np.float32)
    return p


def test_cos_third_acos_fp64_newton():
    # the CFL speed's cos(arccos(a)/3) on [0, 1] in FP64: the FP32 estimate, the FP32 reciprocal
    # of the cubic's derivative, two Newton steps with correctly rounded FMAs as on the device;
    # against 50-digit values: within 2 ulp
    import mpmath as mp
    mp.mp.dps = 40
    src = open(HDR).read()
    assert "for (int k = 0; k < 2; ++k) c = fma(-fma(c, fma(4.0 * c, c, -3.0), -a), r, c);" in src
    pts = np.concatenate([np.linspace(0.0, 1.0, 2001), 1 - np.logspace(-16, -1, 200),
                          np.logspace(-16, -1, 200)])
    cf = _cos_third_acos_f32(pts.astype(np.float32))
    d = (np.float32(12) * cf * cf - np.float32(3)).astype(np.float32)
    r = (np.float32(1) / d).astype(np.float32)
    worst = 0.0
    for a, c0, rr in zip(pts, cf, r):
        c, rr = float(c0), float(rr)
        for _ in range(2):
            f = _fma(c, _fma(4.0 * c, c, -3.0), -a)
            c = _fma(-f, rr, c)
        ref = mp.cos(mp.acos(mp.mpf(float(a))) / 3)
        worst = max(worst, float(abs((mp.mpf(c) - ref) / ref)))
    assert worst < 2 * 2.0 ** -52, worst


def test_cos_third_acos_fp32_polynomial():
    cs = _poly_coeffs("float cos_third_acos(float a)")
    assert len(cs) == 8
    a = np.concatenate([np.linspace(0.0, 1.0, 200001), 1 - np.logspace(-7, -1, 2000)]).astype(np.float32)
    p = _cos_third_acos_f32(a)
    ref = np.cos(np.arccos(a.astype(np.float64)) / 3)
    assert np.max(np.abs(p - ref) / ref) < 4 * 2.0 ** -24


def test_largest_speed_is_the_largest_root_at_abs_froude():
    # the CFL speed takes max_m |mu_m| as mu_3 at |Fr| (k1 even, k2 odd in Fr); checked against
    # all three roots over Froude numbers of both signs, transport from none to strong and both
    # closure forms (kappa = 1 for velocity laws, 7/6 for stress laws), complex roots clamped
    rng = np.random.default_rng(3)
    n = 400_000
    Fr = np.concatenate([rng.uniform(-10, 10, n), rng.uniform(-1.2, 1.2, n)])
    b = np.concatenate([rng.exponential(1.0, n) * 10.0 ** rng.uniform(-8, 2, n), np.zeros(n)])
    kap = np.where(rng.random(2 * n) < 0.5, 1.0, 7.0 / 6.0)

    def roots(F):
        k1 = 3 + F ** 2 + 3 * b
        k2 = F * (18 - 2 * F ** 2 + (18 - 27 * kap) * b)
        ph = np.arccos(np.clip(k2 / np.sqrt(4 * k1 ** 3), -1, 1))
        m, f = 2 / 3 * np.sqrt(k1), 2 / 3 * F
        return f - m * np.cos(ph / 3 - np.pi / 3), f - m * np.cos(ph / 3 + np.pi / 3), f + m * np.cos(ph / 3)

    m1, m2, m3 = roots(Fr)
    mx = np.maximum(np.maximum(np.abs(m1), np.abs(m2)), np.abs(m3))
    assert np.max(np.abs(mx - roots(np.abs(Fr))[2]) / mx) < 1e-14


def test_one_eigenpair_minus_part_matches_lapack():
    # The FP64 kernels take A^- dW = ((A - |A|)/2) dW (Sec. 3.1, Eqs. asbA, ExAbsA) from one
    # eigenpair: mu_3 of the labelled roots is the middle one, so when mu_3 >= 0 only the
    # smallest root o can be negative and A^- dW = c min(mu_o, 0) (l_o . dW) r_o, and when
    # mu_3 < 0 only the largest can be positive and A^- dW = A dW - c max(mu_o, 0) (l_o . dW) r_o;
    # o is labelled 2 when the signs of mu_3 and sign(x) m agree, else 1.  Checked against
    # R min(Lambda, 0) R^-1 dW from LAPACK on the dimensional matrix of the Grass law.
    rng = np.random.default_rng(42)
    g, xi = 9.81, 1.0 / 0.6
    n = 4000
    h = rng.uniform(0.1, 3.0, n)
    Fr_in = rng.uniform(-6.0, 6.0, n)
    Ag = rng.choice([0.0, 1e-4, 1e-2, 5e-2], n)
    c = np.sqrt(g * h)
    u = Fr_in * c
    dW = rng.standard_normal((n, 3)) * np.array([0.1, 0.1, 0.05])
    kqg = 3 * xi * Ag * g
    Fr = u / c
    k1 = 3 + Fr ** 2 * (1 + 3 * kqg)
    k2h = Fr * (9 - Fr ** 2 * (1 + 4.5 * kqg))
    x = k2h / k1 ** 1.5
    keep = 1 - np.abs(x) > 1e-3   # away from coalescing roots, where R^-1 is ill-conditioned
    th = np.arccos(np.abs(x)) / 3
    C, S = np.cos(th), np.sin(th)
    ms = np.copysign(2.0 / 3.0 * np.sqrt(k1), x)
    f = 2.0 / 3.0 * Fr
    r = np.sqrt(3) / 2 * S
    mu1, mu2, mu3 = f + ms * C, f - ms * (0.5 * C + r), f - ms * (0.5 * C - r)
    mus = np.stack([mu1, mu2, mu3])
    # mu_3 is the middle root
    assert np.all(np.sort(mus, axis=0)[1] == mu3)
    up = mu3 >= 0
    two = up == (ms >= 0)
    mo, mx = np.where(two, mu2, mu1), np.where(two, mu1, mu2)
    # every other root has the sign of mu_3 (or is zero)
    other = np.where(two, mu1, mu2)
    assert np.all(np.where(up, other >= 0, other < 0) | (np.abs(other) < 1e-15))
    no = (1 - Fr ** 2 + mu3 * mx) * dW[:, 0] + mo * dW[:, 1] / c + dW[:, 2]
    lo = no / ((mo - mx) * (mo - mu3))
    t = np.where(up, np.minimum(mo, 0), -np.maximum(mo, 0))
    ro = np.stack([np.ones(n), c * mo, (Fr - mo) ** 2 - 1], axis=1)
    A = np.zeros((n, 3, 3))
    A[:, 0, 1] = 1
    A[:, 1, 0], A[:, 1, 1], A[:, 1, 2] = c ** 2 - u ** 2, 2 * u, c ** 2
    A[:, 2, 0], A[:, 2, 1] = xi * (-3 * Ag * u ** 3 / h), xi * (3 * Ag * u ** 2 / h)
    AdW = np.einsum("nij,nj->ni", A, dW)
    got = np.where(up[:, None], 0.0, AdW) + (c * t * lo)[:, None] * ro
    lam, R = np.linalg.eig(A)
    lam, R = lam.real, R.real
    ref = np.einsum("nij,nj->ni", R * np.minimum(lam, 0)[:, None, :], np.linalg.solve(R, dW[..., None])[..., 0])
    scale = np.abs(AdW).max(axis=1) + np.abs(ref).max(axis=1) + 1e-300
    err = np.abs(got - ref).max(axis=1) / scale
    assert keep.mean() > 0.9
    assert err[keep].max() <= 1e-11, (err[keep].max(), np.argmax(np.where(keep, err, 0)))
    # both cases and both labels occur
    assert up[keep].any() and (~up[keep]).any() and two[keep].any() and (~two[keep]).any()
