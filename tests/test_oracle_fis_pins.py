"""Pins of the oracle's Gaussian and filter-importance-sampling filters
(Sec. 4.1 FRS with a discrete Gaussian; Sec. 4.2 FIS; Suppl. S.4.2) against
libm, closed forms, exact counting and statistics, none of which share the
oracle's code."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from paper_2407_06107_amd import inputs

U24 = 2.0 ** -24


# ------------------------------------------------------------ elementary functions
def test_lnc_within_three_ulp_on_every_uniform(orc):
    """ln of every value 1 - u can take (k 2^-24, k = 1..2^24) vs libm."""
    x = (np.arange(1, 2 ** 24 + 1, dtype=np.float64) * U24).astype(np.float32)
    y = orc.lnc(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert y[-1] == 0.0                                  # ln 1
    assert np.all(np.abs(y - ref) <= 3.0 * np.maximum(ulp, 2.0 ** -149))


def test_expc_relative_error_and_range(orc):
    x = np.concatenate([np.linspace(-80, 0, 1_000_001), [-0.0, -1e-30, -79.999]]).astype(np.float32)
    y = orc.expc(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    assert np.all(np.abs(y - ref) <= 2.0 * U24 * ref)
    assert orc.expc(np.array([0.0], np.float32))[0] == 1.0
    assert np.all(orc.expc(np.array([-80.5, -1e4, -np.inf], np.float32)) == 0.0)


def test_sincos_on_every_uniform(orc):
    v = (np.arange(2 ** 24, dtype=np.float64) * U24).astype(np.float32)
    c, s = orc.sincos2pi(v)
    ang = 2.0 * np.pi * v.astype(np.float64)
    assert np.max(np.abs(c - np.cos(ang))) <= 2.0 * U24
    assert np.max(np.abs(s - np.sin(ang))) <= 2.0 * U24
    q = np.array([0.0, 0.25, 0.5, 0.75], np.float32)          # exact quadrant points
    cq, sq = orc.sincos2pi(q)
    assert np.array_equal(cq, [1, 0, -1, 0]) and np.array_equal(sq, [0, 1, 0, -1])


# ------------------------------------------------------------ Gaussian FIS (Box-Muller + nearest)
def test_box_muller_offsets_are_normal(orc):
    """Offsets / sigma from lattice uniforms: standard normal per axis (KS),
    uncorrelated, and the radius bounded by sqrt(2 ln 2^24)."""
    rng = np.random.default_rng(0)
    k = rng.integers(0, 2 ** 24, size=(20000, 2))
    sig = 0.7
    d = np.array([orc.fis_gauss_offset(a * U24, b * U24, sig) for a, b in k]) / sig
    for ax in range(2):
        assert stats.kstest(d[:, ax], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(d[:, 0], d[:, 1])[0, 1]) < 0.03
    rmax = math.sqrt(2 * 24 * math.log(2))
    dx, dy = orc.fis_gauss_offset(1.0 - U24, 0.0, 1.0)            # largest radius, angle 0
    assert dx == pytest.approx(rmax, rel=1e-6) and dy == 0.0
    assert orc.fis_gauss_offset(0.0, 0.3, 2.0) == (0.0, 0.0)       # u1 = 0: radius 0


def _offset_histogram(orc, filt, t, sigma, spp, lo, hi, seed=3):
    """Tap offsets of one query at fraction t past texel 31 of a 64-texel
    axis (clamped texture, so offsets are read back from the taps)."""
    N = 64
    tex = inputs.texture_uniform(N, seed=1)
    u = (31 + t + 0.5) / N
    q = np.array([[u, u, 0.0]], np.float32)
    _, taps = orc.filter2d(orc.Tex2D.rgba32f(tex, wrap=orc.CLAMP), q, filt, orc.STOCHASTIC, spp=spp, seed=seed,
                           taps=True, sigma=sigma)
    p = np.float32(np.float32(u) * np.float32(N)) - np.float32(0.5)
    i0 = int(np.floor(p))
    tt = float(np.float32(p - np.float32(i0)))
    ox = taps[0, :, 1] - i0
    oy = taps[0, :, 2] - i0
    bins = np.arange(lo, hi + 2) - 0.5
    return tt, np.histogram(ox, bins)[0], np.histogram(oy, bins)[0]


@pytest.mark.parametrize("sigma", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("t", [0.0, 0.25, 0.625])
def test_fis_gauss_cell_probabilities(orc, sigma, t):
    """FIS with nearest lookup picks tap offset k with the Gaussian's mass
    over texel k's cell (chi^2 against scipy's normal CDF)."""
    tt, hx, hy = _offset_histogram(orc, orc.GAUSS_FIS, t, sigma, 200_000, -6, 7)
    k = np.arange(-6, 8)
    P = stats.norm.cdf((k + 0.5 - tt) / sigma) - stats.norm.cdf((k - 0.5 - tt) / sigma)
    for h in (hx, hy):
        m = P * h.sum() > 5
        obs = h[m]
        exp = P[m] / P[m].sum() * obs.sum()
        assert h[~m].sum() <= 40
        assert stats.chisquare(obs, exp).pvalue > 1e-4


# ------------------------------------------------------------ cubic B-spline by FIS
def test_fis_bspline_pick_is_exact_floor(orc):
    """The integer decision equals floor(t + (a+b+c) 2^-24 - 1) in exact
    arithmetic for t on the 2^-24 grid, including boundaries."""
    rng = np.random.default_rng(5)
    for _ in range(3000):
        t = int(rng.integers(0, 2 ** 24)) * U24
        w = [int(x) << 8 | int(rng.integers(0, 256)) for x in rng.integers(0, 2 ** 24, 3)]
        S = sum(x >> 8 for x in w)
        ref = math.floor(Fraction(t) + Fraction(S, 2 ** 24) - 1)
        assert orc.fis_bspline_pick(t, *w) == ref
    # boundary: S 2^-24 = 1 - t exactly advances
    t = 0.375
    S = int((1 - t) * 2 ** 24)
    assert orc.fis_bspline_pick(t, S << 8, 0, 0) == 0
    assert orc.fis_bspline_pick(t, (S - 1) << 8, 0, 0) == -1


@pytest.mark.parametrize("t", [0.0, 1e-3, 0.25, 0.5, 0.7, 0.999])
def test_fis_bspline_pmf_is_the_cubic_bspline(orc, t):
    """Sum of three uniforms + nearest = the cubic B-spline tap weights
    (Cox-de Boor), exactly up to the 24-bit lattice."""
    P = orc.fis_bspline_pmf(t)
    tt = float(np.float32(t))
    w = [orc.kbs(tt - (k - 1)) for k in range(4)]
    assert sum(P) == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.abs(P - w) <= 4 * U24)


@pytest.mark.parametrize("t", [0.1, 0.5, 0.8])
def test_fis_bspline_sampled_histogram(orc, t):
    tt, hx, hy = _offset_histogram(orc, orc.BSPLINE3_FIS, t, 0.5, 200_000, -1, 2)
    P = np.array([orc.kbs(tt - (k - 1)) for k in range(4)])
    for h in (hx, hy):
        m = P > 0
        assert h[~m].sum() == 0
        assert stats.chisquare(h[m], P[m] / P[m].sum() * h[m].sum()).pvalue > 1e-4


# ------------------------------------------------------------ discrete Gaussian (FRS)
@pytest.mark.parametrize("sigma", [1 / 16, 0.3, 0.5, 0.8, 2.0, 4.0])
def test_gauss_thresholds_match_fp64_cdf(orc, sigma):
    for t in np.linspace(0, 1, 41).astype(np.float32):
        d = np.arange(-1, 3) - np.float64(t)
        g = np.exp(-d * d / (2 * sigma * sigma))
        ref = np.cumsum(g)[:3] / g.sum()
        C = orc.gauss_thresholds(float(t), sigma)
        assert np.all(np.abs(C - ref) <= 1e-6), (t, C, ref)
        assert np.all(np.diff(C) >= 0)


@pytest.mark.parametrize("t, sigma", [(0.3, 0.3), (0.5, 0.5), (0.9, 0.8), (0.0, 1 / 16)])
def test_gauss_pick_pmf_by_brute_force(orc, t, sigma):
    """Pick probabilities over all 2^24 uniforms, counted in numpy."""
    C = orc.gauss_thresholds(t, sigma)
    u = (np.arange(2 ** 24, dtype=np.float64) * U24).astype(np.float32)
    j = (u >= C[0]).astype(np.int64) + (u >= C[1]) + (u >= C[2])
    counts = np.bincount(j, minlength=4) / 2 ** 24
    assert np.array_equal(counts, orc.gauss_pick_pmf(t, sigma))


# ------------------------------------------------------------ expectations
def _tex_and_queries():
    tex = inputs.texture_uniform(16, seed=4)
    q = inputs.queries_uniform(40, seed=5)
    return tex, q


@pytest.mark.parametrize("filt, sigma", [("GAUSS_FRS", 0.3), ("GAUSS_FRS", 0.8), ("BSPLINE3_FIS", 0.5)])
@pytest.mark.parametrize("shade", [0, 1])
def test_exact_expectation_equals_after(orc, filt, sigma, shade):
    """E[estimator] over the exact 24-bit pick probabilities = the exact
    filter-after value, within sum |P - w| max|shade|."""
    tex, q = _tex_and_queries()
    f = getattr(orc, filt)
    ot = orc.Tex2D.rgba32f(tex)
    E = orc.filter2d_expect(ot, q, f, shade=shade, sigma=sigma)
    A = orc.filter2d(ot, q, f, orc.AFTER, shade=shade, sigma=sigma)
    assert np.max(np.abs(E - A)) <= 16 * 8 * U24 * max(1.0, np.max(np.abs(A)))


def test_fis_bspline_after_is_the_bspline(orc):
    tex, q = _tex_and_queries()
    ot = orc.Tex2D.rgba32f(tex)
    for m in (orc.BEFORE, orc.AFTER):
        assert np.array_equal(orc.filter2d(ot, q, orc.BSPLINE3_FIS, m, shade=1),
                              orc.filter2d(ot, q, orc.BSPLINE3, m, shade=1))


@pytest.mark.parametrize("sigma", [0.3, 0.8, 4.0])
def test_gauss_fis_after_weights_and_constant(orc, sigma):
    """Cell masses sum to one: a constant texture filters to itself, and a
    unit impulse spreads into the product of the axis cell masses."""
    N = 64
    const = np.full((N, N, 4), 0.375, np.float32)
    q = inputs.queries_uniform(30, seed=6)
    out = orc.filter2d(orc.Tex2D.rgba32f(const), q, orc.GAUSS_FIS, orc.AFTER, sigma=sigma)
    assert np.allclose(out, 0.375, rtol=0, atol=0.375 * 4 * stats.norm.cdf(-7.0) + 1e-15)
    imp = np.zeros((N, N, 4), np.float32)
    imp[20, 30] = 1.0
    uq = np.array([[(30 + 0.5 + 0.3) / N, (20 + 0.5 - 0.2) / N, 0.0]], np.float32)
    v = orc.filter2d(orc.Tex2D.rgba32f(imp, wrap=orc.CLAMP), uq, orc.GAUSS_FIS, orc.AFTER, sigma=sigma)[0, 0]
    p = np.float32(uq[0, :2]) * np.float32(N) - np.float32(0.5)
    t = (p - np.floor(p)).astype(np.float64)
    kx, ky = 30.0 - float(np.floor(p[0])), 20.0 - float(np.floor(p[1]))
    s32 = float(np.float32(sigma))                  # the filters take sigma in binary32
    mass = [stats.norm.cdf((k + 0.5 - tt) / s32) - stats.norm.cdf((k - 0.5 - tt) / s32)
            for k, tt in ((kx, t[0]), (ky, t[1]))]
    assert v == pytest.approx(mass[0] * mass[1], rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("filt, sigma", [("GAUSS_FRS", 0.5), ("GAUSS_FIS", 0.3), ("GAUSS_FIS", 0.8),
                                         ("BSPLINE3_FIS", 0.5)])
def test_stochastic_mean_within_five_sigma(orc, filt, sigma):
    tex, q = _tex_and_queries()
    f = getattr(orc, filt)
    ot = orc.Tex2D.rgba32f(tex)
    A = orc.filter2d(ot, q, f, orc.AFTER, shade=1, sigma=sigma)
    spp = 4096
    S = orc.filter2d(ot, q, f, orc.STOCHASTIC, spp=spp, seed=11, shade=1, sigma=sigma)
    # per-sample standard deviation bounded by the range of shaded texel values
    tex_all = orc.filter2d(ot, inputs.queries_uniform(4000, seed=9), orc.NEAREST, orc.AFTER, shade=1)
    sd = (tex_all.max() - tex_all.min()) / 2
    assert np.all(np.abs(S - A) <= 5 * sd / math.sqrt(spp))


def test_sigma_range_is_checked(orc):
    tex, q = _tex_and_queries()
    with pytest.raises(ValueError):
        orc.filter2d(orc.Tex2D.rgba32f(tex), q, orc.GAUSS_FIS, orc.AFTER, sigma=8.0)
