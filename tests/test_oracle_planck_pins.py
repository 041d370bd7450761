"""Pins of the oracle's black-body emission (Sec. 5, "Filtering nonlinear
physical properties": temperatures shaded by Planck's law, filtered before
or after shading) against the laws that Planck's formula must reproduce and
against the filters' closed cases."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_2407_06107_amd import inputs

H, C, K = 6.62607015e-34, 299792458.0, 1.380649e-23       # exact SI values
WIEN_B = 2.897771955e-3                                    # m K (CODATA 2018)
STEFAN = 5.670374419e-8                                    # W m^-2 K^-4 (CODATA 2018)


@pytest.mark.parametrize("T", [800.0, 3000.0, 6000.0, 20000.0])
def test_wien_displacement(orc, T):
    """The spectrum peaks at lambda = b / T."""
    r = optimize.minimize_scalar(lambda l: -orc.planck(l, T), bracket=(0.5e9 * WIEN_B / T, 1e9 * WIEN_B / T,
                                                                      2e9 * WIEN_B / T), tol=1e-12)
    assert abs(r.x * 1e-9 * T / WIEN_B - 1.0) < 1e-6


@pytest.mark.parametrize("T", [800.0, 6000.0])
def test_stefan_boltzmann(orc, T):
    """pi times the integral of B over all wavelengths is sigma T^4."""
    peak = 1e9 * WIEN_B / T
    edges = [peak * f for f in (1e-2, 0.1, 0.3, 1.0, 3.0, 10.0, 100.0, 1e4)]
    tot = sum(integrate.quad(lambda l: orc.planck(l, T), a, b, epsabs=0, epsrel=1e-11, limit=200)[0]
              for a, b in zip(edges[:-1], edges[1:]))
    assert abs(math.pi * tot / (STEFAN * T ** 4) - 1.0) < 1e-6


def test_rayleigh_jeans_and_wien_limits(orc):
    """Long wavelengths: B -> 2 c k T / lambda^4 from below, within x/2
    (x = h c / (lambda k T)); short ones: B -> (2 h c^2 / lambda^5) e^-x from
    above, within a factor 1 + 2 e^-x."""
    for T in (300.0, 6000.0):
        for lam in (1e6, 1e7):                     # nm
            l = lam * 1e-9
            x = H * C / (l * K * T)
            rj = 2 * C * K * T / l ** 4 * 1e-9
            r = orc.planck(lam, T) / rj
            assert 1 - x / 2 - 1e-12 <= r <= 1.0
        for lam in (100.0, 300.0):
            l = lam * 1e-9
            x = H * C / (l * K * T)
            wien = 2 * H * C * C / l ** 5 * math.exp(-x) * 1e-9
            if wien > 0:
                r = orc.planck(lam, T) / wien
                assert 1.0 <= r <= 1 + 2 * math.exp(-x) + 1e-12


def test_special_temperatures(orc):
    assert orc.planck(546.1, 0.0) == 0.0 and orc.planck(546.1, -5.0) == 0.0
    assert math.isnan(orc.planck(546.1, float("nan")))
    # hotter is brighter at every wavelength
    for lam in orc.PLANCK_NM:
        v = [orc.planck(lam, T) for T in (500.0, 1000.0, 2000.0, 4000.0, 8000.0)]
        assert all(a < b for a, b in zip(v, v[1:]))


def _grid(data, side=1.0):
    import oracle
    return oracle.Grid(np.asarray(data), side=side)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode", ["BEFORE", "AFTER", "STOCHASTIC"])
def test_constant_temperature(orc, filt, mode):
    """A uniform 2000 K block: every mode gives B(2000) at a point and
    (t1 - t0) B(2000) along a ray that stays inside (partition of unity)."""
    n, T0 = 24, 2000.0
    g = _grid(np.full((n, n, n), T0, dtype=np.float16))
    B = np.array([orc.planck(l, T0) for l in orc.PLANCK_NM])
    m = getattr(orc, mode)
    f = getattr(orc, filt)
    pts = inputs.random_points(50, 0.3, 0.7, seed=3)
    out = orc.filter3d(g, pts, f, m, spp=3, seed=1, shade=orc.PLANCK)
    assert np.allclose(out, B[None], rtol=1e-13, atol=0)
    rng = np.random.default_rng(2)
    o = 0.35 + 0.3 * rng.random((30, 3))
    d = rng.normal(size=(30, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.concatenate([o, d, np.zeros((30, 1)), np.full((30, 1), 0.2)], 1).astype(np.float32)
    L = orc.raymarch_emission(g, rays, 16, f, m, spp=2, seed=4)
    dt = (np.float32(0.2) / np.float32(16)).astype(np.float64)
    assert np.allclose(L, 16 * dt * B[None], rtol=1e-13, atol=0)


def _fire(n=20, seed=5):
    import torch
    dens = inputs.cloud_grid(n, seed=seed)
    return inputs.temperature_grid(dens).numpy()


def test_before_is_planck_of_the_filtered_temperature(orc):
    """Filtering before shading = B(filtered temperature): the point lookup
    with PLANCK shading equals Planck's law applied to the plain filtered
    value of the same grid."""
    g = _grid(_fire())
    pts = inputs.random_points(200, 0.05, 0.95, seed=7)
    for f in (orc.LINEAR, orc.BSPLINE3):
        Tf = orc.filter3d(g, pts, f, orc.AFTER, shade=orc.DENSITY)
        out = orc.filter3d(g, pts, f, orc.BEFORE, shade=orc.PLANCK)
        ref = np.array([[orc.planck(l, t) for l in orc.PLANCK_NM] for t in Tf])
        assert np.allclose(out, ref, rtol=1e-13, atol=0)


def test_after_exceeds_before_by_convexity(orc):
    """Below h c/(2 lambda k) (13,200 K at 546 nm) B is convex in T, so by
    Jensen filtering after shading gives at least as much emission as
    filtering before, at every point and along every ray — strictly where the
    footprint sees different temperatures."""
    g = _grid(_fire())
    pts = inputs.random_points(300, 0.05, 0.95, seed=8)
    for f in (orc.LINEAR, orc.BSPLINE3):
        a = orc.filter3d(g, pts, f, orc.AFTER, shade=orc.PLANCK)
        b = orc.filter3d(g, pts, f, orc.BEFORE, shade=orc.PLANCK)
        assert np.all(a >= b * (1 - 1e-12))
        assert np.mean(a > b * 1.01) > 0.3
    rays = inputs.random_rays(100, 1.0, seed=9)
    a = orc.raymarch_emission(g, rays, 32, orc.BSPLINE3, orc.AFTER)
    b = orc.raymarch_emission(g, rays, 32, orc.BSPLINE3, orc.BEFORE)
    assert np.all(a >= b * (1 - 1e-12))


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
def test_emission_expectation_equals_after(orc, filt):
    """The stochastic emission's exact expectation (24-bit pick
    probabilities) is the filter-after emission: emission adds over steps, so
    one voxel per step is unbiased for the whole ray.  The 24-bit lattice
    moves each axis's pick probabilities by at most 2^-24 from the weights,
    so a step's expectation is within 3 * 2^-24 of the largest emission in
    its footprint (plus binary32 rounding of the thresholds)."""
    g = _grid(_fire())
    rays = inputs.random_rays(120, 1.0, seed=10)
    f = getattr(orc, filt)
    E = orc.raymarch_emission_expect(g, rays, 24, f)
    A = orc.raymarch_emission(g, rays, 24, f, orc.AFTER)
    Bmax = np.array([orc.planck(l, 6000.0) for l in orc.PLANCK_NM])
    dt = (rays[:, 7] - rays[:, 6]).astype(np.float64)[:, None] / 24
    assert np.all(np.abs(E - A) <= 24 * dt * 8 * 2.0 ** -24 * Bmax[None] + 1e-300)
    assert np.mean(np.abs(E - A) <= 64 * 2.0 ** -24 * np.abs(A)) > 0.9


def test_emission_stochastic_mean(orc):
    g = _grid(_fire())
    rays = inputs.random_rays(40, 1.0, seed=11)
    A = orc.raymarch_emission(g, rays, 24, orc.BSPLINE3, orc.AFTER)
    S = orc.raymarch_emission(g, rays, 24, orc.BSPLINE3, orc.STOCHASTIC, spp=2048, seed=3)
    # per-step emission lies in [0, B(6000)]: the sum over 24 steps has
    # standard deviation at most 24 dt B(6000) / 2 per ray, over sqrt(spp)
    Bmax = np.array([orc.planck(l, 6000.0) for l in orc.PLANCK_NM])
    dt = (rays[:, 7] - rays[:, 6]).astype(np.float64)[:, None] / 24
    assert np.all(np.abs(S - A) <= 5 * 24 * dt * Bmax[None] / 2 / math.sqrt(2048) + 1e-300)


def test_emission_misses_and_nonfinite(orc):
    g = _grid(_fire(8))
    rays = inputs.random_rays(4, 1.0, seed=12)
    rays[0, 6:8] = [0.5, 0.5]                  # empty segment
    rays[1, 0] = np.nan
    rays[2, 3] = 1e30                          # raster position overflows
    L, taps = orc.raymarch_emission(g, rays, 8, orc.BSPLINE3, orc.STOCHASTIC, spp=2, taps=True)
    assert np.all(L[0] == 0) and np.all(np.isnan(L[1])) and np.all(np.isnan(L[2])) and np.all(np.isfinite(L[3]))
    assert np.all(taps[:3] == orc.TAP_NONE)
    for m in (orc.BEFORE, orc.AFTER):
        L = orc.raymarch_emission(g, rays, 8, orc.BSPLINE3, m)
        assert np.all(L[0] == 0) and np.all(np.isnan(L[1:3]))


# ------------------------------------------------------------ perpendicular Gaussian footprint
def test_perp_jitter_is_perpendicular_and_gaussian(orc):
    """World offsets of the jittered steps lie in the plane perpendicular to
    the ray, and their components along any fixed orthonormal pair of that
    plane are independent N(0, sigma^2) (Kolmogorov-Smirnov)."""
    from scipy import stats
    g = _grid(np.zeros((16, 16, 16), np.float16))
    rng = np.random.default_rng(4)
    sigma = 0.03
    for d in ([0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [0.3, -0.5, 0.81], [1.0, 0.0, 0.0]):
        d = np.array(d) / np.linalg.norm(d)
        ray = np.array([0.5, 0.5, 0.5, *d, -0.2, 0.2], np.float32)
        base = orc.perp_jitter(g, ray, 8, 0.0, 0, 0, 3, 1).astype(np.float64)
        offs = np.array([(orc.perp_jitter(g, ray, 8, sigma, i, s, 3, 1) - base) / g.scale
                         for i in range(64) for s in range(32)], dtype=np.float64)
        assert np.max(np.abs(offs @ d)) <= 1e-5 * sigma
        # a fixed orthonormal pair of the plane
        e1 = np.cross(d, [0.0, 1.0, 0.0] if abs(d[1]) < 0.9 else [1.0, 0.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(d, e1)
        for e in (e1, e2):
            assert stats.kstest(offs @ e / sigma, "norm").pvalue > 1e-3
        assert abs(np.corrcoef(offs @ e1, offs @ e2)[0, 1]) < 0.1
    del rng


def test_footprint_blurs_an_edge_by_sigma(orc):
    """A hot half-space (3000 K for x < 1/2) seen by a ray parallel to z at
    x = 1/2 + delta: with the perpendicular Gaussian of standard deviation
    sigma, the expected emission is B(3000) (t1 - t0) times the
    B-spline-smoothed edge averaged over N(delta, sigma^2) — computed here by
    quadrature — and the stochastic mean over 4096 samples matches it."""
    from scipy import stats
    n = 64
    data = np.zeros((n, n, n), np.float16)
    data[:, :, : n // 2] = 3000.0
    g = _grid(data)
    sigma = 4.0 / n
    B = np.array([orc.planck(l, 3000.0) for l in orc.PLANCK_NM])

    def edge(xw):
        # filter-after fraction of the hot side at world x for the cubic B-spline
        p = xw * n - 0.5
        i0 = np.floor(p)
        t = p - i0
        w = [(1 - t) ** 3 / 6, (3 * t ** 3 - 6 * t ** 2 + 4) / 6, (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6, t ** 3 / 6]
        return sum(wk for k, wk in enumerate(w) if i0 - 1 + k < n // 2)

    for delta in (-1.5 * sigma, 0.0, 0.7 * sigma, 2.0 * sigma):
        x = 0.5 + delta
        ray = np.array([[x, 0.5, -1.0, 0.0, 0.0, 1.0, 1.1, 1.9]], np.float32)
        L = orc.raymarch_emission(g, ray, 48, orc.BSPLINE3, orc.STOCHASTIC, spp=4096, seed=9,
                                  footprint=sigma)[0]
        frac, _ = integrate.quad(lambda y: edge(y) * stats.norm.pdf(y, loc=float(np.float32(x)), scale=sigma),
                                 x - 8 * sigma, x + 8 * sigma, points=[0.5], limit=200)
        expect = 0.8 * frac * B
        assert np.all(np.abs(L - expect) <= 5 * 0.8 * B * 0.5 / math.sqrt(4096 * 48) + 1e-9 * B), (delta, L / (0.8 * B),
                                                                                                   frac)


def test_footprint_zero_is_the_plain_march(orc):
    g = _grid(_fire())
    rays = inputs.random_rays(50, 1.0, seed=13)
    a, ta = orc.raymarch_emission(g, rays, 16, orc.BSPLINE3, orc.STOCHASTIC, spp=2, seed=5, taps=True)
    b, tb = orc.raymarch_emission(g, rays, 16, orc.BSPLINE3, orc.STOCHASTIC, spp=2, seed=5, taps=True,
                                  footprint=0.0)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)
