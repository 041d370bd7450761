"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against an
independent fact (a convolution identity, a closed form, brute force on tiny
inputs, a library routine, an invariant), chosen so that a plausible mistake
in the oracle (a dropped term, a shifted tap, a wrong sign) fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2407_06107_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- kernels (S.2)
def _box_power(k: int, h: float):
    """Density of the sum of k unit-width uniforms centred at 0, sampled on a
    grid of spacing h, by repeated discrete convolution of the box."""
    m = int(round(1.0 / h))
    box = np.ones(m) / m
    acc = box
    for _ in range(k - 1):
        acc = np.convolve(acc, box)
    x = (np.arange(acc.size) - (acc.size - 1) / 2.0) * h
    return x, acc / (acc.sum() * h)


@pytest.mark.parametrize("k, name", [(2, "tent"), (4, "bspline")])
def test_kernels_are_box_convolutions(orc, k, name):
    """Suppl. S.2 / Sec. 4.2: the tent is box*box and the cubic B-spline is
    box*box*box*box (Cox-de Boor).  Independent of the closed forms."""
    x, dens = _box_power(k, 1e-3)
    f = orc.ktent if name == "tent" else orc.kbs
    xs = np.linspace(-k / 2 + 0.05, k / 2 - 0.05, 41)
    got = np.array([f(v) for v in xs])
    ref = np.interp(xs, x, dens)
    assert np.max(np.abs(got - ref)) < 3e-3


def test_kbs_special_values_and_partition(orc):
    assert orc.kbs(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert orc.kbs(1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert orc.kbs(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert orc.kbs(2.0) == 0.0 and orc.kbs(-2.5) == 0.0
    # partition of unity and non-negativity for every fractional offset
    for t in np.linspace(0, 1, 101):
        w = orc.axis_weights64(orc.BSPLINE3, t)
        assert np.all(w >= 0.0)
        assert abs(w.sum() - 1.0) < 1e-15
        wt = orc.axis_weights64(orc.LINEAR, t)
        assert abs(wt[:2].sum() - 1.0) < 1e-15


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
def test_linear_reproduction(orc, filt):
    """Tent and cubic B-spline reproduce affine functions:
    sum_k K(x - k) (a + b k) = a + b x.  Pins the tap offsets: a weight set
    shifted by one texel misses by b."""
    f = getattr(orc, filt)
    off = -1 if filt == "BSPLINE3" else 0
    for t in np.linspace(0, 0.999, 37):
        w = orc.axis_weights64(f, t)
        taps = np.arange(4) + off
        assert abs(np.dot(w, 2.0 + 3.0 * taps) - (2.0 + 3.0 * t)) < 1e-13


# -------------------------------------------- binary32 thresholds and picking
def test_thresholds_match_closed_form(orc):
    ts = np.linspace(0.0, 1.0, 2001, dtype=np.float32)
    for t in ts:
        c = orc.thresholds(orc.BSPLINE3, t)
        w = np.array([orc.kbs(1 + float(t)), orc.kbs(float(t)), orc.kbs(1 - float(t)), orc.kbs(2 - float(t))])
        ref = np.array([w[0], w[0] + w[1], 1.0 - w[3]])
        assert np.max(np.abs(c.astype(np.float64) - ref)) < 3e-7
        assert 0.0 <= c[0] <= c[1] <= c[2] <= 1.0
        ct = orc.thresholds(orc.LINEAR, t)
        assert abs(float(ct[0]) - (1.0 - float(t))) < 1e-7


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("t", [0.0, 0.123456, 0.5, 0.75, 0.99999994])
def test_pick_pmf_brute_force(orc, filt, t):
    """The exact pick probabilities over the 2^24-point uniform lattice,
    counted by brute force, match the closed-form count, and lie within
    2^-24 + 2 eps32 of the kernel weights."""
    f = getattr(orc, filt)
    u = np.arange(1 << 24, dtype=np.float32) * np.float32(2.0 ** -24)
    c = orc.thresholds(f, np.float32(t))
    j = np.zeros(u.size, dtype=np.int64)
    for ck in c:
        j += (u >= ck)
    counts = np.bincount(j, minlength=4)[:4] / float(1 << 24)
    pmf = orc.pick_pmf(f, np.float32(t))
    assert np.array_equal(counts, pmf)
    w = orc.axis_weights64(f, float(np.float32(t)))
    assert np.max(np.abs(pmf - w)) <= 2.0 ** -24 + 2.4e-7
    # the per-uniform pick of the oracle agrees with the counted rule
    for k in range(0, 1 << 24, (1 << 24) // 257):
        assert orc.pick(f, np.float32(t), u[k]) == j[k]


def test_zero_weight_tap_never_picked(orc):
    """At t = 0 the B-spline's last tap has weight 0; at t -> 1 the first."""
    assert orc.pick_pmf(orc.BSPLINE3, 0.0)[3] == 0.0
    assert orc.pick_pmf(orc.BSPLINE3, 1.0)[0] == 0.0
    assert orc.pick_pmf(orc.LINEAR, 0.0)[1] == 0.0


def test_fis_sum_of_uniforms_matches_frs_pmf(orc):
    """Sec. 4.2: a degree-3 B-spline tap can be drawn by jittering the point by
    the sum of three uniforms (a degree-2 spline) and taking the nearest
    texel.  The tap histogram of that sampler, which uses no weight code,
    equals the oracle's pick distribution (chi-square, 4 bins)."""
    rng = np.random.default_rng(7)
    n = 4_000_000
    for t in (0.1, 0.37, 0.5, 0.83):
        x = t + rng.random(n) + rng.random(n) + rng.random(n) - 1.5
        tap = np.floor(x + 0.5).astype(np.int64)      # nearest texel, relative to i0
        hist = np.bincount(tap + 1, minlength=4)[:4]
        p = orc.pick_pmf(orc.BSPLINE3, np.float32(t))
        exp = p * n
        mask = exp > 0
        chi2 = np.sum((hist[mask] - exp[mask]) ** 2 / exp[mask])
        assert hist[~mask].sum() == 0
        assert chi2 < 20.0, (t, hist, exp)


def test_sampling_arrays_worked_example(orc):
    """Sec. 4.3 figure (FRS panels): the printed weights -> probabilities,
    under the reading recorded in the fixture."""
    g = json.load(open(os.path.join(GOLD, "frs_worked_example.json")))
    w = np.array(g["weights_read"]).ravel()
    printed = np.array(g["probabilities_percent_as_printed"]).ravel() / 100.0
    assert abs(np.array(g["weights_as_printed"]).sum() - 0.9) < 1e-12     # the garble
    m = 100_000
    xi = (np.arange(m) + 0.5) / m
    picks = np.array([orc.sample_array(w, x) for x in xi])
    freq = np.bincount(picks, minlength=9) / m
    assert np.max(np.abs(freq - printed)) < 1e-4


def test_reuse_variant_distribution(orc):
    """Uniform sample reuse (Sec. 2.2) keeps the joint distribution separable:
    over all 2^24 uniforms the (jx, jy) histogram is the product of the axis
    weights."""
    for tx, ty in ((0.25, 0.6), (0.9, 0.05)):
        h = orc.reuse_histogram2(orc.BSPLINE3, tx, ty) / float(1 << 24)
        wx = orc.axis_weights64(orc.BSPLINE3, tx)
        wy = orc.axis_weights64(orc.BSPLINE3, ty)
        assert np.max(np.abs(h - np.outer(wy, wx))) < 2e-6


def test_weighted_reservoir_matches_inverse_cdf(orc):
    """Weighted reservoir sampling (Sec. 2.2, Chao 1982): keep item i with
    probability w_i / sum_{k<=i} w_k.  Its distribution over a fine uniform
    grid equals the inverse-CDF pick distribution of the oracle."""
    m = 200_000
    for t in (0.2, 0.71):
        w = orc.axis_weights64(orc.BSPLINE3, t)
        rng = np.random.default_rng(3)
        u = rng.random((m, 4))
        sel = np.zeros(m, dtype=np.int64)
        run = np.zeros(m)
        for i in range(4):
            run = run + w[i]
            keep = u[:, i] < w[i] / run
            sel[keep] = i
        freq = np.bincount(sel, minlength=4) / m
        p = orc.pick_pmf(orc.BSPLINE3, np.float32(t))
        assert np.max(np.abs(freq - p)) < 5 * math.sqrt(0.25 / m)


# ----------------------------------------------------------------- RNG hash
def test_pcg4d_uniform_and_mixing(orc):
    """Statistical pins of the hash: distinct keys give distinct outputs (it
    is a bijection), the 24-bit uniforms are uniform (chi-square over 256
    bins) for each word, and flipping one key bit flips about half of the
    output bits for the key bits the filters use."""
    n = 1 << 18
    q = np.arange(n, dtype=np.uint32)
    keys = np.stack([q, q % 16, q // 16 % 256, np.full(n, 12345, np.uint32)], axis=1)
    out = orc.pcg4d(keys)
    packed = out.view(np.dtype((np.void, 16))).ravel()
    assert np.unique(packed).size == n
    for w in range(4):
        b = (out[:, w] >> 24).astype(np.int64)
        h = np.bincount(b, minlength=256)
        chi2 = np.sum((h - n / 256) ** 2 / (n / 256))
        assert chi2 < 340, (w, chi2)     # 255 dof, p ~ 1e-3
    base = keys[:4096].copy()
    o0 = orc.pcg4d(base)
    for word in range(4):
        # keys use the low bits of each word (query, sample, step < 2^24);
        # a multiplicative hash mixes its top input bit weakly by design
        for bit, lo in ((0, 0.45), (7, 0.45), (15, 0.45), (23, 0.3)):
            k = base.copy()
            k[:, word] ^= np.uint32(1 << bit)
            o1 = orc.pcg4d(k)
            flips = np.unpackbits((o0 ^ o1).view(np.uint8)).mean()
            assert lo < flips < 0.55, (word, bit, flips)


# --------------------------------------------------------------- fp16 decode
def test_half_decode_all_patterns(orc):
    bits = np.arange(1 << 16, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = np.array([orc.half_to_double(int(b)) for b in bits[::7]])
    r = ref[::7]
    nan = np.isnan(r)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], r[~nan])


# ---------------------------------------------------------------------- GGX
def _sph_dirs(nt=400, npp=800):
    th = (np.arange(nt) + 0.5) / nt * (math.pi / 2)
    ph = (np.arange(npp) + 0.5) / npp * 2 * math.pi
    T, P = np.meshgrid(th, ph, indexing="ij")
    dw = (math.pi / 2 / nt) * (2 * math.pi / npp) * np.sin(T)
    return T, P, dw


def test_ggx_closed_forms(orc):
    # normal incidence, n = wo = wi = z, alpha = 1 (r = 1): D = 1/pi, G = 1, F = f0
    p = orc.ggx_params(n=(0, 0, 1), wo=(0, 0, 1), wi=(0, 0, 1), radiance=(2.0, 1.0, 0.5), f0=0.04,
                       r_bias=1.0, r_scale=0.0)
    alb = np.array([0.3, 0.6, 0.9, 0.0])
    got = orc.shade_ggx(p, alb)
    ref = np.array([2.0, 1.0, 0.5]) * (alb[:3] / math.pi + (1 / math.pi) * 1.0 * 0.04 / 4.0)
    assert np.allclose(got, ref, rtol=1e-14)


def test_ggx_reciprocity_and_positivity(orc):
    rng = np.random.default_rng(5)
    for _ in range(20):
        wo = rng.normal(size=3); wo[2] = abs(wo[2]) + 0.2
        wi = rng.normal(size=3); wi[2] = abs(wi[2]) + 0.2
        a = orc.ggx_params(wo=wo, wi=wi)
        b = orc.ggx_params(wo=wi, wi=wo)
        rgba = np.array([0.4, 0.5, 0.6, rng.random()])
        fa = orc.shade_ggx(a, rgba) / a[8]      # divide out the cosine n.wi
        fb = orc.shade_ggx(b, rgba) / b[8]
        assert np.allclose(fa, fb, rtol=1e-12)
        assert np.all(fa > 0)


def test_ggx_ndf_normalisation(orc):
    """The microfacet distribution integrates to one over projected solid
    angle: int D(h) (n.h) dw_h = 1.  D is extracted from the shaded value at
    wo = wi = h (so G and F are known) by numerical quadrature."""
    T, P, dw = _sph_dirs(300, 4)
    for r in (0.3, 0.6, 0.9):
        total = 0.0
        for t, d in zip(T[:, 0], dw[:, 0]):
            h = np.array([math.sin(t), 0.0, math.cos(t)])
            p = orc.ggx_params(n=(0, 0, 1), wo=h, wi=h, radiance=(1, 1, 1), f0=1.0, r_bias=r, r_scale=0.0)
            L = orc.shade_ggx(p, np.zeros(4))[0]
            c = math.cos(t)
            a2 = r ** 4
            g1 = 2 * c / (c + math.sqrt(a2 + (1 - a2) * c * c))
            D = L * 4 * c * c / (g1 * g1 * c)  # L = D G F / (4 c c) * c with F = 1
            total += D * c * d * 4           # 4 azimuth cells of 2pi/4 each (isotropic)
        assert abs(total - 1.0) < 2e-3, (r, total)


# ------------------------------------------------------------ 2-D filtering
def _ramp_tex(n=16):
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    tex = np.zeros((n, n, 4), dtype=np.float32)
    tex[..., 0] = 0.1 + 0.02 * x
    tex[..., 1] = 0.2 + 0.03 * y
    tex[..., 2] = 0.05 + 0.01 * x + 0.02 * y
    tex[..., 3] = 0.5
    return tex


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
def test_filter2d_before_reproduces_ramp(orc, filt):
    """Texel centres sit at integer raster coordinates p = u*N - 1/2: a linear
    ramp is reproduced at that point (pins the coordinate convention)."""
    n = 16
    tex = orc.Tex2D.rgba32f(_ramp_tex(n), wrap=orc.CLAMP)
    rng = np.random.default_rng(1)
    q = np.zeros((200, 3), dtype=np.float32)
    q[:, :2] = 0.25 + 0.5 * rng.random((200, 2))
    out = orc.filter2d(tex, q, getattr(orc, filt), orc.BEFORE, shade=0)
    px = q[:, 0].astype(np.float64) * n - 0.5
    py = q[:, 1].astype(np.float64) * n - 0.5
    assert np.allclose(out[:, 0], 0.1 + 0.02 * px, atol=1e-6)
    assert np.allclose(out[:, 1], 0.2 + 0.03 * py, atol=1e-6)
    assert np.allclose(out[:, 2], 0.05 + 0.01 * px + 0.02 * py, atol=1e-6)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
def test_filter2d_affine_before_equals_after(orc, filt):
    """Sec. 3: an affine contribution gives the same result filtered before
    or after shading: shade=none, and GGX with constant roughness (albedo is
    linear in the shaded value)."""
    tex = inputs.texture_uniform(8, seed=3)
    T = orc.Tex2D.rgba32f(tex)
    q = inputs.queries_uniform(300, seed=4)
    f = getattr(orc, filt)
    b = orc.filter2d(T, q, f, orc.BEFORE, shade=0)
    a = orc.filter2d(T, q, f, orc.AFTER, shade=0)
    assert np.allclose(a, b, rtol=0, atol=1e-14)
    tex2 = tex.copy()
    tex2[..., 3] = 0.4
    T2 = orc.Tex2D.rgba32f(tex2)
    b = orc.filter2d(T2, q, f, orc.BEFORE, shade=1)
    a = orc.filter2d(T2, q, f, orc.AFTER, shade=1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)


def test_filter2d_nonlinear_gap(orc):
    """With roughness varying, GGX makes before and after differ."""
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(16, seed=1))
    q = inputs.queries_uniform(200, seed=2)
    b = orc.filter2d(T, q, orc.BSPLINE3, orc.BEFORE, shade=1)
    a = orc.filter2d(T, q, orc.BSPLINE3, orc.AFTER, shade=1)
    assert np.max(np.abs(a - b)) > 1e-3


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter2d_expectation_equals_after(orc, filt, shade):
    """Unbiasedness (Sec. 2.2): the stochastic estimator's exact expectation (exact
    pick probabilities of the 24-bit uniforms) equals the exact filtering
    after shading value, within sum |P - w| * max|shade|."""
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(4, seed=9))
    q = inputs.queries_uniform(64, seed=10)
    f = getattr(orc, filt)
    e = orc.filter2d_expect(T, q, f, shade=shade)
    a = orc.filter2d(T, q, f, orc.AFTER, shade=shade)
    assert np.max(np.abs(e - a)) < 2e-6


@pytest.mark.parametrize("variant", [0, 1])
def test_filter2d_stochastic_mean_converges(orc, variant):
    """The oracle's stochastic estimator, averaged over many samples, is
    within 5 standard errors of its exact expectation."""
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(8, seed=11))
    q = inputs.queries_uniform(16, seed=12)
    spp = 20000
    s = orc.filter2d(T, q, orc.BSPLINE3, orc.STOCHASTIC, spp=spp, seed=5, variant=variant, shade=1)
    e = orc.filter2d_expect(T, q, orc.BSPLINE3, shade=1)
    # per-sample std bounded by the spread of shaded texel values
    one = orc.filter2d(T, q, orc.BSPLINE3, orc.STOCHASTIC, spp=1, seed=5, shade=1)
    sd = 0.5 * (one.max() - one.min()) + 1e-3
    assert np.max(np.abs(s - e)) < 5 * sd / math.sqrt(spp)


def test_filter2d_taps_in_footprint(orc):
    """Every stochastic tap lies in the 4x4 B-spline footprint of its query."""
    n = 16
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(n, seed=1), wrap=orc.CLAMP)
    q = inputs.queries_uniform(500, seed=3)
    _, taps = orc.filter2d(T, q, orc.BSPLINE3, orc.STOCHASTIC, spp=8, seed=1, taps=True)
    i0x = np.floor(q[:, 0] * n - 0.5).astype(int)
    i0y = np.floor(q[:, 1] * n - 0.5).astype(int)
    lo_x = np.clip(i0x - 1, 0, n - 1)[:, None]
    hi_x = np.clip(i0x + 2, 0, n - 1)[:, None]
    lo_y = np.clip(i0y - 1, 0, n - 1)[:, None]
    hi_y = np.clip(i0y + 2, 0, n - 1)[:, None]
    assert np.all((taps[..., 1] >= lo_x) & (taps[..., 1] <= hi_x))
    assert np.all((taps[..., 2] >= lo_y) & (taps[..., 2] <= hi_y))


def test_filter2d_mip_levels(orc):
    """Stochastic level choice between floor(lambda) and floor(lambda)+1 with
    P(upper) = frac(lambda) (Sec. 4.2.1); the expectation of the two-level
    estimator equals the (1-f, f) blend of per-level exact-after values."""
    lv = inputs.mip_chain(inputs.texture_sinusoids(32, seed=3, waves=8))
    q8 = inputs.quantize_unorm8(lv)
    buf, offs = inputs.pack_levels(q8)
    T = orc.Tex2D(buf, 32, 32, len(q8), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    q = inputs.queries_uniform(50, seed=4)
    q[:, 2] = np.linspace(0.0, 4.9, 50, dtype=np.float32)
    e = orc.filter2d_expect(T, q, orc.BSPLINE3, shade=1)
    a = orc.filter2d(T, q, orc.BSPLINE3, orc.AFTER, shade=1)
    assert np.max(np.abs(e - a)) < 2e-6
    _, taps = orc.filter2d(T, q, orc.BSPLINE3, orc.STOCHASTIC, spp=64, seed=2, shade=1, taps=True)
    lam = q[:, 2]
    lvl = taps[..., 0]
    assert np.all((lvl == np.floor(lam)[:, None]) | (lvl == np.floor(lam)[:, None] + 1))
    frac_up = (lvl > np.floor(lam)[:, None]).mean(axis=1)
    f = lam - np.floor(lam)
    assert np.mean(np.abs(frac_up - f)) < 0.1


def test_filter2d_nonfinite_queries(orc):
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(4, seed=1))
    q = np.array([[np.nan, 0.5, 0.0], [0.5, np.inf, 0.0], [0.3, 0.3, 0.0]], dtype=np.float32)
    out, taps = orc.filter2d(T, q, orc.BSPLINE3, orc.STOCHASTIC, spp=2, taps=True, shade=1)
    assert np.all(np.isnan(out[:2])) and np.all(np.isfinite(out[2]))
    assert np.all(taps[:2] == orc.TAP_NONE)


# ------------------------------------------------------------ 3-D path
def _grid(data, side=1.0):
    import oracle
    return oracle.Grid(np.asarray(data), side=side)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode", ["BEFORE", "AFTER", "STOCHASTIC"])
def test_raymarch_constant_density_beer_lambert(orc, filt, mode):
    """Constant sigma = c inside a grid whose rays stay well clear of the
    border: every mode gives exp(-c (t1 - t0)) (Beer-Lambert), with zero
    variance for the stochastic one."""
    n = 24
    c = 3.5
    g = _grid(np.full((n, n, n), c, dtype=np.float16))
    rng = np.random.default_rng(2)
    m = 40
    o = 0.35 + 0.3 * rng.random((m, 3))
    d = rng.normal(size=(m, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((m, 8), np.float32)
    rays[:, :3] = o; rays[:, 3:6] = d
    rays[:, 6] = 0.0; rays[:, 7] = 0.15
    T = orc.raymarch(g, rays, 32, getattr(orc, filt), getattr(orc, mode), spp=3, seed=1)
    L = rays[:, 7].astype(np.float64) - rays[:, 6]
    assert np.allclose(T, np.exp(-c * L), rtol=2e-6)


def test_raymarch_linear_ramp_before_is_exact(orc):
    """sigma linear in x: the B-spline (and tent) reproduce it, and the
    midpoint rule integrates a linear function exactly, so filter-before
    transmittance equals exp(-integral sigma ds) along the ray."""
    n = 32
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    data = (1.0 + 0.25 * x).astype(np.float32)
    g = _grid(data)
    rng = np.random.default_rng(4)
    m = 30
    o = 0.3 + 0.4 * rng.random((m, 3))
    d = rng.normal(size=(m, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((m, 8), np.float32)
    rays[:, :3] = o; rays[:, 3:6] = d; rays[:, 7] = 0.2
    for filt in (orc.LINEAR, orc.BSPLINE3):
        T = orc.raymarch(g, rays, 64, filt, orc.BEFORE)
        # raster x at parameter s: px(s) = (ox + s dx)*n - 0.5; sigma = 1 + 0.25 px
        o64, d64 = rays[:, 0].astype(np.float64), rays[:, 3].astype(np.float64)
        L = rays[:, 7].astype(np.float64)
        integral = L * (1.0 + 0.25 * ((o64 + 0.5 * L * d64) * n - 0.5))
        assert np.allclose(T, np.exp(-integral), rtol=2e-5)


def test_raymarch_jensen_and_expectation(orc):
    """exp is convex, so per ray T_after >= T_before (Jensen); the exact
    expectation of the stochastic estimator equals T_after within the
    24-bit pick-probability error; the stochastic mean converges to it."""
    g = _grid(inputs.cloud_grid(16, seed=4).numpy(), side=1.0)
    rays = inputs.random_rays(64, 1.0, seed=5)
    hit = rays[:, 7] > rays[:, 6]
    for filt in (orc.LINEAR, orc.BSPLINE3):
        b = orc.raymarch(g, rays, 24, filt, orc.BEFORE)
        a = orc.raymarch(g, rays, 24, filt, orc.AFTER)
        e = orc.raymarch_expect(g, rays, 24, filt)
        assert np.all(a[hit] >= b[hit] - 1e-12)
        assert np.max(np.abs(e - a)) < 1e-5
        assert np.all(a[~hit] == 1.0)
    spp = 4000
    s = orc.raymarch(g, rays[:16], 24, orc.BSPLINE3, orc.STOCHASTIC, spp=spp, seed=3)
    e = orc.raymarch_expect(g, rays[:16], 24, orc.BSPLINE3)
    assert np.max(np.abs(s - e)) < 5 * 0.5 / math.sqrt(spp)


def test_filter3d_modes(orc):
    """Point queries: B-spline reproduces a linear field (before), affine
    before == after for shade=none, exp shading obeys Jensen."""
    n = 16
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    g = _grid((0.5 + 0.1 * x + 0.2 * y + 0.05 * z).astype(np.float32))
    p = inputs.random_points(100, 0.3, 0.7, seed=1)
    for filt in (orc.LINEAR, orc.BSPLINE3):
        b = orc.filter3d(g, p, filt, orc.BEFORE)
        a = orc.filter3d(g, p, filt, orc.AFTER)
        r = p.astype(np.float64) * n - 0.5
        assert np.allclose(b, 0.5 + 0.1 * r[:, 0] + 0.2 * r[:, 1] + 0.05 * r[:, 2], atol=1e-6)
        assert np.allclose(a, b, atol=1e-12)
        eb = orc.filter3d(g, p, filt, orc.BEFORE, shade=1, ds=0.7)
        ea = orc.filter3d(g, p, filt, orc.AFTER, shade=1, ds=0.7)
        assert np.all(ea >= eb - 1e-14)


def test_raymarch_border_zero_and_nonfinite(orc):
    g = _grid(np.full((8, 8, 8), 2.0, np.float32))
    rays = np.array([[2.0, 2.0, 2.0, 1, 0, 0, 0.0, 0.5],       # far outside: T = 1
                     [np.nan, 0, 0, 1, 0, 0, 0.0, 0.5],        # NaN -> NaN
                     [0.5, 0.5, 0.5, 1, 0, 0, 0.3, 0.3]],      # empty segment -> 1
                    dtype=np.float32)
    T, taps = orc.raymarch(g, rays, 8, orc.BSPLINE3, orc.STOCHASTIC, taps=True)
    assert T[0] == 1.0 and np.isnan(T[1]) and T[2] == 1.0
    assert np.all(taps[1] == orc.TAP_NONE) and np.all(taps[2] == orc.TAP_NONE)


def test_occupancy_mask_property(orc):
    """A clear occupancy bit means every filter tap around any point of the
    brick reads zero (so skipping the step is exact); a set bit means a
    non-zero voxel lies within 2 voxels of the brick."""
    data = inputs.cloud_grid(24, seed=6).numpy()
    data[:, :, 12:] = 0.0
    g = _grid(data)
    lg, B = 2, 4
    words = orc.build_occupancy(g, lg)
    nb = 24 // B
    rng = np.random.default_rng(0)
    n_clear = 0
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                b = (bz * nb + by) * nb + bx
                bit = (words[b >> 5] >> (b & 31)) & 1
                lo = np.array([bx, by, bz]) * B
                sl = tuple(slice(max(c - 2, 0), c + B + 2) for c in (lo[2], lo[1], lo[0]))
                assert bit == int(np.any(data[sl] != 0))
                if not bit:
                    n_clear += 1
                    # points whose floor(raster) lies in the brick
                    p = (lo[None] + rng.random((20, 3)) * B + 0.5) / 24.0
                    for filt in (orc.LINEAR, orc.BSPLINE3):
                        v = orc.filter3d(g, p.astype(np.float32), filt, orc.BEFORE)
                        assert np.all(v == 0.0)
    assert n_clear > 0


def test_occupancy_nearest_brick_is_exact_outside_the_grid(orc):
    """The deterministic comparators test the brick nearest to a lookup point
    (its brick coordinates clamped to the grid's bricks), also for points
    outside the grid: a point whose trilinear or tricubic value is non-zero never meets a
    clear bit.  Points on a raster range 4 voxels beyond every face; the data
    are zero near the low x and z faces and the high x face, so clamped
    bricks there are clear."""
    data = inputs.cloud_grid(24, seed=6).numpy()
    data[:, :, :6] = 0.0
    data[:, :, 18:] = 0.0
    data[:5] = 0.0
    g = _grid(data)
    lg, nb = 2, 6
    words = orc.build_occupancy(g, lg)
    rng = np.random.default_rng(1)
    raster = rng.uniform(-4.0, 28.0, size=(40000, 3))
    p = ((raster + 0.5) / 24.0).astype(np.float32)
    r32 = (p.astype(np.float64) * 24.0 - 0.5).astype(np.float32)     # fma(p, 24, -1/2) in binary32
    i0 = np.floor(r32).astype(np.int64)
    bc = np.clip(i0 >> lg, 0, nb - 1)
    b = (bc[:, 2] * nb + bc[:, 1]) * nb + bc[:, 0]
    bit = (words[b >> 5] >> (b & 31)) & 1
    outside = np.any((i0 < 0) | (i0 >= 24), axis=1)
    clear = bit == 0
    assert (clear & outside).sum() > 3000 and (~clear & outside).sum() > 3000
    for filt in (orc.LINEAR, orc.BSPLINE3):
        v = orc.filter3d(g, p, filt, orc.BEFORE)
        assert np.all(v[clear] == 0.0)
        assert np.any(v[~clear & outside] != 0.0)


def test_occupancy_lookup_without_clamps_is_exact(orc):
    """The ray march tests a lookup point's brick in the padded mask (one
    bit per brick, 1 = the oracle's clear bit, in rows of nb + 1 bits and
    planes of nb + 1 rows, the padding 0) at bit index (bz*sy + by)*sx + bx
    from arithmetic shifts of floor(raster), reading 0 past the end.  For
    points anywhere on a raster range far beyond every face (brick
    coordinates -10..16 of 6), a point that meets a 1 has trilinear and
    tricubic value exactly 0.  The data are zero near the low x and z faces
    and the high x face, so bricks there hold 1s; points within one brick
    outside the grid always meet a 0 (padding, or past the end), and points
    further out alias onto arbitrary bits, which is exact because all of
    their taps lie outside the grid."""
    data = inputs.cloud_grid(24, seed=6).numpy()
    data[:, :, :6] = 0.0
    data[:, :, 18:] = 0.0
    data[:5] = 0.0
    g = _grid(data)
    lg, nb = 2, 6
    words = orc.build_occupancy(g, lg)
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:nb ** 3].reshape(nb, nb, nb)
    sx = sy = nb + 1
    mask = np.zeros((nb, sy, sx), np.uint8)
    mask[:, :nb, :nb] = 1 - bits
    flat = np.concatenate([mask.ravel(), np.zeros(-mask.size % 32, np.uint8)])   # whole 32-bit words
    rng = np.random.default_rng(1)
    raster = rng.uniform(-40.0, 64.0, size=(60000, 3))
    p = ((raster + 0.5) / 24.0).astype(np.float32)
    r32 = (p.astype(np.float64) * 24.0 - 0.5).astype(np.float32)     # fma(p, 24, -1/2) in binary32
    i0 = np.floor(r32).astype(np.int64)
    b = i0 >> lg
    idx = (b[:, 2] * sy + b[:, 1]) * sx + b[:, 0]        # within 24-bit operands here
    u = idx % 2 ** 32                                    # the unsigned index; word offset (u >> 3) & ~3
    skip = np.zeros(len(u), bool)
    inside = (u >> 5) < flat.size // 32
    skip[inside] = flat[u[inside]] == 1
    near = np.all((b >= -1) & (b <= nb), axis=1)
    outside = np.any((i0 < 0) | (i0 >= 24), axis=1)
    assert (skip & ~outside).sum() > 100                 # empty bricks inside the grid are skipped
    assert not (skip & near & outside).any()             # points just outside meet padding or the end
    assert (skip & ~near).sum() > 2000                   # far points alias onto bytes: any answer is exact
    for filt in (orc.LINEAR, orc.BSPLINE3):
        v = orc.filter3d(g, p, filt, orc.BEFORE)
        assert np.all(v[skip] == 0.0)
        assert np.any(v[~skip & outside & near] != 0.0)


# ------------------------------------------------- Keys cubic, positivisation
def test_keys_cubic_interpolates_and_reproduces_quadratics(orc):
    """S.2's K3 with a = -1/2 interpolates (K3(0) = 1, K3(+-1) = K3(+-2) = 0)
    and, for that a, reproduces polynomials up to degree two (Keys 1981)."""
    assert orc.k3(0.0) == 1.0
    for x in (1.0, -1.0, 2.0, -2.0, 2.5):
        assert orc.k3(x) == 0.0
    for t in np.linspace(0, 0.999, 31):
        w = orc.axis_weights64(orc.KEYS3, t)
        k = np.arange(4) - 1.0
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(np.dot(w, k) - t) < 1e-14
        assert abs(np.dot(w, k * k) - t * t) < 1e-14
        if 0 < t < 1:
            assert w[0] < 0 and w[3] < 0 and w[1] > 0 and w[2] > 0


def test_keys_positivised_expectation_equals_after(orc):
    """The exact expectation of W+ f(t+) - W- f(t-) over the 24-bit uniforms
    (every binary32 decision counted by brute force) equals the exact
    filter-after value (signed Keys weights)."""
    T = orc.Tex2D.rgba32f(inputs.texture_uniform(8, seed=4))
    q = inputs.queries_uniform(4, seed=5)
    e = orc.keys_expect2d(T, q, shade=1)
    a = orc.filter2d(T, q, orc.KEYS3, orc.AFTER, shade=1)
    assert np.max(np.abs(e - a)) < 2e-6


def test_keys_stochastic_mean_and_texel_centres(orc):
    """The stochastic estimator converges to the filter-after value; at texel
    centres (t = 0) the negative set is empty and every sample returns the
    centre texel itself (zero variance)."""
    tex = inputs.texture_uniform(8, seed=4)
    T = orc.Tex2D.rgba32f(tex)
    q = inputs.queries_uniform(8, seed=6)
    spp = 20000
    s = orc.filter2d(T, q, orc.KEYS3, orc.STOCHASTIC, spp=spp, seed=3, shade=1)
    a = orc.filter2d(T, q, orc.KEYS3, orc.AFTER, shade=1)
    one = orc.filter2d(T, q, orc.KEYS3, orc.STOCHASTIC, spp=64, seed=3, shade=1)
    assert np.max(np.abs(s - a)) < 5 * 3.0 / math.sqrt(spp)
    qc = np.array([[(3 + 0.5) / 8, (5 + 0.5) / 8, 0.0]], np.float32)
    v, taps = orc.filter2d(T, qc, orc.KEYS3, orc.STOCHASTIC, spp=16, seed=1, shade=0, taps=True)
    assert np.allclose(v[0], tex[5, 3], rtol=1e-14)
    assert np.all(taps[0, :, 1] == 3) and np.all(taps[0, :, 2] == 5) and np.all(taps[0, :, 3] == orc.TAP_NONE)
    del one


def test_ggx_schlick_fresnel_off_normal(orc):
    """Schlick's Fresnel factor away from normal incidence.  With zero albedo
    the shaded value is proportional to F, so L(f0) / L(1) isolates
    F(f0) / F(1) = f0 + (1 - f0)(1 - wi.h)^5 (Schlick 1994: the fifth power of
    one minus the cosine between the light and the half vector).  The ratio
    must not depend on the surface normal (only wi.h enters F), must be affine
    in f0, and must reach 1 at grazing half-angles (wo nearly opposite wi).
    A wrong exponent, or n.wi / n.h in place of wi.h, fails one of these."""
    rng = np.random.default_rng(11)
    alb = np.zeros(4)
    alb[3] = 0.4

    def ratio(n, wo, wi, f0):
        a = orc.shade_ggx(orc.ggx_params(n=n, wo=wo, wi=wi, f0=f0), alb)[0]
        b = orc.shade_ggx(orc.ggx_params(n=n, wo=wo, wi=wi, f0=1.0), alb)[0]
        return a / b

    for _ in range(40):
        wo = rng.normal(size=3); wo[2] = abs(wo[2]) + 0.3
        wi = rng.normal(size=3); wi[2] = abs(wi[2]) + 0.3
        wo /= np.linalg.norm(wo); wi /= np.linalg.norm(wi)
        h = (wo + wi) / np.linalg.norm(wo + wi)
        c = float(wi @ h)
        r0 = ratio((0, 0, 1), wo, wi, 0.0)
        assert abs(r0 - (1.0 - c) ** 5) <= 1e-12 * max(1.0, r0), (c, r0)
        # tilt the normal (keeping both directions above it): F is unchanged
        n2 = np.array([0.1, -0.15, 1.0]) + 0.05 * rng.normal(size=3)
        n2 /= np.linalg.norm(n2)
        if min(n2 @ wo, n2 @ wi, n2 @ h) > 0.05:
            assert abs(ratio(n2, wo, wi, 0.0) - r0) <= 1e-12 * max(1.0, r0)
        for f0 in (0.04, 0.5, 0.9):
            assert abs(ratio((0, 0, 1), wo, wi, f0) - (f0 + (1 - f0) * r0)) <= 1e-12
    # grazing half-angles: wo and wi nearly opposite in the tangent plane
    for eps in (0.3, 0.1, 0.03):
        wo = np.array([1.0, 0.0, eps]); wi = np.array([-1.0, 0.02, eps])
        wo /= np.linalg.norm(wo); wi /= np.linalg.norm(wi)
        h = (wo + wi) / np.linalg.norm(wo + wi)
        c = float(wi @ h)
        r0 = ratio((0, 0, 1), wo, wi, 0.0)
        assert c < 0.31 and abs(r0 - (1 - c) ** 5) < 1e-12
        assert r0 > (1 - 0.31) ** 5
    # closed values at a fixed geometry: wi.h = cos 30 deg (wo, wi 60 deg apart)
    wo = np.array([math.sin(math.radians(30)), 0.0, math.cos(math.radians(30))])
    wi = np.array([-math.sin(math.radians(30)), 0.0, math.cos(math.radians(30))])
    r0 = ratio((0, 0, 1), wo, wi, 0.0)
    assert abs(r0 - (1 - math.sqrt(3) / 2) ** 5) < 1e-15
