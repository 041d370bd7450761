"""Pins of the oracle's Mitchell-Netravali cubic (B = C = 1/3) and its
positivised stochastic estimator (Sec. 2.2 "Positivization"; the paper's
bicubic listing sorts each weight into a positive or a negative reservoir by
its sign) against the kernel's closed-form properties, brute-force
expectation over the 24-bit uniforms and linear reproduction."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2407_06107_amd import inputs

U24 = 2.0 ** -24


def test_kernel_closed_forms(orc):
    """k(0) = (6 - 2B)/6 = 8/9, k(1) = B/6 = 1/18, k(2) = 0, the outer lobe's
    root at 8/7, symmetry, unit integral, C1 continuity at 1 and 2."""
    k = orc.kmn
    assert abs(k(0.0) - 8 / 9) < 1e-15 and abs(k(1.0) - 1 / 18) < 1e-15 and k(2.0) == 0.0
    assert abs(k(8 / 7)) < 1e-15 and k(1.1) > 0 and k(1.2) < 0
    for x in (0.1, 0.7, 1.3, 1.9):
        assert k(x) == k(-x)
    assert abs(integrate.quad(k, -2, 2, points=[-1, 0, 1], epsabs=1e-14)[0] - 1.0) < 1e-12
    h = 1e-6
    for x0 in (1.0, 2.0):
        left, right = k(x0 - h), k(x0 + h) if x0 < 2 else 0.0
        assert abs(left - right) < 1e-5
        dl = (k(x0 - h) - k(x0 - 2 * h)) / h
        dr = (k(x0 + 2 * h) - k(x0 + h)) / h if x0 < 2 else 0.0
        assert abs(dl - dr) < 1e-4


@pytest.mark.parametrize("t", np.linspace(0.0, 1.0, 37))
def test_partition_of_unity_and_linear_reproduction(orc, t):
    """B + 2C = 1: the four taps' weights sum to one and reproduce linear
    functions (sum_k (k - 1) w_k = t)."""
    w = [orc.kmn(t - (k - 1)) for k in range(4)]
    assert abs(sum(w) - 1.0) < 1e-14
    assert abs(sum((k - 1) * wk for k, wk in enumerate(w)) - t) < 1e-14


def test_binary32_weights_and_sign_sets(orc):
    """The factored binary32 weights equal the kernel within a few ulp, the
    positive set holds the inner taps always, w0 only for t < 1/7 and w3 only
    for t > 6/7, and P+ - P- = 1 to binary32 rounding."""
    for t in np.concatenate([np.linspace(0, 1, 1001)[:-1], [1 / 7, 6 / 7, 1e-7, 1 - 2 ** -24]]):
        t32 = float(np.float32(t))
        w, pp, pm = orc.mitchell_axis(t32)
        ref = np.array([orc.kmn(t32 - (k - 1)) for k in range(4)])
        assert np.all(np.abs(w.astype(np.float64) - ref) <= 4 * 2.0 ** -24)
        assert w[1] > 0 and w[2] > 0
        if t32 < 1 / 7 - 1e-6:
            assert w[0] > 0
        if t32 > 1 / 7 + 1e-6:
            assert w[0] < 0
        if t32 > 6 / 7 + 1e-6:
            assert w[3] > 0
        if 1e-6 < t32 < 6 / 7 - 1e-6:
            assert w[3] < 0
        assert abs(pp - pm - 1.0) <= 4 * 2.0 ** -24
        assert abs(pp - w[w > 0].astype(np.float64).sum()) <= 2 * 2.0 ** -24


def test_picks_respect_the_sign_sets(orc):
    """Every positive draw lands on a product weight > 0 and every negative
    draw on one < 0."""
    rng = np.random.default_rng(3)
    for _ in range(3000):
        tx, ty = (float(np.float32(x)) for x in rng.random(2))
        u = (np.floor(rng.random(6) * 2 ** 24) * U24).astype(np.float32)
        off, has_neg = orc.mitchell_pick(tx, ty, u)
        wx, _, _ = orc.mitchell_axis(tx)
        wy, _, _ = orc.mitchell_axis(ty)
        assert wx[off[0] + 1] * wy[off[1] + 1] > 0
        if has_neg:
            assert wx[off[2] + 1] * wy[off[3] + 1] < 0


def test_exact_expectation_equals_after(orc):
    """The positivised estimator's expectation over the 24-bit uniforms
    (every decision counted by brute force) is the filter-after value, within
    the lattice's 2^-24 per decision times the block sums (< 1.15)."""
    tex = inputs.texture_uniform(16, seed=4)
    t = orc.Tex2D.rgba32f(tex)
    q = inputs.queries_uniform(6, seed=5)
    q[0, :2] = [(3 + 1 / 7 + 0.5) / 16, (5 + 6 / 7 + 0.5) / 16]     # on the sign changes
    q[1, :2] = [3.5 / 16, 7.5 / 16]                                 # texel centre: t = 0
    for shade in (0, 1):
        E = orc.mitchell_expect2d(t, q, shade=shade)
        A = orc.filter2d(t, q, orc.MITCHELL, orc.AFTER, shade=shade)
        assert np.max(np.abs(E - A)) <= 16 * 2.0 ** -24 * 1.15 * max(1.0, np.abs(A).max())


def test_stochastic_mean_and_linear_texture(orc):
    """Stochastic means within 5 sigma of the filter-after value; on a
    texture linear in u (away from the wrap) every deterministic mode returns
    the linear value (B + 2C = 1 reproduces linear functions)."""
    tex = inputs.texture_uniform(32, seed=6)
    t = orc.Tex2D.rgba32f(tex)
    q = inputs.queries_uniform(50, seed=7)
    A = orc.filter2d(t, q, orc.MITCHELL, orc.AFTER, shade=1)
    spp = 8192
    S = orc.filter2d(t, q, orc.MITCHELL, orc.STOCHASTIC, spp=spp, seed=8, shade=1)
    # a sample is W+ f+ - W- f-, |W+| + |W-| < 1.15, shaded values below 1
    assert np.all(np.abs(S - A) <= 5 * 1.15 / math.sqrt(spp))
    ramp = np.zeros((8, 64, 4), np.float32)
    ramp[..., 0] = np.arange(64)[None, :] / 64.0
    ramp[..., 1:] = 0.5
    tr = orc.Tex2D.rgba32f(ramp, wrap=orc.CLAMP)
    x = np.linspace(4.0, 59.0, 40)
    qr = np.stack([(x + 0.5) / 64, np.full_like(x, 0.5), np.zeros_like(x)], 1).astype(np.float32)
    for m in (orc.BEFORE, orc.AFTER):
        out = orc.filter2d(tr, qr, orc.MITCHELL, m)
        px = qr[:, 0].astype(np.float32) * np.float32(64) - np.float32(0.5)
        assert np.allclose(out[:, 0], px / 64.0, atol=1e-12)


def test_taps_and_nonfinite(orc):
    tex = inputs.texture_uniform(16, seed=9)
    t = orc.Tex2D.rgba32f(tex)
    q = np.array([[np.nan, 0.5, 0.0], [0.31, 0.62, 0.0]], np.float32)
    out, taps = orc.filter2d(t, q, orc.MITCHELL, orc.STOCHASTIC, spp=4, seed=2, taps=True, shade=1)
    assert taps.shape == (2, 4, 5) and np.all(taps[0] == orc.TAP_NONE) and np.all(np.isnan(out[0]))
    assert np.all(np.isfinite(out[1]))
