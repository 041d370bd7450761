"""Pins of the oracle's split-filtering estimator (Sec. 3 eq.
split-filtering-shading and its Monte Carlo form in Sec. 4: the low-pass
filter — the MIP level choice, and for pixels the jitter over the footprint
— sampled, the reconstruction filter evaluated before shading) against the
plain filters it is made of."""
import math

import numpy as np
import pytest

from paper_2407_06107_amd import inputs

FILTERS = ["NEAREST", "LINEAR", "BSPLINE3", "KEYS3"]


def _pyr(orc, n=64, mip=None, seed=12):
    lv = inputs.mip_chain(inputs.texture_uniform(n, seed=seed))
    buf, offs = inputs.pack_levels([x.astype(np.float32) for x in lv])
    t = orc.Tex2D(buf, n, n, len(lv), orc.RGBA32F, offs, orc.REPEAT, orc.MIP_LINEAR if mip is None else mip)
    return lv, t


@pytest.mark.parametrize("filt", FILTERS)
@pytest.mark.parametrize("shade", [0, 1])
def test_single_level_split_is_before(orc, filt, shade):
    """With one level there is nothing to sample: split == filter-before
    exactly, for any sample count."""
    lv, _ = _pyr(orc)
    t = orc.Tex2D.rgba32f(lv[0].astype(np.float32))
    q = inputs.queries_uniform(300, seed=3)
    f = getattr(orc, filt)
    a = orc.filter2d(t, q, f, orc.SPLIT, spp=5, seed=1, shade=shade)
    b = orc.filter2d(t, q, f, orc.BEFORE, shade=shade)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
def test_split_levels_and_their_blend(orc, filt):
    """Per sample the split estimator shades the reconstruction of ONE level,
    floor(lambda) or floor(lambda) + 1, picked with probability f: taps hold
    only those levels (no texel), at frequency f, and the mean over many
    samples is (1 - f) shade(recon l0) + f shade(recon l1), the levels'
    own filter-before values, within 5 sigma."""
    lv, t = _pyr(orc)
    q = inputs.queries_uniform(40, seed=4)
    q[:, 2] = np.linspace(0.05, 4.95, 40).astype(np.float32)
    f = getattr(orc, filt)
    spp = 4096
    S, taps = orc.filter2d(t, q, f, orc.SPLIT, spp=spp, seed=2, shade=1, taps=True)
    l0 = np.floor(q[:, 2]).astype(int)
    frac = (q[:, 2] - np.floor(q[:, 2])).astype(np.float64)
    assert np.all(taps[..., 1:] == orc.TAP_NONE)
    assert np.all((taps[..., 0] == l0[:, None]) | (taps[..., 0] == l0[:, None] + 1))
    p1 = np.mean(taps[..., 0] == l0[:, None] + 1, axis=1)
    assert np.all(np.abs(p1 - frac) <= 5 * np.sqrt(frac * (1 - frac) / spp) + 1e-12)
    single = [orc.Tex2D.rgba32f(x.astype(np.float32)) for x in lv]
    B = np.array([[orc.filter2d(single[l], qq[None] * np.array([1, 1, 0], np.float32), f, orc.BEFORE, shade=1)[0]
                   for l in (a, a + 1)] for qq, a in zip(q, l0)])          # [n, 2, 3]
    E = (1 - frac)[:, None] * B[:, 0] + frac[:, None] * B[:, 1]
    sd = np.sqrt(frac * (1 - frac) / spp)[:, None] * np.abs(B[:, 1] - B[:, 0])
    assert np.all(np.abs(S - E) <= 5 * sd + 1e-12)


def test_split_affine_shading_equals_trilinear_before(orc):
    """Without shading (an affine use of the texture) the split estimator is
    unbiased for the trilinear filter-before value."""
    lv, t = _pyr(orc)
    q = inputs.queries_uniform(40, seed=5)
    q[:, 2] = np.linspace(0.1, 5.9, 40).astype(np.float32)
    spp = 4096
    S = orc.filter2d(t, q, orc.BSPLINE3, orc.SPLIT, spp=spp, seed=3)
    A = orc.filter2d(t, q, orc.BSPLINE3, orc.BEFORE)
    assert np.all(np.abs(S - A) <= 5 * 0.5 / math.sqrt(spp))


def test_aniso_split_zero_footprint_is_level0_before(orc):
    """A zero footprint has no jitter and level 0: split == the level-0
    filter-before value for every sample."""
    lv, t = _pyr(orc)
    q = inputs.plane_queries_aniso(20, 10)
    q[:, 2:] = 0.0
    t0 = orc.Tex2D.rgba32f(lv[0].astype(np.float32))
    for filt in ("LINEAR", "BSPLINE3", "KEYS3"):
        f = getattr(orc, filt)
        S, taps = orc.filter2d_aniso(t, q, f, orc.SPLIT, spp=3, seed=4, shade=1, taps=True)
        B = orc.filter2d(t0, np.concatenate([q[:, :2], np.zeros((q.shape[0], 1), np.float32)], 1), f, orc.BEFORE,
                         shade=1)
        assert np.allclose(S, B, rtol=1e-13, atol=1e-14)
        assert np.all(taps[..., 0] == 0) and np.all(taps[..., 1:] == orc.TAP_NONE)


def test_aniso_split_and_stochastic_share_the_unshaded_mean(orc):
    """Unshaded, the split estimator (reconstruction evaluated) and the
    stochastic one (reconstruction sampled) estimate the same value: the
    jitter-and-level average of the reconstructed texture."""
    lv, t = _pyr(orc)
    q = inputs.plane_queries_aniso(40, 30)[::30]
    spp = 4096
    S = orc.filter2d_aniso(t, q, orc.BSPLINE3, orc.SPLIT, spp=spp, seed=6, amax=16)
    T = orc.filter2d_aniso(t, q, orc.BSPLINE3, orc.STOCHASTIC, spp=spp, seed=7, amax=16)
    assert np.all(np.abs(S - T) <= 5 * math.sqrt(2) * 0.5 / math.sqrt(spp))


def test_split_nonfinite(orc):
    lv, t = _pyr(orc)
    q = np.array([[np.nan, 0.5, 0.0], [0.3, 0.3, 1.5]], np.float32)
    out, taps = orc.filter2d(t, q, orc.KEYS3, orc.SPLIT, spp=2, taps=True, shade=1)
    assert np.all(np.isnan(out[0])) and np.all(np.isfinite(out[1]))
    assert taps.shape == (2, 2, 3) and np.all(taps[0] == orc.TAP_NONE)
