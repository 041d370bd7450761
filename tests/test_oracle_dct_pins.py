"""Pins of the oracle's DCT-compressed textures and triplanar mapping
(Sec. 5 "Texture compression" and "Triplanar mapping") against scipy's DCT,
exact counting and the plain 2-D filter."""
import math

import numpy as np
import pytest
from scipy import fft

from paper_2407_06107_amd import inputs

ZIGZAG = [(0, 0), (1, 0), (0, 1), (0, 2), (1, 1), (2, 0)]      # (u horizontal, v vertical)


def test_basis_is_the_orthonormal_dct(orc):
    B = orc.dct_basis32().astype(np.float64)
    x = np.arange(8)
    ref = np.stack([np.sqrt(1 / 8) * np.ones(8)] + [0.5 * np.cos((2 * x + 1) * k * np.pi / 16) for k in (1, 2)])
    assert np.array_equal(B, ref.astype(np.float32).astype(np.float64))
    assert np.allclose(B @ B.T, np.eye(3), atol=1e-7)


def _scipy_coeffs(lv):
    """Six zigzag coefficients of every 8x8 block (edge-replicated), fp64."""
    h, w = lv.shape[:2]
    bh, bw = -(-h // 8), -(-w // 8)
    v = lv.astype(np.float64) / 255.0
    pad = np.pad(v, ((0, bh * 8 - h), (0, bw * 8 - w), (0, 0)), mode="edge")
    blocks = pad.reshape(bh, 8, bw, 8, 4).transpose(0, 2, 4, 1, 3)          # by, bx, c, y, x
    C = fft.dctn(blocks, type=2, norm="ortho", axes=(3, 4))                  # [.., v, u]
    return np.stack([C[..., vv, uu] for uu, vv in ZIGZAG], axis=-1)          # by, bx, c, k


def _codes(tex, level):
    """Unpack the oracle's codes of one level: by, bx, c, k (DC 0..127, AC -15..15)."""
    wl, hl = max(1, tex.w >> level), max(1, tex.h >> level)
    bw, bh = -(-wl // 8), -(-hl // 8)
    words = tex.buf[tex.off[level]:tex.off[level] + 16 * bw * bh].view(np.uint32).reshape(bh, bw, 4)
    out = np.empty((bh, bw, 4, 6), np.int64)
    out[..., 0] = words & 127
    for k in range(1, 6):
        out[..., k] = ((words >> (7 + 5 * (k - 1))) & 31).astype(np.int64) - 15
    return out


def test_codes_quantise_scipy_coefficients(orc):
    """DC in 7 bits over [0, 8], AC in 5 bits over [-R, R], R = max |AC| of the
    channel: the oracle's codes equal the quantised fp64 coefficients except
    where a coefficient sits within binary32 rounding of a code boundary."""
    lv = inputs.quantize_unorm8([inputs.texture_sinusoids(64, seed=5, waves=10)[:44, :60]])[0]
    tex = orc.Tex2D.dct([lv])
    C = _scipy_coeffs(lv)
    codes = _codes(tex, 0)
    R = np.abs(C[..., 1:]).max(axis=(0, 1, 3))                   # per channel
    assert np.allclose(tex.dct_range[:4], R, rtol=1e-6)
    dc = np.clip(np.floor(C[..., 0] * 127 / 8 + 0.5), 0, 127)
    ac = np.clip(np.floor(C[..., 1:] * (15 / R[None, None, :, None]) + 0.5), -15, 15)
    ref = np.concatenate([dc[..., None], ac], axis=-1)
    diff = codes != ref
    assert diff.mean() < 2e-3
    assert np.all(np.abs(codes - ref) <= 1)
    # the disagreements are rounding ties: the scaled coefficient is within 1e-4 of k + 1/2
    scaled = np.concatenate([C[..., :1] * 127 / 8, C[..., 1:] * (15 / R[None, None, :, None])], axis=-1)
    frac = scaled - np.floor(scaled)
    assert np.all(np.abs(frac[diff] - 0.5) < 1e-4)


def test_decode_is_the_truncated_inverse_dct(orc):
    """Decoded texels (read back through the nearest filter at texel
    centres) = clamp(inverse DCT of the dequantised six coefficients)."""
    lv = inputs.quantize_unorm8([inputs.texture_sinusoids(64, seed=6, waves=8)[:40, :48]])[0]
    tex = orc.Tex2D.dct([lv], wrap=orc.CLAMP)
    codes = _codes(tex, 0).astype(np.float64)
    R = tex.dct_range[:4].astype(np.float64)
    deq = np.concatenate([codes[..., :1] * 8 / 127, codes[..., 1:] * R[None, None, :, None] / 15], axis=-1)
    full = np.zeros(codes.shape[:3] + (8, 8))
    for k, (u, v) in enumerate(ZIGZAG):
        full[..., v, u] = deq[..., k]
    rec = fft.idctn(full, type=2, norm="ortho", axes=(3, 4))                 # by, bx, c, y, x
    img = np.clip(rec.transpose(0, 3, 1, 4, 2).reshape(codes.shape[0] * 8, codes.shape[1] * 8, 4), 0, 1)
    h, w = lv.shape[:2]
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    q = np.stack([(xx.ravel() + 0.5) / w, (yy.ravel() + 0.5) / h, np.zeros(h * w)], 1).astype(np.float32)
    out = orc.filter2d(tex, q, orc.NEAREST, orc.AFTER)
    assert np.allclose(out, img[:h, :w].reshape(-1, 4), atol=1e-12)


def test_constant_and_quantisation_error(orc):
    """A constant texture decodes to the constant within half a DC step,
    with zero AC range."""
    lv = np.full((24, 32, 4), 77, np.uint8)
    tex = orc.Tex2D.dct([lv])
    q = inputs.queries_uniform(200, seed=1)
    out = orc.filter2d(tex, q, orc.NEAREST, orc.AFTER)
    assert np.all(np.abs(out - 77 / 255) <= 0.5 * 8 / 127 / 8 + 1e-12)
    assert np.all(tex.dct_range[:4] < 1e-6)


def test_dct_filters_expectation(orc):
    """Filtering a DCT texture: the exact expectation of the stochastic
    estimator equals the exact filter-after value (the decode is just the
    texel fetch)."""
    lvs = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(32, seed=7, waves=6)))
    tex = orc.Tex2D.dct(lvs, mip=orc.MIP_LINEAR)
    q = inputs.queries_uniform(40, seed=2)
    q[:, 2] = np.linspace(0, 3.5, 40)
    for f in (orc.LINEAR, orc.BSPLINE3):
        E = orc.filter2d_expect(tex, q, f, shade=1)
        A = orc.filter2d(tex, q, f, orc.AFTER, shade=1)
        assert np.max(np.abs(E - A)) <= 64 * 2.0 ** -24 * max(1.0, np.abs(A).max())


# ------------------------------------------------------------------ triplanar
def test_plane_pick_probabilities(orc):
    """P(plane j) over all 2^24 uniforms = b_j = n_j^4 / sum n^4 within 2^-23."""
    u = (np.arange(2 ** 24, dtype=np.float64) * 2.0 ** -24).astype(np.float32)
    for nrm in ([0.36, 0.48, 0.8], [1.0, 0.0, 0.0], [0.0, 0.6, -0.8], [-0.577, 0.577, 0.578]):
        n = np.array(nrm, np.float64)
        b = n ** 4 / np.sum(n ** 4)
        picks = np.array([orc.tri_pick(nrm, float(x)) for x in u[:: 2 ** 12]])
        P = np.bincount(picks, minlength=3) / picks.size
        assert np.all(np.abs(P - b) <= 2 ** -12 + 1e-12)         # on the 2^12-subsampled lattice
    assert all(orc.tri_pick([1.0, 0.0, 0.0], float(x)) == 0 for x in (0.0, 0.5, 1 - 2 ** -24))
    assert all(orc.tri_pick([0.0, 0.0, -1.0], float(x)) == 2 for x in (0.0, 0.5, 1 - 2 ** -24))


def _tri_inputs():
    lvs = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(64, seed=8, waves=8)))
    buf, offs = inputs.pack_levels(lvs)
    q = inputs.sphere_queries(48, 32, tex_size=64, levels=len(lvs))
    return lvs, buf, offs, q


@pytest.mark.parametrize("mode", ["BEFORE", "AFTER"])
def test_triplanar_blend_is_the_weighted_plane_filters(orc, mode):
    """The deterministic blend equals sum_j b_j times the plain 2-D filter
    at plane j's coordinates (after), or the shaded blend of the unshaded
    plane filters (before)."""
    lvs, buf, offs, q = _tri_inputs()
    tex = orc.Tex2D(buf, 64, 64, len(lvs), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    m = getattr(orc, mode)
    scale = 1.5
    out = orc.triplanar(tex, q, scale, 0, orc.BSPLINE3, m, shade=1)
    n = q[:, 3:6].astype(np.float64)
    b = n ** 4 / np.sum(n ** 4, axis=1, keepdims=True)
    planes = [(1, 2), (0, 2), (0, 1)]
    acc = np.zeros((q.shape[0], 4 if m == orc.BEFORE else 3))
    for j, (a, c) in enumerate(planes):
        qj = np.stack([q[:, a] * np.float32(scale), q[:, c] * np.float32(scale), q[:, 6]], 1).astype(np.float32)
        # after: blend of shaded plane filters; before: blend of unshaded ones, shaded below
        acc += b[:, j:j + 1] * orc.filter2d(tex, qj, orc.BSPLINE3, orc.AFTER, shade=1 if m == orc.AFTER else 0)
    if m == orc.BEFORE:
        acc = np.array([orc.shade_ggx(orc.ggx_params(), row) for row in acc])
    assert np.allclose(out, acc, rtol=1e-12, atol=1e-13)


def test_triplanar_stochastic_means(orc):
    """Picking one plane per sample (and one texel) is unbiased for the
    blend: mean of many samples within 5 sigma."""
    lvs, buf, offs, q = _tri_inputs()
    tex = orc.Tex2D(buf, 64, 64, len(lvs), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    q = q[::25]
    A = orc.triplanar(tex, q, 1.5, 0, orc.LINEAR, orc.AFTER, shade=1)
    spp = 4096
    for pm, fm in ((1, orc.STOCHASTIC), (1, orc.AFTER), (0, orc.STOCHASTIC)):
        S = orc.triplanar(tex, q, 1.5, pm, orc.LINEAR, fm, spp=spp, seed=3, shade=1)
        assert np.all(np.abs(S - A) <= 5 * 1.0 / math.sqrt(spp)), (pm, fm)
