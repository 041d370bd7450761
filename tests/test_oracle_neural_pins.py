"""Pins of the neural part of the CPU oracle (codecs, MLP gradients, Adam,
neural filtering) against facts independent of its code."""
import math

import numpy as np
import pytest
import torch

from paper_2407_06107_amd import inputs

H = 64


def _rand_params(C, O, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    import oracle
    return rng.normal(size=oracle.mlp_nparams(C, H, O)) * scale


def test_bf16_matches_torch(orc):
    """Round-to-nearest-even to bfloat16 agrees with torch's conversion."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=3000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 3000),
                        np.array([1.0039062, 1.00390625, 1.01171875, -2.5, 0.0, 65504.0, 1e-40], np.float32)])
    ours = orc.f32_to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    back = orc.bf16_to_double(ours)
    assert np.array_equal(back, torch.from_numpy(x).to(torch.bfloat16).double().numpy())


def test_fp8_decode_and_encode_match_torch(orc):
    """OCP E4M3: the oracle's 256-code table equals torch.float8_e4m3fn's
    decoding; encoding rounds to nearest even like torch below 464 (torch
    gives NaN above, the oracle saturates at 448 as the format's
    saturating conversion does)."""
    table = orc.fp8_table()
    ref = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn).double().numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(table), nan)
    assert np.array_equal(table[~nan], ref[~nan])
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-463, 463, 2000), rng.normal(size=2000) * 0.01,
                        [2.0 ** -10, 3 * 2.0 ** -10, 0.0, 448.0, 460.0]]).astype(np.float32)
    ours = np.array([orc.f32_to_fp8(v) for v in x], dtype=np.uint8)
    theirs = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, theirs)
    assert orc.f32_to_fp8(1000.0) == 0x7E and orc.f32_to_fp8(-1e9) == 0xFE


def test_fp8_block_quantisation_error_bound(orc):
    """Per-block scaling: |z - dequant(code)| <= half an E4M3 step of the
    scaled value (relative 2^-4 for normals, 2^-10 s absolute below)."""
    rng = np.random.default_rng(2)
    res = (12, 10, 9)
    C = 16
    lat = (rng.normal(size=(9, 10, 12, C)) * rng.uniform(0.01, 5.0, size=(9, 10, 12, 1))).astype(np.float32)
    lat[:4, :4, :4] = 0.0
    codes, scales = orc.quantize_fp8(lat.ravel(), 3, res, C, 2)
    table = orc.fp8_table()
    B = 4
    nb = [-(-r // B) for r in res]
    z, y, x = np.meshgrid(np.arange(9), np.arange(10), np.arange(12), indexing="ij")
    blk = ((z // B) * nb[1] + (y // B)) * nb[0] + (x // B)
    s = scales[blk][..., None].astype(np.float64)
    deq = table[codes.reshape(lat.shape)] * s
    err = np.abs(deq - lat)
    bound = np.maximum(np.abs(lat) * 2.0 ** -4, s * 2.0 ** -10) * 1.0001
    assert np.all(err <= bound)
    assert np.all(scales[blk[:4, :4, :4]] == 1.0)          # all-zero block


def test_fp8_dequant_is_bf16_of_binary32_product(orc):
    """An E4M3 latent enters the BF16 MLP as bf16(binary32(code value x
    scale)): torch's E4M3 decoding, a float32 product and torch's
    round-to-nearest-even BF16 conversion give the same values; three
    products worked by hand pin the rounding (two ties to even, one below
    half an ulp)."""
    rng = np.random.default_rng(5)
    C = 16
    codes = rng.integers(0, 256, size=(500, C), dtype=np.uint8)
    codes[(codes & 0x7F) == 0x7F] = 0x3A                 # no NaN codes
    scale = np.exp(rng.uniform(-20, 5, size=500)).astype(np.float32)
    ours = orc.dequant_fp8(codes, scale, C)
    z = torch.from_numpy(codes).view(torch.float8_e4m3fn).float()
    ref = (z * torch.from_numpy(scale)[:, None]).to(torch.bfloat16).double().numpy()
    assert np.array_equal(ours, ref)
    # 1.0 x (1 + 2^-8) = 1.00000001b: a tie, to the even 1.0
    # 1.0 x (1 + 3 2^-8) = 1.00000011b: a tie, to the even 1.0000010b
    # 1.125 x (1 + 2^-7) = 1.0010001001b: below half an ulp, to 1.0010001b
    hand = orc.dequant_fp8(np.array([[0x38], [0x38], [0x39]], np.uint8),
                           np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7], np.float32), 1)
    assert hand.ravel().tolist() == [1.0, 1.0 + 2.0 ** -6, 1.1328125]


@pytest.mark.parametrize("C, O", [(8, 4), (16, 1)])
def test_mlp_gradient_finite_differences(orc, C, O):
    """Backward pass vs central differences of the batch loss (FP64)."""
    rng = np.random.default_rng(3)
    P = _rand_params(C, O, 4)
    Z = rng.normal(size=(5, C))
    T = rng.normal(size=(5, O))
    loss, gP, gZ = orc.mlp_grad(C, H, O, P, Z, T)
    h = 1e-6

    def L(P_, Z_):
        return orc.mlp_grad(C, H, O, P_, Z_, T)[0]

    idx = rng.choice(P.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(P)
        e[i] = h
        fd = (L(P + e, Z) - L(P - e, Z)) / (2 * h)
        assert abs(fd - gP[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, gP[i])
    for s in range(2):
        for c in range(C):
            e = np.zeros_like(Z)
            e[s, c] = h
            fd = (L(P, Z + e) - L(P, Z - e)) / (2 * h)
            assert abs(fd - gZ[s, c]) <= 1e-7 * max(1.0, abs(fd))
    # loss is the batch mean of squared errors
    Y = orc.mlp_forward(C, H, O, P, Z)
    assert loss == pytest.approx(np.sum((Y - T) ** 2) / 5, rel=1e-12)


@pytest.mark.parametrize("C, O", [(8, 4), (16, 1)])
def test_mlp_gradient_with_bf16_activations(orc, C, O):
    """With the hidden activations stored in BF16, the oracle's gradients are
    those of backpropagation (numpy matrix form, FP64) through the network
    whose stored activations are the rounded ones: rectifier masks from the
    pre-activations, weight gradients from the rounded activations."""
    import torch
    rng = np.random.default_rng(8)
    P = _rand_params(C, O, 9)
    Z = rng.normal(size=(40, C))
    T = rng.normal(size=(40, O))
    B = Z.shape[0]
    bf = lambda x: torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).double().numpy()
    W1 = P[:C * H].reshape(C, H); b1 = P[C * H:C * H + H]
    o = C * H + H
    W2 = P[o:o + H * H].reshape(H, H); b2 = P[o + H * H:o + H * H + H]
    o += H * H + H
    W3 = P[o:o + H * O].reshape(H, O); b3 = P[o + H * O:]
    A1 = Z @ W1 + b1
    H1 = bf(np.maximum(A1, 0.0))
    A2 = H1 @ W2 + b2
    H2 = bf(np.maximum(A2, 0.0))
    Y = H2 @ W3 + b3
    dY = 2.0 * (Y - T) / B
    dA2 = (dY @ W3.T) * (A2 > 0)
    dA1 = (dA2 @ W2.T) * (A1 > 0)
    ref = np.concatenate([(Z.T @ dA1).ravel(), dA1.sum(0), (H1.T @ dA2).ravel(), dA2.sum(0),
                          (H2.T @ dY).ravel(), dY.sum(0)])
    loss, gP, gZ = orc.mlp_grad(C, H, O, P, Z, T, act_bf16=True)
    assert np.allclose(gP, ref, rtol=1e-10, atol=1e-13)
    assert np.allclose(gZ, dA1 @ W1.T, rtol=1e-10, atol=1e-13)
    assert loss == pytest.approx(np.sum((Y - T) ** 2) / B, rel=1e-12)
    # the rounding matters: the plain FP64 gradient differs
    assert not np.allclose(orc.mlp_grad(C, H, O, P, Z, T)[1], gP, rtol=1e-6, atol=0)


def test_mlp_forward_is_the_textbook_network(orc):
    """Forward pass = numpy matmul/relu on the unpacked parameters."""
    C, O = 8, 4
    P = _rand_params(C, O, 5)
    Z = np.random.default_rng(6).normal(size=(7, C))
    W1 = P[:C * H].reshape(C, H); b1 = P[C * H:C * H + H]
    o = C * H + H
    W2 = P[o:o + H * H].reshape(H, H); b2 = P[o + H * H:o + H * H + H]
    o += H * H + H
    W3 = P[o:o + H * O].reshape(H, O); b3 = P[o + H * O:]
    ref = np.maximum(np.maximum(Z @ W1 + b1, 0) @ W2 + b2, 0) @ W3 + b3
    assert np.allclose(orc.mlp_forward(C, H, O, P, Z), ref, rtol=1e-13, atol=1e-13)


def test_adam_first_step_closed_form(orc):
    """After one step from zero moments, m_hat = g and v_hat = g^2, so the
    update is lr * g / (|g| + eps) (Kingma & Ba 2015)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0, 3e-9])
    th = np.ones(5)
    m, v = np.zeros(5), np.zeros(5)
    orc.adam(th, m, v, g, 1, 0.01)
    assert np.allclose(th, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _identity_params(C, O):
    """An MLP that passes the first O latent channels through (for
    non-negative inputs): W1, W2, W3 are identity blocks, biases zero."""
    import oracle
    P = np.zeros(oracle.mlp_nparams(C, H, O))
    W1 = np.zeros((C, H)); W1[:O, :O] = np.eye(O)
    W2 = np.eye(H)
    W3 = np.zeros((H, O)); W3[:O, :O] = np.eye(O)
    P[:C * H] = W1.ravel()
    o = C * H + H
    P[o:o + H * H] = W2.ravel()
    o += H * H + H
    P[o:o + H * O] = W3.ravel()
    return P


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode", ["STOCHASTIC", "BEFORE", "AFTER"])
def test_neural_filter2d_identity_equals_plain(orc, filt, mode):
    """With an MLP that decodes latent c to the texel of c, the neural
    texture filter is the plain texture filter (taps, shading and all)."""
    R = 16
    tex = inputs.texture_uniform(R, seed=2)
    Z = np.zeros((R * R, 8))
    Z[:, :4] = tex.reshape(-1, 4)
    P = _identity_params(8, 4)
    q = inputs.queries_uniform(300, seed=3)
    f, m = getattr(orc, filt), getattr(orc, mode)
    a = orc.neural_filter2d((R, R), 8, H, 4, Z, P, q, f, m, spp=4, seed=9, shade=1, act_bf16=False)
    b = orc.filter2d(orc.Tex2D.rgba32f(tex), q, f, m, spp=4, seed=9, shade=1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mode", ["STOCHASTIC", "BEFORE", "AFTER"])
def test_neural_raymarch_identity_equals_plain(orc, mode):
    n = 12
    data = inputs.cloud_grid(n, seed=3).numpy().astype(np.float32)
    Z = np.zeros((n ** 3, 16))
    Z[:, 0] = data.ravel()
    P = _identity_params(16, 1)
    rays = inputs.random_rays(40, 1.0, seed=4)
    scale = np.array([n, n, n], np.float32)
    m = getattr(orc, mode)
    a = orc.neural_raymarch((n, n, n), 16, H, Z, P, (0, 0, 0), scale, rays, 16, orc.BSPLINE3, m, spp=2, seed=5,
                            act_bf16=False)
    b = orc.raymarch(orc.Grid(data, side=1.0), rays, 16, orc.BSPLINE3, m, spp=2, seed=5)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)
