"""GPU parity of the neural latent texture / volume path against the oracle.

Integer decisions (lattice taps, quantised codes, scales) are bit-exact.
Decoded values: the matrix cores take BF16 operands and round the hidden
activations to BF16; the oracle emulates that storage in FP64, so the
residual differences are FP32-vs-FP64 accumulation and the rare BF16
rounding flip it causes (one activation off by one BF16 step, ~0.4%).
Tolerance: normwise relative 2e-3 and elementwise 2e-2 of the output scale.
Training gradients: the FP32 step (vector ALU) vs FP64 in the oracle,
normwise 1e-5; the matrix-core step (BF16 operands, FP32 accumulation) vs
the FP64 oracle on the BF16-rounded weights and latents, normwise 2e-2.
"""
import math

import numpy as np
import pytest
import torch

from paper_2407_06107_amd import inputs

pytestmark = pytest.mark.gpu
H = 64


@pytest.fixture(scope="module")
def sf():
    import paper_2407_06107_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sf.lib()
    return sf


def _case(*a):
    print("CASE", *a, flush=True)


def _bf16(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).double().numpy()


def _close_bf16(g, o, norm_tol=2e-3, elem_tol=2e-2):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    assert g.shape == o.shape
    assert np.array_equal(np.isnan(g), np.isnan(o))
    m = ~np.isnan(o)
    g, o = g[m], o[m]
    scale = max(np.sqrt(np.mean(o ** 2)), 1e-6)
    assert np.linalg.norm(g - o) <= norm_tol * np.linalg.norm(o) + 1e-9, \
        f"normwise {np.linalg.norm(g - o) / (np.linalg.norm(o) + 1e-30):.2e}"
    worst = np.max(np.abs(g - o)) / scale if g.size else 0.0
    assert worst <= elem_tol, f"elementwise {worst:.2e} of the output scale"


def _params(C, O, seed, scale=0.25):
    rng = np.random.default_rng(seed)
    n = C * H + H + H * H + H + H * O + O
    P = rng.normal(size=n).astype(np.float32) * scale
    # a positive output bias keeps the clamped 2-D outputs inside (0, 1) mostly
    P[-O:] = 0.5
    return P


def _grid(sf, orc, dims, res, C, fmt, seed, block_log2=2, wmin=(0, 0, 0), scale=(1, 1, 1)):
    rng = np.random.default_rng(seed)
    npts = int(np.prod(res))
    lat = (rng.normal(size=(npts, C)) * rng.uniform(0.2, 2.0, size=(npts, 1))).astype(np.float32)
    lat_d = torch.from_numpy(lat.ravel()).cuda()
    grid = sf.sf_neural_quantize(lat_d, dims, res, C, fmt, block_log2, wmin, scale)
    if fmt == sf.SF_LATENT_BF16:
        Z = _bf16(lat)
    else:
        codes, scales = orc.quantize_fp8(lat.ravel(), dims, res, C, block_log2)
        assert np.array_equal(grid.latents.cpu().numpy(), codes)
        assert np.array_equal(grid.scales.cpu().numpy(), scales)
        B = 1 << block_log2
        nb = [-(-r // B) for r in list(res) + [1] * (3 - len(res))]
        r3 = list(res) + [1] * (3 - len(res))
        z, y, x = np.meshgrid(np.arange(r3[2]), np.arange(r3[1]), np.arange(r3[0]), indexing="ij")
        blk = (((z // B) * nb[1] + (y // B)) * nb[0] + (x // B)).ravel()
        Z = orc.dequant_fp8(codes, scales[blk], C)
    return grid, Z


def test_to_bf16_parity(sf):
    _case("to_bf16")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=50000) * 10.0 ** rng.integers(-30, 30, 50000),
                        [np.inf, -np.inf, 0.0, -0.0, 1e-45, 3.4e38, 1.00390625, 1.01171875]]).astype(np.float32)
    got = sf.sf_to_bf16(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dims, res, C, lg", [(3, (20, 18, 17), 16, 2), (2, (40, 33), 8, 3), (3, (16, 16, 16), 16, 3)])
def test_quantize_fp8_parity(sf, orc, dims, res, C, lg):
    _case("quantize_fp8", dims, res, lg)
    _grid(sf, orc, dims, res, C, sf.SF_LATENT_FP8E4M3, seed=1, block_log2=lg)   # asserts codes and scales


@pytest.mark.parametrize("C, O, dims, res", [(8, 4, 2, (32, 24)), (16, 1, 3, (10, 9, 8))])
@pytest.mark.parametrize("fmt", [1, 2])
def test_decode_lattice_parity(sf, orc, C, O, dims, res, fmt):
    _case("decode_lattice", C, O, fmt)
    grid, Z = _grid(sf, orc, dims, res, C, fmt, seed=2)
    P = _params(C, O, 3)
    mlp = sf.MLP(torch.from_numpy(P).cuda(), C, O)
    npts = int(np.prod(res))
    idx = np.random.default_rng(4).permutation(npts).astype(np.int64)[: npts - 7]   # ragged
    out = sf.sf_neural_decode_lattice(grid, mlp, torch.from_numpy(idx).cuda()).cpu().numpy()
    ref = orc.mlp_forward(C, H, O, _bf16(P), Z[idx], act_bf16=True)
    _close_bf16(out, ref)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode, spp", [("STOCHASTIC", 3), ("STOCHASTIC", 1), ("BEFORE", 1), ("AFTER", 1)])
@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("shade", [0, 1])
def test_neural_filter2d_parity(sf, orc, filt, mode, spp, fmt, shade):
    _case("neural_filter2d", filt, mode, spp, fmt, shade)
    res = (32, 24)
    grid, Z = _grid(sf, orc, 2, res, 8, fmt, seed=5)
    P = _params(8, 4, 6)
    mlp = sf.MLP(torch.from_numpy(P).cuda(), 8, 4)
    q = inputs.queries_uniform(3001, seed=7)
    q[:3, 0] = [-0.3, 1.25, np.nan]
    f, m = getattr(sf, "SF_" + filt), getattr(sf, "SF_" + mode.replace("AFTER", "AFTER_EXACT"))
    smp = sf.sampling(f, m, spp, seed=11)
    taps = torch.empty((q.shape[0], spp, 2), dtype=torch.int32, device="cuda") if mode == "STOCHASTIC" else None
    out = sf.sf_neural_decode(grid, mlp, torch.from_numpy(q).cuda(), smp, shade=shade, ggx_params=sf.ggx(),
                              dbg_taps=taps).cpu().numpy()
    om = {"STOCHASTIC": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    res_ = orc.neural_filter2d(res, 8, H, 4, Z, _bf16(P), q, getattr(orc, filt), om, spp=spp, seed=11, shade=shade,
                               act_bf16=True, taps=mode == "STOCHASTIC")
    if mode == "STOCHASTIC":
        ref, rt = res_
        assert np.array_equal(taps.cpu().numpy(), rt)
    else:
        ref = res_
    _close_bf16(out, ref)


@pytest.mark.parametrize("mode", ["STOCHASTIC", "AFTER"])
@pytest.mark.parametrize("fmt", [1, 2])
def test_neural_filter2d_many_tiles(sf, orc, mode, fmt):
    """More queries than one pass of the decoder's grid holds (as many
    workgroups of 256 as the device keeps resident, far below 2048 x 2):
    every workgroup walks several query tiles.  3000 sampled queries, the
    ragged last tile among them, against the oracle (taps bit-exact)."""
    _case("neural_filter2d_many_tiles", mode, fmt)
    res = (64, 48)
    grid, Z = _grid(sf, orc, 2, res, 8, fmt, seed=8)
    P = _params(8, 4, 9)
    mlp = sf.MLP(torch.from_numpy(P).cuda(), 8, 4)
    n = 2 * 2048 * 256 + 777
    q = inputs.queries_uniform(n, seed=19)
    rng = np.random.default_rng(3)
    sub = np.unique(np.concatenate([rng.choice(n - 1000, 2000, replace=False), np.arange(n - 1000, n)]))
    f = sf.SF_BSPLINE3
    m = sf.SF_STOCHASTIC if mode == "STOCHASTIC" else sf.SF_AFTER_EXACT
    smp = sf.sampling(f, m, 1, seed=13)
    taps = torch.empty((n, 1, 2), dtype=torch.int32, device="cuda") if mode == "STOCHASTIC" else None
    out = sf.sf_neural_decode(grid, mlp, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx(),
                              dbg_taps=taps).cpu().numpy()
    om = orc.STOCHASTIC if mode == "STOCHASTIC" else orc.AFTER
    res_ = orc.neural_filter2d(res, 8, H, 4, Z, _bf16(P), q, orc.BSPLINE3, om, spp=1, seed=13, shade=1,
                               act_bf16=True, taps=mode == "STOCHASTIC", subset=sub)
    if mode == "STOCHASTIC":
        ref, rt = res_
        assert np.array_equal(taps.cpu().numpy()[sub], rt)
    else:
        ref = res_
    _close_bf16(out[sub], ref)


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("addr64", [False, True])
def test_neural_raymarch_parity(sf, orc, filt, fmt, addr64, monkeypatch):
    """addr64: the variant lattices of more than 2^31 bytes of latents take
    (64-bit addresses instead of buffer offsets), forced on this small one."""
    _case("neural_raymarch", filt, fmt, addr64)
    if addr64:
        monkeypatch.setenv("SF_NEURAL_ADDR64", "1")
    res = (12, 11, 10)
    grid, Z = _grid(sf, orc, 3, res, 16, fmt, seed=8, wmin=(0, 0, 0), scale=res)
    P = _params(16, 1, 9, scale=0.2)
    P[-1] = 0.3
    mlp = sf.MLP(torch.from_numpy(P).cuda(), 16, 1)
    rays = inputs.random_rays(1001, 1.0, seed=10)
    rays[0, 0] = np.nan
    steps, spp = 24, 2
    f = getattr(sf, "SF_" + filt)
    smp = sf.sampling(f, sf.SF_STOCHASTIC, spp, seed=12)
    taps = torch.empty((rays.shape[0], spp, steps, 3), dtype=torch.int32, device="cuda")
    T = sf.sf_neural_raymarch(grid, mlp, torch.from_numpy(rays).cuda(), steps, smp, dbg_taps=taps).cpu().numpy()
    ref, rt = orc.neural_raymarch(res, 16, H, Z, _bf16(P), (0, 0, 0), np.array(res, np.float32), rays, steps,
                                  getattr(orc, filt), orc.STOCHASTIC, spp=spp, seed=12, act_bf16=True, taps=True)
    assert np.array_equal(taps.cpu().numpy(), rt)
    # compare optical depths (T = mean of exp(-tau)); relative decode error carries to tau
    _close_bf16(T, ref)
    # without the tap dump the same stream gives the same result
    T2 = sf.sf_neural_raymarch(grid, mlp, torch.from_numpy(rays).cuda(), steps, smp).cpu().numpy()
    assert np.array_equal(T, T2, equal_nan=True)


def _normwise(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("C, O, B", [(8, 4, 700), (16, 1, 700), (8, 4, 690), (16, 1, 32769)])
def test_train_step_parity(sf, orc, C, O, B):
    """Gradients of one FP32 step (vector ALU) vs the FP64 oracle at the same
    inputs; the Adam updates follow from the GPU's own gradients; latents
    outside the batch are untouched.  Batch 690 leaves one chunk with an odd
    number of two-sample groups; batch 32769 makes 17-sample chunks and
    leaves the last workgroups without samples."""
    _case("train_step", C, O, B)
    rng = np.random.default_rng(20)
    nlat = max(2000, B + 1000)
    lat = rng.normal(size=(nlat, C)).astype(np.float32)
    P = _params(C, O, 21, scale=0.2)
    targets = rng.uniform(0, 1, size=(nlat, O)).astype(np.float32)
    idx = rng.permutation(nlat)[:B].astype(np.int32)
    st = sf.TrainState(torch.from_numpy(lat.ravel()).cuda(), torch.from_numpy(P).cuda(), C, O,
                       compute=sf.SF_TRAIN_FP32)
    gP = torch.zeros(P.size, dtype=torch.float32, device="cuda")
    gZ = torch.zeros((B, C), dtype=torch.float32, device="cuda")
    loss = sf.sf_neural_train_step(st, torch.from_numpy(idx).cuda(), torch.from_numpy(targets.ravel()).cuda(),
                                   lr_latent=1e-2, lr_mlp=1e-3, grad_params=gP, grad_latents=gZ)
    oloss, ogP, ogZ = orc.mlp_grad(C, H, O, P.astype(np.float64), lat[idx].astype(np.float64),
                                   targets[idx].astype(np.float64))
    assert abs(loss.item() - oloss) <= 1e-5 * oloss
    gp = gP.cpu().numpy()
    offs = np.cumsum([0, C * H, H, H * H, H, H * O, O])
    for a, b in zip(offs[:-1], offs[1:]):
        assert _normwise(gp[a:b], ogP[a:b]) <= 1e-5, (a, b, _normwise(gp[a:b], ogP[a:b]))
    assert _normwise(gZ.cpu().numpy(), ogZ) <= 1e-5
    # Adam step from the GPU's own gradients (first step: lr g / (|g| + eps))
    newP = st.params.cpu().numpy().astype(np.float64)
    g = gp.astype(np.float64)
    assert np.allclose(newP, P + -1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=2e-7)
    newZ = st.latents.cpu().numpy().reshape(nlat, C).astype(np.float64)
    gz = gZ.cpu().numpy().astype(np.float64)
    assert np.allclose(newZ[idx], lat[idx] - 1e-2 * gz / (np.abs(gz) + 1e-8), rtol=0, atol=2e-6)
    rest = np.setdiff1d(np.arange(nlat), idx)
    assert np.array_equal(newZ[rest], lat[rest].astype(np.float64))


def _weights_bf16(P, C, O):
    """The parameter vector with its weight blocks rounded to BF16 and its
    biases kept in FP32: the operands of the matrix-core step."""
    offs = np.cumsum([0, C * H, H, H * H, H, H * O, O])
    Q = P.astype(np.float64).copy()
    for k in (0, 2, 4):
        Q[offs[k]:offs[k + 1]] = _bf16(P[offs[k]:offs[k + 1]])
    return Q


@pytest.mark.parametrize("C, O, B", [(8, 4, 700), (16, 1, 700), (8, 4, 4099), (16, 1, 32769)])
def test_train_step_bf16_parity(sf, orc, C, O, B):
    """One matrix-core step (BF16 operands, FP32 accumulation): loss and
    gradients within 2e-2 normwise of the FP64 oracle run on the BF16-rounded
    weights and latents with its hidden activations stored in BF16 (so that
    both sides rectify the same second-layer pre-activations; the backward
    signals are rounded to BF16 on the GPU only, a relative 2^-9 each); Adam
    moves the FP32 master copies by the GPU's own gradients; latents outside
    the batch are untouched.  Batches of 4099 and 32769 leave ragged 16-sample tiles and
    empty trailing tiles."""
    _case("train_step_bf16", C, O, B)
    rng = np.random.default_rng(22)
    nlat = max(2000, B + 1000)
    lat = rng.normal(size=(nlat, C)).astype(np.float32)
    P = _params(C, O, 23, scale=0.2)
    targets = rng.uniform(0, 1, size=(nlat, O)).astype(np.float32)
    idx = rng.permutation(nlat)[:B].astype(np.int32)
    st = sf.TrainState(torch.from_numpy(lat.ravel()).cuda(), torch.from_numpy(P).cuda(), C, O)
    assert st.compute == sf.SF_TRAIN_BF16
    gP = torch.zeros(P.size, dtype=torch.float32, device="cuda")
    gZ = torch.zeros((B, C), dtype=torch.float32, device="cuda")
    loss = sf.sf_neural_train_step(st, torch.from_numpy(idx).cuda(), torch.from_numpy(targets.ravel()).cuda(),
                                   lr_latent=1e-2, lr_mlp=1e-3, grad_params=gP, grad_latents=gZ)
    oloss, ogP, ogZ = orc.mlp_grad(C, H, O, _weights_bf16(P, C, O), _bf16(lat[idx]), targets[idx].astype(np.float64),
                                   act_bf16=True)
    assert abs(loss.item() - oloss) <= 2e-2 * oloss
    gp = gP.cpu().numpy()
    offs = np.cumsum([0, C * H, H, H * H, H, H * O, O])
    for a, b in zip(offs[:-1], offs[1:]):
        assert _normwise(gp[a:b], ogP[a:b]) <= 2e-2, (a, b, _normwise(gp[a:b], ogP[a:b]))
    assert _normwise(gZ.cpu().numpy(), ogZ) <= 2e-2
    newP = st.params.cpu().numpy().astype(np.float64)
    g = gp.astype(np.float64)
    assert np.allclose(newP, P + -1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=2e-7)
    newZ = st.latents.cpu().numpy().reshape(nlat, C).astype(np.float64)
    gz = gZ.cpu().numpy().astype(np.float64)
    assert np.allclose(newZ[idx], lat[idx] - 1e-2 * gz / (np.abs(gz) + 1e-8), rtol=0, atol=2e-6)
    rest = np.setdiff1d(np.arange(nlat), idx)
    assert np.array_equal(newZ[rest], lat[rest].astype(np.float64))


def test_checkpoint_resume_is_bit_exact(sf, tmp_path):
    """Training state saved after k steps and restored (latents, MLP, both
    Adam moments, step, seed) continues to the same state, bit for bit, as an
    uninterrupted run over the same batches; both compute modes."""
    _case("checkpoint_resume")
    rng = np.random.default_rng(30)
    C, O, nlat, B, steps, k = 16, 1, 6000, 1024, 12, 5
    lat0 = rng.normal(size=nlat * C).astype(np.float32)
    P0 = _params(C, O, 31, scale=0.2)
    tg = torch.from_numpy(rng.uniform(0, 1, size=nlat * O).astype(np.float32)).cuda()

    def batches(seed, first, last):
        for s in range(first, last):
            r = np.random.default_rng([seed, s])
            yield torch.from_numpy(r.permutation(nlat)[:B].astype(np.int32)).cuda()

    for compute in (sf.SF_TRAIN_BF16, sf.SF_TRAIN_FP32):
        full = sf.TrainState(torch.from_numpy(lat0.copy()).cuda(), torch.from_numpy(P0.copy()).cuda(), C, O,
                             compute=compute)
        for b in batches(7, 0, steps):
            sf.sf_neural_train_step(full, b, tg, 1e-2, 1e-3)
        part = sf.TrainState(torch.from_numpy(lat0.copy()).cuda(), torch.from_numpy(P0.copy()).cuda(), C, O,
                             compute=compute)
        for b in batches(7, 0, k):
            sf.sf_neural_train_step(part, b, tg, 1e-2, 1e-3)
        path = str(tmp_path / f"ckpt{compute}.npz")
        part.save(path, seed=7)
        del part
        res, seed = sf.TrainState.load(path)
        assert seed == 7 and res.step == k and res.compute == compute
        for b in batches(seed, k, steps):
            sf.sf_neural_train_step(res, b, tg, 1e-2, 1e-3)
        torch.cuda.synchronize()
        for a, b in ((full.latents, res.latents), (full.params, res.params), (full.m_lat, res.m_lat),
                     (full.v_lat, res.v_lat), (full.m_par, res.m_par), (full.v_par, res.v_par)):
            assert torch.equal(a, b)
        assert res.step == full.step == steps


def test_training_converges_and_decodes(sf, orc):
    """A small neural texture trained on the matrix cores (BF16) on plain
    B-spline magnification targets: the loss drops by more than 20x and the
    BF16 matrix-core decoder reproduces the targets closely."""
    _case("train_converge")
    src = inputs.texture_uniform(8, seed=1)
    R = 64
    lat_uv = np.zeros((R * R, 3), np.float32)
    yy, xx = np.mgrid[0:R, 0:R]
    lat_uv[:, 0] = ((xx + 0.5) / R).ravel()
    lat_uv[:, 1] = ((yy + 0.5) / R).ravel()
    tex = sf.Texture2D([src])
    targets = sf.sf_filter2d(tex, torch.from_numpy(lat_uv).cuda(), sf.sampling(sf.SF_BSPLINE3, sf.SF_BEFORE, 1))
    rng = np.random.default_rng(3)
    lat = (rng.normal(size=(R * R, 8)) * 0.1).astype(np.float32)
    P = _params(8, 4, 4, scale=0.15)
    st = sf.TrainState(torch.from_numpy(lat.ravel()).cuda(), torch.from_numpy(P).cuda(), 8, 4)
    losses = []
    gen = torch.Generator(device="cuda").manual_seed(0)
    for it in range(600):
        perm = torch.randperm(R * R, device="cuda", generator=gen)[:1024].to(torch.int32)
        l = sf.sf_neural_train_step(st, perm, targets, lr_latent=1e-2, lr_mlp=2e-3)
        if it % 50 == 0 or it == 599:
            losses.append(l.item())
    assert losses[-1] < losses[0] / 20, losses
    grid = sf.sf_neural_quantize(st.latents, 2, (R, R), 8, sf.SF_LATENT_BF16)
    mlp = sf.MLP(st.params, 8, 4)
    dec = sf.sf_neural_decode_lattice(grid, mlp, torch.arange(R * R, device="cuda", dtype=torch.int64))
    rmse = torch.sqrt(torch.mean((dec - targets) ** 2)).item()
    assert rmse < 0.05, rmse


# ------------------------------------------------ config 4 and 5 at full size
def test_neural_filter2d_config4_full_sampled(sf, orc):
    """Config 4 at its size, in the launch the benchmark times: a 1024^2 x 8
    BF16 latent texture, the 8-64-64-4 MLP, 2 Mi uniform queries shaded by
    GGX + Lambert, stochastic B-spline (one decode) and the 16-decode
    filter-after and filter-before comparators.  3000 sampled queries (the
    ragged tail among them) against the oracle; every stochastic tap of the
    sample bit-exact.  Latents and weights are seeded random values: the
    decoder's arithmetic does not depend on them being trained."""
    R, n = 1024, 2 * 1024 * 1024
    rng = np.random.default_rng(61)
    lat = (rng.standard_normal(R * R * 8, dtype=np.float32) * np.float32(0.7)).reshape(R * R, 8)
    grid = sf.sf_neural_quantize(torch.from_numpy(lat.ravel()).cuda(), 2, (R, R), 8, sf.SF_LATENT_BF16)
    Z = _bf16(lat)
    P = _params(8, 4, 62)
    mlp = sf.MLP(torch.from_numpy(P).cuda(), 8, 4)
    q = inputs.queries_uniform(n, seed=6)
    qd = torch.from_numpy(q).cuda()
    sub = np.unique(np.concatenate([rng.choice(n - 500, 2500, replace=False), np.arange(n - 500, n)]))
    for mode in ("STOCHASTIC", "AFTER", "BEFORE"):
        _case("neural_filter2d_config4_full", mode)
        m = {"STOCHASTIC": sf.SF_STOCHASTIC, "AFTER": sf.SF_AFTER_EXACT, "BEFORE": sf.SF_BEFORE}[mode]
        smp = sf.sampling(sf.SF_BSPLINE3, m, 1, seed=3)
        out = sf.sf_neural_decode(grid, mlp, qd, smp, shade=sf.SF_SHADE_GGX, ggx_params=sf.ggx()).cpu().numpy()
        om = {"STOCHASTIC": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
        res_ = orc.neural_filter2d((R, R), 8, H, 4, Z, _bf16(P), q, orc.BSPLINE3, om, spp=1, seed=3, shade=1,
                                   act_bf16=True, taps=mode == "STOCHASTIC", subset=sub)
        if mode == "STOCHASTIC":
            ref, rt = res_
            taps = torch.empty((n, 1, 2), dtype=torch.int32, device="cuda")
            out_t = sf.sf_neural_decode(grid, mlp, qd, smp, shade=sf.SF_SHADE_GGX, ggx_params=sf.ggx(),
                                        dbg_taps=taps).cpu().numpy()
            assert np.array_equal(taps.cpu().numpy()[sub], rt)
            assert np.array_equal(out_t, out)   # the tap dump changes nothing else
        else:
            ref = res_
        _close_bf16(out[sub], ref)


def test_neural_quantize_config5_full_sampled_blocks(sf, orc):
    """The E4M3 quantiser at config 5's size (256^3 x 16 FP32 latents, 8^3
    blocks): the codes and scale of 48 sampled blocks, corner blocks among
    them, equal the oracle's quantisation of each block alone, bit for bit
    (a block's scale and codes depend only on its own values)."""
    _case("quantize_config5_full")
    L, C, B = 256, 16, 8
    rng = np.random.default_rng(63)
    lat = rng.standard_normal(L ** 3 * C, dtype=np.float32) * np.float32(0.5)
    lat[: 4096 * C] *= np.float32(100.0)        # a slab of much larger values
    grid = sf.sf_neural_quantize(torch.from_numpy(lat).cuda(), 3, (L, L, L), C, sf.SF_LATENT_FP8E4M3, 3,
                                 (0.0, 0.0, 0.0), (L / 0.25,) * 3)
    nb = L // B
    blocks = np.concatenate([[0, nb - 1, nb ** 3 - 1, nb * nb * (nb - 1)], rng.choice(nb ** 3, 44, replace=False)])
    lat4 = lat.reshape(L, L, L, C)
    scales = grid.scales.cpu().numpy()
    for b in blocks:
        bz, by, bx = b // (nb * nb), (b // nb) % nb, b % nb
        vals = np.ascontiguousarray(lat4[bz * B:(bz + 1) * B, by * B:(by + 1) * B, bx * B:(bx + 1) * B])
        codes, sc = orc.quantize_fp8(vals.ravel(), 3, (B, B, B), C, 3)
        zz, yy, xx = np.meshgrid(np.arange(bz * B, bz * B + B), np.arange(by * B, by * B + B),
                                 np.arange(bx * B, bx * B + B), indexing="ij")
        lin = ((zz * L + yy) * L + xx).ravel()
        got = grid.latents.view(L ** 3, C)[torch.from_numpy(lin).cuda()].cpu().numpy()
        assert np.array_equal(got.ravel(), codes), b
        assert scales[b] == sc[0], (b, scales[b], sc[0])


def test_neural_raymarch_config5_full_sampled(sf, orc):
    """Config 5 at its size, in the launch the benchmark times: a 256^3 x 16
    E4M3 latent volume with 8^3 block scales over a cube of side 0.25, the
    16-64-64-1 MLP, 512^2 pixels x 16 orthographic rays (4 Mi) x 128 steps,
    stochastic tricubic on the latent lattice.  The codes and scales are
    seeded inputs given to both sides.  450 sampled rays (misses among them)
    against the oracle; their taps, taken from a tap-dump launch over all
    4 Mi rays, bit-exact; and that launch's transmittances equal the timed
    launch's."""
    _case("neural_raymarch_config5_full")
    L, C, side, steps = 256, 16, 0.25, 128
    rng = np.random.default_rng(64)
    # E4M3 codes of magnitudes 1/4 .. 7.5 (exponent fields 5..9, any mantissa), either sign
    codes = (rng.integers(5, 10, size=L ** 3 * C, dtype=np.uint8) << 3) | rng.integers(0, 8, size=L ** 3 * C,
                                                                                          dtype=np.uint8)
    codes[rng.random(codes.size) < 0.5] |= 0x80
    nb = L // 8
    scales = rng.uniform(0.1, 0.5, size=nb ** 3).astype(np.float32)
    grid = sf.LatentGrid(3, (L, L, L), C, sf.SF_LATENT_FP8E4M3, torch.from_numpy(codes).cuda(),
                         torch.from_numpy(scales).cuda(), 3, (0.0, 0.0, 0.0), (L / side,) * 3)
    P = _params(C, 1, 65, scale=0.2)
    P[-1] = 3.0
    mlp = sf.MLP(torch.from_numpy(P).cuda(), C, 1)
    rays = inputs.ortho_rays(512, 16, side=side, seed=12)
    n = rays.shape[0]
    rd = torch.from_numpy(rays).cuda()
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=4)
    T = sf.sf_neural_raymarch(grid, mlp, rd, steps, smp).cpu().numpy()
    taps_d = torch.empty((n, 1, steps, 3), dtype=torch.int32, device="cuda")
    T_dbg = sf.sf_neural_raymarch(grid, mlp, rd, steps, smp, dbg_taps=taps_d).cpu().numpy()
    assert np.array_equal(T_dbg, T, equal_nan=True)
    hit = np.nonzero(rays[:, 7] > rays[:, 6])[0]
    miss = np.nonzero(~(rays[:, 7] > rays[:, 6]))[0]
    sub = np.unique(np.concatenate([rng.choice(hit, 400, replace=False), rng.choice(miss, 50, replace=False),
                                    np.arange(n - 8, n)]))
    taps = taps_d[torch.from_numpy(sub).cuda()].cpu().numpy()
    del taps_d
    torch.cuda.empty_cache()
    # the oracle decodes the same codes: E4M3 value times the block scale, as a BF16 operand
    i = np.arange(L)
    blk = ((i[:, None, None] >> 3) * nb * nb + (i[None, :, None] >> 3) * nb + (i[None, None, :] >> 3)).ravel()
    Z = orc.dequant_fp8(codes, scales[blk], C)
    ref, rt = orc.neural_raymarch((L, L, L), C, H, Z, _bf16(P), (0, 0, 0), np.array((L / side,) * 3, np.float32),
                                  rays, steps, orc.BSPLINE3, orc.STOCHASTIC, spp=1, seed=4, act_bf16=True, taps=True,
                                  subset=sub)
    assert np.array_equal(taps, rt)
    assert np.all(T[miss] == 1.0)
    assert 0.05 < np.median(ref[np.isin(sub, hit)]) < 0.95   # a medium neither empty nor opaque
    _close_bf16(T[sub], ref)
