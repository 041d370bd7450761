"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: tap indices bit-exact given the same random stream; values within
1e-5 relative (the floating-point tolerance stated for the method's shaded
values with FP32 texels), with a 1e-7 absolute floor for exact zeros.  Small
cases span several 256-lane blocks and a ragged tail; full-size cases run in
the launch configuration the benchmark times and are checked on sampled
outputs the oracle computes one by one.
"""
import math

import numpy as np
import pytest
import torch

from paper_2407_06107_amd import inputs

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-7


@pytest.fixture(scope="module")
def sf():
    import paper_2407_06107_amd as sf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sf.lib()
    return sf


def _close(gpu, ref, rtol=RTOL, atol=ATOL):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    nan_g, nan_r = np.isnan(gpu), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), "NaN pattern differs"
    g, r = gpu[~nan_g], ref[~nan_r]
    err = np.abs(g - r)
    bad = err > atol + rtol * np.abs(r)
    assert not bad.any(), f"{bad.sum()} of {bad.size} outside tolerance; worst rel {np.max(err / (np.abs(r) + atol)):.3e}"


def _print_case(*args):
    print("CASE", *args, flush=True)


# ------------------------------------------------------------------ 3-D grids
@pytest.fixture(scope="module")
def small_cloud():
    g = inputs.cloud_grid(48, seed=4).numpy()[:40, :36, :44].copy()   # nz, ny, nx: non-cubic
    return g


def _grids(orc, sf, data, side=1.0):
    nz, ny, nx = data.shape
    scale = (nx / side, ny / side, nz / side)
    og = orc.Grid(data, scale=scale)
    vol = sf.Volume(torch.from_numpy(data).cuda(), scale=scale)
    return og, vol


MODES3 = [("STOCH", 1, 0), ("STOCH", 3, 1), ("BEFORE", 1, 0), ("AFTER", 1, 0)]


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode, spp, variant", MODES3)
@pytest.mark.parametrize("dtype", ["float16", "float32"])
def test_raymarch_small(sf, orc, small_cloud, filt, mode, spp, variant, dtype):
    _print_case("raymarch_small", filt, mode, spp, variant, dtype)
    data = small_cloud.astype(dtype)
    og, vol = _grids(orc, sf, data)
    rays = inputs.random_rays(3001, 1.0, seed=21)       # 11 full blocks + a ragged tail, some misses
    steps = 48
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, spp, seed=77, rng_variant=variant)
    rays_d = torch.from_numpy(rays).cuda()
    taps_d = torch.empty((rays.shape[0], spp, steps, 3), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    T = sf.sf_raymarch(vol, rays_d, steps, smp, dbg_taps=taps_d)
    torch.cuda.synchronize()
    if m == orc.STOCHASTIC:
        ref, taps = orc.raymarch(og, rays, steps, f, m, spp=spp, seed=77, variant=variant, taps=True)
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = orc.raymarch(og, rays, steps, f, m, spp=spp, seed=77, variant=variant)
    _close(T.cpu().numpy(), ref)


def test_raymarch_edge_cases(sf, orc, small_cloud):
    _print_case("raymarch_edge_cases")
    og, vol = _grids(orc, sf, small_cloud)
    rays = np.array([
        [0.5, 0.5, -1.0, 0, 0, 1, 1.0, 2.0],       # through the grid
        [np.nan, 0.5, 0.5, 0, 0, 1, 0.0, 1.0],     # non-finite -> NaN
        [0.5, 0.5, 0.5, 0, 0, 1, 0.4, 0.4],        # empty segment -> 1
        [5.0, 5.0, 5.0, 1, 0, 0, 0.0, 1.0],        # entirely outside -> 1 (zero density)
        [1e9, 0.5, 0.5, 1, 0, 0, 0.0, 1.0],        # beyond 2^22 voxels -> NaN
        [0.5, 0.5, 0.5, 0, 1, 0, -0.6, 0.6],       # enters and leaves through the border
    ], dtype=np.float32)
    rays_d = torch.from_numpy(rays).cuda()
    for steps in (1, 7, 64):
        for filt in (orc.LINEAR, orc.BSPLINE3):
            for m in (orc.STOCHASTIC, orc.BEFORE, orc.AFTER):
                smp = sf.sampling(filt, m, 2, seed=3)
                taps_d = torch.full((6, 2, steps, 3), 7, dtype=torch.int32, device="cuda")
                T = sf.sf_raymarch(vol, rays_d, steps, smp, dbg_taps=taps_d if m == orc.STOCHASTIC else None)
                if m == orc.STOCHASTIC:
                    ref, taps = orc.raymarch(og, rays, steps, filt, m, spp=2, seed=3, taps=True)
                    assert np.array_equal(taps_d.cpu().numpy(), taps)
                else:
                    ref = orc.raymarch(og, rays, steps, filt, m, spp=2, seed=3)
                _close(T.cpu().numpy(), ref)
                t = T.cpu().numpy()
                assert np.isnan(t[1]) and t[2] == 1.0 and t[3] == 1.0 and np.isnan(t[4])
    # n = 0 is a no-op
    empty = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    out = sf.sf_raymarch(vol, empty, 16, sf.sampling(2, 2, 1))
    assert out.numel() == 0


def test_raymarch_deterministic_repeat(sf, orc, small_cloud):
    _print_case("raymarch_deterministic_repeat")
    _, vol = _grids(orc, sf, small_cloud)
    rays = torch.from_numpy(inputs.random_rays(5000, 1.0, seed=2)).cuda()
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=9)
    a = sf.sf_raymarch(vol, rays, 64, smp).clone()
    b = sf.sf_raymarch(vol, rays, 64, smp)
    assert torch.equal(a, b)


def test_raymarch_stochastic_mean_matches_expectation(sf, orc, small_cloud):
    """Unbiasedness on the GPU: the mean over many samples is within 5
    standard errors of the oracle's exact expectation (= exact after)."""
    _print_case("raymarch_stochastic_mean")
    og, vol = _grids(orc, sf, small_cloud)
    rays = inputs.random_rays(64, 1.0, seed=8)
    spp = 4096
    T = sf.sf_raymarch(vol, torch.from_numpy(rays).cuda(), 24, sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, spp, seed=1))
    e = orc.raymarch_expect(og, rays, 24, orc.BSPLINE3)
    assert np.max(np.abs(T.cpu().numpy() - e)) < 5 * 0.5 / math.sqrt(spp)


@pytest.fixture(scope="module")
def full_cloud():
    """Config-3 workload: 512^3 fp16 cloud (cube side 0.25) and 256^2 px x 16 rays."""
    _print_case("full_cloud generate")
    side = 0.25
    data = inputs.cloud_grid(512, seed=4, device="cuda")
    rays = inputs.ortho_rays(256, 16, side=side, seed=11)
    return data, rays, side


@pytest.mark.parametrize("filt, mode", [("BSPLINE3", "STOCH"), ("LINEAR", "STOCH"), ("BSPLINE3", "BEFORE"),
                                        ("BSPLINE3", "AFTER"), ("LINEAR", "AFTER")])
def test_raymarch_full_size_sampled(sf, orc, full_cloud, filt, mode):
    _print_case("raymarch_full_size", filt, mode)
    data, rays, side = full_cloud
    steps = 256
    vol = sf.Volume(data, side=side)
    host = data.cpu().numpy()
    og = orc.Grid(host, side=side)
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, 1, seed=2024)
    rays_d = torch.from_numpy(rays).cuda()
    T = sf.sf_raymarch(vol, rays_d, steps, smp).cpu().numpy()
    vol_skip = sf.Volume(data, side=side, brick_log2=3)            # the benchmark's configuration
    T_skip = sf.sf_raymarch(vol_skip, rays_d, steps, smp).cpu().numpy()
    # a skipped step adds an exact zero (or multiplies by exactly 1), which the
    # compensated sum and the pair product leave bit-identical
    assert np.array_equal(T, T_skip, equal_nan=True)
    rng = np.random.default_rng(5)
    sub = np.sort(rng.choice(rays.shape[0], 400, replace=False))
    ref = orc.raymarch(og, rays, steps, f, m, spp=1, seed=2024, subset=sub)
    _close(T[sub], ref)
    if m == orc.STOCHASTIC:
        # taps of a prefix of the same stream (same ray indices, same keys)
        k = 1024
        taps_d = torch.empty((k, 1, steps, 3), dtype=torch.int32, device="cuda")
        Tk = sf.sf_raymarch(vol, rays_d[:k].contiguous(), steps, smp, dbg_taps=taps_d)
        refk, taps = orc.raymarch(og, rays[:k], steps, f, m, spp=1, seed=2024, taps=True)
        assert np.array_equal(taps_d.cpu().numpy(), taps)
        _close(Tk.cpu().numpy(), refk)
        assert np.array_equal(Tk.cpu().numpy(), T[:k])


@pytest.mark.parametrize("lg", [1, 2, 3, 5, 6])
def test_occupancy_parity(sf, orc, small_cloud, lg):
    _print_case("occupancy_parity", lg)
    data = small_cloud.copy()
    data[:, :, 30:] = 0.0                                  # a slab of empty space
    og, vol = _grids(orc, sf, data)
    nz, ny, nx = data.shape
    occ = sf.sf_build_occupancy(vol, lg).cpu().numpy().view(np.uint32)
    ref = orc.build_occupancy(og, lg)
    B = 1 << lg
    nb = [-(-n // B) for n in (nx, ny, nz)]
    sx, sy = nb[0] + 1, nb[1] + 1
    assert occ.size == -(-(sx * sy * nb[2]) // 32)
    bits = np.unpackbits(occ.view(np.uint8), bitorder="little")
    m = bits[:sx * sy * nb[2]].reshape(nb[2], sy, sx)
    rbits = np.unpackbits(ref.view(np.uint8), bitorder="little")[:nb[0] * nb[1] * nb[2]]
    # one bit per brick, 1 = provably empty = the oracle's clear bit; padding and tail 0
    assert np.array_equal(m[:, :nb[1], :nb[0]].ravel(), 1 - rbits)
    assert not m[:, nb[1]:, :].any() and not m[:, :, nb[0]:].any()
    assert not bits[sx * sy * nb[2]:].any()


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
def test_raymarch_occupancy_skip_is_exact(sf, orc, small_cloud, filt):
    """Skipping empty bricks leaves every mode's result bit-identical (a
    skipped step adds an exact zero to a compensated sum, or multiplies a pair
    product by exactly 1); the oracle agrees."""
    _print_case("raymarch_occupancy_skip", filt)
    data = small_cloud.copy()
    data[:, :, 30:] = 0.0
    og, plain = _grids(orc, sf, data)
    nz, ny, nx = data.shape
    skip = sf.Volume(plain.data, scale=(nx, ny, nz), brick_log2=2)
    rays_d = torch.from_numpy(inputs.random_rays(3001, 1.0, seed=21)).cuda()
    f = getattr(sf, "SF_" + filt)
    for mode, spp in ((sf.SF_STOCHASTIC, 1), (sf.SF_STOCHASTIC, 2), (sf.SF_BEFORE, 1), (sf.SF_AFTER_EXACT, 1)):
        smp = sf.sampling(f, mode, spp, seed=13)
        a = sf.sf_raymarch(plain, rays_d, 40, smp).cpu().numpy()
        b = sf.sf_raymarch(skip, rays_d, 40, smp).cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True)
        ref = orc.raymarch(og, rays_d.cpu().numpy(), 40, getattr(orc, filt), mode, spp=spp, seed=13)
        _close(b, ref)


@pytest.mark.parametrize("steps", [1, 2, 3, 7, 41])
@pytest.mark.parametrize("filt, spp, variant", [("BSPLINE3", 1, 0), ("BSPLINE3", 3, 0), ("LINEAR", 1, 0),
                                                ("BSPLINE3", 2, 1)])
def test_raymarch_occupancy_pow2_odd_steps(sf, orc, filt, spp, variant, steps):
    """The skipping march on a grid with power-of-two x and y (the
    benchmark's addressing) over odd and even step counts (its loop takes two
    steps per pass and a last single step): bit-identical to the march without
    the mask, and equal to the oracle, for bricks of 2^2 and 2^3 voxels."""
    _print_case("raymarch_occupancy_pow2", filt, spp, variant, steps)
    data = inputs.cloud_grid(64, seed=9).numpy()[:40, :32, :64].copy()   # nz, ny, nx = 40, 32, 64
    data[:, :, 40:] = 0.0
    data[:6] = 0.0
    og, plain = _grids(orc, sf, data)
    nz, ny, nx = data.shape
    rays = inputs.random_rays(2049, 1.0, seed=23)
    rays_d = torch.from_numpy(rays).cuda()
    f = getattr(sf, "SF_" + filt)
    smp = sf.sampling(f, sf.SF_STOCHASTIC, spp, seed=29, rng_variant=variant)
    a = sf.sf_raymarch(plain, rays_d, steps, smp).cpu().numpy()
    for lg in (2, 3, 6):   # 6: one brick per axis, mask rows and planes of two
        skip = sf.Volume(plain.data, scale=(nx, ny, nz), brick_log2=lg)
        b = sf.sf_raymarch(skip, rays_d, steps, smp).cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), lg
    ref = orc.raymarch(og, rays, steps, getattr(orc, filt), orc.STOCHASTIC, spp=spp, seed=29, variant=variant)
    _close(a, ref)


# ------------------------------------------------------------------ 2-D
@pytest.fixture(scope="module")
def c1(orc):
    tex = inputs.texture_uniform(64, seed=1)
    q = inputs.queries_uniform(4096, seed=2)
    q[:7, 0] = [-0.25, 1.0, 1.75, 0.999999, -1e-9, 0.5, 0.25]     # wrap cases
    q[7, 1] = np.nan                                            # non-finite -> NaN
    return tex, q


MODES2 = [("STOCH", 16, 0), ("STOCH", 5, 1), ("STOCH", 1, 0), ("BEFORE", 1, 0), ("AFTER", 1, 0)]


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode, spp, variant", MODES2)
@pytest.mark.parametrize("shade", [0, 1])
@pytest.mark.parametrize("wrap", [0, 1])
def test_filter2d_config1(sf, orc, c1, filt, mode, spp, variant, shade, wrap):
    _print_case("filter2d_c1", filt, mode, spp, variant, shade, wrap)
    tex, q = c1
    ot = orc.Tex2D.rgba32f(tex, wrap=wrap)
    gt = sf.Texture2D([tex], wrap=wrap)
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, spp, seed=123, rng_variant=variant)
    qd = torch.from_numpy(q).cuda()
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, qd, smp, shade=shade, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, f, m, spp=spp, seed=123, variant=variant, shade=shade, taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("texkind", ["rgba32f_64", "rgba8_64_mips", "rgba8_100x60_mips"])
@pytest.mark.parametrize("spp, variant, shade", [(16, 0, 1), (5, 1, 0), (1, 0, 1)])
def test_filter2d_texture_in_lds_equals_global(sf, c1, filt, texkind, spp, variant, shade, monkeypatch):
    """Textures of at most 64 KiB are staged in LDS by the stochastic kernel
    (RGBA32F 64^2 is exactly 64 KiB; the RGBA8 pyramids end on a 4-byte
    tail): outputs and taps equal, bit for bit, those of the same launch
    reading global memory (SF_NO_LDS_TEXTURE=1)."""
    _print_case("tex_lds", filt, texkind, spp, variant, shade)
    _, q = c1
    if texkind == "rgba32f_64":
        gt = sf.Texture2D([inputs.texture_uniform(64, seed=1)])
    else:
        full = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(128, seed=4, waves=6)))
        if texkind == "rgba8_64_mips":
            lv = full[1:]
        else:
            lv = [np.ascontiguousarray(f[:max(1, 60 >> l), :max(1, 100 >> l)]) for l, f in enumerate(full[:7])]
        gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    qq = q.copy()
    qq[:, 2] = np.linspace(0.0, 7.0, qq.shape[0], dtype=np.float32)   # levels across the pyramid
    qd = torch.from_numpy(qq).cuda()
    smp = sf.sampling(getattr(sf, "SF_" + filt), sf.SF_STOCHASTIC, spp, seed=17, rng_variant=variant)
    res = []
    for flag in ("0", "1"):
        monkeypatch.setenv("SF_NO_LDS_TEXTURE", flag)
        taps = torch.empty((qq.shape[0], spp, 3), dtype=torch.int32, device="cuda")
        out = sf.sf_filter2d(gt, qd, smp, shade=shade, ggx_params=sf.ggx() if shade else None, dbg_taps=taps)
        res.append((out.cpu().numpy(), taps.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0], equal_nan=True)
    assert np.array_equal(res[0][1], res[1][1])


@pytest.fixture(scope="module")
def c2_small(orc):
    size = 256
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(size, seed=3, waves=12)))
    q = inputs.plane_queries(160, 90, tex_size=size, levels=len(lv))
    return lv, q


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mip", [1, 2])
@pytest.mark.parametrize("mode, spp", [("STOCH", 16), ("STOCH", 1), ("BEFORE", 1), ("AFTER", 1)])
def test_filter2d_mips_rgba8(sf, orc, c2_small, filt, mip, mode, spp):
    _print_case("filter2d_mips", filt, mip, mode, spp)
    lv, q = c2_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, mip)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=mip)
    assert list(gt.offsets) == list(offs)
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, spp, seed=5)
    qd = torch.from_numpy(q).cuda()
    taps_d = torch.empty((q.shape[0], spp, 3), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, qd, smp, shade=1, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, f, m, spp=spp, seed=5, shade=1, taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.fixture(scope="module")
def c2_full():
    _print_case("c2_full generate")
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(4096, seed=3)))
    q = inputs.plane_queries(1920, 1080, tex_size=4096, levels=len(lv))
    return lv, q


@pytest.mark.parametrize("filt, mode, spp", [("BSPLINE3", "STOCH", 16), ("BSPLINE3", "STOCH", 1),
                                             ("LINEAR", "STOCH", 16), ("BSPLINE3", "AFTER", 1),
                                             ("BSPLINE3", "BEFORE", 1)])
def test_filter2d_config2_full_sampled(sf, orc, c2_full, filt, mode, spp):
    _print_case("filter2d_c2_full", filt, mode, spp)
    lv, q = c2_full
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, spp, seed=31)
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx()).cpu().numpy()
    sub = np.sort(np.random.default_rng(1).choice(q.shape[0], 3000, replace=False))
    ref = orc.filter2d(ot, q, f, m, spp=spp, seed=31, shade=1, subset=sub)
    _close(out[sub], ref)


# ------------------------------------------------------------------ 2-D Keys cubic (positivised)
def _close_signed(gpu, ref, scale):
    """Positivised estimates subtract a negative-lobe term from a positive
    one, so the binary32 rounding error scales with the terms' magnitude
    (at most about 1.6 times the largest shaded value: the Keys block sums
    are below 1.28 and 0.28), not with the possibly near-zero difference."""
    _close(gpu, ref, atol=RTOL * 1.6 * scale)


@pytest.mark.parametrize("filt", ["KEYS3", "MITCHELL"])
@pytest.mark.parametrize("mode, spp", [("STOCH", 16), ("STOCH", 5), ("STOCH", 1), ("BEFORE", 1), ("AFTER", 1)])
@pytest.mark.parametrize("shade", [0, 1])
@pytest.mark.parametrize("wrap", [0, 1])
def test_filter2d_keys_config1(sf, orc, c1, filt, mode, spp, shade, wrap):
    _print_case("filter2d_keys_c1", filt, mode, spp, shade, wrap)
    tex, q = c1
    ot = orc.Tex2D.rgba32f(tex, wrap=wrap)
    gt = sf.Texture2D([tex], wrap=wrap)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=77)
    taps_d = torch.full((q.shape[0], spp, 5), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=shade, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, getattr(orc, filt), m, spp=spp, seed=77, shade=shade, taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close_signed(out.cpu().numpy(), ref, np.nanmax(np.abs(ref)))


@pytest.mark.parametrize("filt", ["KEYS3", "MITCHELL"])
@pytest.mark.parametrize("mip", [0, 2])
@pytest.mark.parametrize("mode, spp", [("STOCH", 8), ("AFTER", 1), ("BEFORE", 1)])
def test_filter2d_keys_mips_rgba8(sf, orc, c2_small, filt, mip, mode, spp):
    _print_case("filter2d_keys_mips", filt, mip, mode, spp)
    lv, q = c2_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, mip)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=mip)
    m = {"STOCH": orc.STOCHASTIC, "AFTER": orc.AFTER, "BEFORE": orc.BEFORE}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=6)
    taps_d = torch.empty((q.shape[0], spp, 5), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, getattr(orc, filt), m, spp=spp, seed=6, shade=1, taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close_signed(out.cpu().numpy(), ref, np.nanmax(np.abs(ref)))


def test_filter2d_keys_texel_centres_exact(sf, orc):
    """At texel centres the Keys cubic interpolates: t = 0 on both axes
    leaves no negative weight, so every sample reads the centre texel and
    the estimate is that texel exactly."""
    R = 32
    tex = inputs.texture_uniform(R, seed=8)
    iy, ix = np.meshgrid(np.arange(R), np.arange(R), indexing="ij")
    q = np.stack([(ix.ravel() + 0.5) / R, (iy.ravel() + 0.5) / R, np.zeros(R * R)], 1).astype(np.float32)
    gt = sf.Texture2D([tex])
    taps_d = torch.empty((R * R, 4, 5), dtype=torch.int32, device="cuda")
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), sf.sampling(sf.SF_KEYS3, sf.SF_STOCHASTIC, 4, seed=1),
                         dbg_taps=taps_d).cpu().numpy()
    t = taps_d.cpu().numpy()
    assert np.all(t[..., 3:] == orc.TAP_NONE)
    assert np.array_equal(t[..., 1], np.repeat(ix.ravel()[:, None], 4, 1))
    assert np.array_equal(out, tex.reshape(-1, 4))


@pytest.mark.parametrize("filt", ["KEYS3", "MITCHELL"])
def test_filter2d_keys_config2_full_sampled(sf, orc, c2_full, filt):
    _print_case("filter2d_keys_c2_full", filt)
    lv, q = c2_full
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    smp = sf.sampling(getattr(sf, "SF_" + filt), sf.SF_STOCHASTIC, 16, seed=32)
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx()).cpu().numpy()
    sub = np.sort(np.random.default_rng(2).choice(q.shape[0], 3000, replace=False))
    ref = orc.filter2d(ot, q, getattr(orc, filt), orc.STOCHASTIC, spp=16, seed=32, shade=1, subset=sub)
    _close_signed(out[sub], ref, np.nanmax(np.abs(ref)))


# ------------------------------------------------------------------ 2-D Gaussian FRS / FIS, B-spline FIS
GAUSS = [("GAUSS_FRS", 0.3), ("GAUSS_FRS", 0.8), ("GAUSS_FRS", 1 / 16), ("GAUSS_FIS", 0.3), ("GAUSS_FIS", 0.8),
         ("GAUSS_FIS", 4.0), ("BSPLINE3_FIS", 0.5)]


@pytest.mark.parametrize("filt, sigma", GAUSS)
@pytest.mark.parametrize("mode, spp", [("STOCH", 16), ("STOCH", 3), ("BEFORE", 1), ("AFTER", 1)])
@pytest.mark.parametrize("shade", [0, 1])
@pytest.mark.parametrize("wrap", [0, 1])
def test_filter2d_gauss_fis_config1(sf, orc, c1, filt, sigma, mode, spp, shade, wrap):
    _print_case("filter2d_gauss_c1", filt, sigma, mode, spp, shade, wrap)
    tex, q = c1
    ot = orc.Tex2D.rgba32f(tex, wrap=wrap)
    gt = sf.Texture2D([tex], wrap=wrap)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=91, sigma=sigma)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=shade, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, getattr(orc, filt), m, spp=spp, seed=91, shade=shade, taps=m == orc.STOCHASTIC,
                       sigma=sigma)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("filt, sigma", [("GAUSS_FRS", 0.5), ("GAUSS_FIS", 0.5), ("GAUSS_FIS", 2.0),
                                         ("BSPLINE3_FIS", 0.5)])
@pytest.mark.parametrize("mode, spp", [("STOCH", 8), ("AFTER", 1)])
def test_filter2d_gauss_fis_mips_rgba8(sf, orc, c2_small, filt, sigma, mode, spp):
    """MIP pyramid down to 1x1 levels: the FIS Gaussian's wide offsets wrap
    several times around the small levels."""
    _print_case("filter2d_gauss_mips", filt, sigma, mode, spp)
    lv, q = c2_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    qq = q.copy()
    qq[::7, 2] = len(lv) - 1.0                                 # some queries on the 1x1 level
    m = {"STOCH": orc.STOCHASTIC, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=17, sigma=sigma)
    taps_d = torch.empty((q.shape[0], spp, 3), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, torch.from_numpy(qq).cuda(), smp, shade=1, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, qq, getattr(orc, filt), m, spp=spp, seed=17, shade=1, taps=m == orc.STOCHASTIC,
                       sigma=sigma)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("filt, sigma", [("GAUSS_FIS", 0.5), ("BSPLINE3_FIS", 0.5), ("GAUSS_FRS", 0.5)])
def test_filter2d_gauss_fis_config2_full_sampled(sf, orc, c2_full, filt, sigma):
    _print_case("filter2d_gauss_c2_full", filt, sigma)
    lv, q = c2_full
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    smp = sf.sampling(getattr(sf, "SF_" + filt), sf.SF_STOCHASTIC, 16, seed=33, sigma=sigma)
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx()).cpu().numpy()
    sub = np.sort(np.random.default_rng(3).choice(q.shape[0], 3000, replace=False))
    ref = orc.filter2d(ot, q, getattr(orc, filt), orc.STOCHASTIC, spp=16, seed=33, shade=1, subset=sub,
                       sigma=sigma)
    _close(out[sub], ref)


# ------------------------------------------------------------------ split filtering
@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3", "KEYS3", "MITCHELL"])
@pytest.mark.parametrize("mip", [0, 1, 2])
@pytest.mark.parametrize("spp", [1, 8])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter2d_split(sf, orc, c2_small, filt, mip, spp, shade):
    """Split filtering: the level pick bit-exact, the reconstruction of
    that level before shading to the float tolerance."""
    _print_case("filter2d_split", filt, mip, spp, shade)
    lv, q = c2_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, mip)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=mip)
    f = getattr(orc, filt)
    smp = sf.sampling(f, sf.SF_SPLIT, spp, seed=8)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda")
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=shade, ggx_params=sf.ggx(), dbg_taps=taps_d)
    ref, taps = orc.filter2d(ot, q, f, orc.SPLIT, spp=spp, seed=8, shade=shade, taps=True)
    assert np.array_equal(taps_d.cpu().numpy(), taps)
    if filt in ("KEYS3", "MITCHELL"):
        _close_signed(out.cpu().numpy(), ref, np.nanmax(np.abs(ref)))
    else:
        _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("wrap", [0, 1])
def test_filter2d_split_single_level_is_before(sf, orc, c1, wrap):
    """One level: the split estimator returns the filter-before value."""
    _print_case("filter2d_split_single", wrap)
    tex, q = c1
    gt = sf.Texture2D([tex], wrap=wrap)
    qd = torch.from_numpy(q).cuda()
    for f in (sf.SF_LINEAR, sf.SF_BSPLINE3):
        a = sf.sf_filter2d(gt, qd, sf.sampling(f, sf.SF_SPLIT, 4, seed=2), shade=1, ggx_params=sf.ggx())
        b = sf.sf_filter2d(gt, qd, sf.sampling(f, sf.SF_BEFORE, 1), shade=1, ggx_params=sf.ggx())
        _close(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-6)


# ------------------------------------------------------------------ 2-D anisotropic minification
@pytest.fixture(scope="module")
def aniso_small(orc):
    size = 256
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(size, seed=3, waves=12)))
    q = inputs.plane_queries_aniso(160, 90)
    q[5, 2:] = 0.0                                 # zero footprint: level 0, no jitter
    q[6, 0] = np.inf                               # non-finite -> NaN
    q[7, 2:] = [3e-3, 0.0, 0.0, 1e-7]              # anisotropy far beyond the limit
    q[8, 2:] = [3e38, 0.0, 3e38, 0.0]              # jittered coordinates overflow -> NaN
    return lv, q


@pytest.mark.parametrize("filt, sigma", [("NEAREST", 0.5), ("LINEAR", 0.5), ("BSPLINE3", 0.5), ("GAUSS_FIS", 0.7)])
@pytest.mark.parametrize("mode, spp", [("STOCH", 8), ("STOCH", 1), ("BEFORE", 1), ("AFTER", 1)])
@pytest.mark.parametrize("amax", [64, 4])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter2d_aniso_parity(sf, orc, aniso_small, filt, sigma, mode, spp, amax, shade):
    if filt == "GAUSS_FIS" and mode != "STOCH":
        pytest.skip("the FIS Gaussian has no probe comparator")
    _print_case("filter2d_aniso", filt, mode, spp, amax, shade)
    lv, q = aniso_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=29, sigma=sigma)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, aniso_max=amax, shade=shade,
                               ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d_aniso(ot, q, getattr(orc, filt), m, spp=spp, seed=29, shade=shade, taps=m == orc.STOCHASTIC,
                             sigma=sigma, amax=amax)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3", "KEYS3", "MITCHELL"])
@pytest.mark.parametrize("spp", [1, 8])
@pytest.mark.parametrize("amax", [64, 4])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter2d_aniso_split(sf, orc, aniso_small, filt, spp, amax, shade):
    """Split filtering over the pixel: jitter and level bit-exact (taps hold
    the level), the level's reconstruction before shading to tolerance."""
    _print_case("filter2d_aniso_split", filt, spp, amax, shade)
    lv, q = aniso_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    f = getattr(orc, filt)
    smp = sf.sampling(f, sf.SF_SPLIT, spp, seed=12)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda")
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, aniso_max=amax, shade=shade,
                               ggx_params=sf.ggx(), dbg_taps=taps_d)
    ref, taps = orc.filter2d_aniso(ot, q, f, orc.SPLIT, spp=spp, seed=12, shade=shade, taps=True, amax=amax)
    assert np.array_equal(taps_d.cpu().numpy(), taps)
    if filt in ("KEYS3", "MITCHELL"):
        _close_signed(out.cpu().numpy(), ref, np.nanmax(np.abs(ref)))
    else:
        _close(out.cpu().numpy(), ref)


@pytest.fixture(scope="module")
def checker_full():
    _print_case("checker_full generate")
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_checker(4096, 64)))
    q = inputs.plane_queries_aniso(1920, 1080)
    return lv, q


@pytest.mark.parametrize("filt, mode, spp", [("BSPLINE3", "STOCH", 1), ("BSPLINE3", "STOCH", 16),
                                             ("LINEAR", "BEFORE", 1), ("LINEAR", "AFTER", 1)])
def test_filter2d_aniso_checker_full_sampled(sf, orc, checker_full, filt, mode, spp):
    _print_case("filter2d_aniso_checker_full", filt, mode, spp)
    lv, q = checker_full
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=41)
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx()).cpu().numpy()
    sub = np.sort(np.random.default_rng(4).choice(q.shape[0], 3000, replace=False))
    ref = orc.filter2d_aniso(ot, q, getattr(orc, filt), m, spp=spp, seed=41, shade=1, subset=sub)
    _close(out[sub], ref)


# ------------------------------------------------------------------ stochastic EWA
@pytest.mark.parametrize("mode, spp", [("STOCH", 8), ("STOCH", 1), ("BEFORE", 1), ("AFTER", 1)])
@pytest.mark.parametrize("amax", [16, 4, 1])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter2d_ewa_parity(sf, orc, aniso_small, mode, spp, amax, shade):
    """EWA on a 256^2 RGBA8 pyramid (zero, over-limit, non-finite and
    overflowing footprints included): picked texels bit-exact, values to
    the float tolerance."""
    _print_case("filter2d_ewa", mode, spp, amax, shade)
    lv, q = aniso_small
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, lv[0].shape[1], lv[0].shape[0], len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(sf.SF_EWA, m, spp, seed=31)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, aniso_max=amax, shade=shade,
                               ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d_aniso(ot, q, orc.EWA, m, spp=spp, seed=31, shade=shade, taps=m == orc.STOCHASTIC, amax=amax)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("mode, spp", [("STOCH", 4), ("AFTER", 1), ("BEFORE", 1)])
def test_filter2d_ewa_nonsquare_clamp(sf, orc, mode, spp):
    """A 256 x 32 float pyramid (aspect 8, one axis reaching 1 texel early),
    clamped addressing, footprints scaled up to wider than the texture."""
    _print_case("filter2d_ewa_nonsquare", mode, spp)
    lv = [x.astype(np.float32) for x in inputs.mip_chain(inputs.texture_sinusoids(256, seed=5, waves=9)[:32])]
    q = inputs.plane_queries_aniso(64, 40)
    q[:, 2:] *= np.float32(1.0) + np.arange(q.shape[0], dtype=np.float32)[:, None] % 7 * np.float32(3.0)
    q[:, :2] = q[:, :2] * np.float32(1.3) - np.float32(0.15)          # some coordinates outside [0, 1]
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 256, 32, len(lv), orc.RGBA32F, offs, orc.CLAMP, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_CLAMP, mip=sf.SF_MIP_LINEAR)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(sf.SF_EWA, m, spp, seed=7)
    taps_d = torch.full((q.shape[0], spp, 3), 99, dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, aniso_max=16, shade=1,
                               ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d_aniso(ot, q, orc.EWA, m, spp=spp, seed=7, shade=1, taps=m == orc.STOCHASTIC, amax=16)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.mark.parametrize("mode, spp", [("STOCH", 1), ("STOCH", 4), ("AFTER", 1)])
def test_filter2d_ewa_checker_full_sampled(sf, orc, checker_full, mode, spp):
    """1920 x 1080 pixels over the 4096^2 checkerboard at aniso_max 16, the
    launch the benchmark times; 3000 sampled pixels against the oracle."""
    _print_case("filter2d_ewa_checker_full", mode, spp)
    lv, q = checker_full
    buf, offs = inputs.pack_levels(lv)
    ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
    gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(sf.SF_EWA, m, spp, seed=43)
    out = sf.sf_filter2d_aniso(gt, torch.from_numpy(q).cuda(), smp, aniso_max=16, shade=1,
                               ggx_params=sf.ggx()).cpu().numpy()
    sub = np.sort(np.random.default_rng(5).choice(q.shape[0], 3000, replace=False))
    ref = orc.filter2d_aniso(ot, q, orc.EWA, m, spp=spp, seed=43, shade=1, subset=sub, amax=16)
    _close(out[sub], ref)


# ------------------------------------------------------------------ DCT-compressed textures, triplanar
@pytest.fixture(scope="module")
def dct_pair(orc, sf):
    """An RGBA8 pyramid whose sizes are not multiples of 8 (edge blocks),
    compressed by the oracle and by the GPU."""
    full = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(256, seed=9, waves=12)))
    lv = [np.ascontiguousarray(f[:max(1, 200 >> l), :max(1, 232 >> l)]) for l, f in enumerate(full[:8])]
    ot = orc.Tex2D.dct(lv, wrap=orc.REPEAT, mip=orc.MIP_LINEAR)
    gt = sf.Texture2D.dct(sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR))
    torch.cuda.synchronize()
    return lv, ot, gt


def test_dct_encoder_codes_bit_exact(sf, orc, dct_pair):
    """The GPU compressor's blocks and AC ranges equal the oracle's bit for bit."""
    _print_case("dct_encode")
    lv, ot, gt = dct_pair
    assert list(gt.offsets) == list(ot.off[:len(lv)])
    gbuf = gt.buffer.cpu().numpy()
    for l in range(len(lv)):
        hl, wl = lv[l].shape[:2]
        nbytes = 16 * (-(-wl // 8)) * (-(-hl // 8))
        o = gt.offsets[l]
        assert np.array_equal(gbuf[o:o + nbytes], ot.buf[o:o + nbytes]), l
    assert np.array_equal(gt.ranges.cpu().numpy(), ot.dct_range)


@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode, spp", [("STOCH", 4), ("BEFORE", 1), ("AFTER", 1)])
def test_dct_filtering_parity(sf, orc, dct_pair, filt, mode, spp):
    _print_case("dct_filter", filt, mode, spp)
    lv, ot, gt = dct_pair
    q = inputs.plane_queries(96, 64, tex_size=232, levels=len(lv))
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=13)
    taps_d = torch.empty((q.shape[0], spp, 3), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx(), dbg_taps=taps_d)
    res = orc.filter2d(ot, q, getattr(orc, filt), m, spp=spp, seed=13, shade=1, taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.fixture(scope="module")
def tri_small(orc, sf):
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(128, seed=10, waves=10)))
    q = inputs.sphere_queries(120, 80, tex_size=128, levels=len(lv))
    q[3, 0] = np.nan
    q[4, 3:6] = [1.0, 0.0, 0.0]                      # axis-aligned normal: one plane only
    q[5, 0] = 3e38                                   # projected coordinate overflows -> NaN
    buf, offs = inputs.pack_levels(lv)
    plain = (orc.Tex2D(buf, 128, 128, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR),
             sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR))
    dct = (orc.Tex2D.dct(lv, wrap=orc.REPEAT, mip=orc.MIP_LINEAR), sf.Texture2D.dct(plain[1]))
    return q, {"rgba8": plain, "dct": dct}


@pytest.mark.parametrize("texkind", ["rgba8", "dct"])
@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("plane_mode, mode, spp", [(1, "STOCH", 4), (1, "STOCH", 1), (1, "AFTER", 3), (1, "BEFORE", 2),
                                                   (0, "STOCH", 2), (0, "BEFORE", 1), (0, "AFTER", 1)])
def test_triplanar_parity(sf, orc, tri_small, texkind, filt, plane_mode, mode, spp):
    _print_case("triplanar", texkind, filt, plane_mode, mode, spp)
    q, texs = tri_small
    ot, gt = texs[texkind]
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, spp, seed=21)
    want_taps = plane_mode == 1
    taps_d = torch.empty((q.shape[0], spp, 4), dtype=torch.int32, device="cuda") if want_taps else None
    out = sf.sf_triplanar(gt, torch.from_numpy(q).cuda(), smp, 1.5, plane_mode, shade=1, ggx_params=sf.ggx(),
                          dbg_taps=taps_d)
    res = orc.triplanar(ot, q, 1.5, plane_mode, getattr(orc, filt), m, spp=spp, seed=21, shade=1, taps=want_taps)
    if want_taps:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


@pytest.fixture(scope="module")
def dct_full(orc, sf, c2_full):
    """The config-2 pyramid (4096^2 RGBA8, 13 levels) compressed by both sides."""
    _print_case("dct_full generate")
    lv, _ = c2_full
    ot = orc.Tex2D.dct(lv, wrap=orc.REPEAT, mip=orc.MIP_LINEAR)
    gt = sf.Texture2D.dct(sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR))
    torch.cuda.synchronize()
    return lv, ot, gt


def test_dct_config2_full_codes_bit_exact(sf, orc, dct_full):
    """Every block and range of the full 4096^2 pyramid equals the oracle's."""
    _print_case("dct_full_codes")
    lv, ot, gt = dct_full
    assert np.array_equal(gt.buffer.cpu().numpy()[:ot.buf.size], ot.buf)
    assert np.array_equal(gt.ranges.cpu().numpy(), ot.dct_range)


@pytest.mark.parametrize("filt, mode", [("LINEAR", "STOCH"), ("LINEAR", "BEFORE"), ("BSPLINE3", "STOCH"),
                                        ("BSPLINE3", "AFTER")])
def test_dct_plane_4k_sampled(sf, orc, dct_full, filt, mode):
    """The DCT pyramid seen by the 3840x2160 plane camera, in the launch the
    suite times: 3000 sampled queries against the oracle, stochastic taps
    bit-exact."""
    _print_case("dct_plane_4k", filt, mode)
    lv, ot, gt = dct_full
    q = inputs.plane_queries(3840, 2160, tex_size=4096, levels=len(lv))
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(getattr(sf, "SF_" + filt), m, 1, seed=5)
    stoch = m == orc.STOCHASTIC
    taps_d = torch.empty((q.shape[0], 1, 3), dtype=torch.int32, device="cuda") if stoch else None
    out = sf.sf_filter2d(gt, torch.from_numpy(q).cuda(), smp, shade=1, ggx_params=sf.ggx(), dbg_taps=taps_d)
    sub = np.sort(np.random.default_rng(8).choice(q.shape[0], 3000, replace=False))
    res = orc.filter2d(ot, q, getattr(orc, filt), m, spp=1, seed=5, shade=1, subset=sub, taps=stoch)
    if stoch:
        ref, taps = res
        assert np.array_equal(taps_d[torch.from_numpy(sub).cuda()].cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy()[sub], ref)


@pytest.mark.parametrize("texkind", ["rgba8", "dct"])
@pytest.mark.parametrize("plane_mode, mode", [(1, "STOCH"), (0, "STOCH"), (0, "BEFORE"), (1, "BEFORE")])
def test_triplanar_sphere_4k_sampled(sf, orc, c2_full, dct_full, texkind, plane_mode, mode):
    """Triplanar mapping of the config-2 pyramid (plain and DCT) on the
    3840x2160 sphere, in the launches the suite times: 3000 sampled hit
    pixels against the oracle, the one-plane pick's taps bit-exact."""
    _print_case("triplanar_4k", texkind, plane_mode, mode)
    lv, _ = c2_full
    if texkind == "dct":
        _, ot, gt = dct_full
    else:
        buf, offs = inputs.pack_levels(lv)
        ot = orc.Tex2D(buf, 4096, 4096, len(lv), orc.RGBA8, offs, orc.REPEAT, orc.MIP_LINEAR)
        gt = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    q = inputs.sphere_queries(3840, 2160, tex_size=4096, levels=len(lv))
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE}[mode]
    smp = sf.sampling(sf.SF_LINEAR, m, 1, seed=5)
    want_taps = plane_mode == 1 and m == orc.STOCHASTIC
    taps_d = torch.empty((q.shape[0], 1, 4), dtype=torch.int32, device="cuda") if want_taps else None
    out = sf.sf_triplanar(gt, torch.from_numpy(q).cuda(), smp, 1.0, plane_mode, shade=1, ggx_params=sf.ggx(),
                          dbg_taps=taps_d)
    sub = np.sort(np.random.default_rng(9).choice(q.shape[0], 3000, replace=False))
    res = orc.triplanar(ot, q, 1.0, plane_mode, orc.LINEAR, m, spp=1, seed=5, shade=1, subset=sub, taps=want_taps)
    if want_taps:
        ref, taps = res
        assert np.array_equal(taps_d[torch.from_numpy(sub).cuda()].cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy()[sub], ref)


# ------------------------------------------------------------------ 3-D points
@pytest.mark.parametrize("filt", ["NEAREST", "LINEAR", "BSPLINE3"])
@pytest.mark.parametrize("mode, spp, variant", [("STOCH", 4, 0), ("STOCH", 3, 1), ("BEFORE", 1, 0), ("AFTER", 1, 0)])
@pytest.mark.parametrize("shade", [0, 1])
def test_filter3d_small(sf, orc, small_cloud, filt, mode, spp, variant, shade):
    _print_case("filter3d", filt, mode, spp, variant, shade)
    og, vol = _grids(orc, sf, small_cloud)
    p = inputs.random_points(2999, -0.05, 1.05, seed=4)
    p[3] = [np.nan, 0.5, 0.5]
    f = getattr(orc, filt)
    m = {"STOCH": orc.STOCHASTIC, "BEFORE": orc.BEFORE, "AFTER": orc.AFTER}[mode]
    smp = sf.sampling(f, m, spp, seed=8, rng_variant=variant)
    taps_d = torch.empty((p.shape[0], spp, 3), dtype=torch.int32, device="cuda") if m == orc.STOCHASTIC else None
    out = sf.sf_filter3d(vol, torch.from_numpy(p).cuda(), smp, shade=shade, ds=0.05, dbg_taps=taps_d)
    res = orc.filter3d(og, p, f, m, spp=spp, seed=8, variant=variant, shade=shade, ds=0.05,
                       taps=m == orc.STOCHASTIC)
    if m == orc.STOCHASTIC:
        ref, taps = res
        assert np.array_equal(taps_d.cpu().numpy(), taps)
    else:
        ref = res
    _close(out.cpu().numpy(), ref)


# ------------------------------------------------------------------ reductions
def test_error_stats(sf):
    _print_case("error_stats")
    rng = np.random.default_rng(0)
    for n in (1, 1000, 300_001, 3_000_000):
        ref = rng.random(n) + 0.1
        est = (ref + 1e-3 * rng.normal(size=n)).astype(np.float32)
        if n > 3:
            est[:3] = np.nan
        out = sf.sf_error_stats(torch.from_numpy(est).cuda(), torch.from_numpy(ref).cuda()).cpu().numpy()
        e = est.astype(np.float64)
        fin = np.isfinite(e)
        d = e[fin] - ref[fin]
        assert out[4] == fin.sum() and out[6] == (~fin).sum()
        assert np.isclose(out[0], np.sum(d * d), rtol=1e-12)
        assert np.isclose(out[1], np.sum(d), rtol=1e-9, atol=1e-12)
        assert out[2] == np.max(np.abs(d))
        assert out[3] == np.max(np.abs(d) / np.abs(ref[fin]))
        assert np.isclose(out[5], np.sum(ref[fin] ** 2), rtol=1e-12)
        again = sf.sf_error_stats(torch.from_numpy(est).cuda(), torch.from_numpy(ref).cuda()).cpu().numpy()
        assert np.array_equal(out, again)
