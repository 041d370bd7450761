"""Benchmark of the stochastic-filtering hot path on one MI355X.

Workload (the paper's offline case, Sec. 5, on a synthetic stand-in for the
Disney Cloud): a 512^3 float16 fractal-noise density cloud (~30% exact
zeros, sigma in [0, 50], cube side 0.25), 256x256 pixels x 16 jittered
orthographic rays = 1,048,576 rays, 256 fixed ray-march steps, transmittance
with the stochastic tricubic (cubic B-spline) filter: one voxel per step.

One step of the benchmark = one sf_raymarch launch over all rays.  The
inputs are resident in HBM before timing starts.  ``value`` is shaded
density queries per second (one query = one ray step: a filtered density
lookup shaded by exp(-sigma*dt)).

Beside it the line reports (outside the timed region): the deterministic
64-tap tricubic exact-after and filter-before rates, the trilinear pair, the
equal-RMSE throughput ratio against the 64-tap exact-after path, the
roofline of the timed kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shaded queries/s: stochastic vs 64-tap tricubic at equal RMSE; HBM GB/s"
N_PIX, RAYS_PER_PIX, STEPS, SIDE, GRID = 256, 16, 256, 0.25, 512
HBM_PEAK_GBS = 8000.0
# Vector-ALU peak in tera lane-operations per second: the published binary32
# vector rate, 157.3 TFLOP/s = 256 CUs x 128 lanes x 2.4 GHz x 2 flops per
# fused multiply-add, i.e. two wave64 instructions per CU per cycle (simple
# binary32 and 32-bit integer operations on vector registers reach about
# that rate; the issue-rate probe of libsf_bench.so measures it).
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# One wave64 instruction per CU per cycle: the rate of conversions, compares,
# three-operand integer operations and instructions that read a scalar
# register (the probe's slower class).
VALU_ONE_ISSUE_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic HBM bytes of one ray of the stochastic march: one binary16
# voxel per step (256 x 2 B) plus the 32-byte ray record read and the 4-byte
# transmittance written.
BYTES_PER_RAY = STEPS * 2 + 32 + 4
BRICK_LOG2 = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_launches(fn, steps, warmup, torch):
    """Average duration of `fn` (one kernel launch on the current stream),
    timed with HIP events recorded on that stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def equal_rmse(sf, torch, vol, rays_d, t_stoch, t_det, seed, t_before=None):
    """Pixel-integral equal-RMSE protocol.

    Reference pixel value R_p = mean of the exact-after 64-tap transmittance
    over 16 independent sets of 16 stratified rays per pixel (256 rays); its
    own sampling variance, the variance of the 16 set means over 16, is
    subtracted.  Both 16-ray estimates are compared with R_p; the
    stochastic path needs spp* = 16 (RMSE_s/RMSE_d)^2 rays per pixel to match
    the deterministic path, so the throughput ratio at equal RMSE is
    (t_det / t_stoch) (RMSE_d / RMSE_s)^2.  The stochastic march is then run
    at ceil(spp*/16) sets of 16 rays per pixel, timed, and its RMSE checked.
    The 64-tap filter-before image (biased: the density is filtered before
    the exponential) is compared with the same reference beside it."""
    import numpy as np
    from paper_2407_06107_amd import inputs

    P = N_PIX * N_PIX
    after = sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1)
    stoch = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=seed)
    T_s = sf.sf_raymarch(vol, rays_d, STEPS, stoch).double().view(P, RAYS_PER_PIX).mean(1)
    T_d = sf.sf_raymarch(vol, rays_d, STEPS, after).double().view(P, RAYS_PER_PIX).mean(1)
    before = sf.sampling(sf.SF_BSPLINE3, sf.SF_BEFORE, 1)
    T_b = sf.sf_raymarch(vol, rays_d, STEPS, before).double().view(P, RAYS_PER_PIX).mean(1)
    # reference: 16 sets of 16 stratified rays per pixel (independent jitter);
    # the rays of one set are stratified, so the spread of the set means (not
    # of single rays) measures the reference's own error
    acc = torch.zeros(P, dtype=torch.float64, device="cuda")
    acc2 = torch.zeros(P, dtype=torch.float64, device="cuda")
    sets = 16
    for c in range(sets):
        r = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=1000 + c)
        M = sf.sf_raymarch(vol, torch.from_numpy(r).cuda(), STEPS, after).double().view(P, RAYS_PER_PIX).mean(1)
        acc += M
        acc2 += M * M
    m = sets * RAYS_PER_PIX
    R = acc / sets
    var_R = (acc2 / sets - R * R).clamp(min=0) / (sets - 1)
    bias_corr = float(var_R.mean())
    mse_s = float(((T_s - R) ** 2).mean()) - bias_corr
    mse_d = float(((T_d - R) ** 2).mean()) - bias_corr
    mse_b = float(((T_b - R) ** 2).mean()) - bias_corr
    rmse_s, rmse_d = math.sqrt(max(mse_s, 0.0)), math.sqrt(max(mse_d, 0.0))
    spp_star = RAYS_PER_PIX * (rmse_s / rmse_d) ** 2
    ratio = (t_det / t_stoch) * (rmse_d / rmse_s) ** 2
    # verification at spp*: the stochastic march over ceil(spp* / 16) x 16
    # jittered rays per pixel (new jitter), one launch, timed, and its RMSE
    # against the same reference
    chunks = max(1, math.ceil(spp_star / RAYS_PER_PIX))
    rv = np.concatenate([inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=2000 + c) for c in range(chunks)])
    rv_d = torch.from_numpy(rv).cuda()
    Tv = torch.empty(rv.shape[0], dtype=torch.float32, device="cuda")
    t_v = time_launches(lambda: sf.sf_raymarch(vol, rv_d, STEPS, stoch, T=Tv), 3, 1, torch)
    T_v = Tv.double().view(chunks, P, RAYS_PER_PIX).mean((0, 2))
    rmse_v = math.sqrt(max(float(((T_v - R) ** 2).mean()) - bias_corr, 0.0))
    del rv_d, Tv
    return {"rmse_stochastic_16": rmse_s, "rmse_det_after_16": rmse_d,
            "mse_increase": mse_s / mse_d - 1.0, "spp_star": spp_star, "ratio": ratio,
            "reference_rays_per_pixel": m, "reference_var_subtracted": bias_corr,
            "verified_at_spp_star": {"rays_per_pixel": chunks * RAYS_PER_PIX, "ms": t_v, "rmse": rmse_v,
                                     "rmse_at_most_det": rmse_v <= rmse_d,
                                     "ratio_measured": t_det / t_v},
            "det_before_16": {"rmse": math.sqrt(max(mse_b, 0.0)),
                              "ratio_at_equal_rmse": None if t_before is None else
                              (t_before / t_stoch) * max(mse_b, 0.0) / max(mse_s, 1e-30)}}


def cpu_baseline(grid_host, rays, seed, max_rays):
    """The oracle's stochastic tricubic ray march on the same rays (the first
    ``max_rays`` of the stream, in stream order), all host cores, as shaded
    queries/s."""
    import oracle
    og = oracle.Grid(grid_host, side=SIDE)
    m = min(max_rays, rays.shape[0])
    sub = np.arange(m, dtype=np.int64)
    oracle.raymarch(og, rays, 4, oracle.BSPLINE3, oracle.STOCHASTIC, seed=seed, subset=sub[:256])   # warm
    t0 = time.perf_counter()
    oracle.raymarch(og, rays, STEPS, oracle.BSPLINE3, oracle.STOCHASTIC, seed=seed, subset=sub)
    dt = time.perf_counter() - t0
    return {"value": m * STEPS / dt, "unit": "shaded queries/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {m} of the {rays.shape[0]} rays x {STEPS} steps, stochastic tricubic, "
                      f"{dt:.2f} s wall on {oracle.num_threads()} threads"}


def cpu_comparators(grid_host, rays, seed, nrays=4096):
    """The oracle's other C3 modes (64- and 8-tap filter-before and exact
    filter-after, stochastic trilinear) timed on ``nrays`` rays spread evenly
    over the same stream, all host cores, as shaded queries/s: context beside
    the GPU comparators, not a baseline."""
    import oracle
    og = oracle.Grid(grid_host, side=SIDE)
    sub = np.unique(np.linspace(0, rays.shape[0] - 1, min(nrays, rays.shape[0])).astype(np.int64))
    out = {}
    for name, filt, mode in (("tricubic_after_64tap", oracle.BSPLINE3, oracle.AFTER),
                             ("tricubic_before_64tap", oracle.BSPLINE3, oracle.BEFORE),
                             ("trilinear_after_8tap", oracle.LINEAR, oracle.AFTER),
                             ("trilinear_before_8tap", oracle.LINEAR, oracle.BEFORE),
                             ("trilinear_stochastic", oracle.LINEAR, oracle.STOCHASTIC)):
        t0 = time.perf_counter()
        oracle.raymarch(og, rays, STEPS, filt, mode, seed=seed, subset=sub)
        dt = time.perf_counter() - t0
        out[name] = {"queries_per_s": sub.size * STEPS / dt,
                     "sample": f"{sub.size} rays spread over the stream, {dt:.2f} s"}
    out["cores"] = oracle.num_threads()
    return out


PMC_PROFILE = os.path.join(ROOT, "profiles", "raymarch_stochastic_tricubic_512cloud_pmc.md")


def counters_from_profile(code_digest):
    """Per-launch hardware counters of the timed kernel read from the
    committed rocprofv3 summary (its machine-readable list): HBM bytes
    (FETCH_SIZE + WRITE_SIZE scaled by the plain-copy calibration) and the
    VALU / memory instruction counts.  Empty if the timed kernel's machine
    code differs from the code the counters were taken on."""
    if not os.path.exists(PMC_PROFILE) or code_digest is None:
        return {}
    fields = {}
    for line in open(PMC_PROFILE):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_code_sha256") != code_digest:
        return {}
    out = {}
    for k, v in fields.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def count_occupied_steps(torch, occ, rays_d):
    """Ray steps that the kernel marches (lookup point not in a brick known
    to be empty: those that gather a voxel), from the same raster positions
    evaluated with torch float32 operations and the kernel's lookup in the
    padded bit mask; a step on a brick boundary may round the other way, so
    the count is exact to a few parts per million."""
    words = occ.to(torch.int64) & 0xFFFFFFFF
    nb = GRID >> BRICK_LOG2
    sx = sy = nb + 1                   # rows of nb + 1 bits, planes of nb + 1 rows
    o, d, t0, t1 = rays_d[:, :3], rays_d[:, 3:6], rays_d[:, 6:7], rays_d[:, 7:8]
    hit = (rays_d[:, 7] > rays_d[:, 6])
    dt = (t1 - t0) / STEPS
    scale = GRID / SIDE
    E = torch.addcmul((o * scale - 0.5), t0, d * scale)
    G = dt * d * scale
    total = 0
    for k0 in range(0, STEPS, 32):
        kh = torch.arange(k0, min(STEPS, k0 + 32), device=rays_d.device, dtype=torch.float32) + 0.5
        p = E[:, None, :] + kh[None, :, None] * G[:, None, :]
        b = torch.div(torch.floor(p).to(torch.int64), 1 << BRICK_LOG2, rounding_mode="floor")
        idx = (b[..., 2] * sy + b[..., 1]) * sx + b[..., 0]
        inside = (idx >= 0) & ((idx >> 5) < words.numel())
        empty = torch.zeros_like(inside)
        ii = idx[inside]
        empty[inside] = ((words[ii >> 5] >> (ii & 31)) & 1).bool()
        total += int((~empty & hit[:, None]).sum())
    return total


def valu_issue_rates(torch, reps=5):
    """CU cycles per wave64 instruction of each case of the issue-rate probe
    (libsf_bench.so): 8 resident workgroups of 256 lanes per CU, HIP events
    over `reps` launches, at the nominal 2.4 GHz clock."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2407_06107_amd", "libsf_bench.so"))
    lib.sfb_valu_rate_name.restype = C.c_char_p
    lib.sfb_valu_rate_launch.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * 8
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    insts = lib.sfb_valu_rate_insts()
    rates = {}
    for w in range(lib.sfb_valu_rate_cases()):
        def launch():
            if lib.sfb_valu_rate_launch(w, C.c_void_p(out.data_ptr()), blocks, stream) != 0:
                raise RuntimeError("sfb_valu_rate_launch failed")
        ms = time_launches(launch, reps, 2, torch)
        name = lib.sfb_valu_rate_name(w).decode()
        per = 2 if name.endswith("(pairs)") else 1
        rates[name] = ms * 1e-3 * 2.4e9 / (32 * insts * per)
    return rates


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Streaming rate the chip reaches on a plain device-to-device copy of
    nbytes (torch's copy), in GB/s of bytes read plus written."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del src, dst
    return 2 * nbytes / t / 1e9


def gather_twin(torch, vol_occ, grid, rays_d, T):
    """A launch of the benchmark-only gather twin (libsf_bench.so) on the
    same rays, grid and occupancy mask as the timed kernel, on torch's
    current stream."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2407_06107_amd", "libsf_bench.so"))
    lib.sfb_gather_twin.restype = C.c_int
    lib.sfb_gather_twin.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                    C.c_void_p]
    nz, ny, nx = grid.shape
    wmin = (C.c_float * 3)(0.0, 0.0, 0.0)
    scale = (C.c_float * 3)(nx / SIDE, ny / SIDE, nz / SIDE)
    occ = vol_occ.occupancy

    def launch():
        st = lib.sfb_gather_twin(C.c_void_p(grid.data_ptr()), nx, ny, nz, wmin, scale, C.c_void_p(occ.data_ptr()),
                                 BRICK_LOG2, C.c_void_p(rays_d.data_ptr()), rays_d.shape[0], STEPS,
                                 C.c_void_p(T.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
        if st != 0:
            raise RuntimeError(f"sfb_gather_twin failed: {st}")
    return launch


# The timed kernel: stochastic cubic B-spline, binary16 grid, independent
# uniforms, no tap dump, occupancy mask, power-of-two addressing.
TIMED_KERNEL = "_ZN3sfk11k_ray_stochILi2ELb1ELi0ELb0ELb1ELb1EEEvNS_12RaymarchCallEj"


def kernel_code_digest(lib_path=None, name=TIMED_KERNEL):
    """SHA-256 of a kernel's machine code in the built library: the bytes of
    its function in the gfx950 code objects of libsf.so's offload bundles,
    then its kernel descriptor with the code-entry offset (bytes 16..23,
    which moves with the layout of other code) zeroed.  None if not found."""
    import hashlib
    import struct
    if lib_path is None:
        lib_path = os.path.join(ROOT, "paper_2407_06107_amd", "libsf.so")
    if not os.path.exists(lib_path):
        return None
    data = open(lib_path, "rb").read()
    i = 0
    while True:
        i = data.find(b"__CLANG_OFFLOAD_BUNDLE__", i)
        if i < 0:
            return None
        nent = struct.unpack_from("<Q", data, i + 24)[0]
        off = i + 32
        for _ in range(nent):
            eo, es, tl = struct.unpack_from("<QQQ", data, off)
            triple = data[off + 24:off + 24 + tl].decode()
            off += 24 + tl
            if "amdgcn" not in triple or not es:
                continue
            elf = data[i + eo:i + eo + es]
            shoff = struct.unpack_from("<Q", elf, 0x28)[0]
            shentsize, shnum = struct.unpack_from("<HH", elf, 0x3A)
            secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + k * shentsize) for k in range(shnum)]
            symtabs = [sec for sec in secs if sec[1] == 2]       # SHT_SYMTAB
            if not symtabs:
                continue
            st = symtabs[0]
            strtab = secs[st[6]]
            syms = {}
            for k in range(st[5] // 24):
                nm, _, _, shndx, val, size = struct.unpack_from("<IBBHQQ", elf, st[4] + 24 * k)
                o = strtab[4] + nm
                syms[elf[o:elf.index(b"\0", o)].decode()] = (shndx, val, size)
            if name not in syms or name + ".kd" not in syms:
                continue
            h = hashlib.sha256()
            for sym, zero in ((name, None), (name + ".kd", (16, 24))):
                shndx, val, size = syms[sym]
                sec = secs[shndx]
                start = sec[4] + (val - sec[3])
                blob = bytearray(elf[start:start + size])
                if zero:
                    blob[zero[0]:zero[1]] = bytes(zero[1] - zero[0])
                h.update(blob)
            return h.hexdigest()
        i += 24


# ---------------------------------------------------------------- neural (configs 4 and 5)
MLP_FLOP = {(8, 4): 2 * (8 * 64 + 64 * 64 + 64 * 4), (16, 1): 2 * (16 * 64 + 64 * 64 + 64)}
MFMA_BF16_PEAK_TFLOPS = 2500.0


def _init_mlp(rng, C, O):
    """He-normal weights, zero biases, packed W1 b1 W2 b2 W3 b3."""
    parts = []
    for fan_in, fan_out in ((C, 64), (64, 64), (64, O)):
        parts.append(rng.normal(size=fan_in * fan_out) * math.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def _train(sf, torch, latents, params, targets, C, O, epochs, batch, lr_lat, lr_mlp, seed, compute=None,
           cosine=False):
    """Epochs of shuffled mini-batches through sf_neural_train_step; returns
    (state, first and last epoch losses, milliseconds).  cosine: both
    learning rates follow a cosine from their start value down to 1% of it
    over the epochs (a latent is updated once per epoch, so Adam's step on it
    stays near lr x m / sqrt(v), about 4 lr, until the rate decays)."""
    st = sf.TrainState(latents, params, C, O, compute=sf.SF_TRAIN_BF16 if compute is None else compute)
    n = st.n_lattice
    gen = torch.Generator(device="cuda").manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    first = last = None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen).to(torch.int32)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = 0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            f = max(0.01, 0.5 * (1.0 + math.cos(math.pi * ep / epochs))) if cosine else 1.0
            sf.sf_neural_train_step(st, idx, targets, lr_lat * f, lr_mlp * f, loss_out=loss)
            acc += loss.double()
            nb += 1
        if ep == 0:
            first = float(acc) / nb
        last = acc / nb
    e1.record()
    torch.cuda.synchronize()
    return st, first, float(last), e0.elapsed_time(e1)


def _rmse(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2)))


def aniso_bench(res):
    """Config 2, anisotropic: 4096^2 RGBA8 pyramids under a 1920x1080 plane
    camera, footprint-driven levels; jittered minification, hardware-style
    probes and EWA, against the pixel-integral reference.  Two surfaces: the
    checkerboard shaded as a GGX material, and a bump normal map shaded with
    its texel normals (filtering before shading averages the normals)."""
    import torch
    import oracle
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    g = sf.ggx()
    rng = np.random.default_rng(9)
    qa = inputs.plane_queries_aniso(1920, 1080)
    na = qa.shape[0]
    qad = torch.from_numpy(qa).cuda()
    suba = np.sort(rng.choice(na, 2000, replace=False))
    rows = (("aniso_bicubic_stochastic_1spp", sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, 64),
            ("aniso_bicubic_stochastic_16spp", sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 16, 64),
            ("aniso_bilinear_stochastic_1spp", sf.SF_LINEAR, sf.SF_STOCHASTIC, 1, 64),
            ("aniso_gauss_fis_stochastic_16spp", sf.SF_GAUSS_FIS, sf.SF_STOCHASTIC, 16, 64),
            ("aniso_bicubic_split_1spp", sf.SF_BSPLINE3, sf.SF_SPLIT, 1, 64),
            ("aniso_bicubic_split_16spp", sf.SF_BSPLINE3, sf.SF_SPLIT, 16, 64),
            ("aniso16_trilinear_probes_before", sf.SF_LINEAR, sf.SF_BEFORE, 1, 16),
            ("aniso64_trilinear_probes_before", sf.SF_LINEAR, sf.SF_BEFORE, 1, 64),
            ("aniso64_trilinear_probes_after", sf.SF_LINEAR, sf.SF_AFTER_EXACT, 1, 64),
            ("ewa16_after", sf.SF_EWA, sf.SF_AFTER_EXACT, 1, 16),
            ("ewa16_before", sf.SF_EWA, sf.SF_BEFORE, 1, 16),
            ("ewa16_stochastic_1spp", sf.SF_EWA, sf.SF_STOCHASTIC, 1, 16),
            ("ewa16_stochastic_16spp", sf.SF_EWA, sf.SF_STOCHASTIC, 16, 16))
    for key, label, levels, shade in (
            ("config2_aniso", "checkerboard", lambda: inputs.texture_checker(4096, 64), sf.SF_SHADE_GGX),
            ("config2_aniso_normal_map", "bump normal map",
             lambda: inputs.texture_normal_map(4096, seed=13, slope=3.0), sf.SF_SHADE_GGX_NORMAL)):
        log(f"config 2 anisotropic: {label}")
        lv = inputs.quantize_unorm8(inputs.mip_chain(levels()))
        qi = inputs.plane_queries(1920, 1080, tex_size=4096, levels=len(lv))
        tex = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
        qid = torch.from_numpy(qi).cuda()
        buf, off = inputs.pack_levels(lv)
        ot0 = oracle.Tex2D(buf, 4096, 4096, 1, oracle.RGBA8, off[:1], oracle.REPEAT, oracle.MIP_NONE)
        t0 = time.perf_counter()
        ref_a = oracle.aniso_reference(ot0, qa, K=16, filt=oracle.BSPLINE3, shade=shade, subset=suba)
        dt_ref = time.perf_counter() - t0
        ca = {"queries": na, "texture": label,
              "reference": f"pixel integral, 16x16 midpoints x bicubic filter-after on level 0, "
                           f"{suba.size} pixels ({dt_ref:.1f} s on the CPU)",
              "reference_rms": float(np.sqrt(np.mean(ref_a ** 2)))}
        for name, filt, mode, spp, amax in rows:
            smp = sf.sampling(filt, mode, spp, seed=5, sigma=0.5)
            o = torch.empty((na, 3), dtype=torch.float32, device="cuda")
            t = time_launches(lambda: sf.sf_filter2d_aniso(tex, qad, smp, amax, shade, g, out=o), 10, 3, torch)
            ca[name] = {"ms": t, "queries_per_s": na / (t * 1e-3),
                        "rmse_vs_pixel_reference": _rmse(o.cpu().numpy()[suba], ref_a)}
            if name == "ewa16_after":
                ewa_after = o.cpu().numpy()
            elif filt == sf.SF_EWA:
                ca[name]["rmse_vs_ewa_after"] = _rmse(o.cpu().numpy(), ewa_after)
        smp = sf.sampling(sf.SF_LINEAR, sf.SF_BEFORE, 1)
        o = torch.empty((na, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(tex, qid, smp, shade, g, out=o), 10, 3, torch)
        ca["isotropic_trilinear_before"] = {"ms": t, "queries_per_s": na / (t * 1e-3),
                                            "rmse_vs_pixel_reference": _rmse(o.cpu().numpy()[suba], ref_a)}
        res[key] = ca


def planck_bench(res):
    """Emission: the 512^3 cloud as a fire of temperatures (0 K where the
    density is 0, else 800-6000 K), 1 Mi orthographic rays x 256 steps,
    black-body emission at 700 / 546.1 / 435.8 nm, occupancy mask.  Filtering
    the temperatures before Planck's law against filtering the emission
    after it, and the stochastic filter's one voxel per step."""
    import torch
    import oracle
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    log("emission: temperature grid and rays")
    dens = inputs.cloud_grid(GRID, seed=4, device="cuda")
    temp = inputs.temperature_grid(dens)
    del dens
    rays = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=11)
    rd = torch.from_numpy(rays).cuda()
    n = rays.shape[0]
    vol = sf.Volume(temp, side=SIDE, brick_log2=BRICK_LOG2)
    L = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    ce = {"rays": n, "steps": STEPS, "wavelengths_nm": list(sf.PLANCK_NM)}
    outs = {}
    for name, filt, mode in (("tricubic_stochastic", sf.SF_BSPLINE3, sf.SF_STOCHASTIC),
                             ("trilinear_stochastic", sf.SF_LINEAR, sf.SF_STOCHASTIC),
                             ("tricubic_after_64tap", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT),
                             ("tricubic_before_64tap", sf.SF_BSPLINE3, sf.SF_BEFORE),
                             ("trilinear_after_8tap", sf.SF_LINEAR, sf.SF_AFTER_EXACT),
                             ("trilinear_before_8tap", sf.SF_LINEAR, sf.SF_BEFORE)):
        smp = sf.sampling(filt, mode, 1, seed=7)
        t = time_launches(lambda: sf.sf_raymarch_emission(vol, rd, STEPS, smp, L=L), 5, 2, torch)
        outs[name] = L.double().cpu().numpy().copy()
        ce[name] = {"ms": t, "ray_steps_per_s": n * STEPS / (t * 1e-3)}
    # pixel values (16 rays per pixel) against the tricubic filter-after pixel values
    P = N_PIX * N_PIX
    ref = outs["tricubic_after_64tap"].reshape(P, RAYS_PER_PIX, 3).mean(1)
    scale = np.sqrt(np.mean(ref ** 2, axis=0))
    for name, v in outs.items():
        pix = v.reshape(P, RAYS_PER_PIX, 3).mean(1)
        ce[name]["relative_rmse_vs_tricubic_after"] = [float(x) for x in
                                                       np.sqrt(np.mean((pix - ref) ** 2, axis=0)) / scale]
    ce["note"] = ("relative_rmse_vs_tricubic_after: RMSE over 65,536 pixels (16 rays each) per wavelength, "
                  "divided by the RMS of the reference pixels; the before rows' error is the bias of filtering "
                  "temperatures before the nonlinear shading, the stochastic rows' is variance")
    ce["speedup_stochastic_vs_after"] = ce["tricubic_after_64tap"]["ms"] / ce["tricubic_stochastic"]["ms"]
    res["emission"] = ce

    # ---- minification: 64x64 pixels over the cube (about 10 voxels per pixel)
    log("emission: minification")
    MP, M_REF = 64, 1024
    pw = inputs.ortho_pixel_width(MP, SIDE)
    sigma = 0.5 * pw                       # Gaussian pixel filter, half a pixel
    centre_h = inputs.ortho_rays(MP, 1, side=SIDE, seed=12, strata=0)
    centre = torch.from_numpy(centre_h).cuda()
    nm = centre.shape[0]
    # reference: the Gaussian pixel filter of the exact tricubic filter-after emission on level 0,
    # by M_REF whole rays per pixel offset from the centre ray (same segment and steps, so only the
    # footprint is integrated); their sampling variance is measured and subtracted
    after = sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1)
    acc = torch.zeros((nm, 3), dtype=torch.float64, device="cuda")
    acc2 = torch.zeros((nm, 3), dtype=torch.float64, device="cuda")
    chunk = 256
    for c0 in range(0, M_REF, chunk):
        r = torch.from_numpy(inputs.offset_rays(centre_h, sigma, chunk, seed=100 + c0)).cuda()
        v = sf.sf_raymarch_emission(vol, r, STEPS, after).double().view(nm, chunk, 3)
        acc += v.sum(1)
        acc2 += (v * v).sum(1)
    R = acc / M_REF
    var_R = ((acc2 / M_REF - R * R).clamp(min=0) / (M_REF - 1)).mean(0)
    Rn = R.cpu().numpy()
    scale_m = np.sqrt(np.mean(Rn ** 2, axis=0))
    cm = {"pixels": nm, "voxels_per_pixel": pw * GRID / SIDE, "footprint_sigma_world": sigma,
          "reference": f"Gaussian pixel filter (sigma = 1/2 pixel) of the tricubic filter-after emission on the "
                       f"512^3 level, {M_REF} rays per pixel offset from the centre ray"}
    Lm = torch.empty((nm, 3), dtype=torch.float32, device="cuda")

    def rel_rmse(out):
        mse = np.mean((out.double().cpu().numpy() - Rn) ** 2, axis=0) - var_R.cpu().numpy()
        return [float(x) for x in np.sqrt(np.maximum(mse, 0.0)) / scale_m]

    for lvl in (3, 2):
        coarse = inputs.volume_level(temp, lvl)
        vc = sf.Volume(coarse, side=SIDE, brick_log2=BRICK_LOG2)
        for fname, filt in (("tricubic", sf.SF_BSPLINE3), ("trilinear", sf.SF_LINEAR)):
            smp = sf.sampling(filt, sf.SF_BEFORE, 1)
            t = time_launches(lambda: sf.sf_raymarch_emission(vc, centre, STEPS, smp, L=Lm), 10, 3, torch)
            cm[f"prefiltered_level{lvl}_{fname}_before"] = {"ms": t, "relative_rmse": rel_rmse(Lm)}
        del vc, coarse
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1)
    t = time_launches(lambda: sf.sf_raymarch_emission(vol, centre, STEPS, smp, L=Lm), 5, 2, torch)
    cm["level0_tricubic_after_point_sampled"] = {"ms": t, "relative_rmse": rel_rmse(Lm)}
    for spp in (1, 4, 16, 64):
        smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, spp, seed=31)
        t = time_launches(lambda: sf.sf_raymarch_emission(vol, centre, STEPS, smp, footprint=sigma, L=Lm), 10, 3,
                          torch)
        cm[f"stochastic_gaussian_footprint_{spp}spp"] = {"ms": t, "relative_rmse": rel_rmse(Lm)}
    cm["note"] = ("relative_rmse: per wavelength (700 / 546.1 / 435.8 nm), pixel RMSE against the reference over "
                  "the RMS of the reference, reference sampling variance subtracted; prefiltered rows march a "
                  "box-averaged temperature level (filter before shading), the stochastic rows sample the "
                  "Gaussian footprint on level 0 one voxel per step (filter after shading)")
    res["emission_minification"] = cm


def texture_bench(args, res):
    """Configs 1 and 2: the 2-D path (magnification of a 64^2 RGBA32F texture;
    a 4096^2 RGBA8 pyramid seen by a 1920x1080 camera), GGX + Lambert."""
    import torch
    import oracle
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    g = sf.ggx()
    rng = np.random.default_rng(8)
    # ---- config 1
    log("config 1")
    src = inputs.texture_uniform(64, seed=1)
    q1 = inputs.queries_uniform(4096, seed=2)
    tex1 = sf.Texture2D([src])
    qd1 = torch.from_numpy(q1).cuda()
    ref1 = oracle.filter2d(oracle.Tex2D.rgba32f(src), q1, oracle.BSPLINE3, oracle.AFTER, shade=1)
    c1 = {"queries": 4096}
    for name, filt, mode, spp in (("bicubic_stochastic_16spp", sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 16),
                                  ("bilinear_stochastic_16spp", sf.SF_LINEAR, sf.SF_STOCHASTIC, 16),
                                  ("bicubic_after_16tap", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1),
                                  ("bicubic_before_16tap", sf.SF_BSPLINE3, sf.SF_BEFORE, 1)):
        smp = sf.sampling(filt, mode, spp, seed=5)
        o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
        c1[name] = {"ms": t, "queries_per_s": 4096 / (t * 1e-3)}
        if filt == sf.SF_BSPLINE3:
            c1[name]["rmse_vs_oracle_bicubic_after"] = _rmse(o.cpu().numpy(), ref1)
    # the 64 KiB texture staged in LDS by each workgroup (the stochastic
    # kernel's default for textures up to 64 KiB when each workgroup has one
    # tile of lookups) against texel reads from global memory
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 16, seed=5)
    o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
    lds = {}
    for key, flag in (("lds_ms", "0"), ("global_ms", "1")):
        os.environ["SF_NO_LDS_TEXTURE"] = flag
        lds[key] = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
    os.environ.pop("SF_NO_LDS_TEXTURE", None)
    c1["bicubic_stochastic_16spp_texture_in_lds_vs_global"] = lds
    # interpolating Keys cubic: positivised stochastic (two taps per sample) vs all 16 taps
    ref1k = oracle.filter2d(oracle.Tex2D.rgba32f(src), q1, oracle.KEYS3, oracle.AFTER, shade=1)
    for name, mode, spp in (("keys_positivised_stochastic_16spp", sf.SF_STOCHASTIC, 16),
                            ("keys_positivised_stochastic_1spp", sf.SF_STOCHASTIC, 1),
                            ("keys_after_16tap", sf.SF_AFTER_EXACT, 1)):
        smp = sf.sampling(sf.SF_KEYS3, mode, spp, seed=5)
        o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
        c1[name] = {"ms": t, "queries_per_s": 4096 / (t * 1e-3),
                    "rmse_vs_oracle_keys_after": _rmse(o.cpu().numpy(), ref1k)}
    # Mitchell-Netravali cubic (B = C = 1/3): positivised by per-tap sign vs all 16 taps
    ref1m = oracle.filter2d(oracle.Tex2D.rgba32f(src), q1, oracle.MITCHELL, oracle.AFTER, shade=1)
    for name, mode, spp in (("mitchell_positivised_stochastic_16spp", sf.SF_STOCHASTIC, 16),
                            ("mitchell_positivised_stochastic_1spp", sf.SF_STOCHASTIC, 1),
                            ("mitchell_after_16tap", sf.SF_AFTER_EXACT, 1)):
        smp = sf.sampling(sf.SF_MITCHELL, mode, spp, seed=5)
        o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
        c1[name] = {"ms": t, "queries_per_s": 4096 / (t * 1e-3),
                    "rmse_vs_oracle_mitchell_after": _rmse(o.cpu().numpy(), ref1m)}
    # Gaussian by FRS (4x4 window) and by FIS (Box-Muller + nearest), and the
    # cubic B-spline by FIS (sum of three uniforms): RMSE against each
    # filter's own exact filter-after value, 16 samples per query
    for sigma in (0.3, 0.5, 0.8):
        for fname, filt, ofilt in (("gauss_frs", sf.SF_GAUSS_FRS, oracle.GAUSS_FRS),
                                   ("gauss_fis", sf.SF_GAUSS_FIS, oracle.GAUSS_FIS)):
            ref_after = oracle.filter2d(oracle.Tex2D.rgba32f(src), q1, ofilt, oracle.AFTER, shade=1, sigma=sigma)
            smp = sf.sampling(filt, sf.SF_STOCHASTIC, 16, seed=5, sigma=sigma)
            o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
            t = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
            c1[f"{fname}_sigma{sigma}_stochastic_16spp"] = {"ms": t, "rmse_vs_oracle_own_after": _rmse(o.cpu().numpy(),
                                                                                                    ref_after)}
    smp = sf.sampling(sf.SF_BSPLINE3_FIS, sf.SF_STOCHASTIC, 16, seed=5)
    o = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
    t = time_launches(lambda: sf.sf_filter2d(tex1, qd1, smp, sf.SF_SHADE_GGX, g, out=o), 50, 5, torch)
    c1["bicubic_fis_stochastic_16spp"] = {"ms": t, "rmse_vs_oracle_bicubic_after": _rmse(o.cpu().numpy(), ref1)}
    res["config1"] = c1
    # ---- config 2
    log("config 2: pyramid and camera")
    lv = inputs.quantize_unorm8(inputs.mip_chain(inputs.texture_sinusoids(4096, seed=3)))
    q2 = inputs.plane_queries(1920, 1080, tex_size=4096, levels=len(lv))
    n2 = q2.shape[0]
    tex2 = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    tex2n = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_NEAREST)
    qd2 = torch.from_numpy(q2).cuda()
    buf, offs = inputs.pack_levels(lv)
    otex = oracle.Tex2D(buf, 4096, 4096, len(lv), oracle.RGBA8, offs, oracle.REPEAT, oracle.MIP_LINEAR)
    sub = np.sort(rng.choice(n2, 20000, replace=False))
    ref2 = oracle.filter2d(otex, q2, oracle.BSPLINE3, oracle.AFTER, shade=1, subset=sub)
    ref2k = oracle.filter2d(otex, q2, oracle.KEYS3, oracle.AFTER, shade=1, subset=sub)
    ref2m = oracle.filter2d(otex, q2, oracle.MITCHELL, oracle.AFTER, shade=1, subset=sub)
    c2 = {"queries": n2, "texture_bytes": int(buf.size)}
    for name, tex, filt, mode, spp in (
            ("bicubic_stochastic_1spp", tex2, sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1),
            ("bicubic_stochastic_16spp", tex2, sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 16),
            ("bicubic_after_2x16tap", tex2, sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1),
            ("bicubic_before_2x16tap", tex2, sf.SF_BSPLINE3, sf.SF_BEFORE, 1),
            ("trilinear_stochastic_1spp", tex2, sf.SF_LINEAR, sf.SF_STOCHASTIC, 1),
            ("trilinear_before_2x4tap", tex2, sf.SF_LINEAR, sf.SF_BEFORE, 1),
            ("bilinear_nearest_level_before_4tap", tex2n, sf.SF_LINEAR, sf.SF_BEFORE, 1),
            ("keys_positivised_stochastic_1spp", tex2, sf.SF_KEYS3, sf.SF_STOCHASTIC, 1),
            ("keys_after_2x16tap", tex2, sf.SF_KEYS3, sf.SF_AFTER_EXACT, 1),
            ("mitchell_positivised_stochastic_1spp", tex2, sf.SF_MITCHELL, sf.SF_STOCHASTIC, 1),
            ("mitchell_after_2x16tap", tex2, sf.SF_MITCHELL, sf.SF_AFTER_EXACT, 1),
            ("bicubic_split_1spp", tex2, sf.SF_BSPLINE3, sf.SF_SPLIT, 1),
            ("bicubic_fis_stochastic_1spp", tex2, sf.SF_BSPLINE3_FIS, sf.SF_STOCHASTIC, 1),
            ("bicubic_fis_stochastic_16spp", tex2, sf.SF_BSPLINE3_FIS, sf.SF_STOCHASTIC, 16),
            ("gauss_frs_sigma0.5_stochastic_1spp", tex2, sf.SF_GAUSS_FRS, sf.SF_STOCHASTIC, 1),
            ("gauss_fis_sigma0.5_stochastic_1spp", tex2, sf.SF_GAUSS_FIS, sf.SF_STOCHASTIC, 1)):
        smp = sf.sampling(filt, mode, spp, seed=5, sigma=0.5)
        o = torch.empty((n2, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(tex, qd2, smp, sf.SF_SHADE_GGX, g, out=o), 10, 3, torch)
        cubic = filt in (sf.SF_BSPLINE3, sf.SF_KEYS3, sf.SF_GAUSS_FRS, sf.SF_BSPLINE3_FIS, sf.SF_MITCHELL)
        positivised = filt in (sf.SF_KEYS3, sf.SF_MITCHELL)
        if mode == sf.SF_STOCHASTIC:
            taps = spp * (2 if positivised else 1)
        elif mode == sf.SF_SPLIT:
            taps = spp * (16 if cubic else 4)
        else:
            taps = (2 if tex is tex2 else 1) * (16 if cubic else 4)
        algo = n2 * (taps * 4 + 12 + 12)
        c2[name] = {"ms": t, "queries_per_s": n2 / (t * 1e-3), "texel_reads_per_query": taps,
                    "algorithmic_gbs": algo / (t * 1e-3) / 1e9,
                    "rmse_vs_oracle_bicubic_trilinear_after": _rmse(o.cpu().numpy()[sub], ref2)}
        if filt == sf.SF_KEYS3:
            c2[name]["rmse_vs_oracle_keys_trilinear_after"] = _rmse(o.cpu().numpy()[sub], ref2k)
        if filt == sf.SF_MITCHELL:
            c2[name]["rmse_vs_oracle_mitchell_trilinear_after"] = _rmse(o.cpu().numpy()[sub], ref2m)
    t0 = time.perf_counter()
    oracle.filter2d(otex, q2, oracle.BSPLINE3, oracle.STOCHASTIC, spp=16, seed=5, shade=1, subset=sub)
    dt = time.perf_counter() - t0
    c2["cpu_oracle_bicubic_stochastic_16spp"] = {"queries_per_s": sub.size / dt, "cores": oracle.num_threads(),
                                                 "sample": f"{sub.size} queries, {dt:.2f} s"}
    res["config2"] = c2
    qd2b = qd2
    del tex2, tex2n
    aniso_bench(res)
    # ---- DCT-compressed pyramid (the config 2 texture) and triplanar mapping
    log("DCT texture and triplanar mapping")
    src8 = sf.Texture2D(lv, wrap=sf.SF_WRAP_REPEAT, mip=sf.SF_MIP_LINEAR)
    texd = sf.Texture2D.dct(src8)
    t_enc = time_launches(lambda: sf.Texture2D.dct(src8), 3, 1, torch)
    otd = oracle.Tex2D.dct(lv, wrap=oracle.REPEAT, mip=oracle.MIP_LINEAR)
    cd = {"compressed_bytes": int(texd.buffer.numel()), "rgba8_bytes": int(buf.size), "encode_ms": t_enc,
          "codes_equal_oracle": bool(np.array_equal(texd.buffer.cpu().numpy()[:otd.buf.size], otd.buf))}
    refd = oracle.filter2d(otd, q2, oracle.LINEAR, oracle.BEFORE, shade=1, subset=sub)
    for name, filt, mode in (("dct_trilinear_before_8decodes", sf.SF_LINEAR, sf.SF_BEFORE),
                             ("dct_trilinear_stochastic_1spp", sf.SF_LINEAR, sf.SF_STOCHASTIC),
                             ("dct_bicubic_after_32decodes", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT),
                             ("dct_bicubic_stochastic_1spp", sf.SF_BSPLINE3, sf.SF_STOCHASTIC)):
        smp = sf.sampling(filt, mode, 1, seed=5)
        o = torch.empty((n2, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: sf.sf_filter2d(texd, qd2b, smp, sf.SF_SHADE_GGX, g, out=o), 10, 3, torch)
        cd[name] = {"ms": t, "queries_per_s": n2 / (t * 1e-3),
                    "rmse_vs_oracle_dct_trilinear_before": _rmse(o.cpu().numpy()[sub], refd)}
    cd["stochastic_trilinear_speedup"] = (cd["dct_trilinear_before_8decodes"]["ms"] /
                                          cd["dct_trilinear_stochastic_1spp"]["ms"])
    # the paper measures these speedups at 4K: the plane and the sphere again at 3840 x 2160
    for wx, hy in ((1920, 1080), (3840, 2160)):
        key = f"{wx}x{hy}"
        if (wx, hy) != (1920, 1080):
            qp = inputs.plane_queries(wx, hy, tex_size=4096, levels=len(lv))
            qpd = torch.from_numpy(qp).cuda()
            npq = qp.shape[0]
            subp = np.sort(rng.choice(npq, 5000, replace=False))
            refp = oracle.filter2d(otd, qp, oracle.LINEAR, oracle.BEFORE, shade=1, subset=subp)
            cp = {"queries": npq}
            for name, filt, mode in (("dct_trilinear_before_8decodes", sf.SF_LINEAR, sf.SF_BEFORE),
                                     ("dct_trilinear_stochastic_1spp", sf.SF_LINEAR, sf.SF_STOCHASTIC)):
                smp = sf.sampling(filt, mode, 1, seed=5)
                o = torch.empty((npq, 3), dtype=torch.float32, device="cuda")
                t = time_launches(lambda: sf.sf_filter2d(texd, qpd, smp, sf.SF_SHADE_GGX, g, out=o), 10, 3, torch)
                cp[name] = {"ms": t, "queries_per_s": npq / (t * 1e-3),
                            "rmse_vs_oracle_dct_trilinear_before": _rmse(o.cpu().numpy()[subp], refp)}
            cp["stochastic_trilinear_speedup"] = (cp["dct_trilinear_before_8decodes"]["ms"] /
                                                  cp["dct_trilinear_stochastic_1spp"]["ms"])
            cd[f"plane_{key}"] = cp
            del qpd, o
        qs = inputs.sphere_queries(wx, hy, tex_size=4096, levels=len(lv))
        qsd = torch.from_numpy(qs).cuda()
        ns = qs.shape[0]
        subs = np.sort(rng.choice(ns, 5000, replace=False))
        reft = oracle.triplanar(otd, qs, 1.0, 0, oracle.LINEAR, oracle.BEFORE, shade=1, subset=subs)
        ct = {"queries": ns}
        for name, pm, mode in (("blend_trilinear_before_24decodes", 0, sf.SF_BEFORE),
                               ("blend_trilinear_stochastic_3decodes", 0, sf.SF_STOCHASTIC),
                               ("pick_trilinear_before_8decodes", 1, sf.SF_BEFORE),
                               ("pick_trilinear_stochastic_1decode", 1, sf.SF_STOCHASTIC)):
            smp = sf.sampling(sf.SF_LINEAR, mode, 1, seed=5)
            o = torch.empty((ns, 3), dtype=torch.float32, device="cuda")
            t = time_launches(lambda: sf.sf_triplanar(texd, qsd, smp, 1.0, pm, sf.SF_SHADE_GGX, g, out=o), 10, 3,
                              torch)
            ct[name] = {"ms": t, "queries_per_s": ns / (t * 1e-3),
                        "rmse_vs_oracle_blend_trilinear_before": _rmse(o.cpu().numpy()[subs], reft)}
        ct["fully_stochastic_speedup"] = (ct["blend_trilinear_before_24decodes"]["ms"] /
                                          ct["pick_trilinear_stochastic_1decode"]["ms"])
        cd[f"triplanar_sphere_{key}"] = ct
        del qsd, o
    res["dct_triplanar"] = cd


def neural_bench(args):
    import torch
    import oracle
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    torch.cuda.set_device(0)
    rng = np.random.default_rng(5)
    res = {}
    texture_bench(args, res)
    planck_bench(res)

    # ---- config 4: 1024^2 x 8 BF16 latent texture of the 64^2 RGBA32F texture
    log("config 4: targets and training")
    src = inputs.texture_uniform(64, seed=1)
    R = 1024
    yy, xx = np.mgrid[0:R, 0:R]
    uv = np.zeros((R * R, 3), np.float32)
    uv[:, 0] = ((xx + 0.5) / R).ravel()
    uv[:, 1] = ((yy + 0.5) / R).ravel()
    tex = sf.Texture2D([src])
    targets = sf.sf_filter2d(tex, torch.from_numpy(uv).cuda(), sf.sampling(sf.SF_BSPLINE3, sf.SF_BEFORE, 1))
    lat0 = torch.from_numpy((rng.normal(size=R * R * 8) * 0.5).astype(np.float32)).cuda()
    par0 = torch.from_numpy(_init_mlp(rng, 8, 4)).cuda()
    st, l_first, l_last, ms_train = _train(sf, torch, lat0, par0, targets, 8, 4, args.epochs4, 65536, 1e-2, 1e-3, 1)
    grid = sf.sf_neural_quantize(st.latents, 2, (R, R), 8, sf.SF_LATENT_BF16)
    mlp = sf.MLP(st.params, 8, 4)
    fit = sf.sf_neural_decode_lattice(grid, mlp, torch.arange(R * R, device="cuda", dtype=torch.int64))
    q = inputs.queries_uniform(2 * 1024 * 1024, seed=6)
    qd = torch.from_numpy(q).cuda()
    g = sf.ggx()
    nq = q.shape[0]
    runs = {
        "neural_stochastic_1_decode": lambda o: sf.sf_neural_decode(grid, mlp, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=3), sf.SF_SHADE_GGX, g, out=o),
        "neural_after_16_decodes": lambda o: sf.sf_neural_decode(grid, mlp, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1), sf.SF_SHADE_GGX, g, out=o),
        "neural_before_16_decodes": lambda o: sf.sf_neural_decode(grid, mlp, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_BEFORE, 1), sf.SF_SHADE_GGX, g, out=o),
        "plain_stochastic": lambda o: sf.sf_filter2d(tex, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=3), sf.SF_SHADE_GGX, g, out=o),
        "plain_after": lambda o: sf.sf_filter2d(tex, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1), sf.SF_SHADE_GGX, g, out=o),
        # equal memory: the 1024^2 targets as an RGBA32F texture (16 B per texel, as the BF16 latents)
        "plain1024_equal_memory_stochastic": lambda o: sf.sf_filter2d(eqmem_tex, qd, sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=3), sf.SF_SHADE_GGX, g, out=o),
    }
    eqmem_tex = sf.Texture2D([targets.cpu().numpy().reshape(R, R, 4)])
    sub = np.sort(rng.choice(nq, 20000, replace=False))
    ref_after = oracle.filter2d(oracle.Tex2D.rgba32f(src), q, oracle.BSPLINE3, oracle.AFTER, shade=1, subset=sub)
    c4 = {"training": {"epochs": args.epochs4, "batch": 65536, "steps": args.epochs4 * 16, "ms": ms_train,
                       "loss_first_epoch": l_first, "loss_last_epoch": l_last,
                       "rmse_decoded_vs_targets": float(torch.sqrt(torch.mean((fit - targets) ** 2)))},
          "queries": nq, "memory_bytes": {"latents_bf16": R * R * 8 * 2, "plain_rgba32f_64x64": 64 * 64 * 16}}
    for name, fn in runs.items():
        o = torch.empty((nq, 3), dtype=torch.float32, device="cuda")
        t = time_launches(lambda: fn(o), 10, 3, torch)
        c4[name] = {"ms": t, "queries_per_s": nq / (t * 1e-3), "rmse_vs_oracle_plain_after": _rmse(o.cpu().numpy()[sub], ref_after)}
        if name.startswith("neural"):
            dec = nq * (1 if "stochastic" in name else 16)
            c4[name]["decodes_per_s"] = dec / (t * 1e-3)
            c4[name]["mfma_useful_tflops"] = dec * MLP_FLOP[(8, 4)] / (t * 1e-3) / 1e12
    c4["gain"] = {
        "equal_lookups_rmse_ratio_plain64_over_neural": c4["plain_stochastic"]["rmse_vs_oracle_plain_after"]
        / c4["neural_stochastic_1_decode"]["rmse_vs_oracle_plain_after"],
        "equal_memory_rmse_ratio_neural_over_plain1024": c4["neural_stochastic_1_decode"]["rmse_vs_oracle_plain_after"]
        / c4["plain1024_equal_memory_stochastic"]["rmse_vs_oracle_plain_after"],
        "decodes_saved_vs_exact_after": 16,
        "time_ratio_after_over_stochastic": c4["neural_after_16_decodes"]["ms"] / c4["neural_stochastic_1_decode"]["ms"]}
    res["config4"] = c4
    del st, grid, fit, targets, lat0, par0
    torch.cuda.empty_cache()

    # ---- config 5: 256^3 x 16 E4M3 latent volume of a 1024^3 fp16 cloud
    log("config 5: 1024^3 source and targets")
    side = 0.25
    src3 = inputs.cloud_grid(1024, seed=7, device="cuda")
    vol1024 = sf.Volume(src3, side=side, brick_log2=3)
    L = 256
    cz, cy, cx = torch.meshgrid(*(torch.arange(L, device="cuda", dtype=torch.float32),) * 3, indexing="ij")
    pos = torch.stack([cx, cy, cz], -1).reshape(-1, 3).add_(0.5).mul_(side / L).contiguous()
    sig_t = sf.sf_filter3d(vol1024, pos, sf.sampling(sf.SF_BSPLINE3, sf.SF_BEFORE, 1))
    del pos, cx, cy, cz
    sigma_max = 50.0
    targets = (sig_t / sigma_max).contiguous()
    log("config 5: training")
    lat0 = torch.from_numpy((rng.normal(size=L ** 3 * 16) * 0.5).astype(np.float32)).cuda()
    par0 = torch.from_numpy(_init_mlp(rng, 16, 1)).cuda()
    all_pts = torch.arange(L ** 3, device="cuda", dtype=torch.int64)

    def c5_network(compute):
        """Train the C5 network in one compute mode; the E4M3 grid and MLP it
        decodes with, the training record, and the lattice RMSE of its
        decoded density with E4M3 and with BF16 latents."""
        st, l_first, l_last, ms_train = _train(sf, torch, lat0.clone(), par0.clone(), targets, 16, 1, args.epochs5,
                                               262144, 1e-2, 1e-3, 2, compute=compute, cosine=True)
        # the network was fitted to sigma / sigma_max: fold sigma_max into the last layer
        o3 = 16 * 64 + 64 + 64 * 64 + 64
        params = st.params.clone()
        params[o3:] *= sigma_max
        mlp = sf.MLP(params, 16, 1)
        rmse = {}
        for tag, fmt in (("e4m3", sf.SF_LATENT_FP8E4M3), ("bf16", sf.SF_LATENT_BF16)):
            gq = sf.sf_neural_quantize(st.latents, 3, (L, L, L), 16, fmt, 3, (0, 0, 0), (L / side,) * 3)
            fit = sf.sf_neural_decode_lattice(gq, mlp, all_pts)
            rmse[tag] = float(torch.sqrt(torch.mean((fit.view(-1).clamp(min=0) - sig_t) ** 2)))
            if tag == "e4m3":
                grid = gq
            del fit
        rec = {"epochs": args.epochs5, "batch": 262144, "steps": args.epochs5 * 64, "ms": ms_train,
               "learning_rates": "latents 1e-2, MLP 1e-3, cosine decay to 1%",
               "loss_first_epoch": l_first, "loss_last_epoch": l_last, "sigma_scale": sigma_max,
               "rmse_decoded_sigma_vs_targets": rmse["e4m3"],
               "rmse_decoded_sigma_vs_targets_bf16_latents": rmse["bf16"]}
        del st
        return grid, mlp, rec

    grid, mlp, train_rec = c5_network(sf.SF_TRAIN_BF16)
    log("config 5: training in FP32 (comparison)")
    grid32, mlp32, train_rec32 = c5_network(sf.SF_TRAIN_FP32)
    del lat0, par0
    torch.cuda.empty_cache()
    # equal-memory (512^3 fp16 = 256 MiB) and equal-lattice (256^3) plain grids, box-averaged
    log("config 5: rays and timing")
    f32 = src3.float()[None, None]
    g512 = torch.nn.functional.avg_pool3d(f32, 2)[0, 0].half().contiguous()
    g256 = torch.nn.functional.avg_pool3d(f32, 4)[0, 0].half().contiguous()
    del f32
    v512 = sf.Volume(g512, side=side, brick_log2=3)
    v256 = sf.Volume(g256, side=side, brick_log2=3)
    rays = inputs.ortho_rays(512, 16, side=side, seed=12)
    rd = torch.from_numpy(rays).cuda()
    nr, steps = rays.shape[0], 128
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=4)
    hit = int((rays[:, 7] > rays[:, 6]).sum())
    sub = np.nonzero(rays[:, 7] > rays[:, 6])[0]
    sub = np.sort(rng.choice(sub, 1500, replace=False))
    log("config 5: oracle filter-after reference on the 1024^3 grid")
    ref_after = oracle.raymarch(oracle.Grid(src3.cpu().numpy(), side=side), rays, steps, oracle.BSPLINE3, oracle.AFTER,
                            subset=sub)
    c5 = {"training": dict(train_rec, compute="bf16 matrix cores"),
          "training_fp32_comparison": dict(train_rec32, compute="fp32 vector ALU"),
          "rays": nr, "hit_rays": hit, "steps": steps,
          "memory_bytes": {"latents_fp8": L ** 3 * 16, "block_scales": int(grid.scales.numel()) * 4,
                           "plain_1024": 1024 ** 3 * 2, "plain_512": 512 ** 3 * 2, "plain_256": 256 ** 3 * 2}}
    T = torch.empty(nr, dtype=torch.float32, device="cuda")
    for name, fn in (("neural_stochastic_1_decode", lambda: sf.sf_neural_raymarch(grid, mlp, rd, steps, smp, T=T)),
                     ("neural_fp32_trained_stochastic_1_decode",
                      lambda: sf.sf_neural_raymarch(grid32, mlp32, rd, steps, smp, T=T)),
                     ("plain1024_stochastic", lambda: sf.sf_raymarch(vol1024, rd, steps, smp, T=T)),
                     ("plain512_stochastic_equal_memory", lambda: sf.sf_raymarch(v512, rd, steps, smp, T=T)),
                     ("plain256_stochastic_equal_lattice", lambda: sf.sf_raymarch(v256, rd, steps, smp, T=T))):
        t = time_launches(fn, 5, 2, torch)
        c5[name] = {"ms": t, "ray_steps_per_s": hit * steps / (t * 1e-3),
                    "rmse_vs_oracle_plain1024_after": _rmse(T.cpu().numpy()[sub], ref_after)}
        if name.startswith("neural"):
            c5[name]["decodes_per_s"] = hit * steps / (t * 1e-3)
            c5[name]["mfma_useful_tflops"] = hit * steps * MLP_FLOP[(16, 1)] / (t * 1e-3) / 1e12
            c5[name]["mfma_frac_of_bf16_peak"] = c5[name]["mfma_useful_tflops"] / MFMA_BF16_PEAK_TFLOPS
    c5["gain"] = {
        "equal_memory_rmse_ratio_neural_over_plain512": c5["neural_stochastic_1_decode"]["rmse_vs_oracle_plain1024_after"]
        / c5["plain512_stochastic_equal_memory"]["rmse_vs_oracle_plain1024_after"],
        "equal_lattice_rmse_ratio_neural_over_plain256": c5["neural_stochastic_1_decode"]["rmse_vs_oracle_plain1024_after"]
        / c5["plain256_stochastic_equal_lattice"]["rmse_vs_oracle_plain1024_after"],
        "winner_equal_memory": "plain" if c5["plain512_stochastic_equal_memory"]["rmse_vs_oracle_plain1024_after"]
        < c5["neural_stochastic_1_decode"]["rmse_vs_oracle_plain1024_after"] else "neural"}
    res["config5"] = c5
    n5 = c5["neural_stochastic_1_decode"]
    line = {"metric": "neural decodes/s: stochastic tricubic through a 256^3x16 E4M3 latent volume (1 decode per "
                      "ray step)", "value": n5["decodes_per_s"], "unit": "decodes/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "configs 1 and 2 (2-D path), 4 and 5 (neural latent texture and volume)"},
            "roofline": {"bound": "mfma", "achieved": n5["mfma_useful_tflops"], "peak": MFMA_BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": n5["mfma_frac_of_bf16_peak"], "traffic": None}}
    line.update(res)
    print(json.dumps(line))


def neural_pmc(args):
    """Counter runs of the neural kernels at the config-4 and config-5 shapes:
    seeded random latents (E4M3 codes and block scales for config 5, BF16
    for config 4) and MLP weights built on the host and copied to the device,
    so that no torch device kernel runs.  The decoders' work does not depend
    on trained values: the same launches as the suite times (4 Mi rays x 128
    steps; 2 Mi queries), then training steps of both shapes."""
    import torch
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    torch.cuda.set_device(0)
    rng = np.random.default_rng(41)
    side, L, C5 = 0.25, 256, 16
    codes = rng.integers(0, 0x7E, size=L ** 3 * C5, dtype=np.uint8)       # finite E4M3 codes
    codes[rng.random(codes.size) < 0.5] |= 0x80                             # either sign
    scales = rng.uniform(1e-3, 1e-2, size=(L // 8) ** 3).astype(np.float32)
    grid5 = sf.LatentGrid(3, (L, L, L), C5, sf.SF_LATENT_FP8E4M3, torch.from_numpy(codes).cuda(),
                          torch.from_numpy(scales).cuda(), 3, (0.0, 0.0, 0.0), (L / side,) * 3)
    mlp5 = sf.MLP(torch.from_numpy(_init_mlp(rng, C5, 1)).cuda(), C5, 1)
    rays = torch.from_numpy(inputs.ortho_rays(512, 16, side=side, seed=12)).cuda()
    T = torch.empty(rays.shape[0], dtype=torch.float32, device="cuda")
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=4)
    t5 = time_launches(lambda: sf.sf_neural_raymarch(grid5, mlp5, rays, 128, smp, T=T), 3, 1, torch)
    del grid5, codes
    R = 1024
    b16 = rng.integers(0x3C00, 0x3F80, size=R * R * 8, dtype=np.uint16)   # BF16 bits of 2^-7 .. 1
    b16[rng.random(b16.size) < 0.5] |= 0x8000
    lat4 = torch.from_numpy(b16.view(np.int16)).cuda()
    grid4 = sf.LatentGrid(2, (R, R), 8, sf.SF_LATENT_BF16, lat4)
    mlp4 = sf.MLP(torch.from_numpy(_init_mlp(rng, 8, 4)).cuda(), 8, 4)
    q = torch.from_numpy(inputs.queries_uniform(2 * 1024 * 1024, seed=6)).cuda()
    out = torch.empty((q.shape[0], 3), dtype=torch.float32, device="cuda")
    s4 = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=3)
    t4 = time_launches(lambda: sf.sf_neural_decode(grid4, mlp4, q, s4, sf.SF_SHADE_GGX, sf.ggx(), out=out), 3, 1,
                       torch)
    times = {"neural_ray_ms": t5, "neural2d_ms": t4}
    for name, (n, C, O, batch) in {"train5": (L ** 3, 16, 1, 262144), "train4": (R * R, 8, 4, 65536)}.items():
        lat = torch.from_numpy((rng.standard_normal(n * C, dtype=np.float32) * 0.5)).cuda()
        tg = torch.from_numpy(rng.random(n * O, dtype=np.float32)).cuda()
        idx = torch.from_numpy(rng.permutation(n)[:batch].astype(np.int32)).cuda()
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        for tag, compute in (("", sf.SF_TRAIN_BF16), ("_fp32", sf.SF_TRAIN_FP32)):
            st = sf.TrainState(lat, torch.from_numpy(_init_mlp(rng, C, O)).cuda(), C, O, compute=compute)
            times[name + tag + "_ms"] = time_launches(
                lambda: sf.sf_neural_train_step(st, idx, tg, 1e-2, 1e-3, loss_out=loss), 3, 1, torch)
            del st
        del lat, tg
    print(json.dumps(times))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--pmc-comparators", action="store_true",
                    help="with --pmc-run: also launch each ray-march comparator three times")
    ap.add_argument("--no-compare", action="store_true", help="skip comparators and the equal-RMSE protocol")
    ap.add_argument("--cpu-rays", type=int, default=1 << 20, help="rays in the CPU oracle sample")
    ap.add_argument("--suite", action="store_true",
                    help="configs 1, 2 (2-D path), 4 and 5 (neural forms): one JSON line beside the headline run")
    ap.add_argument("--suite-aniso", action="store_true", help="only the anisotropic section of the suite")
    ap.add_argument("--suite-planck", action="store_true", help="only the emission section of the suite")
    ap.add_argument("--epochs4", type=int, default=200)
    ap.add_argument("--epochs5", type=int, default=120)
    ap.add_argument("--save-inputs", default="", help="write the headline workload (grid, rays) to this .npz and exit")
    ap.add_argument("--load-inputs", default="", help="read the headline workload from this .npz")
    ap.add_argument("--pmc-neural", action="store_true",
                    help="counter runs of the neural decoders and training steps on seeded random data")
    ap.add_argument("--pmc-run", action="store_true",
                    help="counter runs: time the headline kernel and its gather twin only, launch nothing else")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (HBM counter calibration)")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only the vector-ALU issue-rate probe (CU cycles per wave64 instruction)")
    ap.add_argument("--dense-probe", action="store_true",
                    help="only the timed launch on constant-density grids of 16^3 to 512^3 (every step marched)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the path is single-GPU (rays are independent, so more GPUs "
              f"would each march a contiguous share of the ray stream). --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)
    if args.suite_aniso or args.suite_planck:
        res = {}
        if args.suite_aniso:
            aniso_bench(res)
        if args.suite_planck:
            planck_bench(res)
        print(json.dumps(res))
        return
    if args.suite:
        neural_bench(args)
        return
    if args.pmc_neural:
        neural_pmc(args)
        return

    import torch
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    torch.cuda.set_device(0)
    if args.dense_probe:
        # the timed launch (same rays, steps, mask and filter) on grids of
        # constant density 0.5 filling the cube: every step gathers, so the
        # instruction count is the same for every grid size and the time shows
        # what the grid's size (its place in the cache hierarchy) costs
        rays_d = torch.from_numpy(inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=1.0, seed=11)).cuda()
        T = torch.empty(rays_d.shape[0], dtype=torch.float32, device="cuda")
        smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=2024)
        out = {}
        for n in (16, 64, 256, 512):
            g = torch.full((n, n, n), 0.5, dtype=torch.float16, device="cuda")
            v = sf.Volume(g, side=1.0, brick_log2=BRICK_LOG2)
            out[f"dense_{n}^3_ms"] = time_launches(lambda: sf.sf_raymarch(v, rays_d, STEPS, smp, T=T), 50, 5, torch)
            del v, g
        print(json.dumps(out))
        return
    if args.valu_rates:
        print(json.dumps({"valu_issue_probe_cu_cycles_per_inst": valu_issue_rates(torch, reps=20),
                          "device": torch.cuda.get_device_name(0)}))
        return
    if args.save_inputs:
        # the workload, written once for counter runs (which then launch no
        # torch device kernel besides the calibration copy)
        log("generating workload")
        grid = inputs.cloud_grid(GRID, seed=4, device="cuda").cpu()
        rays = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=11)
        np.savez(args.save_inputs, grid=grid.view(torch.int16).numpy(), rays=rays)
        log(f"wrote {args.save_inputs}")
        return
    if args.copy_probe:
        # a plain streaming kernel of known traffic: reads and writes
        # copy_probe bytes (torch's elementwise negation)
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.load_inputs:
        log(f"loading workload from {args.load_inputs}")
        z = np.load(args.load_inputs)
        grid = torch.from_numpy(z["grid"]).view(torch.float16).cuda()   # host-to-device copies only
        rays = z["rays"]
    else:
        log("generating workload")
        grid = inputs.cloud_grid(GRID, seed=4, device="cuda")
        rays = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=11)
    rays_d = torch.from_numpy(rays).cuda()
    n = rays.shape[0]
    # Every path runs with the 8^3 occupancy mask (exact empty-space
    # skipping); the stochastic march without it is timed beside.
    vol_plain = sf.Volume(grid, side=SIDE)
    vol_occ = sf.Volume(grid, side=SIDE, brick_log2=BRICK_LOG2)
    vol = vol_occ
    T = torch.empty(n, dtype=torch.float32, device="cuda")
    seed = 2024
    smp = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=seed)
    torch.cuda.synchronize()

    log("timing stochastic tricubic")
    fn = lambda: sf.sf_raymarch(vol, rays_d, STEPS, smp, T=T)
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    queries = n * STEPS
    value = queries / (ms * 1e-3)

    log("timing the gather-only twin")
    twin_fn = gather_twin(torch, vol_occ, grid, rays_d, T)
    t_twin = time_launches(twin_fn, args.steps, args.warmup, torch)
    t_real = time_launches(fn, args.steps, args.warmup, torch)
    if args.pmc_run:
        # counter runs: the kernels have run; nothing else touches the device
        # but, with --pmc-comparators, three launches of each comparator
        out = {"ms_per_step": ms, "gather_twin_ms": t_twin, "ms_again": t_real}
        if args.pmc_comparators:
            for name, filt, mode in (("tricubic_after_64tap", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT),
                                     ("tricubic_before_64tap", sf.SF_BSPLINE3, sf.SF_BEFORE),
                                     ("trilinear_after_8tap", sf.SF_LINEAR, sf.SF_AFTER_EXACT),
                                     ("trilinear_before_8tap", sf.SF_LINEAR, sf.SF_BEFORE)):
                s2 = sf.sampling(filt, mode, 1, seed=seed)
                out[name + "_ms"] = time_launches(lambda: sf.sf_raymarch(vol_occ, rays_d, STEPS, s2, T=T), 3, 0,
                                                  torch)
        print(json.dumps(out))
        return

    # algorithmic HBM bytes of one launch (548 B per ray: one binary16 voxel
    # per step, the ray record and the result), and the bytes of the steps
    # the kernel actually gathers (steps of rays that meet the grid, in
    # occupied bricks)
    hit = rays[:, 7] > rays[:, 6]
    hit_steps = int(hit.sum()) * STEPS
    occ_steps = count_occupied_steps(torch, vol_occ.occupancy, rays_d)
    algo_bytes = n * BYTES_PER_RAY
    gathered_bytes = occ_steps * 2 + n * 36
    counters = counters_from_profile(kernel_code_digest())
    valu = counters.get("valu_insts_per_launch")
    achieved_tops = valu * 64 / (ms * 1e-3) / 1e12 if valu else None

    extra = {}
    if not args.no_compare:
        log("timing comparators")
        rates = {}
        for name, filt, mode in (("tricubic_after_64tap", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT),
                                 ("tricubic_before_64tap", sf.SF_BSPLINE3, sf.SF_BEFORE),
                                 ("trilinear_after_8tap", sf.SF_LINEAR, sf.SF_AFTER_EXACT),
                                 ("trilinear_before_8tap", sf.SF_LINEAR, sf.SF_BEFORE),
                                 ("trilinear_stochastic", sf.SF_LINEAR, sf.SF_STOCHASTIC),
                                 ("tricubic_stochastic_without_mask", sf.SF_BSPLINE3, sf.SF_STOCHASTIC)):
            s2 = sf.sampling(filt, mode, 1, seed=seed)
            v2 = vol_plain if name.endswith("without_mask") else vol_occ
            t = time_launches(lambda: sf.sf_raymarch(v2, rays_d, STEPS, s2, T=T), 5, 2, torch)
            rates[name] = {"ms": t, "queries_per_s": queries / (t * 1e-3)}
        extra["comparators"] = rates
        log("equal-RMSE protocol")
        extra["equal_rmse_vs_tricubic_after"] = equal_rmse(sf, torch, vol_occ, rays_d, ms,
                                                           rates["tricubic_after_64tap"]["ms"], seed,
                                                           rates["tricubic_before_64tap"]["ms"])
        extra["speedup_vs_tricubic_after_same_rays"] = rates["tricubic_after_64tap"]["ms"] / ms
        extra["speedup_vs_tricubic_before_same_rays"] = rates["tricubic_before_64tap"]["ms"] / ms

    copy_gbs = copy_bandwidth(torch)
    valu_rates = valu_issue_rates(torch)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(grid.cpu().numpy(), rays, seed, args.cpu_rays)
        if not args.no_compare:
            extra["cpu_oracle_comparators"] = cpu_comparators(grid.cpu().numpy(), rays, seed)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "shaded queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision": "binary16 texels, binary32 decisions, compensated binary32 optical depth",
        "data": "synthetic: fractal-noise cloud stands in for the Disney Cloud",
        "config": {"workload": "512^3 fp16 cloud, 1,048,576 rays (256x256 px x 16), 256 steps, "
                               "stochastic tricubic transmittance, 1 lookup per step, 8^3 occupancy bricks",
                   "rays": n, "steps": STEPS, "grid": [GRID, GRID, GRID], "parallelism": "single GPU"},
        "rays_per_s": n / (ms * 1e-3),
        # the kernel is bound by VALU issue: achieved = the VALU lane-operations
        # it issues per launch (the SQ_INSTS_VALU counter of the committed
        # rocprofv3 run x 64 lanes) over the launch's HIP-event duration, null
        # when the counters were taken on other machine code
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved_tops / VALU_PEAK_TOPS if achieved_tops else None,
                     "frac_of_one_issue_per_cu_cycle": achieved_tops / VALU_ONE_ISSUE_TOPS if achieved_tops else None,
                     "valu_issue_probe_cu_cycles_per_inst": valu_rates,
                     "traffic": counters.get("hbm_bytes_per_launch"),
                     "valu_insts_per_launch": valu,
                     "valu_busy_frac": counters.get("valu_busy_frac"),
                     "counters": os.path.relpath(PMC_PROFILE, ROOT)},
        # the gather ceiling of this access pattern: the same launch with the
        # random pick replaced by a fixed tap (libsf_bench.so), t(twin) / t(real)
        "gather_twin_frac": t_twin / t_real,
        "gather_twin_ms": t_twin,
        "hbm_roofline": {"achieved": algo_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": algo_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_ray": BYTES_PER_RAY,
                         "algorithmic_bytes": algo_bytes, "gathered_bytes": gathered_bytes,
                         "copy_gbs": copy_gbs},
        "ray_steps": hit_steps,
        "ray_steps_in_occupied_bricks": occ_steps,
        # the same launch counted by the steps that meet the grid, and by the
        # steps that gather a voxel (value counts every step of every ray)
        "ray_steps_per_s": hit_steps / (ms * 1e-3),
        "gathering_steps_per_s": occ_steps / (ms * 1e-3),
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
