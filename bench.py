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
# Non-packed VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, in
# tera lane-operations per second (an FMA counts as one operation).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Lane operations per ray step of the stochastic tricubic decision contract
# plus its gather and accumulation (itemised in the design doc): every step forms
# its position (13) and tests its brick (12); a step in an occupied brick
# then hashes, picks, gathers and accumulates (88 more).
OPS_POSITION, OPS_BRICK_TEST, OPS_OCCUPIED = 13, 12, 88
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


def equal_rmse(sf, torch, vol, rays_d, t_stoch, t_det, seed):
    """Pixel-integral equal-RMSE protocol.

    Reference pixel value R_p = mean of the exact-after 64-tap transmittance
    over 256 stratified rays per pixel (its own sampling variance is measured
    and subtracted).  Both 16-ray estimates are compared with R_p; the
    stochastic path needs spp* = 16 (RMSE_s/RMSE_d)^2 rays per pixel to match
    the deterministic path, so the throughput ratio at equal RMSE is
    (t_det / t_stoch) (RMSE_d / RMSE_s)^2."""
    import numpy as np
    from paper_2407_06107_amd import inputs

    P = N_PIX * N_PIX
    after = sf.sampling(sf.SF_BSPLINE3, sf.SF_AFTER_EXACT, 1)
    stoch = sf.sampling(sf.SF_BSPLINE3, sf.SF_STOCHASTIC, 1, seed=seed)
    T_s = sf.sf_raymarch(vol, rays_d, STEPS, stoch).double().view(P, RAYS_PER_PIX).mean(1)
    T_d = sf.sf_raymarch(vol, rays_d, STEPS, after).double().view(P, RAYS_PER_PIX).mean(1)
    # reference: 256 rays per pixel in 16 chunks of 16 rays (different jitter)
    acc = torch.zeros(P, dtype=torch.float64, device="cuda")
    acc2 = torch.zeros(P, dtype=torch.float64, device="cuda")
    m = 0
    for c in range(16):
        r = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=1000 + c)
        T = sf.sf_raymarch(vol, torch.from_numpy(r).cuda(), STEPS, after).double().view(P, RAYS_PER_PIX)
        acc += T.sum(1)
        acc2 += (T * T).sum(1)
        m += RAYS_PER_PIX
    R = acc / m
    var_R = (acc2 / m - R * R).clamp(min=0) / (m - 1)
    bias_corr = float(var_R.mean())
    mse_s = float(((T_s - R) ** 2).mean()) - bias_corr
    mse_d = float(((T_d - R) ** 2).mean()) - bias_corr
    rmse_s, rmse_d = math.sqrt(max(mse_s, 0.0)), math.sqrt(max(mse_d, 0.0))
    spp_star = RAYS_PER_PIX * (rmse_s / rmse_d) ** 2
    ratio = (t_det / t_stoch) * (rmse_d / rmse_s) ** 2
    return {"rmse_stochastic_16": rmse_s, "rmse_det_after_16": rmse_d,
            "mse_increase": mse_s / mse_d - 1.0, "spp_star": spp_star, "ratio": ratio,
            "reference_rays_per_pixel": m, "reference_var_subtracted": bias_corr}


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


def traffic_from_profile(source_digest):
    """HBM bytes per launch measured by rocprofv3 FETCH_SIZE + WRITE_SIZE
    (scaled by the plain-copy calibration), read from the committed profile
    summary; None if the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "raymarch_stochastic_tricubic_512cloud_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != source_digest:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def count_occupied_steps(torch, occ, rays_d):
    """Ray steps whose lookup point lies in an occupied brick (those the
    kernel does not skip), from the same raster positions evaluated with
    torch float32 operations; a step on a brick boundary may round the other
    way, so the count is exact to a few parts per million."""
    words = occ.to(torch.int64) & 0xFFFFFFFF
    nb = GRID >> BRICK_LOG2
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
        inr = ((b >= 0) & (b < nb)).all(-1)
        bc = b.clamp(0, nb - 1)
        lin = (bc[..., 2] * nb + bc[..., 1]) * nb + bc[..., 0]
        bit = (words[lin >> 5] >> (lin & 31)) & 1
        occupied = (bit.bool() | ~inr) & hit[:, None]
        total += int(occupied.sum())
    return total


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("sf_device.hpp", "sf_internal.hpp", "volume.hip"):
        h.update(open(os.path.join(ROOT, "paper_2407_06107_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip comparators and the equal-RMSE protocol")
    ap.add_argument("--cpu-rays", type=int, default=1 << 20, help="rays in the CPU oracle sample")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the path is single-GPU (rays are independent; sharding is "
              f"a split of the ray stream, described in DESIGN.md). --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_06107_amd as sf
    from paper_2407_06107_amd import inputs

    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain streaming kernel of known traffic: reads and writes
        # copy_probe bytes (torch's elementwise negation)
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    log("generating workload")
    grid = inputs.cloud_grid(GRID, seed=4, device="cuda")
    rays = inputs.ortho_rays(N_PIX, RAYS_PER_PIX, side=SIDE, seed=11)
    rays_d = torch.from_numpy(rays).cuda()
    n = rays.shape[0]
    vol = sf.Volume(grid, side=SIDE, brick_log2=BRICK_LOG2)
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

    # algorithmic work of one launch: every ray of the stream is read (32 B)
    # and its T written (4 B); every step of a ray that meets the grid forms
    # its position and tests its brick; each step in an occupied brick gathers
    # one binary16 voxel and executes the rest of the decision contract.
    hit = rays[:, 7] > rays[:, 6]
    hit_steps = int(hit.sum()) * STEPS
    occ_steps = count_occupied_steps(torch, vol.occupancy, rays_d)
    algo_bytes = occ_steps * 2 + n * 32 + n * 4
    achieved_gbs = algo_bytes / (ms * 1e-3) / 1e9
    algo_ops = hit_steps * (OPS_POSITION + OPS_BRICK_TEST) + occ_steps * OPS_OCCUPIED
    achieved_tops = algo_ops / (ms * 1e-3) / 1e12
    traffic = traffic_from_profile(kernel_source_digest())

    extra = {}
    if not args.no_compare:
        log("timing comparators")
        rates = {}
        for name, filt, mode in (("tricubic_after_64tap", sf.SF_BSPLINE3, sf.SF_AFTER_EXACT),
                                 ("tricubic_before_64tap", sf.SF_BSPLINE3, sf.SF_BEFORE),
                                 ("trilinear_after_8tap", sf.SF_LINEAR, sf.SF_AFTER_EXACT),
                                 ("trilinear_before_8tap", sf.SF_LINEAR, sf.SF_BEFORE),
                                 ("trilinear_stochastic", sf.SF_LINEAR, sf.SF_STOCHASTIC)):
            s2 = sf.sampling(filt, mode, 1, seed=seed)
            t = time_launches(lambda: sf.sf_raymarch(vol, rays_d, STEPS, s2, T=T), 5, 2, torch)
            rates[name] = {"ms": t, "queries_per_s": queries / (t * 1e-3)}
        extra["comparators"] = rates
        log("equal-RMSE protocol")
        extra["equal_rmse_vs_tricubic_after"] = equal_rmse(sf, torch, vol, rays_d, ms,
                                                           rates["tricubic_after_64tap"]["ms"], seed)
        extra["speedup_vs_tricubic_after_same_rays"] = rates["tricubic_after_64tap"]["ms"] / ms
        extra["speedup_vs_tricubic_before_same_rays"] = rates["tricubic_before_64tap"]["ms"] / ms

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(grid.cpu().numpy(), rays, seed, args.cpu_rays)

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
        "precision": "binary16 texels, binary32 decisions, binary64 optical depth",
        "data": "synthetic: fractal-noise cloud stands in for the Disney Cloud",
        "config": {"workload": "512^3 fp16 cloud, 1,048,576 rays (256x256 px x 16), 256 steps, "
                               "stochastic tricubic transmittance, 1 lookup per step, 8^3 occupancy bricks",
                   "rays": n, "steps": STEPS, "grid": [GRID, GRID, GRID], "parallelism": "single GPU"},
        "rays_per_s": n / (ms * 1e-3),
        "hbm_algorithmic_gbs": achieved_gbs,
        "hbm_algorithmic_frac": achieved_gbs / HBM_PEAK_GBS,
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved_tops / VALU_PEAK_TOPS, "traffic": traffic,
                     "algorithmic_ops": algo_ops, "algorithmic_bytes": algo_bytes},
        "ray_steps": hit_steps,
        "ray_steps_in_occupied_bricks": occ_steps,
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
