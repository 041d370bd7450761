"""Seeded synthetic workloads for the stochastic texture filtering path.

This module only *makes inputs*: textures, MIP chains, query streams, density
grids and rays.  It holds none of the filtering, sampling or shading
arithmetic, so that the CPU oracle and the HIP path can both be fed from it
without sharing any of the method's code.

The paper measures on the Disney Cloud (a NanoVDB volume), on ambientCG PBR
materials and with STBN blue-noise masks (Section 5).  None of those assets
is available here, so the generators below build stand-ins with the same
structure: a sparse fractal-noise density cloud with exact zeros, band-limited
tileable RGBA textures with a full MIP pyramid, an oblique textured plane seen
by a pinhole camera, and orthographic rays through the volume.

Every generator is deterministic given its seed.  NumPy generators use
``numpy.random.default_rng`` (PCG64); the 3-D noise uses an integer lattice
hash evaluated with exact integer arithmetic, so it gives the same lattice on
any device.
"""
from __future__ import annotations

import math

import numpy as np

# ----------------------------------------------------------------------------
# 2-D textures
# ----------------------------------------------------------------------------


def texture_uniform(size: int = 64, seed: int = 1) -> np.ndarray:
    """RGBA32F texture, RGB ~ U[0,1) (albedo), A ~ U[0.05, 1) (roughness).

    Layout: ``[size, size, 4]`` float32, row-major (y, x, channel).
    """
    rng = np.random.default_rng(seed)
    tex = np.empty((size, size, 4), dtype=np.float32)
    tex[..., :3] = rng.random((size, size, 3))
    tex[..., 3] = 0.05 + 0.95 * rng.random((size, size))
    return tex


def queries_uniform(n: int, seed: int = 2, lod: float = 0.0) -> np.ndarray:
    """``n`` uniform uv in [0,1)^2 with a constant level of detail.

    Layout: ``[n, 3]`` float32 rows ``{u, v, lambda}``.
    """
    rng = np.random.default_rng(seed)
    q = np.empty((n, 3), dtype=np.float32)
    q[:, :2] = rng.random((n, 2))
    q[:, 2] = lod
    return q


def _wave_set(rng, waves: int, size: int):
    """Integer wave vectors with |f| log-uniform in [1, size/2], a ~ 1/|f|."""
    fx = np.zeros(waves, dtype=np.int64)
    fy = np.zeros(waves, dtype=np.int64)
    for k in range(waves):
        while True:
            mag = math.exp(rng.random() * math.log(size / 2))
            ang = rng.random() * 2.0 * math.pi
            a = int(round(mag * math.cos(ang)))
            b = int(round(mag * math.sin(ang)))
            a = max(-size // 2, min(size // 2, a))
            b = max(-size // 2, min(size // 2, b))
            if a != 0 or b != 0:
                fx[k], fy[k] = a, b
                break
    amp = 1.0 / np.hypot(fx, fy)
    phase = rng.random(waves) * 2.0 * math.pi
    return fx, fy, amp, phase


def texture_sinusoids(size: int = 4096, seed: int = 3, waves: int = 32) -> np.ndarray:
    """Tileable band-limited RGBA texture in [0,1], float64 ``[size,size,4]``.

    Each channel is 1/2 + 1/2 * sum_k a_k sin(2 pi f_k . x / size + phi_k) / sum_k a_k
    over ``waves`` integer wave vectors (so it tiles exactly), |f_k| <= size/2
    (at most Nyquist) and a_k proportional to 1/|f_k|.  The sum factors as
    two matrix products per channel, so 4096^2 texels take well under a second.
    """
    rng = np.random.default_rng(seed)
    x = np.arange(size, dtype=np.float64)
    out = np.empty((size, size, 4), dtype=np.float64)
    for c in range(4):
        fx, fy, amp, phase = _wave_set(rng, waves, size)
        ax = 2.0 * math.pi * np.outer(x, fx) / size            # [size, waves] along x
        by = 2.0 * math.pi * np.outer(x, fy) / size + phase    # [size, waves] along y
        # sin(ax + by) = sin(ax) cos(by) + cos(ax) sin(by)
        v = (np.cos(by) * amp) @ np.sin(ax).T + (np.sin(by) * amp) @ np.cos(ax).T
        out[..., c] = 0.5 + 0.5 * v / amp.sum()
    return np.clip(out, 0.0, 1.0)


def texture_normal_map(size: int = 4096, seed: int = 13, waves: int = 24, slope: float = 1.0,
                       roughness: float = 0.15) -> np.ndarray:
    """Tileable normal map of a bumpy surface, float64 ``[size,size,4]``:
    height h = sum_k a_k sin(2 pi f_k . x / size + phi_k) scaled so that the
    largest analytic slope |grad h| (texel units) is about ``slope``; RGB =
    (n + 1)/2 with n = normalize(-dh/dx, -dh/dy, 1) (tangent space), A =
    ``roughness`` (the roughness parameter of the GGX shading)."""
    rng = np.random.default_rng(seed)
    fx, fy, amp, phase = _wave_set(rng, waves, size)
    x = np.arange(size, dtype=np.float64)
    w = 2.0 * math.pi / size
    ax = w * np.outer(x, fx)                    # [size, waves] along x
    by = w * np.outer(x, fy) + phase            # [size, waves] along y
    # d/dx sin(ax + by) = w fx cos(ax + by); cos(ax + by) = cos(ax) cos(by) - sin(ax) sin(by)
    cosxy = lambda A: (np.cos(by) * A) @ np.cos(ax).T - (np.sin(by) * A) @ np.sin(ax).T
    gx = cosxy(amp * w * fx)
    gy = cosxy(amp * w * fy)
    scale = slope / np.sum(amp * w * np.hypot(fx, fy))
    n = np.stack([-gx * scale, -gy * scale, np.ones_like(gx)], axis=-1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    out = np.empty((size, size, 4), dtype=np.float64)
    out[..., :3] = 0.5 * (n + 1.0)
    out[..., 3] = roughness
    return out


def mip_chain(level0: np.ndarray) -> list[np.ndarray]:
    """Full MIP pyramid by 2x2 box averaging in float64, down to 1x1.

    ``level0`` is float64 ``[h, w, c]`` with power-of-two sides.  Each level
    is averaged from the previous *unquantised* level.
    """
    levels = [level0]
    cur = level0
    while cur.shape[0] > 1 or cur.shape[1] > 1:
        h, w = cur.shape[:2]
        h2, w2 = max(1, h // 2), max(1, w // 2)
        if h > 1 and w > 1:
            cur = 0.25 * (cur[0::2, 0::2] + cur[1::2, 0::2] + cur[0::2, 1::2] + cur[1::2, 1::2])
        elif h > 1:
            cur = 0.5 * (cur[0::2] + cur[1::2])
        else:
            cur = 0.5 * (cur[:, 0::2] + cur[:, 1::2])
        assert cur.shape[:2] == (h2, w2)
        levels.append(cur)
    return levels


def quantize_unorm8(levels: list[np.ndarray]) -> list[np.ndarray]:
    """Round-to-nearest-even to 8-bit unorm, per level."""
    return [np.rint(np.clip(lv, 0.0, 1.0) * 255.0).astype(np.uint8) for lv in levels]


def pack_levels(levels: list[np.ndarray]) -> tuple[np.ndarray, list[int]]:
    """Concatenate levels into one byte buffer; return (buffer, byte offsets).

    Offsets are aligned to 256 bytes.
    """
    offs, cur = [], 0
    for lv in levels:
        offs.append(cur)
        cur += (lv.nbytes + 255) // 256 * 256
    buf = np.zeros(cur, dtype=np.uint8)
    for lv, o in zip(levels, offs):
        buf[o:o + lv.nbytes] = np.frombuffer(np.ascontiguousarray(lv).tobytes(), dtype=np.uint8)
    return buf, offs


def _morton2(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0xFFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v
    return spread(x) | (spread(y) << np.uint64(1))


def tile_order(width: int, height: int, tile: int = 8) -> np.ndarray:
    """Pixel visiting order: ``tile x tile`` tiles in row-major order, Morton
    order inside each tile.  Returns flat pixel indices (y*width + x)."""
    ys, xs = np.mgrid[0:height, 0:width]
    tx, ty = xs // tile, ys // tile
    ntx = (width + tile - 1) // tile
    key = (ty * ntx + tx).astype(np.uint64) * np.uint64(tile * tile) + _morton2(xs % tile, ys % tile)
    return np.argsort(key.ravel(), kind="stable")


def plane_queries(width: int = 1920, height: int = 1080, tex_size: int = 4096, levels: int = 13,
                  height_above: float = 1.0, pitch_deg: float = 35.0, vfov_deg: float = 40.0,
                  tile: int = 8) -> np.ndarray:
    """Queries from a pinhole camera looking down at the textured plane z=0.

    The camera sits ``height_above`` over the plane, pitched ``pitch_deg``
    below the horizon, with vertical field of view ``vfov_deg``; uv is the
    world xy of the hit point (the texture repeats with period 1).  The level
    of detail is log2 of the longer uv footprint of one pixel step, measured
    in level-0 texels, from the hit points of neighbouring pixel rays
    (a ray-differential estimate) in float64, clamped to [0, levels-1].
    Output ``[width*height, 3]`` float32 ``{u, v, lambda}`` in
    :func:`tile_order`.
    """
    pitch = math.radians(pitch_deg)
    fwd = np.array([0.0, math.cos(pitch), -math.sin(pitch)])
    right = np.array([1.0, 0.0, 0.0])
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    tw = th * width / height
    cam = np.array([0.3, 0.1, height_above])

    def hit(px, py):
        sx = (2.0 * (px + 0.5) / width - 1.0) * tw
        sy = (1.0 - 2.0 * (py + 0.5) / height) * th
        d = fwd[None] + sx[:, None] * right[None] + sy[:, None] * up[None]
        t = -cam[2] / d[:, 2]
        return cam[None, :2] + t[:, None] * d[:, :2]

    order = tile_order(width, height, tile)
    px = (order % width).astype(np.float64)
    py = (order // width).astype(np.float64)
    p = hit(px, py)
    dx = hit(px + 1.0, py) - p
    dy = hit(px, py + 1.0) - p
    foot = np.maximum(np.hypot(dx[:, 0], dx[:, 1]), np.hypot(dy[:, 0], dy[:, 1])) * tex_size
    lam = np.clip(np.log2(np.maximum(foot, 1e-30)), 0.0, levels - 1)
    q = np.empty((order.size, 3), dtype=np.float32)
    q[:, 0] = p[:, 0]
    q[:, 1] = p[:, 1]
    q[:, 2] = lam
    return q


def plane_queries_aniso(width: int = 1920, height: int = 1080, height_above: float = 1.0,
                        pitch_deg: float = 35.0, vfov_deg: float = 40.0, tile: int = 8) -> np.ndarray:
    """Pixel queries of the :func:`plane_queries` camera for anisotropic
    filtering: ``[width*height, 6]`` float32 ``{u, v, du/dx, dv/dx, du/dy,
    dv/dy}``, uv at the pixel centre and its screen derivatives from the hit
    points of the neighbouring pixel rays (float64 differences), in
    :func:`tile_order`."""
    pitch = math.radians(pitch_deg)
    fwd = np.array([0.0, math.cos(pitch), -math.sin(pitch)])
    right = np.array([1.0, 0.0, 0.0])
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    tw = th * width / height
    cam = np.array([0.3, 0.1, height_above])

    def hit(px, py):
        sx = (2.0 * (px + 0.5) / width - 1.0) * tw
        sy = (1.0 - 2.0 * (py + 0.5) / height) * th
        d = fwd[None] + sx[:, None] * right[None] + sy[:, None] * up[None]
        t = -cam[2] / d[:, 2]
        return cam[None, :2] + t[:, None] * d[:, :2]

    order = tile_order(width, height, tile)
    px = (order % width).astype(np.float64)
    py = (order // width).astype(np.float64)
    p = hit(px, py)
    q = np.empty((order.size, 6), dtype=np.float32)
    q[:, 0:2] = p
    q[:, 2:4] = hit(px + 1.0, py) - p
    q[:, 4:6] = hit(px, py + 1.0) - p
    return q


def texture_checker(size: int = 4096, squares: int = 64) -> np.ndarray:
    """High-contrast checkerboard ``[size, size, 4]`` float32 (the
    minification test pattern): dark squares albedo 0.04 with roughness
    parameter 0.1, light squares albedo 0.9 with roughness parameter 0.9,
    so the GGX shading is non-linear across the pattern."""
    cell = size // squares
    i = np.arange(size) // cell
    light = ((i[:, None] + i[None, :]) & 1).astype(bool)
    tex = np.empty((size, size, 4), dtype=np.float32)
    tex[..., :3] = np.where(light[..., None], 0.9, 0.04)
    tex[..., 3] = np.where(light, 0.9, 0.1)
    return tex


def sphere_queries(width: int = 1920, height: int = 1080, tex_size: int = 4096, levels: int = 13,
                   scale: float = 1.0, distance: float = 3.0, vfov_deg: float = 40.0, tile: int = 8) -> np.ndarray:
    """Triplanar-mapping queries: a unit sphere at the origin seen by a
    pinhole camera at (0.3, 0.2, distance) looking at the origin.  One query
    per pixel whose ray hits the sphere, in :func:`tile_order`:
    ``[n, 8]`` float32 {p.x, p.y, p.z, n.x, n.y, n.z, lambda, 0}, with n = p
    (unit normal) and lambda = log2 of the pixel's footprint on the surface
    in level-0 texels (texture scale ``scale`` repeats per world unit),
    ``tex_size * scale * t * pixel_angle / |n . d|``, clamped to
    [0, levels-1]; float64 throughout."""
    eye = np.array([0.3, 0.2, distance])
    fwd = -eye / np.linalg.norm(eye)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    tw = th * width / height
    order = tile_order(width, height, tile)
    px = (order % width).astype(np.float64)
    py = (order // width).astype(np.float64)
    sx = (2.0 * (px + 0.5) / width - 1.0) * tw
    sy = (1.0 - 2.0 * (py + 0.5) / height) * th
    d = fwd[None] + sx[:, None] * right[None] + sy[:, None] * up[None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    b = d @ eye
    disc = b * b - (eye @ eye - 1.0)
    hit = disc > 0
    t = -b[hit] - np.sqrt(disc[hit])
    p = eye[None] + t[:, None] * d[hit]
    nrm = p / np.linalg.norm(p, axis=1, keepdims=True)
    cosv = np.abs(np.sum(nrm * d[hit], axis=1))
    pix = 2.0 * th / height
    foot = tex_size * scale * t * pix / np.maximum(cosv, 1e-3)
    lam = np.clip(np.log2(foot), 0.0, levels - 1)
    q = np.zeros((p.shape[0], 8), dtype=np.float32)
    q[:, 0:3] = p
    q[:, 3:6] = nrm
    q[:, 6] = lam
    return q


# ----------------------------------------------------------------------------
# 3-D density grids
# ----------------------------------------------------------------------------

_MASK32 = 0xFFFFFFFF


def _lattice_value(ix, iy, iz, salt: int):
    """Integer hash of lattice coordinates -> float64 in [0,1).

    Works on int64 torch tensors; all arithmetic is masked to 32 bits so it
    is exact on any device.
    """
    h = (ix * 73856093) ^ (iy * 19349663) ^ (iz * 83492791) ^ (salt * 40503)
    h = h & _MASK32
    h = ((h ^ (h >> 16)) * 0x45D9F3B) & _MASK32
    h = ((h ^ (h >> 16)) * 0x45D9F3B) & _MASK32
    h = h ^ (h >> 16)
    return (h & 0xFFFFFF).double() * (1.0 / 16777216.0)


def _value_noise(x, y, z, salt: int):
    """Quintic-faded trilinear value noise on the integer lattice."""
    import torch
    fx, fy, fz = torch.floor(x), torch.floor(y), torch.floor(z)
    ix, iy, iz = fx.long(), fy.long(), fz.long()
    tx, ty, tz = x - fx, y - fy, z - fz

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    ux, uy, uz = fade(tx), fade(ty), fade(tz)
    acc = torch.zeros_like(x)
    for dz in (0, 1):
        wz = uz if dz else 1.0 - uz
        for dy in (0, 1):
            wy = uy if dy else 1.0 - uy
            for dx in (0, 1):
                wx = ux if dx else 1.0 - ux
                acc = acc + wx * wy * wz * _lattice_value(ix + dx, iy + dy, iz + dz, salt)
    return acc


def cloud_grid(n: int = 512, seed: int = 4, device: str = "cpu", octaves: int = 6,
               base_cells: float = 4.0, sigma_max: float = 50.0, empty_frac: float = 0.30,
               chunk: int = 32):
    """Fractal-noise density cloud, ``[n, n, n]`` float16 torch tensor (z, y, x).

    fBm of value noise (``octaves`` octaves, lacunarity 2, gain 0.5, lowest
    octave ``base_cells`` cells across the grid) minus a radial falloff
    0.6*(r/r_max)^2 about the centre.  The ``empty_frac`` quantile theta of that
    field (over a strided sample of 2^27 voxels for larger grids) maps to exactly zero and sigma = sigma_max*((n-theta)/(n_max-theta))^2
    above it, so about ``empty_frac`` of the voxels are exact zeros and sigma
    lies in [0, sigma_max].  Computed in float64, rounded once to float16.
    """
    import torch
    dev = torch.device(device)
    coords = (torch.arange(n, dtype=torch.float64, device=dev) + 0.5) / n
    field = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    norm = sum(0.5 ** o for o in range(octaves))
    rmax = math.sqrt(3.0) * 0.5
    for z0 in range(0, n, chunk):
        z1 = min(n, z0 + chunk)
        zz, yy, xx = torch.meshgrid(coords[z0:z1], coords, coords, indexing="ij")
        acc = torch.zeros_like(xx)
        for o in range(octaves):
            f = base_cells * (2.0 ** o)
            acc = acc + (0.5 ** o) * _value_noise(xx * f, yy * f, zz * f, seed * 97 + o)
        r2 = (xx - 0.5) ** 2 + (yy - 0.5) ** 2 + (zz - 0.5) ** 2
        field[z0:z1] = acc / norm - 0.6 * r2 / (rmax * rmax)
    flat = field.reshape(-1)
    if flat.numel() > (1 << 27):
        # beyond 2^27 voxels the quantile is taken on an evenly strided sample
        # of 2^27 of them
        flat_q = flat[:: flat.numel() >> 27].contiguous()
    else:
        flat_q = flat
    k = max(1, int(round(empty_frac * flat_q.numel())))
    theta = torch.kthvalue(flat_q.cpu() if dev.type == "cpu" else flat_q, k).values
    nmax = flat.max()
    sig = torch.clamp(field - theta, min=0.0) / (nmax - theta)
    sig = sigma_max * sig * sig
    return sig.to(torch.float16)


def temperature_grid(density, t_min: float = 800.0, t_max: float = 6000.0):
    """Temperature field (kelvin, float16, same shape) of a fire shaped like a
    density cloud: 0 where the density is 0 (no emission), else
    t_min + (t_max - t_min) sqrt(sigma / max sigma).  Computed in float32,
    rounded once to float16 (spacing 4 K near 6000 K)."""
    import torch
    d = density.to(torch.float32)
    peak = float(d.max())
    T = t_min + (t_max - t_min) * torch.sqrt(d / peak if peak > 0 else d)
    return torch.where(d > 0, T, torch.zeros_like(T)).to(torch.float16)


def volume_level(grid, level: int):
    """Level ``level`` of a 3-D MIP pyramid of a grid [nz, ny, nx] (sides
    divisible by 2^level): means of 2^level-cubes, in float32, rounded once
    to the grid's dtype — the prefiltered volume a filter-before renderer
    minifies with."""
    import torch
    k = 1 << level
    x = grid.to(torch.float32)[None, None]
    return torch.nn.functional.avg_pool3d(x, kernel_size=k, stride=k)[0, 0].to(grid.dtype).contiguous()


def ortho_pixel_width(pixels: int, side: float, direction=(0.3, 0.2, 1.0)) -> float:
    """World width of one pixel of :func:`ortho_rays`' image plane."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    a = np.cross(d, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(a, d)
    corners = np.array([[x, y, z] for x in (0, side) for y in (0, side) for z in (0, side)], dtype=np.float64)
    pa, pb = corners @ a, corners @ b
    return float(max(pa.max() - pa.min(), pb.max() - pb.min()) / pixels)


def constant_grid(n: int, value: float, device: str = "cpu"):
    import torch
    return torch.full((n, n, n), value, dtype=torch.float16, device=device)


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------


def _clip_box(o: np.ndarray, d: np.ndarray, lo: np.ndarray, hi: np.ndarray):
    """Slab test in float64; returns (t0, t1), with t1 <= t0 for a miss."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        ta = (lo[None] - o) * inv
        tb = (hi[None] - o) * inv
    tmin = np.minimum(ta, tb)
    tmax = np.maximum(ta, tb)
    t0 = np.max(tmin, axis=1)
    t1 = np.min(tmax, axis=1)
    t0 = np.maximum(t0, 0.0)
    return t0, t1


def ortho_rays(pixels: int = 256, spp: int = 16, side: float = 0.25, seed: int = 11,
               direction=(0.3, 0.2, 1.0), strata: int = 4, gauss_px: float | None = None) -> np.ndarray:
    """Orthographic rays through the cube [0, side]^3.

    The image plane is perpendicular to ``direction`` and its square extent
    covers the cube's projection; ``pixels x pixels`` pixels, ``spp`` rays per
    pixel, jittered within a ``strata x strata`` grid of strata (``spp`` must
    be a multiple of strata^2); ``strata = 0`` puts every ray through its
    pixel's centre, and ``gauss_px`` instead offsets each ray from the
    centre by a 2-D normal of that standard deviation in pixels (a Gaussian
    pixel filter).  Rays are clipped to the cube in float64.
    Output ``[pixels*pixels*spp, 8]`` float32 rows
    ``{ox, oy, oz, dx, dy, dz, t0, t1}``, d of unit length, ordered by pixel in
    8x8-tile Morton order with the ``spp`` rays of one pixel consecutive.  A
    ray that misses the cube has t0 = t1 = 0.
    """
    rng = np.random.default_rng(seed)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    # orthonormal frame (a, b) of the image plane
    a = np.cross(d, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(a, d)
    corners = np.array([[x, y, z] for x in (0, side) for y in (0, side) for z in (0, side)], dtype=np.float64)
    pa, pb = corners @ a, corners @ b
    ext = max(pa.max() - pa.min(), pb.max() - pb.min())
    ca, cb = 0.5 * (pa.max() + pa.min()), 0.5 * (pb.max() + pb.min())
    back = (corners @ d).min() - side          # plane behind the cube

    order = tile_order(pixels, pixels, 8)
    px = (order % pixels).astype(np.float64)
    py = (order // pixels).astype(np.float64)
    s = np.arange(spp)
    if gauss_px is not None:
        off = rng.normal(size=(order.size, spp, 2)) * gauss_px
        fx = (px[:, None] + 0.5 + off[..., 0]) / pixels - 0.5
        fy = (py[:, None] + 0.5 + off[..., 1]) / pixels - 0.5
    elif strata == 0:
        fx = np.broadcast_to((px[:, None] + 0.5) / pixels - 0.5, (order.size, spp))
        fy = np.broadcast_to((py[:, None] + 0.5) / pixels - 0.5, (order.size, spp))
    else:
        sx = (s % strata).astype(np.float64)
        sy = ((s // strata) % strata).astype(np.float64)
        jit = rng.random((order.size, spp, 2))
        fx = (px[:, None] + (sx[None] + jit[..., 0]) / strata) / pixels - 0.5
        fy = (py[:, None] + (sy[None] + jit[..., 1]) / strata) / pixels - 0.5
    fa = ca + fx.ravel() * ext
    fb = cb + fy.ravel() * ext
    o = fa[:, None] * a[None] + fb[:, None] * b[None] + back * d[None]
    dd = np.broadcast_to(d, o.shape)
    t0, t1 = _clip_box(o, dd, np.zeros(3), np.full(3, side))
    miss = ~(t1 > t0)
    t0[miss] = 0.0
    t1[miss] = 0.0
    rays = np.empty((o.shape[0], 8), dtype=np.float32)
    rays[:, :3] = o
    rays[:, 3:6] = dd
    rays[:, 6] = t0
    rays[:, 7] = t1
    return rays


def offset_rays(rays: np.ndarray, sigma: float, count: int, seed: int) -> np.ndarray:
    """``count`` copies of every ray ``[n, 8]``, each with its origin moved by
    a 2-D normal offset of standard deviation ``sigma`` (world units) in the
    plane perpendicular to its direction, the segment [t0, t1] kept (a
    Gaussian pixel footprint realised by whole rays).  ``[n*count, 8]``,
    the copies of one ray consecutive."""
    rng = np.random.default_rng(seed)
    r = np.repeat(np.asarray(rays, dtype=np.float64), count, axis=0)
    d = r[:, 3:6]
    helper = np.where(np.abs(d[:, 1:2]) < 0.9, np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(d, helper)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(d, e1)
    g = rng.normal(size=(r.shape[0], 2)) * sigma
    r[:, :3] += g[:, :1] * e1 + g[:, 1:] * e2
    return r.astype(np.float32)


def random_rays(n: int, side: float, seed: int) -> np.ndarray:
    """Rays between two uniform points on the cube's boundary region, for
    parity tests: origin uniform in the cube, direction uniform on the sphere,
    clipped to the cube (float64), float32 output as :func:`ortho_rays`."""
    rng = np.random.default_rng(seed)
    o = rng.random((n, 3)) * side
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t0, t1 = _clip_box(o - 2.0 * side * d, d, np.zeros(3), np.full(3, side))
    o = o - 2.0 * side * d
    miss = ~(t1 > t0)
    t0[miss] = 0.0
    t1[miss] = 0.0
    rays = np.empty((n, 8), dtype=np.float32)
    rays[:, :3] = o
    rays[:, 3:6] = d
    rays[:, 6] = t0
    rays[:, 7] = t1
    return rays


def random_points(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (lo + (hi - lo) * rng.random((n, 3))).astype(np.float32)
