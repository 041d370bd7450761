"""Python binding of libsf (stochastic texture filtering on MI355X).

Thin ctypes marshalling over the C ABI declared in ``include/sf.h``: every
function here has the name of the C entry point it calls, checks tensor
dtype / device / contiguity, builds the descriptor structs and passes device
pointers plus the current HIP stream.  All computation runs in the HIP
kernels of ``libsf.so``; there is no fallback path, and importing a function
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsf.so")

# enums (values fixed by include/sf.h)
SF_OK, SF_E_NULL, SF_E_RANGE, SF_E_UNSUPPORTED, SF_E_DEVICE, SF_E_WORKSPACE = range(6)
SF_NEAREST, SF_LINEAR, SF_BSPLINE3, SF_KEYS3, SF_GAUSS_FRS, SF_GAUSS_FIS, SF_BSPLINE3_FIS, SF_EWA, SF_MITCHELL = range(9)
SF_MAX_ANISO, SF_EWA_MAX_ANISO, SF_EWA_MAX_ASPECT = 64, 16, 8
SF_SIGMA_MIN, SF_SIGMA_MAX = 0.0625, 4.0
SF_BEFORE, SF_AFTER_EXACT, SF_STOCHASTIC, SF_SPLIT = 0, 1, 2, 3
SF_RGBA32F, SF_RGBA8_UNORM, SF_R16F, SF_R32F, SF_DCT8 = 0, 1, 2, 3, 4
SF_WRAP_REPEAT, SF_WRAP_CLAMP = 0, 1
SF_MIP_NONE, SF_MIP_NEAREST, SF_MIP_LINEAR = 0, 1, 2
SF_SHADE_NONE, SF_SHADE_GGX, SF_SHADE_GGX_NORMAL = 0, 1, 2
SF_SHADE_DENSITY, SF_SHADE_TRANSMITTANCE, SF_SHADE_PLANCK = 0, 1, 2
PLANCK_NM = (700.0, 546.1, 435.8)
SF_TAP_NONE = -(2 ** 31)
SF_MAX_LEVELS = 16

EXPORTED = ("sf_filter2d", "sf_filter2d_aniso", "sf_dct_layout", "sf_dct_encode", "sf_triplanar",
            "sf_filter3d", "sf_raymarch", "sf_raymarch_emission", "sf_build_occupancy",
            "sf_occupancy_words", "sf_mlp_nparams", "sf_neural_decode", "sf_neural_raymarch", "sf_neural_decode_lattice", "sf_to_bf16",
            "sf_neural_quantize", "sf_neural_train_step", "sf_neural_train_workspace",
            "sf_error_stats", "sf_error_stats_workspace", "sf_error_stats_noalloc",
            "sf_error_stats_noalloc_max_bytes", "sf_last_error", "sf_abi_version", "sf_rng_version")
SF_LATENT_F32, SF_LATENT_BF16, SF_LATENT_FP8E4M3 = 0, 1, 2
SF_TRAIN_BF16, SF_TRAIN_FP32 = 0, 1


class sf_sampling(C.Structure):
    _fields_ = [("filter", C.c_int32), ("mode", C.c_int32), ("spp", C.c_int32), ("seed", C.c_uint32),
                ("rng_variant", C.c_int32), ("sigma", C.c_float)]


class sf_tex2d(C.Structure):
    _fields_ = [("base", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32), ("levels", C.c_int32),
                ("format", C.c_int32), ("wrap", C.c_int32), ("mip", C.c_int32),
                ("level_offset", C.c_int64 * SF_MAX_LEVELS), ("dct_range", C.c_void_p)]


class sf_ggx(C.Structure):
    _fields_ = [("n", C.c_float * 3), ("wo", C.c_float * 3), ("wi", C.c_float * 3), ("radiance", C.c_float * 3),
                ("f0", C.c_float), ("r_bias", C.c_float), ("r_scale", C.c_float)]


class sf_volume(C.Structure):
    _fields_ = [("base", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("format", C.c_int32), ("wmin", C.c_float * 3), ("scale", C.c_float * 3),
                ("occupancy", C.c_void_p), ("brick_log2", C.c_int32), ("reserved", C.c_int32)]


class sf_latent_grid(C.Structure):
    _fields_ = [("latents", C.c_void_p), ("block_scale", C.c_void_p), ("dims", C.c_int32), ("res", C.c_int32 * 3),
                ("channels", C.c_int32), ("format", C.c_int32), ("block_log2", C.c_int32),
                ("wmin", C.c_float * 3), ("scale", C.c_float * 3)]


class sf_mlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("in_dim", C.c_int32), ("hidden", C.c_int32), ("out_dim", C.c_int32),
                ("reserved", C.c_int32)]


class sf_train_state(C.Structure):
    _fields_ = [("latents", C.c_void_p), ("params", C.c_void_p), ("m_latents", C.c_void_p),
                ("v_latents", C.c_void_p), ("m_params", C.c_void_p), ("v_params", C.c_void_p),
                ("n_lattice", C.c_int64), ("channels", C.c_int32), ("hidden", C.c_int32), ("out_dim", C.c_int32),
                ("compute", C.c_int32)]


class SFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsf status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libsf.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2407_06107_amd.build.build() "
                              "(hipcc, gfx950).  There is no CPU fallback.")
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.sf_filter2d.argtypes = [P, P, i64, P, i32, P, P, P, P]
        L.sf_filter2d_aniso.argtypes = [P, P, i64, P, i32, i32, P, P, P, P]
        L.sf_dct_layout.argtypes = [i32, i32, i32, P]
        L.sf_dct_layout.restype = i64
        L.sf_dct_encode.argtypes = [P, P, P, P, P]
        L.sf_triplanar.argtypes = [P, P, i64, P, C.c_float, i32, i32, P, P, P, P]
        L.sf_filter3d.argtypes = [P, P, i64, P, i32, C.c_float, P, P, P]
        L.sf_raymarch.argtypes = [P, P, i64, i32, P, P, P, P]
        L.sf_raymarch_emission.argtypes = [P, P, i64, i32, P, C.c_float, P, P, P]
        L.sf_error_stats.argtypes = [P, P, i64, i32, P, P, C.c_size_t, P]
        L.sf_build_occupancy.argtypes = [P, P, i64, P]
        L.sf_build_occupancy.restype = i32
        L.sf_occupancy_words.argtypes = [i32, i32, i32, i32]
        L.sf_occupancy_words.restype = i64
        L.sf_mlp_nparams.argtypes = [i32, i32, i32]
        L.sf_mlp_nparams.restype = i64
        L.sf_neural_decode.argtypes = [P, P, P, i64, P, i32, P, P, P, P]
        L.sf_neural_raymarch.argtypes = [P, P, P, i64, i32, P, P, P, P]
        L.sf_neural_decode_lattice.argtypes = [P, P, P, i64, P, P]
        L.sf_to_bf16.argtypes = [P, i64, P, P]
        L.sf_neural_quantize.argtypes = [P, P, P, P, P]
        L.sf_neural_train_step.argtypes = [P, P, P, i64, i32, C.c_float, C.c_float, P, P, P, P, C.c_size_t, P]
        L.sf_neural_train_workspace.argtypes = [i32, i32, i64]
        L.sf_neural_train_workspace.restype = C.c_size_t
        for f in ("sf_neural_decode", "sf_neural_raymarch", "sf_neural_decode_lattice", "sf_to_bf16",
                  "sf_neural_quantize", "sf_neural_train_step"):
            getattr(L, f).restype = i32
        L.sf_error_stats_noalloc.argtypes = [P, P, i64, i32, P, P]
        L.sf_error_stats_noalloc.restype = i32
        L.sf_error_stats_noalloc_max_bytes.argtypes = []
        L.sf_error_stats_noalloc_max_bytes.restype = C.c_size_t
        L.sf_error_stats_workspace.argtypes = [i64]
        L.sf_error_stats_workspace.restype = C.c_size_t
        for f in ("sf_filter2d", "sf_filter2d_aniso", "sf_dct_encode", "sf_triplanar", "sf_filter3d", "sf_raymarch",
                  "sf_error_stats"):
            getattr(L, f).restype = i32
        L.sf_last_error.restype = C.c_char_p
        L.sf_abi_version.restype = i32
        L.sf_rng_version.restype = i32
        _lib = L
    return _lib


def sf_last_error() -> str:
    return lib().sf_last_error().decode()


def sf_abi_version() -> int:
    return int(lib().sf_abi_version())


def sf_rng_version() -> int:
    return int(lib().sf_rng_version())


def _check(status: int):
    if status != SF_OK:
        raise SFError(status, sf_last_error())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, dtype, name: str, numel: int | None = None):
    """Type, device, layout and (for buffers the library writes) size checks:
    the C ABI trusts the sizes it is given."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")


def sampling(filter: int, mode: int, spp: int = 1, seed: int = 0, rng_variant: int = 0,
             sigma: float = 0.5) -> sf_sampling:
    """``sigma``: standard deviation (texels) of the Gaussian filters."""
    return sf_sampling(filter, mode, spp, seed & 0xFFFFFFFF, rng_variant, sigma)


def ggx(n=(0.0, 0.0, 1.0), wo=(0.2, 0.3, 1.0), wi=(-0.4, 0.1, 1.0), radiance=(1.0, 1.0, 1.0), f0=0.04,
        r_bias=0.05, r_scale=0.95) -> sf_ggx:
    """GGX + Lambert parameters; direction vectors are normalised here."""
    import math

    def nrm(v):
        ln = math.sqrt(sum(x * x for x in v))
        return (C.c_float * 3)(*[x / ln for x in v])
    return sf_ggx(nrm(n), nrm(wo), nrm(wi), (C.c_float * 3)(*radiance), f0, r_bias, r_scale)


class Texture2D:
    """A device texture: one byte buffer holding every level plus its
    descriptor.  ``levels`` is a list of [h, w, 4] arrays (float32 or uint8)."""

    def __init__(self, levels, wrap: int = SF_WRAP_REPEAT, mip: int = SF_MIP_NONE, device="cuda"):
        import numpy as np
        levels = [np.ascontiguousarray(lv) for lv in levels]
        dt = levels[0].dtype
        if dt == np.float32:
            fmt, align = SF_RGBA32F, 16
        elif dt == np.uint8:
            fmt, align = SF_RGBA8_UNORM, 4
        else:
            raise TypeError("levels must be float32 or uint8 RGBA arrays")
        offs, cur = [], 0
        for lv in levels:
            offs.append(cur)
            cur += (lv.nbytes + 255) // 256 * 256
        buf = np.zeros(cur, dtype=np.uint8)
        for lv, o in zip(levels, offs):
            buf[o:o + lv.nbytes] = np.frombuffer(lv.tobytes(), dtype=np.uint8)
        self.buffer = torch.from_numpy(buf).to(device)
        self.offsets = offs
        self.desc = sf_tex2d()
        self.desc.base = self.buffer.data_ptr()
        self.desc.width, self.desc.height = levels[0].shape[1], levels[0].shape[0]
        self.desc.levels = len(levels)
        self.desc.format = fmt
        self.desc.wrap = wrap
        self.desc.mip = mip
        for i, o in enumerate(offs):
            self.desc.level_offset[i] = o
        del align

    @classmethod
    def dct(cls, src: "Texture2D", stream=None) -> "Texture2D":
        """Compress an RGBA8 device texture into SF_DCT8 (sf_dct_encode)."""
        if src.desc.format != SF_RGBA8_UNORM:
            raise TypeError("the DCT compressor takes an RGBA8 texture")
        d = src.desc
        offs = (C.c_int64 * SF_MAX_LEVELS)()
        nbytes = sf_dct_layout(d.width, d.height, d.levels, offs)
        dev = src.buffer.device
        self = cls.__new__(cls)
        self.buffer = torch.zeros(max(nbytes, 16), dtype=torch.uint8, device=dev)
        self.ranges = torch.zeros(4 * d.levels, dtype=torch.float32, device=dev)
        self.offsets = [offs[i] for i in range(d.levels)]
        self.desc = sf_tex2d()
        self.desc.base = self.buffer.data_ptr()
        self.desc.width, self.desc.height, self.desc.levels = d.width, d.height, d.levels
        self.desc.format, self.desc.wrap, self.desc.mip = SF_DCT8, d.wrap, d.mip
        for i in range(d.levels):
            self.desc.level_offset[i] = offs[i]
        self.desc.dct_range = self.ranges.data_ptr()
        _check(lib().sf_dct_encode(C.byref(d), _ptr(self.buffer), offs, _ptr(self.ranges), _stream(stream)))
        self.source = src
        return self

    def with_sampling(self, wrap: int | None = None, mip: int | None = None) -> "Texture2D":
        """The same texture memory with another wrap or MIP mode."""
        t = Texture2D.__new__(Texture2D)
        t.__dict__.update(self.__dict__)
        t.desc = sf_tex2d.from_buffer_copy(self.desc)
        if wrap is not None:
            t.desc.wrap = wrap
        if mip is not None:
            t.desc.mip = mip
        return t


def sf_dct_layout(width: int, height: int, levels: int, level_offset=None) -> int:
    """Bytes of an SF_DCT8 pyramid; fills ``level_offset`` (c_int64 array)."""
    n = int(lib().sf_dct_layout(width, height, levels, level_offset))
    if n < 0:
        raise ValueError("texture size or level count out of range")
    return n


class Volume:
    """A device density grid [nz, ny, nx] (float16 or float32) over the world
    box starting at ``wmin`` with ``scale`` voxels per unit.  With
    ``brick_log2`` set, an occupancy mask is built (sf_build_occupancy) and
    the ray march skips empty bricks."""

    def __init__(self, data: torch.Tensor, wmin=(0.0, 0.0, 0.0), scale=None, side: float = 1.0,
                 brick_log2: int | None = None, stream=None):
        if data.dtype not in (torch.float16, torch.float32):
            raise TypeError("volume must be float16 or float32")
        if not data.is_cuda or not data.is_contiguous() or data.dim() != 3:
            raise ValueError("volume must be a contiguous 3-D device tensor")
        self.data = data
        nz, ny, nx = data.shape
        if scale is None:
            scale = (nx / side, ny / side, nz / side)
        self.desc = sf_volume(data.data_ptr(), nx, ny, nz, SF_R16F if data.dtype == torch.float16 else SF_R32F,
                              (C.c_float * 3)(*wmin), (C.c_float * 3)(*scale), None, 0, 0)
        self.occupancy = None
        if brick_log2 is not None:
            self.occupancy = sf_build_occupancy(self, brick_log2, stream=stream)
            self.desc.occupancy = self.occupancy.data_ptr()
            self.desc.brick_log2 = brick_log2


def sf_filter2d(tex: Texture2D, queries: torch.Tensor, smp: sf_sampling, shade: int = SF_SHADE_NONE,
                ggx_params: sf_ggx | None = None, out: torch.Tensor | None = None,
                dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    _need(queries, torch.float32, "queries")
    n = queries.numel() // 3
    ch = 3 if shade != SF_SHADE_NONE else 4
    if out is None:
        out = torch.empty((n, ch), dtype=torch.float32, device=queries.device)
    _need(out, torch.float32, "out", n * ch)
    if dbg_taps is not None:
        tw = 5 if (smp.filter in (SF_KEYS3, SF_MITCHELL) and smp.mode == SF_STOCHASTIC) else 3
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * tw)
    g = C.byref(ggx_params) if ggx_params is not None else None
    _check(lib().sf_filter2d(C.byref(tex.desc), _ptr(queries), n, C.byref(smp), shade, g, _ptr(out),
                             _ptr(dbg_taps), _stream(stream)))
    return out


def sf_filter2d_aniso(tex: Texture2D, queries: torch.Tensor, smp: sf_sampling, aniso_max: int = 64,
                      shade: int = SF_SHADE_NONE, ggx_params: sf_ggx | None = None, out: torch.Tensor | None = None,
                      dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Anisotropic minification; queries ``[n, 6]`` {u, v, du/dx, dv/dx, du/dy, dv/dy}."""
    _need(queries, torch.float32, "queries")
    if queries.numel() % 6:
        raise ValueError("queries must hold 6 floats per pixel")
    n = queries.numel() // 6
    ch = 3 if shade != SF_SHADE_NONE else 4
    if out is None:
        out = torch.empty((n, ch), dtype=torch.float32, device=queries.device)
    _need(out, torch.float32, "out", n * ch)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * 3)
    g = C.byref(ggx_params) if ggx_params is not None else None
    _check(lib().sf_filter2d_aniso(C.byref(tex.desc), _ptr(queries), n, C.byref(smp), aniso_max, shade, g,
                                   _ptr(out), _ptr(dbg_taps), _stream(stream)))
    return out


def sf_triplanar(tex: Texture2D, queries: torch.Tensor, smp: sf_sampling, tex_scale: float = 1.0,
                 plane_mode: int = 1, shade: int = SF_SHADE_NONE, ggx_params: sf_ggx | None = None,
                 out: torch.Tensor | None = None, dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Triplanar mapping; queries ``[n, 8]`` {p, n, lambda, unused}."""
    _need(queries, torch.float32, "queries")
    if queries.numel() % 8:
        raise ValueError("queries must hold 8 floats per point")
    n = queries.numel() // 8
    ch = 3 if shade == SF_SHADE_GGX else 4
    if out is None:
        out = torch.empty((n, ch), dtype=torch.float32, device=queries.device)
    _need(out, torch.float32, "out", n * ch)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * 4)
    g = C.byref(ggx_params) if ggx_params is not None else None
    _check(lib().sf_triplanar(C.byref(tex.desc), _ptr(queries), n, C.byref(smp), tex_scale, plane_mode, shade, g,
                              _ptr(out), _ptr(dbg_taps), _stream(stream)))
    return out


def sf_filter3d(vol: Volume, pos: torch.Tensor, smp: sf_sampling, shade: int = SF_SHADE_DENSITY, ds: float = 1.0,
                out: torch.Tensor | None = None, dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    _need(pos, torch.float32, "pos")
    n = pos.numel() // 3
    ch = 3 if shade == SF_SHADE_PLANCK else 1
    if out is None:
        out = torch.empty((n, 3) if ch == 3 else n, dtype=torch.float32, device=pos.device)
    _need(out, torch.float32, "out", n * ch)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * 3)
    _check(lib().sf_filter3d(C.byref(vol.desc), _ptr(pos), n, C.byref(smp), shade, ds, _ptr(out), _ptr(dbg_taps),
                             _stream(stream)))
    return out


def sf_raymarch(vol: Volume, rays: torch.Tensor, steps: int, smp: sf_sampling, T: torch.Tensor | None = None,
                dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    _need(rays, torch.float32, "rays")
    n = rays.numel() // 8
    if T is None:
        T = torch.empty(n, dtype=torch.float32, device=rays.device)
    _need(T, torch.float32, "T", n)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * steps * 3)
    _check(lib().sf_raymarch(C.byref(vol.desc), _ptr(rays), n, steps, C.byref(smp), _ptr(T), _ptr(dbg_taps),
                             _stream(stream)))
    return T


def sf_raymarch_emission(vol: Volume, rays: torch.Tensor, steps: int, smp: sf_sampling, footprint: float = 0.0,
                         L: torch.Tensor | None = None, dbg_taps: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """Black-body emission gathered along rays through a temperature grid:
    [n, 3] float32 at PLANCK_NM; ``footprint`` > 0 samples a Gaussian pixel
    footprint perpendicular to the ray (stochastic mode)."""
    _need(rays, torch.float32, "rays")
    n = rays.numel() // 8
    if L is None:
        L = torch.empty((n, 3), dtype=torch.float32, device=rays.device)
    _need(L, torch.float32, "L", 3 * n)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * steps * 3)
    _check(lib().sf_raymarch_emission(C.byref(vol.desc), _ptr(rays), n, steps, C.byref(smp), float(footprint),
                                      _ptr(L), _ptr(dbg_taps), _stream(stream)))
    return L


def sf_occupancy_words(nx: int, ny: int, nz: int, brick_log2: int) -> int:
    return int(lib().sf_occupancy_words(nx, ny, nz, brick_log2))


def sf_build_occupancy(vol: Volume, brick_log2: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Brick occupancy mask of ``vol``: int32 words holding the padded bit
    mask of sf.h (one bit per brick, 1 = provably empty)."""
    d = vol.desc
    words = sf_occupancy_words(d.nx, d.ny, d.nz, brick_log2)
    if out is None:
        out = torch.zeros(max(words, 1), dtype=torch.int32, device=vol.data.device)
    _need(out, torch.int32, "out")
    desc = sf_volume(d.base, d.nx, d.ny, d.nz, d.format, d.wmin, d.scale, None, brick_log2, 0)
    _check(lib().sf_build_occupancy(C.byref(desc), _ptr(out), out.numel(), _stream(stream)))
    return out


def sf_error_stats_workspace(count: int) -> int:
    return int(lib().sf_error_stats_workspace(count))


def sf_error_stats(est: torch.Tensor, ref: torch.Tensor, out: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Returns 8 float64 on the device: sum e^2, sum e, max|e|, max rel, count,
    sum ref^2, non-finite count, 0."""
    _need(est, torch.float32, "est")
    _need(ref, torch.float64, "ref")
    if est.numel() != ref.numel():
        raise ValueError("est and ref differ in size")
    count = est.numel()
    if out is None:
        out = torch.zeros(8, dtype=torch.float64, device=est.device)
    _need(out, torch.float64, "out", 8)
    if workspace is None:
        workspace = torch.empty(max(1, sf_error_stats_workspace(count)), dtype=torch.uint8, device=est.device)
    _check(lib().sf_error_stats(_ptr(est), _ptr(ref), count, 1, _ptr(out), _ptr(workspace), workspace.numel(),
                                _stream(stream)))
    return out


def sf_error_stats_noalloc_max_bytes() -> int:
    return int(lib().sf_error_stats_noalloc_max_bytes())


def sf_error_stats_noalloc(est: torch.Tensor, ref: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """sf_error_stats without a workspace: the library's static per-device
    scratch holds the partial rows, so the call allocates nothing (the caller
    passes `out`, 8 float64 on the device).  Calls that overlap on one device
    race."""
    _need(est, torch.float32, "est")
    _need(ref, torch.float64, "ref")
    if est.numel() != ref.numel():
        raise ValueError("est and ref differ in size")
    _need(out, torch.float64, "out", 8)
    _check(lib().sf_error_stats_noalloc(_ptr(est), _ptr(ref), est.numel(), 1, _ptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------ neural
def sf_mlp_nparams(in_dim: int, hidden: int, out_dim: int) -> int:
    return int(lib().sf_mlp_nparams(in_dim, hidden, out_dim))


def sf_to_bf16(x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """bfloat16 bits (int16 tensor) of a float32 tensor, round to nearest even."""
    _need(x, torch.float32, "x")
    if out is None:
        out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _need(out, torch.int16, "out", x.numel())
    _check(lib().sf_to_bf16(_ptr(x), x.numel(), _ptr(out), _stream(stream)))
    return out


class LatentGrid:
    """Device latent grid (BF16 or E4M3 + block scales) and its descriptor."""

    def __init__(self, dims, res, channels, fmt, latents, scales=None, block_log2=0, wmin=(0.0, 0.0, 0.0),
                 scale=(1.0, 1.0, 1.0)):
        self.latents, self.scales = latents, scales
        r = list(res) + [1] * (3 - len(res))
        self.desc = sf_latent_grid(latents.data_ptr(), scales.data_ptr() if scales is not None else None, dims,
                                   (C.c_int32 * 3)(*r), channels, fmt, block_log2, (C.c_float * 3)(*wmin),
                                   (C.c_float * 3)(*scale))


def sf_neural_quantize(latents: torch.Tensor, dims: int, res, channels: int, fmt: int, block_log2: int = 3,
                       wmin=(0.0, 0.0, 0.0), scale=(1.0, 1.0, 1.0), stream=None) -> LatentGrid:
    _need(latents, torch.float32, "latents")
    r = list(res) + [1] * (3 - len(res))
    npts = r[0] * r[1] * r[2]
    if latents.numel() != npts * channels:
        raise ValueError("latents do not match res x channels")
    if fmt == SF_LATENT_BF16:
        out = torch.empty(npts * channels, dtype=torch.int16, device=latents.device)
        scales = None
    elif fmt == SF_LATENT_FP8E4M3:
        out = torch.empty(npts * channels, dtype=torch.uint8, device=latents.device)
        B = 1 << block_log2
        nb = 1
        for a in range(dims):
            nb *= -(-r[a] // B)
        scales = torch.empty(nb, dtype=torch.float32, device=latents.device)
    else:
        raise ValueError("fmt must be SF_LATENT_BF16 or SF_LATENT_FP8E4M3")
    grid = LatentGrid(dims, r, channels, fmt, out, scales, block_log2 if fmt == SF_LATENT_FP8E4M3 else 0, wmin,
                      scale)
    _check(lib().sf_neural_quantize(_ptr(latents), C.byref(grid.desc), _ptr(out), _ptr(scales), _stream(stream)))
    return grid


class MLP:
    """BF16 packed MLP parameters for decoding."""

    def __init__(self, params_f32: torch.Tensor, in_dim: int, out_dim: int, hidden: int = 64, stream=None):
        _need(params_f32, torch.float32, "params")
        if params_f32.numel() != sf_mlp_nparams(in_dim, hidden, out_dim):
            raise ValueError("parameter count does not match the shape")
        self.bits = sf_to_bf16(params_f32, stream=stream)
        self.desc = sf_mlp(self.bits.data_ptr(), in_dim, hidden, out_dim, 0)


def sf_neural_decode(grid: LatentGrid, mlp: MLP, queries: torch.Tensor, smp: sf_sampling, shade: int = SF_SHADE_NONE,
                     ggx_params: sf_ggx | None = None, out: torch.Tensor | None = None,
                     dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    _need(queries, torch.float32, "queries")
    n = queries.numel() // 3
    ch = 3 if shade == SF_SHADE_GGX else 4
    if out is None:
        out = torch.empty((n, ch), dtype=torch.float32, device=queries.device)
    _need(out, torch.float32, "out", n * ch)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * 2)
    g = C.byref(ggx_params) if ggx_params is not None else None
    _check(lib().sf_neural_decode(C.byref(grid.desc), C.byref(mlp.desc), _ptr(queries), n, C.byref(smp), shade, g,
                                  _ptr(out), _ptr(dbg_taps), _stream(stream)))
    return out


def sf_neural_raymarch(grid: LatentGrid, mlp: MLP, rays: torch.Tensor, steps: int, smp: sf_sampling,
                       T: torch.Tensor | None = None, dbg_taps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    _need(rays, torch.float32, "rays")
    n = rays.numel() // 8
    if T is None:
        T = torch.empty(n, dtype=torch.float32, device=rays.device)
    _need(T, torch.float32, "T", n)
    if dbg_taps is not None:
        _need(dbg_taps, torch.int32, "dbg_taps", n * smp.spp * steps * 3)
    _check(lib().sf_neural_raymarch(C.byref(grid.desc), C.byref(mlp.desc), _ptr(rays), n, steps, C.byref(smp),
                                    _ptr(T), _ptr(dbg_taps), _stream(stream)))
    return T


def sf_neural_decode_lattice(grid: LatentGrid, mlp: MLP, idx: torch.Tensor, out: torch.Tensor | None = None,
                             stream=None) -> torch.Tensor:
    _need(idx, torch.int64, "idx")
    n = idx.numel()
    if out is None:
        out = torch.empty((n, mlp.desc.out_dim), dtype=torch.float32, device=idx.device)
    _need(out, torch.float32, "out", n * mlp.desc.out_dim)
    _check(lib().sf_neural_decode_lattice(C.byref(grid.desc), C.byref(mlp.desc), _ptr(idx), n, _ptr(out),
                                          _stream(stream)))
    return out


class TrainState:
    """FP32 master latents and MLP parameters with their Adam moments, the
    step count, and how the steps compute (SF_TRAIN_BF16 on the matrix cores,
    SF_TRAIN_FP32 on the vector ALU)."""

    def __init__(self, latents: torch.Tensor, params: torch.Tensor, channels: int, out_dim: int, hidden: int = 64,
                 compute: int = SF_TRAIN_BF16):
        _need(latents, torch.float32, "latents")
        _need(params, torch.float32, "params")
        if params.numel() != sf_mlp_nparams(channels, hidden, out_dim) or latents.numel() % channels:
            raise ValueError("latents or params do not match the shape")
        self.latents, self.params = latents, params
        self.m_lat, self.v_lat = torch.zeros_like(latents), torch.zeros_like(latents)
        self.m_par, self.v_par = torch.zeros_like(params), torch.zeros_like(params)
        self.channels, self.out_dim, self.hidden = channels, out_dim, hidden
        self.n_lattice = latents.numel() // channels
        self.step = 0
        self.compute = compute
        self._bind()
        self._ws = None

    def _bind(self):
        self.desc = sf_train_state(self.latents.data_ptr(), self.params.data_ptr(), self.m_lat.data_ptr(),
                                   self.v_lat.data_ptr(), self.m_par.data_ptr(), self.v_par.data_ptr(),
                                   self.n_lattice, self.channels, self.hidden, self.out_dim, self.compute)

    def save(self, path: str, seed: int = 0, stream=None):
        """Checkpoint: latents, parameters, both Adam moments (FP32, exact),
        the step count, the compute mode and the caller's batch-sampling
        seed, to an .npz file (no pickled objects)."""
        import numpy as np
        (stream or torch.cuda.current_stream()).synchronize()
        np.savez(path, latents=self.latents.cpu().numpy(), params=self.params.cpu().numpy(),
                 m_latents=self.m_lat.cpu().numpy(), v_latents=self.v_lat.cpu().numpy(),
                 m_params=self.m_par.cpu().numpy(), v_params=self.v_par.cpu().numpy(),
                 meta=np.array([self.step, self.channels, self.out_dim, self.hidden, self.compute, seed],
                               dtype=np.int64))

    @classmethod
    def load(cls, path: str, device="cuda"):
        """A state restored from save(); returns (state, seed).  Resuming and
        taking the same steps gives the same state, bit for bit, as never
        stopping."""
        import numpy as np
        z = np.load(path, allow_pickle=False)
        step, ch, od, hid, comp, seed = (int(v) for v in z["meta"])
        st = cls(torch.from_numpy(z["latents"]).to(device), torch.from_numpy(z["params"]).to(device), ch, od, hid,
                 comp)
        st.m_lat.copy_(torch.from_numpy(z["m_latents"]))
        st.v_lat.copy_(torch.from_numpy(z["v_latents"]))
        st.m_par.copy_(torch.from_numpy(z["m_params"]))
        st.v_par.copy_(torch.from_numpy(z["v_params"]))
        st.step = step
        return st, seed


def sf_neural_train_workspace(channels: int, out_dim: int, batch: int) -> int:
    return int(lib().sf_neural_train_workspace(channels, out_dim, batch))


def sf_neural_train_step(st: TrainState, batch_idx: torch.Tensor, targets: torch.Tensor, lr_latent: float,
                         lr_mlp: float, loss_out: torch.Tensor | None = None, grad_params: torch.Tensor | None = None,
                         grad_latents: torch.Tensor | None = None, step: int | None = None,
                         workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """One Adam step; returns the device loss tensor (1 float)."""
    _need(batch_idx, torch.int32, "batch_idx")
    _need(targets, torch.float32, "targets", st.n_lattice * st.out_dim)
    B = batch_idx.numel()
    if step is None:
        st.step += 1
        step = st.step
    if loss_out is None:
        loss_out = torch.empty(1, dtype=torch.float32, device=batch_idx.device)
    need = sf_neural_train_workspace(st.channels, st.out_dim, B)
    if workspace is None:
        if st._ws is None or st._ws.numel() < need:
            st._ws = torch.empty(max(need, 4), dtype=torch.uint8, device=batch_idx.device)
        workspace = st._ws
    _need(loss_out, torch.float32, "loss_out", 1)
    for t, name, k in ((grad_params, "grad_params", st.params.numel()), (grad_latents, "grad_latents",
                                                                         B * st.channels)):
        if t is not None:
            _need(t, torch.float32, name, k)
    _check(lib().sf_neural_train_step(C.byref(st.desc), _ptr(batch_idx), _ptr(targets), B, step, lr_latent, lr_mlp,
                                      _ptr(loss_out), _ptr(grad_params), _ptr(grad_latents), _ptr(workspace),
                                      workspace.numel(), _stream(stream)))
    return loss_out
