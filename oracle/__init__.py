"""CPU oracle: ctypes wrapper around ``oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library; the two are fed the same inputs from
``paper_2407_06107_amd.inputs`` and compared.

All arrays here are host NumPy arrays.  Results are float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "neural.c")]
# ORACLE_SANITIZE=1 selects a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (errors abort); the process must then preload the
# compiler's libasan (a test runs the pins that way in a child process).
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

# enums of the oracle (its own copy; it does not include the library header)
NEAREST, LINEAR, BSPLINE3, KEYS3, GAUSS_FRS, GAUSS_FIS, BSPLINE3_FIS, EWA, MITCHELL = 0, 1, 2, 3, 4, 5, 6, 7, 8
SIGMA_MIN, SIGMA_MAX = 1.0 / 16.0, 4.0     # Gaussian standard deviation, texels
BEFORE, AFTER, STOCHASTIC, SPLIT = 0, 1, 2, 3
RGBA32F, RGBA8, R16F, R32F, DCT8 = 0, 1, 2, 3, 4
REPEAT, CLAMP = 0, 1
MIP_NONE, MIP_NEAREST, MIP_LINEAR = 0, 1, 2
TAP_NONE = np.iinfo(np.int32).min
DENSITY, TRANSMITTANCE, PLANCK = 0, 1, 2     # 3-D shading
SHADE_NONE, SHADE_GGX, SHADE_GGX_NORMAL = 0, 1, 2   # 2-D shading
PLANCK_NM = (700.0, 546.1, 435.8)           # wavelengths of an emission result


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (OpenMP, no FP contraction)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fvisibility=hidden", *(_SAN_FLAGS if _SANITIZE else []), *_SRCS, "-o", tmp,
               "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, u32, f32 = C.c_int, C.c_int64, C.c_uint32, C.c_float
        L.orc_kbs.restype = C.c_double
        L.orc_kbs.argtypes = [C.c_double]
        L.orc_ktent.restype = C.c_double
        L.orc_ktent.argtypes = [C.c_double]
        L.orc_thresholds.argtypes = [i32, f32, P]
        L.orc_pick.argtypes = [i32, f32, f32]
        L.orc_reuse.restype = f32
        L.orc_reuse.argtypes = [i32, f32, f32, i32]
        L.orc_pick_pmf.argtypes = [i32, f32, P]
        L.orc_axis_weights64.argtypes = [i32, C.c_double, P]
        L.orc_sample_array.argtypes = [P, i32, C.c_double]
        L.orc_half_to_double.restype = C.c_double
        L.orc_half_to_double.argtypes = [C.c_uint16]
        L.orc_pcg4d_batch.argtypes = [P, P, i64]
        L.orc_shade_ggx.argtypes = [P, P, P]
        L.orc_filter2d.argtypes = [P, i32, i32, i32, i32, i32, i32, P, P, P, i64, i32, i32, i32, u32,
                                   i32, f32, i32, P, P, P, P, i64]
        L.orc_filter2d_expect.argtypes = [P, i32, i32, i32, i32, i32, i32, P, P, P, i64, i32, f32, i32, P, P]
        L.orc_dct_basis32.argtypes = [i32, i32]
        L.orc_dct_basis32.restype = f32
        L.orc_dct_encode_level.argtypes = [P, i32, i32, P, P]
        L.orc_tri_pick.argtypes = [P, f32]
        L.orc_tri_pick.restype = i32
        L.orc_triplanar.argtypes = [P, i32, i32, i32, i32, i32, i32, P, P, P, i64, f32, i32, i32, i32, i32, u32,
                                    i32, P, P, P, P, i64]
        L.orc_lnc.argtypes = [f32]
        L.orc_lnc.restype = f32
        L.orc_expc.argtypes = [f32]
        L.orc_expc.restype = f32
        L.orc_elementary_batch.argtypes = [i32, P, P, P, i64]
        L.orc_fis_gauss_offset.argtypes = [f32, f32, f32, P, P]
        L.orc_fis_nearest.argtypes = [f32, f32]
        L.orc_fis_nearest.restype = i32
        L.orc_fis_bspline_pick.argtypes = [f32, u32, u32, u32]
        L.orc_fis_bspline_pick.restype = i32
        L.orc_fis_bspline_pmf.argtypes = [f32, P]
        L.orc_gauss_thresholds.argtypes = [f32, f32, P]
        L.orc_gauss_h.argtypes = [f32]
        L.orc_gauss_h.restype = f32
        L.orc_gauss_pick_pmf.argtypes = [f32, f32, P]
        L.orc_ewa_gauss.argtypes = [f32]
        L.orc_ewa_gauss.restype = f32
        L.orc_ewa_frame.argtypes = [P, i32, i32, i32, P]
        L.orc_ewa_lod.argtypes = [P, i32, i32, i32]
        L.orc_ewa_box.argtypes = [i32, i32, i32, P, i32, i32, P]
        L.orc_ewa_lod.restype = f32
        L.orc_ewa_pick_pmf.argtypes = [i32, i32, i32, i32, P, i32, i32, P, i32, P]
        L.orc_ewa_weights.argtypes = [i32, i32, i32, i32, P, i32, i32, P, i32]
        L.orc_log2c.argtypes = [f32]
        L.orc_log2c.restype = f32
        L.orc_aniso_lod.argtypes = [i32, i32, P, i32, P, P]
        L.orc_aniso_lod.restype = f32
        L.orc_filter2d_aniso.argtypes = [P, i32, i32, i32, i32, i32, P, P, P, i64, i32, i32, i32, u32, f32, i32,
                                         i32, P, P, P, P, i64]
        L.orc_aniso_reference.argtypes = [P, i32, i32, i32, i32, P, P, i64, i32, i32, f32, i32, P, P, P, i64]
        L.orc_reuse_histogram2.argtypes = [i32, f32, f32, P]
        L.orc_filter3d.argtypes = [P, i32, i32, i32, i32, P, P, P, i64, i32, i32, i32, u32, i32,
                                   i32, f32, P, P, P, i64]
        L.orc_raymarch.argtypes = [P, i32, i32, i32, i32, P, P, P, i64, i32, i32, i32, i32, u32, i32,
                                   P, P, P, i64]
        L.orc_raymarch_expect.argtypes = [P, i32, i32, i32, i32, P, P, P, i64, i32, i32, P]
        L.orc_raymarch_emission.argtypes = [P, i32, i32, i32, i32, P, P, P, i64, i32, i32, i32, i32, u32,
                                            i32, f32, P, P, P, i64]
        L.orc_perp_jitter.argtypes = [P, P, P, i32, f32, i64, i32, i32, u32, P]
        L.orc_raymarch_emission_expect.argtypes = [P, i32, i32, i32, i32, P, P, P, i64, i32, i32, P]
        L.orc_planck.argtypes = [C.c_double, C.c_double]
        L.orc_planck.restype = C.c_double
        L.orc_build_occupancy.argtypes = [P, i32, i32, i32, i32, i32, P]
        L.orc_k3.restype = C.c_double
        L.orc_k3.argtypes = [C.c_double]
        L.orc_keys_pick.argtypes = [f32, f32, P, P, P]
        L.orc_keys_expect2d.argtypes = [P, i32, i32, i32, i32, P, i64, i32, P, P]
        L.orc_shade_ggx_normal.argtypes = [P, P, P]
        L.orc_kmn.restype = C.c_double
        L.orc_kmn.argtypes = [C.c_double]
        L.orc_mitchell_pick.argtypes = [f32, f32, P, P, P]
        L.orc_mitchell_axis.argtypes = [f32, P, P, P]
        L.orc_mitchell_expect2d.argtypes = [P, i32, i32, i32, i32, P, i64, i32, P, P]
        L.orc_f32_to_bf16.restype = C.c_uint16
        L.orc_f32_to_bf16.argtypes = [f32]
        L.orc_bf16_to_double.restype = C.c_double
        L.orc_bf16_to_double.argtypes = [C.c_uint16]
        L.orc_fp8_to_double.restype = C.c_double
        L.orc_fp8_to_double.argtypes = [C.c_uint8]
        L.orc_f32_to_fp8.restype = C.c_uint8
        L.orc_f32_to_fp8.argtypes = [f32]
        L.orc_quantize_fp8.argtypes = [P, i32, P, i32, i32, P, P]
        L.orc_dequant_fp8.argtypes = [P, P, i64, i32, P]
        L.orc_mlp_forward.argtypes = [i32, i32, i32, P, P, i64, i32, P]
        L.orc_mlp_grad.restype = C.c_double
        L.orc_mlp_grad.argtypes = [i32, i32, i32, P, P, P, i64, i32, P, P]
        L.orc_adam.argtypes = [P, P, P, P, i64, i32, C.c_double]
        L.orc_neural_filter2d.argtypes = [i32, i32, i32, i32, i32, P, P, i32, P, i64, i32, i32, i32, u32, i32, P,
                                          P, P, P, i64]
        L.orc_neural_raymarch.argtypes = [i32, i32, i32, i32, i32, P, P, i32, P, P, P, i64, i32, i32, i32, i32,
                                          u32, P, P, P, i64]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- primitives
def pcg4d(keys: np.ndarray) -> np.ndarray:
    keys = _c(keys, np.uint32).reshape(-1, 4)
    out = np.empty_like(keys)
    lib().orc_pcg4d_batch(_p(keys), _p(out), keys.shape[0])
    return out


def kbs(x: float) -> float:
    return lib().orc_kbs(float(x))


def ktent(x: float) -> float:
    return lib().orc_ktent(float(x))


def thresholds(filt: int, t: float) -> np.ndarray:
    c = np.zeros(3, dtype=np.float32)
    n = lib().orc_thresholds(filt, float(t), _p(c))
    return c[:n]


def pick(filt: int, t: float, u: float) -> int:
    return int(lib().orc_pick(filt, float(t), float(u)))


def reuse(filt: int, t: float, u: float, j: int) -> float:
    return float(lib().orc_reuse(filt, float(t), float(u), int(j)))


def pick_pmf(filt: int, t: float) -> np.ndarray:
    p = np.zeros(4)
    lib().orc_pick_pmf(filt, float(t), _p(p))
    return p


def sample_array(w, xi: float) -> int:
    w = _c(w, np.float64).reshape(-1)
    return int(lib().orc_sample_array(_p(w), w.size, float(xi)))


def axis_weights64(filt: int, t: float) -> np.ndarray:
    w = np.zeros(4)
    lib().orc_axis_weights64(filt, float(t), _p(w))
    return w


def half_to_double(bits: int) -> float:
    return lib().orc_half_to_double(int(bits))


def ggx_params(n=(0.0, 0.0, 1.0), wo=(0.2, 0.3, 1.0), wi=(-0.4, 0.1, 1.0), radiance=(1.0, 1.0, 1.0),
               f0=0.04, r_bias=0.05, r_scale=0.95) -> np.ndarray:
    """16 doubles: n, wo, wi (normalised here), radiance, f0, r_bias, r_scale, 0."""
    def nrm(v):
        v = np.asarray(v, dtype=np.float64)
        return v / np.linalg.norm(v)
    p = np.zeros(16)
    p[0:3], p[3:6], p[6:9] = nrm(n), nrm(wo), nrm(wi)
    p[9:12] = radiance
    p[12], p[13], p[14] = f0, r_bias, r_scale
    return p


def shade_ggx(params: np.ndarray, rgba) -> np.ndarray:
    params = _c(params, np.float64)
    rgba = _c(rgba, np.float64)
    out = np.zeros(3)
    lib().orc_shade_ggx(_p(params), _p(rgba), _p(out))
    return out


def shade_ggx_normal(params: np.ndarray, rgba) -> np.ndarray:
    """GGX + Lambert of a grey material (albedo 1/2) with the tangent-space
    normal encoded in rgb (2 rgb - 1, renormalised), roughness parameter a."""
    params = _c(params, np.float64)
    rgba = _c(rgba, np.float64)
    out = np.zeros(3)
    lib().orc_shade_ggx_normal(_p(params), _p(rgba), _p(out))
    return out


def reuse_histogram2(filt: int, tx: float, ty: float) -> np.ndarray:
    c = np.zeros(16, dtype=np.int64)
    lib().orc_reuse_histogram2(filt, float(tx), float(ty), _p(c))
    return c.reshape(4, 4)


# ------------------------------------------------------------------ 2-D path
class Tex2D:
    """Host texture: packed level buffer + per-level byte offsets."""

    def __init__(self, buf: np.ndarray, w: int, h: int, levels: int, fmt: int, offsets,
                 wrap: int = REPEAT, mip: int = MIP_NONE, dct_range=None):
        self.buf = np.ascontiguousarray(buf).view(np.uint8).reshape(-1)
        self.w, self.h, self.levels, self.fmt = w, h, levels, fmt
        self.off = np.zeros(16, dtype=np.int64)
        self.off[:levels] = offsets
        self.wrap, self.mip = wrap, mip
        self.dct_range = None if dct_range is None else _c(dct_range, np.float32).reshape(-1)
        if fmt == DCT8 and (self.dct_range is None or self.dct_range.size < 4 * levels):
            raise ValueError("a DCT texture needs 4 AC ranges per level")

    @classmethod
    def dct(cls, levels, wrap: int = REPEAT, mip: int = MIP_NONE):
        """Encode RGBA8 levels (list of [h, w, 4] uint8) with the oracle's DCT
        encoder: blocks of each level at 256-byte aligned offsets."""
        chunks, offs, ranges, pos = [], [], [], 0
        for lv in levels:
            lv = _c(lv, np.uint8)
            hl, wl = lv.shape[:2]
            bw, bh = (wl + 7) // 8, (hl + 7) // 8
            blocks = np.zeros(bw * bh * 4, dtype=np.uint32)
            rng = np.zeros(4, dtype=np.float32)
            lib().orc_dct_encode_level(_p(lv), wl, hl, _p(blocks), _p(rng))
            pad = (-pos) % 256
            if pad:
                chunks.append(np.zeros(pad, np.uint8))
                pos += pad
            offs.append(pos)
            chunks.append(blocks.view(np.uint8))
            pos += blocks.nbytes
            ranges.append(rng)
        buf = np.concatenate(chunks) if chunks else np.zeros(0, np.uint8)
        w0, h0 = levels[0].shape[1], levels[0].shape[0]
        return cls(buf, w0, h0, len(levels), DCT8, offs, wrap, mip, np.concatenate(ranges))

    @classmethod
    def rgba32f(cls, tex: np.ndarray, wrap=REPEAT):
        tex = np.ascontiguousarray(tex, dtype=np.float32)
        return cls(tex, tex.shape[1], tex.shape[0], 1, RGBA32F, [0], wrap, MIP_NONE)


def _check_sigma(filt, sigma):
    if filt in (GAUSS_FRS, GAUSS_FIS) and not (SIGMA_MIN <= sigma <= SIGMA_MAX):
        raise ValueError(f"sigma {sigma} outside [{SIGMA_MIN}, {SIGMA_MAX}]")


def filter2d(tex: Tex2D, q: np.ndarray, filt: int, mode: int, spp: int = 1, seed: int = 0,
             variant: int = 0, shade: int = 0, ggx=None, taps: bool = False, subset=None, sigma: float = 0.5):
    """Filter every query, or only the rows listed in ``subset`` (their own
    index keys the random stream).  Taps: {level, x, y} per sample, or
    {level, x+, y+, x-, y-} for the positivised Keys cubic.  ``sigma``: the
    Gaussian filters' standard deviation in texels of the level read."""
    _check_sigma(filt, sigma)
    q = _c(q, np.float32).reshape(-1, 3)
    n = q.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    ch = 3 if shade else 4
    out = np.zeros((m, ch))
    tp = np.zeros((m, spp, 5 if (filt in (KEYS3, MITCHELL) and mode == STOCHASTIC) else 3), dtype=np.int32) \
        if taps else None
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_filter2d(_p(tex.buf), tex.w, tex.h, tex.levels, tex.fmt, tex.wrap, tex.mip, _p(tex.off),
                       _p(tex.dct_range), _p(q), n, filt, mode, spp, seed & 0xFFFFFFFF, variant, sigma, shade, _p(g), _p(out), _p(tp),
                       _p(sub), 0 if sub is None else sub.size)
    return (out, tp) if taps else out


def filter2d_expect(tex: Tex2D, q: np.ndarray, filt: int, shade: int = 0, ggx=None, sigma: float = 0.5):
    """Exact expectation of the stochastic estimator (not for KEYS3 or GAUSS_FIS)."""
    _check_sigma(filt, sigma)
    q = _c(q, np.float32).reshape(-1, 3)
    n = q.shape[0]
    ch = 3 if shade else 4
    out = np.zeros((n, ch))
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    st = lib().orc_filter2d_expect(_p(tex.buf), tex.w, tex.h, tex.levels, tex.fmt, tex.wrap, tex.mip,
                                   _p(tex.off), _p(tex.dct_range), _p(q), n, filt, sigma, shade, _p(g), _p(out))
    if st != 0:
        raise ValueError("no exact expectation for this filter")
    return out


# ------------------------------------------------------------------ anisotropic minification
def log2c(x: float) -> float:
    return lib().orc_log2c(x)


def aniso_lod(w: int, h: int, d, amax: int = 64):
    """(lambda, major axis is the y derivative, probe count)."""
    dd = _c(d, np.float32)
    my, npb = C.c_int(), C.c_int()
    lam = lib().orc_aniso_lod(w, h, _p(dd), amax, C.byref(my), C.byref(npb))
    return lam, bool(my.value), npb.value


def filter2d_aniso(tex: Tex2D, q: np.ndarray, filt: int, mode: int, spp: int = 1, seed: int = 0, shade: int = 0,
                   ggx=None, taps: bool = False, subset=None, sigma: float = 0.5, amax: int = 64):
    """Anisotropic minification (screen-space jitter + minor-axis level);
    queries ``[n, 6]`` {u, v, du/dx, dv/dx, du/dy, dv/dy}."""
    _check_sigma(filt, sigma)
    q = _c(q, np.float32).reshape(-1, 6)
    n = q.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    ch = 3 if shade else 4
    out = np.zeros((m, ch))
    tp = np.zeros((m, spp, 3), dtype=np.int32) if taps else None
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_filter2d_aniso(_p(tex.buf), tex.w, tex.h, tex.levels, tex.fmt, tex.wrap, _p(tex.off),
                             _p(tex.dct_range), _p(q), n, filt,
                             mode, spp, seed & 0xFFFFFFFF, sigma, amax, shade, _p(g), _p(out), _p(tp), _p(sub),
                             0 if sub is None else sub.size)
    return (out, tp) if taps else out


def ewa_gauss(r2: float) -> float:
    """The EWA weight e^(-2 r^2) - e^(-2) (0 for r^2 >= 1), binary32."""
    return float(lib().orc_ewa_gauss(float(r2)))


def ewa_frame(q, w: int, h: int, amax: int = 8) -> np.ndarray:
    """{lod, S_ss, S_tt, S_st, det S}: the footprint covariance in level-0
    texels after the anisotropy limit, binary32."""
    out = np.zeros(5, np.float32)
    lib().orc_ewa_frame(_p(_c(q, np.float32)), w, h, amax, _p(out))
    return out


def ewa_lod(q, w: int, h: int, amax: int = 8) -> float:
    """Level of detail of the EWA footprint: max(0, log2(shorter axis in
    level-0 texels)) after the anisotropy limit (binary32)."""
    return float(lib().orc_ewa_lod(_p(_c(q, np.float32)), w, h, amax))


def ewa_box(w: int, h: int, levels: int, q, level: int, amax: int = 8):
    """The ellipse's bounding box (s0, s1, t0, t1) at one level."""
    box = np.zeros(4, dtype=np.int32)
    lib().orc_ewa_box(w, h, levels, _p(_c(q, np.float32)), amax, level, _p(box))
    return tuple(int(b) for b in box)


def ewa_pick_pmf(w: int, h: int, levels: int, q, level: int, amax: int = 8, wrap: int = REPEAT, maxcells: int = 4096):
    """Exact pick probabilities of the inverse-CDF pick over the level's
    bounding box (all 2^24 uniforms), with the box (s0, s1, t0, t1)."""
    qq = _c(q, np.float32)
    P = np.zeros(maxcells)
    box = np.zeros(4, dtype=np.int32)
    k = lib().orc_ewa_pick_pmf(w, h, levels, wrap, _p(qq), amax, level, _p(P), maxcells, _p(box))
    if k < 0:
        raise ValueError("bounding box too large")
    nx, ny = box[1] - box[0] + 1, box[3] - box[2] + 1
    return P[:k].reshape(ny, nx), tuple(int(b) for b in box)


def ewa_weights(w: int, h: int, levels: int, q, level: int, amax: int = 8, wrap: int = REPEAT, maxcells: int = 4096):
    qq = _c(q, np.float32)
    P = np.zeros(maxcells)
    k = lib().orc_ewa_weights(w, h, levels, wrap, _p(qq), amax, level, _p(P), maxcells)
    if k < 0:
        raise ValueError("bounding box too large")
    return P[:k]


def aniso_reference(tex: Tex2D, q: np.ndarray, K: int = 16, filt: int = BSPLINE3, shade: int = 0, ggx=None,
                    subset=None, sigma: float = 0.5):
    """Pixel integral of the level-0 filter-after value (K x K midpoints)."""
    q = _c(q, np.float32).reshape(-1, 6)
    sub = None if subset is None else _c(subset, np.int64)
    m = q.shape[0] if sub is None else sub.size
    ch = 3 if shade else 4
    out = np.zeros((m, ch))
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_aniso_reference(_p(tex.buf), tex.w, tex.h, tex.fmt, tex.wrap, _p(tex.dct_range), _p(q), q.shape[0],
                              K, filt, sigma,
                              shade, _p(g), _p(out), _p(sub), 0 if sub is None else sub.size)
    return out


# ------------------------------------------------------------------ DCT textures, triplanar mapping
def dct_basis32() -> np.ndarray:
    """The encoder's binary32 basis c_k(x), k = 0..2, x = 0..7."""
    return np.array([[lib().orc_dct_basis32(k, x) for x in range(8)] for k in range(3)], dtype=np.float32)


def tri_pick(nrm, u: float) -> int:
    nn = _c(nrm, np.float32)
    return lib().orc_tri_pick(_p(nn), u)


def triplanar(tex: Tex2D, q: np.ndarray, scale: float, plane_mode: int, filt: int, mode: int, spp: int = 1,
              seed: int = 0, shade: int = 0, ggx=None, taps: bool = False, subset=None):
    """Triplanar mapping; queries ``[n, 8]`` {p, n, lambda, unused}.
    plane_mode 0 blends the planes, 1 picks one per sample."""
    q = _c(q, np.float32).reshape(-1, 8)
    n = q.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    ch = 3 if shade else 4
    out = np.zeros((m, ch))
    tp = np.zeros((m, spp, 4), dtype=np.int32) if taps else None
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_triplanar(_p(tex.buf), tex.w, tex.h, tex.levels, tex.fmt, tex.wrap, tex.mip, _p(tex.off),
                        _p(tex.dct_range), _p(q), n, scale, plane_mode, filt, mode, spp, seed & 0xFFFFFFFF, shade,
                        _p(g), _p(out), _p(tp), _p(sub), 0 if sub is None else sub.size)
    return (out, tp) if taps else out


# ------------------------------------------------------------------ Gaussian / FIS contract
def lnc(x):
    x = _c(x, np.float32).ravel()
    y = np.empty_like(x)
    lib().orc_elementary_batch(0, _p(x), _p(y), None, x.size)
    return y


def expc(x):
    x = _c(x, np.float32).ravel()
    y = np.empty_like(x)
    lib().orc_elementary_batch(1, _p(x), _p(y), None, x.size)
    return y


def sincos2pi(v):
    v = _c(v, np.float32).ravel()
    c, s = np.empty_like(v), np.empty_like(v)
    lib().orc_elementary_batch(2, _p(v), _p(c), _p(s), v.size)
    return c, s


def fis_gauss_offset(u1: float, u2: float, sigma: float):
    dx, dy = C.c_float(), C.c_float()
    lib().orc_fis_gauss_offset(u1, u2, sigma, C.byref(dx), C.byref(dy))
    return dx.value, dy.value


def fis_nearest(t: float, d: float) -> int:
    return lib().orc_fis_nearest(t, d)


def fis_bspline_pick(t: float, a: int, b: int, c: int) -> int:
    return lib().orc_fis_bspline_pick(t, a, b, c)


def fis_bspline_pmf(t: float) -> np.ndarray:
    P = np.zeros(4)
    lib().orc_fis_bspline_pmf(t, _p(P))
    return P


def gauss_h(sigma: float) -> float:
    return lib().orc_gauss_h(sigma)


def gauss_thresholds(t: float, sigma: float) -> np.ndarray:
    Cv = np.zeros(3, dtype=np.float32)
    lib().orc_gauss_thresholds(t, gauss_h(sigma), _p(Cv))
    return Cv


def gauss_pick_pmf(t: float, sigma: float) -> np.ndarray:
    P = np.zeros(4)
    lib().orc_gauss_pick_pmf(t, gauss_h(sigma), _p(P))
    return P


# ------------------------------------------------------------------ 3-D path
class Grid:
    """Host density grid ``[nz, ny, nx]`` (float16 or float32), world box
    starting at ``wmin`` with ``scale`` voxels per world unit."""

    def __init__(self, data: np.ndarray, wmin=(0.0, 0.0, 0.0), scale=None, side: float = None):
        self.data = np.ascontiguousarray(data)
        assert self.data.dtype in (np.float16, np.float32)
        self.nz, self.ny, self.nx = self.data.shape
        self.fmt = R16F if self.data.dtype == np.float16 else R32F
        self.wmin = np.asarray(wmin, dtype=np.float32)
        if scale is None:
            side = 1.0 if side is None else side
            scale = (self.nx / side, self.ny / side, self.nz / side)
        self.scale = np.asarray(scale, dtype=np.float32)


def filter3d(g: Grid, pos: np.ndarray, filt: int, mode: int, spp: int = 1, seed: int = 0, variant: int = 0,
             shade: int = 0, ds: float = 1.0, taps: bool = False, subset=None):
    pos = _c(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    out = np.zeros((m, 3)) if shade == PLANCK else np.zeros(m)
    tp = np.zeros((m, spp, 3), dtype=np.int32) if taps else None
    lib().orc_filter3d(_p(g.data), g.nx, g.ny, g.nz, g.fmt, _p(g.wmin), _p(g.scale), _p(pos), n, filt, mode,
                       spp, seed & 0xFFFFFFFF, variant, shade, float(ds), _p(out), _p(tp), _p(sub),
                       0 if sub is None else sub.size)
    return (out, tp) if taps else out


def raymarch(g: Grid, rays: np.ndarray, steps: int, filt: int, mode: int, spp: int = 1, seed: int = 0,
             variant: int = 0, taps: bool = False, subset=None):
    rays = _c(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    T = np.zeros(m)
    tp = np.zeros((m, spp, steps, 3), dtype=np.int32) if taps else None
    lib().orc_raymarch(_p(g.data), g.nx, g.ny, g.nz, g.fmt, _p(g.wmin), _p(g.scale), _p(rays), n, steps, filt,
                       mode, spp, seed & 0xFFFFFFFF, variant, _p(T), _p(tp), _p(sub), 0 if sub is None else sub.size)
    return (T, tp) if taps else T


def raymarch_expect(g: Grid, rays: np.ndarray, steps: int, filt: int):
    rays = _c(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    T = np.zeros(n)
    lib().orc_raymarch_expect(_p(g.data), g.nx, g.ny, g.nz, g.fmt, _p(g.wmin), _p(g.scale), _p(rays), n, steps,
                              filt, _p(T))
    return T


def planck(lambda_nm: float, T: float) -> float:
    """Black-body spectral radiance, W sr^-1 m^-2 nm^-1 (float64)."""
    return lib().orc_planck(float(lambda_nm), float(T))


def raymarch_emission(g: Grid, rays: np.ndarray, steps: int, filt: int, mode: int, spp: int = 1, seed: int = 0,
                      variant: int = 0, taps: bool = False, subset=None, footprint: float = 0.0):
    """Emission gathered along rays through a temperature grid: [m, 3]
    (700, 546.1, 435.8 nm); ``footprint`` > 0 (stochastic) jitters every
    step by a Gaussian of that standard deviation (world units)
    perpendicular to the ray."""
    rays = _c(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    L = np.zeros((m, 3))
    tp = np.zeros((m, spp, steps, 3), dtype=np.int32) if taps else None
    lib().orc_raymarch_emission(_p(g.data), g.nx, g.ny, g.nz, g.fmt, _p(g.wmin), _p(g.scale), _p(rays), n, steps,
                                filt, mode, spp, seed & 0xFFFFFFFF, variant, float(footprint), _p(L), _p(tp),
                                _p(sub), 0 if sub is None else sub.size)
    return (L, tp) if taps else L


def perp_jitter(g: Grid, ray, steps: int, sigma: float, ri: int, s: int, k: int, seed: int) -> np.ndarray:
    """Jittered raster position of step k of a ray (sample s)."""
    out = np.zeros(3, dtype=np.float32)
    r = _c(ray, np.float32)
    lib().orc_perp_jitter(_p(g.wmin), _p(g.scale), _p(r), steps, float(sigma), ri, s, k, seed & 0xFFFFFFFF, _p(out))
    return out


def raymarch_emission_expect(g: Grid, rays: np.ndarray, steps: int, filt: int):
    rays = _c(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    L = np.zeros((n, 3))
    lib().orc_raymarch_emission_expect(_p(g.data), g.nx, g.ny, g.nz, g.fmt, _p(g.wmin), _p(g.scale), _p(rays), n,
                                       steps, filt, _p(L))
    return L


def build_occupancy(g: Grid, brick_log2: int) -> np.ndarray:
    B = 1 << brick_log2
    nb = -(-g.nx // B) * -(-g.ny // B) * -(-g.nz // B)
    words = np.zeros((nb + 31) // 32, dtype=np.uint32)
    lib().orc_build_occupancy(_p(g.data), g.nx, g.ny, g.nz, g.fmt, brick_log2, _p(words))
    return words


# ------------------------------------------------------------------ neural
def f32_to_bf16(x) -> np.ndarray:
    """Vectorised over an array via the oracle's scalar routine (slow; tests only)."""
    x = np.asarray(x, dtype=np.float32)
    f = lib().orc_f32_to_bf16
    return np.array([f(float(v)) for v in x.ravel()], dtype=np.uint16).reshape(x.shape)


def bf16_to_double(b) -> np.ndarray:
    b = np.asarray(b, dtype=np.uint16)
    f = lib().orc_bf16_to_double
    return np.array([f(int(v)) for v in b.ravel()]).reshape(b.shape)


def fp8_table() -> np.ndarray:
    """binary64 value of each of the 256 E4M3 codes."""
    return np.array([lib().orc_fp8_to_double(c) for c in range(256)])


def f32_to_fp8(x: float) -> int:
    return int(lib().orc_f32_to_fp8(float(x)))


def quantize_fp8(lat: np.ndarray, dims: int, res, C: int, block_log2: int):
    lat = _c(lat, np.float32)
    r = np.array(list(res) + [1] * (3 - len(res)), dtype=np.int32)
    B = 1 << block_log2
    nb = int(np.prod([-(-int(r[a]) // B) for a in range(dims)]))
    codes = np.zeros(lat.size, dtype=np.uint8)
    scales = np.zeros(nb, dtype=np.float32)
    lib().orc_quantize_fp8(_p(lat), dims, _p(r), C, block_log2, _p(codes), _p(scales))
    return codes, scales


def dequant_fp8(codes: np.ndarray, point_scale: np.ndarray, C: int) -> np.ndarray:
    """The BF16 values an MLP reads from E4M3 latents: codes n x C, one
    block scale per lattice point; binary32 product rounded to BF16."""
    codes = _c(codes, np.uint8).reshape(-1, C)
    s = _c(point_scale, np.float32).reshape(-1)
    assert s.size == codes.shape[0]
    out = np.zeros(codes.shape)
    lib().orc_dequant_fp8(_p(codes), _p(s), codes.shape[0], C, _p(out))
    return out


def mlp_nparams(C: int, H: int, O: int) -> int:
    return C * H + H + H * H + H + H * O + O


def mlp_forward(C, H, O, P, Z, act_bf16=False):
    P = _c(P, np.float64)
    Z = _c(Z, np.float64).reshape(-1, C)
    Y = np.zeros((Z.shape[0], O))
    lib().orc_mlp_forward(C, H, O, _p(P), _p(Z), Z.shape[0], int(act_bf16), _p(Y))
    return Y


def mlp_grad(C, H, O, P, Z, T, act_bf16=False):
    P = _c(P, np.float64)
    Z = _c(Z, np.float64).reshape(-1, C)
    T = _c(T, np.float64).reshape(-1, O)
    gP = np.zeros(P.size)
    gZ = np.zeros_like(Z)
    loss = lib().orc_mlp_grad(C, H, O, _p(P), _p(Z), _p(T), Z.shape[0], int(act_bf16), _p(gP), _p(gZ))
    return loss, gP, gZ


def adam(theta, m, v, g, step, lr):
    """In place on float64 arrays."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().orc_adam(_p(theta), _p(m), _p(v), _p(g), theta.size, step, float(lr))


def neural_filter2d(res, C, H, O, Z, P, q, filt, mode, spp=1, seed=0, shade=0, ggx=None, act_bf16=True,
                    taps=False, subset=None):
    Z = _c(Z, np.float64)
    P = _c(P, np.float64)
    q = _c(q, np.float32).reshape(-1, 3)
    n = q.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    ch = 3 if shade == 1 else O
    out = np.zeros((m, ch))
    tp = np.zeros((m, spp, 2), dtype=np.int32) if taps else None
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_neural_filter2d(res[0], res[1], C, H, O, _p(Z), _p(P), int(act_bf16), _p(q), n, filt, mode, spp,
                              seed & 0xFFFFFFFF, shade, _p(g), _p(out), _p(tp), _p(sub), 0 if sub is None else sub.size)
    return (out, tp) if taps else out


def neural_raymarch(res, C, H, Z, P, wmin, scale, rays, steps, filt, mode, spp=1, seed=0, act_bf16=True,
                    taps=False, subset=None):
    Z = _c(Z, np.float64)
    P = _c(P, np.float64)
    rays = _c(rays, np.float32).reshape(-1, 8)
    n = rays.shape[0]
    sub = None if subset is None else _c(subset, np.int64)
    m = n if sub is None else sub.size
    T = np.zeros(m)
    tp = np.zeros((m, spp, steps, 3), dtype=np.int32) if taps else None
    wmin = _c(wmin, np.float32)
    scale = _c(scale, np.float32)
    lib().orc_neural_raymarch(res[0], res[1], res[2], C, H, _p(Z), _p(P), int(act_bf16), _p(wmin), _p(scale),
                              _p(rays), n, steps, filt, mode, spp, seed & 0xFFFFFFFF, _p(T), _p(tp), _p(sub),
                              0 if sub is None else sub.size)
    return (T, tp) if taps else T


def k3(x: float) -> float:
    return lib().orc_k3(float(x))


def keys_pick(tx: float, ty: float, u) -> tuple:
    uu = _c(u, np.float32)
    off = np.zeros(4, dtype=np.int32)
    hn = np.zeros(1, dtype=np.int32)
    lib().orc_keys_pick(float(tx), float(ty), _p(uu), _p(off), _p(hn))
    return off, bool(hn[0])


def keys_expect2d(tex: Tex2D, q: np.ndarray, shade: int = 0, ggx=None):
    q = _c(q, np.float32).reshape(-1, 3)
    ch = 3 if shade else 4
    out = np.zeros((q.shape[0], ch))
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_keys_expect2d(_p(tex.buf), tex.w, tex.h, tex.fmt, tex.wrap, _p(q), q.shape[0], shade, _p(g), _p(out))
    return out


def kmn(x: float) -> float:
    """Mitchell-Netravali cubic, B = C = 1/3 (binary64)."""
    return lib().orc_kmn(float(x))


def mitchell_axis(t: float):
    """Binary32 tap weights (taps i0-1..i0+2) and the positive / negative
    sums of one axis."""
    w = np.zeros(4, dtype=np.float32)
    pp = np.zeros(1, dtype=np.float32)
    pm = np.zeros(1, dtype=np.float32)
    lib().orc_mitchell_axis(float(t), _p(w), _p(pp), _p(pm))
    return w, float(pp[0]), float(pm[0])


def mitchell_pick(tx: float, ty: float, u) -> tuple:
    uu = _c(u, np.float32)
    off = np.zeros(4, dtype=np.int32)
    hn = np.zeros(1, dtype=np.int32)
    lib().orc_mitchell_pick(float(tx), float(ty), _p(uu), _p(off), _p(hn))
    return off, bool(hn[0])


def mitchell_expect2d(tex: Tex2D, q: np.ndarray, shade: int = 0, ggx=None):
    q = _c(q, np.float32).reshape(-1, 3)
    ch = 3 if shade else 4
    out = np.zeros((q.shape[0], ch))
    g = _c(ggx if ggx is not None else ggx_params(), np.float64)
    lib().orc_mitchell_expect2d(_p(tex.buf), tex.w, tex.h, tex.fmt, tex.wrap, _p(q), q.shape[0], shade, _p(g),
                                _p(out))
    return out
