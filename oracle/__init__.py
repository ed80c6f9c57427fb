"""FP64 CPU oracle for stochastic texture filtering -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it, and
it shares no code with the HIP path.

This module is argument marshalling around ``liboracle.so`` (compiled from the
C sources next to it by ``oracle/build.py``); all arithmetic is in C.
Every function states the passage of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# storage formats / filters / modes (the oracle's own numbering)
F32, F16, BF16, FP8_E4M3, U8 = 0, 1, 2, 3, 4
LINEAR, CUBIC, KEYS, MITCHELL = 0, 1, 2, 3
POSITIVIZED = (KEYS, MITCHELL)
DET, STOCH, STOCH_REUSE, DET_ABS, STOCH_FIS = 0, 1, 2, 3, 4   # DET_ABS: sum |w_k| |t_k| (tolerance scale)
G_FIS, G_FIS_MEAN, G_DISCRETE, G_DISCRETE_MEAN = 0, 1, 2, 3
BAD_INDEX = -(2 ** 31)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle/liboracle.so is not built; run oracle/build.py")
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


class using_library:
    """Context manager: every function of this module calls the library at
    `path` (a separately built copy of the oracle's C sources) instead of
    liboracle.so until the block ends.  The tests use it to check that a
    pin fails when a mistake is planted in a copy of the oracle."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        self.saved = lib()
        alt = C.CDLL(self.path)
        _declare(alt)
        _lib = alt
        return alt

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _declare(L):
    vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    L.orc_pcg.argtypes, L.orc_pcg.restype = [u32], u32
    L.orc_seed_key.argtypes, L.orc_seed_key.restype = [u64], u32
    L.orc_uniform.argtypes, L.orc_uniform.restype = [u64, u32, u32], C.c_float
    L.orc_decode.argtypes, L.orc_decode.restype = [i32, vp, i64], dbl
    L.orc_kernel_tent.argtypes, L.orc_kernel_tent.restype = [dbl], dbl
    L.orc_kernel_bspline.argtypes, L.orc_kernel_bspline.restype = [dbl], dbl
    L.orc_axis_weights.argtypes, L.orc_axis_weights.restype = [i32, dbl, vp], None
    L.orc_kernel_keys.argtypes, L.orc_kernel_keys.restype = [dbl], dbl
    L.orc_kernel_mitchell.argtypes, L.orc_kernel_mitchell.restype = [dbl], dbl
    L.orc_kernel.argtypes, L.orc_kernel.restype = [i32, dbl], dbl
    L.orc_interp_weights32.argtypes, L.orc_interp_weights32.restype = [i32, C.c_float, vp], None
    L.orc_cumulative_choice.argtypes, L.orc_cumulative_choice.restype = [vp, i32, C.c_float], i32
    L.orc_positivized_taps.argtypes = [i32, i32, vp, u64, u32, vp, vp]
    L.orc_positivized_taps.restype = i32
    L.orc_positivized_masses.argtypes, L.orc_positivized_masses.restype = [i32, i32, vp, vp, vp], None
    L.orc_positivized_wrs2d.argtypes = [i32, dbl, dbl, dbl, vp, vp]
    L.orc_positivized_wrs2d.restype = i32
    L.orc_filter2d_moments.argtypes = [vp, i32, i32, i32, i32, vp, i64, i32, vp, vp, i32]
    L.orc_filter2d_moments.restype = i32
    L.orc_select.argtypes, L.orc_select.restype = [i32, C.c_float, C.c_float], i32
    L.orc_max_threads.argtypes, L.orc_max_threads.restype = [], i32
    L.orc_cubic_breakpoints.argtypes, L.orc_cubic_breakpoints.restype = [C.c_float, vp], None
    L.orc_cubic_breakpoints_disorder.argtypes, L.orc_cubic_breakpoints_disorder.restype = [], i64
    L.orc_filter2d.argtypes = [vp, i32, i32, i32, i32, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_filter2d.restype = i32
    L.orc_filter2d_brute.argtypes = [vp, i32, i32, i32, i32, vp, i64, i32, vp]
    L.orc_filter2d_brute.restype = i32
    L.orc_grid_create.argtypes = [i32, i32, i32, i32, i64, vp, vp, dbl]
    L.orc_grid_create.restype = vp
    L.orc_grid_destroy.argtypes, L.orc_grid_destroy.restype = [vp], None
    L.orc_grid_texel.argtypes, L.orc_grid_texel.restype = [vp, i32, i32, i32], dbl
    L.orc_filter3d.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_filter3d.restype = i32
    L.orc_filter3d_at.argtypes = [vp, vp, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_filter3d_at.restype = i32
    L.orc_filter3d_brute.argtypes = [vp, vp, i64, i32, vp]
    L.orc_filter3d_brute.restype = i32
    L.orc_filter3d_moments.argtypes = [vp, vp, i64, i32, vp, vp, i32]
    L.orc_filter3d_moments.restype = i32
    L.orc_dct_coefficient.argtypes, L.orc_dct_coefficient.restype = [vp, i32, i32], dbl
    L.orc_dct_dequant.argtypes, L.orc_dct_dequant.restype = [u32, i32], dbl
    L.orc_dct_encode.argtypes, L.orc_dct_encode.restype = [vp, i32, i32, i32, vp], i32
    L.orc_dct_texel.argtypes, L.orc_dct_texel.restype = [vp, i32, i32, i32, i32, i32], dbl
    L.orc_dct_filter2d.argtypes = [vp, i32, i32, i32, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_dct_filter2d.restype = i32
    L.orc_dct_filter2d_at.argtypes = [vp, i32, i32, i32, vp, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_dct_filter2d_at.restype = i32
    L.orc_dct_moments2d.argtypes = [vp, i32, i32, i32, vp, i64, i32, vp, vp, i32]
    L.orc_dct_moments2d.restype = i32
    L.orc_fis_tap.argtypes, L.orc_fis_tap.restype = [i32, dbl, u64, u32, i32], i32
    L.orc_ewa_lut_value.argtypes, L.orc_ewa_lut_value.restype = [i32], C.c_float
    L.orc_ewa_lods.argtypes, L.orc_ewa_lods.restype = [vp, i64, i32, C.c_float, vp], i32
    L.orc_ewa_weights.argtypes = [i32, i32, C.c_float, C.c_float, vp, vp, i64, vp, vp]
    L.orc_ewa_weights.restype = i64
    L.orc_ewa_listing_draws.argtypes = [i32, i32, C.c_float, C.c_float, vp, vp, u64, i64, vp]
    L.orc_ewa_listing_draws.restype = i64
    L.orc_ewa_filter2d.argtypes = [vp, vp, vp, i32, i32, i32, vp, i64, C.c_float, i32, u64, vp, vp, i32]
    L.orc_ewa_filter2d.restype = i32
    L.orc_ewa_filter2d_at.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, i64, C.c_float, i32, u64, vp, vp, i32]
    L.orc_ewa_filter2d_at.restype = i32
    L.orc_gauss_radius.argtypes, L.orc_gauss_radius.restype = [dbl], i32
    L.orc_gauss_filter2d.argtypes = [vp, i32, i32, i32, i32, vp, i64, dbl, i32, u64, vp, vp, i32]
    L.orc_gauss_filter2d.restype = i32
    L.orc_dct_gauss_filter2d.argtypes = [vp, i32, i32, i32, vp, i64, dbl, i32, u64, vp, vp, i32]
    L.orc_dct_gauss_filter2d.restype = i32
    L.orc_dct_gauss_filter2d_at.argtypes = [vp, i32, i32, i32, vp, vp, i64, dbl, i32, u64, vp, vp, i32]
    L.orc_dct_gauss_filter2d_at.restype = i32
    L.orc_material_filter2d_at.argtypes = [vp, i32, i32, vp, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_material_filter2d_at.restype = i32
    L.orc_material_gauss_filter2d_at.argtypes = [vp, i32, i32, vp, vp, i64, dbl, i32, u64, vp, vp, i32]
    L.orc_material_gauss_filter2d_at.restype = i32
    L.orc_gauss_fis_positions_at.argtypes = [i32, i32, vp, vp, i64, dbl, u64, vp]
    L.orc_gauss_fis_positions_at.restype = i32
    L.orc_gauss_fis_positions.argtypes = [i32, i32, vp, i64, dbl, u64, vp]
    L.orc_gauss_fis_positions.restype = i32
    if hasattr(L, "orc_shade"):
        _declare_shade(L)
    if hasattr(L, "orc_ntex_decode"):
        _declare_neural(L)


def _declare_shade(L):
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
    L.orc_shade.argtypes = [vp, vp, vp, i32, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_shade.restype = i32
    L.orc_shade_at.argtypes = [vp, vp, vp, i32, vp, vp, i64, i32, i32, u64, vp, vp, i32]
    L.orc_shade_at.restype = i32
    L.orc_shade_moments.argtypes = [vp, vp, vp, i32, vp, i64, i32, vp, vp]
    L.orc_shade_moments.restype = i32
    L.orc_shade_eval.argtypes = [vp, vp, vp, vp]
    L.orc_shade_eval.restype = None
    L.orc_ggx_D.argtypes = [vp, vp, dbl]
    L.orc_ggx_D.restype = dbl
    L.orc_ggx_terms.argtypes = [vp, vp, vp, dbl, vp]
    L.orc_ggx_terms.restype = None
    L.orc_shade_level.argtypes = [C.c_float, i32]
    L.orc_shade_level.restype = i32


def _declare_neural(L):
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
    L.orc_ntex_nparams.argtypes, L.orc_ntex_nparams.restype = [], i32
    L.orc_round_bf16.argtypes, L.orc_round_bf16.restype = [dbl], dbl
    L.orc_ntex_decode.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, i32, vp]
    L.orc_ntex_decode.restype = None
    L.orc_ntex_filter.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, i64, i32, i32, u64, i32, vp, vp, i32]
    L.orc_ntex_filter.restype = i32
    L.orc_ntex_loss_grad.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, i64, vp, vp]
    L.orc_ntex_loss_grad.restype = dbl


# ----------------------------------------------------------------------------
# scalar helpers
# ----------------------------------------------------------------------------
def pcg(x: int) -> int:
    return lib().orc_pcg(x & 0xFFFFFFFF)


def uniform(seed: int, qid: int, axis: int) -> float:
    return lib().orc_uniform(seed, qid, axis)


def kernel_tent(d: float) -> float:
    return lib().orc_kernel_tent(d)


def kernel_bspline(d: float) -> float:
    return lib().orc_kernel_bspline(d)


def kernel(filt: int, d: float) -> float:
    return lib().orc_kernel(filt, d)


def interp_weights32(filt: int, t: float) -> np.ndarray:
    """Pinned binary32 per-axis weights of an interpolating cubic, scaled
    (Keys by 2, Mitchell by 18)."""
    w = np.zeros(4, np.float32)
    lib().orc_interp_weights32(filt, float(np.float32(t)), _p(w))
    return w


def cumulative_choice(masses, u: float) -> int:
    m = np.ascontiguousarray(masses, np.float32)
    return lib().orc_cumulative_choice(_p(m), m.size, float(np.float32(u)))


def positivized_taps(filt: int, t, seed: int, qid: int):
    """Tap offsets (-1..2 per axis) of the positive and negative draws and
    whether a negative tap exists."""
    t = np.ascontiguousarray(t, np.float32)
    D = t.size
    op = np.zeros(D, np.int32)
    on = np.zeros(D, np.int32)
    neg = lib().orc_positivized_taps(filt, D, _p(t), seed, qid & 0xFFFFFFFF, _p(op), _p(on))
    return op, on, bool(neg)


def positivized_masses(filt: int, t):
    t = np.ascontiguousarray(t, np.float64)
    sp, sn = C.c_double(), C.c_double()
    lib().orc_positivized_masses(filt, t.size, _p(t), C.byref(sp), C.byref(sn))
    return sp.value, sn.value


def positivized_wrs2d(filt: int, tx: float, ty: float, u: float):
    op = np.zeros(2, np.int32)
    on = np.zeros(2, np.int32)
    neg = lib().orc_positivized_wrs2d(filt, float(tx), float(ty), float(u), _p(op), _p(on))
    return op, on, bool(neg)


def index_width(filt: int, dims: int) -> int:
    """Index entries per stochastic query: the tap, or for positivized filters
    the positive tap followed by the negative tap."""
    return 2 * dims if filt in POSITIVIZED else dims


def axis_weights(filt: int, t: float) -> np.ndarray:
    w = np.zeros(4, np.float64)
    lib().orc_axis_weights(filt, float(t), _p(w))
    return w


def select(filt: int, t: float, u: float) -> int:
    return lib().orc_select(filt, float(np.float32(t)), float(np.float32(u)))


def cubic_breakpoints(t: float) -> np.ndarray:
    c = np.zeros(3, np.float32)
    lib().orc_cubic_breakpoints(float(np.float32(t)), _p(c))
    return c


def cubic_breakpoints_disorder() -> int:
    return lib().orc_cubic_breakpoints_disorder()


def max_threads() -> int:
    return lib().orc_max_threads()


def decode(fmt: int, raw: np.ndarray) -> np.ndarray:
    raw = np.ascontiguousarray(raw)
    out = np.empty(raw.size, np.float64)
    L = lib()
    for k in range(raw.size):
        out[k] = L.orc_decode(fmt, _p(raw), k)
    return out.reshape(raw.shape)


# ----------------------------------------------------------------------------
# 2D textures
# ----------------------------------------------------------------------------
def filter2d(tex: np.ndarray, fmt: int, uv: np.ndarray, filt: int, mode: int, seed: int = 0,
             want_index: bool = True, nthreads: int = 0):
    """tex: (H, W, C) raw texels of the storage format; uv: (n, 2) float32.
    Returns (values (n, C) float64, indices (n, 2) int32 or None)."""
    tex = np.ascontiguousarray(tex)
    H, W, Ch = tex.shape
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    n = uv.shape[0]
    out = np.empty((n, Ch), np.float64)
    idx = np.empty((n, index_width(filt, 2)), np.int32) if (want_index and mode in (STOCH, STOCH_REUSE, STOCH_FIS)) \
        else None
    rc = lib().orc_filter2d(_p(tex), W, H, Ch, fmt, _p(uv), n, filt, mode, seed, _p(out), _p(idx), nthreads)
    if rc != 0:
        raise ValueError("orc_filter2d rejected its arguments")
    return out, idx


def moments2d(tex: np.ndarray, fmt: int, uv: np.ndarray, filt: int, nthreads: int = 0):
    """Exact mean and variance (n, C) of the stochastic estimator."""
    tex = np.ascontiguousarray(tex)
    H, W, Ch = tex.shape
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    n = uv.shape[0]
    mean = np.empty((n, Ch), np.float64)
    var = np.empty((n, Ch), np.float64)
    if lib().orc_filter2d_moments(_p(tex), W, H, Ch, fmt, _p(uv), n, filt, _p(mean), _p(var), nthreads) != 0:
        raise ValueError("orc_filter2d_moments rejected its arguments")
    return mean, var


def filter2d_brute(tex: np.ndarray, fmt: int, uv: np.ndarray, filt: int) -> np.ndarray:
    tex = np.ascontiguousarray(tex)
    H, W, Ch = tex.shape
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    out = np.empty((uv.shape[0], Ch), np.float64)
    lib().orc_filter2d_brute(_p(tex), W, H, Ch, fmt, _p(uv), uv.shape[0], filt, _p(out))
    return out


# ----------------------------------------------------------------------------
# filter importance sampling and Gaussian filters
# ----------------------------------------------------------------------------
def fis_tap(filt: int, x: float, seed: int, qid: int, axis: int) -> int:
    return lib().orc_fis_tap(filt, float(x), seed, qid & 0xFFFFFFFF, axis)


def gauss_radius(sigma: float) -> int:
    return lib().orc_gauss_radius(float(sigma))


def gauss_filter2d(tex: np.ndarray, fmt: int, uv: np.ndarray, sigma: float, gmode: int, seed: int = 0,
                   want_index: bool = True, nthreads: int = 0):
    tex = np.ascontiguousarray(tex)
    H, W, Ch = tex.shape
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    n = uv.shape[0]
    out = np.empty((n, Ch), np.float64)
    idx = np.empty((n, 2), np.int32) if (want_index and gmode in (G_FIS, G_DISCRETE)) else None
    if lib().orc_gauss_filter2d(_p(tex), W, H, Ch, fmt, _p(uv), n, float(sigma), gmode, seed, _p(out), _p(idx),
                                nthreads) != 0:
        raise ValueError("orc_gauss_filter2d rejected its arguments")
    return out, idx


def dct_gauss_filter2d(blocks: np.ndarray, uv: np.ndarray, sigma: float, gmode: int, seed: int = 0,
                       want_index: bool = True, nthreads: int = 0, qids=None):
    b = np.ascontiguousarray(blocks, np.uint32)
    H, W, Ch = b.shape[0] * 8, b.shape[1] * 8, b.shape[2]
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    qi = _qids(qids)
    n = uv.shape[0] if qi is None else qi.shape[0]
    out = np.empty((n, Ch), np.float64)
    idx = np.empty((n, 2), np.int32) if (want_index and gmode in (G_FIS, G_DISCRETE)) else None
    if lib().orc_dct_gauss_filter2d_at(_p(b), W, H, Ch, _p(uv), _p(qi), n, float(sigma), gmode, seed, _p(out),
                                       _p(idx), nthreads) != 0:
        raise ValueError("orc_dct_gauss_filter2d rejected its arguments")
    return out, idx


def gauss_fis_positions(W: int, H: int, uv: np.ndarray, sigma: float, seed: int, qids=None) -> np.ndarray:
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    qi = _qids(qids)
    n = uv.shape[0] if qi is None else qi.shape[0]
    pos = np.empty((n, 2), np.float64)
    lib().orc_gauss_fis_positions_at(W, H, _p(uv), _p(qi), n, float(sigma), seed, _p(pos))
    return pos


# ----------------------------------------------------------------------------
# elliptically weighted average (EWA) filtering over a MIP pyramid
# ----------------------------------------------------------------------------
def ewa_lut(i: int) -> float:
    return lib().orc_ewa_lut_value(i)


def ewa_weights(W: int, H: int, s: float, t: float, d0, d1):
    """The taps of positive EWA weight on a W x H level for the query (s, t)
    with derivative vectors d0, d1 (texture units): (xy int32 (k, 2), w
    float32 (k,)) in scan order, coordinates not clamped."""
    a = np.ascontiguousarray(d0, np.float32)
    b = np.ascontiguousarray(d1, np.float32)
    n = lib().orc_ewa_weights(W, H, float(np.float32(s)), float(np.float32(t)), _p(a), _p(b), 0, None, None)
    xy = np.zeros((max(n, 1), 2), np.int32)
    w = np.zeros(max(n, 1), np.float32)
    lib().orc_ewa_weights(W, H, float(np.float32(s)), float(np.float32(t)), _p(a), _p(b), n, _p(xy), _p(w))
    return xy[:n], w[:n]


def ewa_listing_draws(W: int, H: int, s: float, t: float, d0, d1, seed: int, K: int) -> np.ndarray:
    """K taps drawn by the supplement's single-uniform reservoir sampler
    (distribution tests only): int32 (K, 2)."""
    a = np.ascontiguousarray(d0, np.float32)
    b = np.ascontiguousarray(d1, np.float32)
    xy = np.zeros((K, 2), np.int32)
    lib().orc_ewa_listing_draws(W, H, float(np.float32(s)), float(np.float32(t)), _p(a), _p(b), seed, K, _p(xy))
    return xy


def ewa_lods(q: np.ndarray, levels: int, max_aniso: float) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float32)
    out = np.empty(q.shape[0])
    lib().orc_ewa_lods(_p(q), q.shape[0], levels, float(max_aniso), _p(out))
    return out


def ewa_filter2d(levels, fmt: int, q: np.ndarray, max_aniso: float, mode: int, seed: int = 0,
                 want_index: bool = True, nthreads: int = 0, qids=None):
    """levels: list of (H_l, W_l, C) raw texel arrays; q: (n, 6) float32
    (s, t, ds/dx, dt/dx, ds/dy, dt/dy).  Returns values (n, C) and, in
    stochastic mode, indices (n, 3) = (x, y, level)."""
    lv = [np.ascontiguousarray(a) for a in levels]
    ptrs = (C.c_void_p * len(lv))(*[a.ctypes.data for a in lv])
    Ws = (C.c_int * len(lv))(*[a.shape[1] for a in lv])
    Hs = (C.c_int * len(lv))(*[a.shape[0] for a in lv])
    Ch = lv[0].shape[2]
    q = np.ascontiguousarray(q, np.float32)
    qi = _qids(qids)
    n = q.shape[0] if qi is None else qi.shape[0]
    out = np.empty((n, Ch))
    idx = np.empty((n, 3), np.int32) if (want_index and mode == STOCH) else None
    if lib().orc_ewa_filter2d_at(ptrs, Ws, Hs, len(lv), Ch, fmt, _p(q), _p(qi), n, float(max_aniso), mode, seed,
                                 _p(out), _p(idx), nthreads) != 0:
        raise ValueError("orc_ewa_filter2d rejected its arguments")
    return out, idx


# ----------------------------------------------------------------------------
# DCT-compressed textures
# ----------------------------------------------------------------------------
def dct_coefficient(block: np.ndarray, u: int, v: int) -> float:
    """Orthonormal DCT-II coefficient F(u, v) of an 8x8 block f[y][x]."""
    b = np.ascontiguousarray(block, np.float64)
    assert b.shape == (8, 8)
    return lib().orc_dct_coefficient(_p(b), u, v)


def dct_dequant(word: int, k: int) -> float:
    return lib().orc_dct_dequant(word & 0xFFFFFFFF, k)


def dct_encode(texels: np.ndarray) -> np.ndarray:
    """(H, W, C) uint8 texels -> (H/8, W/8, C) uint32 words."""
    t = np.ascontiguousarray(texels, np.uint8)
    H, W, Ch = t.shape
    out = np.zeros((H // 8, W // 8, Ch), np.uint32)
    if lib().orc_dct_encode(_p(t), W, H, Ch, _p(out)) != 0:
        raise ValueError("orc_dct_encode rejected its arguments")
    return out


def dct_texel(blocks: np.ndarray, x: int, y: int, c: int) -> float:
    b = np.ascontiguousarray(blocks, np.uint32)
    return lib().orc_dct_texel(_p(b), b.shape[1] * 8, b.shape[2], x, y, c)


def dct_decode_all(blocks: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(blocks, np.uint32)
    H, W, Ch = b.shape[0] * 8, b.shape[1] * 8, b.shape[2]
    L = lib()
    out = np.empty((H, W, Ch))
    for y in range(H):
        for x in range(W):
            for c in range(Ch):
                out[y, x, c] = L.orc_dct_texel(_p(b), W, Ch, x, y, c)
    return out


def _qids(qids):
    return None if qids is None else np.ascontiguousarray(qids, np.int64)


def dct_filter2d(blocks: np.ndarray, uv: np.ndarray, filt: int, mode: int, seed: int = 0, want_index: bool = True,
                 nthreads: int = 0, qids=None):
    """qids: optional indices of the queries of the batch uv to evaluate (as
    members of the whole batch); results follow their order."""
    b = np.ascontiguousarray(blocks, np.uint32)
    H, W, Ch = b.shape[0] * 8, b.shape[1] * 8, b.shape[2]
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    qi = _qids(qids)
    n = uv.shape[0] if qi is None else qi.shape[0]
    out = np.empty((n, Ch), np.float64)
    idx = np.empty((n, index_width(filt, 2)), np.int32) if (want_index and mode in (STOCH, STOCH_REUSE, STOCH_FIS)) \
        else None
    if lib().orc_dct_filter2d_at(_p(b), W, H, Ch, _p(uv), _p(qi), n, filt, mode, seed, _p(out), _p(idx),
                                 nthreads) != 0:
        raise ValueError("orc_dct_filter2d rejected its arguments")
    return out, idx


def material_filter2d(tex: np.ndarray, uv: np.ndarray, filt: int, mode: int, seed: int = 0,
                      want_index: bool = True, nthreads: int = 0, qids=None):
    """tex: (H, W, 8) uint8 material texels (albedo RGB, roughness UNORM8,
    normal x, y binary16), filtered as six channels; qids as dct_filter2d."""
    t = np.ascontiguousarray(tex, np.uint8)
    H, W = t.shape[0], t.shape[1]
    assert t.shape[2] == 8
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    qi = _qids(qids)
    n = uv.shape[0] if qi is None else qi.shape[0]
    out = np.empty((n, 6), np.float64)
    idx = np.empty((n, index_width(filt, 2)), np.int32) if (want_index and mode in (STOCH, STOCH_REUSE, STOCH_FIS)) \
        else None
    if lib().orc_material_filter2d_at(_p(t), W, H, _p(uv), _p(qi), n, filt, mode, seed, _p(out), _p(idx),
                                      nthreads) != 0:
        raise ValueError("orc_material_filter2d rejected its arguments")
    return out, idx


def material_gauss_filter2d(tex: np.ndarray, uv: np.ndarray, sigma: float, gmode: int, seed: int = 0,
                            want_index: bool = True, nthreads: int = 0, qids=None):
    t = np.ascontiguousarray(tex, np.uint8)
    H, W = t.shape[0], t.shape[1]
    assert t.shape[2] == 8
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    qi = _qids(qids)
    n = uv.shape[0] if qi is None else qi.shape[0]
    out = np.empty((n, 6), np.float64)
    idx = np.empty((n, 2), np.int32) if (want_index and gmode in (G_FIS, G_DISCRETE)) else None
    if lib().orc_material_gauss_filter2d_at(_p(t), W, H, _p(uv), _p(qi), n, float(sigma), gmode, seed, _p(out),
                                            _p(idx), nthreads) != 0:
        raise ValueError("orc_material_gauss_filter2d rejected its arguments")
    return out, idx


def dct_moments2d(blocks: np.ndarray, uv: np.ndarray, filt: int, nthreads: int = 0):
    b = np.ascontiguousarray(blocks, np.uint32)
    H, W, Ch = b.shape[0] * 8, b.shape[1] * 8, b.shape[2]
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    n = uv.shape[0]
    mean = np.empty((n, Ch))
    var = np.empty((n, Ch))
    if lib().orc_dct_moments2d(_p(b), W, H, Ch, _p(uv), n, filt, _p(mean), _p(var), nthreads) != 0:
        raise ValueError("orc_dct_moments2d rejected its arguments")
    return mean, var


# ----------------------------------------------------------------------------
# 3D sparse grids
# ----------------------------------------------------------------------------
class Grid:
    """Oracle view of a sparse grid: leaf origins (n, 3) int32 and leaf values
    (n, 8, 8, 8) raw storage (z, y, x order, x fastest)."""

    def __init__(self, dims, fmt: int, origins: np.ndarray, values: np.ndarray, background: float = 0.0):
        self.origins = np.ascontiguousarray(origins, dtype=np.int32)
        self.values = np.ascontiguousarray(values)
        self.fmt = fmt
        self.dims = tuple(int(d) for d in dims)
        h = lib().orc_grid_create(self.dims[0], self.dims[1], self.dims[2], fmt, self.origins.shape[0],
                                  _p(self.origins), _p(self.values), float(background))
        if not h:
            raise ValueError("orc_grid_create rejected the leaf list")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_grid_destroy(h)
            self._h = None

    def texel(self, x: int, y: int, z: int) -> float:
        return lib().orc_grid_texel(self._h, x, y, z)

    def filter(self, p: np.ndarray, filt: int, mode: int, seed: int = 0, want_index: bool = True,
               nthreads: int = 0):
        p = np.ascontiguousarray(p, dtype=np.float32)
        n = p.shape[0]
        out = np.empty(n, np.float64)
        idx = np.empty((n, index_width(filt, 3)), np.int32) if (want_index and mode in (STOCH, STOCH_REUSE, STOCH_FIS)) \
            else None
        rc = lib().orc_filter3d(self._h, _p(p), n, filt, mode, seed, _p(out), _p(idx), nthreads)
        if rc != 0:
            raise ValueError("orc_filter3d failed")
        return out, idx

    def filter_at(self, p: np.ndarray, qids: np.ndarray, filt: int, mode: int, seed: int = 0,
                  nthreads: int = 0):
        """Filter the queries p[qids] as members of the whole batch p (the
        random draw of a query depends on its index in the batch)."""
        p = np.ascontiguousarray(p, dtype=np.float32)
        qids = np.ascontiguousarray(qids, dtype=np.int64)
        m = qids.shape[0]
        out = np.empty(m, np.float64)
        idx = np.empty((m, index_width(filt, 3)), np.int32) if mode in (STOCH, STOCH_REUSE, STOCH_FIS) else None
        rc = lib().orc_filter3d_at(self._h, _p(p), _p(qids), m, filt, mode, seed, _p(out), _p(idx), nthreads)
        if rc != 0:
            raise ValueError("orc_filter3d_at failed")
        return out, idx

    def filter_brute(self, p: np.ndarray, filt: int) -> np.ndarray:
        p = np.ascontiguousarray(p, dtype=np.float32)
        out = np.empty(p.shape[0], np.float64)
        lib().orc_filter3d_brute(self._h, _p(p), p.shape[0], filt, _p(out))
        return out

    def moments(self, p: np.ndarray, filt: int, nthreads: int = 0):
        p = np.ascontiguousarray(p, dtype=np.float32)
        n = p.shape[0]
        mean = np.empty(n, np.float64)
        var = np.empty(n, np.float64)
        if lib().orc_filter3d_moments(self._h, _p(p), n, filt, _p(mean), _p(var), nthreads) != 0:
            raise ValueError("orc_filter3d_moments rejected its arguments")
        return mean, var


# ----------------------------------------------------------------------------
# filtering with shading (material textures)
# ----------------------------------------------------------------------------
SH_AFTER_FILTER, SH_FILTER_AFTER, SH_STOCH = 0, 1, 2


class Material:
    """Oracle view of a material: list of (H, W) structured or (H, W, 8) uint8
    level arrays (8-byte texels)."""

    def __init__(self, levels):
        self.levels = [np.ascontiguousarray(lv).view(np.uint8).reshape(lv.shape[0], lv.shape[1], 8) for lv in levels]
        self._ptrs = (C.c_void_p * len(self.levels))(*[lv.ctypes.data for lv in self.levels])
        self._W = (C.c_int * len(self.levels))(*[lv.shape[1] for lv in self.levels])
        self._H = (C.c_int * len(self.levels))(*[lv.shape[0] for lv in self.levels])

    def shade(self, recs, filt: int, mode: int, seed: int = 0, want_index: bool = True, nthreads: int = 0):
        recs = np.ascontiguousarray(recs, dtype=np.float32)
        n = recs.shape[0]
        out = np.empty((n, 3), np.float64)
        idx = np.empty((n, 3), np.int32) if (want_index and mode == SH_STOCH) else None
        rc = lib().orc_shade(self._ptrs, self._W, self._H, len(self.levels), _p(recs), n, filt, mode, seed,
                             _p(out), _p(idx), nthreads)
        if rc != 0:
            raise ValueError("orc_shade failed")
        return out, idx

    def shade_at(self, recs, qids, filt: int, mode: int, seed: int = 0, nthreads: int = 0):
        """Shade recs[qids] as members of the whole batch recs."""
        recs = np.ascontiguousarray(recs, dtype=np.float32)
        qids = np.ascontiguousarray(qids, dtype=np.int64)
        m = qids.shape[0]
        out = np.empty((m, 3), np.float64)
        idx = np.empty((m, 3), np.int32) if mode == SH_STOCH else None
        rc = lib().orc_shade_at(self._ptrs, self._W, self._H, len(self.levels), _p(recs), _p(qids), m, filt, mode,
                                seed, _p(out), _p(idx), nthreads)
        if rc != 0:
            raise ValueError("orc_shade_at failed")
        return out, idx

    def moments(self, recs, filt: int):
        recs = np.ascontiguousarray(recs, dtype=np.float32)
        n = recs.shape[0]
        mean = np.empty((n, 3), np.float64)
        var = np.empty((n, 3), np.float64)
        lib().orc_shade_moments(self._ptrs, self._W, self._H, len(self.levels), _p(recs), n, filt, _p(mean), _p(var))
        return mean, var


def shade_eval(mat6, wo, wi) -> np.ndarray:
    """f^ for one decoded material (albedo r, g, b, roughness, nx, ny)."""
    m = np.ascontiguousarray(mat6, np.float64)
    a = np.ascontiguousarray(wo, np.float32)
    b = np.ascontiguousarray(wi, np.float32)
    out = np.zeros(3, np.float64)
    lib().orc_shade_eval(_p(m), _p(a), _p(b), _p(out))
    return out


def ggx_D(n, h, alpha: float) -> float:
    return lib().orc_ggx_D(_p(np.ascontiguousarray(n, np.float64)), _p(np.ascontiguousarray(h, np.float64)), alpha)


def ggx_terms(n, wo, wi, alpha: float) -> dict:
    """D(h), Lambda(wo), Lambda(wi), G2 and Schlick F of the GGX lobe used by
    shade_eval, for unit vectors n, wo, wi."""
    a = np.ascontiguousarray(n, np.float64)
    b = np.ascontiguousarray(wo, np.float64)
    c = np.ascontiguousarray(wi, np.float64)
    out = np.zeros(5, np.float64)
    lib().orc_ggx_terms(_p(a), _p(b), _p(c), float(alpha), _p(out))
    return dict(D=out[0], lambda_o=out[1], lambda_i=out[2], G2=out[3], F=out[4])


def shade_level(s: float, levels: int) -> int:
    return lib().orc_shade_level(float(np.float32(s)), levels)


# ----------------------------------------------------------------------------
# neural texture
# ----------------------------------------------------------------------------
NTEX_PARAMS = 5256


def round_bf16(x: float) -> float:
    return lib().orc_round_bf16(float(x))


class NeuralTexture:
    """Oracle view of a neural texture: latents (LH, LW, 8) and the MLP
    parameter vector (5256) in binary64; decoded texture size W x H."""

    def __init__(self, latents, mlp, width: int, height: int):
        self.lat = np.ascontiguousarray(latents, np.float64)
        self.mlp = np.ascontiguousarray(mlp, np.float64)
        assert self.mlp.size == NTEX_PARAMS and self.lat.shape[2] == 8
        self.LH, self.LW = self.lat.shape[:2]
        self.W, self.H = width, height

    def decode(self, i: int, j: int, emulate: bool = False) -> np.ndarray:
        out = np.zeros(8, np.float64)
        lib().orc_ntex_decode(_p(self.lat), self.LW, self.LH, self.W, self.H, _p(self.mlp), i, j, int(emulate),
                              _p(out))
        return out

    def decode_all(self, emulate: bool = False) -> np.ndarray:
        """(H, W, 8) decoded texels (texel-centre queries through the filter)."""
        js, is_ = np.meshgrid(np.arange(self.H), np.arange(self.W), indexing="ij")
        uv = np.stack([(is_ + 0.5) / self.W, (js + 0.5) / self.H], axis=-1).reshape(-1, 2).astype(np.float32)
        out, _ = self.filter(uv, LINEAR, DET, emulate=emulate)
        return out.reshape(self.H, self.W, 8)

    def filter(self, uv, filt: int, mode: int, seed: int = 0, qids=None, emulate: bool = False, nthreads: int = 0):
        uv = np.ascontiguousarray(uv, np.float32)
        qids_a = None if qids is None else np.ascontiguousarray(qids, np.int64)
        m = uv.shape[0] if qids_a is None else qids_a.shape[0]
        out = np.empty((m, 8), np.float64)
        idx = np.empty((m, 2), np.int32) if mode != DET else None
        lib().orc_ntex_filter(_p(self.lat), self.LW, self.LH, self.W, self.H, _p(self.mlp), _p(uv), _p(qids_a), m,
                              filt, mode, seed, int(emulate), _p(out), _p(idx), nthreads)
        return out, idx

    def loss_grad(self, target, pos, want_grad: bool = True):
        """target (H, W, 8) float32; pos (B, 2) int32 texel (i, j)."""
        target = np.ascontiguousarray(target, np.float32)
        pos = np.ascontiguousarray(pos, np.int32)
        gl = np.zeros_like(self.lat) if want_grad else None
        gm = np.zeros(NTEX_PARAMS) if want_grad else None
        loss = lib().orc_ntex_loss_grad(_p(self.lat), self.LW, self.LH, self.W, self.H, _p(self.mlp), _p(target),
                                        _p(pos), pos.shape[0], _p(gl), _p(gm))
        return loss, gl, gm
