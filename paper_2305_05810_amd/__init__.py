"""Python binding of libstf (stochastic texture filtering on MI355X).

Argument marshalling only: every call goes straight to the C ABI declared in
``include/stf.h`` with the same name.  Device buffers are torch tensors on the
GPU; host arrays are numpy arrays.  The binding has no compute path of its own:
if ``libstf.so`` is missing it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstf.so")

# enums of include/stf.h
STF_OK, STF_E_INVALID, STF_E_OOM, STF_E_UNSUPPORTED, STF_E_DEVICE, STF_E_BUSY, STF_E_CANCELLED = 0, -1, -2, -3, -4, -5, -6
STF_FMT_F32, STF_FMT_F16, STF_FMT_BF16, STF_FMT_FP8_E4M3, STF_FMT_U8 = 0, 1, 2, 3, 4
STF_LINEAR, STF_CUBIC_BSPLINE, STF_CUBIC_KEYS, STF_CUBIC_MITCHELL = 0, 1, 2, 3
STF_GAUSS_FIS, STF_GAUSS_FIS_MEAN, STF_GAUSS_DISCRETE, STF_GAUSS_DISCRETE_MEAN = 0, 1, 2, 3
POSITIVIZED_FILTERS = (STF_CUBIC_KEYS, STF_CUBIC_MITCHELL)
STF_DETERMINISTIC, STF_STOCHASTIC, STF_STOCHASTIC_FIS = 0, 1, 2
STF_SHADE_AFTER_FILTER, STF_FILTER_AFTER_SHADE, STF_SHADE_STOCHASTIC = 0, 1, 2


def index_width(filter: int, dims: int) -> int:
    """int32 index entries per query in stochastic mode: the tap, or for the
    interpolating cubics the positive tap followed by the negative tap."""
    return 2 * dims if filter in POSITIVIZED_FILTERS else dims


FORMATS = {"f32": STF_FMT_F32, "f16": STF_FMT_F16, "bf16": STF_FMT_BF16, "fp8_e4m3": STF_FMT_FP8_E4M3,
           "u8": STF_FMT_U8}
FORMAT_BYTES = {STF_FMT_F32: 4, STF_FMT_F16: 2, STF_FMT_BF16: 2, STF_FMT_FP8_E4M3: 1, STF_FMT_U8: 1}

_STATUS = {0: "STF_OK", -1: "STF_E_INVALID", -2: "STF_E_OOM", -3: "STF_E_UNSUPPORTED", -4: "STF_E_DEVICE",
           -5: "STF_E_BUSY", -6: "STF_E_CANCELLED"}


class STFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libstf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                              "python paper_2305_05810_amd/build.py")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    vp, i32, i64, u32, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
    L.stf_last_error.restype = C.c_char_p
    L.stf_last_error.argtypes = []
    L.stf_version.restype = C.c_char_p
    L.stf_version.argtypes = []
    L.stf_create_texture2d.argtypes = [i32, i32, i32, i32, i32, C.POINTER(vp), C.POINTER(vp)]
    L.stf_create_material2d.argtypes = [i32, i32, i32, C.POINTER(vp), C.POINTER(vp)]
    L.stf_create_sparse_grid3d.argtypes = [i32, i32, i32, i32, i64, vp, vp, f32, C.POINTER(vp)]
    L.stf_destroy.argtypes = [vp]
    L.stf_destroy.restype = None
    L.stf_texture_bytes.argtypes = [vp, C.POINTER(i64)]
    L.stf_filter.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, u32, vp]
    L.stf_filter_moments.argtypes = [vp, vp, i64, i32, u64, i32, vp, vp, vp]
    L.stf_shade_filter.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, vp]
    L.stf_dct_encode.argtypes = [i32, i32, i32, vp, vp]
    L.stf_filter_gaussian.argtypes = [vp, vp, i64, f32, i32, u64, vp, vp, vp]
    L.stf_filter_ewa.argtypes = [vp, vp, i64, f32, i32, u64, vp, vp, vp]
    L.stf_create_dct_texture2d.argtypes = [i32, i32, i32, vp, C.POINTER(vp)]
    L.stf_stage_counting.argtypes = [i32]
    L.stf_stage_counts.argtypes = [C.POINTER(u64), C.POINTER(u64)]
    for name in ("stf_create_texture2d", "stf_create_material2d", "stf_create_sparse_grid3d",
                 "stf_texture_bytes", "stf_filter", "stf_filter_moments", "stf_shade_filter", "stf_dct_encode",
                 "stf_create_dct_texture2d", "stf_filter_gaussian", "stf_filter_ewa", "stf_stage_counting",
                 "stf_stage_counts"):
        getattr(L, name).restype = i32


def _check(status: int):
    if status != STF_OK:
        raise STFError(status, stf_last_error())


def stf_last_error() -> str:
    return lib().stf_last_error().decode()


def stf_version() -> str:
    return lib().stf_version().decode()


def stf_stage_counting(on: bool):
    _check(lib().stf_stage_counting(1 if on else 0))


def stf_stage_counts():
    """(blocks that staged their taps in LDS, blocks) since counting began."""
    a, b = C.c_uint64(), C.c_uint64()
    _check(lib().stf_stage_counts(C.byref(a), C.byref(b)))
    return a.value, b.value


class Texture:
    """Owning handle of an stf_texture (freed by stf_destroy)."""

    def __init__(self, handle: int, kind: str, channels: int, dims: int):
        self.handle = handle
        self.kind = kind
        self.channels = channels
        self.dims = dims

    def destroy(self):
        if self.handle:
            lib().stf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()


def _host(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a)


def _check_level_sizes(levels, width, height, texel_bytes):
    """The C call reads w_l * h_l texels per level from host memory: make sure
    the arrays hold that many bytes (positive sizes only; the library rejects
    the rest)."""
    if width <= 0 or height <= 0:
        return
    for l, a in enumerate(levels):
        w, h = max(1, width >> l), max(1, height >> l)
        if a.nbytes != w * h * texel_bytes:
            raise ValueError(f"level {l} holds {a.nbytes} bytes, expected {w * h * texel_bytes}")


def stf_create_texture2d(width: int, height: int, channels: int, fmt: int,
                         level_texels: Sequence[np.ndarray]) -> Texture:
    """level_texels[l]: raw texels of level l (any dtype whose bytes are the
    storage format), row-major, channels interleaved."""
    lv = [_host(a) for a in level_texels]
    if fmt in FORMAT_BYTES and 1 <= channels <= 4:
        _check_level_sizes(lv, width, height, channels * FORMAT_BYTES[fmt])
    arr = (C.c_void_p * len(lv))(*[a.ctypes.data for a in lv])
    h = C.c_void_p()
    _check(lib().stf_create_texture2d(width, height, channels, fmt, len(lv), arr, C.byref(h)))
    return Texture(h.value, "tex2d", channels, 2)


def stf_dct_encode(texels: np.ndarray) -> np.ndarray:
    """(H, W, C) uint8 texels (H, W multiples of 8, C <= 16) -> (H/8, W/8, C)
    uint32 DCT block words, encoded by the library on the host."""
    t = _host(np.ascontiguousarray(texels, np.uint8))
    if t.ndim != 3:
        raise ValueError("texels must be (H, W, C)")
    H, W, Ch = t.shape
    out = np.zeros((max(H // 8, 0), max(W // 8, 0), Ch), np.uint32)
    _check(lib().stf_dct_encode(W, H, Ch, t.ctypes.data, out.ctypes.data))
    return out


def stf_create_dct_texture2d(width: int, height: int, channels: int, blocks: np.ndarray) -> Texture:
    """blocks: (height/8, width/8, channels) uint32 DCT words."""
    b = _host(np.ascontiguousarray(blocks, np.uint32))
    if b.size != (width // 8) * (height // 8) * channels:
        raise ValueError(f"blocks hold {b.size} words, {(width // 8) * (height // 8) * channels} needed")
    h = C.c_void_p()
    _check(lib().stf_create_dct_texture2d(width, height, channels, b.ctypes.data, C.byref(h)))
    return Texture(h.value, "dct2d", channels, 2)


def stf_create_material2d(width: int, height: int, level_texels: Sequence[np.ndarray]) -> Texture:
    lv = [_host(a) for a in level_texels]
    _check_level_sizes(lv, width, height, 8)
    arr = (C.c_void_p * len(lv))(*[a.ctypes.data for a in lv])
    h = C.c_void_p()
    _check(lib().stf_create_material2d(width, height, len(lv), arr, C.byref(h)))
    return Texture(h.value, "material", 6, 2)   # filtered: albedo RGB, roughness, normal x, y


def stf_create_sparse_grid3d(dims, fmt: int, leaf_origins: np.ndarray, leaf_values: np.ndarray,
                             background: float = 0.0) -> Texture:
    """leaf_origins: (n, 3) int32; leaf_values: n*512 values in storage format."""
    o = _host(np.asarray(leaf_origins, np.int32))
    v = _host(leaf_values)
    n = o.shape[0]
    if v.nbytes != n * 512 * FORMAT_BYTES[fmt]:
        raise ValueError("leaf_values has the wrong size for the format")
    h = C.c_void_p()
    _check(lib().stf_create_sparse_grid3d(int(dims[0]), int(dims[1]), int(dims[2]), fmt, n,
                                          o.ctypes.data if n else None, v.ctypes.data if n else None,
                                          float(background), C.byref(h)))
    return Texture(h.value, "grid3d", 1, 3)


def stf_destroy(tex: Texture):
    tex.destroy()


def stf_texture_bytes(tex: Texture) -> int:
    b = C.c_int64()
    _check(lib().stf_texture_bytes(tex.handle, C.byref(b)))
    return b.value


# Element type of every buffer the library reads or writes, by argument name
# (the library sees raw pointers, so a wrong type would be read or written
# past its end).
_DTYPES = {"queries": "float32", "sorted_queries": "float32", "sorted_out": "float32", "out": "float32",
           "out_rgb": "float32", "target": "float32", "grad_latents": "float32", "grad_mlp": "float32",
           "loss": "float32", "out_index": "int32", "order": "int32", "order_out": "int32",
           "positions": "int32", "sum": "float64", "sumsq": "float64", "workspace": "uint8"}


_TORCH_DTYPES = None


def _dev_ptr(t, name):
    global _TORCH_DTYPES
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if _TORCH_DTYPES is None:
        import torch
        _TORCH_DTYPES = {k: getattr(torch, v) for k, v in _DTYPES.items()}
    if t.dtype != _TORCH_DTYPES[name]:
        raise ValueError(f"{name} must be {_DTYPES[name]}, not {t.dtype}")
    return t.data_ptr()


def _stream(stream):
    """The HIP stream to launch on: the given torch stream, else torch's
    current stream on the current device (read as a raw handle when torch
    offers that, which skips building a Stream object: ~0.3 instead of ~3 us
    per call, which matters for small batches)."""
    if stream is not None:
        return stream.cuda_stream
    import torch
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return raw(torch.cuda.current_device())
    return torch.cuda.current_stream().cuda_stream


def _check_queries(tex: Texture, queries, n: int):
    """The library reads n x dims binary32 coordinates through a raw pointer."""
    if queries.numel() < n * tex.dims:
        raise ValueError(f"queries hold {queries.numel()} values, {n * tex.dims} needed ({tex.dims} per query)")


def _check_outputs(tex: Texture, n: int, filter: int, out, out_index):
    """The library writes n x channels results and n x index_width indices
    through raw pointers; refuse buffers that are too small."""
    if out is not None and out.numel() < n * tex.channels:
        raise ValueError(f"out holds {out.numel()} values, {n * tex.channels} needed")
    if out_index is not None and out_index.numel() < n * index_width(filter, tex.dims):
        raise ValueError(f"out_index holds {out_index.numel()} entries, {n * index_width(filter, tex.dims)} needed")


def stf_filter(tex: Texture, queries, filter: int, mode: int, seed: int, out, out_index=None, flags: int = 0,
               stream=None):
    """queries: (n, 2|3) float32 GPU tensor; out: (n, channels) float32 GPU
    tensor; out_index: None or (n, index_width(filter, dims)) int32 GPU
    tensor (stochastic)."""
    n = queries.shape[0]
    _check_queries(tex, queries, n)
    _check_outputs(tex, n, filter, out, out_index)
    _check(lib().stf_filter(tex.handle, _dev_ptr(queries, "queries"), n, filter, mode, seed & (2 ** 64 - 1),
                            _dev_ptr(out, "out"), _dev_ptr(out_index, "out_index"), flags, _stream(stream)))


def stf_filter_gaussian(tex: Texture, queries, sigma: float, mode: int, seed: int, out, out_index=None, stream=None):
    """Gaussian filtering of a 2D texture (STF_GAUSS_* modes); out: (n,
    channels) float32; out_index: None or (n, 2) int32 (stochastic modes)."""
    n = queries.shape[0]
    _check_queries(tex, queries, n)
    if out.numel() < n * tex.channels:
        raise ValueError("out is too small")
    if out_index is not None and out_index.numel() < 2 * n:
        raise ValueError("out_index is too small")
    _check(lib().stf_filter_gaussian(
        tex.handle, _dev_ptr(queries, "queries"), n, float(sigma), mode, seed & (2 ** 64 - 1), _dev_ptr(out, "out"),
        _dev_ptr(out_index, "out_index"), _stream(stream)))


def stf_filter_ewa(tex: Texture, queries, max_anisotropy: float, mode: int, seed: int, out, out_index=None,
                   stream=None):
    """EWA filtering: queries (n, 6) float32 GPU tensor; out (n, channels);
    out_index None or (n, 3) int32 (stochastic)."""
    n = queries.shape[0]
    if queries.numel() < 6 * n or out.numel() < n * tex.channels:
        raise ValueError("queries or out is too small")
    if out_index is not None and out_index.numel() < 3 * n:
        raise ValueError("out_index is too small")
    _check(lib().stf_filter_ewa(tex.handle, _dev_ptr(queries, "queries"), n, float(max_anisotropy), mode,
                                seed & (2 ** 64 - 1), _dev_ptr(out, "out"), _dev_ptr(out_index, "out_index"),
                                _stream(stream)))


def stf_filter_moments(tex: Texture, queries, filter: int, seed_base: int, n_seeds: int, sum_out, sumsq_out,
                       stream=None):
    n = queries.shape[0]
    _check_queries(tex, queries, n)
    if sum_out.numel() < n or sumsq_out.numel() < n:
        raise ValueError("sum/sumsq hold fewer than n values")
    _check(lib().stf_filter_moments(tex.handle, _dev_ptr(queries, "queries"), n, filter, seed_base, n_seeds,
                                    _dev_ptr(sum_out, "sum"), _dev_ptr(sumsq_out, "sumsq"), _stream(stream)))


def stf_shade_filter(material: Texture, queries, filter: int, mode: int, seed: int, out_rgb, out_index=None,
                     stream=None):
    """queries: (n, 9) float32 shading records; out_rgb: (n, 3) float32;
    out_index: None or (n, 3) int32 (x, y, level; stochastic mode)."""
    n = queries.shape[0]
    if queries.numel() < 9 * n or out_rgb.numel() < 3 * n:
        raise ValueError("queries or out_rgb is too small")
    if out_index is not None and out_index.numel() < 3 * n:
        raise ValueError("out_index is too small")
    _check(lib().stf_shade_filter(material.handle, _dev_ptr(queries, "queries"), n, filter, mode,
                                  seed & (2 ** 64 - 1), _dev_ptr(out_rgb, "out_rgb"),
                                  _dev_ptr(out_index, "out_index"), _stream(stream)))


# ----------------------------------------------------------------------------
# conveniences over the calls above (allocation of outputs only)
# ----------------------------------------------------------------------------
def filter(tex: Texture, queries, filter: int, mode: int, seed: int = 0, want_index: bool = False, stream=None):
    import torch
    n = queries.shape[0]
    out = torch.empty((n, tex.channels), dtype=torch.float32, device=queries.device)
    idx = None
    if want_index and mode in (STF_STOCHASTIC, STF_STOCHASTIC_FIS):
        idx = torch.empty((n, index_width(filter, tex.dims)), dtype=torch.int32, device=queries.device)
    stf_filter(tex, queries, filter, mode, seed, out, idx, 0, stream)
    return out, idx


# ----------------------------------------------------------------------------
# neural texture
# ----------------------------------------------------------------------------
def _declare_ntex(L):
    vp, i32, i64, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
    L.stf_ntex_param_count.argtypes, L.stf_ntex_param_count.restype = [], i32
    L.stf_ntex_create.argtypes = [i32, i32, i32, i32, vp, vp, C.POINTER(vp)]
    L.stf_ntex_destroy.argtypes, L.stf_ntex_destroy.restype = [vp], None
    L.stf_ntex_train.argtypes = [vp, vp, i32, i32, f32, f32, u64, vp, vp]
    L.stf_ntex_gradients.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    L.stf_ntex_get_params.argtypes = [vp, vp, vp]
    L.stf_ntex_prepare_inference.argtypes = [vp, vp]
    L.stf_ntex_filter.argtypes = [vp, vp, i64, i32, i32, u64, vp, vp, vp]
    for name in ("stf_ntex_create", "stf_ntex_train", "stf_ntex_gradients", "stf_ntex_get_params",
                 "stf_ntex_prepare_inference", "stf_ntex_filter"):
        getattr(L, name).restype = i32


class NeuralTexture:
    """Owning handle of an stf_neural."""

    def __init__(self, handle, tex_w, tex_h, lat_w, lat_h):
        self.handle, self.W, self.H, self.LW, self.LH = handle, tex_w, tex_h, lat_w, lat_h

    def destroy(self):
        if self.handle:
            lib().stf_ntex_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _ntex_lib():
    L = lib()
    if not getattr(L, "_ntex_declared", False):
        _declare_ntex(L)
        L._ntex_declared = True
    return L


def stf_ntex_param_count() -> int:
    return _ntex_lib().stf_ntex_param_count()


def stf_ntex_create(tex_w: int, tex_h: int, latents: np.ndarray, mlp: np.ndarray) -> NeuralTexture:
    """latents: (lat_h, lat_w, 8) float32; mlp: (5256,) float32."""
    lat = _host(np.asarray(latents, np.float32))
    m = _host(np.asarray(mlp, np.float32))
    if lat.ndim != 3 or lat.shape[2] != 8 or m.size != stf_ntex_param_count():
        raise ValueError("latents must be (lat_h, lat_w, 8) and mlp must hold 5256 values")
    h = C.c_void_p()
    _check(_ntex_lib().stf_ntex_create(tex_w, tex_h, lat.shape[1], lat.shape[0], lat.ctypes.data, m.ctypes.data,
                                       C.byref(h)))
    return NeuralTexture(h.value, tex_w, tex_h, lat.shape[1], lat.shape[0])


def stf_ntex_destroy(nt: NeuralTexture):
    nt.destroy()


def stf_ntex_train(nt: NeuralTexture, target, steps: int, batch: int, lr_latent: float, lr_mlp: float, seed: int,
                   loss=None, stream=None):
    """target: (tex_h, tex_w, 8) float32 GPU tensor; loss: None or (steps,) float32 GPU tensor."""
    _check(_ntex_lib().stf_ntex_train(nt.handle, _dev_ptr(target, "target"), steps, batch, lr_latent, lr_mlp,
                                      seed & (2 ** 64 - 1), _dev_ptr(loss, "loss"), _stream(stream)))


def stf_ntex_gradients(nt: NeuralTexture, target, positions, grad_latents, grad_mlp, loss=None, stream=None):
    _check(_ntex_lib().stf_ntex_gradients(nt.handle, _dev_ptr(target, "target"), _dev_ptr(positions, "positions"),
                                          positions.shape[0], _dev_ptr(grad_latents, "grad_latents"),
                                          _dev_ptr(grad_mlp, "grad_mlp"), _dev_ptr(loss, "loss"), _stream(stream)))


def stf_ntex_get_params(nt: NeuralTexture):
    lat = np.empty((nt.LH, nt.LW, 8), np.float32)
    m = np.empty(stf_ntex_param_count(), np.float32)
    _check(_ntex_lib().stf_ntex_get_params(nt.handle, lat.ctypes.data, m.ctypes.data))
    return lat, m


def stf_ntex_prepare_inference(nt: NeuralTexture, stream=None):
    _check(_ntex_lib().stf_ntex_prepare_inference(nt.handle, _stream(stream)))


def stf_ntex_filter(nt: NeuralTexture, queries, filter: int, mode: int, seed: int, out, out_index=None, stream=None):
    """queries: (n, 2) float32 GPU tensor; out: (n, 8) float32 GPU tensor;
    out_index: None or (n, 2) int32 (stochastic mode)."""
    n = queries.shape[0]
    if queries.numel() < 2 * n or out.numel() < 8 * n:
        raise ValueError("queries or out is too small")
    if out_index is not None and out_index.numel() < 2 * n:
        raise ValueError("out_index is too small")
    _check(_ntex_lib().stf_ntex_filter(nt.handle, _dev_ptr(queries, "queries"), n, filter, mode,
                                       seed & (2 ** 64 - 1), _dev_ptr(out, "out"), _dev_ptr(out_index, "out_index"),
                                       _stream(stream)))


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
STF_SERVE_QUERIES_ON_DEVICE, STF_SERVE_RESULTS_ON_DEVICE = 1, 2


class ServerConfig(C.Structure):
    _fields_ = [("memory_budget_bytes", C.c_int64), ("max_resident", C.c_int32), ("chunk_queries", C.c_int32)]


class ServeStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("completed", "cancelled", "queries", "launches", "rounds", "peak_resident",
                                         "peak_arena_bytes", "pending", "resident")] + \
               [(n, C.c_double) for n in ("p50_ms", "p99_ms", "max_ms", "mean_ms", "lookups_per_s", "span_s")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServeRequest(C.Structure):
    _fields_ = [("tex", C.c_void_p), ("queries", C.c_void_p), ("n", C.c_int64), ("filter", C.c_int32),
                ("seed", C.c_uint64), ("out", C.c_void_p), ("out_index", C.c_void_p), ("arrival_s", C.c_double)]


def _declare_server(L):
    vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    L.stf_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(vp)]
    L.stf_server_destroy.argtypes, L.stf_server_destroy.restype = [vp], None
    L.stf_server_submit.argtypes = [vp, vp, vp, i64, i32, u64, vp, vp, u32, C.POINTER(u64)]
    L.stf_server_poll.argtypes = [vp, u64, C.POINTER(i32)]
    L.stf_server_wait.argtypes = [vp, u64, dbl]
    L.stf_server_cancel.argtypes = [vp, u64]
    L.stf_server_release.argtypes = [vp, u64]
    L.stf_server_stats.argtypes = [vp, C.POINTER(ServeStats)]
    L.stf_server_reset_stats.argtypes = [vp]
    L.stf_server_replay.argtypes = [vp, C.POINTER(ServeRequest), i64, u32, dbl]
    for name in ("stf_server_create", "stf_server_submit", "stf_server_poll", "stf_server_wait", "stf_server_cancel",
                 "stf_server_release", "stf_server_stats", "stf_server_reset_stats", "stf_server_replay"):
        getattr(L, name).restype = i32


def _srv_lib():
    L = lib()
    if not getattr(L, "_srv_declared", False):
        _declare_server(L)
        L._srv_declared = True
    return L


class Server:
    """Owning handle of an stf_server; keeps host buffers of in-flight
    requests alive until they are released."""

    def __init__(self, handle):
        self.handle = handle
        self._keep = {}

    def destroy(self):
        if self.handle:
            _srv_lib().stf_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def stf_server_create(memory_budget_bytes: int, max_resident: int, chunk_queries: int) -> Server:
    cfg = ServerConfig(memory_budget_bytes, max_resident, chunk_queries)
    h = C.c_void_p()
    _check(_srv_lib().stf_server_create(C.byref(cfg), C.byref(h)))
    return Server(h.value)


def stf_server_destroy(s: Server):
    s.destroy()


def _buf(x, name):
    """(pointer, on_device) of a torch tensor or numpy array."""
    if x is None:
        return None, None
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError(f"{name} must be contiguous")
        if x.dtype != np.dtype(_DTYPES[name]):
            raise ValueError(f"{name} must be {_DTYPES[name]}, not {x.dtype}")
        return x.ctypes.data, False
    return _dev_ptr(x, name), True


def stf_server_submit(s: Server, tex: Texture, queries, filter: int, seed: int, out, out_index=None) -> int:
    """queries/out/out_index: numpy arrays (host) or GPU tensors (device);
    queries and results may live on different sides."""
    qp, qdev = _buf(queries, "queries")
    op, odev = _buf(out, "out")
    ip, idev = _buf(out_index, "out_index")
    if ip is not None and idev != odev:
        raise ValueError("out and out_index must be on the same side")
    flags = (STF_SERVE_QUERIES_ON_DEVICE if qdev else 0) | (STF_SERVE_RESULTS_ON_DEVICE if odev else 0)
    t = C.c_uint64()
    _check(_srv_lib().stf_server_submit(s.handle, tex.handle, qp, queries.shape[0], filter, seed & (2 ** 64 - 1), op,
                                        ip, flags, C.byref(t)))
    s._keep[t.value] = (queries, out, out_index)
    return t.value


def stf_server_poll(s: Server, ticket: int) -> bool:
    d = C.c_int32()
    _check(_srv_lib().stf_server_poll(s.handle, ticket, C.byref(d)))
    return bool(d.value)


def stf_server_wait(s: Server, ticket: int, timeout_s: float = 60.0):
    _check(_srv_lib().stf_server_wait(s.handle, ticket, timeout_s))


def stf_server_cancel(s: Server, ticket: int):
    _check(_srv_lib().stf_server_cancel(s.handle, ticket))


def stf_server_release(s: Server, ticket: int):
    _check(_srv_lib().stf_server_release(s.handle, ticket))
    s._keep.pop(ticket, None)


def stf_server_stats(s: Server) -> dict:
    st = ServeStats()
    _check(_srv_lib().stf_server_stats(s.handle, C.byref(st)))
    return st.as_dict()


def stf_server_reset_stats(s: Server):
    _check(_srv_lib().stf_server_reset_stats(s.handle))


def stf_server_replay(s: Server, requests, flags: int, timeout_s: float = 120.0):
    """requests: sequence of (tex, queries_ptr, n, filter, seed, out_ptr,
    out_index_ptr_or_None, arrival_s) with raw pointers (the caller keeps the
    buffers alive); flags: STF_SERVE_* bits."""
    arr = (ServeRequest * len(requests))()
    for k, (tex, qp, n, f, seed, op, ip, t) in enumerate(requests):
        arr[k] = ServeRequest(tex.handle, qp, n, f, seed & (2 ** 64 - 1), op, ip, t)
    _check(_srv_lib().stf_server_replay(s.handle, arr, len(requests), flags, timeout_s))


# ----------------------------------------------------------------------------
# Morton-ordered query streams
# ----------------------------------------------------------------------------
STF_ORDER_SCATTER = 1


def _sort_lib():
    L = lib()
    if not getattr(L, "_sort_declared", False):
        vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        L.stf_sort_workspace_bytes.argtypes = [i64, C.POINTER(C.c_size_t)]
        L.stf_sort_queries.argtypes = [vp, vp, i64, vp, vp, vp, C.c_size_t, vp]
        L.stf_filter_ordered.argtypes = [vp, vp, vp, i64, i32, i32, u64, vp, vp, u32, vp]
        L.stf_sort_queries_noalloc.argtypes = [vp, vp, i64, vp, vp, vp]
        for name in ("stf_sort_workspace_bytes", "stf_sort_queries", "stf_filter_ordered", "stf_sort_queries_noalloc"):
            getattr(L, name).restype = i32
        L._sort_declared = True
    return L


def stf_sort_workspace_bytes(n: int) -> int:
    b = C.c_size_t()
    _check(_sort_lib().stf_sort_workspace_bytes(n, C.byref(b)))
    return b.value


def stf_sort_queries(tex: Texture, queries, sorted_out, order_out, workspace, stream=None):
    """workspace: a uint8 GPU tensor of at least stf_sort_workspace_bytes(n);
    sorted_out: like queries; order_out: n int32."""
    n = queries.shape[0]
    _check_queries(tex, queries, n)
    if sorted_out.numel() < n * tex.dims or order_out.numel() < n:
        raise ValueError("sorted_out or order_out is too small")
    _check(_sort_lib().stf_sort_queries(tex.handle, _dev_ptr(queries, "queries"), n,
                                        _dev_ptr(sorted_out, "sorted_out"), _dev_ptr(order_out, "order_out"),
                                        _dev_ptr(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                                        _stream(stream)))


def stf_filter_ordered(tex: Texture, sorted_queries, order, filter: int, mode: int, seed: int, out, out_index=None,
                       flags: int = 0, stream=None):
    _check_queries(tex, sorted_queries, sorted_queries.shape[0])
    _check_outputs(tex, sorted_queries.shape[0], filter, out, out_index)
    if order.numel() < sorted_queries.shape[0]:
        raise ValueError("order is shorter than the query stream")
    _check(_sort_lib().stf_filter_ordered(tex.handle, _dev_ptr(sorted_queries, "sorted_queries"),
                                          _dev_ptr(order, "order"), sorted_queries.shape[0], filter, mode,
                                          seed & (2 ** 64 - 1), _dev_ptr(out, "out"), _dev_ptr(out_index, "out_index"),
                                          flags, _stream(stream)))


STF_SORT_NOALLOC_MAX_QUERIES = 1 << 20


def stf_sort_queries_noalloc(tex: Texture, queries, sorted_queries, order, stream=None):
    """The allocation-free sort (its workspace is a fixed device array of the
    library; n <= STF_SORT_NOALLOC_MAX_QUERIES)."""
    n = queries.shape[0]
    _check_queries(tex, queries, n)
    if sorted_queries.numel() < n * tex.dims or order.numel() < n:
        raise ValueError("sorted_queries or order is too small")
    _check(_sort_lib().stf_sort_queries_noalloc(tex.handle, _dev_ptr(queries, "queries"), n,
                                                _dev_ptr(sorted_queries, "sorted_queries"),
                                                _dev_ptr(order, "order"), _stream(stream)))


def sort_queries(tex: Texture, queries, stream=None):
    """Convenience: allocate outputs and workspace, return (sorted, order)."""
    import torch
    n = queries.shape[0]
    sorted_q = torch.empty_like(queries)
    order = torch.empty(n, dtype=torch.int32, device=queries.device)
    ws = torch.empty(max(1, stf_sort_workspace_bytes(n)), dtype=torch.uint8, device=queries.device)
    stf_sort_queries(tex, queries, sorted_q, order, ws, stream)
    return sorted_q, order
