"""ctypes binding of libsrp (include/srp.h).

Argument marshalling only: every step of the SRP path runs in the library's
HIP kernels. PyTorch supplies device memory and the current stream. There is
no CPU fallback: if libsrp.so is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsrp.so")

SRP_OK, SRP_ERR_INVALID_ARG, SRP_ERR_OUT_OF_MEMORY, SRP_ERR_DEVICE, SRP_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
DTYPES = {"fp32": 0, "bf16": 1, "fp16": 2, "fp64": 3}


def sample_torch_dtype(dtype: str):
    """Storage type of GCC samples for a map dtype (fp64 maps read float32 samples)."""
    import torch
    return {"fp32": torch.float32, "fp64": torch.float32, "bf16": torch.bfloat16,
            "fp16": torch.float16}[dtype]
# dtypes srp_map_conventional has a kernel for (others return SRP_ERR_UNSUPPORTED)
CONVENTIONAL_DTYPES = ("fp32", "fp64", "bf16", "fp16")


def conventional_supports(dtype: str) -> bool:
    return dtype in CONVENTIONAL_DTYPES


FIELDS = {"near": 0, "far": 1}
WINDOWS = {"hann": 0, "sqrt_hann": 1, "rect": 2}
PHAT = 0

# exported symbols of include/srp.h
EXPORTS = ("srp_pair_layout", "srp_geometry", "srp_geometry_query", "srp_geometry_destroy",
           "srp_cross_spectra_workspace", "srp_cross_spectra", "srp_cross_spectra_noalloc",
           "srp_gcc_samples", "srp_gcc_samples_frames", "srp_spectra_lowp_bytes",
           "srp_spectra_lowp",
           "srp_map_conventional", "srp_map_nyquist", "srp_map_nyquist_batched_workspace",
           "srp_map_nyquist_batched", "srp_nyquist_weights_bytes", "srp_nyquist_weights",
           "srp_map_nyquist_cached", "srp_map_nyquist_points", "srp_argmax", "srp_last_error",
           "srp_version")
BATCH_MAX_F = 8            # frames per item of a batched launch, FP32 samples
BATCH_MAX_F_MX = 16        # ... BF16 / FP16 samples (matrix-core tile)


def batch_max_frames(dtype: str) -> int:
    return BATCH_MAX_F if dtype == "fp32" else BATCH_MAX_F_MX


class SrpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libsrp status {status}: {msg}")
        self.status = status


class GeometryInfo(C.Structure):
    _fields_ = [("M", C.c_int32), ("P", C.c_int32), ("L", C.c_int32), ("K", C.c_int32),
                ("J", C.c_int64), ("S", C.c_int64), ("h_max", C.c_int32), ("n_aux", C.c_int32),
                ("field", C.c_int32), ("window", C.c_int32), ("c", C.c_double),
                ("fs", C.c_double), ("f_max", C.c_double), ("T", C.c_double)]


class BatchItem(C.Structure):
    _fields_ = [("g", C.c_void_p), ("xi_offset", C.c_int64), ("F", C.c_int32),
                ("reserved", C.c_int32), ("map", C.c_void_p), ("peaks", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """Loads libsrp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2012_09499_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.srp_pair_layout.argtypes = [vp, i32, dbl, dbl, i32, vp, vp, vp]
    L.srp_geometry.argtypes = [vp, i32, vp, i64, i32, dbl, dbl, i32, dbl, i32, i32, vp,
                               C.POINTER(vp)]
    L.srp_geometry_query.argtypes = [vp, C.POINTER(GeometryInfo), vp, vp]
    L.srp_geometry_destroy.argtypes = [vp]
    L.srp_geometry_destroy.restype = None
    L.srp_cross_spectra_workspace.argtypes = [vp, i32, C.POINTER(C.c_size_t)]
    L.srp_cross_spectra.argtypes = [vp, vp, i32, i32, vp, C.c_size_t, vp, vp]
    L.srp_cross_spectra_noalloc.argtypes = [vp, vp, i32, i32, vp, vp]
    L.srp_gcc_samples.argtypes = [vp, vp, i32, i32, vp, vp]
    L.srp_gcc_samples_frames.argtypes = [vp, vp, i32, i32, i32, vp, C.c_size_t, vp, vp]
    L.srp_spectra_lowp_bytes.argtypes = [vp, i32, i32, C.POINTER(C.c_size_t)]
    L.srp_spectra_lowp.argtypes = [vp, vp, i32, i32, vp, C.c_size_t, vp]
    L.srp_map_conventional.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.srp_map_nyquist.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.srp_argmax.argtypes = [vp, i32, i64, vp, vp]
    L.srp_map_nyquist_batched_workspace.argtypes = [i32, C.POINTER(C.c_size_t)]
    L.srp_map_nyquist_batched.argtypes = [vp, i32, vp, i64, i32, vp, C.c_size_t, vp]
    L.srp_nyquist_weights_bytes.argtypes = [vp, i32, C.POINTER(C.c_size_t)]
    L.srp_nyquist_weights.argtypes = [vp, i32, vp, C.c_size_t, vp]
    L.srp_map_nyquist_cached.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    L.srp_map_nyquist_points.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    L.srp_last_error.restype = C.c_char_p
    L.srp_last_error.argtypes = []
    L.srp_version.restype = C.c_char_p
    L.srp_version.argtypes = []
    for name in EXPORTS:
        if name not in ("srp_geometry_destroy", "srp_last_error", "srp_version"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != SRP_OK:
        raise SrpError(status, lib().srp_last_error().decode())


def version() -> str:
    return lib().srp_version().decode()


def _stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def pair_layout(mic_xyz, c: float, f_max: float, n_aux: int):
    """Host-only N_p, packed offsets and S (no device work)."""
    mic = np.ascontiguousarray(mic_xyz, dtype=np.float64)
    M = mic.shape[0]
    P = M * (M - 1) // 2
    N_p = np.zeros(max(P, 1), dtype=np.int32)
    off = np.zeros(P + 1, dtype=np.int64)
    S = C.c_int64(0)
    _check(lib().srp_pair_layout(mic.ctypes.data, M, float(c), float(f_max), int(n_aux),
                                 N_p.ctypes.data, off.ctypes.data, C.addressof(S)))
    return N_p[:P], off, int(S.value)


def _need_cuda(t, name, dtype=None, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Geometry:
    """Device-resident array geometry (srp_geometry)."""

    def __init__(self, mic_xyz, candidates, *, fs: float, L: int, c: float = 343.0,
                 f_max: Optional[float] = None, n_aux: int = 2, field: str = "near",
                 window: str = "hann", stream=None):
        mic = np.ascontiguousarray(mic_xyz, dtype=np.float64)
        cand = np.ascontiguousarray(candidates, dtype=np.float64).reshape(-1, 3)
        f_max = fs / 2.0 if f_max is None else f_max
        h = C.c_void_p()
        _check(lib().srp_geometry(mic.ctypes.data, mic.shape[0], cand.ctypes.data,
                                  cand.shape[0], FIELDS[field], float(c), float(fs), int(L),
                                  float(f_max), int(n_aux), WINDOWS[window],
                                  _stream_handle(stream), C.byref(h)))
        self._h = h
        info = GeometryInfo()
        P = mic.shape[0] * (mic.shape[0] - 1) // 2
        self.N_p = np.zeros(P, dtype=np.int32)
        self.offsets = np.zeros(P + 1, dtype=np.int64)
        _check(lib().srp_geometry_query(h, C.byref(info), self.N_p.ctypes.data,
                                        self.offsets.ctypes.data))
        self.info = info
        self.M, self.P, self.L, self.K = info.M, info.P, info.L, info.K
        self.J, self.S, self.h_max, self.n_aux = info.J, info.S, info.h_max, info.n_aux
        self.fs, self.c, self.f_max, self.T = info.fs, info.c, info.f_max, info.T
        self.field = field
        # samples per frame without the layout's alignment gaps (N P of Sec. 3.3)
        self.W = 2 * (self.N_p.astype(np.int64) + self.n_aux) + 1
        self.W_total = int(self.W.sum())

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("geometry closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().srp_geometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, F: int) -> int:
        n = C.c_size_t(0)
        _check(lib().srp_cross_spectra_workspace(self.handle, int(F), C.byref(n)))
        return int(n.value)


def cross_spectra(g: Geometry, frames, out=None, workspace=None, stream=None):
    """frames [F][M][L] float32 -> psi [F][P][K] complex64 (srp_cross_spectra)."""
    import torch
    _need_cuda(frames, "frames", torch.float32)
    F = frames.shape[0]
    if frames.dim() != 3 or frames.shape[1] != g.M or frames.shape[2] != g.L:
        raise ValueError(f"frames must be [F][{g.M}][{g.L}]")
    nbytes = g.workspace_bytes(F)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=frames.device)
    if out is None:
        out = torch.empty((F, g.P, g.K), dtype=torch.complex64, device=frames.device)
    _need_cuda(out, "psi", torch.complex64, (F, g.P, g.K))
    _check(lib().srp_cross_spectra(g.handle, frames.data_ptr(), F, PHAT, workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(), out.data_ptr(),
                                   _stream_handle(stream)))
    return out


CROSS_STATIC_BYTES = 64 << 20  # the library's static phasor buffer per GPU


def cross_spectra_noalloc(g: Geometry, frames, out, stream=None):
    """frames [F][M][L] float32 -> psi [F][P][K] complex64 into `out`, staging the
    per-microphone phasors in the library's static buffer (srp_cross_spectra_noalloc).
    Nothing is allocated: the caller passes the output."""
    import torch
    _need_cuda(frames, "frames", torch.float32)
    F = frames.shape[0]
    if frames.dim() != 3 or frames.shape[1] != g.M or frames.shape[2] != g.L:
        raise ValueError(f"frames must be [F][{g.M}][{g.L}]")
    _need_cuda(out, "psi", torch.complex64, (F, g.P, g.K))
    _check(lib().srp_cross_spectra_noalloc(g.handle, frames.data_ptr(), F, PHAT, out.data_ptr(),
                                           _stream_handle(stream)))
    return out


def gcc_samples(g: Geometry, psi, out=None, dtype: str = "fp32", stream=None):
    """psi [F][P][K] complex64 -> xi [F][S] (float32, bfloat16 or float16) (srp_gcc_samples)."""
    import torch
    _need_cuda(psi, "psi", torch.complex64)
    F = psi.shape[0]
    tdt = sample_torch_dtype(dtype)
    if out is None:
        out = torch.empty((F, g.S), dtype=tdt, device=psi.device)
    _need_cuda(out, "xi", tdt, (F, g.S))
    _check(lib().srp_gcc_samples(g.handle, psi.data_ptr(), F, DTYPES[dtype if dtype != "fp64" else "fp32"],
                                 out.data_ptr(), _stream_handle(stream)))
    return out


def gcc_samples_frames(g: Geometry, frames, out=None, dtype: str = "fp32", workspace=None,
                       stream=None):
    """frames [F][M][L] float32 -> xi [F][S] in one call (srp_gcc_samples_frames):
    the cross-spectra are formed on chip from the per-microphone phasors."""
    import torch
    _need_cuda(frames, "frames", torch.float32)
    F = frames.shape[0]
    if frames.dim() != 3 or frames.shape[1] != g.M or frames.shape[2] != g.L:
        raise ValueError(f"frames must be [F][{g.M}][{g.L}]")
    if workspace is None:
        workspace = torch.empty(g.workspace_bytes(F), dtype=torch.uint8, device=frames.device)
    tdt = sample_torch_dtype(dtype)
    if out is None:
        out = torch.empty((F, g.S), dtype=tdt, device=frames.device)
    _need_cuda(out, "xi", tdt, (F, g.S))
    _check(lib().srp_gcc_samples_frames(g.handle, frames.data_ptr(), F, PHAT,
                                        DTYPES[dtype if dtype != "fp64" else "fp32"],
                                        workspace.data_ptr(),
                                        workspace.numel() * workspace.element_size(),
                                        out.data_ptr(), _stream_handle(stream)))
    return out


def unpack_samples(g: Geometry, xi):
    """Host copy of xi without the alignment gaps: [F][sum_p W_p] float64, pair-major."""
    h = xi.detach().float().cpu().numpy().astype(np.float64)
    cols = np.concatenate([np.arange(int(o), int(o) + int(w))
                           for o, w in zip(g.offsets[:-1], g.W)])
    return h[:, cols]


def _map_outputs(g, F, device, want_map, want_peaks, map_out, peaks_out):
    import torch
    m = map_out
    if m is None and want_map:
        m = torch.empty((F, g.J), dtype=torch.float32, device=device)
    if m is not None:
        _need_cuda(m, "map", torch.float32, (F, g.J))
    pk = peaks_out
    if pk is None and want_peaks:
        pk = torch.empty((F, 2), dtype=torch.int64, device=device)
    if pk is not None:
        _need_cuda(pk, "peaks", torch.int64, (F, 2))
    return m, pk


def map_nyquist(g: Geometry, xi, dtype: str = "fp32", want_map: bool = True,
                want_peaks: bool = True, map_out=None, peaks_out=None, stream=None):
    """xi [F][S] -> (map [F][J] float32 | None, peaks [F][2] int64 | None) (srp_map_nyquist).

    xi must be stored in the type srp_gcc_samples writes for `dtype`.
    """
    _need_cuda(xi, "xi", sample_torch_dtype(dtype))
    F = xi.shape[0]
    if xi.shape[1] != g.S:
        raise ValueError(f"xi must be [F][{g.S}]")
    m, pk = _map_outputs(g, F, xi.device, want_map, want_peaks, map_out, peaks_out)
    _check(lib().srp_map_nyquist(g.handle, xi.data_ptr(), F, DTYPES[dtype],
                                 m.data_ptr() if m is not None else None,
                                 pk.data_ptr() if pk is not None else None,
                                 _stream_handle(stream)))
    return m, pk


def spectra_lowp_buffer(g: Geometry, F: int, dtype: str = "bf16", device="cuda"):
    """An uninitialised [F][P][Kp][2] buffer for spectra_lowp."""
    import torch
    n = C.c_size_t(0)
    _check(lib().srp_spectra_lowp_bytes(g.handle, int(F), DTYPES[dtype], C.byref(n)))
    Kp = int(n.value) // (4 * F * g.P)
    return torch.empty((F, g.P, Kp, 2), dtype=sample_torch_dtype(dtype), device=device)


def spectra_lowp(g: Geometry, psi, dtype: str = "bf16", out=None, stream=None):
    """psi [F][P][K] complex64 -> weighted spectra [F][P][Kp][2] in bf16/fp16
    (srp_spectra_lowp): the input of the BF16/FP16 conventional map."""
    import torch
    _need_cuda(psi, "psi", torch.complex64)
    F = psi.shape[0]
    if out is None:
        out = spectra_lowp_buffer(g, F, dtype, psi.device)
    _need_cuda(out, "spectra", sample_torch_dtype(dtype))
    if out.dim() != 4 or tuple(out.shape[:2]) != (F, g.P) or out.shape[3] != 2:
        raise ValueError(f"spectra must be [{F}][{g.P}][Kp][2]")
    _check(lib().srp_spectra_lowp(g.handle, psi.data_ptr(), F, DTYPES[dtype], out.data_ptr(),
                                  out.numel() * out.element_size(), _stream_handle(stream)))
    return out


def map_conventional(g: Geometry, psi, dtype: str = "fp32", want_map: bool = True,
                     want_peaks: bool = True, map_out=None, peaks_out=None, stream=None):
    """psi [F][P][K] complex64 (FP32/FP64) or the srp_spectra_lowp output
    [F][P][Kp][2] (BF16/FP16) -> (map, peaks) (srp_map_conventional)."""
    import torch
    F = psi.shape[0]
    if dtype in ("bf16", "fp16"):
        _need_cuda(psi, "spectra", sample_torch_dtype(dtype))
        if psi.dim() != 4 or tuple(psi.shape[1:2]) != (g.P,) or psi.shape[3] != 2:
            raise ValueError(f"BF16/FP16 spectra must be [F][{g.P}][Kp][2] (spectra_lowp)")
    else:
        _need_cuda(psi, "psi", torch.complex64)
        if tuple(psi.shape[1:]) != (g.P, g.K):
            raise ValueError(f"psi must be [F][{g.P}][{g.K}]")
    m, pk = _map_outputs(g, F, psi.device, want_map, want_peaks, map_out, peaks_out)
    _check(lib().srp_map_conventional(g.handle, psi.data_ptr(), F, DTYPES[dtype],
                                      m.data_ptr() if m is not None else None,
                                      pk.data_ptr() if pk is not None else None,
                                      _stream_handle(stream)))
    return m, pk


def nyquist_weights_bytes(g: Geometry, dtype: str = "bf16") -> int:
    """Bytes of the cached weight matrix W [J][Sw] (srp_nyquist_weights_bytes)."""
    n = C.c_size_t(0)
    _check(lib().srp_nyquist_weights_bytes(g.handle, DTYPES[dtype], C.byref(n)))
    return int(n.value)


def nyquist_weights(g: Geometry, dtype: str = "bf16", out=None, stream=None):
    """Builds the float64-exact, once-rounded weight matrix W [J][Sw] (srp_nyquist_weights)."""
    import torch
    nbytes = nyquist_weights_bytes(g, dtype)
    cols = nbytes // (2 * g.J)
    tdt = sample_torch_dtype(dtype)
    if out is None:
        out = torch.empty((g.J, cols), dtype=tdt, device="cuda")
    _need_cuda(out, "weights", tdt, (g.J, cols))
    _check(lib().srp_nyquist_weights(g.handle, DTYPES[dtype], out.data_ptr(), nbytes,
                                     _stream_handle(stream)))
    return out


def map_nyquist_cached(g: Geometry, weights, xi, dtype: str = "bf16", want_map: bool = True,
                       want_peaks: bool = True, map_out=None, peaks_out=None, stream=None):
    """xi [F][S] + cached W -> (map [F][J] | None, peaks [F][2] | None) (srp_map_nyquist_cached)."""
    import torch
    tdt = sample_torch_dtype(dtype)
    _need_cuda(xi, "xi", tdt)
    _need_cuda(weights, "weights", tdt)
    F = xi.shape[0]
    if tuple(xi.shape) != (F, g.S):
        raise ValueError(f"xi must have shape (F, {g.S})")
    if weights.shape[0] != g.J or weights.numel() * 2 < nyquist_weights_bytes(g, dtype):
        raise ValueError("weights do not match this geometry")
    m = map_out if map_out is not None else (
        torch.empty((F, g.J), dtype=torch.float32, device=xi.device) if want_map else None)
    pk = peaks_out if peaks_out is not None else (
        torch.empty((F, 2), dtype=torch.int64, device=xi.device) if want_peaks else None)
    if m is not None:
        _need_cuda(m, "map", torch.float32, (F, g.J))
    if pk is not None:
        _need_cuda(pk, "peaks", torch.int64, (F, 2))
    _check(lib().srp_map_nyquist_cached(g.handle, weights.data_ptr(), xi.data_ptr(), F,
                                        DTYPES[dtype], m.data_ptr() if m is not None else None,
                                        pk.data_ptr() if pk is not None else None,
                                        _stream_handle(stream)))
    return m, pk


def map_nyquist_points(g: Geometry, xi, points, out=None, stream=None):
    """xi [F][S] float32, points [F][Q][3] float64 (CUDA) -> values [F][Q] float32
    (srp_map_nyquist_points)."""
    import torch
    _need_cuda(xi, "xi", torch.float32)
    F = xi.shape[0]
    if tuple(xi.shape) != (F, g.S):
        raise ValueError(f"xi must have shape (F, {g.S})")
    _need_cuda(points, "points", torch.float64)
    if points.dim() != 3 or points.shape[0] != F or points.shape[2] != 3:
        raise ValueError("points must have shape (F, Q, 3)")
    Q = points.shape[1]
    if out is None:
        out = torch.empty((F, Q), dtype=torch.float32, device=xi.device)
    _need_cuda(out, "values", torch.float32, (F, Q))
    _check(lib().srp_map_nyquist_points(g.handle, xi.data_ptr(), F, points.data_ptr(), Q,
                                        out.data_ptr(), _stream_handle(stream)))
    return out


def batched_workspace_bytes(n_items: int) -> int:
    n = C.c_size_t(0)
    _check(lib().srp_map_nyquist_batched_workspace(int(n_items), C.byref(n)))
    return int(n.value)


def map_nyquist_batched(items, xi_arena, workspace, stream=None, dtype: str = "fp32"):
    """One ragged launch over many arrays (srp_map_nyquist_batched).

    items: list of (Geometry, xi_offset, F, map tensor or None, peaks tensor or None);
    xi_arena: CUDA tensor holding every item's samples, float32 for dtype "fp32",
    bfloat16 / float16 for "bf16" / "fp16" (then every xi_offset is a multiple
    of 8); workspace: CUDA uint8 tensor of at least
    batched_workspace_bytes(len(items)) bytes.
    """
    import torch
    if dtype not in ("fp32", "bf16", "fp16"):
        raise ValueError(f"batched dtype must be fp32, bf16 or fp16, not {dtype!r}")
    _need_cuda(xi_arena, "xi_arena", sample_torch_dtype(dtype))
    n = len(items)
    arr = (BatchItem * n)()
    for i, (g, off, F, m, pk) in enumerate(items):
        if m is not None:
            _need_cuda(m, "map", torch.float32, (F, g.J))
        if pk is not None:
            _need_cuda(pk, "peaks", torch.int64, (F, 2))
        arr[i].g = g.handle
        arr[i].xi_offset = int(off)
        arr[i].F = int(F)
        arr[i].map = m.data_ptr() if m is not None else None
        arr[i].peaks = pk.data_ptr() if pk is not None else None
    _check(lib().srp_map_nyquist_batched(arr, n, xi_arena.data_ptr(), xi_arena.numel(),
                                         DTYPES[dtype],
                                         workspace.data_ptr(),
                                         workspace.numel() * workspace.element_size(),
                                         _stream_handle(stream)))


def argmax(srp_map, peaks_out=None, stream=None):
    """map [F][J] float32 -> peaks [F][2] int64 (srp_argmax)."""
    import torch
    _need_cuda(srp_map, "map", torch.float32)
    F, J = srp_map.shape
    pk = peaks_out
    if pk is None:
        pk = torch.empty((F, 2), dtype=torch.int64, device=srp_map.device)
    _need_cuda(pk, "peaks", torch.int64, (F, 2))
    _check(lib().srp_argmax(srp_map.data_ptr(), F, J, pk.data_ptr(), _stream_handle(stream)))
    return pk


def decode_peaks(peaks) -> Tuple[np.ndarray, np.ndarray]:
    """srp_peak records [F][2] int64 -> (index int64 [F], value float32 [F]) on the host."""
    h = peaks.detach().cpu().contiguous().numpy()
    idx = h[:, 0].copy()
    val = h.view(np.int32)[:, 2].copy().view(np.float32)
    return idx, val
