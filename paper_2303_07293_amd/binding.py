"""ctypes binding of libsst.so, the C ABI of the shift-and-stack search.

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  PyTorch provides device memory and the stream; NumPy arrays
carry the host-side inputs (timestamps, velocity grids).  If the compiled
library is missing or cannot be loaded every call raises: there is no other
implementation behind these functions.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from ._build import LIB

SST_OK = 0
SST_E_ARG = -1
SST_E_UNSORTED = -2
SST_E_RANGE = -3
SST_E_WORKSPACE = -4
SST_E_DEVICE = -5
SST_E_UNSUPPORTED = -6

SST_F32, SST_BF16, SST_F16 = 0, 1, 2
SST_OP_STACK, SST_OP_DETECT, SST_OP_STATS, SST_OP_QUANT, SST_OP_REFINE = 0, 1, 2, 3, 4
SST_SUM, SST_MEAN = 0, 1

# the 32-byte sst_candidate record
CANDIDATE_DTYPE = np.dtype([
    ("ivx", np.int32), ("ivy", np.int32), ("x", np.int32), ("y", np.int32),
    ("snr", np.float32), ("flux", np.float32), ("coverage", np.int32), ("rank", np.int32),
])

EXPORTS = ("sst_shift_table", "sst_workspace_bytes", "sst_quantize", "sst_median_subtract", "sst_coadd", "sst_bin2x2",
           "sst_frame_stats", "sst_stack", "sst_detect", "sst_refine", "sst_plan_detect", "sst_plan_run",
           "sst_plan_destroy", "sst_batch_workspace_bytes", "sst_batch_create", "sst_batch_run", "sst_batch_destroy",
           "sst_shape_info", "sst_workspace_bytes_shape", "sst_plan_detect_shape", "sst_plan_info",
           "sst_profile_begin", "sst_profile_end", "sst_last_error", "sst_version", "sst_detect_noalloc",
           "sst_noalloc_scratch_bytes", "sst_set_half_search", "sst_set_slot_keep", "sst_set_stack_shape",
           "sst_set_two_pass")


class SstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sst error {code}: {msg}")
        self.code = code


_lib = None

_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_f = ctypes.c_float
_sz = ctypes.c_size_t


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libsst.so (built by `_build.build`) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    lib.sst_shift_table.argtypes = [_p, _i, _d, _p, _i, _p]
    lib.sst_shift_table.restype = _i
    lib.sst_workspace_bytes.argtypes = [_i, _i, _i, _i, _p, _d, _p, _i, _p, _i, _i]
    lib.sst_workspace_bytes.restype = _sz
    lib.sst_workspace_bytes_shape.argtypes = [_i, _i, _i, _i, _i, _p, _d, _p, _i, _p, _i, _i]
    lib.sst_workspace_bytes_shape.restype = _sz
    lib.sst_shape_info.argtypes = [_i, _p, _p]
    lib.sst_shape_info.restype = _i
    lib.sst_plan_detect_shape.argtypes = [_i, _i, _i, _i, _p, _d, _p, _i, _p, _i, _f, _i, _i, _p, _sz, _p, _p]
    lib.sst_plan_detect_shape.restype = _i
    lib.sst_plan_info.argtypes = [_p, _p, _p, _p]
    lib.sst_plan_info.restype = _i
    lib.sst_quantize.argtypes = [_p, _i, _i, _i, _i, _i, _p, _p, _p, _p, _sz, _p]
    lib.sst_quantize.restype = _i
    lib.sst_median_subtract.argtypes = [_p, _i, _i, _i, _p, _p, _p]
    lib.sst_median_subtract.restype = _i
    lib.sst_coadd.argtypes = [_p, _i, _i, _i, _i, _p, _p, _p, _p]
    lib.sst_coadd.restype = _i
    lib.sst_bin2x2.argtypes = [_p, _i, _i, _i, _p, _p]
    lib.sst_bin2x2.restype = _i
    lib.sst_frame_stats.argtypes = [_p, _i, _p, _i, _i, _i, _p, _p, _sz, _p]
    lib.sst_frame_stats.restype = _i
    lib.sst_stack.argtypes = [_p, _i, _p, _i, _i, _i, _p, _d, _p, _i, _p, _i, _p, _i, _p, _p, _p, _sz, _p]
    lib.sst_stack.restype = _i
    lib.sst_detect.argtypes = [_p, _i, _p, _i, _i, _i, _p, _d, _p, _i, _p, _i, _f, _i, _i, _p, _p, _p, _p, _sz,
                               _p]
    lib.sst_detect.restype = _i
    lib.sst_detect_noalloc.argtypes = [_p, _i, _p, _i, _i, _i, _p, _d, _p, _i, _p, _i, _f, _i, _i, _p, _p, _p, _p]
    lib.sst_detect_noalloc.restype = _i
    lib.sst_noalloc_scratch_bytes.argtypes = []
    lib.sst_noalloc_scratch_bytes.restype = _sz
    lib.sst_refine.argtypes = [_p, _i, _p, _i, _i, _i, _p, _d, _i, _p, _i, _f, _i, _f, _p, _p, _p, _sz, _p]
    lib.sst_refine.restype = _i
    lib.sst_plan_detect.argtypes = [_i, _i, _i, _p, _d, _p, _i, _p, _i, _f, _i, _i, _p, _sz, _p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.sst_plan_detect.restype = _i
    lib.sst_plan_run.argtypes = [_p, _p, _i, _p, _p, _p, _p]
    lib.sst_plan_run.restype = _i
    lib.sst_plan_destroy.argtypes = [_p]
    lib.sst_plan_destroy.restype = None
    lib.sst_batch_workspace_bytes.argtypes = [_p, _i]
    lib.sst_batch_workspace_bytes.restype = _sz
    lib.sst_batch_create.argtypes = [_p, _i, _p, _sz, _p, _p]
    lib.sst_batch_create.restype = _i
    lib.sst_batch_run.argtypes = [_p, _p, _p, _p, _p, _p, _p]
    lib.sst_batch_run.restype = _i
    lib.sst_batch_destroy.argtypes = [_p]
    lib.sst_batch_destroy.restype = None
    lib.sst_profile_begin.argtypes = []
    lib.sst_profile_begin.restype = _i
    lib.sst_set_slot_keep.argtypes = [_i]
    lib.sst_set_slot_keep.restype = _i
    lib.sst_set_half_search.argtypes = [_i]
    lib.sst_set_half_search.restype = _i
    lib.sst_set_stack_shape.argtypes = [_i, _p]
    lib.sst_set_stack_shape.restype = _i
    lib.sst_set_two_pass.argtypes = [_i, _p]
    lib.sst_set_two_pass.restype = _i
    lib.sst_profile_end.argtypes = [_p, _p]
    lib.sst_profile_end.restype = _i
    lib.sst_last_error.argtypes = []
    lib.sst_last_error.restype = ctypes.c_char_p
    lib.sst_version.argtypes = []
    lib.sst_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def sst_last_error() -> str:
    return load().sst_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise SstError(rc, sst_last_error())
    return rc


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dev(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def _frames_dtype(frames) -> int:
    import torch
    if frames.dtype == torch.float32:
        return SST_F32
    if frames.dtype == torch.bfloat16:
        return SST_BF16
    if frames.dtype == torch.float16:
        return SST_F16
    raise TypeError(f"frames dtype {frames.dtype} is not float32/bfloat16/float16")


def _check_frames(frames):
    if frames.dim() != 3 or not frames.is_contiguous() or not frames.is_cuda:
        raise ValueError("frames must be a contiguous [n][h][w] tensor on a HIP device")


# ------------------------------------------------------------- entry points
def sst_shift_table(t, t_ref: float, v) -> np.ndarray:
    """int32 [n][nv] table llround(v[a] * (t[i] - t_ref)), computed by the library."""
    t, v = _f64(t), _f64(v)
    out = np.empty((len(t), len(v)), dtype=np.int32)
    _check(load().sst_shift_table(_ptr(t), len(t), float(t_ref), _ptr(v), len(v), _ptr(out)))
    return out


def sst_workspace_bytes(op: int, n: int, h: int, w: int, t=None, t_ref: float = 0.0, vx=None, vy=None,
                        k_max: int = 0, shape: int = -1) -> int:
    """Workspace bytes of an operation (shape -1: the library's default
    velocity-block shape choice)."""
    t = None if t is None else _f64(t)
    vx = None if vx is None else _f64(vx)
    vy = None if vy is None else _f64(vy)
    nb = load().sst_workspace_bytes_shape(op, shape, n, h, w, _ptr(t), float(t_ref), _ptr(vx),
                                          0 if vx is None else len(vx), _ptr(vy), 0 if vy is None else len(vy), k_max)
    if nb == 0:
        raise SstError(SST_E_ARG, sst_last_error())
    return int(nb)


def sst_shapes():
    """The compiled velocity-block shapes: list of (vbx, vby), index = shape."""
    out = []
    k = 0
    while True:
        vbx, vby = ctypes.c_int(0), ctypes.c_int(0)
        nsh = load().sst_shape_info(k, ctypes.byref(vbx), ctypes.byref(vby))
        _check(nsh)
        out.append((vbx.value, vby.value))
        k += 1
        if k >= nsh:
            return out


def _workspace(nbytes: int, device, ws=None):
    import torch
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError(f"workspace too small: {ws.numel() * ws.element_size()} < {nbytes}")
        return ws
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def sst_quantize(frames, dtype, center: bool = False, ws=None):
    """16-bit copy of float32 frames with per-frame scales (see sst.h).

    dtype is torch.bfloat16 or torch.float16.  Returns (q, scale, offset): q
    has that dtype and the frames' shape, scale and offset are float32 [n];
    frame value = scale[i] * q[i] (+ offset[i] for absolute levels; offset is
    zero unless center)."""
    import torch
    _check_frames(frames)
    if frames.dtype != torch.float32:
        raise TypeError("sst_quantize takes float32 frames")
    code = {torch.bfloat16: SST_BF16, torch.float16: SST_F16}.get(dtype)
    if code is None:
        raise TypeError(f"dtype {dtype} is not bfloat16/float16")
    n, h, w = frames.shape
    nb = sst_workspace_bytes(SST_OP_QUANT, n, h, w)
    ws = _workspace(nb, frames.device, ws)
    q = torch.empty((n, h, w), dtype=dtype, device=frames.device)
    scale = torch.empty((n,), dtype=torch.float32, device=frames.device)
    offset = torch.zeros((n,), dtype=torch.float32, device=frames.device)
    _check(load().sst_quantize(_dev(frames), n, h, w, code, int(bool(center)), _dev(q), _dev(scale), _dev(offset),
                               _dev(ws), ws.numel(), _stream(frames.device)))
    return q, scale, offset


def _f32_frames(frames):
    import torch
    _check_frames(frames)
    if frames.dtype != torch.float32:
        raise TypeError("float32 frames expected")
    return frames.shape


def sst_median_subtract(frames, out=None, with_median: bool = False):
    """F_i - (per-pixel median over the frames); float32 [n][h][w] (and the
    median [h][w] if asked)."""
    import torch
    n, h, w = _f32_frames(frames)
    if out is None:
        out = torch.empty_like(frames)
    med = torch.empty((h, w), dtype=torch.float32, device=frames.device) if with_median else None
    _check(load().sst_median_subtract(_dev(frames), n, h, w, _dev(out), _dev(med), _stream(frames.device)))
    return (out, med) if with_median else out


def sst_coadd(frames, group: int, t=None):
    """Sums of each complete group of `group` consecutive frames:
    float32 [n // group][h][w] (and the groups' mean timestamps if t given)."""
    import torch
    n, h, w = _f32_frames(frames)
    ng = n // group if group >= 1 else 0
    out = torch.empty((max(ng, 1), h, w), dtype=torch.float32, device=frames.device)
    tv = None if t is None else _f64(t)
    if tv is not None and len(tv) != n:
        raise ValueError("t must have one value per frame")
    t_out = None if tv is None else np.empty(max(ng, 1), dtype=np.float64)
    _check(load().sst_coadd(_dev(frames), n, h, w, int(group), _dev(out), _ptr(tv), _ptr(t_out),
                            _stream(frames.device)))
    out = out[:ng]
    return (out, t_out[:ng]) if tv is not None else out


def sst_bin2x2(frames):
    """2x2 block sums: float32 [n][h // 2][w // 2]."""
    import torch
    n, h, w = _f32_frames(frames)
    out = torch.empty((n, max(h // 2, 1), max(w // 2, 1)), dtype=torch.float32, device=frames.device)
    _check(load().sst_bin2x2(_dev(frames), n, h, w, _dev(out), _stream(frames.device)))
    return out


def _check_scale(frames, scale):
    import torch
    if frames.dtype == torch.float32:
        return None if scale is None else _dev(scale)
    if scale is None or scale.dtype != torch.float32 or not scale.is_cuda or scale.numel() != frames.shape[0]:
        raise ValueError("16-bit frames need a float32 device tensor of per-frame scales")
    return _dev(scale.contiguous())


def sst_frame_stats(frames, scale=None, ws=None):
    """Per-frame (mean, population variance), float64 [n][2] on the device."""
    import torch
    _check_frames(frames)
    n, h, w = frames.shape
    nb = sst_workspace_bytes(SST_OP_STATS, n, h, w)
    ws = _workspace(nb, frames.device, ws)
    stats = torch.empty((n, 2), dtype=torch.float64, device=frames.device)
    _check(load().sst_frame_stats(_dev(frames), _frames_dtype(frames), _check_scale(frames, scale), n, h, w,
                                  _dev(stats),
                                  _dev(ws), ws.numel(), _stream(frames.device)))
    return stats


def sst_stack(frames, t, t_ref: float, vx, vy, bg=None, mode: int = SST_SUM, with_coverage: bool = False,
              out=None, cov=None, scale=None, ws=None):
    """Plain stacks float32 [nvy][nvx][h][w] (and coverage int32 if asked)."""
    import torch
    _check_frames(frames)
    n, h, w = frames.shape
    t, vx, vy = _f64(t), _f64(vx), _f64(vy)
    bgv = None if bg is None else _f64(bg)
    if bgv is not None and len(bgv) != n:
        raise ValueError("bg must have one value per frame")
    nb = sst_workspace_bytes(SST_OP_STACK, n, h, w, t, t_ref, vx, vy)
    ws = _workspace(nb, frames.device, ws)
    if out is None:
        out = torch.empty((len(vy), len(vx), h, w), dtype=torch.float32, device=frames.device)
    if with_coverage and cov is None:
        cov = torch.empty((len(vy), len(vx), h, w), dtype=torch.int32, device=frames.device)
    _check(load().sst_stack(_dev(frames), _frames_dtype(frames), _check_scale(frames, scale), n, h, w, _ptr(t),
                            float(t_ref),
                            _ptr(vx), len(vx), _ptr(vy), len(vy), _ptr(bgv), mode, _dev(out), _dev(cov), _dev(ws),
                            ws.numel(), _stream(frames.device)))
    return (out, cov) if with_coverage else out


def sst_detect(frames, t, t_ref: float, vx, vy, threshold: float, min_coverage: int = 0, k_max: int = 64,
               want_stats: bool = False, scale=None, ws=None, cand=None, count=None):
    """Per-velocity candidate lists.

    Returns (cand, count[, stats]): cand is an int32 device tensor
    [nvy*nvx][k_max][8] holding sst_candidate records (see `candidates_to_numpy`),
    count an int32 device tensor [nvy*nvx]; stats (host float64 [n][2]) if asked.
    """
    import torch
    _check_frames(frames)
    n, h, w = frames.shape
    t, vx, vy = _f64(t), _f64(vx), _f64(vy)
    nk = len(vx) * len(vy)
    nb = sst_workspace_bytes(SST_OP_DETECT, n, h, w, t, t_ref, vx, vy, k_max)
    ws = _workspace(nb, frames.device, ws)
    if cand is None:
        cand = torch.empty((nk, k_max, 8), dtype=torch.int32, device=frames.device)
    if count is None:
        count = torch.empty((nk,), dtype=torch.int32, device=frames.device)
    stats = np.empty((n, 2), dtype=np.float64) if want_stats else None
    _check(load().sst_detect(_dev(frames), _frames_dtype(frames), _check_scale(frames, scale), n, h, w, _ptr(t),
                             float(t_ref),
                             _ptr(vx), len(vx), _ptr(vy), len(vy), float(threshold), int(min_coverage), int(k_max),
                             _dev(cand), _dev(count), _ptr(stats), _dev(ws), ws.numel(), _stream(frames.device)))
    return (cand, count, stats) if want_stats else (cand, count)


def sst_detect_noalloc(frames, t, t_ref: float, vx, vy, threshold: float, min_coverage: int, k_max: int, cand,
                       count, scale=None):
    """sst_detect on the library's static device scratch: allocates nothing.
    cand (int32 [nvy*nvx][k_max][8]) and count (int32 [nvy*nvx]) are the
    caller's device tensors.  Problems needing more workspace than
    `sst_noalloc_scratch_bytes()` are rejected (SstError)."""
    _check_frames(frames)
    n, h, w = frames.shape
    t, vx, vy = _f64(t), _f64(vx), _f64(vy)
    nk = len(vx) * len(vy)
    if tuple(cand.shape) != (nk, k_max, 8) or tuple(count.shape) != (nk,):
        raise ValueError("cand must be [nvy*nvx][k_max][8] and count [nvy*nvx]")
    _check(load().sst_detect_noalloc(_dev(frames), _frames_dtype(frames), _check_scale(frames, scale), n, h, w,
                                     _ptr(t), float(t_ref), _ptr(vx), len(vx), _ptr(vy), len(vy), float(threshold),
                                     int(min_coverage), int(k_max), _dev(cand), _dev(count), None,
                                     _stream(frames.device)))
    return cand, count


def sst_noalloc_scratch_bytes() -> int:
    return int(load().sst_noalloc_scratch_bytes())


def sst_refine(frames, t, t_ref: float, params, cutout: int = 33, fwhm: float = 2.5, steps: int = 20,
               lr: float = 0.05, scale=None, ws=None):
    """Gradient ascent of the bilinear PSF-weighted stacked S/N (see sst.h).

    params: float32 device tensor [n_cand][4] of (x0, y0, vx, vy); it is not
    modified.  Returns (theta, snr, grad): the final parameters, SN and
    dSN/dtheta there (steps = 0 evaluates at params)."""
    import torch
    _check_frames(frames)
    n, h, w = frames.shape
    t = _f64(t)
    if len(t) != n:
        raise ValueError("t must have one value per frame")
    if params.dim() != 2 or params.shape[1] != 4 or params.dtype != torch.float32 or not params.is_cuda:
        raise ValueError("params must be a float32 device tensor [n_cand][4]")
    nc = params.shape[0]
    theta = params.detach().clone().contiguous()
    snr = torch.empty((nc,), dtype=torch.float32, device=frames.device)
    grad = torch.empty((nc, 4), dtype=torch.float32, device=frames.device)
    nb = sst_workspace_bytes(SST_OP_REFINE, n, h, w)
    ws = _workspace(nb, frames.device, ws)
    _check(load().sst_refine(_dev(frames), _frames_dtype(frames), _check_scale(frames, scale), n, h, w, _ptr(t),
                             float(t_ref), nc, _dev(theta), int(cutout), float(fwhm), int(steps), float(lr),
                             _dev(snr), _dev(grad), _dev(ws), ws.numel(), _stream(frames.device)))
    return theta, snr, grad


class SstPlan:
    """A prepared detect problem (sst_plan_detect).  It owns its workspace
    tensor; `run` enqueues kernels only and may be captured in a graph."""

    def __init__(self, handle, ws, n, h, w, nk, k_max):
        self._h = handle
        self.ws = ws
        self.n, self.h, self.w, self.nk, self.k_max = n, h, w, nk, k_max
        shape, staged, launches = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(load().sst_plan_info(handle, ctypes.byref(shape), ctypes.byref(staged), ctypes.byref(launches)))
        self.shape, self.staged, self.launches = shape.value, bool(staged.value), launches.value

    def run(self, frames, scale=None, cand=None, count=None):
        import torch
        _check_frames(frames)
        if tuple(frames.shape) != (self.n, self.h, self.w):
            raise ValueError(f"frames {tuple(frames.shape)} do not match the plan {(self.n, self.h, self.w)}")
        if self._h is None:
            raise RuntimeError("plan was destroyed")
        if cand is None:
            cand = torch.empty((self.nk, self.k_max, 8), dtype=torch.int32, device=frames.device)
        if count is None:
            count = torch.empty((self.nk,), dtype=torch.int32, device=frames.device)
        _check(load().sst_plan_run(self._h, _dev(frames), _frames_dtype(frames), _check_scale(frames, scale),
                                   _dev(cand), _dev(count), _stream(frames.device)))
        return cand, count

    def close(self):
        if self._h is not None:
            load().sst_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sst_plan_detect(n: int, h: int, w: int, t, t_ref: float, vx, vy, threshold: float, min_coverage: int = 0,
                    k_max: int = 64, device="cuda:0", shape: int = -1) -> SstPlan:
    """Prepare sst_detect for one geometry (uploads the shift tables once),
    with velocity-block shape `shape` (see sst_shapes; -1: the library's
    default choice)."""
    import torch
    t, vx, vy = _f64(t), _f64(vx), _f64(vy)
    nb = sst_workspace_bytes(SST_OP_DETECT, n, h, w, t, t_ref, vx, vy, k_max, shape=shape)
    ws = torch.empty(nb, dtype=torch.uint8, device=device)
    handle = ctypes.c_void_p()
    _check(load().sst_plan_detect_shape(int(shape), n, h, w, _ptr(t), float(t_ref), _ptr(vx), len(vx), _ptr(vy),
                                        len(vy), float(threshold), int(min_coverage), int(k_max), _dev(ws),
                                        ws.numel(), _stream(torch.device(device)), ctypes.byref(handle)))
    return SstPlan(handle, ws, n, h, w, len(vx) * len(vy), k_max)


class SstBatch:
    """Prepared plans searched together (sst_batch_create): `run` enqueues the
    plans' preparation kernels, one persistent stacking launch per round and
    the merges; kernels only, so it may be captured in a graph.  The plans
    must stay open while the batch is used."""

    def __init__(self, plans, device="cuda:0"):
        import torch
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("a batch needs at least one plan")
        if any(p._h is None for p in self.plans):
            raise RuntimeError("plan was destroyed")
        handles = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        self._handles = handles
        nb = load().sst_batch_workspace_bytes(handles, len(self.plans))
        if nb == 0:
            _check(-1)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(load().sst_batch_create(handles, len(self.plans), _dev(self.ws), self.ws.numel(),
                                       _stream(torch.device(device)), ctypes.byref(h)))
        self._h = h

    def run(self, frames, scales=None, cands=None, counts=None):
        """frames: list of [n][h][w] tensors, one per plan (scales likewise
        for 16-bit frames).  Returns (cands, counts), lists as SstPlan.run."""
        import torch
        k = len(self.plans)
        if len(frames) != k:
            raise ValueError(f"{len(frames)} frame tensors for {k} plans")
        if self._h is None:
            raise RuntimeError("batch was destroyed")
        if cands is None:
            cands = [torch.empty((p.nk, p.k_max, 8), dtype=torch.int32, device=f.device)
                     for p, f in zip(self.plans, frames)]
        if counts is None:
            counts = [torch.empty((p.nk,), dtype=torch.int32, device=f.device) for p, f in zip(self.plans, frames)]
        fr, dt, sc = [], [], []
        for j, (p, f) in enumerate(zip(self.plans, frames)):
            _check_frames(f)
            if tuple(f.shape) != (p.n, p.h, p.w):
                raise ValueError(f"frames {j} {tuple(f.shape)} do not match plan {(p.n, p.h, p.w)}")
            fr.append(_dev(f))
            dt.append(_frames_dtype(f))
            sc.append(_check_scale(f, None if scales is None else scales[j]))
        arr = lambda vals: (ctypes.c_void_p * k)(*vals)
        _check(load().sst_batch_run(self._h, arr(fr), (ctypes.c_int * k)(*dt), arr(sc),
                                    arr([_dev(c) for c in cands]), arr([_dev(c) for c in counts]),
                                    _stream(frames[0].device)))
        return cands, counts

    def close(self):
        if self._h is not None:
            load().sst_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sst_set_half_search(on: bool) -> bool:
    """Search IEEE-half frames on their 16-bit samples (True) or on a
    float32 copy (False, the default); returns the previous setting."""
    return bool(load().sst_set_half_search(1 if on else 0))


def sst_set_stack_shape(shape: int) -> int:
    """Work-item shape of sst_stack (-1: automatic); returns the previous
    setting.  Every shape writes the same stacks."""
    prev = ctypes.c_int(0)
    _check(load().sst_set_stack_shape(int(shape), ctypes.byref(prev)))
    return prev.value


SST_TWO_PASS_NEVER, SST_TWO_PASS_AUTO, SST_TWO_PASS_ALWAYS = 0, 1, 2


def sst_set_two_pass(mode: int) -> int:
    """Two-pass search of shape 2: SST_TWO_PASS_NEVER, _AUTO (the default:
    launches of at least 4096 work items) or _ALWAYS; returns the previous
    setting.  Every mode gives the same lists."""
    prev = ctypes.c_int(0)
    _check(load().sst_set_two_pass(int(mode), ctypes.byref(prev)))
    return prev.value


def sst_set_slot_keep(kt: int) -> int:
    """Cap the candidates each slot keeps (0: automatic) for plans made from
    now on; returns the previous cap.  Lists are the same either way."""
    return int(load().sst_set_slot_keep(int(kt)))


def sst_profile_begin() -> None:
    _check(load().sst_profile_begin())


def sst_profile_end() -> Tuple[float, int]:
    """(summed stacking-kernel milliseconds, launches) since sst_profile_begin."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int(0)
    _check(load().sst_profile_end(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def candidates_to_numpy(cand) -> np.ndarray:
    """Copy a candidate tensor to the host as a structured [nk][k_max] array."""
    a = cand.detach().cpu().numpy()
    return np.ascontiguousarray(a).view(CANDIDATE_DTYPE).reshape(a.shape[0], a.shape[1])
