"""Thin Python binding of libbm.so: the C-ABI calls under the same names.

Argument marshalling only.  Every step of block matching runs in the library's HIP
kernels; PyTorch tensors only provide device memory (``data_ptr()``) and the stream
handle.  If the shared library is missing or fails to load, every call raises -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbm.so")

BM_OK = 0
BM_EINVAL = -1
BM_ENOMEM = -2
BM_EDEVICE = -3
BM_EAGAIN = -4
BM_EBUSY = -5
BM_ENOTFOUND = -6
BM_ECANCELED = -7
BM_ENOTSUP = -8

BM_PREC_FP32 = 0
BM_PREC_BF16X4 = 1
BM_PREC_FP16X3 = 2
PRECISIONS = {"fp32": BM_PREC_FP32, "bf16x4": BM_PREC_BF16X4, "fp16x3": BM_PREC_FP16X3}

BM_FLAG_CENTER = 1
BM_FLAG_NCC = 2


class bm_desc(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("channels", C.c_int32),
                ("patch", C.c_int32), ("stride", C.c_int32), ("window", C.c_int32),
                ("k", C.c_int32), ("precision", C.c_int32), ("flags", C.c_uint32),
                ("patch_depth", C.c_int32), ("window_depth", C.c_int32)]


class bm_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32),
                ("max_queue", C.c_int32), ("max_step", C.c_int32)]


class bm_request_stats(C.Structure):
    _fields_ = [("queue_s", C.c_double), ("device_s", C.c_double), ("total_s", C.c_double),
                ("n_ref", C.c_int64)]


class BMError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_status_name(status)} ({status}): {msg}")
        self.status = status


_lib = None
_lock = threading.Lock()

_SIGS = {
    "bm_plan": (C.c_int32, [C.POINTER(bm_desc), C.POINTER(C.c_void_p)]),
    "bm_plan_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "bm_match": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bm_match_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bm_norms": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bm_cross_topk": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "bm_match_batch": (C.c_int32, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p,
                                   C.c_void_p]),
    "bm_batch_workspace": (C.c_int32, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64)]),
    "bm_plan_destroy": (C.c_int32, [C.c_void_p]),
    "bm_gather": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "bm_aggregate_workspace": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "bm_aggregate": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "bm_nlm": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_void_p]),
    "bm_server_create": (C.c_int32, [C.POINTER(bm_server_cfg), C.POINTER(C.c_void_p)]),
    "bm_submit": (C.c_int32, [C.c_void_p, C.POINTER(bm_desc), C.c_void_p, C.POINTER(C.c_uint64)]),
    "bm_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                            C.POINTER(bm_request_stats)]),
    "bm_cancel": (C.c_int32, [C.c_void_p, C.c_uint64]),
    "bm_server_destroy": (C.c_int32, [C.c_void_p]),
    "bm_autotune": (C.c_int32, [C.POINTER(bm_desc), C.c_void_p, C.c_int32, C.c_char_p, C.c_int32]),
    "bm_plan_config": (C.c_int32, [C.c_void_p, C.c_char_p, C.c_int32, C.POINTER(C.c_int32)]),
    "bm_peak_mfma": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    "bm_peak_copy": (C.c_int32, [C.c_int64, C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    "bm_status_str": (C.c_char_p, [C.c_int32]),
    "bm_last_error": (C.c_char_p, []),
}


def lib():
    """Load libbm.so once; raise if it is absent (no fallback path exists)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2006_13714_amd.build_lib` (no CPU fallback exists)")
            h = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(h, name)
                f.restype = res
                f.argtypes = args
            _lib = h
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().bm_status_str(s).decode()
    except Exception:
        return str(s)


def _check(status: int, where: str):
    if status != BM_OK:
        raise BMError(status, where, bm_last_error())


def bm_last_error() -> str:
    return lib().bm_last_error().decode()


def bm_status_str(s: int) -> str:
    return lib().bm_status_str(s).decode()


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def make_desc(height, width, channels, patch, stride, window, k, precision="fp32", flags=0,
              patch_depth=0, window_depth=0):
    """A bm_desc; patch_depth / window_depth > 0 make it a 3D search over `channels` planes."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return bm_desc(height, width, channels, patch, stride, window, k, prec, flags, patch_depth,
                   window_depth)


class Plan:
    """Owns a bm_plan_t; destroyed with the object or by ``close()``."""

    def __init__(self, handle: int, desc: bm_desc):
        self.handle = handle
        self.desc = desc
        n_ref, ws = C.c_int64(), C.c_int64()
        _check(lib().bm_plan_info(handle, C.byref(n_ref), C.byref(ws)), "bm_plan_info")
        self.n_ref = n_ref.value
        self.workspace_bytes = ws.value

    def close(self):
        if self.handle:
            lib().bm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bm_plan(desc: bm_desc) -> Plan:
    h = C.c_void_p()
    _check(lib().bm_plan(C.byref(desc), C.byref(h)), "bm_plan")
    return Plan(h.value, desc)


def bm_plan_info(plan: Plan):
    return plan.n_ref, plan.workspace_bytes


def bm_match(plan: Plan, img, idx, dist, workspace=None, stream=None):
    _check(lib().bm_match(plan.handle, _ptr(img), _ptr(idx), _ptr(dist), _ptr(workspace),
                          _stream(stream)), "bm_match")


def bm_match_noalloc(plan: Plan, img, idx, dist, stream=None):
    _check(lib().bm_match_noalloc(plan.handle, _ptr(img), _ptr(idx), _ptr(dist),
                                  _stream(stream)), "bm_match_noalloc")


def bm_norms(plan: Plan, img, norm, stream=None):
    _check(lib().bm_norms(plan.handle, _ptr(img), _ptr(norm), _stream(stream)), "bm_norms")


def bm_cross_topk(plan: Plan, img, norm, idx, dist, stream=None):
    _check(lib().bm_cross_topk(plan.handle, _ptr(img), _ptr(norm), _ptr(idx), _ptr(dist),
                               _stream(stream)), "bm_cross_topk")


def bm_batch_workspace(plans) -> int:
    arr = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    out = C.c_int64()
    _check(lib().bm_batch_workspace(len(plans), arr, C.byref(out)), "bm_batch_workspace")
    return out.value


def bm_match_batch(plans, imgs, idxs, dists, workspace=None, stream=None):
    n = len(plans)
    P = (C.c_void_p * n)(*[p.handle for p in plans])
    I = (C.c_void_p * n)(*[_ptr(t) for t in imgs])
    X = (C.c_void_p * n)(*[_ptr(t) for t in idxs])
    D = (C.c_void_p * n)(*[_ptr(t) for t in dists])
    _check(lib().bm_match_batch(n, P, I, X, D, _ptr(workspace), _stream(stream)), "bm_match_batch")


def bm_gather(plan: Plan, img, idx, groups, stream=None):
    _check(lib().bm_gather(plan.handle, _ptr(img), _ptr(idx), _ptr(groups), _stream(stream)),
           "bm_gather")


def bm_aggregate_workspace(plan: Plan) -> int:
    out = C.c_int64()
    _check(lib().bm_aggregate_workspace(plan.handle, C.byref(out)), "bm_aggregate_workspace")
    return out.value


def bm_aggregate(plan: Plan, groups, idx, out, workspace=None, stream=None):
    _check(lib().bm_aggregate(plan.handle, _ptr(groups), _ptr(idx), _ptr(out), _ptr(workspace),
                              _stream(stream)), "bm_aggregate")


def bm_nlm(plan: Plan, img, b: float, patch, theta=None, workspace=None, stream=None):
    _check(lib().bm_nlm(plan.handle, _ptr(img), float(b), _ptr(patch), _ptr(theta),
                        _ptr(workspace), _stream(stream)), "bm_nlm")


def bm_plan_destroy(plan: Plan):
    plan.close()


def bm_autotune(desc: bm_desc, img=None, reps: int = 10) -> str:
    out = C.create_string_buffer(128)
    _check(lib().bm_autotune(C.byref(desc), _ptr(img), reps, out, 128), "bm_autotune")
    return out.value.decode()


def bm_plan_config(plan: Plan):
    out = C.create_string_buffer(128)
    src = C.c_int32()
    _check(lib().bm_plan_config(plan.handle, out, 128, C.byref(src)), "bm_plan_config")
    return out.value.decode(), src.value


def bm_peak_mfma(precision, shape: int = 0, iterations: int = 20000, stream=None) -> float:
    """Measured matrix-core rate (TFLOP/s) of a precision form's 16x16 (shape 0, the one the
    kernels issue) or 32x32 (shape 1) matrix instruction."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = C.c_double()
    _check(lib().bm_peak_mfma(prec, shape, iterations, _stream(stream), C.byref(out)),
           "bm_peak_mfma")
    return out.value


def bm_peak_copy(nbytes: int = 1 << 30, repeats: int = 5, stream=None) -> float:
    """Measured streaming device-copy rate (GB/s of bytes read plus written)."""
    out = C.c_double()
    _check(lib().bm_peak_copy(nbytes, repeats, _stream(stream), C.byref(out)), "bm_peak_copy")
    return out.value


def bm_server_create(hbm_budget_bytes: int, max_inflight: int = 64, max_queue: int = 4096,
                     max_step: int = 0) -> int:
    cfg = bm_server_cfg(hbm_budget_bytes, max_inflight, max_queue, max_step)
    h = C.c_void_p()
    _check(lib().bm_server_create(C.byref(cfg), C.byref(h)), "bm_server_create")
    return h.value


def bm_submit(server: int, desc: bm_desc, host_img) -> int:
    """Queue one request; ``host_img`` is a C-contiguous float32 numpy array (C, H, W)."""
    import numpy as np
    a = np.ascontiguousarray(host_img, dtype=np.float32)
    t = C.c_uint64()
    _check(lib().bm_submit(server, C.byref(desc), a.ctypes.data, C.byref(t)), "bm_submit")
    return t.value


def bm_poll(server: int, ticket: int, host_idx=None, host_dist=None):
    """Return (status, stats).  status is BM_OK (buffers filled) or BM_EAGAIN."""
    st = bm_request_stats()
    s = lib().bm_poll(server, ticket, None if host_idx is None else host_idx.ctypes.data,
                      None if host_dist is None else host_dist.ctypes.data, C.byref(st))
    if s in (BM_OK, BM_EAGAIN):
        return s, st
    raise BMError(s, "bm_poll", bm_last_error())


def bm_cancel(server: int, ticket: int):
    _check(lib().bm_cancel(server, ticket), "bm_cancel")


def bm_server_destroy(server: int):
    _check(lib().bm_server_destroy(server), "bm_server_destroy")


# ---- convenience ---------------------------------------------------------------------
_plan_cache: dict = {}


def _call_workspace(plan: Plan, device, stream):
    """A workspace of plan.workspace_bytes for one call, from torch's allocator on the
    call's stream, so calls of one cached plan on different streams never share the
    plan's own workspace (norm map and auxiliary slots)."""
    import torch
    if plan.workspace_bytes <= 0:
        return None
    if stream is None or isinstance(stream, int):
        return torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=device)
    with torch.cuda.stream(stream):
        return torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=device)


def cached_plan(desc: bm_desc) -> Plan:
    key = tuple(getattr(desc, f) for f, _ in bm_desc._fields_)
    p = _plan_cache.get(key)
    if p is None:
        p = _plan_cache[key] = bm_plan(desc)
    return p


def match3d(vol, patch: int, patch_depth: int, stride: int, window: int, window_depth: int,
            k: int, precision="fp32", plan: Plan | None = None, stream=None):
    """3D search over a (q, H, W) float32 CUDA tensor: d x P x P blocks, Wn x Wn x c windows.

    Returns (idx, dist) of shape ((q - d + 1) * n_ref2d, k), references depth-major; indices
    are volume positions (z * H + y) * W + x."""
    import torch
    if vol.dim() != 3 or not vol.is_cuda or vol.dtype != torch.float32:
        raise ValueError("vol must be a (q, H, W) float32 tensor on the GPU")
    vol = vol.contiguous()
    q, H, W = vol.shape
    if plan is None:
        plan = cached_plan(make_desc(H, W, q, patch, stride, window, k, precision, 0,
                                     patch_depth, window_depth))
    idx = torch.empty((plan.n_ref, k), dtype=torch.int32, device=vol.device)
    dist = torch.empty((plan.n_ref, k), dtype=torch.float32, device=vol.device)
    bm_match(plan, vol, idx, dist, _call_workspace(plan, vol.device, stream), stream)
    return idx, dist


def nlm(img, patch: int, stride: int, window: int, b: float, plan: Plan | None = None,
        stream=None):
    """Allocate outputs and run bm_nlm on a (C, H, W) float32 CUDA tensor: (theta, patch)."""
    import torch
    if img.dim() == 2:
        img = img.unsqueeze(0)
    if not img.is_cuda or img.dtype != torch.float32:
        raise ValueError("img must be a float32 tensor on the GPU")
    img = img.contiguous()
    Cn, H, W = img.shape
    if plan is None:
        plan = cached_plan(make_desc(H, W, Cn, patch, stride, window, 16, "fp32", 0))
    out = torch.empty((plan.n_ref, Cn, patch, patch), dtype=torch.float32, device=img.device)
    theta = torch.empty((plan.n_ref,), dtype=torch.float32, device=img.device)
    bm_nlm(plan, img, b, out, theta, _call_workspace(plan, img.device, stream), stream)
    return theta, out


def match(img, patch: int, stride: int, window: int, k: int, precision="fp32", flags=0,
          plan: Plan | None = None, stream=None):
    """Allocate outputs and run bm_match on a (C, H, W) float32 CUDA tensor."""
    import torch
    if img.dim() == 2:
        img = img.unsqueeze(0)
    if not img.is_cuda or img.dtype != torch.float32:
        raise ValueError("img must be a float32 tensor on the GPU")
    img = img.contiguous()
    Cn, H, W = img.shape
    if plan is None:
        plan = cached_plan(make_desc(H, W, Cn, patch, stride, window, k, precision, flags))
    idx = torch.empty((plan.n_ref, k), dtype=torch.int32, device=img.device)
    dist = torch.empty((plan.n_ref, k), dtype=torch.float32, device=img.device)
    bm_match(plan, img, idx, dist, _call_workspace(plan, img.device, stream), stream)
    return idx, dist
