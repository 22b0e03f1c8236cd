"""Python binding of libddm (argument marshalling only).

Every step of the matching runs in the HIP kernels of ``libddm.so``; this
module checks tensor shapes, allocates the workspace and output tensors with
PyTorch (device memory and streams are all PyTorch provides) and calls the C
interface declared in ``include/ddm.h``.  There is no fallback: if the library
is missing or a tensor is not on a GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libddm.so")

DDM_OK = 0
DDM_E_INVAL = -1
DDM_E_CAPACITY = -2
DDM_E_WORKSPACE = -3
DDM_E_DEVICE = -4
DDM_E_UNSUPPORTED = -5

MODES = {"count": 0, "per_update": 1, "pairs": 2}
PATHS = {"auto": 0, "bucketed": 1, "global": 2}
MAX_DIMS = 16


class DDMError(RuntimeError):
    def __init__(self, code: int, where: str = "ddm_match"):
        self.code = code
        super().__init__(f"{where} failed: {code} ({strerror(code)})")


_lib = None


def library() -> ctypes.CDLL:
    """Load libddm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(
                f"{LIBRARY} is missing: build it with `python -m paper_1703_06680_amd.build` "
                "(no CPU fallback exists)")
        lib = ctypes.CDLL(LIBRARY)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.ddm_workspace_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int, i64]
        lib.ddm_workspace_bytes.restype = ctypes.c_size_t
        lib.ddm_match.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                                  ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_uint64), vp, vp, i64]
        lib.ddm_match.restype = ctypes.c_int
        lib.ddm_strerror.argtypes = [ctypes.c_int]
        lib.ddm_strerror.restype = ctypes.c_char_p
        lib.ddm_set_path.argtypes = [ctypes.c_int]
        lib.ddm_set_path.restype = ctypes.c_int
        lib.ddm_last_path.argtypes = []
        lib.ddm_last_path.restype = ctypes.c_int
        lib.ddm_profile.argtypes = [ctypes.c_int]
        lib.ddm_profile.restype = ctypes.c_int
        lib.ddm_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.ddm_profile_report.restype = ctypes.c_int
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    try:
        return library().ddm_strerror(code).decode()
    except Exception:  # library missing: still produce a message
        return "unknown"


def set_path(name: str) -> None:
    """Select the implementation for later calls (process-global): "auto"
    (bucketed where available, global otherwise or on overflow), "bucketed"
    (error instead of falling back) or "global"."""
    rc = library().ddm_set_path(PATHS[name])
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_set_path")


def last_path():
    """Implementation that produced the last successful result."""
    return {0: None, 1: "bucketed", 2: "global"}[library().ddm_last_path()]


def profile(enable: bool) -> None:
    """Start (clearing the totals) or stop per-phase GPU timing."""
    library().ddm_profile(1 if enable else 0)


def profile_report() -> dict:
    """Per-phase totals recorded since profile(True): {phase: {"ms", "launches"}}."""
    import json
    lib = library()
    need = lib.ddm_profile_report(None, 0)
    buf = ctypes.create_string_buffer(max(need, 2) + 64)
    rc = lib.ddm_profile_report(buf, len(buf))
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_profile_report")
    return json.loads(buf.value.decode())


def match_into(upd_lo, upd_hi, sub_lo, sub_hi, mode: str, workspace: torch.Tensor,
               per_update: torch.Tensor | None = None, pairs: torch.Tensor | None = None,
               stream=None) -> int:
    """Low-level call with caller-provided workspace and outputs (no
    allocation); returns the number of pairs, raises DDMError on failure."""
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    cnt = ctypes.c_uint64(0)
    cap = pairs.shape[0] if pairs is not None else 0
    rc = library().ddm_match(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                             MODES[mode], ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                             ctypes.c_void_p(stream.cuda_stream), ctypes.byref(cnt),
                             _ptr(per_update) if per_update is not None else None,
                             _ptr(pairs) if pairs is not None else None, cap)
    if rc != DDM_OK:
        raise DDMError(rc)
    return int(cnt.value)


def workspace_bytes(n: int, m: int, d: int, mode: str = "count", pair_capacity: int = 0) -> int:
    return int(library().ddm_workspace_bytes(n, m, d, MODES[mode], pair_capacity))


def _check_boxes(lo: torch.Tensor, hi: torch.Tensor, name: str):
    if not (isinstance(lo, torch.Tensor) and isinstance(hi, torch.Tensor)):
        raise TypeError(f"{name}: expected torch tensors")
    if lo.device.type != "cuda" or hi.device.type != "cuda":
        raise ValueError(f"{name}: tensors must live on a GPU (no CPU path exists)")
    if lo.dtype != torch.float32 or hi.dtype != torch.float32:
        raise TypeError(f"{name}: expected float32")
    if lo.dim() != 2 or lo.shape != hi.shape:
        raise ValueError(f"{name}: expected lo/hi of the same shape [count, d]")
    if not (lo.is_contiguous() and hi.is_contiguous()):
        raise ValueError(f"{name}: tensors must be contiguous (row-major [count][d])")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def match(upd_lo, upd_hi, sub_lo, sub_hi, mode: str = "count", *, pair_capacity: int | None = None,
          per_update: bool = True, workspace: torch.Tensor | None = None, stream=None):
    """Sort-based matching of update boxes against subscription boxes.

    ``upd_lo``/``upd_hi`` are float32 [n, d], ``sub_lo``/``sub_hi`` float32
    [m, d], all on the same GPU.  Returns
      mode="count":      int K (number of intersecting pairs)
      mode="per_update": (K, int32 tensor [n] of matches per update)
      mode="pairs":      (K, int32 tensor [K, 2] of (update id, subscription
                         id) in lexicographic order, int32 [n] counts or None)
    """
    if mode not in MODES:
        raise ValueError(f"unknown mode {mode!r}")
    _check_boxes(upd_lo, upd_hi, "updates")
    _check_boxes(sub_lo, sub_hi, "subscriptions")
    n, d = upd_lo.shape
    m, d2 = sub_lo.shape
    if d != d2:
        raise ValueError("updates and subscriptions differ in dimension")
    if upd_lo.device != sub_lo.device:
        raise ValueError("all tensors must be on the same device")
    dev = upd_lo.device
    lib = library()
    code = MODES[mode]
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    handle = ctypes.c_void_p(stream.cuda_stream)
    cnt = ctypes.c_uint64(0)
    per = None
    if mode == "per_update" or (mode == "pairs" and per_update):
        per = torch.empty(max(n, 1), dtype=torch.int32, device=dev)

    def run(cap, out):
        need = lib.ddm_workspace_bytes(n, m, d, code, cap)
        if need == 0:
            raise DDMError(DDM_E_INVAL, "ddm_workspace_bytes")
        ws = workspace
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        return lib.ddm_match(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d, code,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), handle, ctypes.byref(cnt),
                             _ptr(per) if per is not None else None,
                             _ptr(out) if out is not None else None, cap)

    with torch.cuda.device(dev):
        if mode != "pairs":
            rc = run(0, None)
            if rc != DDM_OK:
                raise DDMError(rc)
            k = int(cnt.value)
            return k if mode == "count" else (k, per[:n])
        cap = int(pair_capacity) if pair_capacity is not None else max(1024, n + m)
        while True:
            out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
            rc = run(cap, out)
            if rc == DDM_E_CAPACITY and pair_capacity is None:
                cap = int(cnt.value)
                continue
            if rc != DDM_OK:
                raise DDMError(rc)
            k = int(cnt.value)
            return k, out[:k], (per[:n] if per is not None else None)
