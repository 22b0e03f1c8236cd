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
DDM_E_SCRATCH = -6
NOALLOC_SCRATCH_BYTES = 64 << 20  # DDM_NOALLOC_SCRATCH_BYTES

MODES = {"count": 0, "per_update": 1, "pairs": 2}
DDM_CLOSED = 16  # interval flag OR-ed into a mode: closed boxes [lo, hi]
PATHS = {"auto": 0, "bucketed": 1, "global": 2}
MAX_DIMS = 16


class Tuning(ctypes.Structure):
    """Launch shape of the batched path (``ddm_tuning``)."""
    _fields_ = [("target", ctypes.c_int32), ("sweep_threads", ctypes.c_int32),
                ("groups_per_thread", ctypes.c_int32), ("max_blocks", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


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
        lib.ddm_match_csr.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int, vp,
                                      ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_uint64), vp, vp,
                                      i64]
        lib.ddm_match_csr.restype = ctypes.c_int
        lib.ddm_match_noalloc.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, ctypes.c_int,
                                          vp, ctypes.POINTER(ctypes.c_uint64), vp, vp, i64]
        lib.ddm_match_noalloc.restype = ctypes.c_int
        lib.ddm_strerror.argtypes = [ctypes.c_int]
        lib.ddm_strerror.restype = ctypes.c_char_p
        lib.ddm_set_path.argtypes = [ctypes.c_int]
        lib.ddm_set_path.restype = ctypes.c_int
        lib.ddm_set_sweep_axis.argtypes = [ctypes.c_int]
        lib.ddm_set_sweep_axis.restype = ctypes.c_int
        lib.ddm_last_path.argtypes = []
        lib.ddm_last_path.restype = ctypes.c_int
        lib.ddm_profile.argtypes = [ctypes.c_int]
        lib.ddm_profile.restype = ctypes.c_int
        lib.ddm_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        lib.ddm_profile_report.restype = ctypes.c_int
        lib.ddm_copy_probe.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp,
                                       ctypes.POINTER(ctypes.c_double)]
        lib.ddm_copy_probe.restype = ctypes.c_int
        tp = ctypes.POINTER(Tuning)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.ddm_dim_counts_workspace_bytes.argtypes = [i64, i64, ctypes.c_int]
        lib.ddm_dim_counts_workspace_bytes.restype = ctypes.c_size_t
        lib.ddm_dim_counts.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, vp, ctypes.c_size_t,
                                       vp, vp]
        lib.ddm_dim_counts.restype = ctypes.c_int
        lib.ddm_default_tuning.argtypes = [tp]
        lib.ddm_default_tuning.restype = None
        lib.ddm_batch_workspace_bytes.argtypes = [vp, vp, i64, ctypes.c_int, ctypes.c_int, i64, tp]
        lib.ddm_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.ddm_match_batched.argtypes = [vp, vp, vp, vp, vp, vp, i64, ctypes.c_int, ctypes.c_int,
                                          vp, ctypes.c_size_t, vp, tp, vp, u64p, vp, vp, vp, i64]
        lib.ddm_match_batched.restype = ctypes.c_int
        lib.ddm_batch_graph_create.argtypes = [vp, vp, vp, vp, vp, vp, i64, ctypes.c_int,
                                               ctypes.c_int, vp, ctypes.c_size_t, tp, vp, vp, vp,
                                               vp, i64, ctypes.POINTER(vp)]
        lib.ddm_batch_graph_create.restype = ctypes.c_int
        lib.ddm_batch_graph_launch.argtypes = [vp, vp]
        lib.ddm_batch_graph_launch.restype = ctypes.c_int
        lib.ddm_batch_graph_result.argtypes = [vp, vp, u64p]
        lib.ddm_batch_graph_result.restype = ctypes.c_int
        lib.ddm_batch_graph_destroy.argtypes = [vp]
        lib.ddm_batch_graph_destroy.restype = ctypes.c_int
        lib.ddm_batch_autotune.argtypes = [vp, vp, vp, vp, vp, vp, i64, ctypes.c_int, ctypes.c_int,
                                           vp, ctypes.c_size_t, vp, vp, vp, vp, vp, i64, tp,
                                           ctypes.POINTER(ctypes.c_double)]
        lib.ddm_batch_autotune.restype = ctypes.c_int
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


def set_sweep_axis(axis: int | None) -> None:
    """Swept axis of later bucketed calls (process-global): None lets each
    instance's plan choose the axis with the fewest expected 1-D candidates
    (the default); an int forces that input axis."""
    rc = library().ddm_set_sweep_axis(-1 if axis is None else int(axis))
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_set_sweep_axis")


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


def copy_probe(nbytes: int = 256 << 20, reps: int = 10) -> dict:
    """Achievable HBM bandwidth of a plain copy kernel of the library
    (``ddm_copy_probe``): {"bytes_moved", "ms", "gb_per_s"} for one copy of
    ``nbytes`` (read + write = 2 * nbytes)."""
    nbytes = (int(nbytes) + 15) // 16 * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    ms = ctypes.c_double(0.0)
    stream = torch.cuda.current_stream()
    rc = library().ddm_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                  nbytes, int(reps), ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.byref(ms))
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_copy_probe")
    return {"bytes_moved": 2 * nbytes, "ms": ms.value,
            "gb_per_s": 2 * nbytes / (ms.value * 1e-3) / 1e9}


def _code(mode: str, closed: bool) -> int:
    if mode not in MODES:
        raise ValueError(f"unknown mode {mode!r}")
    return MODES[mode] | (DDM_CLOSED if closed else 0)


def match_into(upd_lo, upd_hi, sub_lo, sub_hi, mode: str, workspace: torch.Tensor,
               per_update: torch.Tensor | None = None, pairs: torch.Tensor | None = None,
               stream=None, closed: bool = False) -> int:
    """Low-level call with caller-provided workspace and outputs (no
    allocation); returns the number of pairs, raises DDMError on failure."""
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    cnt = ctypes.c_uint64(0)
    cap = pairs.shape[0] if pairs is not None else 0
    rc = library().ddm_match(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                             _code(mode, closed), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel(),
                             ctypes.c_void_p(stream.cuda_stream), ctypes.byref(cnt),
                             _ptr(per_update) if per_update is not None else None,
                             _ptr(pairs) if pairs is not None else None, cap)
    if rc != DDM_OK:
        raise DDMError(rc)
    return int(cnt.value)


def match_noalloc_into(upd_lo, upd_hi, sub_lo, sub_hi, mode: str,
                       per_update: torch.Tensor | None = None,
                       pairs: torch.Tensor | None = None, stream=None,
                       closed: bool = False) -> int:
    """``ddm_match_noalloc``: the call of ``match_into`` without a workspace
    (the library's static device array serves as one); returns K, raises
    DDMError (code DDM_E_SCRATCH when the sizes need more than the array)."""
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    cnt = ctypes.c_uint64(0)
    cap = pairs.shape[0] if pairs is not None else 0
    rc = library().ddm_match_noalloc(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi),
                                     m, d, _code(mode, closed),
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(cnt),
                                     _ptr(per_update) if per_update is not None else None,
                                     _ptr(pairs) if pairs is not None else None, cap)
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_match_noalloc")
    return int(cnt.value)


def match_csr_into(upd_lo, upd_hi, sub_lo, sub_hi, workspace: torch.Tensor,
                   row_off: torch.Tensor, sub_ids: torch.Tensor, stream=None,
                   closed: bool = False) -> int:
    """Low-level CSR call (``ddm_match_csr``) with caller-provided workspace
    (``workspace_bytes(n, m, d, "pairs", capacity)``), int64 ``row_off``
    [n + 1] and int32 ``sub_ids`` [capacity]; returns K, raises DDMError."""
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    cnt = ctypes.c_uint64(0)
    rc = library().ddm_match_csr(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                                 DDM_CLOSED if closed else 0, ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel(), ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(cnt), ctypes.c_void_p(row_off.data_ptr()),
                                 _ptr(sub_ids), sub_ids.numel())
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_match_csr")
    return int(cnt.value)


def workspace_bytes(n: int, m: int, d: int, mode: str = "count", pair_capacity: int = 0,
                    closed: bool = False) -> int:
    return int(library().ddm_workspace_bytes(n, m, d, _code(mode, closed), pair_capacity))


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
          per_update: bool = True, workspace: torch.Tensor | None = None, stream=None,
          closed: bool = False):
    """Sort-based matching of update boxes against subscription boxes.

    ``upd_lo``/``upd_hi`` are float32 [n, d], ``sub_lo``/``sub_hi`` float32
    [m, d], all on the same GPU; boxes are half-open [lo, hi), or closed
    [lo, hi] with ``closed=True``.  Returns
      mode="count":      int K (number of intersecting pairs)
      mode="per_update": (K, int32 tensor [n] of matches per update)
      mode="pairs":      (K, int32 tensor [K, 2] of (update id, subscription
                         id) in lexicographic order, int32 [n] counts or None)
      mode="csr":        (K, int64 tensor [n + 1] of row offsets, int32 tensor
                         [K] of subscription ids, ascending within each row)
    """
    if mode == "csr":
        return _match_csr(upd_lo, upd_hi, sub_lo, sub_hi, pair_capacity, workspace, stream,
                          closed)
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
    code = _code(mode, closed)
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


def _match_csr(upd_lo, upd_hi, sub_lo, sub_hi, capacity, workspace, stream, closed):
    _check_boxes(upd_lo, upd_hi, "updates")
    _check_boxes(sub_lo, sub_hi, "subscriptions")
    n, d = upd_lo.shape
    m, d2 = sub_lo.shape
    if d != d2:
        raise ValueError("updates and subscriptions differ in dimension")
    dev = upd_lo.device
    lib = library()
    flags = DDM_CLOSED if closed else 0
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    handle = ctypes.c_void_p(stream.cuda_stream)
    cnt = ctypes.c_uint64(0)
    row_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    cap = int(capacity) if capacity is not None else max(1024, n + m)
    with torch.cuda.device(dev):
        while True:
            need = lib.ddm_workspace_bytes(n, m, d, MODES["pairs"] | flags, cap)
            if need == 0:
                raise DDMError(DDM_E_INVAL, "ddm_workspace_bytes")
            ws = workspace
            if ws is None or ws.numel() < need:
                ws = torch.empty(need, dtype=torch.uint8, device=dev)
            ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            rc = lib.ddm_match_csr(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                                   flags, ctypes.c_void_p(ws.data_ptr()), ws.numel(), handle,
                                   ctypes.byref(cnt), ctypes.c_void_p(row_off.data_ptr()),
                                   _ptr(ids), cap)
            if rc == DDM_E_CAPACITY and capacity is None:
                cap = int(cnt.value)
                continue
            if rc != DDM_OK:
                raise DDMError(rc, "ddm_match_csr")
            k = int(cnt.value)
            return k, row_off, ids[:k]


def dim_counts(upd_lo, upd_hi, sub_lo, sub_hi, stream=None):
    """Per-axis 1-D candidate counts K_1D(k), k = 0 .. d-1 (``ddm_dim_counts``)."""
    import numpy as np
    _check_boxes(upd_lo, upd_hi, "updates")
    _check_boxes(sub_lo, sub_hi, "subscriptions")
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    lib = library()
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    ws = torch.empty(max(lib.ddm_dim_counts_workspace_bytes(n, m, d), 256), dtype=torch.uint8,
                     device=upd_lo.device)
    out = np.zeros(d, dtype=np.uint64)
    with torch.cuda.device(upd_lo.device):
        rc = lib.ddm_dim_counts(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(stream.cuda_stream),
                                ctypes.c_void_p(out.ctypes.data))
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_dim_counts")
    return [int(x) for x in out]


# --------------------------------------------------------------- batches

def default_tuning() -> Tuning:
    t = Tuning()
    library().ddm_default_tuning(ctypes.byref(t))
    return t


def _offsets(off, name: str):
    """Host int64 CSR offsets as a contiguous numpy array (kept alive by the caller)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    if a.ndim != 1 or a.size < 2:
        raise ValueError(f"{name}: expected a 1-D array of B + 1 offsets")
    return a


def _aptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Batch:
    """A batch of independent instances stored back to back.

    ``upd_lo``/``upd_hi`` float32 [sum n, d] and ``sub_lo``/``sub_hi``
    float32 [sum m, d] on one GPU; ``upd_off``/``sub_off`` host offsets
    [B + 1] (instance b owns rows upd_off[b]:upd_off[b+1] and
    sub_off[b]:sub_off[b+1]).  Holds the output tensors:
    ``counts`` uint64-as-int64 [B], ``per_update`` int32 [sum n] (modes
    per_update and pairs), ``pairs`` int32 [capacity, 2] and ``pair_off``
    int64 [B + 1] (mode pairs), and the workspace.  ``closed=True`` matches
    closed boxes [lo, hi] instead of half-open ones.
    """

    def __init__(self, upd_lo, upd_hi, upd_off, sub_lo, sub_hi, sub_off, mode: str = "count",
                 pair_capacity: int = 0, workspace: torch.Tensor | None = None,
                 closed: bool = False):
        if mode not in MODES:
            raise ValueError(f"unknown mode {mode!r}")
        _check_boxes(upd_lo, upd_hi, "updates")
        _check_boxes(sub_lo, sub_hi, "subscriptions")
        self.uoff = _offsets(upd_off, "upd_off")
        self.soff = _offsets(sub_off, "sub_off")
        if self.uoff.size != self.soff.size:
            raise ValueError("upd_off and sub_off must have the same length")
        self.B = self.uoff.size - 1
        self.d = upd_lo.shape[1]
        if sub_lo.shape[1] != self.d:
            raise ValueError("updates and subscriptions differ in dimension")
        if int(self.uoff[-1]) != upd_lo.shape[0] or int(self.soff[-1]) != sub_lo.shape[0]:
            raise ValueError("the last offset must equal the number of rows")
        self.mode = mode
        self.code = _code(mode, closed)
        self.dev = upd_lo.device
        self.inputs = (upd_lo, upd_hi, sub_lo, sub_hi)
        self.cap = int(pair_capacity)
        self.ws = workspace
        self._reserve(None)
        n_total = int(self.uoff[-1])
        self.counts = torch.zeros(self.B, dtype=torch.int64, device=self.dev)
        self.per_update = (torch.zeros(max(n_total, 1), dtype=torch.int32, device=self.dev)
                           if mode != "count" else None)
        self.pairs = (torch.empty((max(self.cap, 1), 2), dtype=torch.int32, device=self.dev)
                      if mode == "pairs" else None)
        self.pair_off = (torch.zeros(self.B + 1, dtype=torch.int64, device=self.dev)
                         if mode == "pairs" else None)

    def _reserve(self, tuning) -> None:
        """Grows the workspace to what ``tuning`` (None: the default and the
        autotuner's candidates) needs."""
        need = library().ddm_batch_workspace_bytes(
            _aptr(self.uoff), _aptr(self.soff), self.B, self.d, self.code, self.cap,
            ctypes.byref(tuning) if tuning is not None else None)
        if need == 0:
            raise DDMError(DDM_E_INVAL, "ddm_batch_workspace_bytes")
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.dev)

    def _common(self):
        ul, uh, sl, sh = self.inputs
        return [_ptr(ul), _ptr(uh), _aptr(self.uoff), _ptr(sl), _ptr(sh), _aptr(self.soff),
                self.B, self.d, self.code, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel()]

    def _outs(self):
        return [_ptr(self.counts), _ptr(self.per_update) if self.per_update is not None else None,
                _ptr(self.pairs) if self.pairs is not None else None,
                _ptr(self.pair_off) if self.pair_off is not None else None, self.cap]

    def run(self, tuning: Tuning | None = None, stream=None) -> int:
        """One plain batched call; returns the total number of pairs."""
        if stream is None:
            stream = torch.cuda.current_stream(self.dev)
        total = ctypes.c_uint64(0)
        if tuning is not None:
            self._reserve(tuning)
        c, o = self._common(), self._outs()
        with torch.cuda.device(self.dev):
            rc = library().ddm_match_batched(
                *c, ctypes.c_void_p(stream.cuda_stream),
                ctypes.byref(tuning) if tuning is not None else None, o[0], ctypes.byref(total),
                o[1], o[2], o[3], o[4])
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_match_batched")
        return int(total.value)

    def graph(self, tuning: Tuning | None = None) -> "BatchGraph":
        return BatchGraph(self, tuning)

    def autotune(self, stream=None):
        """Fastest tuning for this batch and its replay time in ms."""
        if stream is None:
            stream = torch.cuda.current_stream(self.dev)
        best = Tuning()
        ms = ctypes.c_double(0.0)
        c, o = self._common(), self._outs()
        with torch.cuda.device(self.dev):
            rc = library().ddm_batch_autotune(*c, ctypes.c_void_p(stream.cuda_stream), *o,
                                              ctypes.byref(best), ctypes.byref(ms))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_batch_autotune")
        return best, float(ms.value)

    # results of the last run / replay, per instance
    def instance_pairs(self, b: int) -> torch.Tensor:
        lo, hi = (int(x) for x in self.pair_off[b:b + 2].cpu())
        return self.pairs[lo:hi]

    def instance_per_update(self, b: int) -> torch.Tensor:
        return self.per_update[int(self.uoff[b]):int(self.uoff[b + 1])]


class BatchGraph:
    """The batch captured as one HIP graph (``ddm_batch_graph_*``)."""

    def __init__(self, batch: Batch, tuning: Tuning | None = None):
        self.batch = batch
        self.handle = ctypes.c_void_p(None)
        # a graph keeps its plan in its workspace: give it one of its own
        need = library().ddm_batch_workspace_bytes(
            _aptr(batch.uoff), _aptr(batch.soff), batch.B, batch.d, batch.code, batch.cap,
            ctypes.byref(tuning) if tuning is not None else None)
        if need == 0:
            raise DDMError(DDM_E_INVAL, "ddm_batch_workspace_bytes")
        self.ws = torch.empty(need, dtype=torch.uint8, device=batch.dev)
        c, o = batch._common(), batch._outs()
        c[9], c[10] = ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel()
        with torch.cuda.device(batch.dev):
            rc = library().ddm_batch_graph_create(
                *c, ctypes.byref(tuning) if tuning is not None else None, *o,
                ctypes.byref(self.handle))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_batch_graph_create")

    def launch(self, stream=None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream(self.batch.dev)
        rc = library().ddm_batch_graph_launch(self.handle, ctypes.c_void_p(stream.cuda_stream))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_batch_graph_launch")

    def result(self, stream=None) -> int:
        if stream is None:
            stream = torch.cuda.current_stream(self.batch.dev)
        total = ctypes.c_uint64(0)
        with torch.cuda.device(self.batch.dev):
            rc = library().ddm_batch_graph_result(self.handle, ctypes.c_void_p(stream.cuda_stream),
                                                  ctypes.byref(total))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_batch_graph_result")
        return int(total.value)

    def close(self) -> None:
        if self.handle and self.handle.value:
            library().ddm_batch_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- serving

SERVE_POLICIES = {"batched": 0, "plain": 1, "incremental": 2}


class ServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("launches", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("peak_arena_bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: (int(getattr(self, f)) if f == "launches" else float(getattr(self, f)))
                for f, _ in self._fields_}


class ResidentInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("rebuilds", ctypes.c_int64),
                ("full_matches", ctypes.c_int64), ("movers", ctypes.c_int64),
                ("buckets", ctypes.c_int32), ("full_mode", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def _serve_prototypes(lib):
    if getattr(lib, "_serve_ready", False):
        return lib
    i64, vp, f32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_float
    lib.ddm_sim_step.argtypes = [vp, vp, i64, vp, vp, i64, ctypes.c_int, f32, f32,
                                 ctypes.c_uint64, ctypes.c_uint32, vp]
    lib.ddm_sim_step.restype = ctypes.c_int
    lib.ddm_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(vp)]
    lib.ddm_server_create.restype = ctypes.c_int
    lib.ddm_server_add_sim.argtypes = [vp, vp, vp, i64, vp, vp, i64, ctypes.c_int, f32, f32,
                                       ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
    lib.ddm_server_add_sim.restype = ctypes.c_int
    lib.ddm_server_run.argtypes = [vp, vp, vp, i64, vp, vp, vp, ctypes.POINTER(ServeStats)]
    lib.ddm_server_run.restype = ctypes.c_int
    lib.ddm_server_destroy.argtypes = [vp]
    lib.ddm_server_destroy.restype = ctypes.c_int
    lib.ddm_server_export.argtypes = [vp, ctypes.c_int32]
    lib.ddm_server_export.restype = ctypes.c_int
    lib.ddm_resident_bytes.argtypes = [i64, i64, ctypes.c_int]
    lib.ddm_resident_bytes.restype = ctypes.c_size_t
    lib.ddm_resident_create.argtypes = [vp, ctypes.c_size_t, vp, vp, i64, vp, vp, i64,
                                        ctypes.c_int, f32, f32, ctypes.c_uint64, vp,
                                        ctypes.POINTER(vp)]
    lib.ddm_resident_create.restype = ctypes.c_int
    lib.ddm_resident_step.argtypes = [vp, ctypes.c_uint32, vp]
    lib.ddm_resident_step.restype = ctypes.c_int
    lib.ddm_resident_finish.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.ddm_resident_finish.restype = ctypes.c_int
    lib.ddm_resident_export.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.ddm_resident_export.restype = ctypes.c_int
    lib.ddm_resident_get_info.argtypes = [vp, ctypes.POINTER(ResidentInfo)]
    lib.ddm_resident_get_info.restype = ctypes.c_int
    lib.ddm_resident_destroy.argtypes = [vp]
    lib.ddm_resident_destroy.restype = ctypes.c_int
    lib._serve_ready = True
    return lib


def sim_step(upd_lo, upd_hi, sub_lo, sub_hi, side: float, sigma: float, seed: int, step: int,
             stream=None) -> None:
    """One random-walk step of a simulation's regions, in place (``ddm_sim_step``)."""
    lib = _serve_prototypes(library())
    _check_boxes(upd_lo, upd_hi, "updates")
    _check_boxes(sub_lo, sub_hi, "subscriptions")
    if stream is None:
        stream = torch.cuda.current_stream(upd_lo.device)
    n, d = upd_lo.shape
    m = sub_lo.shape[0]
    rc = lib.ddm_sim_step(_ptr(upd_lo), _ptr(upd_hi), n, _ptr(sub_lo), _ptr(sub_hi), m, d,
                          float(side), float(sigma), int(seed), int(step),
                          ctypes.c_void_p(stream.cuda_stream))
    if rc != DDM_OK:
        raise DDMError(rc, "ddm_sim_step")


class Server:
    """Serving runtime (``ddm_server_*``): resident simulations, open-loop
    request traces, continuous batching under an HBM budget (``arena``)."""

    def __init__(self, arena_bytes: int, policy: str = "batched", slots: int = 4,
                 max_batch: int = 32, device=None):
        self.lib = _serve_prototypes(library())
        self.dev = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.dev)
        self.sims = []
        self.handle = ctypes.c_void_p(None)
        with torch.cuda.device(self.dev):
            rc = self.lib.ddm_server_create(ctypes.c_void_p(self.arena.data_ptr()),
                                            self.arena.numel(), SERVE_POLICIES[policy], slots,
                                            max_batch, ctypes.byref(self.handle))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_server_create")

    def add_sim(self, upd_lo, upd_hi, sub_lo, sub_hi, side: float, sigma: float,
                seed: int) -> int:
        _check_boxes(upd_lo, upd_hi, "updates")
        _check_boxes(sub_lo, sub_hi, "subscriptions")
        sid = ctypes.c_int32(-1)
        n, d = upd_lo.shape
        rc = self.lib.ddm_server_add_sim(self.handle, _ptr(upd_lo), _ptr(upd_hi), n,
                                         _ptr(sub_lo), _ptr(sub_hi), sub_lo.shape[0], d,
                                         float(side), float(sigma), int(seed), ctypes.byref(sid))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_server_add_sim")
        self.sims.append((upd_lo, upd_hi, sub_lo, sub_hi))  # keep the state alive
        return int(sid.value)

    def run(self, sim_ids, arrival_s):
        """Serves the trace; returns (counts uint64 [R], steps uint32 [R],
        latency_s float64 [R], stats dict)."""
        import numpy as np
        sims = np.ascontiguousarray(np.asarray(sim_ids, dtype=np.int32))
        arr = np.ascontiguousarray(np.asarray(arrival_s, dtype=np.float64))
        if sims.shape != arr.shape or sims.ndim != 1:
            raise ValueError("sim_ids and arrival_s must be 1-D of one length")
        R = sims.size
        counts = np.zeros(max(R, 1), dtype=np.uint64)
        steps = np.zeros(max(R, 1), dtype=np.uint32)
        lat = np.zeros(max(R, 1), dtype=np.float64)
        st = ServeStats()
        with torch.cuda.device(self.dev):
            rc = self.lib.ddm_server_run(self.handle, _aptr(sims), _aptr(arr), R, _aptr(counts),
                                         _aptr(steps), _aptr(lat), ctypes.byref(st))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_server_run")
        return counts[:R], steps[:R], lat[:R], st.as_dict()

    def export(self, sim_id: int) -> None:
        """Brings the arrays simulation ``sim_id`` was registered with up to
        date (incremental policy; a no-op for the others)."""
        with torch.cuda.device(self.dev):
            rc = self.lib.ddm_server_export(self.handle, int(sim_id))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_server_export")

    def close(self) -> None:
        if self.handle and self.handle.value:
            self.lib.ddm_server_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def resident_bytes(n: int, m: int, d: int) -> int:
    return int(_serve_prototypes(library()).ddm_resident_bytes(n, m, d))


class Resident:
    """A simulation matched incrementally (``ddm_resident_*``): its regions
    live in a device state in bucket order; ``step(k)`` moves them by step
    k of the random walk (as ``sim_step``) and returns the count of
    intersecting pairs (as ``match(..., "count")`` on the moved rows)."""

    def __init__(self, upd_lo, upd_hi, sub_lo, sub_hi, side: float, sigma: float, seed: int,
                 stream=None):
        self.lib = _serve_prototypes(library())
        _check_boxes(upd_lo, upd_hi, "updates")
        _check_boxes(sub_lo, sub_hi, "subscriptions")
        self.dev = upd_lo.device
        self.n, self.d = upd_lo.shape
        self.m = sub_lo.shape[0]
        size = self.lib.ddm_resident_bytes(self.n, self.m, self.d)
        if size == 0:
            raise DDMError(DDM_E_INVAL, "ddm_resident_bytes")
        self.state = torch.empty(int(size), dtype=torch.uint8, device=self.dev)
        self.handle = ctypes.c_void_p(None)
        if stream is None:
            stream = torch.cuda.current_stream(self.dev)
        rc = self.lib.ddm_resident_create(ctypes.c_void_p(self.state.data_ptr()), size,
                                          _ptr(upd_lo), _ptr(upd_hi), self.n, _ptr(sub_lo),
                                          _ptr(sub_hi), self.m, self.d, float(side), float(sigma),
                                          int(seed), ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.byref(self.handle))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_resident_create")

    def step_async(self, step: int, stream=None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream(self.dev)
        rc = self.lib.ddm_resident_step(self.handle, int(step), ctypes.c_void_p(stream.cuda_stream))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_resident_step")

    def finish(self) -> int:
        k = ctypes.c_uint64(0)
        rc = self.lib.ddm_resident_finish(self.handle, ctypes.byref(k))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_resident_finish")
        return int(k.value)

    def step(self, step: int, stream=None) -> int:
        self.step_async(step, stream)
        return self.finish()

    def export(self, stream=None):
        """Current (upd_lo, upd_hi, sub_lo, sub_hi) in region order."""
        out = [torch.empty((r, self.d), dtype=torch.float32, device=self.dev)
               for r in (self.n, self.n, self.m, self.m)]
        if stream is None:
            stream = torch.cuda.current_stream(self.dev)
        rc = self.lib.ddm_resident_export(self.handle, *[_ptr(t) for t in out],
                                          ctypes.c_void_p(stream.cuda_stream))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_resident_export")
        return out

    def info(self) -> dict:
        st = ResidentInfo()
        rc = self.lib.ddm_resident_get_info(self.handle, ctypes.byref(st))
        if rc != DDM_OK:
            raise DDMError(rc, "ddm_resident_get_info")
        return st.as_dict()

    def close(self) -> None:
        if self.handle and self.handle.value:
            self.lib.ddm_resident_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
