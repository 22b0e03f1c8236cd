"""CPU oracle for region matching (Data Distribution Management).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path.

Contents, each citing the passage of Marzolla & D'Angelo (DS-RT 2017) it
follows:

* ``Oracle.sbm``        -- Algorithm 4 (Sort-Based-Matching-1D) on axis 0 with
                           the other axes ANDed per pair (Sec. 3, after
                           Algorithm 1), serial C (``sbm_oracle.c``).
* ``Oracle.bruteforce`` -- Algorithm 2 (BruteForce-1D) over d axes, serial C.
* ``bruteforce_numpy``  -- the problem statement of Sec. 3 written as a
                           vectorised definition: box i and box j intersect
                           iff max(lo) < min(hi) on every axis.
* ``closed_form_1d``    -- an identity for one axis: the subscriptions that
                           overlap update u are those that start before u ends
                           minus those that end before (or where) u starts.
* ``parallel_sbm_model``-- Algorithms 5 and 6 (Parallel-SBM-1D and the
                           initialisation of SubSet[p] / UpdSet[p]) in plain
                           Python for small inputs.

Readings of the paper (see the header of ``sbm_oracle.c``): half-open
intervals; ties upper-before-lower, then update-before-subscription, then id;
empty regions (lo == hi on some axis) match nothing; NaN or lo > hi is an
error; 0-based ids; pairs are (update id, subscription id) in lexicographic
order.  ``closed=True`` selects the closed reading instead (Algorithm 1's
tests as printed, lo <= hi' and lo' <= hi): no region is empty and ties sort
lower-before-upper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "sbm_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

OR_OK = 0
OR_E_INVAL = -1
OR_E_CAPACITY = -2


class OracleError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


def build(source: str = SOURCE, output: str = LIBRARY) -> str:
    """Compile the C oracle with the host compiler (no GPU toolchain)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", output, source, "-lm"]
    subprocess.run(cmd, check=True)
    return output


def _f32(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return a


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Oracle:
    """ctypes front end of the C oracle; ``path`` selects the shared object."""

    def __init__(self, path: str | None = None):
        path = path or LIBRARY
        if not os.path.exists(path):
            build(output=path)
        self.path = path
        self.lib = ctypes.CDLL(path)
        fp = ctypes.POINTER(ctypes.c_float)
        sig = [fp, fp, ctypes.c_int64, fp, fp, ctypes.c_int64, ctypes.c_int,
               ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32),
               ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]
        for name in ("oracle_sbm", "oracle_bruteforce", "oracle_sbm_closed",
                     "oracle_bruteforce_closed"):
            fn = getattr(self.lib, name)
            fn.argtypes = sig
            fn.restype = ctypes.c_int
        st = self.lib.oracle_sweep_state
        st.argtypes = [fp, fp, ctypes.c_int64, fp, fp, ctypes.c_int64, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
        st.restype = ctypes.c_int64

    def _run(self, fname, ulo, uhi, slo, shi, pairs: bool, per_update: bool = True,
             capacity: int | None = None):
        ulo, uhi, slo, shi = _f32(ulo), _f32(uhi), _f32(slo), _f32(shi)
        n, m = ulo.shape[0], slo.shape[0]
        d = ulo.shape[1] if n else (slo.shape[1] if m else 1)
        if ulo.shape != uhi.shape or slo.shape != shi.shape:
            raise OracleError("lo/hi shape mismatch", OR_E_INVAL)
        if n and m and ulo.shape[1] != slo.shape[1]:
            raise OracleError("dimension mismatch", OR_E_INVAL)
        fn = getattr(self.lib, fname)
        cnt = ctypes.c_uint64(0)
        per = np.zeros(max(n, 1), dtype=np.int32) if per_update else None
        per_p = _ptr(per, ctypes.c_int32) if per_update else None
        if not pairs:
            rc = fn(_ptr(ulo, ctypes.c_float), _ptr(uhi, ctypes.c_float), n,
                    _ptr(slo, ctypes.c_float), _ptr(shi, ctypes.c_float), m, d,
                    ctypes.byref(cnt), per_p, None, 0)
            if rc != OR_OK:
                raise OracleError(f"{fname} failed with {rc}", rc)
            return int(cnt.value), (per[:n].copy() if per_update else None), None
        cap = capacity if capacity is not None else 1024
        while True:
            buf = np.zeros((max(cap, 1), 2), dtype=np.int32)
            rc = fn(_ptr(ulo, ctypes.c_float), _ptr(uhi, ctypes.c_float), n,
                    _ptr(slo, ctypes.c_float), _ptr(shi, ctypes.c_float), m, d,
                    ctypes.byref(cnt), per_p, _ptr(buf, ctypes.c_int32), cap)
            if rc == OR_E_CAPACITY and capacity is None:
                cap = int(cnt.value)
                continue
            if rc != OR_OK:
                raise OracleError(f"{fname} failed with {rc}", rc)
            k = int(cnt.value)
            return k, (per[:n].copy() if per_update else None), buf[:k].copy()

    def sbm(self, ulo, uhi, slo, shi, pairs: bool = True, per_update: bool = True,
            capacity: int | None = None, closed: bool = False):
        """Algorithm 4 + per-axis AND.  Returns (count, per_update[n] int32,
        pairs[K,2] int32 or None).  ``closed``: closed intervals."""
        name = "oracle_sbm_closed" if closed else "oracle_sbm"
        return self._run(name, ulo, uhi, slo, shi, pairs, per_update, capacity)

    def bruteforce(self, ulo, uhi, slo, shi, pairs: bool = True, per_update: bool = True,
                   closed: bool = False):
        """Algorithm 2 over d axes.  Same return convention as ``sbm``."""
        name = "oracle_bruteforce_closed" if closed else "oracle_bruteforce"
        return self._run(name, ulo, uhi, slo, shi, pairs, per_update)

    def sweep_state(self, ulo, uhi, slo, shi, cuts):
        """Serial SubSet/UpdSet of Algorithm 4 after ``cuts[c]`` endpoints of
        the sorted T.  Returns a list (one per cut) of sets of (kind, id),
        kind 0 = update, 1 = subscription."""
        ulo, uhi, slo, shi = _f32(ulo), _f32(uhi), _f32(slo), _f32(shi)
        n, m = ulo.shape[0], slo.shape[0]
        d = ulo.shape[1] if n else (slo.shape[1] if m else 1)
        cuts = np.ascontiguousarray(np.asarray(cuts, dtype=np.int64))
        off = np.zeros(len(cuts) + 1, dtype=np.int64)
        cap = max(1, (n + m) * max(1, len(cuts)))
        kinds = np.zeros(cap, dtype=np.int32)
        ids = np.zeros(cap, dtype=np.int64)
        rc = self.lib.oracle_sweep_state(
            _ptr(ulo, ctypes.c_float), _ptr(uhi, ctypes.c_float), n,
            _ptr(slo, ctypes.c_float), _ptr(shi, ctypes.c_float), m, d,
            _ptr(cuts, ctypes.c_int64), len(cuts), _ptr(off, ctypes.c_int64),
            _ptr(kinds, ctypes.c_int32), _ptr(ids, ctypes.c_int64), cap)
        if rc < 0:
            raise OracleError(f"oracle_sweep_state failed with {rc}", rc)
        return [set(zip(kinds[off[c]:off[c + 1]].tolist(), ids[off[c]:off[c + 1]].tolist()))
                for c in range(len(cuts))]


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


# ---------------------------------------------------------------------------
# Plain definitions in numpy (independent of the C code)
# ---------------------------------------------------------------------------

def bruteforce_numpy(ulo, uhi, slo, shi, closed: bool = False) -> np.ndarray:
    """The problem statement of Sec. 3 with half-open boxes: returns the
    boolean matrix hit[i, j] = AND_k max(ulo_ik, slo_jk) < min(uhi_ik, shi_jk)
    (<= for closed boxes).  Intended for n*m up to a few million."""
    ulo, uhi, slo, shi = (_f32(a).astype(np.float64) for a in (ulo, uhi, slo, shi))
    lo_max = np.maximum(ulo[:, None, :], slo[None, :, :])
    hi_min = np.minimum(uhi[:, None, :], shi[None, :, :])
    return np.all(lo_max <= hi_min if closed else lo_max < hi_min, axis=2)


def pairs_from_matrix(hit: np.ndarray) -> np.ndarray:
    """Lexicographically ordered (update id, subscription id) pairs."""
    u, s = np.nonzero(hit)
    return np.stack([u, s], axis=1).astype(np.int32).reshape(-1, 2)


def nonempty_mask(lo, hi) -> np.ndarray:
    lo, hi = _f32(lo), _f32(hi)
    return np.all(lo != hi, axis=1)


def closed_form_1d(ulo, uhi, slo, shi, axis: int = 0, closed: bool = False) -> np.ndarray:
    """Per-update overlap counts on one axis among non-empty regions.

    For half-open intervals, subscription s overlaps update u iff
    s.lo < u.hi and not (s.hi <= u.lo); since s.lo < s.hi, the second set is
    contained in the first, so the count is
        #{s : s.lo < u.hi} - #{s : s.hi <= u.lo}.
    Regions that are empty on any axis are excluded on both sides, and an
    empty update gets 0.  For closed intervals (none is empty) the same
    argument with s.lo <= s.hi gives
        #{s : s.lo <= u.hi} - #{s : s.hi < u.lo}.
    Returns int64 counts."""
    ulo, uhi, slo, shi = _f32(ulo), _f32(uhi), _f32(slo), _f32(shi)
    if closed:
        s_lo = np.sort(slo[:, axis].astype(np.float64))
        s_hi = np.sort(shi[:, axis].astype(np.float64))
        starts = np.searchsorted(s_lo, uhi[:, axis].astype(np.float64), side="right")
        ends = np.searchsorted(s_hi, ulo[:, axis].astype(np.float64), side="left")
        return starts.astype(np.int64) - ends.astype(np.int64)
    su = nonempty_mask(ulo, uhi)
    ss = nonempty_mask(slo, shi)
    s_lo = np.sort(slo[ss, axis].astype(np.float64))
    s_hi = np.sort(shi[ss, axis].astype(np.float64))
    u_lo = ulo[:, axis].astype(np.float64)
    u_hi = uhi[:, axis].astype(np.float64)
    starts_before_end = np.searchsorted(s_lo, u_hi, side="left")
    ends_before_start = np.searchsorted(s_hi, u_lo, side="right")
    c = starts_before_end.astype(np.int64) - ends_before_start.astype(np.int64)
    c[~su] = 0
    return c


# ---------------------------------------------------------------------------
# Algorithms 5 and 6 (segment-parallel SBM) as a plain-Python model
# ---------------------------------------------------------------------------

UPD, SUB = 0, 1
UPPER, LOWER = 0, 1


def endpoint_list(ulo, uhi, slo, shi, axis: int = 0):
    """Sorted endpoint list T of the non-empty regions: tuples
    (coord, type, kind, id) in the order coordinate, upper-before-lower,
    update-before-subscription, id."""
    ulo, uhi, slo, shi = _f32(ulo), _f32(uhi), _f32(slo), _f32(shi)
    T = []
    for kind, lo, hi in ((UPD, ulo, uhi), (SUB, slo, shi)):
        ok = nonempty_mask(lo, hi)
        for i in np.nonzero(ok)[0].tolist():
            T.append((float(lo[i, axis]), LOWER, kind, i))
            T.append((float(hi[i, axis]), UPPER, kind, i))
    T.sort()
    return T


def _other_axes_overlap(ulo, uhi, slo, shi, u, s, d):
    for k in range(1, d):
        if not (float(ulo[u, k]) < float(shi[s, k]) and float(slo[s, k]) < float(uhi[u, k])):
            return False
    return True


def alg6_initial_sets(T, cuts, displayed_equation: bool = False):
    """Algorithm 6.  ``cuts`` are the segment start positions in T (cuts[0] is
    0).  Local pass: per segment the sets Sadd/Sdel/Uadd/Udel; master pass:
    SubSet[p] = (SubSet[p-1] U Sadd[p-1]) minus Sdel[p-1], same for updates.
    With ``displayed_equation`` the master pass uses Sadd[p]/Sdel[p] instead,
    which is how the displayed equation after Algorithm 6 reads."""
    P = len(cuts)
    bounds = list(cuts) + [len(T)]
    Sadd, Sdel, Uadd, Udel = ([set() for _ in range(P)] for _ in range(4))
    for p in range(P):
        for (_, typ, kind, i) in T[bounds[p]:bounds[p + 1]]:
            add, dele = (Sadd[p], Sdel[p]) if kind == SUB else (Uadd[p], Udel[p])
            if typ == LOWER:
                add.add(i)
            elif i in add:
                add.discard(i)
            else:
                dele.add(i)
    SubSet, UpdSet = [set() for _ in range(P)], [set() for _ in range(P)]
    for p in range(1, P):
        q = p if displayed_equation else p - 1
        SubSet[p] = (SubSet[p - 1] | Sadd[q]) - Sdel[q]
        UpdSet[p] = (UpdSet[p - 1] | Uadd[q]) - Udel[q]
    return SubSet, UpdSet, (Sadd, Sdel, Uadd, Udel)


def parallel_sbm_model(ulo, uhi, slo, shi, cuts):
    """Algorithm 5: every segment of T is swept from its initial sets
    (Algorithm 6); the union of the per-segment results is returned as a
    sorted pair array together with the initial sets."""
    ulo_, uhi_, slo_, shi_ = _f32(ulo), _f32(uhi), _f32(slo), _f32(shi)
    d = ulo_.shape[1] if ulo_.shape[0] else slo_.shape[1]
    T = endpoint_list(ulo_, uhi_, slo_, shi_)
    SubSet0, UpdSet0, _ = alg6_initial_sets(T, cuts)
    bounds = list(cuts) + [len(T)]
    L = []
    for p in range(len(cuts)):
        SubSet, UpdSet = set(SubSet0[p]), set(UpdSet0[p])
        for (_, typ, kind, i) in T[bounds[p]:bounds[p + 1]]:
            if kind == SUB:
                if typ == LOWER:
                    SubSet.add(i)
                else:
                    SubSet.discard(i)
                    for x in UpdSet:
                        if _other_axes_overlap(ulo_, uhi_, slo_, shi_, x, i, d):
                            L.append((x, i))
            else:
                if typ == LOWER:
                    UpdSet.add(i)
                else:
                    UpdSet.discard(i)
                    for x in SubSet:
                        if _other_axes_overlap(ulo_, uhi_, slo_, shi_, i, x, d):
                            L.append((i, x))
    L.sort()
    pairs = np.asarray(L, dtype=np.int32).reshape(-1, 2)
    return pairs, SubSet0, UpdSet0
