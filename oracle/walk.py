"""CPU reference of the serving workload's motion (random-walk steps).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark to replay, on
the host, the motion that the device applies to a resident simulation, so
that every served count can be checked against the matching oracle.  It
shares no code with the GPU path; both follow the same published definition.

The motion is not part of the paper's method (the paper matches static
region sets); it stands in for the moving regions of a simulation that
issues one matching request per time step.  Definition (bit-exact on any
IEEE float32 implementation):

* generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC 2011): ten rounds on a 4 x 32-bit
  counter with a 2 x 32-bit key; a round multiplies counter words 0 and 2 by
  0xD2511F53 and 0xCD9E8D57 into 64-bit products and returns
  (hi(w2 * M1) ^ w1 ^ k0, lo(w2 * M1), hi(w0 * M0) ^ w3 ^ k1, lo(w0 * M0));
  the key grows by (0x9E3779B9, 0xBB67AE85) after every round;
* z(region, axis, step): the four output words of the draws at counters
  (region, axis, step, j), j = 0, 1, 2, under key (seed mod 2^32, seed >>
  32), each shifted right by 8 and summed as integers (exact, < 2^28), then
  converted to float32, times 2^-24, minus 6: a standard normal by the
  Irwin-Hall approximation (mean 0, variance 1, support [-6, 6]);
* step: lo <- lo + sigma * z, hi <- lo + side, in float32 with one rounding
  per operation.  Updates are regions 0 .. n-1, subscriptions n .. n+m-1.

Parity of this module itself is pinned by the known-answer vectors published
with Philox4x32-10 (tests/golden/), by a second, scalar implementation of the
same definition in the tests and by distribution checks.  ``walk_fast`` runs the same motion through a
C implementation (``walk_oracle.c``, pinned bit for bit to this module by the
tests) for full-size replays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
C_SOURCE = os.path.join(_HERE, "walk_oracle.c")
C_LIBRARY = os.path.join(_HERE, "libwalk.so")
_clib = None


def build_c(source: str = C_SOURCE, output: str = C_LIBRARY) -> str:
    """Compile the C motion with the host compiler, one rounding per float
    operation (no contraction into fused multiply-adds)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", output,
           source]
    subprocess.run(cmd, check=True)
    return output


def _c():
    global _clib
    if _clib is None:
        if not os.path.exists(C_LIBRARY):
            build_c()
        lib = ctypes.CDLL(C_LIBRARY)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.walk_oracle_step.argtypes = [fp, fp, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_uint64,
                                         ctypes.c_uint32]
        lib.walk_oracle_step.restype = None
        _clib = lib
    return _clib

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """Philox4x32-10 of counters ``ctr`` (uint32 [..., 4]) under key (k0, k1)."""
    x = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 &= 0xFFFFFFFF
    k1 &= 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * x[0]
        p1 = _M1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        x = [hi1 ^ x[1] ^ np.uint64(k0), lo1, hi0 ^ x[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([v.astype(np.uint32) for v in x], axis=-1)


def normal_z(regions: np.ndarray, axis: int, step: int, seed: int) -> np.ndarray:
    """Irwin-Hall z for every region index in ``regions`` (float32)."""
    regions = np.asarray(regions, dtype=np.uint32)
    total = np.zeros(regions.shape, dtype=np.uint64)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    for j in range(3):
        ctr = np.stack([regions, np.full_like(regions, axis), np.full_like(regions, step),
                        np.full_like(regions, j)], axis=-1)
        w = philox4x32_10(ctr, k0, k1).astype(np.uint64)
        total += (w >> np.uint64(8)).sum(axis=-1)
    s = total.astype(np.uint32).astype(np.float32)
    return s * np.float32(2.0 ** -24) - np.float32(6.0)


def walk_step(lo: np.ndarray, region0: int, side: float, sigma: float, seed: int,
              step: int):
    """One step of rows ``lo`` (float32 [rows, d]) whose first row is region
    ``region0``; returns the new (lo, hi)."""
    lo = np.asarray(lo, dtype=np.float32)
    rows, d = lo.shape
    out = np.empty_like(lo)
    regions = np.arange(region0, region0 + rows, dtype=np.uint32)
    sig = np.float32(sigma)
    for k in range(d):
        z = normal_z(regions, k, step, seed)
        out[:, k] = lo[:, k] + sig * z
    return out, (out + np.float32(side)).astype(np.float32)


def walk(upd_lo, sub_lo, side: float, sigma: float, seed: int, steps: int, first_step: int = 1):
    """``steps`` steps of a simulation from lower corners (upd_lo, sub_lo);
    yields (step, upd_lo, upd_hi, sub_lo, sub_hi) after every step."""
    ul = np.asarray(upd_lo, dtype=np.float32)
    sl = np.asarray(sub_lo, dtype=np.float32)
    n = ul.shape[0]
    for st in range(first_step, first_step + steps):
        ul, uh = walk_step(ul, 0, side, sigma, seed, st)
        sl, sh = walk_step(sl, n, side, sigma, seed, st)
        yield st, ul, uh, sl, sh


def walk_step_c(lo: np.ndarray, region0: int, side: float, sigma: float, seed: int,
                step: int):
    """``walk_step`` by the C implementation; returns the new (lo, hi)."""
    out = np.ascontiguousarray(np.asarray(lo, dtype=np.float32)).copy()
    rows = out.shape[0]
    d = out.shape[1] if out.ndim == 2 else 1
    hi = np.empty_like(out)
    fp = ctypes.POINTER(ctypes.c_float)
    if rows:
        _c().walk_oracle_step(out.ctypes.data_as(fp), hi.ctypes.data_as(fp), rows, d,
                              region0, float(np.float32(side)), float(np.float32(sigma)),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, int(step))
    return out, hi


def walk_fast(upd_lo, sub_lo, side: float, sigma: float, seed: int, steps: int,
              first_step: int = 1):
    """``walk`` by the C implementation."""
    ul = np.asarray(upd_lo, dtype=np.float32)
    sl = np.asarray(sub_lo, dtype=np.float32)
    n = ul.shape[0]
    for st in range(first_step, first_step + steps):
        ul, uh = walk_step_c(ul, 0, side, sigma, seed, st)
        sl, sh = walk_step_c(sl, n, side, sigma, seed, st)
        yield st, ul, uh, sl, sh
