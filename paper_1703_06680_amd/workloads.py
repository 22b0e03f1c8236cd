"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers: it holds none of the matching arithmetic, and
it is the one piece of code that both the GPU path's tests/benchmarks and the
CPU oracle's tests consume.

The experimental setup of the paper (Sec. 5, "Experimental setup") places
N = n + m extents uniformly on a routing space of length L = 1e6, all of the
same length l chosen from the overlapping degree alpha = N * l / L, i.e.
l = alpha * L / N.  Here the same recipe is applied on every axis of a
d-dimensional routing space [0, L)^d:

* generator: numpy PCG64 seeded with SeedSequence([seed, stream]); stream 0 =
  updates, 1 = subscriptions, 1000 + i = batched instance i, 2000 + j =
  serving simulation j;
* lower corner: float32(U[0,1) * L) per axis, clamped to the largest float32
  below L;
* side: l32 = float32(alpha * L / (n + m)) (computed in float64, rounded
  once);
* upper corner: hi = lo + l32 in float32 (IEEE round-to-nearest-even), so
  tiny alpha produces many empty intervals (lo == hi), as float rounding
  dictates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

L_SPACE = 1.0e6
LO_MAX = np.float32(999999.9375)  # largest float32 strictly below 1e6

UPD_STREAM = 0
SUB_STREAM = 1
BATCH_STREAM_BASE = 1000
SIM_STREAM_BASE = 2000


def generator(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def side_length(alpha: float, n_total: int, L: float = L_SPACE) -> np.float32:
    """l = alpha * L / N, rounded once to float32."""
    return np.float32(alpha * L / max(n_total, 1))


def uniform_regions(rng: np.random.Generator, count: int, d: int, side: np.float32,
                    L: float = L_SPACE):
    """``count`` boxes with float32 lower corners uniform on [0, L)^d and all
    sides equal to ``side``.  Returns (lo, hi), float32 [count, d]."""
    lo = (rng.random((count, d)) * L).astype(np.float32)
    np.minimum(lo, np.nextafter(np.float32(L), np.float32(0)), out=lo)
    hi = (lo + np.float32(side)).astype(np.float32)
    return lo, hi


@dataclass
class Instance:
    upd_lo: np.ndarray
    upd_hi: np.ndarray
    sub_lo: np.ndarray
    sub_hi: np.ndarray
    alpha: float
    name: str = ""

    @property
    def n(self):
        return self.upd_lo.shape[0]

    @property
    def m(self):
        return self.sub_lo.shape[0]

    @property
    def d(self):
        return self.upd_lo.shape[1]


def uniform_instance(n: int, m: int, d: int, alpha: float, seed: int = 0,
                     upd_stream: int = UPD_STREAM, sub_stream: int = SUB_STREAM,
                     name: str = "") -> Instance:
    side = side_length(alpha, n + m)
    ulo, uhi = uniform_regions(generator(seed, upd_stream), n, d, side)
    slo, shi = uniform_regions(generator(seed, sub_stream), m, d, side)
    return Instance(ulo, uhi, slo, shi, alpha, name or f"uniform_d{d}_n{n}_m{m}_a{alpha:g}")


# The paper-shaped configurations (d, n = m, alphas).
CONFIGS = {
    "cfg1": dict(d=1, n=10_000, alphas=(1.0,)),
    "cfg2": dict(d=2, n=500_000, alphas=(0.01, 1.0, 100.0)),
    "cfg3": dict(d=3, n=5_000_000, alphas=(1.0, 10.0, 100.0)),
}


def config_instance(cfg: str, alpha: float | None = None, seed: int = 0) -> Instance:
    c = CONFIGS[cfg]
    a = c["alphas"][0] if alpha is None else alpha
    return uniform_instance(c["n"], c["n"], c["d"], a, seed, name=f"{cfg}_a{a:g}")


def correlated_d3(n: int, alpha: float, seed: int = 0) -> Instance:
    """Stress variant with many true 3-D matches: axis-0 lower corners are
    uniform as above; on axes 1 and 2 the lower corner is the axis-0 lower
    corner plus U[0, 2l), in float32."""
    side = side_length(alpha, 2 * n)
    out = []
    for stream in (UPD_STREAM, SUB_STREAM):
        rng = generator(seed, 100 + stream)
        lo0 = np.minimum((rng.random(n) * L_SPACE).astype(np.float32), LO_MAX)
        lo = np.empty((n, 3), dtype=np.float32)
        lo[:, 0] = lo0
        for k in (1, 2):
            lo[:, k] = (lo0 + (rng.random(n) * (2.0 * float(side))).astype(np.float32)).astype(np.float32)
        hi = (lo + side).astype(np.float32)
        out.append((lo, hi))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, alpha, f"correlated_d3_n{n}_a{alpha:g}")


def loguniform_boxes(n: int, m: int, d: int, alpha: float, seed: int = 0,
                     decades: float = 6.0) -> Instance:
    """Skewed placement: lower corners log-uniform over ``decades`` decades
    from 1 on every axis (half of them below 1e3 for six decades), each side
    proportional to its lower corner, with the overlap degree alpha of the
    uniform workload in logarithmic coordinates: side = lo * alpha *
    ln(10^decades) / (n + m), rounded to float32, upper = lower + side in
    float32."""
    span = decades * math.log(10.0)
    rel = np.float32(alpha * span / max(n + m, 1))
    out = []
    for stream, cnt in ((UPD_STREAM, n), (SUB_STREAM, m)):
        rng = generator(seed, 200 + stream)
        lo = np.exp(rng.random((cnt, d)) * span).astype(np.float32)
        hi = (lo + (lo * rel).astype(np.float32)).astype(np.float32)
        out.append((lo, hi))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, alpha, f"loguniform_d{d}_n{n}_a{alpha:g}")


def clustered_boxes(n: int, m: int, d: int, alpha: float, seed: int = 0, clusters: int = 16,
                    sigma: float = 2.0e4) -> Instance:
    """Clustered placement: lower corners drawn around ``clusters`` centres
    (uniform on [2e5, 8e5)^d, shared by both sets) with a normal spread of
    ``sigma`` per axis, clamped to [0, L).  The side on axis k is chosen so
    that the expected number of 1-D overlaps per box is alpha, as in the
    uniform workload: l_k = alpha / ((n + m) * integral of f_k^2), f_k the
    mixture density of axis k (a sum of normal densities over centre pairs),
    rounded once to float32."""
    centres = 2.0e5 + generator(seed, 300).random((clusters, d)) * 6.0e5
    sides = np.empty(d, dtype=np.float32)
    for k in range(d):
        diff = centres[:, None, k] - centres[None, :, k]
        f2 = np.exp(-diff ** 2 / (4.0 * sigma ** 2)).sum() / (clusters ** 2 * 2.0 * sigma * math.sqrt(math.pi))
        sides[k] = np.float32(alpha / (max(n + m, 1) * f2))
    out = []
    for stream, cnt in ((UPD_STREAM, n), (SUB_STREAM, m)):
        rng = generator(seed, 300 + 1 + stream)
        which = rng.integers(0, clusters, size=cnt)
        lo = (centres[which] + rng.standard_normal((cnt, d)) * sigma).astype(np.float32)
        np.clip(lo, np.float32(0.0), LO_MAX, out=lo)
        hi = (lo + sides).astype(np.float32)
        out.append((lo, hi))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, alpha, f"clustered_d{d}_n{n}_a{alpha:g}")


def anisotropic_boxes(n: int, m: int, d: int, alpha: float, stretch: float = 100.0,
                      seed: int = 0) -> Instance:
    """The uniform workload with boxes ``stretch`` times longer on axis 0
    than on the others (side l32 on axes 1 .. d-1, float32(stretch * l32) on
    axis 0): axis 0 carries ``stretch`` times the 1-D candidates of any other
    axis."""
    side = side_length(alpha, n + m)
    sides = np.full(d, side, dtype=np.float32)
    sides[0] = np.float32(stretch * float(side))
    out = []
    for stream, cnt in ((UPD_STREAM, n), (SUB_STREAM, m)):
        rng = generator(seed, 400 + stream)
        lo = np.minimum((rng.random((cnt, d)) * L_SPACE).astype(np.float32), LO_MAX)
        hi = (lo + sides).astype(np.float32)
        out.append((lo, hi))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, alpha, f"anisotropic_d{d}_n{n}_a{alpha:g}_x{stretch:g}")


def signed_logscale_boxes(n: int, m: int, d: int, alpha: float, seed: int = 0,
                          other_alpha: float | None = None, decades: float = 6.0,
                          straddle: float = 0.01) -> Instance:
    """Axis 0 as in the uniform workload (side alpha L / N); on axes 1 ..
    d-1 lower corners of random sign with magnitudes log-uniform over
    ``decades`` decades from 1, each side proportional to its magnitude
    (side = |lo| * other_alpha * ln(10^decades) / N, other_alpha = alpha by
    default); a fraction ``straddle`` of the boxes instead spans
    [-u, v) with u, v uniform on [0, 1), across zero."""
    oa = alpha if other_alpha is None else other_alpha
    side0 = side_length(alpha, n + m)
    rel = np.float32(oa * decades * math.log(10.0) / max(n + m, 1))
    out = []
    for stream, cnt in ((UPD_STREAM, n), (SUB_STREAM, m)):
        rng = generator(seed, 500 + stream)
        lo = np.empty((cnt, d), dtype=np.float32)
        hi = np.empty((cnt, d), dtype=np.float32)
        lo[:, 0] = np.minimum((rng.random(cnt) * L_SPACE).astype(np.float32), LO_MAX)
        hi[:, 0] = (lo[:, 0] + side0).astype(np.float32)
        for k in range(1, d):
            mag = np.exp(rng.random(cnt) * decades * math.log(10.0)).astype(np.float32)
            sign = np.where(rng.random(cnt) < 0.5, np.float32(-1.0), np.float32(1.0))
            lk = (sign * mag).astype(np.float32)
            lo[:, k] = lk
            hi[:, k] = (lk + (mag * rel).astype(np.float32)).astype(np.float32)
            cross = rng.random(cnt) < straddle
            lo[cross, k] = -rng.random(int(cross.sum())).astype(np.float32)
            hi[cross, k] = rng.random(int(cross.sum())).astype(np.float32)
            fix = hi[:, k] < lo[:, k]
            hi[fix, k] = lo[fix, k]
        out.append((lo, hi))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, alpha, f"signedlog_d{d}_n{n}_a{alpha:g}_o{oa:g}")


def tie_heavy(n: int, m: int, d: int, grid: int = 12, max_len: int = 4, seed: int = 0) -> Instance:
    """Small integer-grid boxes: lower corners in {0..grid}, side lengths in
    {0..max_len}.  Touching, nested, identical and empty intervals are all
    frequent."""
    rng = generator(seed, 7)
    out = []
    for cnt in (n, m):
        lo = rng.integers(0, grid + 1, size=(cnt, d)).astype(np.float32)
        ln = rng.integers(0, max_len + 1, size=(cnt, d)).astype(np.float32)
        out.append((lo, (lo + ln).astype(np.float32)))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, float("nan"), f"ties_d{d}_n{n}_m{m}_g{grid}")


def random_float_boxes(n: int, m: int, d: int, seed: int = 0, extent: float = 100.0,
                       max_side: float = 20.0) -> Instance:
    """Small boxes with random float corners and random (per-box, per-axis)
    sides; some sides are forced to zero."""
    rng = generator(seed, 8)
    out = []
    for cnt in (n, m):
        lo = (rng.random((cnt, d)) * extent).astype(np.float32)
        side = (rng.random((cnt, d)) * max_side).astype(np.float32)
        side[rng.random((cnt, d)) < 0.05] = 0
        out.append((lo, (lo + side).astype(np.float32)))
    (ulo, uhi), (slo, shi) = out
    return Instance(ulo, uhi, slo, shi, float("nan"), f"float_d{d}_n{n}_m{m}")


def batched_sizes(count: int = 512, lo: int = 1_000, hi: int = 200_000,
                  alphas=(0.01, 1.0, 10.0), seed: int = 0):
    """Per-instance (n = m, alpha) for the batched workload: n log-uniform on
    [lo, hi], alpha a uniform choice from ``alphas``."""
    rng = generator(seed, BATCH_STREAM_BASE - 1)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    al = np.asarray(alphas, dtype=np.float64)[rng.integers(0, len(alphas), size=count)]
    return sizes, al


def batched_instances(count: int = 512, d: int = 2, seed: int = 0, lo: int = 1_000,
                      hi: int = 200_000, alphas=(0.01, 1.0, 10.0)):
    sizes, al = batched_sizes(count, lo, hi, alphas, seed)
    insts = []
    for i in range(count):
        n = int(sizes[i])
        side = side_length(float(al[i]), 2 * n)
        rng = generator(seed, BATCH_STREAM_BASE + i)
        ulo, uhi = uniform_regions(rng, n, d, side)
        slo, shi = uniform_regions(rng, n, d, side)
        insts.append(Instance(ulo, uhi, slo, shi, float(al[i]), f"batch{i}"))
    return insts


def concat_instances(insts):
    """Stores instances back to back: (upd_lo, upd_hi, upd_off, sub_lo,
    sub_hi, sub_off) with host int64 offsets [B + 1]; instance b owns rows
    upd_off[b]:upd_off[b+1] and sub_off[b]:sub_off[b+1]."""
    d = insts[0].d if insts else 1
    uoff = np.zeros(len(insts) + 1, dtype=np.int64)
    soff = np.zeros(len(insts) + 1, dtype=np.int64)
    for i, t in enumerate(insts):
        if t.d != d:
            raise ValueError("instances of one batch share d")
        uoff[i + 1] = uoff[i] + t.n
        soff[i + 1] = soff[i] + t.m

    def cat(arrs):
        arrs = [np.asarray(a, dtype=np.float32).reshape(-1, d) for a in arrs]
        return np.ascontiguousarray(np.concatenate(arrs) if arrs else np.zeros((0, d), np.float32))

    return (cat([t.upd_lo for t in insts]), cat([t.upd_hi for t in insts]), uoff,
            cat([t.sub_lo for t in insts]), cat([t.sub_hi for t in insts]), soff)


def serving_sims(count: int = 32, d: int = 2, seed: int = 0, lo: int = 10_000,
                 hi: int = 2_000_000, alpha: float = 1.0):
    """Initial states of the serving workload: simulation j has n = m regions
    (n log-uniform on [lo, hi]) placed uniformly, side alpha * L / (2n);
    returns a list of (Instance, side, sigma = 0.1 * side, seed of its walk)."""
    rng = generator(seed, SIM_STREAM_BASE - 1)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    out = []
    for j in range(count):
        n = int(sizes[j])
        side = side_length(alpha, 2 * n)
        r = generator(seed, SIM_STREAM_BASE + j)
        ulo, uhi = uniform_regions(r, n, d, side)
        slo, shi = uniform_regions(r, n, d, side)
        walk_seed = (int(seed) << 32) | (SIM_STREAM_BASE + j)
        out.append((Instance(ulo, uhi, slo, shi, alpha, f"sim{j}"), float(side),
                    float(np.float32(0.1) * side), walk_seed))
    return out


def poisson_arrivals(count: int, qps: float, seed: int = 0, sims: int = 32):
    """Open-loop trace: ``count`` requests with exponential inter-arrival
    times of mean 1/qps, each for a uniformly chosen simulation.  Returns
    (sim ids int32 [count], arrival times float64 [count] in seconds)."""
    rng = generator(seed, SIM_STREAM_BASE - 2)
    gaps = rng.exponential(1.0 / qps, size=count)
    return rng.integers(0, sims, size=count).astype(np.int32), np.cumsum(gaps)
