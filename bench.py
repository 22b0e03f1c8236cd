#!/usr/bin/env python3
"""Benchmark of sort-based matching on one MI355X.

One step = one complete ``ddm_match`` call (validate/encode, sort, sweep,
per-update counts and total) over the resident synthetic workload: d = 3,
n = m = 5e6 boxes placed uniformly on [0, 1e6)^3, side alpha * 1e6 / (n + m),
the N = n + m = 1e7 configuration the headline metric is quoted on.  Inputs
are uploaded before timing; the timed region covers exactly --steps calls
bracketed by device synchronisations.

Printed: one JSON line with whole-job throughput (regions matched per second),
the roofline of the dominant kernel (algorithmic bytes per launch over its
average duration, timed with HIP events inside the library on the stream the
kernels run on), and the CPU oracle timed on this host as a reported baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
METRIC = "matched regions/sec + HBM GB/s fraction at N=1e7; p50/p99 latency served"


def algorithmic_bytes(phase: str, n: int, m: int, d: int, nonempty: int, mode: str):
    """Bytes a kernel phase must move once per launch (inputs read once,
    outputs written once), independent of caching or re-reads.  A region
    record is 16 bytes (lower and upper key on the swept axis, the region
    index, quantised bounds of the other axes).  Per region:

      bucket.count    8d read (lo and hi rows), + 4 per update written in
                      per-update mode (the count pass clears that output);
      bucket.scatter  8d read + 16 written (one record);
      bucket.sweep    16 read (one record), + what the matches write (not
                      counted: at most 4 bytes per update, in practice
                      negligible next to the records);
      keys            8d read + 8 written (lower/upper keys);
      sort.downsweep  8 read + 8 written per element (first pass: 4 + 8);
      sort.upsweep    4 read per element;
      gather          4 + 4 + 8(d-1) read, 4 + 8(d-1) written;
      sweep.count     12 + 8(d-1) read (+ 4 per update in per-update mode).
    """
    N = n + m
    rec = 16
    out = 4 * n if mode != "count" else 0
    if phase == "bucket.count":
        return N * 8 * d + out
    if phase == "bucket.scatter":
        return N * 8 * d + nonempty * rec
    if phase == "bucket.sweep":
        return nonempty * rec
    if phase == "keys":
        return N * (8 * d + 8)
    if phase == "sort.upsweep":
        return N * 4
    if phase == "sort.downsweep":
        return N * 16
    if phase == "gather":
        return nonempty * (8 + 8 * (d - 1) + 4 + 8 * (d - 1))
    if phase == "sweep.count":
        return nonempty * (12 + 8 * (d - 1)) + (4 * n if mode != "count" else 0)
    return None


def bench_batched(args, ddm, W, torch, np, cpu=None):
    """512 independent d=2 instances (n = m log-uniform on [1e3, 2e5], alpha
    uniform in {0.01, 1, 10}), pairs mode: 512 plain ddm_match calls against
    one batched call and against replays of the autotuned captured graph."""
    dev = torch.device("cuda:0")
    insts = W.batched_instances(args.batch_count, d=2, seed=0)
    ulo, uhi, uoff, slo, shi, soff = W.concat_instances(insts)
    g = [torch.from_numpy(a).to(dev) for a in (ulo, uhi, slo, shi)]
    regions = int(uoff[-1] + soff[-1])
    cap = 1 << 21
    batch = ddm.Batch(g[0], g[1], uoff, g[2], g[3], soff, mode="pairs", pair_capacity=cap)
    stream = torch.cuda.current_stream(dev)

    # plain: one ddm_match per instance, each synchronising
    big = max(range(len(insts)), key=lambda b: insts[b].n + insts[b].m)
    ws = torch.empty(ddm.workspace_bytes(insts[big].n, insts[big].m, 2, "pairs", cap),
                     dtype=torch.uint8, device=dev)
    pbuf = torch.empty((cap, 2), dtype=torch.int32, device=dev)

    def plain_pass(keep=False):
        ks, kept = [], []
        for b in range(len(insts)):
            u0, u1, s0, s1 = int(uoff[b]), int(uoff[b + 1]), int(soff[b]), int(soff[b + 1])
            k = ddm.match_into(g[0][u0:u1], g[1][u0:u1], g[2][s0:s1], g[3][s0:s1], mode="pairs",
                               workspace=ws, pairs=pbuf, stream=stream)
            ks.append(k)
            if keep:
                kept.append(pbuf[:k].clone())
        return ks, kept

    plain_pass()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_reps):
        ks_plain, _ = plain_pass()
    plain_ms = 1e3 * (time.perf_counter() - t) / args.batch_reps
    ks_plain, kept = plain_pass(keep=True)
    pairs_plain = torch.cat(kept) if kept else torch.empty((0, 2), dtype=torch.int32, device=dev)

    # one batched call (plan upload included), default tuning
    batch.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_reps):
        total = batch.run()
    call_ms = 1e3 * (time.perf_counter() - t) / args.batch_reps

    # autotuned graph
    t = time.perf_counter()
    best, best_ms = batch.autotune()
    tune_s = time.perf_counter() - t
    graph = batch.graph(best)
    graph.launch()
    total_g = graph.result()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.batch_reps):
        graph.launch()
    total_g = graph.result()
    graph_ms = 1e3 * (time.perf_counter() - t) / args.batch_reps
    counts = batch.counts.cpu().numpy().astype(np.int64)
    exact = (total_g == total == sum(ks_plain) and counts.tolist() == ks_plain and
             bool(torch.equal(batch.pairs[:total_g], pairs_plain)))
    graph.close()
    cpu_baseline = None
    if cpu is not None:
        exact = exact and [int(counts[b]) for b in cpu["instances"]] == cpu["counts"]
        cpu_baseline = {k: cpu[k] for k in ("one_core", "all_cores", "sample")}
    return {
        "workload": f"{len(insts)} independent d=2 instances, n=m log-uniform on [1e3, 2e5] "
                    f"(sum N = {regions}), alpha uniform in {{0.01, 1, 10}}, pairs mode",
        "instances": len(insts), "regions": regions, "pairs": int(total_g),
        "plain_ms": round(plain_ms, 3), "batched_call_ms": round(call_ms, 3),
        "graph_ms": round(graph_ms, 3),
        "graph_regions_per_s": round(regions / (graph_ms * 1e-3), 1),
        "plain_regions_per_s": round(regions / (plain_ms * 1e-3), 1),
        "speedup_graph_vs_plain": round(plain_ms / graph_ms, 2),
        "tuning": best.as_dict(), "autotune_replay_ms": round(best_ms, 3),
        "autotune_s": round(tune_s, 2), "exact": exact, "cpu_baseline": cpu_baseline,
    }


def bench_output_heavy(args, ddm, W, torch, np):
    """The output-bound case: d = 1, n = m = 5e6, alpha = 100, so about 5e8
    pairs (4 GB as a pair list, 2 GB as CSR).  Times the pair list and the
    CSR output, checks the per-update counts against the 1-D counting
    identity and the order of every row, and reports the written bytes per
    second against HBM peak."""
    dev = torch.device("cuda:0")
    n = m = args.heavy_n
    inst = W.uniform_instance(n, m, 1, 100.0, seed=0)
    g = [torch.from_numpy(a).to(dev) for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]
    # expected per-update counts: #{s.lo < u.hi} - #{s.hi <= u.lo} (no empty boxes here)
    s_lo = torch.sort(g[2][:, 0]).values
    s_hi = torch.sort(g[3][:, 0]).values
    want = (torch.searchsorted(s_lo, g[1][:, 0], right=False) -
            torch.searchsorted(s_hi, g[0][:, 0], right=True))
    K = int(want.sum())
    cap = K
    stream = torch.cuda.current_stream(dev)
    ws = torch.empty(ddm.workspace_bytes(n, m, 1, "pairs", cap), dtype=torch.uint8, device=dev)
    out = {"workload": f"uniform intervals d=1, n=m={n}, alpha=100, side=alpha*1e6/N",
           "pairs": K}
    for kind in ("csr", "pairs"):
        if kind == "csr":
            row_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
            ids = torch.empty(cap, dtype=torch.int32, device=dev)
            call = lambda: ddm.match_csr_into(*g, workspace=ws, row_off=row_off, sub_ids=ids,  # noqa: E731
                                              stream=stream)
            written = 4 * K + 8 * (n + 1)
        else:
            pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
            per = torch.empty(n, dtype=torch.int32, device=dev)
            call = lambda: ddm.match_into(*g, mode="pairs", workspace=ws, per_update=per,  # noqa: E731
                                          pairs=pairs, stream=stream)
            written = 8 * K + 4 * n
        k = call()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.heavy_reps):
            k = call()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / args.heavy_reps
        ddm.profile(True)
        call()
        torch.cuda.synchronize()
        phases = {p: round(v["ms"], 3) for p, v in sorted(ddm.profile_report().items())}
        ddm.profile(False)
        if kind == "csr":
            counts = row_off[1:] - row_off[:-1]
            first = torch.zeros(K, dtype=torch.bool, device=dev)
            first[row_off[:-1][counts > 0]] = True
            ordered = bool((first[1:] | (ids[1:] > ids[:-1])).all())
            ok = k == K and bool(torch.equal(counts, want)) and ordered
            del row_off, ids, first
        else:
            ordered = bool(((pairs[1:, 0] > pairs[:-1, 0]) |
                            ((pairs[1:, 0] == pairs[:-1, 0]) & (pairs[1:, 1] > pairs[:-1, 1]))).all())
            ok = k == K and bool(torch.equal(per.to(torch.int64), want)) and ordered
            del pairs, per
        alg = 8 * (n + m) + written
        out[kind] = {"ms": round(ms, 3), "pairs_per_s": round(K / (ms * 1e-3), 1),
                     "written_bytes": written, "hbm_frac": round(alg / (ms * 1e-3) / 1e9 /
                                                                  HBM_PEAK_GBS, 4),
                     "exact_counts_and_order": ok, "phases_ms": phases}
    del ws
    torch.cuda.empty_cache()
    return out


def bench_served(args, ddm, W, torch, np):
    """32 resident d=2 simulations (n = m log-uniform on [1e4, 2e6], alpha = 1,
    random-walk sigma = 0.1 * side); open-loop Poisson traces at fractions of
    the plain matcher's saturation rate, served by the plain per-request
    policy, by continuous batching and by incremental matching of resident
    states."""
    dev = torch.device("cuda:0")
    sims = W.serving_sims(32, d=2, seed=0)
    init = [[torch.from_numpy(a).to(dev) for a in (t.upd_lo, t.upd_hi, t.sub_lo, t.sub_hi)]
            for t, _, _, _ in sims]
    sizes = np.array([t.n + t.m for t, _, _, _ in sims], dtype=np.int64)
    budget = int(args.serve_budget_gib * (1 << 30))
    # the incremental policy holds every simulation's resident state
    resident = sum((ddm.resident_bytes(t.n, t.m, 2) + 255) // 256 * 256 for t, _, _, _ in sims)
    budgets = {"plain": budget, "batched": budget, "incremental": max(budget, resident)}
    policies = ("plain", "batched", "incremental")

    def serve(policy, ids, arr):
        sv = ddm.Server(budgets[policy], policy=policy, slots=args.serve_slots,
                        max_batch=args.serve_max_batch)
        for (t, side, sigma, seed), g0 in zip(sims, init):
            sv.add_sim(*[x.clone() for x in g0], side, sigma, seed)
        out = sv.run(ids, arr)
        sv.close()
        return out

    # saturation rate of the plain matcher: everything arrives at once
    R = args.serve_requests
    ids_sat, _ = W.poisson_arrivals(R, 1.0, seed=5, sims=32)
    serve("plain", ids_sat[:64], np.zeros(64))  # warm-up
    _, _, _, st = serve("plain", ids_sat, np.zeros(R))
    sat_qps = R / st["wall_s"]
    _, _, _, stb = serve("batched", ids_sat, np.zeros(R))
    sat_batched = R / stb["wall_s"]
    serve("incremental", ids_sat[:64], np.zeros(64))  # warm-up
    _, _, _, sti = serve("incremental", ids_sat, np.zeros(R))
    sat_incremental = R / sti["wall_s"]
    levels = {}
    for frac in (0.5, 0.8, 1.0, 1.2):
        ids, arr = W.poisson_arrivals(R, frac * sat_qps, seed=int(frac * 10), sims=32)
        row = {"qps": round(frac * sat_qps, 1)}
        results = {}
        for policy in policies:
            counts, steps, lat, stt = serve(policy, ids, arr)
            results[policy] = (counts, steps)
            row[policy] = {
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                "regions_per_s": round(float(sizes[ids].sum()) / stt["wall_s"], 1),
                "mean_batch": round(stt["mean_batch"], 2),
                "peak_arena_gib": round(stt["peak_arena_bytes"] / (1 << 30), 3),
            }
        row["exact"] = bool(all(np.array_equal(results["plain"][k], results[p][k])
                                for p in policies[1:] for k in (0, 1)))
        levels[f"{frac:g}x"] = row
    return {
        "workload": "32 resident d=2 simulations, n=m log-uniform on [1e4, 2e6] "
                    f"(sum N = {int(sizes.sum())}), alpha=1, random walk sigma=0.1*side, "
                    f"{R} Poisson requests per level, count mode",
        "plain_saturation_qps": round(sat_qps, 1),
        "batched_saturation_qps": round(sat_batched, 1),
        "incremental_saturation_qps": round(sat_incremental, 1),
        "saturation_regions_per_s": {
            "plain": round(float(sizes[ids_sat].sum()) / st["wall_s"], 1),
            "batched": round(float(sizes[ids_sat].sum()) / stb["wall_s"], 1),
            "incremental": round(float(sizes[ids_sat].sum()) / sti["wall_s"], 1)},
        "budget_gib": args.serve_budget_gib,
        "incremental_state_gib": round(resident / (1 << 30), 3),
        "slots": args.serve_slots, "max_batch": args.serve_max_batch, "levels": levels,
    }


def bench_resident(args, ddm, W, torch, np):
    """One resident simulation of the serving workload's kind at the headline
    scale (d = 2, n = m = 5e6, alpha = 1, random walk sigma = 0.1 side):
    closed-loop steps matched incrementally (ddm_resident_*) against the same
    steps taken by ddm_sim_step followed by the full ddm_match count, with
    equal counts at every step."""
    dev = torch.device("cuda:0")
    n = args.resident_n
    d, alpha = 2, 1.0
    inst = W.uniform_instance(n, n, d, alpha, seed=11)
    side = float(W.side_length(alpha, 2 * n))
    sigma = float(np.float32(0.1) * np.float32(side))
    seed = 0x5EED
    g = [torch.from_numpy(a).to(dev) for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]
    full = [x.clone() for x in g]
    res = ddm.Resident(*g, side, sigma, seed)
    ws = torch.empty(ddm.workspace_bytes(n, n, d, "count"), dtype=torch.uint8, device=dev)
    K, W_ = args.resident_steps, 3
    counts_res, counts_full = [], []
    step = 0
    for _ in range(W_):
        step += 1
        counts_res.append(res.step(step))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step += 1
        counts_res.append(res.step(step))
    t_res = (time.perf_counter() - t0) / K
    ddm.profile(True)
    for _ in range(3):
        step += 1
        counts_res.append(res.step(step))
    phases = {p: round(v["ms"] / 3, 4) for p, v in sorted(ddm.profile_report().items())}
    ddm.profile(False)
    for st in range(1, W_ + 1):
        ddm.sim_step(*full, side, sigma, seed, st)
        counts_full.append(ddm.match_into(*full, "count", ws))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(W_ + 1, W_ + K + 1):
        ddm.sim_step(*full, side, sigma, seed, st)
        counts_full.append(ddm.match_into(*full, "count", ws))
    t_full = (time.perf_counter() - t0) / K
    for st in range(W_ + K + 1, step + 1):
        ddm.sim_step(*full, side, sigma, seed, st)
        counts_full.append(ddm.match_into(*full, "count", ws))
    exact = counts_res == counts_full
    state = res.export()
    exact = exact and all(torch.equal(a, b) for a, b in zip(state, full))
    info = res.info()
    res.close()
    del full, state
    degraded = _resident_burst(ddm, torch, g, side, seed, ws)
    step_ms = phases.get("resident.step")
    # algorithmic bytes of the step kernels per region: read its index and
    # lower corner (4 + 4d), write both corners and the 16-byte sweep record
    # (8d + 16); indices are rewritten only in the few slabs a region left
    bytes_step = 2 * n * (4 + 4 * d + 8 * d + 16)
    return {
        "workload": f"one resident simulation d={d}, n=m={n}, alpha={alpha:g}, "
                    f"random walk sigma=0.1*side, {K} closed-loop steps",
        "ms_per_step": round(1e3 * t_res, 4),
        "full_ms_per_step": round(1e3 * t_full, 4),
        "speedup": round(t_full / t_res, 2),
        "regions_per_s": round(2 * n / t_res, 1),
        "phases_ms": phases,
        "step_kernels_gb_s": round(bytes_step / (step_ms * 1e-3) / 1e9, 1) if step_ms else None,
        "movers_last_step": info["movers"],
        "buckets": info["buckets"],
        "full_matches": info["full_matches"],
        "exact": bool(exact),
        "burst": degraded,
    }


def _resident_burst(ddm, torch, g, side, seed, ws, steps=5, warmup=2):
    """The same simulation in a lasting burst: a random walk whose sigma
    (1e4) is about 65 slab widths, so that most regions leave their slab at
    every step, the mover list and the boundary state overflow and the steps
    run in full-match mode (the walk, then the full count).  Its step time
    against sim_step + ddm_match at the same sigma, counts compared."""
    sigma = 1.0e4
    full = [x.clone() for x in g]
    res = ddm.Resident(*g, side, sigma, seed)
    got, want = [], []
    for st in range(1, warmup + 1):
        got.append(res.step(st))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(warmup + 1, warmup + steps + 1):
        got.append(res.step(st))
    t_res = (time.perf_counter() - t0) / steps
    info = res.info()
    res.close()
    for st in range(1, warmup + 1):
        ddm.sim_step(*full, side, sigma, seed, st)
        want.append(ddm.match_into(*full, "count", ws))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(warmup + 1, warmup + steps + 1):
        ddm.sim_step(*full, side, sigma, seed, st)
        want.append(ddm.match_into(*full, "count", ws))
    t_full = (time.perf_counter() - t0) / steps
    del full
    return {
        "sigma": sigma,
        "steps": steps,
        "ms_per_step": round(1e3 * t_res, 4),
        "full_ms_per_step": round(1e3 * t_full, 4),
        "full_mode": info["full_mode"],
        "full_matches": info["full_matches"],
        "rebuilds": info["rebuilds"],
        "exact": got == want,
    }


def _oracle_count(inst):
    """The oracle's count of one instance (upd_lo, upd_hi, sub_lo, sub_hi)."""
    from oracle import oracle as O
    k, _, _ = O.default().sbm(*inst, pairs=False, per_update=False)
    return k


def cpu_batched_baseline(args, W, np):
    """The oracle on a sample of the batched workload (every 8th instance), on
    one core and over a pool of threads on the host cores (the C oracle
    releases the interpreter lock and keeps no global state, so instances
    run in parallel without extra processes)."""
    from concurrent.futures import ThreadPoolExecutor
    insts = W.batched_instances(args.batch_count, d=2, seed=0)
    picked = list(range(0, len(insts), 8))
    work = [(insts[b].upd_lo, insts[b].upd_hi, insts[b].sub_lo, insts[b].sub_hi)
            for b in picked]
    regions = sum(insts[b].n + insts[b].m for b in picked)
    t = time.perf_counter()
    serial = [_oracle_count(w) for w in work]
    t_serial = time.perf_counter() - t
    procs = max(1, min(16, os.cpu_count() or 1))
    # largest instances first
    order = sorted(range(len(picked)), key=lambda i: -(insts[picked[i]].n + insts[picked[i]].m))
    with ThreadPoolExecutor(procs) as pool:
        list(pool.map(_oracle_count, [work[i] for i in order[-procs:]]))  # threads up
        t = time.perf_counter()
        pooled = list(pool.map(_oracle_count, [work[i] for i in order]))
        t_pool = time.perf_counter() - t
    assert [pooled[order.index(i)] for i in range(len(picked))] == serial
    return {
        "instances": picked, "counts": serial,
        "one_core": {"value": round(regions / t_serial, 1), "unit": "regions/s", "cores": 1,
                     "kind": "oracle"},
        "all_cores": {"value": round(regions / t_pool, 1), "unit": "regions/s", "cores": procs,
                      "kind": "oracle"},
        "sample": f"every 8th instance ({len(picked)} instances, {regions} regions), the C "
                  f"oracle per instance: {t_serial:.2f} s on one core, {t_pool:.2f} s over "
                  f"{procs} threads",
    }


def host_cpu() -> str:
    """Model name of the host CPU (Linux), for the baseline's description."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "host CPU"


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_phase: str):
    """Counter-measured HBM bytes for the dominant kernel, from a committed
    rocprofv3 summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_phase)
    except Exception:
        return None
    if not rec:
        return None
    if rec.get("source_digest") != source_digest(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--alpha", type=float, default=100.0,
                    help="overlap degree of the timed workload")
    ap.add_argument("--also-alphas", default="1,10",
                    help="comma-separated extra alphas reported under per_alpha ('' for none)")
    ap.add_argument("--mode", default="per_update", choices=["count", "per_update"])
    ap.add_argument("--workload", default="uniform",
                    choices=["uniform", "correlated", "loguniform", "clustered"],
                    help="input of the timed steps: the uniform boxes the metric is quoted on "
                         "(default), or a stress input of the same size, for kernel profiles")
    ap.add_argument("--n", type=int, default=5_000_000, help="n = m boxes per side")
    ap.add_argument("--d", type=int, default=3)
    ap.add_argument("--path", default="auto", choices=["auto", "bucketed", "global"],
                    help="implementation of the headline calls (default: the library's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-phase event timing (roofline becomes null)")
    ap.add_argument("--no-closed", action="store_true",
                    help="skip the closed-interval measurement of the headline workload")
    ap.add_argument("--no-anisotropic", action="store_true",
                    help="skip the anisotropic step (swept-axis choice against axis 0)")
    ap.add_argument("--no-skewed", action="store_true",
                    help="skip the skewed-placement (log-uniform, clustered) steps")
    ap.add_argument("--no-correlated", action="store_true",
                    help="skip the correlated d=3 stress measurement (many true matches)")
    ap.add_argument("--no-heavy", action="store_true",
                    help="skip the output-heavy (d=1, alpha=100, ~5e8 pairs) measurement")
    ap.add_argument("--heavy-n", type=int, default=5_000_000)
    ap.add_argument("--heavy-reps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched measurement")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-served", action="store_true", help="skip the serving measurement")
    ap.add_argument("--cpu-runs", type=int, default=3, help="runs of the CPU oracle baseline")
    ap.add_argument("--no-resident", action="store_true",
                    help="skip the incremental (resident simulation) measurement")
    ap.add_argument("--resident-n", type=int, default=5_000_000)
    ap.add_argument("--resident-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-budget-gib", type=float, default=4.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 256 MiB device-to-device copy (the reference kernel "
                         "for scaling HBM traffic counters) and exit")
    args = ap.parse_args()

    if args.copy_probe:
        from paper_1703_06680_amd import ddm as D
        c = D.copy_probe(256 << 20, reps=10)
        print(json.dumps({"copy_bytes": c["bytes_moved"], "ms": round(c["ms"], 4),
                          "gb_per_s": round(c["gb_per_s"], 1)}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py: this library runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "sharding across GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1703_06680_amd import ddm, workloads as W

    batched_cpu = None
    if not args.no_batched and not args.no_cpu_baseline:
        batched_cpu = cpu_batched_baseline(args, W, np)  # before the GPU is touched

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    ddm.set_path(args.path)
    n = m = args.n
    d = args.d
    t0 = time.time()
    if args.workload == "correlated" and d != 3:
        print("bench.py: the correlated workload is three-dimensional (--d 3)", file=sys.stderr)
        sys.exit(2)
    make = {"uniform": lambda: W.uniform_instance(n, m, d, args.alpha, seed=0),
            "correlated": lambda: W.correlated_d3(n, args.alpha, seed=0),
            "loguniform": lambda: W.loguniform_boxes(n, m, d, args.alpha, seed=0),
            "clustered": lambda: W.clustered_boxes(n, m, d, args.alpha, seed=0)}[args.workload]
    inst = make()
    gen_s = time.time() - t0
    g = [torch.from_numpy(a).to(dev) for a in (inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi)]
    ws = torch.empty(ddm.workspace_bytes(n, m, d, args.mode), dtype=torch.uint8, device=dev)
    per = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        return ddm.match_into(*g, mode=args.mode, workspace=ws,
                              per_update=per if args.mode == "per_update" else None, stream=stream)

    for _ in range(args.warmup):
        k = step()
    torch.cuda.synchronize()

    per_step = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        k = step()  # returns after the device result is complete
        per_step.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    head_path = ddm.last_path()
    # per-phase times from HIP events on the library's stream, in a second
    # pass of the same steps (event records are not part of the timed pass)
    phases = {}
    if not args.no_profile:
        ddm.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        phases = ddm.profile_report()
        ddm.profile(False)

    ms_per_step = 1e3 * elapsed / args.steps
    regions = n + m
    value = regions / (elapsed / args.steps)
    nonempty = regions  # every box of this workload has positive side

    roofline = None
    if phases:
        dom = max(phases, key=lambda p: phases[p]["ms"])
        avg_ms = phases[dom]["ms"] / max(phases[dom]["launches"], 1)
        alg = algorithmic_bytes(dom, n, m, d, nonempty, args.mode)
        if dom == "sort.downsweep":
            # the first down-sweep pass reads no values (4 + 8 bytes per
            # element instead of 8 + 8): average over the passes of one call
            passes = phases[dom]["launches"] / args.steps
            alg = regions * (16 * passes - 4) / passes
        if alg is not None:
            achieved = alg / (avg_ms * 1e-3) / 1e9
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": load_traffic(dom),
                        "avg_launch_ms": round(avg_ms, 4),
                        "algorithmic_bytes_per_launch": int(alg)}

    # HBM traffic of the whole step by counters (count + scatter + sweep, the
    # kernels that move the data) over their measured time
    step_traffic = None
    if phases:
        kern = ("bucket.count", "bucket.scatter", "bucket.sweep")
        tb = [load_traffic(k) for k in kern]
        if all(tb) and all(k in phases for k in kern):
            ms = sum(phases[k]["ms"] / max(phases[k]["launches"], 1) for k in kern)
            gbs = sum(tb) / (ms * 1e-3) / 1e9
            step_traffic = {"kernels": list(kern), "bytes": int(sum(tb)), "ms": round(ms, 4),
                            "gb_per_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    # the whole step against the bytes sort-based matching must move: read
    # both corners once (8d per box), write and read the sorted endpoints
    # (2 x 16 per box), write the per-update counts (4 per update)
    step_bytes = regions * (8 * d + 32) + (4 * n if args.mode == "per_update" else 8)
    step_alg = {"bytes": int(step_bytes), "ms": round(ms_per_step, 4),
                "gb_per_s": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                "frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    # achievable-bandwidth reference: a plain 256 MiB copy kernel of the library
    cref = ddm.copy_probe(256 << 20, reps=20)
    copy_ref = {"kernel": "ddm_copy_probe (16-byte loads and stores)",
                "bytes_moved": cref["bytes_moved"], "ms": round(cref["ms"], 4),
                "gb_per_s": round(cref["gb_per_s"], 1),
                "frac": round(cref["gb_per_s"] / HBM_PEAK_GBS, 4)}

    per_alpha = {}
    for a in [float(x) for x in args.also_alphas.split(",") if x.strip()]:
        extra = W.uniform_instance(n, m, d, a, seed=0)
        ge = [torch.from_numpy(x).to(dev) for x in (extra.upd_lo, extra.upd_hi, extra.sub_lo, extra.sub_hi)]
        for _ in range(args.warmup):
            ddm.match_into(*ge, mode=args.mode, workspace=ws,
                           per_update=per if args.mode == "per_update" else None, stream=stream)
        torch.cuda.synchronize()
        te = time.perf_counter()
        for _ in range(args.steps):
            ke = ddm.match_into(*ge, mode=args.mode, workspace=ws,
                                per_update=per if args.mode == "per_update" else None, stream=stream)
        torch.cuda.synchronize()
        dte = (time.perf_counter() - te) / args.steps
        per_alpha[f"{a:g}"] = {"ms_per_step": round(dte * 1e3, 4), "value": round(regions / dte, 1),
                               "matches": ke, "path": ddm.last_path()}
        del ge

    ddm.set_path("auto")  # the other measurements use the library's choice
    correlated = None
    if not args.no_correlated:
        # axis-0 lower corners uniform, axes 1 and 2 within 2 sides of axis 0:
        # the same 1-D candidates as the headline, about 45% of them true 3-D
        # matches; checked against the pairs the d = 1 match of each axis
        # bounds (K_3D <= K_1D on every axis)
        ci = W.correlated_d3(n, args.alpha, seed=0)
        gc = [torch.from_numpy(x).to(dev) for x in (ci.upd_lo, ci.upd_hi, ci.sub_lo, ci.sub_hi)]
        call = lambda: ddm.match_into(*gc, mode="per_update", workspace=ws, per_update=per,  # noqa: E731
                                      stream=stream)
        for _ in range(args.warmup):
            kc = call()
        torch.cuda.synchronize()
        tcl = time.perf_counter()
        for _ in range(args.steps):
            kc = call()
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - tcl) / args.steps
        path_c = ddm.last_path()
        ddm.profile(True)
        call()
        torch.cuda.synchronize()
        ph = {p: round(v["ms"], 4) for p, v in sorted(ddm.profile_report().items())}
        ddm.profile(False)
        consistent = kc == int(per.sum()) and kc <= min(ddm.dim_counts(*gc))
        correlated = {"workload": f"correlated boxes d=3, n=m={n}, alpha={args.alpha:g} (axes 1, 2 "
                                  f"within two sides of axis 0), per_update output",
                      "ms_per_step": round(dtc * 1e3, 4), "value": round(regions / dtc, 1),
                      "matches": kc, "path": path_c, "phases_ms": ph,
                      "counts_consistent": consistent}
        del gc
    skewed = None
    if not args.no_skewed:
        # the headline shape with skewed lower corners (six decades of
        # log-uniform placement; 16 normal clusters), same 1-D overlap degree:
        # the overfull buckets of the sampled linear map are split by their
        # exact totals; the per-update counts are checked against the pairs
        # the d = 1 match of each axis bounds
        skewed = {}
        for kind, make in (("loguniform", W.loguniform_boxes), ("clustered", W.clustered_boxes)):
            si = make(n, m, d, args.alpha, seed=0)
            gs = [torch.from_numpy(x).to(dev) for x in (si.upd_lo, si.upd_hi, si.sub_lo, si.sub_hi)]
            call = lambda: ddm.match_into(*gs, mode=args.mode, workspace=ws,  # noqa: E731
                                          per_update=per if args.mode == "per_update" else None,
                                          stream=stream)
            for _ in range(args.warmup):
                ks = call()
            torch.cuda.synchronize()
            tsk = time.perf_counter()
            for _ in range(args.steps):
                ks = call()
            torch.cuda.synchronize()
            dts = (time.perf_counter() - tsk) / args.steps
            path_s = ddm.last_path()
            ddm.profile(True)
            call()
            torch.cuda.synchronize()
            ph = {p: round(v["ms"], 4) for p, v in sorted(ddm.profile_report().items())}
            ddm.profile(False)
            ok = ks <= min(ddm.dim_counts(*gs))
            if args.mode == "per_update":
                ok = ok and ks == int(per.sum())
            skewed[kind] = {"workload": f"{si.name}: lower corners "
                                        + ("log-uniform over six decades, sides proportional"
                                           if kind == "loguniform" else
                                           "in 16 normal clusters (sigma 2e4)")
                                        + f", {args.mode} output",
                            "ms_per_step": round(dts * 1e3, 4), "value": round(regions / dts, 1),
                            "vs_uniform_step": round(dts * 1e3 / ms_per_step, 3),
                            "matches": ks, "path": path_s, "phases_ms": ph,
                            "counts_consistent": ok}
            del gs
    anisotropic = None
    if not args.no_anisotropic and d >= 2:
        # boxes 100 times longer on axis 0 than on the others, alpha = 1 on
        # the short axes: the plan sweeps another axis; the same step with
        # axis 0 forced shows what the choice saves (counts must agree)
        ai = W.anisotropic_boxes(n, m, d, 1.0, stretch=100.0, seed=0)
        ga = [torch.from_numpy(x).to(dev) for x in (ai.upd_lo, ai.upd_hi, ai.sub_lo, ai.sub_hi)]
        anisotropic = {"workload": f"{ai.name}: sides 100 l on axis 0, l = 1e6/N on the others, "
                                   f"{args.mode} output"}
        for label, axis in (("chosen_axis", None), ("axis_0", 0)):
            ddm.set_sweep_axis(axis)
            call = lambda: ddm.match_into(*ga, mode=args.mode, workspace=ws,  # noqa: E731
                                          per_update=per if args.mode == "per_update" else None,
                                          stream=stream)
            for _ in range(args.warmup):
                ka = call()
            torch.cuda.synchronize()
            tan = time.perf_counter()
            for _ in range(args.steps):
                ka = call()
            torch.cuda.synchronize()
            dta = (time.perf_counter() - tan) / args.steps
            anisotropic[label] = {"ms_per_step": round(dta * 1e3, 4),
                                  "value": round(regions / dta, 1), "matches": ka,
                                  "path": ddm.last_path()}
        ddm.set_sweep_axis(None)
        anisotropic["counts_equal"] = (anisotropic["chosen_axis"]["matches"]
                                       == anisotropic["axis_0"]["matches"])
        anisotropic["speedup"] = round(anisotropic["axis_0"]["ms_per_step"]
                                       / anisotropic["chosen_axis"]["ms_per_step"], 2)
        del ga
    closed = None
    if not args.no_closed:
        # the headline inputs as closed boxes [lo, hi]; checked against the
        # half-open match of [lo, nextafter(hi)), which is the same set
        def closed_step():
            return ddm.match_into(*g, mode=args.mode, workspace=ws,
                                  per_update=per if args.mode == "per_update" else None,
                                  stream=stream, closed=True)
        for _ in range(args.warmup):
            closed_step()
        torch.cuda.synchronize()
        tcl = time.perf_counter()
        for _ in range(args.steps):
            kc = closed_step()
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - tcl) / args.steps
        path_c = ddm.last_path()
        per_c = per.clone() if args.mode == "per_update" else None
        inf = torch.tensor(float("inf"), device=dev)
        up = [torch.nextafter(t, inf) for t in (g[1], g[3])]
        kh = ddm.match(g[0], up[0], g[2], up[1], mode="count")
        same = kh == kc
        if args.mode == "per_update":
            _, per_h = ddm.match(g[0], up[0], g[2], up[1], mode="per_update")
            same = same and bool(torch.equal(per_h, per_c))
        del up
        closed = {"ms_per_step": round(dtc * 1e3, 4), "value": round(regions / dtc, 1),
                  "matches": kc, "path": path_c, "equal_to_half_open_next_float": same}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        o = O.default()
        times = []
        for _ in range(args.cpu_runs):
            tc = time.perf_counter()
            k_cpu, per_cpu, _ = o.sbm(inst.upd_lo, inst.upd_hi, inst.sub_lo, inst.sub_hi,
                                      pairs=False, per_update=args.mode == "per_update")
            times.append(time.perf_counter() - tc)
        dt = statistics.median(times)
        k_chk = step()  # the extra alphas reused the output buffer
        assert k_cpu == k_chk == k, f"GPU count {k} != oracle {k_cpu}"
        if args.mode == "per_update":
            assert np.array_equal(per_cpu, per.cpu().numpy()), "per-update counts differ"
        cpu = {"value": round(regions / dt, 1), "unit": "regions/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload (n = m = {n}, d = {d}, alpha = {args.alpha:g}), "
                         f"{len(times)} serial runs of the C oracle on one core of a {host_cpu()} "
                         f"({os.cpu_count()} logical CPUs visible): median {dt:.2f} s, min "
                         f"{min(times):.2f} s; checked equal to the GPU result"}

    heavy = None if args.no_heavy else bench_output_heavy(args, ddm, W, torch, np)
    batched = None if args.no_batched else bench_batched(args, ddm, W, torch, np, batched_cpu)
    served = None if args.no_served else bench_served(args, ddm, W, torch, np)
    resident = None if args.no_resident else bench_resident(args, ddm, W, torch, np)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "regions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"uniform boxes d={d}, n=m={n} (N={regions}), alpha={args.alpha:g}, "
                                f"side=alpha*1e6/N on [0,1e6)^{d}, {args.mode} output"
                                if args.workload == "uniform" else
                                f"{inst.name} ({args.workload} stress input), {args.mode} output"),
                   "d": d, "n": n, "m": m, "alpha": args.alpha, "mode": args.mode,
                   "parallelism": "single GPU"},
        "matches": k,
        "path": head_path,
        "step_ms_p50": round(1e3 * statistics.median(per_step), 4),
        "step_ms_p99": round(1e3 * float(np.percentile(per_step, 99)), 4),
        "roofline": roofline,
        "step_counter_traffic": step_traffic,
        "step_algorithmic": step_alg,
        "copy_reference": copy_ref,
        "cpu_baseline": cpu,
        "phases_ms_per_step": {p: round(v["ms"] / args.steps, 4) for p, v in sorted(phases.items())},
        "per_alpha": per_alpha,
        "closed": closed,
        "correlated": correlated,
        "skewed": skewed,
        "anisotropic": anisotropic,
        "served_p50_ms": served["levels"]["1x"]["batched"]["p50_ms"] if served else None,
        "served_p99_ms": served["levels"]["1x"]["batched"]["p99_ms"] if served else None,
        "served_incremental_p50_ms":
            served["levels"]["1x"]["incremental"]["p50_ms"] if served else None,
        "served_incremental_p99_ms":
            served["levels"]["1x"]["incremental"]["p99_ms"] if served else None,
        "output_heavy": heavy,
        "batched": batched,
        "served": served,
        "resident": resident,
        "input_generation_s": round(gen_s, 2),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
