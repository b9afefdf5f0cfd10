"""Throughput benchmark of exact (p,q)-biclique counting on one MI355X.

One step = every query of the workload counted once on the resident graph
(the whole device path: candidate pass, planning, rows, enumeration).
Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.

Default workload: Chung-Lu power-law graph, |U| = 100k, |V| = 50k, 2M edges,
exponent 2.1 on both sides, max degree 5k, degree-ordered relabelling.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X dense int8 matrix-core peak (no structured sparsity): 5.0 POP/s.
MFMA_I8_PEAK = 5.0e15
# The leaf pair sums are the int8 product R R^T of 0/1 rows: one 64-bit word
# of both rows is 64 multiply-adds, 128 operations.
OPS_PER_WORD_PAIR = 2 * 64
# One word-intersection (the unit of the enumeration): an 8-byte row word read
# and ANDed with the parent's word, then counted: 2 v_and_b32 + 2
# v_bcnt_u32_b32 on 32-bit lanes.
BYTES_PER_WORD = 8
INT_OPS_PER_WORD = 4
# Nominal figures of MI355X (256 CUs at 2.4 GHz): LDS 128 B/clk/CU, integer
# VALU 64 lanes/clk/CU, HBM3E 8 TB/s.  The LDS and VALU denominators of the
# roofline are measured live by the microbenchmarks of libbc_peaks.so.
LDS_NOMINAL = 256 * 2.4e9 * 128
VALU_INT_NOMINAL = 256 * 2.4e9 * 64
HBM_PEAK = 8.0e12

# HBM bytes of one k_enumerate launch for (4,4) on the power-law 2M-edge graph,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE (each scaled by the same counter on a
# 1 GiB device copy), valid only for the kernel source they were taken on.
TRAFFIC_KERNEL_SHA256_PREFIX = "d93191dce7218f63"
TRAFFIC_WORKLOAD = "power_law_2m"
TRAFFIC_BYTES_Q44 = (923703.125 * 2.0 + 1033914.8125 * 1.0) * 1024

WORKLOADS = {
    "power_law_2m": ("power_law_2m", [(4, 4), (4, 6), (6, 4), (5, 5)]),
    # 1M x 400k, 20M edges: the timed step; (6,6) runs in root ranges under
    # --c3
    "power_law_20m": ("power_law_20m", [(3, 3), (4, 4), (5, 5)]),
    "small_er": ("small_er", [(3, 3)]),
}


def parse_queries(s):
    out = []
    for part in s.split(";"):
        if part.strip():
            p, q = part.split(",")
            out.append((int(p), int(q)))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="power_law_2m", choices=sorted(WORKLOADS))
    ap.add_argument("--queries", default=None, help="e.g. '4,4;4,6'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rank-lo", type=int, default=61000,
                    help="first U degree rank of the roots the oracle and the device both count at (4,4)")
    ap.add_argument("--cpu-rank-hi", type=int, default=63000)
    ap.add_argument("--sweep", default="6:150,7:20,8:20",
                    help="p=q queries counted once after the timed steps, each under a device time limit "
                         "in seconds ('k:seconds,...'; empty = none)")
    ap.add_argument("--batch", action="store_true",
                    help="batched workload: 4096 Chung-Lu graphs with mixed (p,q), one batched launch "
                         "set against one launch set per graph")
    ap.add_argument("--serve", action="store_true",
                    help="served workload: 64 resident graphs, Poisson query streams")
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--c3", action="store_true",
                    help="20M-edge workload: (6,6) over cost-balanced root ranges, and a bitmap-width sweep")
    ap.add_argument("--ranges", type=int, default=16)
    ap.add_argument("--range-workload", default="power_law_20m", choices=sorted(WORKLOADS),
                    help="--c3: the graph whose roots are split into ranges")
    ap.add_argument("--range-query", default="6,6", help="--c3: the (p,q) counted over root ranges")
    ap.add_argument("--range-anchor", default="V", choices=("U", "V"), help="--c3: the side the ranges are of")
    ap.add_argument("--range-calibrate", default="",
                    help="--c3: a cheaper (p,q) timed over 4x as many fine ranges; the ranges are then cut at equal "
                         "sums of its times instead of equal sums of d^2")
    ap.add_argument("--range-budget-s", type=float, default=0.0,
                    help="--c3: start no range after this many seconds (0 = no limit); the rest is reported not run")
    ap.add_argument("--range-cap-s", type=float, default=15.0)
    ap.add_argument("--bitmap-sweep", default="64,128,256,512,1024,0")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave the batched-vs-per-query measurement out of the default line")
    ap.add_argument("--timeout-ms", type=int, default=0, help="device time limit per count (0 = none)")
    ap.add_argument("--serve-queries", type=int, default=200, help="queries per arrival rate")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000")
    ap.add_argument("--serve-graphs", type=int, default=64)
    ap.add_argument("--serve-batch", type=int, default=8, help="most queries per served batch")
    ap.add_argument("--ablation", action="store_true",
                    help="Section VII ablations (HTB, NB comparator, pure DFS, Border, |N2| order, BCPar)")
    ap.add_argument("--ablation-cap-s", type=float, default=30.0, help="device time limit per ablation count")
    ap.add_argument("--border-iters", type=int, default=1024, help="Border swap steps per side (ablation)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the count is additive over root ranges, so each GPU could take its own ranges)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_07858_amd import bc, graphgen as gg

    if args.batch:
        return run_batch(args)
    if args.serve:
        return run_serve(args)
    if args.c3:
        return run_c3(args)
    if args.ablation:
        return run_ablation(args)
    gen_name, default_q = WORKLOADS[args.workload]
    queries = parse_queries(args.queries) if args.queries else default_q
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 18   # float32 elements
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.copy_calibration_mib} MiB read, {args.copy_calibration_mib} MiB written")
        del src, dst
    peaks = measure_peaks(log)
    t0 = time.time()
    g = getattr(gg, gen_name)()
    log(f"[bench] generated {args.workload}: {g.manifest['edges']} edges in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    G = bc.build_graph(g, stream=stream)
    log(f"[bench] bc_build {time.time() - t0:.2f}s")

    # instrumented pass: algorithmic word operations per query (not timed)
    algo = {}
    for p, q in queries:
        c, st = bc.bc_count(G, p, q, with_stats=True, instrument=True, stream=stream)
        algo[(p, q)] = (c, st)
        cyc = {k: st[k] for k in ("cyc_setup", "cyc_compact", "cyc_pair", "cyc_filter")}
        tot = sum(cyc.values()) or 1
        log(f"[bench] ({p},{q}) count={c} anchor={st['anchor']} tasks={st['tasks']} "
            f"pair_words={st['pair_ops']} filter_words={st['filter_ops']} ms_enum={st['ms_enumerate']:.1f} "
            f"ms_cand={st['ms_candidates']:.1f} ms_rows={st['ms_rows']:.1f} ms_plan={st['ms_plan']:.1f} "
            f"cycle share " + " ".join(f"{k[4:]}={v / tot:.2f}" for k, v in cyc.items()) +
            f" pack={st['cyc_pack'] / tot:.2f} task_cycles={tot:.4g}"
            f" pairs={st['pairs']} lane_use={st['pairs'] / max(1, st['pair_slots']):.2f} "
            f"words/pair={st['pair_ops'] / max(1, st['pairs']):.2f} wave makespan={st['ms_wave_makespan']:.1f}ms "
            f"spread={st['ms_wave_spread']:.1f}ms")

    # load balance of the deep queries: per-wave makespan and spread with the
    # runtime split off (the default) and on (heavy tasks queue their level-3 nodes)
    balance = []
    for p, q in queries:
        if min(p, q) < 5:
            continue
        for rows in (0xFFFFFFFF, 256):
            c, st = bc.bc_count(G, p, q, with_stats=True, instrument=True, stream=stream, split_rows=rows)
            assert c == algo[(p, q)][0]
            balance.append({"p": p, "q": q, "split_rows": None if rows == 0xFFFFFFFF else rows,
                            "ms_enumerate": st["ms_enumerate"], "wave_makespan_ms": st["ms_wave_makespan"],
                            "wave_spread_ms": st["ms_wave_spread"]})
            log(f"[bench] ({p},{q}) split_rows={balance[-1]['split_rows']}: enum {st['ms_enumerate']:.1f} ms, "
                f"wave makespan {st['ms_wave_makespan']:.1f} ms, spread {st['ms_wave_spread']:.1f} ms")

    def step():
        out = []
        for p, q in queries:
            c, st = bc.bc_count(G, p, q, with_stats=True, stream=stream)
            out.append((p, q, c, st))
        return out

    for _ in range(args.warmup):
        step()
        log("[bench] warmup step done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        log(f"[bench] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000 / args.steps

    for r in results:
        for (p, q, c, st) in r:
            assert c == algo[(p, q)][0], "count changed between runs"
    total_count = sum(c for (_, _, c, _) in results[0])
    roots = sum(st["roots"] for (_, _, _, st) in results[0])
    value = total_count / (ms_per_step / 1000)

    # roofline of the enumeration kernel (the dominant one): algorithmic
    # word-intersections (leaf pairs and child filters, from the instrumented
    # pass) x 8 bytes per launch, over its mean launch time (HIP events on the
    # stream it runs on), against the LDS bandwidth measured on this device
    enum_ms = {}
    for r in results:
        for (p, q, c, st) in r:
            enum_ms.setdefault((p, q), []).append(st["ms_enumerate"])
    words = sum(algo[k][1]["pair_ops"] + algo[k][1]["filter_ops"] for k in algo)
    launch_ms = sum(sum(v) / len(v) for v in enum_ms.values())
    n_launch = len(enum_ms)
    sec = launch_ms / 1000
    achieved = BYTES_PER_WORD * words / sec if sec > 0 else 0.0
    int_ops = INT_OPS_PER_WORD * words / sec if sec > 0 else 0.0
    mfma_ops = sum(OPS_PER_WORD_PAIR * algo[k][1]["pair_ops"] for k in algo) / sec if sec > 0 else 0.0
    traffic = traffic_bytes(args.workload, queries)
    per_query = []
    for (p, q) in queries:
        c, st = algo[(p, q)]
        ms = sum(enum_ms[(p, q)]) / len(enum_ms[(p, q)])
        tot = [st2 for r in results for (pp, qq, _, st2) in r if (pp, qq) == (p, q)]
        mt = sum(s["ms_total"] for s in tot) / len(tot)
        w = st["pair_ops"] + st["filter_ops"]
        per_query.append({"p": p, "q": q, "count": str(c), "ms_total": round(mt, 3), "ms_enumerate": round(ms, 3),
                          "bicliques_per_s": c / (mt / 1000), "root_vertices_per_s": st["roots"] / (mt / 1000),
                          "anchor": "UV"[st["anchor"]], "tasks": st["tasks"],
                          "word_intersections": w,
                          "wave_makespan_ms": st["ms_wave_makespan"], "wave_spread_ms": st["ms_wave_spread"],
                          "lds_frac": (BYTES_PER_WORD * w / (ms / 1000)) / peaks["lds_bytes_per_s"] if ms > 0 else 0.0,
                          "leaf_pairs_per_s": st["pairs"] / (ms / 1000) if ms > 0 else 0.0})

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, G, stream, args.cpu_rank_lo, args.cpu_rank_hi, log)
    sweep = capped_sweep(G, stream, args.sweep, log) if args.sweep else []
    batch = batch_measure(args.batch_n, 1, args.timeout_ms, log) if args.batch_n and not args.no_batch else None

    line = {
        "metric": "bicliques counted/sec",
        "value": value,
        "unit": "bicliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128",
        "data": "synthetic",
        "config": {"workload": args.workload, "queries": [f"({p},{q})" for p, q in queries],
                   "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges, "seed": g.manifest.get("seed"),
                   "sha256": g.manifest["sha256"]},
        "root_vertices_per_s": roots / (ms_per_step / 1000),
        "per_query": per_query,
        "roofline": {"bound": "lds", "kernel": "k_enumerate", "achieved": achieved / 1e9,
                     "peak": peaks["lds_bytes_per_s"] / 1e9, "unit": "GB/s",
                     "frac": achieved / peaks["lds_bytes_per_s"], "traffic": traffic,
                     "traffic_unit": f"HBM bytes per k_enumerate launch of (4,4) on {TRAFFIC_WORKLOAD}",
                     "algorithmic_bytes_per_launch": BYTES_PER_WORD * words / n_launch,
                     "launch_ms_mean": launch_ms / n_launch, "launches_per_step": n_launch,
                     "unit_of_work": "word-intersection: 8 B row word AND parent word + popcount",
                     "peak_source": "measured: bc_peak_lds (libbc_peaks.so) on this device",
                     "peak_nominal": LDS_NOMINAL / 1e9, "frac_of_nominal": achieved / LDS_NOMINAL,
                     "valu_int": {"achieved_tops": int_ops / 1e12, "peak_tops": peaks["valu_int_ops_per_s"] / 1e12,
                                  "frac": int_ops / peaks["valu_int_ops_per_s"],
                                  "peak_nominal_tops": VALU_INT_NOMINAL / 1e12},
                     "hbm": {"achieved_gb_s": (traffic / ((sum(enum_ms[(4, 4)]) / len(enum_ms[(4, 4)])) / 1000) / 1e9)
                             if traffic and (4, 4) in enum_ms else None,
                             "peak_gb_s": HBM_PEAK / 1e9},
                     "mfma_equivalent": {"achieved_tops": mfma_ops / 1e12, "peak_tops": MFMA_I8_PEAK / 1e12,
                                         "frac": mfma_ops / MFMA_I8_PEAK, "dtype": "int8",
                                         "note": "leaf pair sums as the int8 product of bit-expanded rows"}},
        "cpu_baseline": cpu,
        "capped_sweep": sweep,
        "load_balance": balance,
        "batched_vs_per_query_speedup": batch["batched_vs_per_query_speedup"] if batch else None,
        "batch": batch,
    }
    print(json.dumps(line), flush=True)


def measure_peaks(log):
    """LDS bandwidth and integer VALU rate of this device (libbc_peaks.so)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2403_07858_amd", "libbc_peaks.so"))
    for f in (lib.bc_peak_lds, lib.bc_peak_valu_int):
        f.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        f.restype = ctypes.c_int
    rate, ms = ctypes.c_double(), ctypes.c_double()
    out = {}
    for name, f, iters in (("lds_bytes_per_s", lib.bc_peak_lds, 2048), ("valu_int_ops_per_s", lib.bc_peak_valu_int, 8192)):
        best = 0.0
        for _ in range(3):
            rc = f(iters, ctypes.byref(rate), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"{name} microbenchmark failed with hip error {rc}")
            best = max(best, rate.value)
        out[name] = best
        log(f"[bench] peak {name} = {best:.4g} ({ms.value:.2f} ms launch)")
    return out


def traffic_bytes(workload, queries):
    """Measured HBM bytes of the (4,4) enumeration launch on the 2M-edge graph,
    or None when the kernel source changed since the counters were taken, or
    the workload is another graph, or (4,4) is not run."""
    import hashlib
    src = os.path.join(ROOT, "paper_2403_07858_amd", "csrc", "bc_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if (not sha.startswith(TRAFFIC_KERNEL_SHA256_PREFIX) or workload != TRAFFIC_WORKLOAD
            or (4, 4) not in queries):
        return None
    return TRAFFIC_BYTES_Q44


def cpu_baseline(g, G, stream, rank_lo, rank_hi, log, pq=(4, 4)):
    """The oracle (all host cores) and the device (bc_count_roots) on the
    identical work: the roots with degree rank in [rank_lo, rank_hi) on the
    U side, query (4,4).  Both counts must be equal."""
    import oracle
    from paper_2403_07858_amd import bc

    p, q = pq
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    want = oracle.count(g, p, q, order_key=oracle.ORDER_DEGREE, rank_lo=rank_lo, rank_hi=rank_hi, threads=threads)
    dt = time.perf_counter() - t0
    got, st = bc.bc_count_roots(G, p, q, bc.BC_ANCHOR_U, rank_lo, rank_hi, with_stats=True, stream=stream)
    ms = []
    for _ in range(5):
        c, st = bc.bc_count_roots(G, p, q, bc.BC_ANCHOR_U, rank_lo, rank_hi, with_stats=True, stream=stream)
        assert c == got
        ms.append(st["ms_total"])
    gpu_s = sorted(ms)[len(ms) // 2] / 1000
    log(f"[bench] cpu oracle: ({p},{q}) ranks [{rank_lo},{rank_hi}) count {want} in {dt:.1f}s; "
        f"device {got} in {gpu_s * 1e3:.2f} ms")
    if got != want:
        raise RuntimeError(f"device and oracle differ on the CPU-baseline sample: {got} vs {want}")
    return {"value": want / dt if dt > 0 else 0.0, "unit": "bicliques/s", "cores": threads, "kind": "oracle",
            "sample": f"({p},{q}) anchor U, roots of degree rank [{rank_lo},{rank_hi}) "
                      f"({rank_hi - rank_lo} roots), count {want}",
            "seconds": dt, "device_seconds_same_sample": gpu_s,
            "device_value_same_sample": want / gpu_s if gpu_s > 0 else 0.0,
            "device_speedup_same_sample": dt / gpu_s if gpu_s > 0 else 0.0}


def capped_sweep(G, stream, spec, log):
    """p = q queries beyond the timed step, each counted once under a device
    time limit; a query that hits its limit is reported as capped (no count,
    nothing extrapolated)."""
    from paper_2403_07858_amd import bc

    out = []
    for part in spec.split(","):
        pq, cap = part.split(":")
        k = int(pq)
        cap_s = float(cap)
        log(f"[bench] sweep ({k},{k}) under a {cap_s:.0f} s device time limit")
        t0 = time.perf_counter()
        try:
            c, st = bc.bc_count(G, k, k, with_stats=True, stream=stream, timeout_ms=int(cap_s * 1000))
            dt = time.perf_counter() - t0
            out.append({"p": k, "q": k, "status": "done", "count": str(c), "seconds": dt,
                        "bicliques_per_s": c / dt, "anchor": "UV"[st["anchor"]], "cap_s": cap_s})
        except bc.BCError as e:
            dt = time.perf_counter() - t0
            out.append({"p": k, "q": k, "status": "capped" if e.status == bc.BC_E_TIMEOUT else bc.bc_status_string(e.status),
                        "count": None, "seconds": dt, "cap_s": cap_s})
        log(f"[bench] sweep ({k},{k}): {out[-1]['status']} after {dt:.1f}s")
    return out


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _batch_item(i):
    from paper_2403_07858_amd import graphgen as gg
    return gg.batch_graph(i)


def _served_item(i):
    from paper_2403_07858_amd import graphgen as gg
    return gg.served_graph(i)


def _generate(fn, n, workers):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(fn, range(n), chunksize=8))


def _workers():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return 8


def batch_measure(n, steps, timeout_ms, log):
    """The batched workload: n Chung-Lu graphs, each with its own (p,q), counted
    by one batched launch set (schedule from the autotuner) and by one
    bc_count per graph on the same stream; counts compared item by item."""
    import torch

    from paper_2403_07858_amd import bc

    t0 = time.time()
    items = _generate(_batch_item, n, _workers())
    log(f"[batch] generated {len(items)} graphs, {sum(g.n_edges for g, _, _ in items)} edges "
        f"in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    graphs = [bc.build_graph(g, stream=stream) for g, _, _ in items]
    ps = [p for _, p, _ in items]
    qs = [q for _, _, q in items]
    log(f"[batch] built {len(graphs)} graphs in {time.time() - t0:.1f}s")
    opt = {"stream": stream, "timeout_ms": timeout_ms}
    # the batched path's autotuner picks the schedule on a sample of the items
    t0 = time.perf_counter()
    tuned = bc.bc_tune_batch(graphs, ps, qs, stream=stream, timeout_ms=timeout_ms)
    t_tune = time.perf_counter() - t0
    log(f"[batch] autotuner chose {tuned} in {t_tune * 1e3:.0f} ms")
    opt.update(tuned)
    vals, st, agg = bc.bc_count_batch(graphs, ps, qs, with_stats=True, **opt)
    log(f"[batch] warm pass: ms_cand={agg['ms_candidates']:.1f} ms_plan={agg['ms_plan']:.1f} "
        f"ms_rows={agg['ms_rows']:.1f} ms_enum={agg['ms_enumerate']:.1f} ms_total={agg['ms_total']:.1f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        vals, st = bc.bc_count_batch(graphs, ps, qs, **opt)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    log(f"[batch] batched: {t_batch * 1e3:.1f} ms per pass")
    # the default schedule, for the autotuner's gain
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vals_d, st_d = bc.bc_count_batch(graphs, ps, qs, stream=stream, timeout_ms=timeout_ms)
    torch.cuda.synchronize()
    t_default = time.perf_counter() - t0
    single_vals, single_st = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for G, p, q in zip(graphs, ps, qs):
        try:
            single_vals.append(bc.bc_count(G, p, q, **opt))
            single_st.append(bc.BC_OK)
        except bc.BCError as e:
            single_vals.append(None)
            single_st.append(e.status)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    log(f"[batch] one launch set per graph: {t_single * 1e3:.1f} ms; default schedule batched: "
        f"{t_default * 1e3:.1f} ms")
    # load balance of the batched launch: per-wave makespan and spread with the
    # runtime split off and on (instrumented passes, counts compared)
    balance = []
    for rows in (0xFFFFFFFF, 256):
        o2 = dict(opt)
        o2["split_rows"] = rows
        v2, s2, a2 = bc.bc_count_batch(graphs, ps, qs, with_stats=True, instrument=True, **o2)
        balance.append({"split_rows": None if rows == 0xFFFFFFFF else rows, "ms_enumerate": a2["ms_enumerate"],
                        "wave_makespan_ms": a2["ms_wave_makespan"], "wave_spread_ms": a2["ms_wave_spread"],
                        "same_counts": v2 == vals and s2 == st})
        log(f"[batch] split_rows={balance[-1]['split_rows']}: enum {a2['ms_enumerate']:.1f} ms, wave makespan "
            f"{a2['ms_wave_makespan']:.1f} ms, spread {a2['ms_wave_spread']:.1f} ms")
    mismatch = sum(1 for a, b, s, s2 in zip(vals, single_vals, st, single_st)
                   if s == bc.BC_OK and s2 == bc.BC_OK and a != b)
    mismatch += sum(1 for a, b, s, s2 in zip(vals, vals_d, st, st_d) if s == bc.BC_OK and s2 == bc.BC_OK and a != b)
    total = sum(v for v, s in zip(vals, st) if s == bc.BC_OK)
    return {"graphs": len(graphs), "edges": sum(g.n_edges for g, _, _ in items), "pq": "U{2..6}^2",
            "queries_per_s": len(graphs) / t_batch, "bicliques_per_s": total / t_batch,
            "ms_batched": t_batch * 1e3, "ms_per_query_launches": t_single * 1e3,
            "batched_vs_per_query_speedup": t_single / t_batch,
            "ms_batched_default_schedule": t_default * 1e3, "autotuner_gain": t_default / t_batch,
            "schedule": tuned, "autotune_ms": t_tune * 1e3, "load_balance": balance,
            "completed": sum(1 for s in st if s == bc.BC_OK),
            "statuses": {bc.bc_status_string(s): st.count(s) for s in set(st)},
            "mismatches": mismatch}


def run_batch(args):
    """Batched counting as a bench line of its own."""
    r = batch_measure(args.batch_n, args.steps, args.timeout_ms, _log)
    line = {
        "metric": "batched count queries/sec",
        "value": r["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": r["ms_batched"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128",
        "data": "synthetic",
        "config": {"workload": "batch_chung_lu", "graphs": r["graphs"], "edges": r["edges"], "pq": r["pq"],
                   "timeout_ms": args.timeout_ms},
        "batch": r,
    }
    print(json.dumps(line), flush=True)


def equal_weight_cuts(weights, n_ranges):
    """Cut points 0 = c_0 <= c_1 <= ... <= c_n = len(weights) that split the
    sequence into n_ranges consecutive ranges of about equal weight."""
    import numpy as np
    cum = np.cumsum(np.asarray(weights, dtype=np.float64))
    n = len(cum)
    if n == 0:
        return [0] * (n_ranges + 1)
    return [0] + [int(np.searchsorted(cum, cum[-1] * i / n_ranges)) for i in range(1, n_ranges)] + [n]


def merge_cuts(fine, times, n_ranges):
    """Merges the consecutive ranges [fine[k], fine[k + 1]) with measured times
    into at most n_ranges ranges of about equal total time; returns strictly
    increasing cut points from fine[0] to fine[-1], each one of fine's."""
    import numpy as np
    ct = np.cumsum(np.asarray(times, dtype=np.float64))
    nf = len(times)
    idx = [int(np.searchsorted(ct, ct[-1] * i / n_ranges)) for i in range(1, n_ranges)] if nf else []
    return sorted({fine[0], fine[-1]} | {fine[min(k + 1, nf)] for k in idx})


def run_c3(args):
    """A deep query over cost-balanced root ranges of one anchor, each under a
    device time limit (completed and capped ranges reported, nothing
    extrapolated): by default (6,6) on the 20M-edge power-law graph with 16
    ranges of V; then (with --bitmap-sweep) the bitmap width swept at (4,4):
    roots with more neighbours than W bits take the HTB path."""
    import numpy as np
    import torch

    from paper_2403_07858_amd import bc, graphgen as gg

    log = _log
    t0 = time.time()
    gen_name, _ = WORKLOADS[args.range_workload]
    g = getattr(gg, gen_name)()
    log(f"[c3] generated {g.n_edges} edges in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    G = bc.build_graph(g, stream=stream)
    (rp, rq), = parse_queries(args.range_query)
    side = bc.BC_ANCHOR_U if args.range_anchor == "U" else bc.BC_ANCHOR_V
    # ranges of equal sum over roots of d^2 (a per-root cost proxy), by rank
    deg = g.degrees_u() if side == bc.BC_ANCHOR_U else g.degrees_v()
    dv = np.sort(deg.astype(np.float64))   # ranks follow ascending degree
    n_side = len(dv)
    cuts = equal_weight_cuts(dv * dv, args.ranges)
    calib = []
    if args.range_calibrate:
        # time a cheaper query over 4x finer ranges of equal d^2 sums, then
        # merge them into ranges of equal time: its per-root cost follows the
        # deep query's far more closely than d^2 does
        (cp, cq), = parse_queries(args.range_calibrate)
        fine = equal_weight_cuts(dv * dv, 4 * args.ranges)
        bc.bc_count_roots(G, 2, 2, side, 0, n_side, stream=stream)   # first-launch costs off the clock
        for lo, hi in zip(fine, fine[1:]):
            _, st = bc.bc_count_roots(G, cp, cq, side, lo, hi, with_stats=True, stream=stream)
            calib.append({"rank_lo": lo, "rank_hi": hi, "ms_enumerate": st["ms_enumerate"]})
        times = [c["ms_enumerate"] for c in calib]
        log(f"[c3] calibration ({cp},{cq}) over {len(times)} ranges: {sum(times):.1f} ms of enumeration")
        cuts = merge_cuts(fine, times, args.ranges)
    ranges = []
    t_start = time.perf_counter()
    for lo, hi in zip(cuts, cuts[1:]):
        if args.range_budget_s and time.perf_counter() - t_start > args.range_budget_s:
            ranges.append({"rank_lo": lo, "rank_hi": hi, "status": "not run", "count": None, "seconds": 0.0})
            continue
        t1 = time.perf_counter()
        try:
            c, st = bc.bc_count_roots(G, rp, rq, side, lo, hi, with_stats=True, stream=stream,
                                      timeout_ms=int(args.range_cap_s * 1000))
            ranges.append({"rank_lo": lo, "rank_hi": hi, "status": "done", "count": str(c),
                           "seconds": time.perf_counter() - t1})
        except bc.BCError as e:
            ranges.append({"rank_lo": lo, "rank_hi": hi, "status": "capped" if e.status == bc.BC_E_TIMEOUT
                           else bc.bc_status_string(e.status), "count": None, "seconds": time.perf_counter() - t1})
        log(f"[c3] ({rp},{rq}) {args.range_anchor} ranks [{lo},{hi}): {ranges[-1]['status']} "
            f"{ranges[-1]['seconds']:.1f}s")
    done = [r for r in ranges if r["status"] == "done"]
    done_count = sum(int(r["count"]) for r in done)
    done_s = sum(r["seconds"] for r in done)
    sweep = []
    base = None
    cap_ms = int(args.range_cap_s * 1000)
    for w in [int(x) for x in args.bitmap_sweep.split(",") if x.strip()]:
        try:
            c, st = bc.bc_count(G, 4, 4, anchor=bc.BC_ANCHOR_U, bitmap_bits=w, with_stats=True, stream=stream,
                                timeout_ms=cap_ms)
        except bc.BCError as e:
            if e.status != bc.BC_E_TIMEOUT:
                raise
            sweep.append({"bitmap_bits": w, "status": "capped", "count": None, "ms_total": None,
                          "ms_enumerate": None})
            log(f"[c3] (4,4) bitmap_bits {w}: capped at {args.range_cap_s:.0f} s")
            continue
        ms = []
        for _ in range(2):
            c2, st2 = bc.bc_count(G, 4, 4, anchor=bc.BC_ANCHOR_U, bitmap_bits=w, with_stats=True, stream=stream)
            assert c2 == c
            ms.append(st2["ms_total"])
        base = c if base is None else base
        assert c == base, "the bitmap width changed a count"
        sweep.append({"bitmap_bits": w, "status": "done", "count": str(c), "ms_total": min(ms),
                      "ms_enumerate": st2["ms_enumerate"]})
        log(f"[c3] (4,4) bitmap_bits {w}: {min(ms):.1f} ms")
    line = {
        "metric": "bicliques counted/sec", "value": done_count / done_s if done_s else 0.0, "unit": "bicliques/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": done_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": args.range_workload,
                   "query": f"({rp},{rq}) on {args.range_anchor} root ranges"
                            + ("; (4,4) bitmap sweep" if sweep else ""),
                   "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges, "sha256": g.manifest["sha256"],
                   "range_cap_s": args.range_cap_s},
        "calibration": calib,
        "ranges": ranges, "ranges_done": len(done),
        "ranges_capped": sum(1 for r in ranges if r["status"] == "capped"),
        "ranges_not_run": sum(1 for r in ranges if r["status"] == "not run"),
        "bitmap_sweep_44": sweep,
    }
    print(json.dumps(line), flush=True)


def run_ablation(args):
    """Section VII's ablations, each against the default build (degree order,
    local bitmaps, hybrid DFS-BFS), with every count checked against the
    default's; a count past the device time limit is reported as capped,
    not extrapolated.
    - Whole 2M-edge graph: Border order (Algorithm 2) and the |N_2^q| order
      key (Definition 2) on the local-bitmap path, with the HTB 1-block
      counts of both orders (Table III's measure).
    - A band of roots (ranks [0.61 n, 0.63 n) of the anchor side): the HTB
      global-set path, the binary-search (NB) comparator on sorted id
      lists, pure DFS on the global sets (NH), Border + HTB.
    - BCPar (Algorithm 3) on a 200k-edge graph of the same shape: the groups'
      counts add up to the whole count; groups, largest closure, time.
    - Per-vertex counts against the plain count of the same query."""
    import torch

    from paper_2403_07858_amd import bc, graphgen as gg

    log = _log
    gen_name, _ = WORKLOADS[args.workload]
    queries = parse_queries(args.queries) if args.queries else [(4, 4), (4, 6), (6, 4)]
    g = getattr(gg, gen_name)()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cap_ms = int(args.ablation_cap_s * 1000)
    graphs = {"degree": bc.build_graph(g, stream=stream)}
    t0 = time.perf_counter()
    graphs["border"] = bc.build_graph(g, stream=stream, order_key=bc.BC_ORDER_BORDER, border_iters=args.border_iters)
    border_build_s = time.perf_counter() - t0
    log(f"[ablation] Border build ({args.border_iters} swap steps per side): {border_build_s:.1f} s")
    t0 = time.perf_counter()
    graphs["two_hop"] = bc.build_graph(g, stream=stream, order_key=bc.BC_ORDER_TWO_HOP)
    two_hop_build_s = time.perf_counter() - t0
    log(f"[ablation] |N2| order build: {two_hop_build_s:.1f} s")
    htb = {}
    for name in ("degree", "border"):
        for side in (0, 1):
            words, ones = bc.bc_htb_stats(graphs[name], side)
            htb[f"{name}_side{side}"] = {"words": words, "one_blocks": ones}
        log(f"[ablation] {name} order HTB: {htb[name + '_side0']} (U rows) {htb[name + '_side1']} (V rows)")

    def timed(fn, **opt):
        try:
            c, st = fn(with_stats=True, stream=stream, timeout_ms=cap_ms, **opt)
            return c, st["ms_total"], st["ms_enumerate"]
        except bc.BCError as e:
            if e.status != bc.BC_E_TIMEOUT:
                raise
            return None, None, None

    rows = []
    for p, q in queries:
        want, st = bc.bc_count(graphs["degree"], p, q, with_stats=True, stream=stream)
        anchor = st["anchor"]
        for name, gname in (("default", "degree"), ("border", "border"), ("two_hop_order", "two_hop")):
            c, ms, me = timed(lambda **o: bc.bc_count(graphs[gname], p, q, **o))
            assert c is None or c == want, (name, p, q)
            rows.append({"scope": "graph", "variant": name, "p": p, "q": q, "status": "done" if c is not None
                         else "capped", "count": None if c is None else str(c), "ms_total": ms, "ms_enumerate": me})
            log(f"[ablation] ({p},{q}) whole graph {name}: total {ms} ms, enumeration {me} ms")
        n = g.n_u if anchor == 0 else g.n_v
        lo, hi = int(0.61 * n), int(0.63 * n)
        sub = sub_b = None
        for name, gname, opt in (("default", "degree", {}), ("htb", "degree", {"sets": bc.BC_SETS_HTB}),
                                 ("nb_sorted", "degree", {"sets": bc.BC_SETS_SORTED}),
                                 ("htb_pure_dfs", "degree", {"sets": bc.BC_SETS_HTB, "pure_dfs": True}),
                                 ("border", "border", {}), ("border_htb", "border", {"sets": bc.BC_SETS_HTB})):
            c, ms, me = timed(lambda **o: bc.bc_count_roots(graphs[gname], p, q, anchor, lo, hi, **o), **opt)
            if gname == "degree" and name == "default":
                sub = c
            # Border relabels the side, so its band holds other roots: compared among Border runs
            if name == "border":
                sub_b = c
            ref = sub_b if gname == "border" else sub
            if c is not None and ref is not None:
                assert c == ref, (name, p, q)
            rows.append({"scope": f"ranks [{lo},{hi}) of {'UV'[anchor]}", "variant": name, "p": p, "q": q,
                         "status": "done" if c is not None else "capped", "count": None if c is None else str(c),
                         "ms_total": ms, "ms_enumerate": me})
            log(f"[ablation] ({p},{q}) ranks [{lo},{hi}) {name}: total {ms} ms, enumeration {me} ms")
    # per-vertex counts (the output set of Algorithm 1 as membership counts):
    # their time against the plain count of the same query
    Gd = graphs["degree"]
    for p, q, side in ((2, 3, bc.BC_ANCHOR_U), (2, 4, bc.BC_ANCHOR_U), (3, 2, bc.BC_ANCHOR_V)):
        c, st = bc.bc_count(Gd, p, q, with_stats=True, stream=stream, anchor=side)
        t0 = time.perf_counter()
        try:
            pv = bc.bc_count_per_vertex(Gd, p, q, side, stream=stream, timeout_ms=cap_ms)
            ms = (time.perf_counter() - t0) * 1e3
            assert sum(pv) == (p if side == bc.BC_ANCHOR_U else q) * c
            status = "done"
        except bc.BCError as e:
            if e.status != bc.BC_E_TIMEOUT:
                raise
            ms, status = None, "capped"
        rows.append({"scope": "graph", "variant": f"per-vertex counts, side {'UV'[side]}", "p": p, "q": q,
                     "status": status, "count": str(c), "ms_total": ms, "count_ms_total": st["ms_total"]})
        log(f"[ablation] ({p},{q}) per-vertex side {'UV'[side]}: {status} {ms} ms (count alone {st['ms_total']:.1f} ms)")
    # BCPar on a smaller graph of the same shape
    gs = gg.chung_lu_bipartite(10_000, 5_000, 200_000, 2.1, 2.1, 1000, 1000, seed=5)
    Gs = bc.build_graph(gs, stream=stream)
    for p, q, side in ((4, 4, bc.BC_ANCHOR_U), (4, 4, bc.BC_ANCHOR_V)):
        c, st = bc.bc_count(Gs, p, q, with_stats=True, stream=stream, anchor=side)
        t0 = time.perf_counter()
        pv = bc.bc_count_per_vertex(Gs, p, q, side, stream=stream)
        ms = (time.perf_counter() - t0) * 1e3
        assert sum(pv) == 4 * c
        rows.append({"scope": "graph 10k x 5k, 200k edges", "variant": f"per-vertex counts, side {'UV'[side]}",
                     "p": p, "q": q, "status": "done", "count": str(c), "ms_total": ms,
                     "count_ms_total": st["ms_total"]})
        log(f"[ablation] ({p},{q}) 200k-edge graph per-vertex side {'UV'[side]}: {ms:.1f} ms "
            f"(count alone {st['ms_total']:.1f} ms)")
    for p, q in queries:
        want, st = bc.bc_count(Gs, p, q, with_stats=True, stream=stream)
        anchor = st["anchor"]
        whole_ms = st["ms_total"]
        for budget_kib in (256, 1024):
            t0 = time.perf_counter()
            part, n = bc.bc_partition(Gs, p, q, anchor, budget_kib << 10)
            plan_s = time.perf_counter() - t0
            t0 = time.perf_counter()
            tot, biggest = 0, 0
            for k in range(n):
                c, edges = bc.bc_count_partition(Gs, p, q, anchor, part, k, stream=stream)
                tot += c
                biggest = max(biggest, edges)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            assert tot == want, ("bcpar", p, q)
            rows.append({"scope": "bcpar graph 10k x 5k, 200k edges", "variant": f"bcpar {budget_kib} KiB",
                         "p": p, "q": q, "status": "done", "count": str(tot), "groups": n,
                         "largest_closure_edges": biggest, "partition_s": plan_s, "groups_wall_ms": wall * 1e3,
                         "whole_count_ms": whole_ms})
            log(f"[ablation] ({p},{q}) bcpar {budget_kib} KiB: {n} groups (largest closure {biggest} of "
                f"{gs.n_edges} edges), partition {plan_s:.2f} s, groups {wall * 1e3:.1f} ms, whole {whole_ms:.1f} ms")
    line = {
        "metric": "bicliques counted/sec", "value": None, "unit": "bicliques/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "u128", "data": "synthetic",
        "config": {"workload": args.workload, "queries": [f"({p},{q})" for p, q in queries],
                   "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges, "sha256": g.manifest["sha256"],
                   "cap_s": args.ablation_cap_s, "border_iters": args.border_iters},
        "build_s": {"border": border_build_s, "two_hop": two_hop_build_s},
        "htb": htb, "ablation": rows,
    }
    print(json.dumps(line), flush=True)


def run_serve(args):
    """Served counting: resident graphs, Poisson arrivals at several rates;
    each result is checked against the same query counted alone."""
    import torch

    from paper_2403_07858_amd import bc, graphgen as gg

    t0 = time.time()
    raw = _generate(_served_item, args.serve_graphs, _workers())
    _log(f"[serve] generated {len(raw)} graphs, {sum(g.n_edges for g in raw)} edges in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    graphs = [bc.build_graph(g) for g in raw]
    deadline_ms = args.timeout_ms or 2000
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    per_rate = []
    solo_cache = {}
    for ri, rate in enumerate(rates):
        t_arr, gid, p, q = gg.poisson_arrivals(rate, args.serve_queries, len(graphs), 2, 8, seed=6000 + int(rate))
        srv = bc.Server(max_inflight=3, max_batch=args.serve_batch, batch_timeout_ms=deadline_ms)
        for G in graphs:
            srv.add_graph(G)
        start = srv.now_ns()
        tickets = []
        for k in range(len(t_arr)):
            due = start + int(t_arr[k] * 1e9)
            while srv.now_ns() < due:
                time.sleep(max(0.0, min(0.001, (due - srv.now_ns()) / 1e9)))
            try:
                tickets.append((srv.submit(int(gid[k]), int(p[k]), int(q[k]), deadline_ns=srv.now_ns() +
                                           deadline_ms * 1_000_000), k))
            except bc.BCError as e:
                tickets.append((None, k))
        res = {}
        for t, k in tickets:
            res[k] = srv.poll(t) if t is not None else (bc.BC_E_REJECTED, None, {})
        wall = (srv.now_ns() - start) / 1e9
        stats = srv.stats()
        srv.close()
        # completed results equal the same query counted alone (first 40 checked
        # here; the test suite checks every result of its mixes)
        mism, checked = 0, 0
        for k, (s, v, _) in res.items():
            if s != bc.BC_OK or checked >= 40:
                continue
            checked += 1
            key = (int(gid[k]), int(p[k]), int(q[k]))
            if key not in solo_cache:
                solo_cache[key] = bc.bc_count(graphs[key[0]], key[1], key[2])
            if solo_cache[key] != v:
                mism += 1
        stats.update({"rate": rate, "wall_s": wall, "mismatches_vs_alone": mism})
        per_rate.append(stats)
        _log(f"[serve] rate {rate}: completed {stats['completed']} timed_out {stats['timed_out']} "
             f"p50 {stats['p50_ms']:.1f} ms p99 {stats['p99_ms']:.1f} ms qps {stats['completed'] / wall:.1f} "
             f"mean batch {stats['mean_batch']:.1f} overlap {stats['max_overlap']} mismatches {mism}")
    best = max(per_rate, key=lambda s: s["completed"] / s["wall_s"])
    line = {
        "metric": "served count queries/sec",
        "value": best["completed"] / best["wall_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": len(rates),
        "warmup": 0,
        "ms_per_step": best["wall_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128",
        "data": "synthetic",
        "config": {"workload": "served_chung_lu", "graphs": len(graphs), "edges": sum(g.n_edges for g in raw),
                   "pq": "U{2..8}^2", "queries_per_rate": args.serve_queries, "deadline_ms": deadline_ms,
                   "max_batch": args.serve_batch},
        "per_rate": per_rate,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
