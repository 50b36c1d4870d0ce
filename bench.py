"""Benchmark: census arcs/s of the 16-class directed triad census on one MI355X.

Default workload: R-MAT (0.57, 0.19, 0.19, 0.05), n = 2^20, ~2^24 arcs,
reciprocity 0.20, relabelled; the graph is built once and stays resident in
HBM; a step is one full census (all bucket kernels, the 128-byte read-back and
the 003 finalisation).  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload rmat|citation|er]
                  [--cpu-seconds S] [--no-cpu-baseline]
  python bench.py --workload batch [--batch-count 4096]   # batched mode vs per-graph launches
  python bench.py --workload serve [--rate 2000] [--duration 10] [--pool 64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Library sources that neither build nor launch a census kernel: the serving
# loop (its scheduler and executor) and the autotuner's search.
NOT_CENSUS_SOURCES = ("tc_serve.cpp", "tc_sched.cpp", "tc_sched.h", "tc_tune.cpp")


def census_source_hash() -> str:
    """sha256 (first 16 hex digits) of the code the census kernels are built
    and launched from (every library source but NOT_CENSUS_SOURCES, in name
    order, comments and whitespace removed): a counter summary taken on other
    code no longer describes the kernels."""
    import re
    d = os.path.join(ROOT, "paper_1603_02655_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")) and name not in NOT_CENSUS_SOURCES:
            with open(os.path.join(d, name)) as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(name.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str, kernel: str):
    """HBM bytes per launch of `kernel` (FETCH_SIZE and WRITE_SIZE, scaled by
    the copy calibration) from profiles/hbm_traffic_<workload>.md, when that
    table was taken on the current sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_key}.md")
    if not os.path.exists(path):
        return None
    src = census_source_hash()
    with open(path) as f:
        for line in f:
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 7 and cells[0] == kernel and cells[1] == src:
                try:
                    return float(cells[6])
                except ValueError:
                    return None
    return None


def measured_valu_busy(workload_key: str, kernel: str):
    """VALU busy fraction of `kernel` (SQ_ACTIVE_INST_VALU x 4 cycles over the
    1024 SIMDs' active cycles) from profiles/sq_counters_<workload>.md, when
    that table was taken on the current sources; None otherwise."""
    import re
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload_key}.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    m = re.search(r"Source hash `([0-9a-f]+)`", text)
    if not m or m.group(1) != census_source_hash():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == kernel:
            try:
                return float(cells[3])
            except ValueError:
                return None
    return None


def workload(name: str):
    from paper_1603_02655_amd import synth
    if name == "rmat":
        return synth.config_rmat_2p20()
    if name == "citation":
        return synth.config_citation()
    if name == "er":
        return synth.config_er_small()
    raise SystemExit(f"unknown workload {name}")


def _gen_batch(i):
    from paper_1603_02655_amd import synth
    return synth.batch_graph(i)


def _gen_serve(i):
    from paper_1603_02655_amd import synth
    return synth.serving_graph(i)


def generate_pool(fn, count):
    """Graphs 0..count-1 of a pool, drawn in spawned worker processes (which
    never touch the GPU; spawned, not forked, since this process may already
    hold the HIP runtime)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, range(count), chunksize=max(1, count // (4 * workers))))


def kernel_key(name: str, tri: bool, tuning: dict, chunk: int = 512) -> str:
    """The name rocprofv3 gives the template instance of a census kernel that
    runs with this tuning (namespace and arguments dropped), as used in the
    tables under profiles/; `chunk`: the graph's records per hub task
    (`tri_chunk` or `hub_chunk` of its info), which picks the hub kernel's
    LDS instance."""
    t = "true" if tri else "false"
    if name == "k_census_hub":
        return f"k_census_hub<{t}, {tuning['hub_tile']}u, {256 if chunk <= 256 else 512}u>"
    if name == "k_census_wave":
        return f"k_census_wave<{t}, {tuning['wave_tile']}>"
    if name == "k_census_group":
        return f"k_census_group<{t}, {tuning['group_size']}, {tuning['group_tile']}>"
    if name == "k_census_lane":
        return f"k_census_lane<{t}>"
    return name


def census_bytes(info: dict, n: int, tri: bool) -> float:
    """Algorithmic bytes of one whole census of a graph by the per-kernel
    models (see the roofline comment in main): merge modes 4 B per merged entry
    + 8 B per record, hub mode 4 B per streamed and staged entry + 8 B per
    record, and on the forward-list path the totals pass's 16 B per neighbour
    entry + 16 B per row."""
    if tri:
        cost, recs = info["tri_bucket_cost"], info["tri_bucket_edges"]
        stream, staged = info["tri_stream"], info["tri_staged"]
        p = info["asym_dyads"] + info["mutual_dyads"]
        base = 16.0 * 2 * p + 16.0 * n
    else:
        cost, recs = info["bucket_cost"], info["bucket_dyads"]
        stream, staged = info["hub_stream"], info["hub_staged"]
        base = 0.0
    return (base + 4.0 * sum(cost[:3]) + 8.0 * sum(recs[:3]) + 4.0 * (stream + staged) + 8.0 * recs[3])


def time_shards(ctx, g, full_counts, shard_counts, reps: int = 5) -> dict:
    """Per-shard census times on this one GPU: the work one GPU of a G-GPU run
    would do, without the graph's broadcast and the final 128-byte sum.  Each
    shard's wall time is the median of `reps` calls; the shards' counts must
    add up to the full census."""
    out = {}
    for G in shard_counts:
        ms, total = [], np.zeros(16, np.uint64)
        for k in range(G):
            t = []
            for _ in range(reps):
                ts = time.perf_counter()
                p = ctx.census_shard(g, k, G)
                t.append(1000.0 * (time.perf_counter() - ts))
            ms.append(float(np.median(t)))
            with np.errstate(over="ignore"):
                total = total + p.astype(np.uint64)
        if total[1:].tolist() != [int(x) for x in full_counts[1:]]:
            raise SystemExit(f"the {G} shard censuses do not add up to the full census")
        out[str(G)] = {"max_ms": max(ms), "min_ms": min(ms), "sum_ms": sum(ms)}
    return out


def apply_tuning(ctx, args):
    """--tuning key=value overrides on top of the library's default tuning."""
    if args.tuning:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})


def golden_counts(kind: str, pool):
    """The oracle's stored census of every pool graph (tests/golden/, written by
    the CPU oracle), after checking each graph's arc hash; None when the pool is
    not the stored one (another size)."""
    from tests.golden import make_goldens as goldens
    try:
        gold = goldens.load(kind)
    except OSError:
        return None
    if len(gold) < len(pool):
        return None
    out = []
    for g, rec in zip(pool, gold):
        if (g.n, g.m, goldens.arc_hash(g.src, g.dst)) != (rec["n"], rec["m"], rec["hash"]):
            return None
        out.append(rec["counts"])
    return out


def run_batch(args, autotune_sample: int) -> dict:
    """Batched census of the pool of uneven R-MAT graphs: one persistent launch
    (captured HIP graph) against one launch sequence per graph, on the same
    resident graphs; every graph's counts against the oracle's stored census."""
    from paper_1603_02655_amd import tc
    log(f"[bench] generating {args.batch_count} batch graphs")
    pool = generate_pool(_gen_batch, args.batch_count)
    gold = golden_counts("batch", pool)
    ctx = tc.Context(0)
    apply_tuning(ctx, args)
    log("[bench] building the batch pool")
    hs = [ctx.build_graph(g.n, g.src, g.dst) for g in pool]
    arcs = sum(int(h.info["arcs_kept"]) for h in hs)
    rng = np.random.default_rng(1)
    tune_s = 0.0
    if autotune_sample > 0:
        sample = [hs[i] for i in rng.choice(len(hs), size=min(autotune_sample, len(hs)), replace=False)]
        t = time.perf_counter()
        tuning = ctx.autotune(sample)
        tune_s = time.perf_counter() - t
        for h in hs:
            ctx.rebucket(h)
        log(f"[bench] autotuned in {tune_s:.1f}s: {tuning}")
    else:
        tuning = ctx.get_tuning()
    each = ctx.census_each(hs)
    tc.device_synchronize(0)
    t = time.perf_counter()
    each = ctx.census_each(hs)
    tc.device_synchronize(0)
    each_s = time.perf_counter() - t
    for _ in range(args.warmup):
        out = ctx.census_batch(hs)
    assert out.tolist() == each.tolist(), "batched and per-graph counts differ"
    ctx.reset_kernel_stats()
    ctx.set_timing(True)
    tc.device_synchronize(0)
    steps = max(1, args.batch_steps)
    t = time.perf_counter()
    for _ in range(steps):
        out = ctx.census_batch(hs)
    tc.device_synchronize(0)
    el = time.perf_counter() - t
    ks = ctx.kernel_stats()
    ctx.set_timing(False)
    assert out.tolist() == each.tolist()
    equal_oracle = None if gold is None else out.tolist() == gold
    step_s = el / steps
    launch_ms = ks["batch_ms"] / max(1, ks["batch_launches"])
    tri = bool(ctx.get_tuning()["tri"])
    bytes_alg = sum(census_bytes(h.info, h.n, tri and h.info["fwd_entries"] > 0) for h in hs)
    achieved = bytes_alg / (launch_ms / 1000.0) / 1e9 if launch_ms > 0 else 0.0
    res = {
        "workload": f"batch of {len(hs)} R-MAT digraphs, n log-uniform [50, 20000], mean out-degree U[3,30], "
                    "reciprocity 0.10",
        "graphs": len(hs), "arcs": arcs, "steps": steps, "ms_per_batch": 1000 * step_s,
        "arcs_per_s": arcs / step_s, "graphs_per_s": len(hs) / step_s,
        "per_graph_launches": {"graphs_per_s": len(hs) / each_s, "arcs_per_s": arcs / each_s, "ms": 1000 * each_s},
        "speedup_vs_per_graph": each_s / step_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "kernel": "k_census_batch_hub + k_census_batch",
                     "kernel_ms": launch_ms, "bytes_per_launch": bytes_alg},
        "tuning": tuning, "autotune_s": tune_s,
        "path": "forward-list triangles" if tri else "dyad intersections",
        "results_equal_oracle": equal_oracle,
    }
    for h in hs:
        h.release()
    ctx.close()
    if equal_oracle is False:
        raise SystemExit("batched counts differ from the oracle's stored census")
    return res


def bench_batch(args):
    res = run_batch(args, args.autotune_sample)
    line = {
        "metric": "census arcs/sec (batched)", "value": res["arcs_per_s"], "unit": "arcs/s", "n_gpus": 1,
        "steps": res["steps"], "warmup": args.warmup, "ms_per_step": res["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
        "config": {"workload": res["workload"], "graphs": res["graphs"], "arcs": res["arcs"],
                   "tuning": res["tuning"]},
    }
    line.update({k: v for k, v in res.items() if k not in ("workload", "graphs", "arcs", "tuning", "steps")})
    print(json.dumps(line), flush=True)


def run_serve(args) -> dict:
    """Served census: Poisson arrivals of requests for graphs of a resident
    pool; every result against the same graph's census run alone and, for the
    stored pool, against the oracle's census."""
    from paper_1603_02655_amd import tc
    log(f"[bench] generating serving pool of {args.pool}")
    pool = generate_pool(_gen_serve, args.pool)
    gold = golden_counts("serve", pool)
    ctx = tc.Context(0)
    apply_tuning(ctx, args)
    hs = [ctx.build_graph(g.n, g.src, g.dst) for g in pool]
    arcs = np.array([int(h.info["arcs_kept"]) for h in hs])
    alone = ctx.census_each(hs)
    equal_oracle = None if gold is None else alone.tolist() == gold
    # per-graph launch baseline over a random request sequence
    rng = np.random.default_rng(5)
    seq = rng.integers(0, len(hs), 200)
    t = time.perf_counter()
    for i in seq:
        ctx.census(hs[i])
    base_s = time.perf_counter() - t
    base_rps = len(seq) / base_s
    from paper_1603_02655_amd import synth
    runs = []
    all_ok = True
    plan = [(float(x), 0.0) for x in str(args.rate).split(",")]
    if args.cold_frac > 0:
        plan.append((float(args.cold_rate), float(args.cold_frac)))
    for rate, cold_frac in plan:
        arrivals = synth.poisson_arrivals(rate, args.duration + 1.0, synth.rng_for(5, int(rate)))
        picks = rng.integers(0, len(hs), arrivals.size)
        # cold requests carry the graph's arcs and are built inside their round
        cold = rng.random(arrivals.size) < cold_frac
        log(f"[bench] serving {arrivals.size} requests at {rate:.0f}/s for {args.duration + 1:.0f}s "
            f"({cold.sum()} cold)")
        ctx.serve_reset_stats()
        sub_q = []
        lock = threading.Lock()
        t0 = time.perf_counter()

        def submitter():
            for k in range(arrivals.size):
                delay = arrivals[k] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                if cold[k]:
                    g = pool[picks[k]]
                    tk = ctx.submit_arcs(g.n, g.src, g.dst)
                else:
                    tk = ctx.submit(hs[picks[k]])
                with lock:
                    sub_q.append((tk, k, time.perf_counter()))

        th = threading.Thread(target=submitter)
        th.start()
        outstanding = []
        results = {}
        lat = {}
        while True:
            with lock:
                outstanding.extend(sub_q)
                sub_q.clear()
            keep = []
            for n_polled, (tk, k, ts) in enumerate(outstanding):
                if n_polled >= 512:
                    keep.append((tk, k, ts))
                    continue
                r = ctx.poll(tk)
                if r is None:
                    keep.append((tk, k, ts))
                else:
                    results[k] = r
                    lat[k] = (time.perf_counter() - ts) * 1000.0
            outstanding = keep
            if not th.is_alive() and not outstanding and not sub_q:
                break
            time.sleep(0.0002)
        th.join()
        total_s = time.perf_counter() - t0
        st = ctx.serve_stats()
        ok = all(results[i].tolist() == alone[picks[i]].tolist() for i in range(arrivals.size))
        all_ok &= ok
        meas = [i for i in range(arrivals.size) if arrivals[i] >= 1.0]
        ml = np.array([lat[i] for i in meas]) if meas else np.zeros(1)
        mc = np.array([lat[i] for i in meas if cold[i]])
        mw = np.array([lat[i] for i in meas if not cold[i]])
        runs.append({"rate": rate, "cold_fraction": cold_frac, "cold_requests": int(cold.sum()),
                     "requests": int(arrivals.size), "measured": len(meas),
                     "wall_s": total_s, "completed_per_s": arrivals.size / total_s,
                     "offered_arcs_per_s": float(arcs[picks].mean() * rate),
                     "achieved_arcs_per_s": float(arcs[picks].sum() / total_s),
                     "p50_ms": float(np.percentile(ml, 50)), "p99_ms": float(np.percentile(ml, 99)),
                     "rounds": st["rounds"], "mean_admission_ms": st["mean_admission_ms"],
                     "cold_p50_ms": float(np.percentile(mc, 50)) if mc.size else None,
                     "cold_p99_ms": float(np.percentile(mc, 99)) if mc.size else None,
                     "resident_p50_ms": float(np.percentile(mw, 50)) if mc.size and mw.size else None,
                     "resident_p99_ms": float(np.percentile(mw, 99)) if mc.size and mw.size else None,
                     "results_equal_alone": ok})
        log(f"[bench] rate {rate}: {runs[-1]}")
    warm = [r for r in runs if r["cold_fraction"] == 0.0] or runs
    res = {
        "workload": f"serving pool of {len(hs)} graphs (even ER, odd R-MAT r=0.10), n log-uniform "
                    "[1e3, 1e6], mean out-degree U[4,32]; Poisson arrivals",
        "duration_s": args.duration, "pool_arcs": int(arcs.sum()), "runs": runs,
        "per_graph_launches_rps": base_rps,
        # at the first (nominal) rate: latency; at the last resident-only rate:
        # what the loop sustains
        "requests_per_s": runs[0]["completed_per_s"], "p50_ms": runs[0]["p50_ms"], "p99_ms": runs[0]["p99_ms"],
        "capacity_rps": warm[-1]["completed_per_s"], "capacity_arcs_per_s": warm[-1]["achieved_arcs_per_s"],
        "results_equal_alone": all_ok, "results_equal_oracle": equal_oracle,
    }
    for h in hs:
        h.release()
    ctx.close()
    if not all_ok or equal_oracle is False:
        raise SystemExit("served counts differ from the census alone or from the oracle's stored census")
    return res


def bench_serve(args):
    res = run_serve(args)
    head = res["runs"][0]
    line = {
        "metric": "served census throughput + p50/p99 latency", "value": head["completed_per_s"],
        "unit": "requests/s", "n_gpus": 1, "steps": head["requests"], "warmup": 0,
        "ms_per_step": head["p50_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64", "data": "synthetic",
        "config": {"workload": res["workload"], "duration_s": res["duration_s"], "pool_arcs": res["pool_arcs"]},
    }
    line.update({k: v for k, v in res.items() if k not in ("workload", "duration_s", "pool_arcs")})
    print(json.dumps(line), flush=True)


def copy_calibration(nbytes: int):
    """Three device-to-device copies of nbytes through the HIP runtime the
    library uses (a plain copy kernel of known size, read by the profiler to
    scale the FETCH_SIZE / WRITE_SIZE counters)."""
    import ctypes
    from paper_1603_02655_amd import tc
    h = tc.hip_runtime()
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    if h.hipMalloc(ctypes.byref(a), nbytes) != 0 or h.hipMalloc(ctypes.byref(b), nbytes) != 0:
        raise MemoryError("hipMalloc failed")
    h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
    h.hipMemset(a, 1, nbytes)
    for _ in range(3):
        if h.hipMemcpy(b, a, nbytes, 3) != 0:   # device to device
            raise RuntimeError("hipMemcpy failed")
    tc.device_synchronize(0)
    h.hipFree(a)
    h.hipFree(b)


def copy_bandwidth(nbytes: int = 1 << 30) -> float:
    """Device-to-device copy rate in GB/s (bytes read + bytes written over the
    time of three copies after one untimed), the practical HBM rate the
    census kernels' byte rates are also compared with."""
    import ctypes
    from paper_1603_02655_amd import tc
    h = tc.hip_runtime()
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    if h.hipMalloc(ctypes.byref(a), nbytes) != 0 or h.hipMalloc(ctypes.byref(b), nbytes) != 0:
        raise MemoryError("hipMalloc failed")
    try:
        h.hipMemset.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t]
        h.hipMemset(a, 1, nbytes)
        if h.hipMemcpy(b, a, nbytes, 3) != 0:
            raise RuntimeError("hipMemcpy failed")
        tc.device_synchronize(0)
        t = time.perf_counter()
        for _ in range(3):
            if h.hipMemcpy(b, a, nbytes, 3) != 0:   # device to device
                raise RuntimeError("hipMemcpy failed")
        tc.device_synchronize(0)
        el = time.perf_counter() - t
    finally:
        h.hipFree(a)
        h.hipFree(b)
    return 3 * 2 * nbytes / el / 1e9


def cpu_tuned(g0, m_kept: int) -> dict:
    """The multicore CPU census of the same method (libtc_cpu.so: per-dyad
    merge with typed counts, task queues, local census per thread) on the whole
    graph, timed on the host cores; context only, never the measured value."""
    from paper_1603_02655_amd import cpu_census
    threads = min(16, os.cpu_count() or 1)
    _, secs = cpu_census.census(g0.n, g0.src, g0.dst, threads=threads)
    return {"value": m_kept / secs if secs > 0 else None, "unit": "arcs/s", "cores": threads,
            "kind": "tuned multicore CPU census (per-dyad merge, task queues, local census per thread)",
            "census_s": secs}


def oracle_work(g0):
    """Per-vertex work of the oracle's census (entries it visits): for vertex x
    its own row once, and for every neighbour p > x the row of x twice and the
    row of p three times.  Used only to extrapolate the timed CPU sample."""
    n = g0.n
    s = g0.src.astype(np.int64)
    d = g0.dst.astype(np.int64)
    keep = s != d
    lo = np.minimum(s[keep], d[keep])
    hi = np.maximum(s[keep], d[keep])
    pk = np.unique(lo * n + hi)
    a, b = pk // n, pk % n
    deg = (np.bincount(a, minlength=n) + np.bincount(b, minlength=n)).astype(np.float64)
    return deg + np.bincount(a, weights=2.0 * deg[a] + 3.0 * deg[b], minlength=n)


def cpu_baseline(g0, m_kept: int, seconds: float):
    """The oracle (test infrastructure) on a bounded sample: the vertices are
    cut into chunks of about equal oracle work, threads take chunks in a random
    order (each chunk one call of the oracle's range census) until the time
    budget is spent, and the work rate is extrapolated to the whole graph."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    work = oracle_work(g0)
    total_work = float(work.sum())
    cum = np.concatenate([[0.0], np.cumsum(work)])
    cuts = np.unique(np.searchsorted(cum, np.linspace(0.0, total_work, 4097), side="left").clip(0, g0.n))
    chunks = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    order = np.random.default_rng(0).permutation(len(chunks))
    og = oracle.OracleGraph(g0.n, g0.src, g0.dst)
    lock = threading.Lock()
    state = {"next": 0, "work": 0.0, "chunks": 0}
    deadline = time.perf_counter() + seconds

    def worker():
        while time.perf_counter() < deadline:
            with lock:
                if state["next"] >= len(order):
                    return
                u0, u1 = chunks[order[state["next"]]]
                state["next"] += 1
            og.census_range(u0, u1)
            with lock:
                state["work"] += cum[u1] - cum[u0]
                state["chunks"] += 1

    t0 = time.perf_counter()
    ts = [threading.Thread(target=worker) for _ in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    el = time.perf_counter() - t0
    og.close()
    rate = state["work"] / el
    full_s = total_work / rate
    return {"value": m_kept / full_s, "unit": "arcs/s", "cores": threads, "kind": "oracle",
            "sample": (f"{state['chunks']} of {len(chunks)} vertex-range chunks taken in random order, "
                       f"{state['work']:.3g} of {total_work:.3g} oracle work units (row entries visited) in "
                       f"{el:.1f} s; rate extrapolated to the whole graph ({full_s:.0f} s)")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--rate", default="2000,8000",
                    help="comma-separated arrival rates (requests/s); the last one measures capacity")
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--cold-frac", type=float, default=0.05,
                    help="fraction of cold requests (arcs submitted, built in their round) in one more serving run")
    ap.add_argument("--cold-rate", type=float, default=1000.0, help="arrival rate of the run with cold requests")
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=10, help="timed batched launches")
    ap.add_argument("--autotune-sample", type=int, default=0,
                    help="graphs the batched bench autotunes on (0: keep the default tuning)")
    ap.add_argument("--single-only", action="store_true",
                    help="default workload: leave out the batched and served legs")
    ap.add_argument("--tuning", default="", help="comma-separated key=value overrides, e.g. t_hub=256")
    ap.add_argument("--shards", action="store_true",
                    help="also time the census shards for 2, 4 and 8 GPUs' worth of work (extra launches)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run 3 device-to-device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the census of one graph is "
              "a single-device job here.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)

    from paper_1603_02655_amd import tc

    log(f"[bench] generating workload {args.workload}")
    g0 = workload(args.workload)
    ctx = tc.Context(0)
    apply_tuning(ctx, args)
    log(f"[bench] building n={g0.n} m={g0.m}")
    t = time.perf_counter()
    g = ctx.build_graph(g0.n, g0.src, g0.dst)
    tc.device_synchronize(0)
    build_s = time.perf_counter() - t
    info = g.info
    log(f"[bench] built in {build_s:.2f}s info={info}")
    for _ in range(args.warmup):
        ctx.census(g)
    ctx.reset_kernel_stats()
    ctx.set_timing(True)
    tc.device_synchronize(0)
    t0 = time.perf_counter()
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        counts = ctx.census(g)                      # returns after the counts are on the host
        step_ms.append(1000.0 * (time.perf_counter() - ts))
    tc.device_synchronize(0)
    el = time.perf_counter() - t0
    ctx.set_timing(False)
    ks = ctx.kernel_stats()
    ms_step = 1000.0 * el / args.steps
    m_kept = int(info["arcs_kept"])
    value = m_kept / (el / args.steps)

    # roofline of the dominant kernel, bytes per launch by the algorithmic
    # model of each kernel:
    #   merge modes (lane / wave / group): 4 B per entry of the two rows merged
    #     (|N(u)|+|N(v)| per dyad, |N+(x)|+|N+(y)| per forward-list edge) and
    #     8 B per task (the (u, v<<2|f) pair);
    #   hub mode: 4 B per streamed entry of the non-anchor rows, 4 B per staged
    #     anchor entry (once per task), 8 B per task;
    #   totals pass (forward-list census): per neighbour entry its word, its
    #     row id and one prefix count (16 B), per row its bounds and the prefix
    #     count at its end (16 B).
    tri = bool(ctx.get_tuning()["tri"]) and info["fwd_entries"] > 0
    chunk = info["tri_chunk"] if tri else info["hub_chunk"]
    if tri:
        cost, tasks = info["tri_bucket_cost"], info["tri_bucket_edges"]
        stream, staged = info["tri_stream"], info["tri_staged"]
    else:
        cost, tasks = info["bucket_cost"], info["bucket_dyads"]
        stream, staged = info["hub_stream"], info["hub_staged"]
    p_dyads = info["asym_dyads"] + info["mutual_dyads"]
    kern = [("k_census_lane", 0), ("k_census_wave", 1), ("k_census_group", 2), ("k_census_hub", 3)]
    per_launch_ms = {name: ks["ms"][b] / max(1, ks["launches"][b]) for name, b in kern}
    bytes_of = {name: (4.0 * stream + 4.0 * staged + 8.0 * tasks[3]) if b == 3 else
                (4.0 * cost[b] + 8.0 * tasks[b]) for name, b in kern}
    if tri:
        per_launch_ms["k_census_totals"] = ks["totals_ms"] / max(1, ks["totals_launches"])
        bytes_of["k_census_totals"] = 16.0 * 2 * p_dyads + 16.0 * g0.n
    dom_name = max(per_launch_ms, key=per_launch_ms.get)
    dom_ms = per_launch_ms[dom_name]
    bytes_dom = bytes_of[dom_name]
    achieved = bytes_dom / (dom_ms / 1000.0) / 1e9 if dom_ms > 0 else 0.0
    b_alg = 4.0 * info["sum_d2"] + 8.0 * (info["asym_dyads"] + info["mutual_dyads"]) + 4.0 * (g0.n + 1)
    step_bytes = census_bytes(info, g0.n, tri)
    line = {
        "metric": "census arcs/sec",
        "value": value,
        "unit": "arcs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64",
        "data": "synthetic",
        "config": {"workload": g0.name, "n": g0.n, "arcs": m_kept,
                   "reciprocity": 2.0 * info["mutual_dyads"] / max(1, m_kept),
                   "sum_d2": info["sum_d2"], "max_degree": info["max_degree"],
                   "tuning": ctx.get_tuning()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, kernel_key(dom_name, tri, ctx.get_tuning(), chunk)),
                     "kernel": dom_name, "bytes_per_launch": bytes_dom, "kernel_ms": dom_ms,
                     "source_hash": census_source_hash(),
                     # what the counters say limits the kernel (SQ_ACTIVE_INST_VALU x 4 / SIMD cycles)
                     "valu_busy": measured_valu_busy(args.workload, kernel_key(dom_name, tri, ctx.get_tuning(), chunk))},
        "path": "forward-list triangles" if tri else "dyad intersections",
        "kernels_ms": per_launch_ms,
        "kernel_bytes": bytes_of,
        "step_ms": {"p10": float(np.percentile(step_ms, 10)), "p50": float(np.percentile(step_ms, 50)),
                    "p90": float(np.percentile(step_ms, 90))},
        # the per-dyad merge's byte count (4 sum d^2 + 8p + 4(n+1)), for
        # reference only: the forward-list path never moves most of it
        "merge_b_alg_gb": b_alg / 1e9,
        # every kernel of the step by its own byte model, over the whole step
        "step_roofline": {"bytes": step_bytes, "achieved": step_bytes / (el / args.steps) / 1e9,
                          "unit": "GB/s", "frac": step_bytes / (el / args.steps) / 1e9 / HBM_PEAK_GBS},
        "build_s": build_s,
        "counts": [int(x) for x in counts],
    }
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        line["copy_calibration_bytes"] = args.copy_calibration
    else:
        # the same kernel rate against a measured device copy
        bw = copy_bandwidth()
        line["roofline"]["copy_gbs"] = bw
        line["roofline"]["frac_of_copy"] = achieved / bw
    if args.shards:
        line["shards"] = time_shards(ctx, g, counts, (2, 4, 8))
    gold = golden_counts("rmat", [g0]) if args.workload == "rmat" else None
    line["counts_equal_oracle"] = None if gold is None else line["counts"] == gold[0]
    g.release()
    ctx.close()
    if line["counts_equal_oracle"] is False:
        raise SystemExit("census differs from the oracle's stored census")
    if args.workload == "rmat" and not args.single_only:
        line["batched"] = run_batch(args, args.autotune_sample)
        line["served"] = run_serve(args)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(g0, m_kept, args.cpu_seconds)
        log("[bench] tuned multicore CPU census (context)")
        line["cpu_tuned"] = cpu_tuned(g0, m_kept)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
