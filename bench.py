#!/usr/bin/env python3
"""Benchmark of the DBL hot path on one MI355X (prints one JSON line).

One step is one pass of the whole path over the LiveJournal-shaped synthetic workload
(R-MAT, 2^22 vertices, 68,993,773 unique edges; the inputs are already resident in HBM when the
timed region starts):

  1. build: ingest into forward/reverse CSR, select 64 landmarks, hash the leaves, propagate
     DL and BL labels to the fixpoint;
  2. insert 100,000 R-MAT edges, one edge per request (validate, append, seed, propagate);
  3. answer 1,000,000 queries (about half reachable) in one batch: label rules, then the
     label-pruned BFS for the pairs the labels leave open.

`value` = (inserted edges + answered queries) per second of whole steps. The line also carries
the per-phase rates, the p50/p99 latency of single insertions, the roofline of the dominant
kernel (its launches timed with HIP events inside the timed region) and the CPU oracle timed on
a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "inserted edges/s (label update) + reachability queries/s; p99 latency; HBM GB/s"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per unit of work (the bytes the method must move, not what caches move).
# Query decided by labels: the pair (8 B), the 32-byte label records of u and v, the answer byte.
QUERY_LABEL_BYTES = 8 + 32 + 32 + 1
# Propagation: per relaxed edge the 4-byte neighbour id and a 16-byte read-modify-write of the
# neighbour's direction label; per expanded frontier entry its id (4 B), row offset and degree
# (12 B) and its own 16-byte label.
RELAX_BYTES = 4 + 16
EXPAND_BYTES = 4 + 12 + 16


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def with_counters(rl):
    """Add the counter view to a roofline object: measured HBM-side bytes (rocprofv3
    FETCH_SIZE + WRITE_SIZE, calibrated) over the same launch time."""
    if rl and rl.get("traffic"):
        t = rl["traffic"]
        rl["counter_achieved"] = t / (rl["avg_launch_us"] / 1e6) / 1e9
        rl["counter_frac"] = rl["counter_achieved"] / rl["peak"]
        rl["traffic_over_algorithmic"] = t / rl["algorithmic_bytes_per_launch"]
    return rl


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_2101_09441_amd", "csrc", "dbl_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` ("lj" or "scale") from the committed
    rocprofv3 counter summary, if it was taken on that workload and on the kernel source as it
    is now (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            d = json.load(f)
        e = d.get(workload, {}).get(kernel)
        if not e or e.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return e.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def cpu_baseline(w, n_ins_sample, n_q_sample):
    """Time the oracle on the host: full build, a prefix of the insertions, a prefix of the
    queries; scale each phase to the step's counts."""
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    o = oracle.OracleIndex(w.n, w.src, w.dst)
    o.build(k=64, kp=64, threads=threads)
    t_build = time.perf_counter() - t0
    log(f"cpu oracle build {t_build:.1f}s ({threads} threads)")
    t0 = time.perf_counter()
    o.insert(w.ins_src[:n_ins_sample], w.ins_dst[:n_ins_sample])
    t_ins = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.query_dbl(w.q_u[:n_q_sample], w.q_v[:n_q_sample], threads=threads)
    t_q = time.perf_counter() - t0
    o.close()
    n_ins, n_q = len(w.ins_src), len(w.q_u)
    t_step = t_build + t_ins * n_ins / n_ins_sample + t_q * n_q / n_q_sample
    return {
        "value": (n_ins + n_q) / t_step,
        "unit": "ops/s (inserted edges + answered queries)",
        "cores": threads,
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"oracle build of the full graph ({t_build:.1f} s, {threads} threads), first "
                   f"{n_ins_sample} insertions one at a time ({t_ins * 1e3:.1f} ms, 1 thread), "
                   f"first {n_q_sample} queries ({t_q * 1e3:.1f} ms, {threads} threads); each phase "
                   f"scaled to the step's {n_ins} insertions and {n_q} queries"),
        "step_s_extrapolated": t_step,
    }


def calibration_copy(dev):
    """One 1 GiB device-to-device copy (1 GiB read, 1 GiB written): the reference dispatch for
    scaling memory counters."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    c.copy_(a)
    torch.cuda.synchronize()
    del a, c
    log("calibration copy: 1 GiB read, 1 GiB written")


def bench_scale(args):
    """The batched form at scale: R-MAT 2^25 vertices, the distinct edges of 2^30 draws
    (~1.0e9), 10M insertions in batches of 100k, 10M Zipf(1.1)-skewed queries in batches of
    65,536. A step = build + all insertion batches + all query batches."""
    import numpy as np
    import torch

    import dblgen
    import paper_2101_09441_amd as dbl

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        calibration_copy(dev)
    t0 = time.perf_counter()
    w = dblgen.scale_workload()
    log(f"scale workload generated in {time.perf_counter() - t0:.0f} s: n={w.n} m={w.m}")
    src, dst = dbl.to_device_ids(w.src), dbl.to_device_ids(w.dst)
    isrc, idst = dbl.to_device_ids(w.ins_src), dbl.to_device_ids(w.ins_dst)
    qu, qv = dbl.to_device_ids(w.q_u), dbl.to_device_ids(w.q_v)
    out = torch.empty(len(w.q_u), dtype=torch.uint8, device=dev)
    n_ins, n_q, ib, qb = len(w.ins_src), len(w.q_u), 100_000, 65536

    def step(timed):
        r = {}
        ta = time.perf_counter()
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True,
                             time_kernels="round" if timed else None)
        tb = time.perf_counter()
        if timed:
            r["ktimes_build"] = ix.kernel_times()
            ix.time_kernels("insert_apply,local_rounds,query_label,query_bfs")
        lat_i = []
        for lo in range(0, n_ins, ib):
            t = time.perf_counter()
            ix.insert_edges(isrc[lo:lo + ib], idst[lo:lo + ib])
            lat_i.append(time.perf_counter() - t)
        tc = time.perf_counter()
        lat_q = []
        for lo in range(0, n_q, qb):
            t = time.perf_counter()
            ix.query(qu[lo:lo + qb], qv[lo:lo + qb], out=out[lo:lo + qb])
            lat_q.append(time.perf_counter() - t)
        td = time.perf_counter()
        r.update(build_s=tb - ta, insert_s=tc - tb, query_s=td - tc, lat_i=lat_i, lat_q=lat_q)
        if timed:
            r["ktimes"] = ix.kernel_times()
        ix.close()
        return r

    def diagnostics():
        """Untimed pass over the same inputs: counters after each phase."""
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
        s_b = ix.stats()
        for lo in range(0, n_ins, ib):
            ix.insert_edges(isrc[lo:lo + ib], idst[lo:lo + ib])
        s_i = ix.stats()
        for lo in range(0, n_q, qb):
            ix.query(qu[lo:lo + qb], qv[lo:lo + qb], out=out[lo:lo + qb])
        s_q = ix.stats()
        ix.close()
        return s_b, s_i, s_q

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    res = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - ts) / args.steps * 1e3
    for i, r in enumerate(res):
        log(f"step {i}: build {r['build_s']:.3f} s, inserts {r['insert_s']:.3f} s, "
            f"queries {r['query_s']:.3f} s")
    sb, si, st = diagnostics()
    kt = {}
    for r in res:
        for k, v in list(r["ktimes_build"].items()) + list(r["ktimes"].items()):
            a = kt.setdefault(k, {"launches": 0, "total_ms": 0.0})
            a["launches"] += v["launches"]
            a["total_ms"] += v["total_ms"]
    ans = out.cpu().numpy()
    classes = np.bincount(ans >> 1, minlength=7)

    def bytes_per_launch(kind):
        if kind == "query_label":
            return QUERY_LABEL_BYTES * qb
        if kind == "round":  # build rounds only
            return ((sb["vertices_expanded"] * EXPAND_BYTES + sb["edges_relaxed"] * RELAX_BYTES)
                    / max(sb["build_rounds"], 1))
        if kind == "insert_apply":  # appends and seeds of one 100k batch (section 6 of the
            return 112 * ib          # design notes: ~112 B per edge)
        if kind == "query_bfs":
            return ((st["bfs_edges"] - si["bfs_edges"]) * (4 + 24 + 8)
                    + (st["bfs_vertices"] - si["bfs_vertices"]) * 16) / max(n_q // qb, 1)
        return None

    kernel_rooflines = {}
    for k, d in kt.items():
        per = bytes_per_launch(k)
        if per is None or not d["launches"]:
            kernel_rooflines[k] = None
            continue
        avg = d["total_ms"] / d["launches"] / 1e3
        kernel_rooflines[k] = with_counters({
            "bound": "hbm", "achieved": per / avg / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": per / avg / 1e9 / HBM_PEAK_GBS,
            "traffic": committed_traffic(k, "scale"), "kernel": k,
            "avg_launch_us": avg * 1e6, "launches": d["launches"],
            "algorithmic_bytes_per_launch": per})
    timed_kinds = [k for k in kt if kernel_rooflines.get(k)]
    dominant = max(timed_kinds, key=lambda k: kt[k]["total_ms"]) if timed_kinds else None
    roofline = kernel_rooflines[dominant] if dominant else None
    line = {
        "metric": METRIC, "value": (n_ins + n_q) / (ms / 1e3),
        "unit": "ops/s (inserted edges + answered queries)", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "R-MAT 2^25 vertices, distinct edges of 2^30 draws, 10M "
                               "insertions in 100k batches, 10M Zipf(1.1) queries in 65,536 "
                               "batches, 64 DL + 64 BL bits", "n": w.n, "m": w.m,
                   "insertions": n_ins, "insert_batch": ib, "queries": n_q, "query_batch": qb},
        "build_s": float(np.mean([r["build_s"] for r in res])),
        "insert_edges_per_s": n_ins / float(np.mean([r["insert_s"] for r in res])),
        "insert_batch_ms": {"p50": float(np.percentile(res[-1]["lat_i"], 50) * 1e3),
                            "p99": float(np.percentile(res[-1]["lat_i"], 99) * 1e3),
                            "first": res[-1]["lat_i"][0] * 1e3,
                            "max": float(np.max(res[-1]["lat_i"]) * 1e3)},
        "queries_per_s": n_q / float(np.mean([r["query_s"] for r in res])),
        "query_batch_ms": {"p50": float(np.percentile(res[-1]["lat_q"], 50) * 1e3),
                           "p99": float(np.percentile(res[-1]["lat_q"], 99) * 1e3),
                           "first": res[-1]["lat_q"][0] * 1e3,
                           "max": float(np.max(res[-1]["lat_q"]) * 1e3)},
        "class_histogram": {dbl.CLASS_NAMES[i]: int(classes[i]) for i in range(7)},
        "kernel_times_ms": {k: {"launches": v["launches"],
                                "avg_us": v["total_ms"] / v["launches"] * 1e3}
                            for k, v in kt.items()},
        "build_teps": sb["edges_relaxed"] / float(np.mean([r["build_s"] for r in res])),
        "propagation": {"build_rounds": st["build_rounds"], "edges_relaxed": st["edges_relaxed"],
                        "vertices_expanded": st["vertices_expanded"],
                        "csr_regrows": st["csr_regrows"], "bfs_heavy": st["bfs_heavy"],
                        "pull_rounds": st["pull_rounds"],
                        "bfs_vertices": st["bfs_vertices"] - si["bfs_vertices"],
                        "bfs_edges": st["bfs_edges"] - si["bfs_edges"]},
        "roofline": roofline,
        "kernel_rooflines": kernel_rooflines,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["lj", "tiny", "scale"], default="lj")
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--serving", choices=["on", "off"], default="on")
    ap.add_argument("--extras", choices=["on", "off"], default="on",
                    help="off: skip the launch-per-request comparison, the batched form and "
                         "serving (leaves only same-sized plain passes, e.g. for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy one 1 GiB device buffer (reads 1 GiB, writes 1 GiB), the "
                         "reference for scaling memory counters")
    ap.add_argument("--time-kernels",
                    default="round,insert_stream,insert_server,insert_small,query_label,query_bfs",
                    help="kernel kinds timed with HIP events during the timed steps "
                         "(':N' times one launch in N); 'round' times the build's rounds")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this path "
              "runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import dblgen
    import paper_2101_09441_amd as dbl

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.workload == "scale":
        return bench_scale(args)
    if args.workload == "lj":
        w = dblgen.cached("rmat22-lj-s1", dblgen.lj_workload)
        desc = ("R-MAT (a,b,c,d)=(0.57,0.19,0.19,0.05), 2^22 vertices, 68,993,773 unique edges, "
                "100,000 R-MAT insertions one per request, 1,000,000 queries (35% random-walk "
                "endpoints, 65% uniform) in one batch, 64 DL + 64 BL bits")
    else:
        w = dblgen.cached("rmat14-tiny-s1", dblgen.tiny_workload)
        desc = ("R-MAT 2^14 vertices, 8n draws, 1,000 uniform insertions one per request, "
                "10,000 uniform queries, 64 DL + 64 BL bits")
    log(f"workload {w.name}: n={w.n} m={w.m} insertions={len(w.ins_src)} queries={len(w.q_u)}")
    src, dst = dbl.to_device_ids(w.src), dbl.to_device_ids(w.dst)
    isrc, idst = dbl.to_device_ids(w.ins_src), dbl.to_device_ids(w.ins_dst)
    qu, qv = dbl.to_device_ids(w.q_u), dbl.to_device_ids(w.q_v)
    out = torch.empty(len(w.q_u), dtype=torch.uint8, device=dev)
    if args.calibrate_copy:
        calibration_copy(dev)
    torch.cuda.synchronize()

    kinds = [k for k in args.time_kernels.split(",") if k]

    def step(timed):
        r = {}
        t0 = time.perf_counter()
        # the build's grid propagation rounds are timed from inside dbl_build
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True,
                             time_kernels="round" if timed and "round" in kinds else None)
        t1 = time.perf_counter()
        if timed:
            r["ktimes_build"] = ix.kernel_times()
            ix.time_kernels(",".join(k for k in kinds if k != "round") or None)
        # per-request latencies are recorded in the untimed diagnostic pass (the clock reads
        # are instrumentation, not work)
        ix.insert_edges_each(isrc, idst)
        t2 = time.perf_counter()
        ix.query(qu, qv, out=out)
        t3 = time.perf_counter()
        r.update(build_s=t1 - t0, insert_s=t2 - t1, query_s=t3 - t2)
        if timed:
            r["ktimes"] = ix.kernel_times()
        ix.close()
        return r

    def diagnostics():
        """Untimed pass over the same inputs: counters after each phase, each request's
        latency, final labels."""
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
        s_build = ix.stats()
        lat = ix.insert_edges_each(isrc, idst, latencies=True)
        s_ins = ix.stats()
        ix.query(qu, qv, out=out)
        s_q = ix.stats()
        labels = ix.labels()
        ix.close()
        return s_build, s_ins, s_q, labels, lat

    def launch_per_request(plain_labels):
        """The same single-edge requests with one kernel launch per request instead of the
        resident workgroup (untimed; labels must come out identical)."""
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
        ix.set_tuning(insert_server=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat2 = ix.insert_edges_each(isrc, idst, latencies=True)
        dt = time.perf_counter() - t0
        same = all(torch.equal(a, b) for a, b in zip(ix.labels(), plain_labels))
        ix.close()
        return {"edges_per_s": n_ins / dt,
                "latency_us_p50": float(np.percentile(lat2, 50)),
                "latency_us_p99": float(np.percentile(lat2, 99)),
                "labels_equal_stream": bool(same)}

    def serving():
        """Continuous-batching server on the resident graph: a Poisson stream of query batches
        (1..100k pairs) and insertion batches (1k..10k edges) at 80:20, swept over arrival
        rates up to saturation; next to it the same trace served one request at a time in
        sequence order against the same arrival times (no overlap, no coalescing; queueing
        counts in its latency)."""
        from paper_2101_09441_amd.serve import Request, serve, serve_alone
        res = {}
        n_req = 1200
        for rate in (2000.0, 8000.0, 32000.0, 128000.0, 512000.0):
            spec = dblgen.serving_trace(w.q_u, w.q_v, w.ins_src, w.ins_dst, n_req, rate, seed=5)
            trace = [Request(s_, k, a, b, t) for s_, k, a, b, t in spec]
            ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
            summ = serve(ix, trace, workers=4, max_batch=1 << 17, bfs_slots=256)
            ix.close()
            ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
            alone = [Request(s_, k, a, b, t) for s_, k, a, b, t in spec]
            alone_summ = serve_alone(ix, alone)
            ix.close()
            same = all(r.kind != "query" or np.array_equal(r.answers, m.answers)
                       for r, m in zip(alone, trace))
            res[f"rate_{int(rate)}_per_s"] = {"serving": summ, "one_at_a_time": alone_summ,
                                              "answers_equal_alone": bool(same)}
            log(f"serving rate {rate}: queries/s {summ['query']['per_s']:.3g} "
                f"(alone {alone_summ['query']['per_s']:.3g}), query p99 "
                f"{summ['query']['latency_ms_p99']:.2f} ms (alone "
                f"{alone_summ['query']['latency_ms_p99']:.2f}), equal {same}")
        return res

    T4_SAMPLE = 8192

    def table4(plain_answers):
        """The shape of the paper's Table 4 on this workload: queries answered with DL only, BL
        only and both (DBL), on the index after the plain form's insertions; the share each
        decides by labels alone, its class histogram and its batch time. The answers are exact
        in every mode. DL only and DBL run on all the queries. Without the DL rules and prune,
        every reachable pair needs a pruned BFS that explores much of the graph, so BL only
        runs on the first T4_SAMPLE queries (the other two modes too, for a like-for-like
        comparison); the searches that outgrow their wave's slot go to the whole-device BFS
        from both ends."""
        ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
        ix.insert_edges(isrc, idst)
        ctx = ix.query_context()
        k = min(T4_SAMPLE, n_q)
        res = {"all": {"queries": n_q}, "sample": {"queries": k, "which": "the first queries"}}
        for part, cnt, modes in (("all", n_q, (("DL", 1), ("DBL", 3))),
                                 ("sample", k, (("DL", 1), ("BL", 2), ("DBL", 3)))):
            for name, rules in modes:
                o = torch.empty(cnt, dtype=torch.uint8, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.query_rules(qu[:cnt], qv[:cnt], rules, out=o)
                dt = time.perf_counter() - t0
                a = o.cpu().numpy()
                cls = np.bincount(a >> 1, minlength=7)
                res[part][name] = {
                    "label_decided_frac": float(cls[:5].sum() / cnt),
                    "class_histogram": {dbl.CLASS_NAMES[i]: int(cls[i]) for i in range(7)},
                    "batch_ms": dt * 1e3,
                    "answers_equal_plain": bool(np.array_equal(a & 1, plain_answers[:cnt] & 1))}
                log(f"table 4 shape ({part}, {cnt} queries), {name}: "
                    f"{res[part][name]['label_decided_frac']:.4f} decided by labels, "
                    f"{dt * 1e3:.1f} ms")
        ctx.close()
        ix.close()
        return res

    def host_requests(plain_labels):
        """The single-edge requests as a host client issues them: the request server takes
        each edge from pinned host memory after the previous one was reported (a PCIe round
        trip per request), without and with its cache warm-up (untimed; labels must equal the
        stream's)."""
        res = {}
        for warm in (0, 1):
            ix = dbl.Index.build(w.n, src, dst, edges_unique=True)
            ix.set_tuning(insert_server=1, server_warm=warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat2 = ix.insert_edges_each(isrc, idst, latencies=True)
            dt = time.perf_counter() - t0
            st = ix.stats()
            same = all(torch.equal(a, b) for a, b in zip(ix.labels(), plain_labels))
            ix.close()
            res[f"server_warm_{warm}"] = {
                "edges_per_s": n_ins / dt,
                "latency_us_p50": float(np.percentile(lat2, 50)),
                "latency_us_p99": float(np.percentile(lat2, 99)),
                "device_us_per_request": st["server_busy_us"] / max(st["server_requests"], 1),
                "labels_equal_stream": bool(same)}
        return res

    def batched(plain_labels, plain_answers):
        """The batched form on the same inputs: insertion batches of 1k/10k/100k edges and query
        batches of 65,536 pairs; labels and answers must equal the plain form's."""
        from paper_2101_09441_amd import autotune
        res = {}
        qb = 65536
        mk = lambda: dbl.Index.build(w.n, src, dst, edges_unique=True)  # noqa: E731
        def insert_stream(make, tuning, bsz):
            """Insert the whole stream in batches of bsz, on fresh indexes with `tuning`, repeated
            until at least 10 batches were timed (the 100k stream is one batch); the timing
            entry, with the median pass as its rate."""
            times, passes, same, stalls = [], [], True, 0
            while len(times) < 10:
                ix = make()
                ix.set_tuning(**tuning)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for lo in range(0, n_ins, bsz):
                    tb = time.perf_counter()
                    ix.insert_edges(isrc[lo:lo + bsz], idst[lo:lo + bsz])
                    times.append(time.perf_counter() - tb)
                passes.append(time.perf_counter() - t0)
                same &= all(torch.equal(a, b) for a, b in zip(ix.labels(), plain_labels))
                stalls += ix.stats()["batch_stalls"]
                ix.close()
            t_ins = float(np.median(passes))
            return {"edges_per_s": n_ins / t_ins, "batches": len(times), "passes": len(passes),
                    "batch_ms_p50": float(np.percentile(times, 50) * 1e3),
                    "batch_ms_p99": float(np.percentile(times, 99) * 1e3),
                    "speedup_vs_plain": (n_ins / t_ins) / (n_ins / insert_s),
                    "labels_equal_plain": bool(same), "batch_stalls": stalls}

        # the three forms of an insertion batch above the single-workgroup limit, default knobs
        forms = {"multi_launch": dict(insert_persistent=0),
                 "persistent": dict(insert_persistent=1, insert_graph=0),
                 "persistent_graph": dict(insert_persistent=1, insert_graph=1)}
        for bsz in (1000, 10000, 100000):
            if bsz > n_ins:
                continue
            tuned = autotune.tune_insertions(mk, isrc, idst, bsz, w.m, max_batches=30,
                                             progress=log)
            knobs = {k: tuned[k] for k in autotune.INSERT_KNOBS}
            entry = insert_stream(mk, knobs, bsz)
            entry["tuning"] = knobs
            log(f"batches of {bsz}: {entry['edges_per_s']:.3g} edges/s with {entry['tuning']}")
            if bsz == 1000:
                # query batches on the index after every insertion
                ix = mk()
                ix.insert_edges(isrc, idst)
                qtuned = autotune.tune_queries(ix, qu, qv, qb, w.m)
                # each batch as two kernel launches, then as one graph launch (the graph is
                # instantiated by an untimed first batch and replayed with new arguments)
                for graph in (0, 1):
                    ix.set_tuning(query_graph=graph)
                    qout = torch.empty_like(out)
                    ix.query(qu[:qb], qv[:qb], out=qout[:qb])
                    qt = []
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for lo in range(0, n_q, qb):
                        tb = time.perf_counter()
                        ix.query(qu[lo:lo + qb], qv[lo:lo + qb], out=qout[lo:lo + qb])
                        qt.append(time.perf_counter() - tb)
                    t_q = time.perf_counter() - t0
                    res["query_batches_65536" + ("_graph" if graph else "")] = {
                        "queries_per_s": n_q / t_q, "batches": len(qt),
                        "batch_ms_p50": float(np.percentile(qt, 50) * 1e3),
                        "batch_ms_p99": float(np.percentile(qt, 99) * 1e3),
                        "answers_equal_plain": bool(torch.equal(qout, plain_answers)),
                        "tuning": {"bfs_slots": qtuned["bfs_slots"], "query_graph": graph}}
                ix.close()
            entry["forms"] = {name: insert_stream(mk, dict(small_batch=min(bsz - 1, 2048), **kw),
                                                  bsz)
                              for name, kw in forms.items()}
            # the autotuner times a few batches per candidate, so its pick can lose to a fixed
            # form on the whole stream: the entry's rate is the fastest setting measured here
            best = max([("tuned", entry)] + list(entry["forms"].items()),
                       key=lambda kv: kv[1]["edges_per_s"])
            entry["tuned_edges_per_s"] = entry["edges_per_s"]
            entry["edges_per_s"] = best[1]["edges_per_s"]
            entry["speedup_vs_plain"] = best[1]["speedup_vs_plain"]
            entry["fastest"] = best[0]
            res[f"insert_batch_{bsz}"] = entry
        return res

    for i in range(args.warmup):
        r = step(False)
        log(f"warmup {i}: build {r['build_s']*1e3:.1f} ms, inserts {r['insert_s']:.2f} s, "
            f"queries {r['query_s']*1e3:.1f} ms")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = step(True)
        results.append(r)
        log(f"step {i}: build {r['build_s']*1e3:.1f} ms, inserts {r['insert_s']:.2f} s, "
            f"queries {r['query_s']*1e3:.1f} ms")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = t_total / args.steps * 1e3
    n_ins, n_q = len(w.ins_src), len(w.q_u)
    value = (n_ins + n_q) / (ms_per_step / 1e3)

    build_s = float(np.mean([r["build_s"] for r in results]))
    insert_s = float(np.mean([r["insert_s"] for r in results]))
    query_s = float(np.mean([r["query_s"] for r in results]))
    s_build, s_ins, s_q, plain_labels, lat = diagnostics()
    log("diagnostic pass done")
    extras = args.extras == "on"
    per_request = launch_per_request(plain_labels) if extras else None
    host_req = host_requests(plain_labels) if extras else None
    if extras:
        log("single-request comparisons done")
    table4_res = table4(out.cpu().numpy()) if extras else None
    batched_res = batched(plain_labels, out.clone()) if extras else None
    serving_res = (serving() if extras and args.workload == "lj" and args.serving == "on"
                   else None)
    ins_expanded = s_ins["vertices_expanded"] - s_build["vertices_expanded"]
    ins_relaxed = s_ins["edges_relaxed"] - s_build["edges_relaxed"]
    answers = out.cpu().numpy()
    classes = np.bincount(answers >> 1, minlength=7)

    # kernel times accumulated over all timed steps
    kt = {}
    for r in results:
        for k, v in list(r["ktimes_build"].items()) + list(r["ktimes"].items()):
            a = kt.setdefault(k, {"launches": 0, "total_ms": 0.0})
            a["launches"] += v["launches"]
            a["total_ms"] += v["total_ms"]
    dominant = max(kt, key=lambda k: kt[k]["total_ms"]) if kt else None

    def bytes_per_launch(kind):
        """Algorithmic bytes of one launch of `kind` over this step's work."""
        if kind == "query_label":
            return QUERY_LABEL_BYTES * n_q
        if kind in ("insert_server", "insert_stream"):
            # every request of the timed steps, spread over the launches that served them
            prop = ins_expanded * EXPAND_BYTES + ins_relaxed * RELAX_BYTES
            per_req = 8 + 8 + 24 + 8 + 32 + 32 + prop / n_ins
            return per_req * n_ins * len(results) / kt[kind]["launches"]
        if kind == "insert_small":
            # one edge per launch: the two appends and two seeds (ids 8 B, two degree RMWs 8 B,
            # two row offsets and capacities 24 B, two column writes 8 B, labels read 32 B and
            # OR-ed 32 B), plus the propagation the insertions triggered, averaged per launch
            prop = ins_expanded * EXPAND_BYTES + ins_relaxed * RELAX_BYTES
            return 8 + 8 + 24 + 8 + 32 + 32 + prop / n_ins
        if kind == "round":
            prop = (s_build["vertices_expanded"] * EXPAND_BYTES
                    + s_build["edges_relaxed"] * RELAX_BYTES)
            return prop / max(s_build["build_rounds"], 1)
        if kind == "query_bfs":
            # per scanned edge: 4 B id + 24 B of labels + the visited word; per vertex 16 B
            return (s_q["bfs_edges"] - s_ins["bfs_edges"]) * (4 + 24 + 8) + \
                (s_q["bfs_vertices"] - s_ins["bfs_vertices"]) * 16
        return None

    per_request_device_us = (s_ins["server_busy_us"] / s_ins["server_requests"]
                             if s_ins["server_requests"] else None)
    lat_p50_us = float(np.percentile(lat, 50))

    def roofline_of(kind):
        d = kt[kind]
        per_launch = bytes_per_launch(kind)
        if per_launch is None or not d["launches"]:
            return None
        avg_s = d["total_ms"] / d["launches"] / 1e3
        achieved = per_launch / avg_s / 1e9
        r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic(kind, "lj"),
             "kernel": kind, "avg_launch_us": avg_s * 1e6, "launches": d["launches"],
             "algorithmic_bytes_per_launch": per_launch}
        if kind == "insert_stream" and per_request_device_us is not None:
            # one launch serves the whole request stream, one request after another
            r["note"] = (f"one resident workgroup applies the requests in order: "
                         f"{per_request_device_us:.2f} us per request on average, "
                         f"{lat_p50_us:.2f} us at p50 (requests go in windows of 32: a window "
                         f"waits for one memory round trip, its reads and the stores of the "
                         f"window before, and a request that changes no label then takes a "
                         f"dozen instructions in one wave; the few that change labels end their "
                         f"window and add their propagation rounds), so the bound is that "
                         f"chain of memory latencies, not HBM bandwidth")
        return with_counters(r)

    roofline = roofline_of(dominant) if dominant else None
    kernel_rooflines = {k: roofline_of(k) for k in kt}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "ops/s (inserted edges + answered queries)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "n": w.n, "m": w.m, "insertions": n_ins,
                   "insertion_form": ("one edge per request, read from HBM and applied in "
                                      "order by one resident workgroup (no host step per "
                                      "request; a host client's round trip per request is "
                                      "in insert_host_requests)"),
                   "insertion_note": ("R-MAT insertions continuing the build stream: "
                                      f"{ins_relaxed} edges relaxed over all {n_ins} requests, "
                                      "so most requests change no label"),
                   "queries": n_q,
                   "query_batch": n_q, "landmarks": 64, "bl_bits": 64},
        "build_ms": build_s * 1e3,
        "insert_edges_per_s": n_ins / insert_s,
        "insert_latency_us": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99)),
                              "max": float(lat.max())},
        "queries_per_s": n_q / query_s,
        "query_batch_ms": query_s * 1e3,
        "label_decided_frac": float(classes[:5].sum() / max(n_q, 1)),
        "reachable_frac": float((answers & 1).mean()),
        "class_histogram": {dbl.CLASS_NAMES[i]: int(classes[i]) for i in range(7)},
        "kernel_times_ms": {k: {"launches": v["launches"], "avg_us": v["total_ms"] / v["launches"]
                                * 1e3} for k, v in kt.items()},
        "build_teps": s_build["edges_relaxed"] / build_s,
        "propagation": {"build_rounds": s_build["build_rounds"],
                        "build_edges_relaxed": s_build["edges_relaxed"],
                        "build_vertices_expanded": s_build["vertices_expanded"],
                        "insert_edges_relaxed": ins_relaxed,
                        "insert_vertices_expanded": ins_expanded,
                        "csr_regrows": s_ins["csr_regrows"],
                        "bfs_edges": s_q["bfs_edges"], "bfs_vertices": s_q["bfs_vertices"]},
        "insert_device_us_per_request": per_request_device_us,
        "insert_launch_per_request": per_request,
        "insert_host_requests": host_req,
        "table4_shape": table4_res,
        "batched": batched_res,
        "serving": serving_res,
        "roofline": roofline,
        "kernel_rooflines": kernel_rooflines,
        "cpu_baseline": None,
    }
    if args.cpu_baseline == "on":
        n_ins_s = min(n_ins, 10000)
        n_q_s = min(n_q, 100000)
        line["cpu_baseline"] = cpu_baseline(w, n_ins_s, n_q_s)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
