"""Autotuner for the batched form: picks the runtime tuning of an index by measurement.

Insertion knobs (the single-workgroup batch limit and the local-round limits, the grid-round
block count, the pull threshold of grid rounds, the persistent one-launch form and its graph
replay) are timed on fresh indexes built from the same graph, because insertions change the
index; query knobs (BFS slots) are timed on the index itself, because queries do not. The
choice is cached per (device, graph size, phase, batch size) in a JSON file. No knob can change
a label or an answer, only the time they take.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Optional

import torch

# the multi-launch form (host-driven rounds) over its knobs, then the persistent form (one launch
# per batch above small_batch, plain or as a graph replay) over the knobs that reach it
INSERT_CANDIDATES: List[dict] = [
    dict(small_batch=sb, local_max_frontier=lf, local_max_edges=le, round_grid=rg,
         pull_threshold=pt, insert_persistent=0, insert_graph=0)
    for sb in (256, 2048, 16384)
    for lf, le in ((8192, 1 << 16), (32768, 1 << 18))
    for rg in (1024, 2048)
    for pt in (0, 128)
] + [
    dict(small_batch=sb, local_max_frontier=lf, local_max_edges=le, round_grid=2048,
         pull_threshold=128, insert_persistent=1, insert_graph=gr)
    for sb in (0, 256, 2048)
    for lf, le in ((8192, 1 << 16), (32768, 1 << 18))
    for gr in (0, 1)
]
INSERT_KNOBS = ("small_batch", "local_max_frontier", "local_max_edges", "round_grid",
                "pull_threshold", "insert_persistent", "insert_graph")
QUERY_CANDIDATES: List[dict] = [dict(bfs_slots=s) for s in (256, 512, 1024, 2048)]


def _cache_path() -> str:
    return os.environ.get("DBL_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dbl_tuning.json"))


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    c = _load_cache()
    c[key] = value
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, p)
    except OSError:
        pass


def _key(index, m: int, phase: str, batch: int) -> str:
    name = torch.cuda.get_device_name(index.device)
    return f"{name}|n={index.n}|m={m}|{phase}|batch={batch}"


def tune_insertions(make_index: Callable, src: torch.Tensor, dst: torch.Tensor, batch: int,
                    m: int, max_batches: int = 20, use_cache: bool = True,
                    progress: Optional[Callable[[str], None]] = None) -> dict:
    """Time inserting up to `max_batches` batches of `batch` edges for every insertion
    candidate, each on a fresh index from make_index(); return the fastest setting.
    progress(msg), if given, is called after every eighth candidate."""
    probe = make_index()
    key = _key(probe, m, "insert", batch)
    cache = _load_cache()
    if use_cache and key in cache and all(k in cache[key] for k in INSERT_KNOBS):
        probe.close()
        return cache[key]
    probe.close()
    n_edges = min(src.numel(), batch * max_batches)
    results = []
    for cand in INSERT_CANDIDATES:
        # the better of two trials, each on a fresh index
        dt = float("inf")
        for _ in range(2):
            ix = make_index()
            ix.set_tuning(**cand)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for lo in range(0, n_edges, batch):
                ix.insert_edges(src[lo:lo + batch], dst[lo:lo + batch])
            dt = min(dt, time.perf_counter() - t0)
            ix.close()
        results.append((dt, cand))
        if progress is not None and len(results) % 8 == 0:
            progress(f"tuning batches of {batch}: {len(results)} of "
                     f"{len(INSERT_CANDIDATES)} candidates timed")
    dt, best = min(results, key=lambda r: r[0])
    out = dict(best, seconds=dt, timed_edges=n_edges,
               candidates=[dict(c, seconds=t) for t, c in results])
    _store(key, out)
    return out


def tune_queries(index, u: torch.Tensor, v: torch.Tensor, batch: int, m: int, reps: int = 3,
                 use_cache: bool = True) -> dict:
    """Time query batches of `batch` pairs for every query candidate on `index` (queries do not
    change it) and leave the fastest setting applied."""
    key = _key(index, m, "query", batch)
    cache = _load_cache()
    if use_cache and key in cache:
        index.set_tuning(bfs_slots=cache[key]["bfs_slots"])
        return cache[key]
    out = torch.empty(min(u.numel(), batch), dtype=torch.uint8, device=u.device)
    nb = min(u.numel(), batch * 8)
    results = []
    for cand in QUERY_CANDIDATES:
        index.set_tuning(**cand)
        index.query(u[:batch], v[:batch], out=out)  # warm the context
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for lo in range(0, nb, batch):
                k = min(batch, nb - lo)
                index.query(u[lo:lo + k], v[lo:lo + k], out=out[:k])
            best = min(best, time.perf_counter() - t0)
        results.append((best, cand))
    dt, bestc = min(results, key=lambda r: r[0])
    index.set_tuning(**bestc)
    res = dict(bestc, seconds=dt, timed_pairs=nb,
               candidates=[dict(c, seconds=t) for t, c in results])
    _store(key, res)
    return res
