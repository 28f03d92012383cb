"""Seeded synthetic inputs for the DBL reachability index (input only: no index arithmetic).

Both the CPU oracle and the GPU path consume what this module produces. The arithmetic lives in
``dblgen.c`` (xoshiro256** seeded through splitmix64, R-MAT descent, Fisher-Yates relabelling,
query mixtures); this file compiles it with gcc and wraps it with ctypes and numpy.

Workloads (the shapes of the paper's experiments, stood in for by R-MAT graphs because the
paper's SNAP datasets are not available):

* ``tiny``: 2^14 vertices, 8*n R-MAT draws (loops and duplicates removed), 1,000 uniform new
  edges inserted one at a time, 10,000 uniform queries.
* ``lj``: 2^22 vertices, 68,993,773 unique edges (the LiveJournal edge count of the paper's
  dataset table), 100,000 insertion edges continuing the R-MAT stream, 1,000,000 queries of which
  about 35% are random-walk endpoints (reachable by construction) and the rest uniform.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dblgen.c")
# DBL_SANITIZE=1 selects a build instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (a library of its own name; the process must preload the ASan runtime).
_SANITIZE = os.environ.get("DBL_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libdblgen_san.so" if _SANITIZE else "libdblgen.so")
_SAN_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined"]
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build() -> str:
    """Compile ``dblgen.c`` into ``libdblgen.so`` (always recompiles)."""
    tmp = _LIB + ".tmp"
    opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
    subprocess.check_call(["gcc", *opt, "-std=gnu11", "-fPIC", "-shared", "-pthread", "-o", tmp,
                           _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    u32, u64, f64, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_int64
    lib.dblgen_rmat_new.restype = P
    lib.dblgen_rmat_new.argtypes = [u32, u64, f64, f64, f64, u64]
    lib.dblgen_rmat_free.argtypes = [P]
    lib.dblgen_rmat_free.restype = None
    lib.dblgen_rmat_n.argtypes = [P]
    lib.dblgen_rmat_n.restype = u32
    lib.dblgen_rmat_draws.argtypes = [P]
    lib.dblgen_rmat_draws.restype = u64
    lib.dblgen_rmat_next.argtypes = [P, u64, u64, P, P]
    lib.dblgen_rmat_next.restype = i64
    lib.dblgen_rmat_uniform_new.argtypes = [P, u64, u64, P, P]
    lib.dblgen_rmat_uniform_new.restype = i64
    lib.dblgen_rmat_contains.argtypes = [P, u32, u32]
    lib.dblgen_rmat_contains.restype = ctypes.c_int
    lib.dblgen_queries_uniform.argtypes = [u32, u64, u64, P, P]
    lib.dblgen_queries_uniform.restype = None
    lib.dblgen_queries_mixed.argtypes = [u32, u64, P, P, u64, u64, f64, u32, P, P]
    lib.dblgen_queries_mixed.restype = ctypes.c_int
    lib.dblgen_queries_zipf.argtypes = [u32, u64, u64, f64, P, P]
    lib.dblgen_queries_zipf.restype = ctypes.c_int
    lib.dblgen_rmat_large.argtypes = [u32, u64, f64, f64, f64, u64, u64, u32, P, P, P, u64, P, P]
    lib.dblgen_rmat_large.restype = ctypes.c_int
    lib.dblgen_xoshiro_outputs.argtypes = [u64, u64, P]
    lib.dblgen_xoshiro_outputs.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class RmatStream:
    """A seeded R-MAT edge stream over 2^scale vertices with duplicate/loop rejection."""

    def __init__(self, scale: int, seed: int, expected_edges: int = 0,
                 a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C):
        lib = _load()
        self._h = lib.dblgen_rmat_new(scale, seed, a, b, c, max(expected_edges, 1024))
        if not self._h:
            raise MemoryError("dblgen_rmat_new failed")
        self.n = int(lib.dblgen_rmat_n(self._h))

    def close(self):
        if self._h:
            _load().dblgen_rmat_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def draws(self) -> int:
        return int(_load().dblgen_rmat_draws(self._h))

    def next_edges(self, max_unique: int, max_draws: int = 0):
        src = np.empty(max(max_unique, 1), dtype=np.uint32)
        dst = np.empty(max(max_unique, 1), dtype=np.uint32)
        got = _load().dblgen_rmat_next(self._h, max_unique, max_draws, _ptr(src), _ptr(dst))
        if got < 0:
            raise MemoryError("dblgen_rmat_next failed")
        return src[:got].copy(), dst[:got].copy()

    def uniform_new_edges(self, seed: int, count: int):
        src = np.empty(max(count, 1), dtype=np.uint32)
        dst = np.empty(max(count, 1), dtype=np.uint32)
        got = _load().dblgen_rmat_uniform_new(self._h, seed, count, _ptr(src), _ptr(dst))
        if got < 0:
            raise MemoryError("dblgen_rmat_uniform_new failed")
        return src[:got].copy(), dst[:got].copy()

    def contains(self, u: int, v: int) -> bool:
        return bool(_load().dblgen_rmat_contains(self._h, u, v))


def queries_uniform(n: int, seed: int, count: int):
    u = np.empty(max(count, 1), dtype=np.uint32)
    v = np.empty(max(count, 1), dtype=np.uint32)
    _load().dblgen_queries_uniform(n, seed, count, _ptr(u), _ptr(v))
    return u[:count].copy(), v[:count].copy()


def queries_mixed(n: int, src: np.ndarray, dst: np.ndarray, seed: int, count: int,
                  p_walk: float = 0.35, max_len: int = 16):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    u = np.empty(max(count, 1), dtype=np.uint32)
    v = np.empty(max(count, 1), dtype=np.uint32)
    rc = _load().dblgen_queries_mixed(n, len(src), _ptr(src), _ptr(dst), seed, count, p_walk,
                                      max_len, _ptr(u), _ptr(v))
    if rc:
        raise MemoryError("dblgen_queries_mixed failed")
    return u[:count].copy(), v[:count].copy()


def queries_zipf(n: int, seed: int, count: int, s: float = 1.1):
    u = np.empty(max(count, 1), dtype=np.uint32)
    v = np.empty(max(count, 1), dtype=np.uint32)
    rc = _load().dblgen_queries_zipf(n, seed, count, s, _ptr(u), _ptr(v))
    if rc:
        raise MemoryError("dblgen_queries_zipf failed")
    return u[:count].copy(), v[:count].copy()


def xoshiro_outputs(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().dblgen_xoshiro_outputs(seed, count, _ptr(out))
    return out


@dataclass
class Workload:
    """One synthetic workload: build edges, an insertion stream and a query stream."""
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    ins_src: np.ndarray
    ins_dst: np.ndarray
    q_u: np.ndarray
    q_v: np.ndarray
    draws: int

    @property
    def m(self) -> int:
        return len(self.src)


def make_rmat_workload(name: str, scale: int, seed: int, *, draws: int = 0, m_target: int = 0,
                       n_insert: int = 0, insert_kind: str = "rmat", n_query: int = 0,
                       query_kind: str = "uniform", p_walk: float = 0.35) -> Workload:
    """Build edges (by draw count or unique-edge target), insertion edges, queries."""
    if not draws and not m_target:
        raise ValueError("give draws or m_target")
    expected = (m_target or draws) + n_insert
    st = RmatStream(scale, seed, expected_edges=expected)
    src, dst = st.next_edges(m_target if m_target else draws, draws if not m_target else 0)
    n_draws = st.draws
    if n_insert:
        if insert_kind == "rmat":
            isrc, idst = st.next_edges(n_insert)
        elif insert_kind == "uniform":
            isrc, idst = st.uniform_new_edges(seed + 3, n_insert)
        else:
            raise ValueError(insert_kind)
    else:
        isrc = idst = np.empty(0, dtype=np.uint32)
    st.close()
    n = 1 << scale
    if n_query:
        if query_kind == "uniform":
            qu, qv = queries_uniform(n, seed + 2, n_query)
        elif query_kind == "mixed":
            qu, qv = queries_mixed(n, src, dst, seed + 2, n_query, p_walk=p_walk)
        elif query_kind == "zipf":
            qu, qv = queries_zipf(n, seed + 2, n_query)
        else:
            raise ValueError(query_kind)
    else:
        qu = qv = np.empty(0, dtype=np.uint32)
    return Workload(name, n, src, dst, isrc, idst, qu, qv, n_draws)


def serving_trace(q_u, q_v, ins_src, ins_dst, n_requests: int, rate: float, p_query: float = 0.8,
                  q_size=(1, 100_000), i_size=(1_000, 10_000), seed: int = 7):
    """A Poisson arrival stream of query and insertion requests.

    Inter-arrival times are exponential with mean 1/rate; a request is a query batch with
    probability p_query, else an insertion batch; sizes are log-uniform integers in the given
    ranges. Query pairs are taken in order from (q_u, q_v) (wrapping around); insertion edges in
    order from (ins_src, ins_dst) (once they run out, further requests are queries).
    Returns a list of (seq, kind, a, b, arrival_seconds).
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out, qi, ii = [], 0, 0
    nq, ni = len(q_u), len(ins_src)

    def logu(lo, hi):
        return int(np.exp(rng.uniform(np.log(lo), np.log(hi + 1))))

    for s in range(n_requests):
        want_q = rng.random() < p_query
        if not want_q and ii < ni:
            k = min(logu(*i_size), ni - ii)
            out.append((s, "insert", ins_src[ii:ii + k].copy(), ins_dst[ii:ii + k].copy(), float(t[s])))
            ii += k
        else:
            k = max(1, min(logu(*q_size), nq))
            idx = (qi + np.arange(k)) % nq
            out.append((s, "query", q_u[idx].copy(), q_v[idx].copy(), float(t[s])))
            qi = (qi + k) % nq
    return out


def rmat_large(scale: int, seed: int, draws: int, n_insert: int, threads: int = 0,
               chunk: int = 1 << 20):
    """Chunked-stream R-MAT (see dblgen.c): the distinct non-loop edges of `draws` draws,
    sorted, plus `n_insert` new edges continuing the stream."""
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    src = np.empty(max(draws, 1), dtype=np.uint32)
    dst = np.empty(max(draws, 1), dtype=np.uint32)
    isrc = np.empty(max(n_insert, 1), dtype=np.uint32)
    idst = np.empty(max(n_insert, 1), dtype=np.uint32)
    m = ctypes.c_uint64()
    rc = _load().dblgen_rmat_large(scale, seed, RMAT_A, RMAT_B, RMAT_C, draws, chunk, threads,
                                   _ptr(src), _ptr(dst), ctypes.addressof(m), n_insert,
                                   _ptr(isrc), _ptr(idst))
    if rc:
        raise MemoryError("dblgen_rmat_large failed")
    mm = int(m.value)
    return src[:mm], dst[:mm], isrc[:n_insert], idst[:n_insert]


def scale_workload(scale: int = 25, draws: int = 1 << 30, n_insert: int = 10_000_000,
                   n_query: int = 10_000_000, seed: int = 1) -> Workload:
    """Large R-MAT (2^25 vertices, the distinct edges of 2^30 draws, about 1.0e9), insertions
    continuing the stream, Zipf(1.1)-skewed query sources with uniform targets."""
    src, dst, isrc, idst = rmat_large(scale, seed, draws, n_insert)
    qu, qv = queries_zipf(1 << scale, seed + 2, n_query)
    return Workload(f"rmat{scale}-scale", 1 << scale, src, dst, isrc, idst, qu, qv, draws)


def cached(name: str, make, cache_dir: str = None) -> Workload:
    """Return make() through an on-disk cache (uncompressed .npz keyed by `name`)."""
    cache_dir = cache_dir or os.environ.get("DBLGEN_CACHE", "/tmp/dblgen_cache")
    path = os.path.join(cache_dir, name + ".npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            return Workload(str(z["name"]), int(z["n"]), z["src"], z["dst"], z["ins_src"],
                            z["ins_dst"], z["q_u"], z["q_v"], int(z["draws"]))
        except Exception:
            pass
    w = make()
    try:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, name=w.name, n=w.n, src=w.src, dst=w.dst, ins_src=w.ins_src,
                 ins_dst=w.ins_dst, q_u=w.q_u, q_v=w.q_v, draws=w.draws)
        os.replace(tmp, path)
    except OSError:
        pass
    return w


def tiny_workload(seed: int = 1) -> Workload:
    """2^14 vertices, 8n draws, 1,000 uniform new edges, 10,000 uniform queries."""
    return make_rmat_workload("rmat14-tiny", 14, seed, draws=8 << 14, n_insert=1000,
                              insert_kind="uniform", n_query=10000, query_kind="uniform")


LJ_EDGES = 68_993_773


def lj_workload(seed: int = 1, n_insert: int = 100_000, n_query: int = 1_000_000,
                scale: int = 22, m_target: int = LJ_EDGES) -> Workload:
    """LiveJournal-shaped: 2^22 vertices, 68,993,773 unique edges, R-MAT insertions, mixed queries."""
    return make_rmat_workload(f"rmat{scale}-lj", scale, seed, m_target=m_target,
                              n_insert=n_insert, insert_kind="rmat", n_query=n_query,
                              query_kind="mixed")
