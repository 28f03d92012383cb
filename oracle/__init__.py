"""DBL oracle — TEST INFRASTRUCTURE ONLY.

A plain CPU implementation of the DBL reachability index (arXiv 2101.09441), written from the
paper's definitions and Algorithms 1-3 in ``dbl_oracle.c`` and wrapped here with ctypes. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may use it; the GPU library never
imports or links it, and the two share no code.

Class codes of ``query_dbl`` (``out = answer | class << 1``):
0 self, 1 DL hit (Lemma 1), 2 BL miss (Lemma 2), 3 Theorem 1, 4 Theorem 2, 5 BFS true,
6 BFS false.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dbl_oracle.c")
# DBL_SANITIZE=1 selects a build instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (a library of its own name; the process must preload the ASan runtime, see
# tests/test_sanitizers.py).
_SANITIZE = os.environ.get("DBL_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined"]
_lib = None

CLASS_SELF, CLASS_R1, CLASS_R2, CLASS_R3, CLASS_R4, CLASS_BFS_TRUE, CLASS_BFS_FALSE = range(7)
CLASS_NAMES = ["self", "R1_dl_hit", "R2_bl_miss", "R3_thm1", "R4_thm2", "bfs_true", "bfs_false"]
RULES_DL, RULES_BL = 1, 2
RANK_PRODUCT, RANK_MAX, RANK_MIN, RANK_SUM = range(4)


def build() -> str:
    """Compile the oracle with gcc (always recompiles; instrumented under DBL_SANITIZE=1)."""
    tmp = _LIB + ".tmp"
    opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
    subprocess.check_call(["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp,
                           _SRC])
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
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.orc_new.restype = P
    lib.orc_new.argtypes = [u32, u64, P, P]
    lib.orc_free.argtypes = [P]
    lib.orc_free.restype = None
    lib.orc_build.argtypes = [P, u32, u32, P, P, P, u32]
    lib.orc_build.restype = i32
    lib.orc_select_landmarks.argtypes = [P, u32, P]
    lib.orc_select_landmarks.restype = u32
    lib.orc_hash.argtypes = [u32, u32]
    lib.orc_hash.restype = u32
    for name in ("orc_query_dbl", "orc_query_truth"):
        f = getattr(lib, name)
        f.argtypes = [P, u64, P, P, P, u32]
        f.restype = i32
    lib.orc_query_dbl_rules.argtypes = [P, u64, P, P, P, u32, u32]
    lib.orc_query_dbl_rules.restype = i32
    lib.orc_set_selection.argtypes = [P, u32, u64]
    lib.orc_set_selection.restype = None
    lib.orc_insert.argtypes = [P, u64, P, P]
    lib.orc_insert.restype = i32
    lib.orc_label_words.argtypes = [P, ctypes.POINTER(u32), ctypes.POINTER(u32)]
    lib.orc_label_words.restype = None
    lib.orc_read_labels.argtypes = [P, P, P, P, P]
    lib.orc_read_labels.restype = None
    lib.orc_landmarks.argtypes = [P, P]
    lib.orc_landmarks.restype = u32
    lib.orc_leaves.argtypes = [P, P, P, P]
    lib.orc_leaves.restype = None
    lib.orc_num_edges.argtypes = [P]
    lib.orc_num_edges.restype = u64
    lib.orc_closure.argtypes = [P, P]
    lib.orc_closure.restype = i32
    lib.orc_in_degree.argtypes = [P, u32]
    lib.orc_in_degree.restype = u32
    lib.orc_out_degree.argtypes = [P, u32]
    lib.orc_out_degree.restype = u32
    lib.orc_add_vertices.argtypes = [P, u32]
    lib.orc_add_vertices.restype = u32
    lib.orc_big_new.argtypes = [u32, u64, P, P]
    lib.orc_big_new.restype = P
    lib.orc_big_free.argtypes = [P]
    lib.orc_big_free.restype = None
    lib.orc_big_landmarks.argtypes = [P, u32, P]
    lib.orc_big_landmarks.restype = u32
    lib.orc_big_degrees.argtypes = [P, P, P]
    lib.orc_big_degrees.restype = None
    lib.orc_big_reach.argtypes = [P, u64, P, ctypes.c_int, P]
    lib.orc_big_reach.restype = ctypes.c_int64
    lib.orc_big_query_truth.argtypes = [P, u64, P, P, P, u32]
    lib.orc_big_query_truth.restype = i32
    lib.orc_big_labels.argtypes = [P, u32, P, u32, P, P, P, u32, u32, P, P, P, P]
    lib.orc_big_labels.restype = i32
    lib.orc_big_query_dbl.argtypes = [P, P, P, P, P, u64, P, P, P, u32]
    lib.orc_big_query_dbl.restype = i32
    lib.orc_big_query_bibfs.argtypes = [P, u64, P, P, P, u32]
    lib.orc_big_query_bibfs.restype = i32
    _lib = lib
    return lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def fib_hash(x: int, kp: int) -> int:
    """The oracle's leaf hash h(x) (Fibonacci hashing into kp buckets)."""
    return int(_load().orc_hash(x, kp))


class OracleIndex:
    """Graph + DBL labels held by the oracle."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        src, dst = _u32(src), _u32(dst)
        if len(src) != len(dst):
            raise ValueError("src/dst length mismatch")
        self.n = int(n)
        self._keep = (src, dst)
        self._h = lib.orc_new(self.n, len(src), src.ctypes.data, dst.ctypes.data)
        if not self._h:
            raise ValueError("orc_new failed (vertex id out of range or out of memory)")
        self.k = 0
        self.kp = 0

    def close(self):
        if self._h:
            _load().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- construction (Algorithm 1)
    def build(self, k: int = 64, kp: int = 64, landmarks=None, bucket_table=None,
              leaf_flags=None, threads: int = 1, rank: int = RANK_PRODUCT,
              leaf_threshold: int = 0) -> "OracleIndex":
        """Algorithm 1. ``leaf_flags``: optional uint8[n], bit 0 = in S_in, bit 1 = in S_out.
        ``rank``: landmark ranking (product, max, min, sum of |Pre| and |Suc|);
        ``leaf_threshold``: r of the generalised leaf rule (0 = zero in/out degree)."""
        lib = _load()
        lib.orc_set_selection(self._h, rank, leaf_threshold)
        lm = None if landmarks is None else _u32(landmarks)
        if lm is not None and len(lm) < min(k, self.n):
            raise ValueError("need k landmarks")
        bt = None if bucket_table is None else np.ascontiguousarray(bucket_table, dtype=np.uint8)
        lf = None if leaf_flags is None else np.ascontiguousarray(leaf_flags, dtype=np.uint8)
        rc = lib.orc_build(self._h, k, kp, None if lm is None else lm.ctypes.data,
                           None if bt is None else bt.ctypes.data,
                           None if lf is None else lf.ctypes.data, threads)
        if rc:
            raise ValueError("orc_build failed")
        self.k = min(k, self.n)
        self.kp = kp
        return self

    def select_landmarks(self, k: int) -> np.ndarray:
        out = np.zeros(max(k, 1), dtype=np.uint32)
        got = _load().orc_select_landmarks(self._h, k, out.ctypes.data)
        return out[:got].copy()

    def landmarks(self) -> np.ndarray:
        out = np.zeros(256, dtype=np.uint32)
        got = _load().orc_landmarks(self._h, out.ctypes.data)
        return out[:got].copy()

    def leaves(self):
        a = np.zeros(self.n, np.uint8)
        b = np.zeros(self.n, np.uint8)
        c = np.zeros(self.n, np.uint8)
        _load().orc_leaves(self._h, a.ctypes.data, b.ctypes.data, c.ctypes.data)
        return a.astype(bool), b.astype(bool), c

    def label_words(self):
        wd, wb = ctypes.c_uint32(), ctypes.c_uint32()
        _load().orc_label_words(self._h, ctypes.byref(wd), ctypes.byref(wb))
        return wd.value, wb.value

    def labels(self):
        """(DL_in, DL_out, BL_in, BL_out): uint64[n] for 64-bit labels, else uint64[n, words]
        (bit i in word i // 64)."""
        wd, wb = self.label_words()
        arrs = [np.zeros((self.n, w), dtype=np.uint64) for w in (wd, wd, wb, wb)]
        _load().orc_read_labels(self._h, *[a.ctypes.data for a in arrs])
        return tuple(a[:, 0].copy() if a.shape[1] == 1 else a for a in arrs)

    # -- queries (Algorithm 2)
    def _q(self, fn, u, v, threads):
        u, v = _u32(u), _u32(v)
        out = np.zeros(max(len(u), 1), dtype=np.uint8)
        rc = fn(self._h, len(u), u.ctypes.data, v.ctypes.data, out.ctypes.data, threads)
        if rc:
            raise ValueError("query failed (vertex id out of range?)")
        return out[:len(u)].copy()

    def query_dbl(self, u, v, threads: int = 1) -> np.ndarray:
        """Algorithm 2: answer | class << 1 per pair."""
        return self._q(_load().orc_query_dbl, u, v, threads)

    def query_rules(self, u, v, rules: int, threads: int = 1) -> np.ndarray:
        """Algorithm 2 using only the labels in ``rules`` (RULES_DL | RULES_BL)."""
        u, v = _u32(u), _u32(v)
        out = np.zeros(max(len(u), 1), dtype=np.uint8)
        rc = _load().orc_query_dbl_rules(self._h, len(u), u.ctypes.data, v.ctypes.data,
                                         out.ctypes.data, rules, threads)
        if rc:
            raise ValueError("query failed (vertex id out of range?)")
        return out[:len(u)].copy()

    def query_truth(self, u, v, threads: int = 1) -> np.ndarray:
        """Plain BFS reachability (no labels): 1 if u reaches v."""
        return self._q(_load().orc_query_truth, u, v, threads)

    # -- insertion (Algorithm 3)
    def insert(self, src, dst) -> "OracleIndex":
        src, dst = _u32(src), _u32(dst)
        rc = _load().orc_insert(self._h, len(src), src.ctypes.data, dst.ctypes.data)
        if rc:
            raise ValueError("orc_insert failed (vertex id out of range?)")
        return self

    def add_vertices(self, count: int) -> int:
        """Append `count` vertices without edges; returns the first new id."""
        first = _load().orc_add_vertices(self._h, count)
        if first == 0xFFFFFFFF:
            raise MemoryError("orc_add_vertices failed")
        self.n += count
        return int(first)

    def num_edges(self) -> int:
        return int(_load().orc_num_edges(self._h))

    def degrees(self):
        lib = _load()
        indeg = np.array([lib.orc_in_degree(self._h, x) for x in range(self.n)], dtype=np.uint32)
        outdeg = np.array([lib.orc_out_degree(self._h, x) for x in range(self.n)], dtype=np.uint32)
        return indeg, outdeg

    def closure(self) -> np.ndarray:
        """Boolean n x n reachability matrix by bitset Warshall (small n only)."""
        if self.n > 4096:
            raise ValueError("closure is for small graphs")
        words = (self.n + 63) // 64
        rows = np.zeros(self.n * words, dtype=np.uint64)
        _load().orc_closure(self._h, rows.ctypes.data)
        bits = np.unpackbits(rows.view(np.uint8).reshape(self.n, words * 8), axis=1,
                             bitorder="little")
        return bits[:, :self.n].astype(bool)


class BigGraph:
    """Oracle view of a large graph for sampled checks: CSR both ways, selection, the reachable
    set of a source set (one BFS of Algorithm 1), plain BFS reachability per pair."""

    def __init__(self, n: int, src, dst):
        src, dst = _u32(src), _u32(dst)
        self.n = int(n)
        self._h = _load().orc_big_new(self.n, len(src), src.ctypes.data, dst.ctypes.data)
        if not self._h:
            raise ValueError("orc_big_new failed (id out of range or out of memory)")

    def close(self):
        if self._h:
            _load().orc_big_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def landmarks(self, k: int = 64) -> np.ndarray:
        out = np.zeros(max(k, 1), dtype=np.uint32)
        got = _load().orc_big_landmarks(self._h, k, out.ctypes.data)
        return out[:got].copy()

    def degrees(self):
        indeg = np.zeros(self.n, np.uint32)
        outdeg = np.zeros(self.n, np.uint32)
        _load().orc_big_degrees(self._h, indeg.ctypes.data, outdeg.ctypes.data)
        return indeg, outdeg

    def leaves(self, landmarks, kp: int = 64):
        """(S_in mask, S_out mask, bucket) under the default leaf rule and Fibonacci hashing."""
        indeg, outdeg = self.degrees()
        lm = np.zeros(self.n, bool)
        lm[np.asarray(landmarks, dtype=np.int64)] = True
        bits = int(kp).bit_length() - 1
        x = np.arange(self.n, dtype=np.uint64)
        bucket = ((x * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(64 - bits)).astype(np.uint8) \
            if bits else np.zeros(self.n, np.uint8)
        return (indeg == 0) & ~lm, (outdeg == 0) & ~lm, bucket

    def reach(self, sources, forward: bool = True) -> np.ndarray:
        """Boolean mask of the vertices reached from the source set (sources included)."""
        s = _u32(sources)
        words = (self.n + 63) // 64
        bm = np.zeros(words, dtype=np.uint64)
        got = _load().orc_big_reach(self._h, len(s), s.ctypes.data, 1 if forward else 0,
                                    bm.ctypes.data)
        if got < 0:
            raise MemoryError("orc_big_reach failed")
        bits = np.unpackbits(bm.view(np.uint8), bitorder="little")[:self.n]
        return bits.astype(bool)

    def query_truth(self, u, v, threads: int = 1) -> np.ndarray:
        u, v = _u32(u), _u32(v)
        out = np.zeros(max(len(u), 1), dtype=np.uint8)
        rc = _load().orc_big_query_truth(self._h, len(u), u.ctypes.data, v.ctypes.data,
                                         out.ctypes.data, threads)
        if rc:
            raise ValueError("query failed")
        return out[:len(u)].copy()

    def labels(self, landmarks, s_in, s_out, bucket, kp: int = 64, threads: int = 1,
               on_label=None):
        """(DL_in, DL_out, BL_in, BL_out) as uint64[n] (k, k' <= 64) from one BFS per bit
        column (Definitions 1 and 2), given the landmarks, leaf masks and leaf hash. The labels
        are computed one after another; on_label(name) is called after each."""
        lm = _u32(landmarks)
        si = np.ascontiguousarray(s_in, dtype=np.uint8)
        so = np.ascontiguousarray(s_out, dtype=np.uint8)
        bk = np.ascontiguousarray(bucket, dtype=np.uint8)
        if len(si) != self.n or len(so) != self.n or len(bk) != self.n:
            raise ValueError("leaf masks and bucket need n entries")
        labs = [np.zeros(max(self.n, 1), dtype=np.uint64) for _ in range(4)]
        for i, name in enumerate(("DL_in", "DL_out", "BL_in", "BL_out")):
            rc = _load().orc_big_labels(self._h, len(lm), lm.ctypes.data, kp, si.ctypes.data,
                                        so.ctypes.data, bk.ctypes.data, 1 << i, threads,
                                        *[a.ctypes.data for a in labs])
            if rc:
                raise ValueError("orc_big_labels failed (bad sizes or out of memory)")
            if on_label is not None:
                on_label(name)
        return tuple(a[:self.n] for a in labs)

    def query_dbl(self, labels, u, v, threads: int = 1) -> np.ndarray:
        """Algorithm 2 on this graph with the given one-word labels: answer | class << 1."""
        labs = [np.ascontiguousarray(a, dtype=np.uint64) for a in labels]
        if any(len(a) != self.n for a in labs):
            raise ValueError("labels need n entries")
        u, v = _u32(u), _u32(v)
        out = np.zeros(max(len(u), 1), dtype=np.uint8)
        rc = _load().orc_big_query_dbl(self._h, *[a.ctypes.data for a in labs], len(u),
                                       u.ctypes.data, v.ctypes.data, out.ctypes.data, threads)
        if rc:
            raise ValueError("query failed")
        return out[:len(u)].copy()

    def query_bibfs(self, u, v, threads: int = 1) -> np.ndarray:
        """Reachability per pair by bidirectional BFS without labels: 1 if u reaches v."""
        u, v = _u32(u), _u32(v)
        out = np.zeros(max(len(u), 1), dtype=np.uint8)
        rc = _load().orc_big_query_bibfs(self._h, len(u), u.ctypes.data, v.ctypes.data,
                                         out.ctypes.data, threads)
        if rc:
            raise ValueError("query failed")
        return out[:len(u)].copy()


def build_index(n, src, dst, **kw) -> OracleIndex:
    return OracleIndex(n, src, dst).build(**kw)
