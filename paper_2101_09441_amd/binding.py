"""ctypes binding of libdbl (include/dbl.h): argument marshalling only.

Device memory and streams come from PyTorch tensors; every step of the method runs in the HIP
kernels of libdbl. The binding refuses to run without the compiled library.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbl.so")

DBL_OK, DBL_ERR_INVALID_ARG, DBL_ERR_VERTEX_RANGE, DBL_ERR_OUT_OF_MEMORY, DBL_ERR_DEVICE = range(5)
CLASS_NAMES = ["self", "dl_hit", "bl_miss", "thm1", "thm2", "bfs_true", "bfs_false"]

# every symbol declared in include/dbl.h
EXPORTS = [
    "dbl_default_options", "dbl_build", "dbl_add_vertices", "dbl_insert_edges",
    "dbl_insert_edges_each",
    "dbl_query_batch", "dbl_query_ctx_bytes", "dbl_query_ctx_create", "dbl_query_batch_ctx",
    "dbl_query_ctx_destroy", "dbl_query_batch_rules", "dbl_query_batch_noalloc",
    "dbl_read_labels", "dbl_get_landmarks", "dbl_get_leaves", "dbl_get_stats",
    "dbl_time_kernels", "dbl_read_kernel_times", "dbl_get_tuning", "dbl_set_tuning",
    "dbl_num_vertices", "dbl_label_words", "dbl_destroy",
    "dbl_release_cache", "dbl_set_cache_limit", "dbl_cached_bytes", "dbl_live_bytes",
    "dbl_set_device_limit",
    "dbl_status_str",
]


class DblOptions(ctypes.Structure):
    _fields_ = [
        ("num_landmarks", ctypes.c_uint32),
        ("bl_bits", ctypes.c_uint32),
        ("landmarks", ctypes.c_void_p),
        ("leaf_bucket", ctypes.c_void_p),
        ("leaf_flags", ctypes.c_void_p),
        ("slack_fraction", ctypes.c_float),
        ("slack_min", ctypes.c_uint32),
        ("bfs_slots", ctypes.c_uint32),
        ("bfs_queue_cap", ctypes.c_uint32),
        ("edges_unique", ctypes.c_uint32),
        ("landmark_rank", ctypes.c_uint32),
        ("leaf_threshold", ctypes.c_uint64),
        ("time_kernels", ctypes.c_char_p),
        ("pull_threshold", ctypes.c_uint32),
        ("pull_all_threshold", ctypes.c_uint32),
        ("row_fill", ctypes.c_uint32),
    ]


class DblStats(ctypes.Structure):
    _fields_ = [
        ("num_edges", ctypes.c_uint64),
        ("build_rounds", ctypes.c_uint64),
        ("insert_calls", ctypes.c_uint64),
        ("insert_rounds", ctypes.c_uint64),
        ("vertices_expanded", ctypes.c_uint64),
        ("edges_relaxed", ctypes.c_uint64),
        ("csr_regrows", ctypes.c_uint64),
        ("queries", ctypes.c_uint64),
        ("query_class", ctypes.c_uint64 * 7),
        ("bfs_vertices", ctypes.c_uint64),
        ("bfs_edges", ctypes.c_uint64),
        ("bfs_heavy", ctypes.c_uint64),
        ("pull_rounds", ctypes.c_uint64),
        ("server_requests", ctypes.c_uint64),
        ("server_busy_us", ctypes.c_double),
        ("batch_stalls", ctypes.c_uint64),
        ("build_long_bins", ctypes.c_uint64),
    ]


class DblTuning(ctypes.Structure):
    _fields_ = [
        ("small_batch", ctypes.c_uint32),
        ("local_max_frontier", ctypes.c_uint32),
        ("local_max_edges", ctypes.c_uint32),
        ("round_grid", ctypes.c_uint32),
        ("bfs_slots", ctypes.c_uint32),
        ("insert_server", ctypes.c_uint32),
        ("server_idle_us", ctypes.c_uint32),
        ("pull_threshold", ctypes.c_uint32),
        ("server_polls", ctypes.c_uint32),
        ("query_graph", ctypes.c_uint32),
        ("server_warm", ctypes.c_uint32),
        ("pull_all_threshold", ctypes.c_uint32),
        ("insert_persistent", ctypes.c_uint32),
        ("insert_graph", ctypes.c_uint32),
        ("batch_max_frontier", ctypes.c_uint32),
        ("gather_wait_us", ctypes.c_uint32),
        ("barrier_wait_us", ctypes.c_uint32),
        ("batch_grid", ctypes.c_uint32),
    ]


class DblKernelTime(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
    ]


class DblError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


_lib = None


def load_library():
    """Load libdbl.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python paper_2101_09441_amd/build.py` "
            "(or __graft_entry__.build()); the DBL index has no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    lib.dbl_default_options.argtypes = [ctypes.POINTER(DblOptions)]
    lib.dbl_default_options.restype = None
    lib.dbl_build.argtypes = [u32, u64, P, P, ctypes.POINTER(DblOptions), P, ctypes.POINTER(P)]
    lib.dbl_build.restype = i32
    lib.dbl_add_vertices.argtypes = [P, u32, ctypes.POINTER(u32), P]
    lib.dbl_add_vertices.restype = i32
    lib.dbl_insert_edges.argtypes = [P, u64, P, P, P]
    lib.dbl_insert_edges.restype = i32
    lib.dbl_insert_edges_each.argtypes = [P, u64, P, P, P, P]
    lib.dbl_insert_edges_each.restype = i32
    lib.dbl_query_batch.argtypes = [P, u64, P, P, P, P]
    lib.dbl_query_batch.restype = i32
    lib.dbl_query_batch_noalloc.argtypes = [P, u64, P, P, P, P]
    lib.dbl_query_batch_noalloc.restype = i32
    lib.dbl_query_ctx_bytes.argtypes = [P, u32, u32, u64]
    lib.dbl_query_ctx_bytes.restype = u64
    lib.dbl_query_ctx_create.argtypes = [P, u32, u32, ctypes.POINTER(P)]
    lib.dbl_query_ctx_create.restype = i32
    lib.dbl_query_batch_ctx.argtypes = [P, P, u64, P, P, P, P]
    lib.dbl_query_batch_ctx.restype = i32
    lib.dbl_query_batch_rules.argtypes = [P, P, u64, P, P, P, u32, P]
    lib.dbl_query_batch_rules.restype = i32
    lib.dbl_query_ctx_destroy.argtypes = [P]
    lib.dbl_query_ctx_destroy.restype = None
    lib.dbl_read_labels.argtypes = [P, P, P, P, P, P]
    lib.dbl_read_labels.restype = i32
    lib.dbl_get_landmarks.argtypes = [P, P, ctypes.POINTER(u32)]
    lib.dbl_get_landmarks.restype = i32
    lib.dbl_get_leaves.argtypes = [P, P, P]
    lib.dbl_get_leaves.restype = i32
    lib.dbl_get_stats.argtypes = [P, ctypes.POINTER(DblStats)]
    lib.dbl_get_stats.restype = i32
    lib.dbl_time_kernels.argtypes = [P, ctypes.c_char_p]
    lib.dbl_time_kernels.restype = i32
    lib.dbl_read_kernel_times.argtypes = [P, ctypes.POINTER(DblKernelTime), u32,
                                          ctypes.POINTER(u32)]
    lib.dbl_read_kernel_times.restype = i32
    lib.dbl_get_tuning.argtypes = [P, ctypes.POINTER(DblTuning)]
    lib.dbl_get_tuning.restype = i32
    lib.dbl_set_tuning.argtypes = [P, ctypes.POINTER(DblTuning)]
    lib.dbl_set_tuning.restype = i32
    lib.dbl_num_vertices.argtypes = [P]
    lib.dbl_num_vertices.restype = u32
    lib.dbl_label_words.argtypes = [P]
    lib.dbl_label_words.restype = u32
    lib.dbl_destroy.argtypes = [P]
    lib.dbl_destroy.restype = None
    lib.dbl_release_cache.argtypes = []
    lib.dbl_release_cache.restype = None
    lib.dbl_set_cache_limit.argtypes = [u64]
    lib.dbl_set_cache_limit.restype = None
    lib.dbl_cached_bytes.argtypes = []
    lib.dbl_cached_bytes.restype = u64
    lib.dbl_live_bytes.argtypes = []
    lib.dbl_live_bytes.restype = u64
    lib.dbl_set_device_limit.argtypes = [u64]
    lib.dbl_set_device_limit.restype = None
    lib.dbl_status_str.argtypes = [i32]
    lib.dbl_status_str.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_str(s: int) -> str:
    try:
        return load_library().dbl_status_str(s).decode()
    except Exception:
        return "status"


def _check(status: int, what: str):
    if status != DBL_OK:
        raise DblError(status, what)


def _ids(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name} must hold 32-bit vertex ids (int32 or uint32)")
    return t.contiguous()


try:  # the current stream's raw handle without building a Stream object
    _raw_stream = torch._C._cuda_getCurrentRawStream
except AttributeError:  # pragma: no cover - older torch
    _raw_stream = None


def _stream_ptr(stream, device=None) -> int:
    if stream is None:
        if _raw_stream is not None:
            idx = device.index if isinstance(device, torch.device) else device
            return int(_raw_stream(torch.cuda.current_device() if idx is None else idx))
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def release_cache() -> None:
    """Return every device / pinned block the library keeps for reuse to the driver."""
    load_library().dbl_release_cache()


def set_cache_limit(nbytes: int) -> None:
    """Cap the bytes the library keeps cached for reuse (0 = cache nothing)."""
    load_library().dbl_set_cache_limit(int(nbytes))


def cached_bytes() -> int:
    return int(load_library().dbl_cached_bytes())


def live_bytes() -> int:
    """Device bytes the library holds in use (indexes, query contexts, scratch)."""
    return int(load_library().dbl_live_bytes())


def set_device_limit(nbytes: int) -> None:
    """Cap the device bytes the library may hold in use (0 = no cap); an allocation beyond it
    fails as out of memory."""
    load_library().dbl_set_device_limit(int(nbytes))


def to_device_ids(a, device="cuda") -> torch.Tensor:
    """numpy/sequence of ids -> int32 device tensor (bit pattern of uint32)."""
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.uint32)).view(np.int32)
    return torch.from_numpy(arr.copy()).to(device)


class QueryContext:
    """Scratch for one in-flight query batch; several contexts let batches overlap on the device
    (each on its own stream, driven from its own host thread)."""

    def __init__(self, index: "Index", bfs_slots: int = 0, queue_cap: int = 0):
        self.index = index
        h = ctypes.c_void_p()
        with torch.cuda.device(index.device):
            _check(load_library().dbl_query_ctx_create(index._handle(), bfs_slots, queue_cap,
                                                       ctypes.byref(h)), "dbl_query_ctx_create")
        self._h = h

    def query(self, u: torch.Tensor, v: torch.Tensor, out: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
        u, v = _ids(u, "u"), _ids(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        if out is None:
            out = torch.empty(u.numel(), dtype=torch.uint8, device=u.device)
        elif out.dtype != torch.uint8 or out.numel() < u.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 tensor with room for every pair")
        if self._h is None or not self._h.value:
            raise RuntimeError("query context is closed")
        with torch.cuda.device(self.index.device):
            st = load_library().dbl_query_batch_ctx(self.index._handle(), self._h, u.numel(),
                                                    u.data_ptr(), v.data_ptr(), out.data_ptr(),
                                                    _stream_ptr(stream))
        _check(st, "dbl_query_batch_ctx")
        return out

    def query_rules(self, u: torch.Tensor, v: torch.Tensor, rules: int,
                    out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Queries on this context using only the labels in `rules` (1 = DL, 2 = BL, 3 = both)."""
        u, v = _ids(u, "u"), _ids(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        if out is None:
            out = torch.empty(u.numel(), dtype=torch.uint8, device=u.device)
        if self._h is None or not self._h.value:
            raise RuntimeError("query context is closed")
        with torch.cuda.device(self.index.device):
            st = load_library().dbl_query_batch_rules(self.index._handle(), self._h, u.numel(),
                                                      u.data_ptr(), v.data_ptr(), out.data_ptr(),
                                                      rules, _stream_ptr(stream))
        _check(st, "dbl_query_batch_rules")
        return out

    def close(self):
        if self._h is not None and self._h.value and self.index._h is not None \
                and self.index._h.value:
            with torch.cuda.device(self.index.device):
                load_library().dbl_query_ctx_destroy(self._h)
        self._h = None


class Index:
    """A DBL index resident on one GPU."""

    def __init__(self, handle: int, n: int, device: torch.device):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.device = device

    @classmethod
    def build(cls, n: int, src: torch.Tensor, dst: torch.Tensor, *, num_landmarks: int = 64,
              bl_bits: int = 64, landmarks=None, leaf_bucket=None, leaf_flags=None,
              slack_fraction: float = 0.25, slack_min: int = 4, bfs_slots: int = 0,
              bfs_queue_cap: int = 0, edges_unique: bool = False, landmark_rank: int = 0,
              leaf_threshold: int = 0, time_kernels: Optional[str] = None,
              pull_threshold: Optional[int] = None, pull_all_threshold: Optional[int] = None,
              row_fill: int = 0, stream=None) -> "Index":
        lib = load_library()
        src, dst = _ids(src, "src"), _ids(dst, "dst")
        if src.numel() != dst.numel():
            raise ValueError("src and dst differ in length")
        opt = DblOptions()
        lib.dbl_default_options(ctypes.byref(opt))
        opt.num_landmarks = num_landmarks
        opt.bl_bits = bl_bits
        keep = []
        if landmarks is not None:
            lm = np.ascontiguousarray(np.asarray(landmarks, dtype=np.uint32))
            keep.append(lm)
            opt.landmarks = lm.ctypes.data
        if leaf_bucket is not None:
            lb = np.ascontiguousarray(np.asarray(leaf_bucket, dtype=np.uint8))
            if lb.size != n:
                raise ValueError("leaf_bucket needs n entries")
            keep.append(lb)
            opt.leaf_bucket = lb.ctypes.data
        if leaf_flags is not None:
            lf = np.ascontiguousarray(np.asarray(leaf_flags, dtype=np.uint8))
            if lf.size != n:
                raise ValueError("leaf_flags needs n entries")
            keep.append(lf)
            opt.leaf_flags = lf.ctypes.data
        opt.slack_fraction = slack_fraction
        opt.slack_min = slack_min
        opt.bfs_slots = bfs_slots
        opt.bfs_queue_cap = bfs_queue_cap
        opt.edges_unique = 1 if edges_unique else 0
        opt.landmark_rank = landmark_rank
        opt.leaf_threshold = leaf_threshold
        if pull_threshold is not None:
            opt.pull_threshold = pull_threshold
        if pull_all_threshold is not None:
            opt.pull_all_threshold = pull_all_threshold
        opt.row_fill = row_fill
        if time_kernels:
            tk = time_kernels.encode()
            keep.append(tk)
            opt.time_kernels = tk
        out = ctypes.c_void_p()
        with torch.cuda.device(src.device):
            st = lib.dbl_build(n, src.numel(), src.data_ptr(), dst.data_ptr(), ctypes.byref(opt),
                               _stream_ptr(stream), ctypes.byref(out))
        _check(st, "dbl_build")
        return cls(out.value, n, src.device)

    def close(self):
        if self._h is not None and self._h.value:
            load_library().dbl_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("index is closed")
        return self._h

    def add_vertices(self, count: int, stream=None) -> int:
        """Append `count` vertices without edges; returns the first new id."""
        first = ctypes.c_uint32()
        with torch.cuda.device(self.device):
            st = load_library().dbl_add_vertices(self._handle(), count, ctypes.byref(first),
                                                 _stream_ptr(stream))
        _check(st, "dbl_add_vertices")
        self.n += count
        return int(first.value)

    def insert_edges(self, src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
        src, dst = _ids(src, "src"), _ids(dst, "dst")
        if src.numel() != dst.numel():
            raise ValueError("src and dst differ in length")
        # the library makes the index's device current itself
        st = load_library().dbl_insert_edges(self._handle(), src.numel(), src.data_ptr(),
                                             dst.data_ptr(), _stream_ptr(stream, self.device))
        _check(st, "dbl_insert_edges")

    def insert_edges_each(self, src: torch.Tensor, dst: torch.Tensor, latencies: bool = False,
                          stream=None):
        """Insert the edges one request at a time; optionally return per-request wall times (us)."""
        src, dst = _ids(src, "src"), _ids(dst, "dst")
        if src.numel() != dst.numel():
            raise ValueError("src and dst differ in length")
        lat = np.zeros(max(src.numel(), 1), dtype=np.float32) if latencies else None
        with torch.cuda.device(self.device):
            st = load_library().dbl_insert_edges_each(
                self._handle(), src.numel(), src.data_ptr(), dst.data_ptr(),
                None if lat is None else lat.ctypes.data, _stream_ptr(stream))
        _check(st, "dbl_insert_edges_each")
        return None if lat is None else lat[:src.numel()]

    def query(self, u: torch.Tensor, v: torch.Tensor, out: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
        """Answer bytes: bit 0 = u reaches v, bits 1-3 = decision class."""
        u, v = _ids(u, "u"), _ids(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        if out is None:
            out = torch.empty(u.numel(), dtype=torch.uint8, device=u.device)
        elif out.dtype != torch.uint8 or out.numel() < u.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 tensor with room for every pair")
        st = load_library().dbl_query_batch(self._handle(), u.numel(), u.data_ptr(),
                                            v.data_ptr(), out.data_ptr(),
                                            _stream_ptr(stream, self.device))
        _check(st, "dbl_query_batch")
        return out

    def query_noalloc(self, u: torch.Tensor, v: torch.Tensor, out: torch.Tensor,
                      stream=None) -> torch.Tensor:
        """dbl_query_batch_noalloc: the library allocates nothing; `out` is the caller's."""
        u, v = _ids(u, "u"), _ids(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        if out.dtype != torch.uint8 or out.numel() < u.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 tensor with room for every pair")
        with torch.cuda.device(self.device):
            st = load_library().dbl_query_batch_noalloc(self._handle(), u.numel(), u.data_ptr(),
                                                        v.data_ptr(), out.data_ptr(),
                                                        _stream_ptr(stream))
        _check(st, "dbl_query_batch_noalloc")
        return out

    def query_rules(self, u: torch.Tensor, v: torch.Tensor, rules: int,
                    out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Queries using only the labels in `rules` (1 = DL, 2 = BL, 3 = both)."""
        u, v = _ids(u, "u"), _ids(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        if out is None:
            out = torch.empty(u.numel(), dtype=torch.uint8, device=u.device)
        with torch.cuda.device(self.device):
            st = load_library().dbl_query_batch_rules(self._handle(), None, u.numel(),
                                                      u.data_ptr(), v.data_ptr(), out.data_ptr(),
                                                      rules, _stream_ptr(stream))
        _check(st, "dbl_query_batch_rules")
        return out

    def query_context(self, bfs_slots: int = 0, queue_cap: int = 0) -> QueryContext:
        return QueryContext(self, bfs_slots, queue_cap)

    def query_context_bytes(self, bfs_slots: int = 0, queue_cap: int = 0, batch: int = 0) -> int:
        return int(load_library().dbl_query_ctx_bytes(self._handle(), bfs_slots, queue_cap, batch))

    def label_words(self) -> int:
        """64-bit words per label: 1, 2 or 4 (labels of up to 64, 128, 256 bits)."""
        return int(load_library().dbl_label_words(self._handle()))

    def labels(self, stream=None):
        """(DL_in, DL_out, BL_in, BL_out) as int64 device tensors holding the bit patterns:
        shape (n,) for 64-bit labels, else (n, W) with bit i in word i // 64."""
        w = self.label_words()
        shape = (self.n,) if w == 1 else (self.n, w)
        outs = [torch.empty(shape, dtype=torch.int64, device=self.device) for _ in range(4)]
        with torch.cuda.device(self.device):
            st = load_library().dbl_read_labels(self._handle(), *[o.data_ptr() for o in outs],
                                                _stream_ptr(stream))
        _check(st, "dbl_read_labels")
        return tuple(outs)

    def labels_numpy(self):
        return tuple(t.cpu().numpy().view(np.uint64) for t in self.labels())

    def landmarks(self) -> np.ndarray:
        buf = np.zeros(256, dtype=np.uint32)
        k = ctypes.c_uint32()
        _check(load_library().dbl_get_landmarks(self._handle(), buf.ctypes.data, ctypes.byref(k)),
               "dbl_get_landmarks")
        return buf[:k.value].copy()

    def leaves(self):
        """(flags uint8[n]: bit 0 in S_in, bit 1 in S_out; bucket uint8[n])."""
        flags = np.zeros(self.n, dtype=np.uint8)
        bucket = np.zeros(self.n, dtype=np.uint8)
        with torch.cuda.device(self.device):
            _check(load_library().dbl_get_leaves(self._handle(), flags.ctypes.data,
                                                 bucket.ctypes.data), "dbl_get_leaves")
        return flags, bucket

    def tuning(self) -> dict:
        t = DblTuning()
        _check(load_library().dbl_get_tuning(self._handle(), ctypes.byref(t)), "dbl_get_tuning")
        return {name: getattr(t, name) for name, _ in DblTuning._fields_}

    def set_tuning(self, **kw) -> None:
        """Change tuning fields (small_batch, local_max_frontier, local_max_edges, round_grid,
        bfs_slots, insert_server, server_idle_us, pull_threshold, server_polls, query_graph,
        server_warm, pull_all_threshold, insert_persistent, insert_graph, batch_max_frontier,
        gather_wait_us, barrier_wait_us, batch_grid); results never change."""
        cur = self.tuning()
        bad = set(kw) - set(cur)
        if bad:
            raise KeyError(f"unknown tuning fields {sorted(bad)}")
        cur.update(kw)
        t = DblTuning(**cur)
        with torch.cuda.device(self.device):
            _check(load_library().dbl_set_tuning(self._handle(), ctypes.byref(t)),
                   "dbl_set_tuning")

    def time_kernels(self, kinds: Optional[str]) -> None:
        """Time launches of the given kernel kinds with HIP events ("all", a comma list, None)."""
        _check(load_library().dbl_time_kernels(self._handle(), kinds.encode() if kinds else None),
               "dbl_time_kernels")

    def kernel_times(self) -> dict:
        """{kind: {"launches", "total_ms", "avg_ms", "max_ms"}} for timed kinds."""
        buf = (DblKernelTime * 16)()
        cnt = ctypes.c_uint32()
        with torch.cuda.device(self.device):
            _check(load_library().dbl_read_kernel_times(self._handle(), buf, 16, ctypes.byref(cnt)),
                   "dbl_read_kernel_times")
        out = {}
        for i in range(cnt.value):
            r = buf[i]
            out[r.name.decode()] = {"launches": int(r.launches), "total_ms": r.total_ms,
                                    "avg_ms": r.total_ms / max(r.launches, 1), "max_ms": r.max_ms}
        return out

    def stats(self) -> dict:
        s = DblStats()
        with torch.cuda.device(self.device):
            _check(load_library().dbl_get_stats(self._handle(), ctypes.byref(s)), "dbl_get_stats")
        d = {name: getattr(s, name) for name, _ in DblStats._fields_ if name != "query_class"}
        d["query_class"] = {CLASS_NAMES[i]: int(s.query_class[i]) for i in range(7)}
        return d
