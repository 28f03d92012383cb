"""dbl_query_batch_noalloc (scratch in a static device array, no allocation) against
dbl_query_batch on the same index, byte for byte, over the C ABI.

Two calls follow each other, the second on a smaller batch, so the second finds the array as the
first left it. A device cap at the bytes already in use makes any allocation by the library
fail, so the calls pass only if they allocate nothing.
"""
import numpy as np
import pytest
import torch

import dblgen
import oracle

pytestmark = pytest.mark.gpu

dbl = pytest.importorskip("paper_2101_09441_amd")


def dev(a):
    return dbl.to_device_ids(a)


def _noalloc(g, u, v, out):
    """Run the allocation-free entry point with the library capped at what it holds now."""
    lib = dbl.load_library()
    live, cached = dbl.live_bytes(), dbl.cached_bytes()
    dbl.set_device_limit(max(live, 1))
    try:
        g.query_noalloc(u, v, out)
    finally:
        dbl.set_device_limit(0)
    torch.cuda.synchronize()
    assert dbl.live_bytes() == live and dbl.cached_bytes() == cached
    return lib


def _check_pairs(g, o, u, v, sizes):
    """Calls in a row on prefixes of (u, v) of the given sizes; each equals dbl_query_batch and
    the oracle."""
    for m in sizes:
        du, dv = dev(u[:m]), dev(v[:m])
        want = g.query(du, dv).cpu().numpy()
        out = torch.full((m,), 0xAB, dtype=torch.uint8, device="cuda")
        _noalloc(g, du, dv, out)
        got = out.cpu().numpy()
        bad = np.flatnonzero(got != want)
        assert len(bad) == 0, (f"{len(bad)} of {m} answers differ, first {bad[:5]}: "
                               f"noalloc {got[bad[:5]]} query_batch {want[bad[:5]]}")
        assert np.array_equal(got, o.query_dbl(u[:m], v[:m], threads=8))


def test_noalloc_matches_query_batch_rmat():
    """2^14 R-MAT, 20,000 mixed pairs (78 label-kernel tiles and a ragged tail), then 3,001."""
    w = dblgen.make_rmat_workload("tiny", 14, 1, draws=8 << 14, n_insert=500,
                                  insert_kind="uniform", n_query=20000, query_kind="mixed")
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    _check_pairs(g, o, w.q_u, w.q_v, [20000, 3001])
    # after insertions the same two calls see the grown labels
    g.insert_edges(dev(w.ins_src), dev(w.ins_dst))
    o.insert(w.ins_src, w.ins_dst)
    _check_pairs(g, o, w.q_u, w.q_v, [12345, 1])
    g.close()


def test_noalloc_overflowing_slots_use_whole_device_bfs():
    """A chain with no landmarks and one BL bucket, 8-entry BFS queues: long searches leave
    their slot for the whole-device BFS inside the static array; then a small batch."""
    n = 3000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    g = dbl.Index.build(n, dev(src), dev(dst), num_landmarks=0, bl_bits=1, bfs_slots=4,
                        bfs_queue_cap=8)
    o = oracle.OracleIndex(n, src, dst).build(k=0, kp=1)
    rng = np.random.default_rng(11)
    u = rng.integers(0, n, 300).astype(np.uint32)
    v = rng.integers(0, n, 300).astype(np.uint32)
    u[:4] = [0, 10, 2000, 5]
    v[:4] = [n - 1, 12, 1000, 5]
    _check_pairs(g, o, u, v, [300, 7])
    g.close()


def test_noalloc_errors():
    w = dblgen.make_rmat_workload("err", 10, 2, draws=8 << 10, n_insert=0,
                                  insert_kind="uniform", n_query=0, query_kind="uniform")
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=4)
    out = torch.zeros(4, dtype=torch.uint8, device="cuda")
    # an id out of range: reported, the index is never modified by a query
    with pytest.raises(dbl.DblError) as e:
        g.query_noalloc(dev([0, 1, w.n, 3]), dev([1, 2, 3, 4]), out)
    assert e.value.status == dbl.DBL_ERR_VERTEX_RANGE
    # a batch too large for the static array is refused before any device work
    lib = dbl.load_library()
    u = dev([0])
    st = lib.dbl_query_batch_noalloc(g._handle(), 1 << 31, u.data_ptr(), u.data_ptr(),
                                     out.data_ptr(), None)
    assert st == dbl.DBL_ERR_INVALID_ARG
    # and the next call is exact again
    rng = np.random.default_rng(3)
    qu = rng.integers(0, w.n, 5000).astype(np.uint32)
    qv = rng.integers(0, w.n, 5000).astype(np.uint32)
    _check_pairs(g, o, qu, qv, [5000, 999])
    g.close()
