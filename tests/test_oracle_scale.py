"""Oracle properties on the 2^14-vertex R-MAT workload (sizes the oracle finishes in seconds)."""
import numpy as np

import dblgen
import oracle


def _edge_monotone(labs, src, dst):
    dl_in, dl_out, bl_in, bl_out = labs
    # for every edge (a, b): fwd labels grow along the edge, bwd labels grow against it
    assert not np.any(dl_in[src] & ~dl_in[dst])
    assert not np.any(bl_in[src] & ~bl_in[dst])
    assert not np.any(dl_out[dst] & ~dl_out[src])
    assert not np.any(bl_out[dst] & ~bl_out[src])


def test_tiny_workload_invariants_and_answers():
    w = dblgen.tiny_workload(1)
    ix = oracle.OracleIndex(w.n, w.src, w.dst).build(k=64, kp=64)
    labs = ix.labels()
    _edge_monotone(labs, w.src, w.dst)
    lm = ix.landmarks()
    assert len(lm) == 64
    # seed bits: landmark i carries bit i in both DL labels
    for i, l in enumerate(lm):
        assert labs[0][l] >> np.uint64(i) & np.uint64(1) and labs[1][l] >> np.uint64(i) & np.uint64(1)
    in_leaf, out_leaf, bucket = ix.leaves()
    one = np.uint64(1)
    assert np.all((labs[2][in_leaf] >> bucket[in_leaf].astype(np.uint64)) & one)
    assert np.all((labs[3][out_leaf] >> bucket[out_leaf].astype(np.uint64)) & one)
    q = ix.query_dbl(w.q_u, w.q_v, threads=4)
    t = ix.query_truth(w.q_u, w.q_v, threads=4)
    assert np.array_equal(q & 1, t)
    cls = q >> 1
    assert np.all(t[cls == oracle.CLASS_R1] == 1)
    assert np.all(t[np.isin(cls, [oracle.CLASS_R2, oracle.CLASS_R3, oracle.CLASS_R4])] == 0)


def test_tiny_workload_incremental_equals_rebuild():
    w = dblgen.tiny_workload(1)
    ix = oracle.OracleIndex(w.n, w.src, w.dst).build(k=64, kp=64)
    in_leaf, out_leaf, bucket = ix.leaves()
    lm = ix.landmarks()
    ix.insert(w.ins_src, w.ins_dst)
    allsrc = np.concatenate([w.src, w.ins_src])
    alldst = np.concatenate([w.dst, w.ins_dst])
    flags = in_leaf.astype(np.uint8) | (out_leaf.astype(np.uint8) << 1)
    rb = oracle.OracleIndex(w.n, allsrc, alldst).build(k=64, kp=64, landmarks=lm,
                                                        bucket_table=bucket, leaf_flags=flags)
    for a, b in zip(ix.labels(), rb.labels()):
        assert np.array_equal(a, b)
    _edge_monotone(ix.labels(), allsrc, alldst)


def test_threads_do_not_change_labels():
    w = dblgen.tiny_workload(2)
    a = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=1).labels()
    b = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=6).labels()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_big_graph_view_agrees_with_definitions():
    """The large-graph view (CSR + one BFS per source set) against the per-vertex-list oracle,
    itself pinned against brute force: landmarks, leaves, hash, every label bit column, and
    plain reachability."""
    w = dblgen.tiny_workload(1)
    src = np.concatenate([w.src, w.ins_src])
    dst = np.concatenate([w.dst, w.ins_dst])
    big = oracle.BigGraph(w.n, src, dst)
    ix = oracle.OracleIndex(w.n, src, dst).build(threads=4)
    lm = big.landmarks(64)
    assert np.array_equal(lm, ix.landmarks())
    s_in, s_out, bucket = big.leaves(lm)
    oi, oo, ob = ix.leaves()
    assert np.array_equal(s_in, oi) and np.array_equal(s_out, oo) and np.array_equal(bucket, ob)
    dl_in, dl_out, bl_in, bl_out = ix.labels()
    one = np.uint64(1)
    for i in range(0, 64, 7):
        assert np.array_equal(big.reach([lm[i]], True), (dl_in >> np.uint64(i)) & one == 1)
        assert np.array_equal(big.reach([lm[i]], False), (dl_out >> np.uint64(i)) & one == 1)
    for j in range(0, 64, 5):
        srcs = np.flatnonzero(s_in & (bucket == j))
        assert np.array_equal(big.reach(srcs, True), (bl_in >> np.uint64(j)) & one == 1)
        tgts = np.flatnonzero(s_out & (bucket == j))
        assert np.array_equal(big.reach(tgts, False), (bl_out >> np.uint64(j)) & one == 1)
    t = big.query_truth(w.q_u, w.q_v, threads=4)
    assert np.array_equal(t, ix.query_truth(w.q_u, w.q_v, threads=4))
