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
