"""Pins of the oracle's large-graph view (CSR both ways) against brute force on small graphs.

``BigGraph.labels`` (one BFS per bit column), ``BigGraph.query_dbl`` (Algorithm 2 over given
labels) and ``BigGraph.query_bibfs`` (bidirectional BFS without labels) are what the at-scale GPU
parity test compares against. Here their results are checked against reachability from scipy's
shortest paths and against labels, answers and classes written out from the definitions as set
operations (the helpers of ``test_oracle_brute``), and on the 2^14-vertex workload against the
per-vertex-list oracle.
"""
import numpy as np
import pytest

import dblgen
import oracle
from test_oracle_brute import (FAMILIES, as_sets, expected_labels, expected_landmarks,
                               expected_leaves, expected_query, random_bucket, reach_matrix)


def _masks(n, s_in, s_out):
    a = np.zeros(n, np.uint8)
    b = np.zeros(n, np.uint8)
    a[np.asarray(s_in, dtype=np.int64)] = 1
    b[np.asarray(s_out, dtype=np.int64)] = 1
    return a, b


def _words(sets):
    out = np.zeros(len(sets), np.uint64)
    for x, s in enumerate(sets):
        for b in s:
            out[x] |= np.uint64(1) << np.uint64(b)
    return out


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("k,kp", [(64, 64), (3, 4), (8, 64), (0, 1)])
def test_big_view_vs_definitions(name, g, k, kp):
    n, src, dst = g
    R = reach_matrix(n, src, dst)
    bucket = random_bucket(n, kp, 3 * n + k + kp)
    lm = expected_landmarks(n, src, dst, k)
    s_in, s_out = expected_leaves(n, src, dst, lm)
    exp = expected_labels(R, lm, s_in, s_out, bucket)
    big = oracle.BigGraph(n, src, dst)
    mi, mo = _masks(n, s_in, s_out)
    got = big.labels(np.asarray(lm, np.uint32), mi, mo, bucket, kp=kp, threads=3)
    for what, e, w in zip(("DL_in", "DL_out", "BL_in", "BL_out"), exp, got):
        assert as_sets(w) == e, what
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    labs = tuple(_words(s) for s in exp)
    assert np.array_equal(big.query_dbl(labs, u, v, threads=2), want)
    assert np.array_equal(big.query_bibfs(u, v, threads=2), R[u, v].astype(np.uint8))
    big.close()


def test_big_view_agrees_with_list_oracle_on_rmat_workload():
    """Every label word, every answer byte and the bidirectional truth on the 2^14 workload
    (after its 1,000 insertions), against the per-vertex-list oracle."""
    w = dblgen.tiny_workload(1)
    src = np.concatenate([w.src, w.ins_src])
    dst = np.concatenate([w.dst, w.ins_dst])
    ix = oracle.OracleIndex(w.n, src, dst).build(threads=4)
    big = oracle.BigGraph(w.n, src, dst)
    lm = ix.landmarks()
    s_in, s_out, bucket = ix.leaves()
    labs = big.labels(lm, s_in, s_out, bucket, threads=4)
    for a, b in zip(labs, ix.labels()):
        assert np.array_equal(a, b)
    assert np.array_equal(big.query_dbl(labs, w.q_u, w.q_v, threads=4),
                          ix.query_dbl(w.q_u, w.q_v, threads=4))
    assert np.array_equal(big.query_bibfs(w.q_u, w.q_v, threads=4),
                          ix.query_truth(w.q_u, w.q_v, threads=4))


def test_big_view_rejects_bad_sizes():
    n, src, dst = FAMILIES[4][1]
    big = oracle.BigGraph(n, src, dst)
    z = np.zeros(n, np.uint8)
    with pytest.raises(ValueError):
        big.labels(np.array([n], np.uint32), z, z, z)            # landmark out of range
    with pytest.raises(ValueError):
        big.labels(np.array([0], np.uint32), z, z, z + 70, kp=64)  # bucket >= k'
    with pytest.raises(ValueError):
        big.query_bibfs([0], [n])
