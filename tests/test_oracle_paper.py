"""Pins of the oracle against the values the paper prints for its running example.

Fixtures (tests/golden): Figure 1(b,c) labels, Figure 3(b,c) after inserting (v9,v2), and the
query examples of Section 3 (Examples 1 and 2). The graph drawing of Figure 1(a) is not in the
text; the edge set in fig1_graph.txt is a reconstruction whose closure reproduces every printed
label (the labels depend on reachability only).
"""
import numpy as np
import pytest

import oracle
from golden_io import bucket_word, examples, fig1_graph, fig1_labels, fig3_insert, landmark_word


def _fig1_index():
    n, src, dst = fig1_graph()
    landmarks, bucket, _ = fig1_labels()
    ix = oracle.OracleIndex(n, src, dst).build(k=2, kp=2, landmarks=landmarks, bucket_table=bucket)
    return ix


def test_fig1_landmark_selection_by_M():
    """Section 3.1 ranks by |Pre|*|Suc|; Example 1 uses L = {v5, v8} (M = 4 each)."""
    n, src, dst = fig1_graph()
    landmarks, _, _ = fig1_labels()
    ix = oracle.OracleIndex(n, src, dst)
    assert list(ix.select_landmarks(2)) == landmarks


def test_fig1_leaves():
    """Section 3.1, hash-set paragraph: the leaves are {v1, v2, v3, v10, v11}."""
    n, src, dst = fig1_graph()
    landmarks, bucket, _ = fig1_labels()
    ix = oracle.OracleIndex(n, src, dst).build(k=2, kp=2, landmarks=landmarks, bucket_table=bucket)
    in_leaf, out_leaf, _ = ix.leaves()
    assert set(np.flatnonzero(in_leaf) + 1) == {1, 2, 3}
    assert set(np.flatnonzero(out_leaf) + 1) == {10, 11}


def test_fig1_labels_match_paper():
    ix = _fig1_index()
    landmarks, _, rows = fig1_labels()
    dl_in, dl_out, bl_in, bl_out = ix.labels()
    for x, (e_dli, e_dlo, e_bli, e_blo) in rows.items():
        assert int(dl_in[x]) == landmark_word(e_dli, landmarks), f"DL_in(v{x+1})"
        assert int(dl_out[x]) == landmark_word(e_dlo, landmarks), f"DL_out(v{x+1})"
        assert int(bl_in[x]) == bucket_word(e_bli), f"BL_in(v{x+1})"
        assert int(bl_out[x]) == bucket_word(e_blo), f"BL_out(v{x+1})"


def test_fig3_insertion_matches_paper():
    ix = _fig1_index()
    landmarks, _, _ = fig1_labels()
    before = ix.labels()
    (u, v), rows = fig3_insert()
    ix.insert([u], [v])
    dl_in, dl_out, bl_in, bl_out = ix.labels()
    for x, (e_dli, e_bli) in rows.items():
        assert int(dl_in[x]) == landmark_word(e_dli, landmarks), f"DL_in(v{x+1})"
        assert int(bl_in[x]) == bucket_word(e_bli), f"BL_in(v{x+1})"
    changed = np.flatnonzero(dl_in != before[0])
    assert list(changed) == [1]  # only v2 changes (Figure 3(b))
    # DL_out and BL_out: u = v9 already has DL_out = {v5, v8} and reaches every out-leaf that
    # v2 reaches, so nothing upstream of v9 changes either.
    assert np.array_equal(dl_out, before[1]) and np.array_equal(bl_out, before[3])
    # after the insertion, v5 reaches v2 and the DL labels show it (Lemma 1)
    q = ix.query_dbl([4], [1])
    assert q[0] & 1 == 1 and q[0] >> 1 == oracle.CLASS_R1


@pytest.mark.parametrize("u,v,ans,why", examples())
def test_examples_of_section3(u, v, ans, why):
    ix = _fig1_index()
    q = int(ix.query_dbl([u], [v])[0])
    cls = q >> 1
    assert q & 1 == ans
    if why == "dl_hit":
        assert cls == oracle.CLASS_R1
    elif why == "not_dl":
        assert cls != oracle.CLASS_R1
    elif why == "bl_miss":
        assert cls == oracle.CLASS_R2
    elif why == "not_bl":
        assert cls not in (oracle.CLASS_R1, oracle.CLASS_R2)


def test_fig1_all_pairs_against_closure():
    ix = _fig1_index()
    n = ix.n
    u = np.repeat(np.arange(n), n)
    v = np.tile(np.arange(n), n)
    q = ix.query_dbl(u, v)
    truth = ix.closure()[u, v]
    assert np.array_equal(q & 1, truth.astype(np.uint8))


def test_fig1_class_histogram_cross_check():
    """Cross-check (not a paper value): the per-class counts over all 121 ordered pairs, before
    and after inserting (v9, v2), with the rule order self, Lemma 1, Lemma 2, Theorem 1,
    Theorem 2, BFS."""
    ix = _fig1_index()
    n = ix.n
    u = np.repeat(np.arange(n), n)
    v = np.tile(np.arange(n), n)
    hist = np.bincount(ix.query_dbl(u, v) >> 1, minlength=7)
    assert list(hist) == [11, 26, 64, 4, 6, 4, 6]
    (a, b), _ = fig3_insert()
    ix.insert([a], [b])
    hist = np.bincount(ix.query_dbl(u, v) >> 1, minlength=7)
    assert list(hist) == [11, 29, 64, 1, 8, 4, 4]
