"""Pins of the oracle against brute force on small graphs.

The expected values here never use the oracle's own arithmetic: reachability comes from scipy's
shortest-path routine (finite distance = reachable, u reaches u), and every label, answer and
decision class is then written out from the paper's definitions as Python set operations:

* Definition 1: DL_in(x) = {l in L : l reaches x}, DL_out(x) = {l in L : x reaches l}.
* Definition 2 + hashing: BL_in(x) = {h(s) : s in S_in reaches x}, BL_out(x) = {h(t) : x reaches
  t in S_out}.
* Algorithm 2's rule order: self, Lemma 1 (DL hit), Lemma 2 (BL containment fails), Theorem 1,
  Theorem 2, then BFS (the answer is exact reachability).
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import dblgen
import oracle


def reach_matrix(n, src, dst):
    if n == 0:
        return np.zeros((0, 0), bool)
    a = csr_matrix((np.ones(len(src)), (np.asarray(src, np.int64), np.asarray(dst, np.int64))),
                   shape=(n, n))
    d = shortest_path(a, method="D", unweighted=True, directed=True)
    r = np.isfinite(d)
    np.fill_diagonal(r, True)
    return r


def distinct_degrees(n, src, dst):
    pairs = {(int(a), int(b)) for a, b in zip(src, dst) if a != b}
    indeg = np.zeros(n, np.int64)
    outdeg = np.zeros(n, np.int64)
    for a, b in pairs:
        outdeg[a] += 1
        indeg[b] += 1
    return indeg, outdeg


RANKS = {0: lambda p, s: p * s, 1: max, 2: min, 3: lambda p, s: p + s}


def expected_landmarks(n, src, dst, k, rank=0):
    indeg, outdeg = distinct_degrees(n, src, dst)
    f = RANKS[rank]
    order = sorted(range(n), key=lambda x: (-f(int(indeg[x]), int(outdeg[x])), x))
    return order[:min(k, n)]


def expected_leaves(n, src, dst, landmarks, r=0):
    indeg, outdeg = distinct_degrees(n, src, dst)
    lm = set(landmarks)
    if r:
        s = [x for x in range(n) if int(indeg[x]) * int(outdeg[x]) <= r and x not in lm]
        return s, s
    s_in = [x for x in range(n) if indeg[x] == 0 and x not in lm]
    s_out = [x for x in range(n) if outdeg[x] == 0 and x not in lm]
    return s_in, s_out


def expected_labels(R, landmarks, s_in, s_out, bucket):
    n = R.shape[0]
    dl_in = [{i for i, l in enumerate(landmarks) if R[l, x]} for x in range(n)]
    dl_out = [{i for i, l in enumerate(landmarks) if R[x, l]} for x in range(n)]
    bl_in = [{int(bucket[s]) for s in s_in if R[s, x]} for x in range(n)]
    bl_out = [{int(bucket[t]) for t in s_out if R[x, t]} for x in range(n)]
    return dl_in, dl_out, bl_in, bl_out


def as_sets(words):
    """Bit sets of a label array: uint64[n] or uint64[n, W] (bit i in word i // 64)."""
    if words.ndim == 1:
        return [{b for b in range(64) if (int(w) >> b) & 1} for w in words]
    return [{64 * j + b for j in range(words.shape[1]) for b in range(64)
             if (int(row[j]) >> b) & 1} for row in words]


def expected_query(R, lab, u, v, dl=True, bl=True):
    dl_in, dl_out, bl_in, bl_out = lab
    if u == v:
        return 1 | (oracle.CLASS_SELF << 1)
    if dl and dl_out[u] & dl_in[v]:
        return 1 | (oracle.CLASS_R1 << 1)
    if bl and not (bl_in[u] <= bl_in[v] and bl_out[v] <= bl_out[u]):
        return 0 | (oracle.CLASS_R2 << 1)
    if dl and dl_out[v] & dl_in[u]:
        return 0 | (oracle.CLASS_R3 << 1)
    if dl and ((dl_out[u] & dl_in[u]) or (dl_out[v] & dl_in[v])):
        return 0 | (oracle.CLASS_R4 << 1)
    ans = int(R[u, v])
    return ans | ((oracle.CLASS_BFS_TRUE if ans else oracle.CLASS_BFS_FALSE) << 1)


# ----------------------------------------------------------------------------- graph families

def g_er(n, p, seed, loops=False, dups=False):
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < p
    if not loops:
        np.fill_diagonal(mask, False)
    src, dst = np.nonzero(mask)
    if dups and len(src):
        extra = rng.integers(0, len(src), size=len(src) // 3 + 1)
        src = np.concatenate([src, src[extra]])
        dst = np.concatenate([dst, dst[extra]])
    return n, src.astype(np.uint32), dst.astype(np.uint32)


def g_dag(n, p, seed):
    rng = np.random.default_rng(seed)
    mask = np.triu(rng.random((n, n)) < p, 1)
    src, dst = np.nonzero(mask)
    return n, src.astype(np.uint32), dst.astype(np.uint32)


def g_chain(n, cycle=False):
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    if cycle and n > 1:
        src = np.append(src, n - 1).astype(np.uint32)
        dst = np.append(dst, 0).astype(np.uint32)
    return n, src, dst


def g_sccs(n_scc, size, bridges, seed):
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for c in range(n_scc):
        base = c * size
        for i in range(size):
            src.append(base + i)
            dst.append(base + (i + 1) % size)
        for _ in range(size):
            a, b = rng.integers(0, size, 2)
            src.append(base + a)
            dst.append(base + b)
    for _ in range(bridges):
        a, b = sorted(rng.integers(0, n_scc, 2))
        if a != b:
            src.append(a * size + rng.integers(0, size))
            dst.append(b * size + rng.integers(0, size))
    return n_scc * size, np.array(src, np.uint32), np.array(dst, np.uint32)


def g_rmat(scale, draws, seed):
    st = dblgen.RmatStream(scale, seed, expected_edges=draws)
    src, dst = st.next_edges(draws, draws)
    return 1 << scale, src, dst


def g_star(n, out=True):
    hub = np.zeros(n - 1, np.uint32)
    leaves = np.arange(1, n, dtype=np.uint32)
    return (n, hub, leaves) if out else (n, leaves, hub)


FAMILIES = [
    ("single", (1, np.zeros(0, np.uint32), np.zeros(0, np.uint32))),
    ("pair", (2, np.array([0], np.uint32), np.array([1], np.uint32))),
    ("isolated", (7, np.zeros(0, np.uint32), np.zeros(0, np.uint32))),
    ("er_sparse", g_er(60, 0.02, 1)),
    ("er_mid", g_er(80, 0.04, 2)),
    ("er_dense", g_er(40, 0.15, 3)),
    ("er_loops_dups", g_er(50, 0.05, 4, loops=True, dups=True)),
    ("dag", g_dag(70, 0.05, 5)),
    ("chain", g_chain(90)),
    ("cycle", g_chain(33, cycle=True)),
    ("sccs", g_sccs(6, 8, 9, 6)),
    ("star_out", g_star(30, True)),
    ("star_in", g_star(30, False)),
    ("rmat7", g_rmat(7, 600, 7)),
    ("rmat8", g_rmat(8, 1200, 8)),
]


def random_bucket(n, kp, seed):
    return np.random.default_rng(seed).integers(0, kp, size=n).astype(np.uint8)


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("k,kp", [(64, 64), (3, 4), (1, 1), (0, 2), (8, 64)])
def test_labels_and_queries_vs_definitions(name, g, k, kp):
    n, src, dst = g
    R = reach_matrix(n, src, dst)
    bucket = random_bucket(n, kp, n + k + kp)
    ix = oracle.OracleIndex(n, src, dst).build(k=k, kp=kp, bucket_table=bucket)
    lm = expected_landmarks(n, src, dst, k)
    assert list(ix.landmarks()) == lm
    s_in, s_out = expected_leaves(n, src, dst, lm)
    in_leaf, out_leaf, _ = ix.leaves()
    assert list(np.flatnonzero(in_leaf)) == s_in and list(np.flatnonzero(out_leaf)) == s_out
    exp = expected_labels(R, lm, s_in, s_out, bucket)
    got = [as_sets(w) for w in ix.labels()]
    for name_, e, g_ in zip(("DL_in", "DL_out", "BL_in", "BL_out"), exp, got):
        assert e == g_, name_
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    q = ix.query_dbl(u, v)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    assert np.array_equal(q, want)
    assert np.array_equal(ix.query_truth(u, v), R[u, v].astype(np.uint8))
    assert np.array_equal(ix.closure(), R)


@pytest.mark.parametrize("name,g", FAMILIES[3:], ids=[f[0] for f in FAMILIES[3:]])
@pytest.mark.parametrize("rank,r", [(1, 0), (2, 0), (3, 0), (0, 2), (3, 6)])
def test_selection_variants_vs_definitions(name, g, rank, r):
    """Table 3's landmark rankings and the leaf threshold r, against the definitions."""
    n, src, dst = g
    R = reach_matrix(n, src, dst)
    bucket = random_bucket(n, 8, n + rank)
    ix = oracle.OracleIndex(n, src, dst).build(k=5, kp=8, bucket_table=bucket, rank=rank,
                                               leaf_threshold=r)
    lm = expected_landmarks(n, src, dst, 5, rank)
    assert list(ix.landmarks()) == lm
    s_in, s_out = expected_leaves(n, src, dst, lm, r)
    exp = expected_labels(R, lm, s_in, s_out, bucket)
    assert [as_sets(w_) for w_ in ix.labels()] == list(exp)
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    assert np.array_equal(ix.query_dbl(u, v), want)


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("rules", [1, 2, 0])
def test_rule_ablations_vs_definitions(name, g, rules):
    """Table 4's ablations: DL only, BL only, neither; answers stay exact."""
    n, src, dst = g
    R = reach_matrix(n, src, dst)
    bucket = random_bucket(n, 4, n)
    ix = oracle.OracleIndex(n, src, dst).build(k=3, kp=4, bucket_table=bucket)
    lm = expected_landmarks(n, src, dst, 3)
    s_in, s_out = expected_leaves(n, src, dst, lm)
    exp = expected_labels(R, lm, s_in, s_out, bucket)
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    want = np.array([expected_query(R, exp, int(a), int(b), dl=bool(rules & 1),
                                    bl=bool(rules & 2)) for a, b in zip(u, v)], np.uint8)
    got = ix.query_rules(u, v, rules)
    assert np.array_equal(got, want)
    assert np.array_equal(got & 1, R[u, v].astype(np.uint8))


@pytest.mark.parametrize("name,g", [f for f in FAMILIES if f[0] in
                                    ("er_mid", "sccs", "rmat7", "rmat8", "star_out", "chain")],
                         ids=lambda x: x if isinstance(x, str) else "")
@pytest.mark.parametrize("k,kp", [(128, 64), (64, 256), (256, 128), (100, 128)])
def test_multiword_labels_vs_definitions(name, g, k, kp):
    """Labels longer than 64 bits (Table 5's sizes): labels, insertion and answers against the
    definitions."""
    n, src, dst = g
    bucket = random_bucket(n, kp, n + k)
    ix = oracle.OracleIndex(n, src, dst).build(k=k, kp=kp, bucket_table=bucket)
    lm = expected_landmarks(n, src, dst, k)
    assert list(ix.landmarks()) == lm
    s_in, s_out = expected_leaves(n, src, dst, lm)
    rng = np.random.default_rng(n)
    iu = rng.integers(0, n, 20).astype(np.uint32)
    iv = rng.integers(0, n, 20).astype(np.uint32)
    ix.insert(iu, iv)
    src = np.concatenate([src, iu]).astype(np.uint32)
    dst = np.concatenate([dst, iv]).astype(np.uint32)
    R = reach_matrix(n, src, dst)
    exp = expected_labels(R, lm, s_in, s_out, bucket)
    assert [as_sets(w_) for w_ in ix.labels()] == list(exp)
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    assert np.array_equal(ix.query_dbl(u, v), want)


def test_fibonacci_hash_range_and_spread():
    for kp in (1, 2, 4, 64, 256):
        hs = [oracle.fib_hash(x, kp) for x in range(4096)]
        assert min(hs) >= 0 and max(hs) < kp
        if kp > 1:
            counts = np.bincount(hs, minlength=kp)
            assert counts.min() > 0.7 * 4096 / kp and counts.max() < 1.3 * 4096 / kp
    # h(x) = floor(x * 0x9E3779B97F4A7C15 / 2^64 * kp) for kp a power of two
    for x in (0, 1, 2, 12345, 2**31 - 1, 2**32 - 1):
        frac = (x * 0x9E3779B97F4A7C15) % (1 << 64)
        assert oracle.fib_hash(x, 64) == frac >> 58
        assert oracle.fib_hash(x, 2) == frac >> 63
        assert oracle.fib_hash(x, 256) == frac >> 56


@pytest.mark.parametrize("seed", range(6))
def test_incremental_equals_definition_on_grown_graph(seed):
    """Algorithm 3 edge by edge == labels of the grown graph with the build's L, leaves and h."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 90))
    _, src, dst = g_er(n, float(rng.uniform(0.01, 0.05)), 200 + seed)
    kp = 8
    bucket = random_bucket(n, kp, seed)
    k = int(rng.integers(1, 10))
    ix = oracle.OracleIndex(n, src, dst).build(k=k, kp=kp, bucket_table=bucket)
    lm = list(ix.landmarks())
    s_in, s_out = expected_leaves(n, src, dst, lm)
    ins_u = rng.integers(0, n, 40).astype(np.uint32)
    ins_v = rng.integers(0, n, 40).astype(np.uint32)
    for a, b in zip(ins_u, ins_v):  # one at a time, checking after every insertion
        ix.insert([a], [b])
        src = np.append(src, a).astype(np.uint32)
        dst = np.append(dst, b).astype(np.uint32)
        R = reach_matrix(n, src, dst)
        exp = expected_labels(R, lm, s_in, s_out, bucket)
        got = [as_sets(w) for w in ix.labels()]
        assert list(exp) == got
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    q = ix.query_dbl(u, v)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    assert np.array_equal(q, want)


def test_batch_order_does_not_matter():
    n, src, dst = g_sccs(5, 6, 4, 11)
    rng = np.random.default_rng(5)
    iu = rng.integers(0, n, 30).astype(np.uint32)
    iv = rng.integers(0, n, 30).astype(np.uint32)
    ref = None
    for perm_seed in range(5):
        p = np.random.default_rng(perm_seed).permutation(30)
        ix = oracle.OracleIndex(n, src, dst).build(k=4, kp=4)
        ix.insert(iu[p], iv[p])
        labs = ix.labels()
        if ref is None:
            ref = labs
        for a, b in zip(ref, labs):
            assert np.array_equal(a, b)


def test_insert_rejects_out_of_range():
    ix = oracle.OracleIndex(4, [0, 1], [1, 2]).build(k=2, kp=2)
    with pytest.raises(ValueError):
        ix.insert([0], [4])


@pytest.mark.parametrize("seed", range(4))
def test_vertex_insertion_vs_definitions(seed):
    """New vertices (no edges, empty labels, not BL sources) then edges touching them: labels
    equal the definitions on the grown graph with the build's landmarks, leaves and hash."""
    rng = np.random.default_rng(300 + seed)
    n0 = int(rng.integers(15, 60))
    _, src, dst = g_er(n0, 0.05, 400 + seed)
    kp = 8
    bucket = random_bucket(n0, kp, seed)
    ix = oracle.OracleIndex(n0, src, dst).build(k=4, kp=kp, bucket_table=bucket)
    lm = list(ix.landmarks())
    s_in, s_out = expected_leaves(n0, src, dst, lm)
    add = int(rng.integers(1, 12))
    assert ix.add_vertices(add) == n0
    n = n0 + add
    full_bucket = np.concatenate([bucket, np.array([oracle.fib_hash(x, kp) for x in range(n0, n)],
                                                   np.uint8)])
    iu = rng.integers(0, n, 30).astype(np.uint32)
    iv = rng.integers(0, n, 30).astype(np.uint32)
    iu[:5] = n - 1  # the newest vertex gains out-edges
    ix.insert(iu, iv)
    src = np.concatenate([src, iu]).astype(np.uint32)
    dst = np.concatenate([dst, iv]).astype(np.uint32)
    R = reach_matrix(n, src, dst)
    exp = expected_labels(R, lm, s_in, s_out, full_bucket)
    assert [as_sets(w_) for w_ in ix.labels()] == list(exp)
    u = np.repeat(np.arange(n), n).astype(np.uint32)
    v = np.tile(np.arange(n), n).astype(np.uint32)
    want = np.array([expected_query(R, exp, int(a), int(b)) for a, b in zip(u, v)], np.uint8)
    assert np.array_equal(ix.query_dbl(u, v), want)
