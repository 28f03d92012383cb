"""GPU parity: labels and answers of libdbl (through the C ABI) against the oracle, bit for bit.

Every expected value comes from the CPU oracle on the same seeded inputs. Labels are compared
word for word; answers and decision classes byte for byte (the class is a function of the exact
labels, so it is unique too).
"""
import numpy as np
import pytest
import torch

import dblgen
import oracle
from golden_io import fig1_graph, fig1_labels, fig3_insert
from test_oracle_brute import FAMILIES, random_bucket

pytestmark = pytest.mark.gpu

dbl = pytest.importorskip("paper_2101_09441_amd")


def dev(a):
    return dbl.to_device_ids(a)


def gpu_index(n, src, dst, **kw):
    return dbl.Index.build(n, dev(src), dev(dst), **kw)


def _words(a, w):
    """A label array as (n, w) words: (n,) is one word; missing high words are zero."""
    a = a.reshape(len(a), -1)
    out = np.zeros((len(a), w), dtype=np.uint64)
    out[:, :a.shape[1]] = a
    return out


def assert_labels_equal(gix, oix, what=""):
    g = gix.labels_numpy()
    o = oix.labels()
    for name, a, b in zip(("DL_in", "DL_out", "BL_in", "BL_out"), g, o):
        w = max(a.reshape(len(a), -1).shape[1], b.reshape(len(b), -1).shape[1])
        a, b = _words(a, w), _words(b, w)
        if not np.array_equal(a, b):
            bad = np.flatnonzero((a != b).any(axis=1))
            raise AssertionError(f"{what} {name} differs at {len(bad)} vertices, first {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")


def all_pairs(n):
    return (np.repeat(np.arange(n), n).astype(np.uint32),
            np.tile(np.arange(n), n).astype(np.uint32))


def assert_queries_equal(gix, oix, u, v, threads=8):
    got = gix.query(dev(u), dev(v)).cpu().numpy()
    want = oix.query_dbl(u, v, threads=threads)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{len(bad)} answers differ, first pairs "
                             f"{list(zip(u[bad[:5]], v[bad[:5]]))}: gpu {got[bad[:5]]} "
                             f"oracle {want[bad[:5]]}")
    return got


# ------------------------------------------------------------------ the paper's running example

def test_fig1_labels_queries_and_fig3_insert():
    n, src, dst = fig1_graph()
    landmarks, bucket, _ = fig1_labels()
    g = gpu_index(n, src, dst, num_landmarks=2, bl_bits=2, landmarks=landmarks, leaf_bucket=bucket)
    o = oracle.OracleIndex(n, src, dst).build(k=2, kp=2, landmarks=landmarks, bucket_table=bucket)
    assert_labels_equal(g, o, "Figure 1")
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)
    (a, b), _ = fig3_insert()
    g.insert_edges(dev([a]), dev([b]))
    o.insert([a], [b])
    assert_labels_equal(g, o, "Figure 3")
    assert_queries_equal(g, o, u, v)


def test_fig1_selection_on_gpu():
    n, src, dst = fig1_graph()
    landmarks, _, _ = fig1_labels()
    g = gpu_index(n, src, dst, num_landmarks=2, bl_bits=2)
    assert list(g.landmarks()) == landmarks
    flags, _ = g.leaves()
    assert set(np.flatnonzero(flags & 1) + 1) == {1, 2, 3}
    assert set(np.flatnonzero(flags & 2) + 1) == {10, 11}


# ------------------------------------------------------------------ small graph families

@pytest.mark.parametrize("name,gr", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("k,kp", [(64, 64), (3, 4), (0, 2)])
def test_families_build_and_all_pairs(name, gr, k, kp):
    n, src, dst = gr
    bucket = random_bucket(n, kp, n + k + kp)
    g = gpu_index(n, src, dst, num_landmarks=k, bl_bits=kp, leaf_bucket=bucket)
    o = oracle.OracleIndex(n, src, dst).build(k=k, kp=kp, bucket_table=bucket)
    assert list(g.landmarks()) == list(o.landmarks())
    flags, bk = g.leaves()
    oi, oo, ob = o.leaves()
    assert np.array_equal(flags & 1, oi.astype(np.uint8))
    assert np.array_equal((flags >> 1) & 1, oo.astype(np.uint8))
    assert np.array_equal(bk, ob)
    assert_labels_equal(g, o, name)
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("name,gr", FAMILIES[3:], ids=[f[0] for f in FAMILIES[3:]])
def test_families_insert_batches(name, gr):
    n, src, dst = gr
    rng = np.random.default_rng(7)
    iu = rng.integers(0, n, 60).astype(np.uint32)
    iv = rng.integers(0, n, 60).astype(np.uint32)
    g = gpu_index(n, src, dst, num_landmarks=6, bl_bits=8)
    o = oracle.OracleIndex(n, src, dst).build(k=6, kp=8)
    for lo, hi in [(0, 1), (1, 8), (8, 60)]:
        g.insert_edges(dev(iu[lo:hi]), dev(iv[lo:hi]))
        o.insert(iu[lo:hi], iv[lo:hi])
        assert_labels_equal(g, o, f"{name} after {hi}")
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("name,gr", FAMILIES, ids=[f[0] for f in FAMILIES])
@pytest.mark.parametrize("row_fill", [1, 2])
@pytest.mark.parametrize("unique", [False, True])
def test_row_fill_modes(name, gr, row_fill, unique):
    """Direct and LDS-assembled row fills (staging in the dedup table or in a buffer of its
    own): labels and all-pairs answers equal the oracle's."""
    n, src, dst = gr
    if unique:
        pairs = np.unique(np.stack([src, dst], 1), axis=0)
        src, dst = pairs[:, 0].copy(), pairs[:, 1].copy()
    g = gpu_index(n, src, dst, num_landmarks=64, bl_bits=64, row_fill=row_fill,
                  edges_unique=unique)
    o = oracle.OracleIndex(n, src, dst).build(k=64, kp=64)
    assert_labels_equal(g, o, f"{name} fill {row_fill}")
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("order", ["shuffled", "by_src", "by_dst"])
@pytest.mark.parametrize("slack_min", [0, 40, 3000])
def test_row_fill_assembled_sub_bins(slack_min, order):
    """Assembled fill over bins of several sub-bins: many short rows, rows wider than the LDS
    stage (filled directly) and sub-bins where no row starts; labels and queries as the oracle.
    Input sorted by one endpoint sends whole waves of the ingest's counters to one bin or key
    (one atomic per wave or per run) in that direction."""
    rng = np.random.default_rng(17 + slack_min)
    n = 20000
    src = rng.integers(0, n, 120000).astype(np.uint32)
    dst = rng.integers(0, n, 120000).astype(np.uint32)
    # hubs with rows longer than the stage, in and out; bins hold 8 vertices here, so the out-hub
    # 79 is the last row of its bin and leaves sub-bins where no row starts at the bin's end
    hub_dst = rng.integers(0, n, 30000).astype(np.uint32)
    src = np.concatenate([src, np.full(30000, 79, np.uint32), hub_dst])
    dst = np.concatenate([dst, hub_dst, np.full(30000, 12345, np.uint32)])
    perm = {"shuffled": rng.permutation(src.size),
            "by_src": np.lexsort((dst, src)),
            "by_dst": np.lexsort((src, dst))}[order]
    src, dst = src[perm], dst[perm]
    outs = {}
    for row_fill in (0, 1, 2):
        g = gpu_index(n, src, dst, num_landmarks=16, bl_bits=16, row_fill=row_fill,
                      slack_min=slack_min)
        outs[row_fill] = g
    o = oracle.OracleIndex(n, src, dst).build(k=16, kp=16, threads=8)
    u = rng.integers(0, n, 20000).astype(np.uint32)
    v = rng.integers(0, n, 20000).astype(np.uint32)
    for row_fill, g in outs.items():
        assert_labels_equal(g, o, f"fill {row_fill} slack {slack_min}")
        assert_queries_equal(g, o, u, v)
    # rows keep their slack: insertions after the build land in place and stay exact
    iu = rng.integers(0, n, 200).astype(np.uint32)
    iv = rng.integers(0, n, 200).astype(np.uint32)
    outs[2].insert_edges(dev(iu), dev(iv))
    o.insert(iu, iv)
    assert_labels_equal(outs[2], o, f"fill 2 slack {slack_min} after inserts")
    assert_queries_equal(outs[2], o, u, v)


# ------------------------------------------------------------------ memory cache

def test_memory_cache_reuse_and_release(tiny):
    """Blocks of a destroyed index are cached and reused by the next build of the same graph;
    labels stay the oracle's; releasing and a zero limit empty the cache."""
    w = tiny
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    dbl.release_cache()
    g = gpu_index(w.n, w.src, w.dst)
    g.query(dev(w.q_u[:1000]), dev(w.q_v[:1000]))
    g.close()
    held = dbl.cached_bytes()
    assert held > 0
    g = gpu_index(w.n, w.src, w.dst)
    assert dbl.cached_bytes() < held  # the build took blocks back out of the cache
    assert_labels_equal(g, o, "build on reused blocks")
    assert_queries_equal(g, o, w.q_u, w.q_v)
    g.close()
    dbl.release_cache()
    assert dbl.cached_bytes() == 0
    dbl.set_cache_limit(0)
    g = gpu_index(w.n, w.src, w.dst)
    g.close()
    assert dbl.cached_bytes() == 0
    dbl.set_cache_limit(64 << 30)


# ------------------------------------------------------------------ push and pull rounds

@pytest.mark.parametrize("pull,pull_all", [(0, 0), (1, 0), (1, 1), (1 << 20, 0)])
@pytest.mark.parametrize("name,gr", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_pull_rounds_families(name, gr, pull, pull_all):
    """Build rounds forced to push only (0), to pull any direction with frontier edges (1) with
    or without the frontier test (pull_all 0 / 1), or never to pull (2^20): labels and answers
    equal the oracle's."""
    n, src, dst = gr
    g = gpu_index(n, src, dst, num_landmarks=6, bl_bits=8, pull_threshold=pull,
                  pull_all_threshold=pull_all)
    o = oracle.OracleIndex(n, src, dst).build(k=6, kp=8)
    assert_labels_equal(g, o, f"{name} pull {pull} pull_all {pull_all}")
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("words", [1, 4])
def test_pull_rounds_rmat_equal_counts(words):
    """On a 2^16-vertex R-MAT graph with hub rows, builds that push only, pull whenever a
    direction has frontier edges, or follow the default threshold all give the oracle's labels
    (the least fixpoint; how many edges each relaxes depends on the schedule). Then grid-round
    insertion batches with pulls (tiny single-workgroup bounds)."""
    k, kp = (64, 64) if words == 1 else (200, 256)
    w = dblgen.make_rmat_workload(f"pr{words}", 16, 21, draws=16 << 16, n_insert=30000,
                                  insert_kind="rmat", n_query=50000, query_kind="mixed")
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(k=k, kp=kp, threads=8)
    stats = {}
    for pull, pull_all in ((0, 0), (1, 0), (128, 512), (1, 1)):
        g = gpu_index(w.n, w.src, w.dst, num_landmarks=k, bl_bits=kp, pull_threshold=pull,
                      pull_all_threshold=pull_all)
        assert g.label_words() == words
        assert_labels_equal(g, o, f"pull {pull} pull_all {pull_all}")
        stats[pull] = g.stats()
        g.close()
    assert stats[0]["pull_rounds"] == 0
    assert stats[1]["pull_rounds"] >= stats[128]["pull_rounds"] > 0
    g = gpu_index(w.n, w.src, w.dst, num_landmarks=k, bl_bits=kp, pull_threshold=1)
    g.set_tuning(small_batch=0, local_max_frontier=16, local_max_edges=256)
    o.insert(w.ins_src, w.ins_dst)
    for lo in range(0, 30000, 10000):
        g.insert_edges(dev(w.ins_src[lo:lo + 10000]), dev(w.ins_dst[lo:lo + 10000]))
    assert_labels_equal(g, o, "insertion rounds after a pulled build")
    assert_queries_equal(g, o, w.q_u, w.q_v)


@pytest.mark.parametrize("form", [dict(insert_persistent=0), dict(batch_max_frontier=16)])
@pytest.mark.parametrize("pull_all", [0, 1])
def test_pull_rounds_in_insertion_batches(pull_all, form):
    """Insertion batches on a 2^12-vertex graph with the single-workgroup bounds tiny, so the
    batches propagate in grid rounds, and the threshold at its minimum, so those rounds pull
    (with and without the frontier test): in the multi-launch form, and in the persistent form
    with every frontier above 16 entries handed to the host's rounds."""
    w = dblgen.make_rmat_workload("pri", 12, 5, draws=8 << 12, n_insert=6000,
                                  insert_kind="uniform", n_query=20000, query_kind="mixed")
    g = gpu_index(w.n, w.src, w.dst, pull_threshold=1, pull_all_threshold=pull_all)
    g.set_tuning(small_batch=0, local_max_frontier=4, local_max_edges=32, **form)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    built = g.stats()["pull_rounds"]
    for lo in range(0, 6000, 1500):
        g.insert_edges(dev(w.ins_src[lo:lo + 1500]), dev(w.ins_dst[lo:lo + 1500]))
        o.insert(w.ins_src[lo:lo + 1500], w.ins_dst[lo:lo + 1500])
        assert_labels_equal(g, o, f"after {lo + 1500} insertions")
    assert g.stats()["pull_rounds"] > built
    assert_queries_equal(g, o, w.q_u, w.q_v)


# ------------------------------------------------------------------ labels longer than 64 bits

@pytest.mark.parametrize("k,kp,words", [(65, 2, 2), (128, 128, 2), (3, 256, 4), (200, 256, 4),
                                        (256, 64, 4)])
def test_multiword_labels_build_insert_query(k, kp, words):
    """k landmarks and k' buckets beyond one 64-bit word: labels word for word, answers and
    classes byte for byte, through a build, single-workgroup batches, a grid batch and
    single-edge requests (the device-fed stream, then the request server)."""
    w = dblgen.make_rmat_workload(f"mw{k}_{kp}", 11, 4, draws=6 << 11, n_query=30000,
                                  query_kind="mixed")
    bucket = random_bucket(w.n, kp, k + kp)
    g = gpu_index(w.n, w.src, w.dst, num_landmarks=k, bl_bits=kp, leaf_bucket=bucket)
    assert g.label_words() == words
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(k=k, kp=kp, bucket_table=bucket, threads=8)
    assert list(g.landmarks()) == list(o.landmarks())
    assert_labels_equal(g, o, "build")
    assert_queries_equal(g, o, w.q_u, w.q_v)
    rng = np.random.default_rng(k * 1000 + kp)
    iu = rng.integers(0, w.n, 6000).astype(np.uint32)
    iv = rng.integers(0, w.n, 6000).astype(np.uint32)
    for lo, hi in [(0, 1), (1, 100), (100, 6000)]:
        g.insert_edges(dev(iu[lo:hi]), dev(iv[lo:hi]))
        o.insert(iu[lo:hi], iv[lo:hi])
        assert_labels_equal(g, o, f"after {hi} insertions")
    ju = rng.integers(0, w.n, 400).astype(np.uint32)
    jv = rng.integers(0, w.n, 400).astype(np.uint32)
    for server, lo, hi in ((2, 0, 200), (1, 200, 400)):
        g.set_tuning(insert_server=server)
        g.insert_edges_each(dev(ju[lo:hi]), dev(jv[lo:hi]))
        o.insert(ju[lo:hi], jv[lo:hi])
        assert_labels_equal(g, o, f"after single-edge requests (form {server})")
    assert_queries_equal(g, o, w.q_u, w.q_v)
    for rules in (1, 2):
        got = g.query_rules(dev(w.q_u), dev(w.q_v), rules).cpu().numpy()
        assert np.array_equal(got, o.query_rules(w.q_u, w.q_v, rules, threads=8))


def test_multiword_default_selection_and_hash():
    """Top-256 landmark selection (ties by id) and the Fibonacci hash into 256 buckets."""
    w = dblgen.make_rmat_workload("mwsel", 12, 3, draws=8 << 12)
    g = gpu_index(w.n, w.src, w.dst, num_landmarks=256, bl_bits=256)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(k=256, kp=256, threads=8)
    assert list(g.landmarks()) == list(o.landmarks())
    _, bk = g.leaves()
    assert np.array_equal(bk, o.leaves()[2])
    assert_labels_equal(g, o, "k = k' = 256")


def test_multiword_small_bfs_slots_overflow():
    """The slot BFS and the whole-device BFS with multi-word prunes: on a 3000-vertex chain with
    k = 130 the landmarks are vertices 1..130, so q(u, 2999) for u > 130 is left to a BFS that
    walks the chain and outgrows a queue of 8 entries."""
    n = 3000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    g = gpu_index(n, src, dst, num_landmarks=130, bl_bits=256, bfs_slots=4, bfs_queue_cap=8)
    o = oracle.OracleIndex(n, src, dst).build(k=130, kp=256)
    assert_labels_equal(g, o, "chain")
    u = np.concatenate([np.arange(200, 2999, 97), np.full(20, 2999)]).astype(np.uint32)
    v = np.concatenate([np.full(len(range(200, 2999, 97)), 2999), np.arange(20) * 101]
                       ).astype(np.uint32)
    got = assert_queries_equal(g, o, u, v)
    assert ((got >> 1) == 5).sum() > 0
    assert g.stats()["bfs_heavy"] > 0
    w = dblgen.make_rmat_workload("mwbfs", 11, 4, draws=6 << 11, n_query=5000,
                                  query_kind="mixed")
    g = gpu_index(w.n, w.src, w.dst, num_landmarks=130, bl_bits=256, bfs_slots=4,
                  bfs_queue_cap=8)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(k=130, kp=256, threads=8)
    assert_queries_equal(g, o, w.q_u, w.q_v)


@pytest.mark.parametrize("rank,r", [(1, 0), (2, 0), (3, 0), (0, 3)])
def test_selection_variants(rank, r):
    """Table 3's landmark rankings and the leaf threshold r."""
    w = dblgen.make_rmat_workload("sv", 11, 4, draws=8 << 11, n_query=20000,
                                  query_kind="mixed")
    g = gpu_index(w.n, w.src, w.dst, landmark_rank=rank, leaf_threshold=r)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(rank=rank, leaf_threshold=r)
    assert list(g.landmarks()) == list(o.landmarks())
    assert_labels_equal(g, o, f"rank {rank} r {r}")
    assert_queries_equal(g, o, w.q_u, w.q_v)


@pytest.mark.parametrize("rules", [1, 2, 0, 3])
def test_rule_ablations(tiny, rules):
    """Table 4's ablations on the 2^14 workload: DL only, BL only, neither, both."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    got = g.query_rules(dev(w.q_u), dev(w.q_v), rules).cpu().numpy()
    want = o.query_rules(w.q_u, w.q_v, rules, threads=8)
    assert np.array_equal(got, want)


def test_default_hash_matches_oracle():
    w = dblgen.make_rmat_workload("h", 10, 5, draws=8 << 10)
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build()
    _, bk = g.leaves()
    _, _, ob = o.leaves()
    assert np.array_equal(bk, ob)
    assert_labels_equal(g, o, "default hash")


# ------------------------------------------------------------------ the 2^14-vertex workload

@pytest.fixture(scope="module")
def tiny():
    return dblgen.tiny_workload(1)


def test_tiny_build_labels(tiny):
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    assert list(g.landmarks()) == list(o.landmarks())
    assert_labels_equal(g, o, "tiny build")


def test_tiny_single_insertions_then_queries(tiny):
    """1,000 uniform new edges inserted one at a time; labels checked after every insertion."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    su, sv = dev(w.ins_src), dev(w.ins_dst)
    for i in range(len(w.ins_src)):
        g.insert_edges(su[i:i + 1], sv[i:i + 1])
        o.insert(w.ins_src[i:i + 1], w.ins_dst[i:i + 1])
        assert_labels_equal(g, o, f"after insertion {i}")
    got = assert_queries_equal(g, o, w.q_u, w.q_v)
    truth = o.query_truth(w.q_u, w.q_v, threads=8)
    assert np.array_equal(got & 1, truth)


def test_tiny_insert_each_equals_single_calls(tiny):
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    lat = g.insert_edges_each(dev(w.ins_src), dev(w.ins_dst), latencies=True)
    o.insert(w.ins_src, w.ins_dst)
    # the default form's latencies are device clock ticks (10 ns): a quick request may take none
    assert lat.shape == (len(w.ins_src),) and np.all(lat >= 0) and lat.sum() > 0
    assert_labels_equal(g, o, "insert_each")
    assert g.stats()["insert_calls"] == len(w.ins_src)
    with pytest.raises(dbl.DblError):
        g.insert_edges_each(dev([1, 2, w.n]), dev([3, 4, 5]))


@pytest.mark.parametrize("server,idle_us,polls", [(0, 200000, 4), (1, 0, 4), (1, 200000, 1),
                                                  (2, 200000, 4)])
def test_insert_each_forms(tiny, server, idle_us, polls):
    """One launch per request; the request server with a zero idle limit (a launch ends as soon
    as the next request is not there yet, so most requests start a new launch); the server
    reading its doorbell one read at a time; the device-fed stream."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    g.set_tuning(insert_server=server, server_idle_us=idle_us, server_polls=polls)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    k = 300
    lat = g.insert_edges_each(dev(w.ins_src[:k]), dev(w.ins_dst[:k]), latencies=True)
    o.insert(w.ins_src[:k], w.ins_dst[:k])
    # the stream's latencies are device clock ticks (10 ns): a quick request may take none
    assert np.all(lat > 0) if server != 2 else (np.all(lat >= 0) and lat.sum() > 0)
    assert_labels_equal(g, o, f"server {server} idle {idle_us} polls {polls}")
    assert g.stats()["insert_calls"] == k


@pytest.mark.parametrize("server", [1, 2])
def test_insert_each_server_hands_back_to_host(tiny, server):
    """Requests that fill a row (no slack) or grow a frontier past one workgroup (tiny local
    bounds) end the server launch (request server or device-fed stream); the host regrows the
    CSR or runs grid rounds, and a new launch serves the rest."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst, slack_fraction=0.0, slack_min=0)
    g.set_tuning(local_max_frontier=4, local_max_edges=64, insert_server=server)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    g.insert_edges_each(dev(w.ins_src), dev(w.ins_dst))
    o.insert(w.ins_src, w.ins_dst)
    st = g.stats()
    assert st["csr_regrows"] > 0 and st["insert_rounds"] > 0
    assert_labels_equal(g, o, "server with host hand-offs")
    assert_queries_equal(g, o, w.q_u, w.q_v)


@pytest.mark.parametrize("server", [1, 2])
def test_insert_each_stops_at_bad_id(tiny, server):
    """A request with an out-of-range id fails; the requests before it stay applied, the ones
    after it are not run, and the next call serves normally (request server or device-fed
    stream; in the stream the bad request sits inside a window of requests read together)."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    g.set_tuning(insert_server=server)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    a = np.array(list(w.ins_src[:10]) + [w.n] + list(w.ins_src[10:15]), dtype=np.uint32)
    b = np.array(list(w.ins_dst[:10]) + [0] + list(w.ins_dst[10:15]), dtype=np.uint32)
    with pytest.raises(dbl.DblError):
        g.insert_edges_each(dev(a), dev(b))
    o.insert(w.ins_src[:10], w.ins_dst[:10])
    assert g.stats()["insert_calls"] == 10
    assert_labels_equal(g, o, "stopped at the bad id")
    g.insert_edges_each(dev(w.ins_src[10:200]), dev(w.ins_dst[10:200]))
    o.insert(w.ins_src[10:200], w.ins_dst[10:200])
    assert_labels_equal(g, o, "served after the failure")
    # ids of all ones, as the first request and after a good one
    full = np.uint32(0xFFFFFFFF)
    for k in (0, 1):
        a = np.array(list(w.ins_src[200:200 + k]) + [full], dtype=np.uint32)
        b = np.array(list(w.ins_dst[200:200 + k]) + [full], dtype=np.uint32)
        with pytest.raises(dbl.DblError):
            g.insert_edges_each(dev(a), dev(b))
        o.insert(w.ins_src[200:200 + k], w.ins_dst[200:200 + k])
    assert_labels_equal(g, o, "refused ids of all ones")
    g.insert_edges_each(dev(w.ins_src[201:300]), dev(w.ins_dst[201:300]))
    o.insert(w.ins_src[201:300], w.ins_dst[201:300])
    assert_labels_equal(g, o, "served after ids of all ones")


@pytest.mark.parametrize("slack", [0, 3])
def test_insert_stream_repeated_rows_and_full_rows(slack):
    """The device-fed stream on requests that keep hitting the same rows: five hubs as tails and
    heads, and one whole window on a single row, so a window's later requests take their row's
    degree from the earlier ones; self-loops and repeated edges; rows that fill up inside a
    window (no slack, or three free slots), which hand the request to the host. Labels and
    answers equal the oracle's; every request that is not a self-loop stores one entry (the
    library keeps repeated edges, the oracle drops them)."""
    rng = np.random.default_rng(31)
    n = 3000
    src = rng.integers(0, n, 12000).astype(np.uint32)
    dst = rng.integers(0, n, 12000).astype(np.uint32)
    g = gpu_index(n, src, dst, num_landmarks=8, bl_bits=16, slack_fraction=0.0, slack_min=slack)
    g.set_tuning(insert_server=2)
    o = oracle.OracleIndex(n, src, dst).build(k=8, kp=16, threads=8)
    hubs = np.array([3, 77, 1500, 2999, 42], np.uint32)
    k = 4000
    a = rng.integers(0, n, k).astype(np.uint32)
    b = rng.integers(0, n, k).astype(np.uint32)
    sel = rng.random(k)
    a[sel < 0.4] = hubs[rng.integers(0, 5, int((sel < 0.4).sum()))]
    m = (sel >= 0.4) & (sel < 0.7)
    b[m] = hubs[rng.integers(0, 5, int(m.sum()))]
    a[sel > 0.97] = b[sel > 0.97]              # self-loops
    a[96:160] = 77                             # windows of requests on one row
    b[300:340] = 1500
    a[500:510], b[500:510] = a[499], b[499]    # one edge ten more times
    stored = g.stats()["num_edges"]
    lat = g.insert_edges_each(dev(a), dev(b), latencies=True)
    o.insert(a, b)
    assert_labels_equal(g, o, f"stream, slack {slack}")
    st = g.stats()
    assert st["num_edges"] == stored + int((a != b).sum())
    assert st["insert_calls"] == k and st["server_requests"] >= k
    if slack == 0:
        assert st["csr_regrows"] > 0
    assert lat.shape == (k,) and np.all(lat >= 0) and lat.sum() > 0
    u = rng.integers(0, n, 5000).astype(np.uint32)
    v = rng.integers(0, n, 5000).astype(np.uint32)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("server", [2, 1])
def test_insert_each_chain_and_hub(server):
    """Single-edge requests whose propagation is long or wide: a 20,000-vertex path closed into
    a cycle (thousands of rounds, all small enough for one wave in the stream), then requests
    that reach a hub of 60,000 out-edges (too many edges for one wave: the workgroup's rounds
    take over) and lead back from its leaves. Labels after each request and the answers equal
    the oracle's."""
    n = 20000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    hub = np.full(60000, n, dtype=np.uint32)
    leaves = np.arange(n + 1, n + 60001, dtype=np.uint32)
    nn = n + 60001
    bsrc = np.concatenate([src, hub])
    bdst = np.concatenate([dst, leaves])
    g = gpu_index(nn, bsrc, bdst, num_landmarks=4, bl_bits=8)
    g.set_tuning(insert_server=server)
    o = oracle.OracleIndex(nn, bsrc, bdst).build(k=4, kp=8, threads=8)
    steps = [([n - 1, 5], [0, 17]),            # closes the cycle
             ([100, 7], [n, 3]),               # the cycle now reaches the hub
             ([n + 5, n + 70], [n + 9, 250])]  # leaves of the hub reach back into the cycle
    for a, b in steps:
        g.insert_edges_each(dev(a), dev(b))
        o.insert(a, b)
        assert_labels_equal(g, o, f"server {server} after {a}->{b}")
    rng = np.random.default_rng(2)
    u = rng.integers(0, nn, 4000).astype(np.uint32)
    v = rng.integers(0, nn, 4000).astype(np.uint32)
    assert_queries_equal(g, o, u, v)


@pytest.mark.parametrize("server", [2, 1])
def test_insert_each_label_bit_31(server):
    """Landmarks 0..63 fixed in id order, so landmark 31 is DL bit 31. Vertex 100 is reached by
    landmark 31 alone; the request (100, 101) gives 101 exactly bit 31 and the rounds carry it
    on to 102 and 103 (in the stream, by the single wave: a label word whose low half has bit
    31 set must reach the targets unchanged, bits 32..63 untouched). Labels equal the
    oracle's."""
    n = 200
    src = np.array([31, 101, 102, 150], dtype=np.uint32)
    dst = np.array([100, 102, 103, 151], dtype=np.uint32)
    lm = list(range(64))
    g = gpu_index(n, src, dst, num_landmarks=64, bl_bits=1, landmarks=lm)
    g.set_tuning(insert_server=server)
    o = oracle.OracleIndex(n, src, dst).build(k=64, kp=1, landmarks=lm)
    g.insert_edges_each(dev([100]), dev([101]))
    o.insert([100], [101])
    assert_labels_equal(g, o, f"form {server}")
    dl_in = g.labels_numpy()[0].reshape(n, -1)[:, 0]
    assert dl_in[102] == dl_in[103] == (1 << 31)


def test_query_graph_replays(tiny):
    """Query batches as graph launches: instantiated on the first batch, then replayed with new
    arguments. Every replay (sizes from 1 to 10,000, DL-only and BL-only rules, direct-launch
    batches and insertions in between) gives the oracle's answers."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    lo = 0
    for k in (10000, 7, 4096, 1, 9999, 10000):
        qu, qv = w.q_u[:k], w.q_v[:k]
        want = o.query_dbl(qu, qv, threads=8)
        g.set_tuning(query_graph=1)
        assert np.array_equal(g.query(dev(qu), dev(qv)).cpu().numpy(), want)
        for rules in (1, 2):
            got = g.query_rules(dev(qu), dev(qv), rules).cpu().numpy()
            assert np.array_equal(got, o.query_rules(qu, qv, rules, threads=8))
        g.set_tuning(query_graph=0)
        assert np.array_equal(g.query(dev(qu), dev(qv)).cpu().numpy(), want)
        g.insert_edges(dev(w.ins_src[lo:lo + 150]), dev(w.ins_dst[lo:lo + 150]))
        o.insert(w.ins_src[lo:lo + 150], w.ins_dst[lo:lo + 150])
        lo += 150
    # a slot queue too small for the BFS: the whole-device BFS runs after the graph launch
    n = 3000
    src = np.arange(n - 1, dtype=np.uint32)
    g = gpu_index(n, src, src + 1, num_landmarks=0, bl_bits=1, bfs_slots=4, bfs_queue_cap=8)
    g.set_tuning(query_graph=1)
    o = oracle.OracleIndex(n, src, src + 1).build(k=0, kp=1)
    u = np.array([0, 5, 100, 2999, 7], dtype=np.uint32)
    v = np.array([2999, 4, 2500, 0, 7], dtype=np.uint32)
    for _ in range(3):
        assert np.array_equal(g.query(dev(u), dev(v)).cpu().numpy(), o.query_dbl(u, v))
    assert g.stats()["bfs_heavy"] > 0


@pytest.mark.parametrize("batch", [1000, 333, 7])
def test_tiny_batched_insertions_equal_sequential(tiny, batch):
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    o.insert(w.ins_src, w.ins_dst)
    for lo in range(0, len(w.ins_src), batch):
        g.insert_edges(dev(w.ins_src[lo:lo + batch]), dev(w.ins_dst[lo:lo + batch]))
    assert_labels_equal(g, o, f"batch {batch}")
    assert_queries_equal(g, o, w.q_u, w.q_v)


def test_tiny_no_slack_forces_regrow(tiny):
    """Zero per-vertex slack: every insertion overflows its row and the CSR is regrown."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst, slack_fraction=0.0, slack_min=0)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    for lo, hi in [(0, 1), (1, 2), (2, 300), (300, 1000)]:
        g.insert_edges(dev(w.ins_src[lo:hi]), dev(w.ins_dst[lo:hi]))
        o.insert(w.ins_src[lo:hi], w.ins_dst[lo:hi])
        assert_labels_equal(g, o, f"no slack after {hi}")
    assert g.stats()["csr_regrows"] > 0
    assert_queries_equal(g, o, w.q_u, w.q_v)


def test_small_bfs_slots_overflow_to_device_bfs(tiny):
    """Four BFS slots with 8-entry queues: long BFS overflow their slot and run on the device."""
    n = 3000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    # no landmarks and one BL bucket: the labels decide nothing, every pair needs the BFS
    g = gpu_index(n, src, dst, num_landmarks=0, bl_bits=1, bfs_slots=4, bfs_queue_cap=8)
    o = oracle.OracleIndex(n, src, dst).build(k=0, kp=1)
    rng = np.random.default_rng(4)
    u = rng.integers(0, n, 40).astype(np.uint32)
    v = rng.integers(0, n, 40).astype(np.uint32)
    u[:5] = [0, 10, 2000, 5, 2999]
    v[:5] = [n - 1, 12, 1000, 5, 0]
    got = assert_queries_equal(g, o, u, v)
    assert np.array_equal(got & 1, (u <= v).astype(np.uint8))
    assert g.stats()["bfs_heavy"] > 0
    w = tiny
    g = gpu_index(w.n, w.src, w.dst, bfs_slots=4, bfs_queue_cap=8)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    assert_queries_equal(g, o, w.q_u, w.q_v)


@pytest.mark.parametrize("rules", [0, 2])
def test_whole_device_bfs_from_both_ends(rules):
    """Four landmarks, 8 BL bits and 8-entry BFS queues send many undecided pairs of a 2^15
    R-MAT to the whole-device BFS, which searches from u and from v and expands the side with
    fewer pending edges: hubs on either side, paths that meet anywhere, pairs with no path. With
    no label rules nothing is pruned; with BL alone both sides' containment prunes apply.
    Answers equal the oracle's. (With DL on, the hub landmarks stop these searches early; the
    layered graph below covers that.)"""
    w = dblgen.make_rmat_workload("bidir", 15, 9, draws=6 << 15, n_insert=2000,
                                  insert_kind="rmat", n_query=3000, query_kind="mixed")
    g = gpu_index(w.n, w.src, w.dst, num_landmarks=4, bl_bits=8, bfs_slots=4, bfs_queue_cap=8)
    g.insert_edges(dev(w.ins_src), dev(w.ins_dst))
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(k=4, kp=8, threads=8)
    o.insert(w.ins_src, w.ins_dst)
    before = g.stats()["bfs_heavy"]
    got = g.query_rules(dev(w.q_u), dev(w.q_v), rules).cpu().numpy()
    want = o.query_rules(w.q_u, w.q_v, rules, threads=8)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, f"rules {rules}: {len(bad)} answers differ, first {bad[:5]}"
    cls = got >> 1
    heavy = g.stats()["bfs_heavy"] - before
    assert heavy > 0 and (cls == 5).sum() > 0 and (cls == 6).sum() > 0, (heavy, np.bincount(cls))



@pytest.mark.parametrize("rules", [1, 3])
def test_whole_device_bfs_landmark_prunes(rules):
    """A layered DAG (48 layers of 64 vertices, three edges from each vertex into the next
    layer) with the landmarks fixed in layer 30: a search from the first layers covers more than
    a slot before the landmark prune (DL_out(u) & DL_in(x) forward, DL_out(y) & DL_in(v)
    backward) cuts it off, so it runs on the whole device with both sides' DL prunes."""
    rng = np.random.default_rng(21)
    layers, width = 48, 64
    n = layers * width
    src = np.repeat(np.arange((layers - 1) * width), 3).astype(np.uint32)
    dst = ((src // width + 1) * width + rng.integers(0, width, src.size)).astype(np.uint32)
    lm = [30 * width + i for i in (0, 17, 40)]
    g = gpu_index(n, src, dst, num_landmarks=3, bl_bits=1, landmarks=lm, bfs_slots=4,
                  bfs_queue_cap=8)
    o = oracle.OracleIndex(n, src, dst).build(k=3, kp=1, landmarks=lm)
    u = rng.integers(0, 10 * width, 800).astype(np.uint32)
    v = rng.integers(0, n, 800).astype(np.uint32)
    before = g.stats()["bfs_heavy"]
    got = g.query_rules(dev(u), dev(v), rules).cpu().numpy()
    want = o.query_rules(u, v, rules, threads=8)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, f"rules {rules}: {len(bad)} answers differ, first {bad[:5]}"
    cls = got >> 1
    heavy = g.stats()["bfs_heavy"] - before
    assert heavy > 0 and (cls == 5).sum() > 0 and (cls == 6).sum() > 0, (heavy, np.bincount(cls))

# ------------------------------------------------------------------ edge cases

def test_out_of_range_ids_leave_index_unchanged(tiny):
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    before = g.labels_numpy()
    edges_before = g.stats()["num_edges"]
    for src, dst in ([[0], [w.n]], [[w.n + 5], [1]], [list(range(300)), [w.n] * 300],
                     [[1, 2, 3], [4, 5, 0xFFFFFFFF]]):
        with pytest.raises(dbl.DblError) as e:
            g.insert_edges(dev(src), dev(dst))
        assert e.value.status == dbl.DBL_ERR_VERTEX_RANGE
    after = g.labels_numpy()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert g.stats()["num_edges"] == edges_before
    # batches above the single-workgroup limit (validated by the grid path), and a small one
    # with that limit at zero, each with a single bad id somewhere in it
    rng = np.random.default_rng(9)
    for count, small_batch in ((5000, None), (70000, None), (10, 0)):
        if small_batch is not None:
            g.set_tuning(small_batch=small_batch)
        a = rng.integers(0, w.n, count).astype(np.uint32)
        b = rng.integers(0, w.n, count).astype(np.uint32)
        bad = int(rng.integers(0, count))
        (a if bad % 2 else b)[bad] = w.n + bad
        with pytest.raises(dbl.DblError) as e:
            g.insert_edges(dev(a), dev(b))
        assert e.value.status == dbl.DBL_ERR_VERTEX_RANGE
        for x, y in zip(before, g.labels_numpy()):
            assert np.array_equal(x, y), f"labels changed by a refused batch of {count}"
        assert g.stats()["num_edges"] == edges_before
    g.set_tuning(small_batch=2048)
    with pytest.raises(dbl.DblError) as e:
        g.query(dev([0, w.n]), dev([1, 2]))
    assert e.value.status == dbl.DBL_ERR_VERTEX_RANGE
    # the index still works
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    assert_queries_equal(g, o, w.q_u[:500], w.q_v[:500])
    with pytest.raises(dbl.DblError):
        dbl.Index.build(10, dev([0, 10]), dev([1, 2]))


def test_empty_loops_duplicates_and_degenerate_graphs():
    # single vertex, no edges
    g = gpu_index(1, [], [])
    assert g.query(dev([0]), dev([0])).cpu().numpy()[0] == 1
    g.insert_edges(dev([]), dev([]))
    assert g.query(dev([]), dev([])).numel() == 0
    # no edges at all: every vertex is both leaves; k > n
    n = 50
    g = gpu_index(n, [], [], num_landmarks=64)
    o = oracle.OracleIndex(n, [], []).build(k=64)
    assert_labels_equal(g, o, "edgeless")
    u, v = all_pairs(n)
    assert_queries_equal(g, o, u, v)
    # self-loops and duplicates in the build and in insertions
    src = [0, 0, 1, 1, 2, 3, 3, 4]
    dst = [0, 1, 2, 2, 3, 3, 1, 4]
    g = gpu_index(6, src, dst, num_landmarks=2, bl_bits=4)
    o = oracle.OracleIndex(6, src, dst).build(k=2, kp=4)
    assert_labels_equal(g, o, "loops/dups build")
    g.insert_edges(dev([5, 5, 2, 2]), dev([5, 0, 3, 3]))
    o.insert([5, 5, 2, 2], [5, 0, 3, 3])
    assert_labels_equal(g, o, "loops/dups insert")
    u, v = all_pairs(6)
    assert_queries_equal(g, o, u, v)


def test_wide_vertex_range_ingest_fallback():
    """Above 2^26 vertices a bin spans more vertices than LDS counters hold, and the build
    counts degrees and fills rows with global atomics instead. A 3,000-vertex R-MAT graph is
    spread over 2^26 + 3 ids (every other id isolated); with the same explicit landmarks and
    leaf hash, its labels and answers must equal the oracle's on the compact graph, and an
    isolated vertex carries only its own BL bit."""
    n_big = (1 << 26) + 3
    w = dblgen.make_rmat_workload("wide", 11, 13, draws=8 << 11, n_insert=500,
                                  insert_kind="uniform", n_query=20000, query_kind="mixed")
    rng = np.random.default_rng(17)
    ids = np.sort(rng.choice(n_big - 2, size=w.n - 2, replace=False) + 1)
    ids = np.concatenate([[0], ids, [n_big - 1]]).astype(np.uint32)  # compact -> wide
    kp = 64
    bucket_big = rng.integers(0, kp, n_big).astype(np.uint8)
    o = oracle.OracleIndex(w.n, w.src, w.dst)
    lm_small = o.select_landmarks(16)
    o.build(k=16, kp=kp, landmarks=lm_small, bucket_table=bucket_big[ids], threads=8)
    g = gpu_index(n_big, ids[w.src], ids[w.dst], num_landmarks=16, bl_bits=kp,
                  landmarks=ids[lm_small], leaf_bucket=bucket_big, bfs_slots=64)

    def check(what):
        got = g.labels()
        t_ids = torch.from_numpy(ids.astype(np.int64)).to(got[0].device)
        for name, a, b in zip(("DL_in", "DL_out", "BL_in", "BL_out"), got, o.labels()):
            sub = a[t_ids].cpu().numpy().view(np.uint64)
            assert np.array_equal(sub, b), f"{what}: {name} differs on the graph's vertices"
        iso = torch.from_numpy(rng.choice(n_big, 200000).astype(np.int64)).to(got[0].device)
        iso = iso[~torch.isin(iso, t_ids)]
        own = torch.from_numpy(bucket_big.astype(np.int64)).to(got[0].device)[iso]
        assert torch.all(got[0][iso] == 0) and torch.all(got[1][iso] == 0), what
        assert torch.equal(got[2][iso], torch.ones_like(own) << own), what
        assert torch.equal(got[3][iso], torch.ones_like(own) << own), what

    check("build")
    qa = g.query(dev(ids[w.q_u]), dev(ids[w.q_v])).cpu().numpy()
    assert np.array_equal(qa, o.query_dbl(w.q_u, w.q_v, threads=8))
    g.insert_edges(dev(ids[w.ins_src]), dev(ids[w.ins_dst]))
    o.insert(w.ins_src, w.ins_dst)
    check("after insertions")
    qa = g.query(dev(ids[w.q_u]), dev(ids[w.q_v])).cpu().numpy()
    assert np.array_equal(qa, o.query_dbl(w.q_u, w.q_v, threads=8))


def test_long_chain_many_rounds():
    """A 20,000-vertex path: propagation needs one round per hop, grid and local forms both."""
    n = 20000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    g = gpu_index(n, src, dst, num_landmarks=4, bl_bits=4)
    o = oracle.OracleIndex(n, src, dst).build(k=4, kp=4)
    assert_labels_equal(g, o, "chain")
    # closing the cycle changes every label
    g.insert_edges(dev([n - 1]), dev([0]))
    o.insert([n - 1], [0])
    assert_labels_equal(g, o, "chain closed")
    rng = np.random.default_rng(3)
    u = rng.integers(0, n, 3000).astype(np.uint32)
    v = rng.integers(0, n, 3000).astype(np.uint32)
    assert_queries_equal(g, o, u, v)


def test_star_hub_heavy_rows():
    """A hub with 200,000 out-edges and 100,000 in-edges exercises the chunked heavy rows."""
    n = 300001
    leaves_out = np.arange(1, 200001, dtype=np.uint32)
    leaves_in = np.arange(200001, n, dtype=np.uint32)
    src = np.concatenate([np.zeros(200000, np.uint32), leaves_in])
    dst = np.concatenate([leaves_out, np.zeros(100000, np.uint32)])
    g = gpu_index(n, src, dst, num_landmarks=8, bl_bits=64)
    o = oracle.OracleIndex(n, src, dst).build(k=8, kp=64, threads=8)
    assert_labels_equal(g, o, "star")
    # the hub's rows are wider than the LDS stage of the assembled fill
    assert_labels_equal(gpu_index(n, src, dst, num_landmarks=8, bl_bits=64, row_fill=2), o,
                        "star, assembled fill")
    rng = np.random.default_rng(9)
    u = rng.integers(0, n, 5000).astype(np.uint32)
    v = rng.integers(0, n, 5000).astype(np.uint32)
    assert_queries_equal(g, o, u, v)
    g.insert_edges(dev([5, 250000]), dev([250001, 7]))
    o.insert([5, 250000], [250001, 7])
    assert_labels_equal(g, o, "star insert")


# ------------------------------------------------------------------ skewed vertex numbering

def _degree_numbering(n, src, dst):
    """New ids by descending total degree (ties by old id), so that the high-degree vertices
    share the first id ranges: new_of[old id]."""
    deg = np.bincount(src, minlength=n).astype(np.int64) + np.bincount(dst, minlength=n)
    order = np.argsort(-deg, kind="stable")
    new_of = np.empty(n, np.uint32)
    new_of[order] = np.arange(n, dtype=np.uint32)
    return new_of


@pytest.mark.parametrize("row_fill", [1, 2])
def test_degree_numbered_ids_split_long_bins(row_fill):
    """R-MAT 2^18 numbered by descending degree: the first vertex-range bins hold far more than
    their share of the edges and are split over several workgroups (direct and LDS-assembled
    fill of the other bins); then a block of hubs with 40,000 edges each. Labels, answers and
    insertions into the kept slack against the oracle."""
    w = dblgen.make_rmat_workload("skew18", 18, 13, draws=8 << 18, n_insert=3000,
                                  insert_kind="rmat", n_query=30000, query_kind="mixed")
    new_of = _degree_numbering(w.n, w.src, w.dst)
    src, dst = new_of[w.src], new_of[w.dst]
    isrc, idst = new_of[w.ins_src], new_of[w.ins_dst]
    g = gpu_index(w.n, src, dst, row_fill=row_fill)
    assert g.stats()["build_long_bins"] > 0
    o = oracle.OracleIndex(w.n, src, dst).build(threads=8)
    assert_labels_equal(g, o, "degree-numbered build")
    assert_queries_equal(g, o, w.q_u, w.q_v)
    g.insert_edges(dev(isrc), dev(idst))
    o.insert(isrc, idst)
    assert_labels_equal(g, o, "degree-numbered, after insertions")
    # hubs 0..7 with 40,000 out-edges and 40,000 in-edges each, over a sparse random rest
    n = 1 << 16
    rng = np.random.default_rng(21)
    hs = np.repeat(np.arange(8, dtype=np.uint32), 40000)
    ht = rng.integers(8, n, len(hs)).astype(np.uint32)
    rs = rng.integers(8, n, 200000).astype(np.uint32)
    rt = rng.integers(8, n, 200000).astype(np.uint32)
    bsrc = np.concatenate([hs, ht, rs])
    bdst = np.concatenate([ht, hs[::-1], rt])
    g = gpu_index(n, bsrc, bdst, row_fill=row_fill, num_landmarks=16, bl_bits=16)
    assert g.stats()["build_long_bins"] > 0
    o = oracle.OracleIndex(n, bsrc, bdst).build(k=16, kp=16, threads=8)
    assert_labels_equal(g, o, "hub block")
    u = rng.integers(0, n, 20000).astype(np.uint32)
    v = rng.integers(0, n, 20000).astype(np.uint32)
    assert_queries_equal(g, o, u, v)


# ------------------------------------------------------------------ several tiles, heavy rows

def test_rmat18_build_insert_query():
    w = dblgen.make_rmat_workload("r18", 18, 11, draws=8 << 18, n_insert=20000,
                                  insert_kind="rmat", n_query=100000, query_kind="mixed")
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    assert list(g.landmarks()) == list(o.landmarks())
    assert_labels_equal(g, o, "rmat18 build")
    assert_queries_equal(g, o, w.q_u, w.q_v)
    o.insert(w.ins_src, w.ins_dst)
    for lo in range(0, 20000, 5000):
        g.insert_edges(dev(w.ins_src[lo:lo + 5000]), dev(w.ins_dst[lo:lo + 5000]))
    assert_labels_equal(g, o, "rmat18 after inserts")
    got = assert_queries_equal(g, o, w.q_u, w.q_v)
    st = g.stats()
    assert st["queries"] == 200000
    assert sum(st["query_class"].values()) == 200000
    assert np.bincount(got >> 1, minlength=7)[5:].sum() > 0  # some BFS ran


@pytest.mark.parametrize("tuning", [
    dict(small_batch=0, local_max_frontier=0, local_max_edges=0, round_grid=1, bfs_slots=4),
    dict(small_batch=0, local_max_frontier=0, local_max_edges=0, pull_threshold=1,
         pull_all_threshold=1),
    dict(small_batch=0, local_max_frontier=1 << 20, local_max_edges=1 << 30, round_grid=3),
    dict(small_batch=65536, local_max_frontier=16, local_max_edges=64, round_grid=2048,
         bfs_slots=2048),
])
def test_tuning_never_changes_results(tiny, tuning):
    """Schedule independence: extreme tunings (every round on the grid, every round in one
    workgroup, tiny grids, few or many BFS slots) give bit-identical labels and answers."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    g.set_tuning(**tuning)
    assert all(g.tuning()[k] == v for k, v in tuning.items() if k != "bfs_slots")
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    for lo, hi in [(0, 1), (1, 400), (400, 1000)]:
        g.insert_edges(dev(w.ins_src[lo:hi]), dev(w.ins_dst[lo:hi]))
        o.insert(w.ins_src[lo:hi], w.ins_dst[lo:hi])
    assert_labels_equal(g, o, str(tuning))
    assert_queries_equal(g, o, w.q_u, w.q_v)


def test_autotuner_picks_a_candidate(tiny, tmp_path, monkeypatch):
    from paper_2101_09441_amd import autotune
    monkeypatch.setenv("DBL_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = tiny
    src, dst = dev(w.src), dev(w.dst)
    mk = lambda: dbl.Index.build(w.n, src, dst)  # noqa: E731
    r = autotune.tune_insertions(mk, dev(w.ins_src), dev(w.ins_dst), 100, w.m, max_batches=5)
    assert {k: r[k] for k in ("small_batch", "round_grid")} in [
        {k: c[k] for k in ("small_batch", "round_grid")} for c in autotune.INSERT_CANDIDATES]
    g = mk()
    q = autotune.tune_queries(g, dev(w.q_u), dev(w.q_v), 2000, w.m, reps=1)
    assert g.tuning()["bfs_slots"] == q["bfs_slots"]
    # cached second time
    assert autotune.tune_queries(g, dev(w.q_u), dev(w.q_v), 2000, w.m)["bfs_slots"] == q["bfs_slots"]
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    assert_queries_equal(g, o, w.q_u, w.q_v)


def test_vertex_insertion(tiny):
    """Vertices added after the build (no edges, empty labels, not BL sources), then edges to
    and from them, in several rounds that grow the per-vertex arrays more than once."""
    w = tiny
    g = gpu_index(w.n, w.src, w.dst)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    rng = np.random.default_rng(12)
    n = w.n
    for add in (1, 100, 20000, 7):
        assert g.add_vertices(add) == n
        assert o.add_vertices(add) == n
        n += add
        iu = rng.integers(0, n, 300).astype(np.uint32)
        iv = rng.integers(0, n, 300).astype(np.uint32)
        iu[:50] = rng.integers(n - add, n, 50)
        iv[50:100] = rng.integers(n - add, n, 50)
        g.insert_edges(dev(iu), dev(iv))
        o.insert(iu, iv)
        assert_labels_equal(g, o, f"after adding {add}")
        qu = rng.integers(0, n, 5000).astype(np.uint32)
        qv = rng.integers(0, n, 5000).astype(np.uint32)
        assert_queries_equal(g, o, qu, qv)
    flags, bucket = g.leaves()
    assert len(flags) == n and not flags[w.n:].any()
    _, _, ob = o.leaves()
    assert np.array_equal(bucket, ob)
    with pytest.raises(dbl.DblError):
        g.insert_edges(dev([0]), dev([n]))


def test_build_out_of_memory_leaks_nothing(tiny):
    """Every device allocation of a build can fail: under a device cap swept from just above
    what the library already holds up to what a build needs, each build either fails with
    OUT_OF_MEMORY and leaves the library's bytes in use exactly as before, or succeeds with
    labels equal to the oracle's."""
    w = tiny
    src, dst = dev(w.src), dev(w.dst)
    dbl.release_cache()
    base = dbl.live_bytes()
    g = gpu_index(w.n, w.src, w.dst)
    need = dbl.live_bytes() - base
    g.close()
    assert dbl.live_bytes() == base
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    failures = 0
    try:
        for frac in np.linspace(0.0, 1.2, 41):
            dbl.set_device_limit(base + int(frac * need) + 1)
            try:
                g = dbl.Index.build(w.n, src, dst)
            except dbl.DblError as e:
                assert e.status == dbl.DBL_ERR_OUT_OF_MEMORY
                assert dbl.live_bytes() == base, f"build failing at {frac:.2f} leaked"
                failures += 1
                continue
            dbl.set_device_limit(0)
            assert_labels_equal(g, o, f"build under a cap of {frac:.2f}")
            g.close()
            assert dbl.live_bytes() == base
    finally:
        dbl.set_device_limit(0)
    assert failures >= 20
