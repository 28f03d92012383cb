"""The persistent insertion kernel (one launch per batch, rounds separated by grid barriers) and
its graph form, against the oracle, bit for bit.

Batches of 1, 7, 1,000, 10,000 and 100,000 edges of a continued R-MAT stream (so components
merge) on a 2^17-vertex graph, plain launches and replays of the instantiated graph; the graph
replays are also compared after every batch with the multi-launch form on a second index.
Stalls forced from the host (a launch with more workgroups than fit at once, which never
gathers; a zero wait at the later barriers) drive both recovery paths, and degenerate shapes
(one long chain, a hub with chunked rows, every round on the grid, a frontier handed to the
host's rounds) the rest of the kernel.
"""
import numpy as np
import pytest
import torch

import dblgen
import oracle

pytestmark = pytest.mark.gpu

dbl = pytest.importorskip("paper_2101_09441_amd")

N_SMALL = 2800  # prefix inserted by the 1- and 7-edge batches


def dev(a):
    return dbl.to_device_ids(a)


def assert_labels_equal(g, want, what):
    for name, a, b in zip(("DL_in", "DL_out", "BL_in", "BL_out"), g.labels_numpy(), want):
        bad = np.flatnonzero(a != b)
        assert len(bad) == 0, f"{what}: {name} differs at {len(bad)} vertices, first {bad[:5]}"


@pytest.fixture(scope="module")
def stream():
    """2^17-vertex R-MAT, 100,000 insertions continuing the stream, 50,000 mixed queries, and
    the oracle's labels and answers after the first N_SMALL insertions and after all of them."""
    w = dblgen.make_rmat_workload("b17", 17, 21, draws=8 << 17, n_insert=100_000,
                                  insert_kind="rmat", n_query=50_000, query_kind="mixed")
    want = {}
    for cnt in (N_SMALL, len(w.ins_src)):
        o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
        o.insert(w.ins_src[:cnt], w.ins_dst[:cnt])
        want[cnt] = (o.labels(), o.query_dbl(w.q_u, w.q_v, threads=8), o.num_edges())
        o.close()
    return w, want


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("batch", [1, 7, 1000, 10_000, 100_000])
def test_persistent_batches_match_oracle(stream, batch, graph):
    w, want = stream
    cnt = N_SMALL if batch < 1000 else len(w.ins_src)
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    g.set_tuning(small_batch=0, insert_persistent=1, insert_graph=graph)
    isrc, idst = dev(w.ins_src[:cnt]), dev(w.ins_dst[:cnt])
    g.time_kernels("insert_batch")
    for lo in range(0, cnt, batch):
        g.insert_edges(isrc[lo:lo + batch], idst[lo:lo + batch])
    labels, answers, edges = want[cnt]
    assert_labels_equal(g, labels, f"batches of {batch}, graph {graph}")
    st = g.stats()
    assert st["num_edges"] == edges and st["batch_stalls"] == 0
    assert g.kernel_times()["insert_batch"]["launches"] == (cnt + batch - 1) // batch
    got = g.query(dev(w.q_u), dev(w.q_v)).cpu().numpy()
    assert np.array_equal(got, answers)
    g.close()


def test_graph_replays_equal_multi_launch_after_every_batch(stream):
    """Every replay of the graph form against the multi-launch form on a second index, with the
    libraries' own eager work (status reads, host rounds) between replays."""
    w, want = stream
    a = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    b = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    a.set_tuning(small_batch=0, insert_graph=1)
    b.set_tuning(small_batch=0, insert_persistent=0)
    isrc, idst = dev(w.ins_src), dev(w.ins_dst)
    for lo in range(0, 30_000, 1000):
        a.insert_edges(isrc[lo:lo + 1000], idst[lo:lo + 1000])
        b.insert_edges(isrc[lo:lo + 1000], idst[lo:lo + 1000])
        for x, y in zip(a.labels(), b.labels()):
            assert torch.equal(x, y), f"graph replay of the batch at {lo}"
    a.insert_edges(isrc[30_000:], idst[30_000:])
    labels, answers, _ = want[len(w.ins_src)]
    assert_labels_equal(a, labels, "graph form, all insertions")
    a.close()
    b.close()


@pytest.mark.parametrize("stall", ["gather", "barrier"])
def test_forced_stalls_recover(stream, stall):
    """Stalls forced from the host. A launch of 2,048 workgroups (more than fit on the device at
    once) never gathers: its resident blocks give up after the gathering wait, nothing has
    changed, and the batch runs in several launches. A zero wait at the later barriers makes
    the first block to wait there give up: the rounds stop and the host re-propagates from
    every vertex. Labels and answers stay exact; every wait ends."""
    w, want = stream
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    g.set_tuning(small_batch=0, **({"batch_grid": 2048, "gather_wait_us": 2000}
                                   if stall == "gather" else {"barrier_wait_us": 0}))
    isrc, idst = dev(w.ins_src), dev(w.ins_dst)
    for lo in range(0, len(w.ins_src), 10_000):
        g.insert_edges(isrc[lo:lo + 10_000], idst[lo:lo + 10_000])
    labels, answers, edges = want[len(w.ins_src)]
    assert_labels_equal(g, labels, f"forced {stall} stalls")
    st = g.stats()
    assert st["batch_stalls"] > 0 and st["num_edges"] == edges
    assert np.array_equal(g.query(dev(w.q_u), dev(w.q_v)).cpu().numpy(), answers)
    g.close()


@pytest.mark.parametrize("tuning", [
    dict(),                                                  # single-workgroup passes
    dict(local_max_frontier=0, local_max_edges=0),           # every round on the grid
    dict(batch_max_frontier=1),                              # every round left to the host
])
def test_chain_and_hub_shapes(tuning):
    """A 20,000-vertex path closed into a cycle by a batch (20,000 rounds: the single-workgroup
    passes run out of their round budget many times over), then a batch that links a hub of
    60,000 out-edges (rows split into chunks)."""
    n = 20000
    src = np.arange(n - 1, dtype=np.uint32)
    dst = src + 1
    hub = np.full(60000, n, dtype=np.uint32)
    leaves = np.arange(n + 1, n + 60001, dtype=np.uint32)
    nn = n + 60001
    bsrc = np.concatenate([src, hub])
    bdst = np.concatenate([dst, leaves])
    g = dbl.Index.build(nn, dev(bsrc), dev(bdst), num_landmarks=4, bl_bits=8)
    g.set_tuning(small_batch=0, **tuning)
    o = oracle.OracleIndex(nn, bsrc, bdst).build(k=4, kp=8, threads=8)
    steps = [([n - 1, 5], [0, 17]),            # closes the cycle
             ([100, 7], [n, 3]),               # the cycle now reaches the hub
             ([n + 5, n + 70], [n + 9, 250])]  # leaves of the hub reach back into the cycle
    for a, b in steps:
        g.insert_edges(dev(a), dev(b))
        o.insert(a, b)
        assert_labels_equal(g, o.labels(), f"{tuning} after {a}->{b}")
    rng = np.random.default_rng(2)
    u = rng.integers(0, nn, 4000).astype(np.uint32)
    v = rng.integers(0, nn, 4000).astype(np.uint32)
    assert np.array_equal(g.query(dev(u), dev(v)).cpu().numpy(), o.query_dbl(u, v, threads=8))
    assert g.stats()["batch_stalls"] == 0
    g.close()
