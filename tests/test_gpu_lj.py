"""GPU parity at the LiveJournal-shaped configuration, in the form the benchmark times.

R-MAT, 2^22 vertices, 68,993,773 unique edges: build, the 100,000 R-MAT insertions one request
at a time (the device-fed stream), then the 1,000,000 mixed queries as one batch. Every label
word of every vertex and every answer byte (answer and decision class) must equal the oracle's
(the oracle builds with 16 threads, applies Algorithm 3 edge by edge, answers with Algorithm 2).
"""
import numpy as np
import pytest

import dblgen
import oracle

pytestmark = pytest.mark.gpu

dbl = pytest.importorskip("paper_2101_09441_amd")


def test_lj_shaped_full_parity():
    w = dblgen.cached("rmat22-lj-s1", dblgen.lj_workload)
    print(f"workload n={w.n} m={w.m} insertions={len(w.ins_src)} queries={len(w.q_u)}",
          flush=True)
    g = dbl.Index.build(w.n, dbl.to_device_ids(w.src), dbl.to_device_ids(w.dst),
                        edges_unique=True)
    lat = g.insert_edges_each(dbl.to_device_ids(w.ins_src), dbl.to_device_ids(w.ins_dst),
                              latencies=True)
    got = g.query(dbl.to_device_ids(w.q_u), dbl.to_device_ids(w.q_v)).cpu().numpy()
    st = g.stats()
    assert st["server_requests"] == len(w.ins_src) and np.all(lat >= 0) and lat.sum() > 0
    print("GPU done; oracle build", flush=True)
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=16)
    print("oracle insertions", flush=True)
    o.insert(w.ins_src, w.ins_dst)
    for name, a, b in zip(("DL_in", "DL_out", "BL_in", "BL_out"), g.labels_numpy(), o.labels()):
        bad = np.flatnonzero(a != b)
        assert len(bad) == 0, f"{name} differs at {len(bad)} vertices, first {bad[:5]}"
    print("labels equal; oracle queries", flush=True)
    want = o.query_dbl(w.q_u, w.q_v, threads=16)
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, f"{len(bad)} answers differ, first {bad[:5]}"
    assert 0.4 < (got & 1).mean() < 0.6  # the mixture is about half reachable
    o.close()
