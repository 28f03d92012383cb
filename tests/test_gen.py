"""The seeded input generator against the published definitions of its parts."""
import numpy as np

import dblgen

M64 = (1 << 64) - 1


def _splitmix64(state):
    state = (state + 0x9E3779B97F4A7C15) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def _rotl(x, k):
    return ((x << k) | (x >> (64 - k))) & M64


def _xoshiro_ref(seed, count):
    """xoshiro256** as published by Blackman and Vigna, seeded through splitmix64."""
    st, s = seed, []
    for _ in range(4):
        st, z = _splitmix64(st)
        s.append(z)
    out = []
    for _ in range(count):
        out.append((_rotl((s[1] * 5) & M64, 7) * 9) & M64)
        t = (s[1] << 17) & M64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
    return out


def test_xoshiro_matches_published_definition():
    for seed in (0, 1, 12345):
        got = [int(x) for x in dblgen.xoshiro_outputs(seed, 50)]
        assert got == _xoshiro_ref(seed, 50)


def test_rmat_stream_is_unique_loop_free_and_deterministic():
    w1 = dblgen.tiny_workload(1)
    w2 = dblgen.tiny_workload(1)
    assert np.array_equal(w1.src, w2.src) and np.array_equal(w1.q_v, w2.q_v)
    assert w1.n == 1 << 14 and w1.draws == 8 << 14
    assert np.all(w1.src != w1.dst)
    keys = w1.src.astype(np.uint64) << np.uint64(32) | w1.dst.astype(np.uint64)
    assert len(np.unique(keys)) == len(keys)
    ikeys = w1.ins_src.astype(np.uint64) << np.uint64(32) | w1.ins_dst.astype(np.uint64)
    assert len(np.intersect1d(keys, ikeys)) == 0 and len(np.unique(ikeys)) == len(ikeys)
    assert np.all(w1.ins_src != w1.ins_dst)
    assert 0.85 * w1.draws < w1.m <= w1.draws


def test_rmat_degree_skew():
    w = dblgen.tiny_workload(1)
    outdeg = np.bincount(w.src, minlength=w.n)
    assert outdeg.max() > 50 * outdeg.mean()  # power-law: hubs far above the mean
    assert (np.bincount(np.concatenate([w.src, w.dst]), minlength=w.n) == 0).mean() > 0.2


def test_mixed_queries_walk_endpoints_are_reachable():
    st = dblgen.RmatStream(10, 3, expected_edges=8192)
    src, dst = st.next_edges(8192, 8192)
    u, v = dblgen.queries_mixed(1 << 10, src, dst, seed=9, count=2000, p_walk=1.0, max_len=4)
    adj = {}
    for a, b in zip(src, dst):
        adj.setdefault(int(a), set()).add(int(b))
    for a, b in zip(u[:300], v[:300]):
        seen, todo = {int(a)}, [int(a)]
        while todo:
            x = todo.pop()
            for y in adj.get(x, ()):
                if y not in seen:
                    seen.add(y)
                    todo.append(y)
        assert int(b) in seen


def test_zipf_sources_are_skewed():
    u, v = dblgen.queries_zipf(1 << 12, seed=4, count=20000, s=1.1)
    counts = np.sort(np.bincount(u, minlength=1 << 12))[::-1]
    assert counts[0] > 0.05 * 20000 and counts[:10].sum() > 0.2 * 20000
    assert v.max() < 1 << 12


def test_large_chunked_stream_is_sorted_unique_and_thread_independent():
    src, dst, isrc, idst = dblgen.rmat_large(15, 3, 1 << 19, 3000, threads=4, chunk=1 << 13)
    keys = src.astype(np.uint64) << np.uint64(32) | dst.astype(np.uint64)
    assert np.all(keys[1:] > keys[:-1]) and np.all(src != dst)
    ik = isrc.astype(np.uint64) << np.uint64(32) | idst.astype(np.uint64)
    assert len(np.intersect1d(keys, ik)) == 0 and len(np.unique(ik)) == len(ik)
    s2, d2, i2, j2 = dblgen.rmat_large(15, 3, 1 << 19, 3000, threads=3, chunk=1 << 13)
    assert np.array_equal(src, s2) and np.array_equal(dst, d2) and np.array_equal(isrc, i2)
    assert 0.8 * (1 << 19) < len(src) < (1 << 19)
