"""Seeded input generators: determinism, exact sizes, structure (CPU only)."""
import numpy as np

import graphgen


def test_draws_are_counter_based():
    a = graphgen.draws(5, 3, 100)
    b = graphgen.draws(5, 3, 40, start=60)
    assert np.array_equal(a[60:], b)
    assert not np.array_equal(graphgen.draws(5, 4, 100), a)


def test_permutation_is_a_permutation_and_seeded():
    p = graphgen.permutation(10007, seed=1)
    assert np.array_equal(np.sort(p), np.arange(10007))
    assert np.array_equal(p, graphgen.permutation(10007, seed=1))
    assert not np.array_equal(p, graphgen.permutation(10007, seed=2))


def test_er_planted_sizes_and_cliques():
    u, v, n, cl = graphgen.er_planted(seed=1001)
    assert n == 1 << 16
    assert len(u) == len(v) == (1 << 19) + 64 * 6
    assert cl.shape == (64, 4) and len(np.unique(cl)) == 256
    er_u, er_v = u[:1 << 19], v[:1 << 19]
    # random pairs never touch a clique vertex
    assert not np.isin(er_u, cl).any() and not np.isin(er_v, cl).any()
    assert u.min() >= 0 and max(u.max(), v.max()) < n
    u2, v2, _, _ = graphgen.er_planted(seed=1001)
    assert np.array_equal(u, u2) and np.array_equal(v, v2)


def test_rmat_skew_and_symmetry():
    u, v, n = graphgen.rmat(16, 8, seed=3, permute=False)
    assert n == 1 << 16 and len(u) == 8 << 16
    # unpermuted: vertex 0 is the top hub, P(bit = 0) = a + b = 0.76 per level for u
    deg = np.bincount(u, minlength=n)
    assert deg.argmax() == 0
    bit0 = 1.0 - np.mean((u >> 15) & 1)
    assert abs(bit0 - 0.76) < 0.005
    vbit0 = 1.0 - np.mean((v >> 15) & 1)
    assert abs(vbit0 - 0.76) < 0.005  # a + c
    us, vs, _ = graphgen.rmat(10, 4, seed=3, symmetrize=True)
    m = 4 << 10
    assert np.array_equal(us[m:], vs[:m]) and np.array_equal(vs[m:], us[:m])
    # permutation preserves the multiset of degrees
    up, vp, _ = graphgen.rmat(16, 8, seed=3, permute=True)
    assert np.array_equal(np.sort(np.bincount(up, minlength=n)), np.sort(deg))


def test_grid_exact_counts():
    assert graphgen.grid_edge_count(4096, 4096) == 33546240
    u, v, n = graphgen.grid(64, 32, 3, 10, seed=4)
    E = 63 * 32 + 64 * 31
    assert len(u) == E - E * 3 // 10
    d = v - u
    assert set(np.unique(d).tolist()) <= {1, 64}
    assert np.all(u[d == 1] % 64 != 63)
    # edges are emitted in enumeration order
    key = u.astype(np.int64) * 2 + (d == 64)
    assert np.all(np.diff(key) > 0)


def test_batch_sizes_in_range():
    nv, me = graphgen.batch_sizes(10000, seed=1004)
    assert nv.min() >= 256 and nv.max() <= 65536
    deg = 2.0 * me / nv
    assert deg.min() >= 0.99 and deg.max() <= 16.01
    # log-uniform: the median size is near 2^12
    assert 2 ** 11.5 < np.median(nv) < 2 ** 12.5
    u, v, vo, eo = graphgen.batch_er(50, seed=9)
    for g in range(50):
        s, e = eo[g], eo[g + 1]
        assert u[s:e].max(initial=0) < vo[g + 1] - vo[g]


def test_serving_shapes():
    sc, ef = graphgen.serving_request_shapes(5000, seed=1005)
    assert sc.min() == 10 and sc.max() == 22 and ef.min() == 8 and ef.max() == 32
    u, v, n = graphgen.serving_request(3, 10, 8)
    assert n == 1024 and len(u) == 8 * 1024
    t = graphgen.poisson_arrivals(20000, rate=100.0, seed=1)
    assert abs(np.mean(np.diff(t)) - 0.01) < 0.0005
