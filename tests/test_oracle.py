"""Pins of the CPU oracle against things other than itself (CPU only).

The oracle's definition is Section 2's: each vertex gets the id of a
representative of its component, read here as the smallest id (the root that
the high-to-low hooking of Figs. 2-3 leaves).  Each test below checks the
oracle against an independent source of truth: brute-force transitive
closure, a breadth-first traversal labeller, scipy, closed forms, and output
invariants.  ``test_mutants_are_caught`` plants plausible mistakes in a copy
of the oracle's source and checks that these pins reject every one.
"""
import itertools
import os
import shutil
import tempfile

import numpy as np
import pytest

import graphgen
import oracle
from tests import pins


def _rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------------------- brute force
def test_exhaustive_small_graphs_match_transitive_closure():
    """Every edge set on n <= 5 vertices (2^10 sets at n = 5), each in a
    shuffled order with random orientations, plus a self-loop/duplicate variant."""
    rng = _rng(1)
    for n in range(0, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            chosen = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
            rng.shuffle(chosen)
            u = [a if rng.random() < 0.5 else b for a, b in chosen]
            v = [b if uu == a else a for (a, b), uu in zip(chosen, u)]
            want = pins.closure_labels(u, v, n)
            got = oracle.labels(u, v, n)
            assert np.array_equal(got, want), (n, chosen)
            if n and chosen and mask % 7 == 0:
                # self-loops and a duplicated edge change nothing
                extra_u = u + [u[0], 0, n - 1]
                extra_v = v + [v[0], 0, n - 1]
                assert np.array_equal(oracle.labels(extra_u, extra_v, n), want)


def test_random_graphs_match_closure_and_traversal():
    rng = _rng(2)
    for trial in range(400):
        n = int(rng.integers(1, 65))
        m = int(rng.integers(0, 3 * n + 1))
        u = rng.integers(0, n, m)
        v = rng.integers(0, n, m)
        got = oracle.labels(u, v, n)
        assert np.array_equal(got, pins.closure_labels(u, v, n)), trial
        assert np.array_equal(got, pins.traversal_labels(u, v, n)), trial


# ----------------------------------------------------------------------------- library routine
@pytest.mark.parametrize("family", ["er", "rmat", "grid", "sparse"])
def test_medium_graphs_match_scipy(family):
    if family == "er":
        u, v, n, _ = graphgen.er_planted(n=1 << 12, m_er=1 << 13, cliques=16, seed=7)
    elif family == "rmat":
        u, v, n = graphgen.rmat(14, 4, seed=8, permute=True, symmetrize=True)
    elif family == "grid":
        u, v, n = graphgen.grid(128, 96, 3, 10, seed=9)
    else:  # below the ER threshold: many small trees
        u, v = graphgen.uniform_pairs(3000, 10000, seed=10, stream=0)
        n = 10000
    got = oracle.labels(u, v, n)
    assert np.array_equal(got, pins.scipy_labels(u, v, n))
    pins.check_invariants(u, v, n, got)


def test_traversal_matches_on_medium_graph():
    u, v, n = graphgen.rmat(12, 8, seed=11, permute=True)
    assert np.array_equal(oracle.labels(u, v, n), pins.traversal_labels(u, v, n))


# ----------------------------------------------------------------------------- closed forms
def test_closed_forms():
    n = 1000
    ids = np.arange(n, dtype=np.int32)
    # no edges: every vertex is its own component
    assert np.array_equal(oracle.labels([], [], n), ids)
    # self-loops only
    assert np.array_equal(oracle.labels(ids, ids, n), ids)
    # path 0-1-...-(n-1), listed in increasing and in decreasing order, both orientations
    a, b = ids[:-1], ids[1:]
    zeros = np.zeros(n, np.int32)
    for uu, vv in [(a, b), (b, a), (a[::-1], b[::-1]), (b[::-1], a[::-1])]:
        assert np.array_equal(oracle.labels(uu, vv, n), zeros)
    # star centred on the largest id
    assert np.array_equal(oracle.labels(np.full(n - 1, n - 1), ids[:-1], n), zeros)
    # perfect matching (2i, 2i+1) -> 2*floor(v/2)
    assert np.array_equal(oracle.labels(ids[1::2], ids[0::2], n), (ids // 2) * 2)
    # matching of i with n-1-i -> min(i, n-1-i)
    assert np.array_equal(oracle.labels(ids, ids[::-1], n), np.minimum(ids, ids[::-1]))
    # two interleaved cycles: evens and odds
    ev, od = ids[0::2], ids[1::2]
    got = oracle.labels(np.concatenate([ev, od]), np.concatenate([np.roll(ev, 1), np.roll(od, 1)]), n)
    assert np.array_equal(got, ids % 2)


def test_grid_closed_forms():
    W, H = 64, 48
    n = W * H
    r = np.arange(n) // W
    # full lattice: one component
    u, v, _ = graphgen.grid(W, H, 0, 10, seed=1)
    assert len(u) == (W - 1) * H + W * (H - 1)
    assert np.array_equal(oracle.labels(u, v, n), np.zeros(n, np.int32))
    # horizontal edges only: one component per row, labelled by its first vertex
    horiz = (v - u) == 1
    assert np.array_equal(oracle.labels(u[horiz], v[horiz], n), (r * W).astype(np.int32))
    # vertical edges only: one component per column
    vert = ~horiz
    assert np.array_equal(oracle.labels(u[vert], v[vert], n), (np.arange(n) % W).astype(np.int32))


def test_planted_cliques_are_isolated_components():
    u, v, n, cliques = graphgen.er_planted(n=1 << 12, m_er=1 << 14, cliques=64, seed=3)
    lab = oracle.labels(u, v, n)
    for c in cliques:
        assert np.all(lab[c] == c.min())
        # nothing outside the clique shares its label
        assert np.count_nonzero(lab == c.min()) == 4


def test_partition_is_invariant_under_relabelling():
    u, v, n = graphgen.rmat(12, 4, seed=5, permute=False)
    p = graphgen.permutation(n, seed=77)
    lab = oracle.labels(u, v, n)
    lab_p = oracle.labels(p[u], p[v], n)
    # vertices x, y share a component iff p[x], p[y] do
    inv = np.empty(n, np.int64)
    inv[p] = np.arange(n)
    # map each relabelled component back and compare partitions via their minima
    back = lab_p[p]  # label (in permuted ids) of original vertex x
    pair = {}
    for a, b in zip(lab.tolist(), back.tolist()):
        assert pair.setdefault(a, b) == b
    assert len(set(pair.values())) == len(pair)


def test_output_invariants_on_generators():
    for u, v, n in [graphgen.rmat(13, 8, seed=21, symmetrize=True),
                    graphgen.grid(100, 100, 3, 10, seed=22)]:
        pins.check_invariants(u, v, n, oracle.labels(u, v, n))


# ----------------------------------------------------------------------------- errors, batch
def test_argument_and_range_errors():
    with pytest.raises(ValueError):
        oracle.labels([0, 5], [1, 2], 5)
    with pytest.raises(ValueError):
        oracle.labels([-1], [0], 3)
    with pytest.raises(ValueError):
        oracle.labels([], [], -1)
    assert len(oracle.labels([], [], 0)) == 0


def test_batch_is_disjoint_union():
    u, v, vo, eo = graphgen.batch_er(40, seed=31, lo_exp=3, hi_exp=9)
    lab = oracle.labels_batch(u, v, vo, eo)
    # one big graph with global ids = offset + local id
    gid = np.repeat(vo[:-1], np.diff(eo))
    big = oracle.labels(u + gid, v + gid, int(vo[-1]))
    vid = np.repeat(vo[:-1], np.diff(vo))
    assert np.array_equal(lab + vid, big)
    for g in range(40):
        s, e = eo[g], eo[g + 1]
        n_g = int(vo[g + 1] - vo[g])
        assert np.array_equal(lab[vo[g]:vo[g + 1]], pins.traversal_labels(u[s:e], v[s:e], n_g))


# ----------------------------------------------------------------------------- mutation check
_MUTANTS = {
    "link_to_max": ("if (ru < rv) parent[rv] = ru;\n        else parent[ru] = rv;",
                    "if (ru < rv) parent[ru] = rv;\n        else parent[rv] = ru;"),
    "drop_last_edge": ("for (int64_t i = 0; i < m; ++i) {\n        int32_t ru",
                       "for (int64_t i = 0; i + 1 < m; ++i) {\n        int32_t ru"),
    "parent_as_label": ("label[x] = (parent[x] == x) ? x : label[parent[x]];",
                        "label[x] = parent[x];"),
    "single_step_find": ("while (parent[x] != x) {", "if (parent[x] != x) {"),
    "transposed_operand": ("int32_t rv = find_root(parent, v[i]);",
                           "int32_t rv = find_root(parent, u[i]);"),
    "no_halving_target": ("parent[x] = parent[parent[x]];", "parent[x] = x;"),
}


def _pins_pass(lib) -> bool:
    try:
        rng = _rng(99)
        for _ in range(200):
            n = int(rng.integers(1, 24))
            m = int(rng.integers(0, 2 * n + 1))
            u = rng.integers(0, n, m)
            v = rng.integers(0, n, m)
            if not np.array_equal(oracle.labels(u, v, n, lib=lib), pins.closure_labels(u, v, n)):
                return False
        ids = np.arange(300, dtype=np.int32)
        if not np.array_equal(oracle.labels(ids[1:], ids[:-1], 300, lib=lib), np.zeros(300)):
            return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_mutants_are_caught(name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "cc_oracle.c")).read()
    old, new = _MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved: " + name
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        path = os.path.join(d, "mut.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        so = oracle.build(src=path, out=os.path.join(d, "libmut.so"))
        assert not _pins_pass(oracle.load(so)), "pins did not catch mutant " + name
    finally:
        shutil.rmtree(d, ignore_errors=True)


def test_unmutated_oracle_passes_mutation_pins():
    assert _pins_pass(oracle.load())


# ----------------------------------------------------------------------------- hand fixtures
def test_hand_worked_fixtures():
    from tests.golden.cases import hand_cases
    cases = list(hand_cases())
    assert len(cases) >= 10
    for name, n, u, v, want in cases:
        assert np.array_equal(pins.closure_labels(u, v, n), want), name  # fixture is right
        assert np.array_equal(oracle.labels(u, v, n), want), name
