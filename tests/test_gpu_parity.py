"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Labels are integers with a unique correct answer (the smallest id of each
component), so every comparison is bit-exact.  Small and medium cases are
compared element by element with the oracle run live; the full-size
workloads are compared through the SHA-256 digests of the oracle's labels
stored in tests/golden/oracle_digests.json (written by make_golden.py, which
calls only the oracle).
"""
import hashlib
import itertools
import json
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import pins
from tests.golden.cases import hand_cases

torch = pytest.importorskip("torch")
import paper_1612_01178_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")

VARIANTS = {
    "default": cc.Options(),
    "plain": cc.Options(hook="plain"),
    "atomic": cc.Options(hook="atomic"),
    "s1": cc.Options(hook="atomic", segments=1, filter="off"),
    "s3_nohalve": cc.Options(hook="atomic", segments=3, filter="off", path_halving="off"),
    "s8_giant_nohalve": cc.Options(hook="atomic", segments=8, filter="giant", path_halving="off",
                                   hot_cache="on"),
    "s7_b64_e4": cc.Options(hook="atomic", segments=7, filter="off", edges_per_thread=4, block=64),
    "s5_giant_b1024_e16": cc.Options(hook="atomic", segments=5, filter="giant", filter_after=1,
                                     edges_per_thread=16, block=1024),
    "s9_giant_after3": cc.Options(hook="atomic", segments=9, filter="giant", filter_after=3,
                                  edges_per_thread=8, block=512),
    "s6_giant_nohot_e4": cc.Options(hook="atomic", segments=6, filter="giant", hot_cache="off",
                                    edges_per_thread=4),
    "s12_giant_hotlarge_e16": cc.Options(hook="atomic", segments=12, filter="giant",
                                         hot_cache="large", edges_per_thread=16),
    "s10_giant_hotvertex": cc.Options(hook="atomic", segments=10, filter="giant",
                                      hot_cache="vertex"),
    "s6_giant_hotvertex_nohalve_after2": cc.Options(hook="atomic", segments=6, filter="giant",
                                                    filter_after=2, hot_cache="vertex",
                                                    path_halving="off"),
    "plain_b128_e16_k1": cc.Options(hook="plain", edges_per_thread=16, block=128,
                                    rounds_per_check=1),
    "plain_e4_k7": cc.Options(hook="plain", edges_per_thread=4, rounds_per_check=7),
    # frontier rewritten only below a surviving fraction of 0.1 % / 50 %
    "plain_tau1_k1": cc.Options(hook="plain", compact_threshold=1, rounds_per_check=1),
    "plain_tau500_e16": cc.Options(hook="plain", compact_threshold=500, edges_per_thread=16),
    "coherent_giant": cc.Options(hook="atomic", coherent_loads=True, segments=6, filter="giant"),
    "coherent_s3": cc.Options(hook="atomic", coherent_loads=True, segments=3, filter="off",
                              block=128),
    "hybrid": cc.Options(hook="hybrid"),
    "hybrid_nohalve_e4": cc.Options(hook="hybrid", path_halving="off", edges_per_thread=4),
    "hostloop_jump": cc.Options(hook="plain", host_loop="jump"),
    "hostloop_multijump": cc.Options(hook="plain", host_loop="multijump", edges_per_thread=16),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cc.load()
    return torch.device("cuda:0")


def to_dev(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)


def to_dev64(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int64)).to(dev)


def solve(u, v, n, dev, options=None, offset=0):
    """GPU labels as numpy.  ``offset`` shifts the edge arrays inside a larger
    allocation so that their base is not 16-byte aligned."""
    if offset:
        U = torch.zeros(len(u) + offset, dtype=torch.int32, device=dev)
        V = torch.zeros(len(v) + offset, dtype=torch.int32, device=dev)
        U[offset:] = to_dev(u, dev)
        V[offset:] = to_dev(v, dev)
        du, dv = U[offset:], V[offset:]
    else:
        du, dv = to_dev(u, dev), to_dev(v, dev)
    return cc.labels(du, dv, n, options=options).cpu().numpy()


def digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()


# ----------------------------------------------------------------------------- small, exact
@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_hand_fixtures(dev, variant):
    for name, n, u, v, want in hand_cases():
        say("hand case", name, variant)
        got = solve(u, v, n, dev, VARIANTS[variant])
        assert np.array_equal(got, want), (name, got, want)


def test_exhaustive_tiny_graphs_single_calls(dev):
    rng = np.random.default_rng(5)
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    masks = rng.choice(1 << len(pairs), 96, replace=False)
    for i, mask in enumerate(masks):
        chosen = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
        u = np.array([a for a, _ in chosen], np.int32)
        v = np.array([b for _, b in chosen], np.int32)
        if i % 2:
            u, v = v, u
        want = pins.closure_labels(u, v, n)
        for name in ("default", "plain", "s7_b64_e4"):
            assert np.array_equal(solve(u, v, n, dev, VARIANTS[name]), want), (chosen, name)


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_random_graphs_against_oracle(dev, variant):
    """Sizes span several tiles with ragged tails; densities from forests to
    dense; both aligned and unaligned edge arrays."""
    rng = np.random.default_rng(11)
    for trial in range(14):
        n = int(rng.choice([1, 2, 3, 17, 100, 1000, 4099, 65537, 200003]))
        deg = float(rng.choice([0.3, 1.0, 2.0, 5.0, 16.0]))
        m = int(deg * n) + int(rng.integers(0, 7))
        u, v = graphgen.uniform_pairs(m, n, seed=1000 + trial, stream=3)
        off = int(rng.choice([0, 0, 1, 3]))
        say("random", variant, "trial", trial, "n", n, "m", m, "offset", off)
        got = solve(u, v, n, dev, VARIANTS[variant], offset=off)
        want = oracle.labels(u, v, n)
        assert np.array_equal(got, want), (variant, trial, n, m, int(np.sum(got != want)))


@pytest.mark.parametrize("variant", ["default", "plain", "atomic", "s5_giant_b1024_e16", "s1"])
def test_adversarial_shapes(dev, variant):
    opt = VARIANTS[variant]
    n = 100003
    ids = np.arange(n, dtype=np.int32)
    cases = {
        "path_up": (ids[:-1], ids[1:]),
        "path_down": (ids[1:][::-1].copy(), ids[:-1][::-1].copy()),
        "star_top": (np.full(n - 1, n - 1, np.int32), ids[:-1]),
        "star_zero": (ids[1:], np.zeros(n - 1, np.int32)),
        "matching": (ids[1::2], ids[0::2][:len(ids[1::2])]),
        "mirror": (ids, ids[::-1].copy()),
        "self_loops": (ids, ids),
        "no_edges": (np.zeros(0, np.int32), np.zeros(0, np.int32)),
    }
    for name, (u, v) in cases.items():
        say("shape", name, variant)
        got = solve(u, v, n, dev, opt)
        assert np.array_equal(got, oracle.labels(u, v, n)), name
    # complete graph on 300 vertices (every ordered pair)
    a, b = np.meshgrid(np.arange(300, dtype=np.int32), np.arange(300, dtype=np.int32))
    got = solve(a.ravel(), b.ravel(), 300, dev, opt)
    assert np.array_equal(got, np.zeros(300, np.int32))
    # long chains of a lattice: rows only, columns only
    W, H = 700, 300
    u, v, nn = graphgen.grid(W, H, 0, 10, seed=2)
    horiz = (v - u) == 1
    got = solve(u[horiz], v[horiz], nn, dev, opt)
    assert np.array_equal(got, (np.arange(nn) // W * W).astype(np.int32))
    got = solve(u[~horiz][::-1].copy(), v[~horiz][::-1].copy(), nn, dev, opt)
    assert np.array_equal(got, (np.arange(nn) % W).astype(np.int32))


def test_generator_families_against_oracle(dev):
    fams = {
        "er_planted": graphgen.er_planted(n=1 << 14, m_er=1 << 17, cliques=64, seed=17)[:3],
        "rmat_sym": graphgen.rmat(16, 16, seed=18, symmetrize=True),
        "rmat_plain": graphgen.rmat(15, 8, seed=19, permute=False),
        "grid_perc": graphgen.grid(512, 384, 3, 10, seed=20),
        "grid_sparse": graphgen.grid(400, 400, 6, 10, seed=21),
    }
    for name, (u, v, n) in fams.items():
        want = oracle.labels(u, v, n)
        for variant, opt in VARIANTS.items():
            say("family", name, variant)
            got = solve(u, v, n, dev, opt)
            assert np.array_equal(got, want), (name, variant)


# ----------------------------------------------------------------------------- metamorphic
def test_metamorphic_invariance(dev):
    u, v, n = graphgen.rmat(15, 12, seed=23, symmetrize=False)
    want = oracle.labels(u, v, n)
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(u))
    variants = {
        "shuffled": (u[perm], v[perm]),
        "swapped": (v, u),
        "duplicated": (np.concatenate([u, u[:5000]]), np.concatenate([v, v[:5000]])),
        "self_loops_added": (np.concatenate([u, np.arange(n, dtype=np.int32)]),
                             np.concatenate([v, np.arange(n, dtype=np.int32)])),
    }
    for name, (uu, vv) in variants.items():
        for opt in ("default", "plain", "atomic", "s9_giant_after3"):
            say("metamorphic", name, opt)
            assert np.array_equal(solve(uu, vv, n, dev, VARIANTS[opt]), want), (name, opt)


def test_repeated_solves_are_identical(dev):
    """The races in Hook / Multi-Jump change the intermediate trees, never the labels."""
    u, v, n, _ = graphgen.er_planted(seed=1001)
    want = oracle.labels(u, v, n)
    du, dv = to_dev(u, dev), to_dev(v, dev)
    for opt in ("default", "plain", "atomic", "s5_giant_b1024_e16"):
        for rep in range(15):
            got = cc.labels(du, dv, n, options=VARIANTS[opt]).cpu().numpy()
            assert np.array_equal(got, want), (opt, rep)


# ----------------------------------------------------------------------------- errors
def test_range_errors_are_reported(dev):
    for opt in ("default", "plain", "atomic", "s5_giant_b1024_e16"):
        for bad in (10, -1, 1 << 30):
            u = np.array([0, 1, 2, bad, 3], np.int32)
            v = np.array([1, 2, 3, 4, 0], np.int32)
            with pytest.raises(cc.CCError) as ei:
                solve(u, v, 10, dev, VARIANTS[opt])
            assert ei.value.code == cc.CC_ERR_RANGE
    # the library stays usable afterwards
    assert np.array_equal(solve(np.array([1], np.int32), np.array([0], np.int32), 3, dev),
                          np.array([0, 0, 2], np.int32))


def test_round_cap_and_workspace_errors(dev):
    n = 5000
    u = np.full(n - 1, n - 1, np.int32)   # star on the top id: hooks collide on one slot
    v = np.arange(n - 1, dtype=np.int32)
    with pytest.raises(cc.CCError) as ei:
        solve(u, v, n, dev, cc.Options(hook="plain", max_rounds=1, rounds_per_check=1))
    assert ei.value.code == cc.CC_ERR_NOCONVERGE
    opt = cc.Options(hook="plain")
    need = cc.workspace_bytes(n, len(u), opt)
    small = torch.empty(need // 2, dtype=torch.uint8, device=dev)
    with pytest.raises(cc.CCError) as ei:
        cc.labels(to_dev(u, dev), to_dev(v, dev), n, options=opt, workspace=small)
    assert ei.value.code == cc.CC_ERR_NOMEM
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    got = cc.labels(to_dev(u, dev), to_dev(v, dev), n, options=opt, workspace=ws)
    assert np.array_equal(got.cpu().numpy(), np.zeros(n, np.int32))


def test_stats_are_reported(dev):
    u, v, n = graphgen.rmat(16, 16, seed=31, symmetrize=True)
    du, dv = to_dev(u, dev), to_dev(v, dev)
    lab, st = cc.labels(du, dv, n, options=cc.Options(hook="atomic", filter="giant", profile=True),
                        return_stats=True)
    assert st["segments"] == 32 and st["filter_used"] == 1 and st["host_syncs"] == 1
    assert st["hook_ms"] > 0 and st["compress_ms"] > 0
    assert np.array_equal(lab.cpu().numpy(), oracle.labels(u, v, n))
    lab, st = cc.labels(du, dv, n, options=cc.Options(hook="plain"), return_stats=True)
    assert st["rounds"] >= 1 and st["active_edges"] >= 0


# ----------------------------------------------------------------------------- batches
def test_batch_exhaustive_tiny_graphs(dev):
    graphs = []
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            chosen = [pairs[k] for k in range(len(pairs)) if mask >> k & 1]
            graphs.append((n, chosen))
    vo = np.zeros(len(graphs) + 1, np.int64)
    eo = np.zeros(len(graphs) + 1, np.int64)
    us, vs, want = [], [], []
    for g, (n, chosen) in enumerate(graphs):
        vo[g + 1] = vo[g] + n
        eo[g + 1] = eo[g] + len(chosen)
        uu = np.array([b for _, b in chosen], np.int32)
        vv = np.array([a for a, _ in chosen], np.int32)
        us.append(uu)
        vs.append(vv)
        want.append(pins.closure_labels(uu, vv, n))
    u = np.concatenate(us).astype(np.int32)
    v = np.concatenate(vs).astype(np.int32)
    got = cc.labels_batch(to_dev(u, dev), to_dev(v, dev), vo, eo).cpu().numpy()
    assert np.array_equal(got, np.concatenate(want))


def test_batch_mixed_sizes_against_oracle(dev):
    rng = np.random.default_rng(8)
    sizes = [0, 1, 2, 300, 65536, 65537, 150000, 7, 40000, 0, 1000]
    us, vs = [], []
    vo, eo = [0], [0]
    for i, n in enumerate(sizes):
        m = 0 if n == 0 else int(rng.integers(0, 3 * n + 2))
        if i == 4:
            m = 0  # a large graph with no edges
        uu, vv = graphgen.uniform_pairs(m, max(n, 1), seed=50 + i, stream=0)
        us.append(uu)
        vs.append(vv)
        vo.append(vo[-1] + n)
        eo.append(eo[-1] + m)
    u, v = np.concatenate(us), np.concatenate(vs)
    vo, eo = np.array(vo, np.int64), np.array(eo, np.int64)
    want = oracle.labels_batch(u, v, vo, eo)
    got, st = cc.labels_batch(to_dev(u, dev), to_dev(v, dev), vo, eo, return_stats=True)
    assert np.array_equal(got.cpu().numpy(), want)
    for cap, halve in ((1, "auto"), (2, "on"), (5, "auto"), (0, "off"), (3, "off")):
        got = cc.labels_batch(to_dev(u, dev), to_dev(v, dev), vo, eo,
                              options=cc.Options(segments=cap, path_halving=halve))
        assert np.array_equal(got.cpu().numpy(), want), (cap, halve)


def test_batch_range_error(dev):
    u = np.array([0, 1, 5], np.int32)
    v = np.array([1, 2, 0], np.int32)
    vo = np.array([0, 3, 8], np.int64)
    eo = np.array([0, 2, 3], np.int64)
    with pytest.raises(cc.CCError) as ei:
        cc.labels_batch(to_dev(u, dev), to_dev(v, dev), vo, eo)
    assert ei.value.code == cc.CC_ERR_RANGE


def _batch_device(u, v, vo, eo, dev, max_n, options=None, stream=None):
    import torch
    # as many labels as the largest offset, so that invalid offsets never
    # make a valid graph's labels land outside the tensor
    out = torch.full((max(int(np.max(vo)), 1),), -1, dtype=torch.int32, device=dev)
    dvo, deo = to_dev64(vo, dev), to_dev64(eo, dev)
    return cc.labels_batch_device(to_dev(u, dev), to_dev(v, dev), dvo, deo, max_n, out,
                                  options=options, stream=stream)


def test_batch_device_offsets_match_oracle(dev):
    """Offsets in device memory: graphs ordered and described on the device.
    Empty graphs, single vertices, every slot width (32-bit up to 32,768
    vertices, 16-bit above) and every segment schedule equal the oracle."""
    rng = np.random.default_rng(18)
    sizes = [0, 1, 2, 300, 65536, 7, 40000, 0, 1000, 32768, 32769, 5]
    us, vs, vo, eo = [], [], [0], [0]
    for i, n in enumerate(sizes):
        m = 0 if n == 0 else int(rng.integers(0, 3 * n + 2))
        uu, vv = graphgen.uniform_pairs(m, max(n, 1), seed=150 + i, stream=0)
        us.append(uu)
        vs.append(vv)
        vo.append(vo[-1] + n)
        eo.append(eo[-1] + m)
    u, v = np.concatenate(us), np.concatenate(vs)
    vo, eo = np.array(vo, np.int64), np.array(eo, np.int64)
    want = oracle.labels_batch(u, v, vo, eo)
    for opt in (None, cc.Options(segments=1), cc.Options(segments=5, path_halving="off"),
                cc.Options(segments=0, path_halving="off"), cc.Options(block=256)):
        say("batch device offsets", opt)
        got = _batch_device(u, v, vo, eo, dev, 65536, options=opt).cpu().numpy()
        assert np.array_equal(got, want), opt
    # a tight bound on the vertex count (smaller LDS, more workgroups per CU)
    small = [i for i, n in enumerate(sizes) if n <= 1000]
    su = np.concatenate([us[i] for i in small])
    sv = np.concatenate([vs[i] for i in small])
    svo = np.concatenate([[0], np.cumsum([sizes[i] for i in small])]).astype(np.int64)
    seo = np.concatenate([[0], np.cumsum([len(us[i]) for i in small])]).astype(np.int64)
    got = _batch_device(su, sv, svo, seo, dev, 1000).cpu().numpy()
    assert np.array_equal(got, oracle.labels_batch(su, sv, svo, seo))
    # exhaustive tiny graphs, the same as the host-offset test
    graphs = []
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            graphs.append((n, [pairs[k] for k in range(len(pairs)) if mask >> k & 1]))
    tvo = np.concatenate([[0], np.cumsum([n for n, _ in graphs])]).astype(np.int64)
    teo = np.concatenate([[0], np.cumsum([len(c) for _, c in graphs])]).astype(np.int64)
    tu = np.array([b for _, c in graphs for _, b in c], np.int32)
    tv = np.array([a for _, c in graphs for a, _ in c], np.int32)
    want = np.concatenate([pins.closure_labels(tu[teo[g]:teo[g + 1]], tv[teo[g]:teo[g + 1]], n)
                           for g, (n, _) in enumerate(graphs)])
    assert np.array_equal(_batch_device(tu, tv, tvo, teo, dev, 5).cpu().numpy(), want)
    # one graph; graphs without vertices only; more graphs than one preparation
    # workgroup takes (1,024), most of them empty
    one_u, one_v = np.array([3, 1], np.int32), np.array([1, 0], np.int32)
    got = _batch_device(one_u, one_v, np.array([0, 5], np.int64), np.array([0, 2], np.int64), dev, 5)
    assert np.array_equal(got.cpu().numpy(), [0, 0, 2, 0, 4])
    empty = np.zeros(4, np.int64)
    got = _batch_device(np.zeros(0, np.int32), np.zeros(0, np.int32), empty, empty, dev, 1)
    assert (got.cpu().numpy() == -1).all()  # nothing written
    B = 2500
    nv = np.where(np.arange(B) % 7 == 3, 3, 0).astype(np.int64)
    me = np.where(nv > 0, 1, 0).astype(np.int64)
    bvo = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    beo = np.concatenate([[0], np.cumsum(me)]).astype(np.int64)
    bu = np.full(int(beo[-1]), 2, np.int32)
    bv = np.zeros(int(beo[-1]), np.int32)
    got = _batch_device(bu, bv, bvo, beo, dev, 3).cpu().numpy()
    assert np.array_equal(got, oracle.labels_batch(bu, bv, bvo, beo))


def test_batch_preparation_scan_path(dev):
    """More than 32 preparation workgroups (32,768 graphs): a scan launch
    turns the per-workgroup class counts into prefix sums before the
    descriptors are placed.  Sizes spread over many classes, with empty
    graphs; offsets on the device and on the host; an invalid graph among
    them is reported and the valid ones are still solved."""
    import torch
    rs = np.random.default_rng(19)
    B = 40000
    nv = rs.integers(0, 40, B).astype(np.int64)
    nv[rs.integers(0, B, 25)] = rs.integers(1000, 5000, 25)
    me = (nv * rs.uniform(0.0, 1.5, B)).astype(np.int64)
    me[nv == 0] = 0
    vo = np.concatenate([[0], np.cumsum(nv)]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum(me)]).astype(np.int64)
    gid = np.repeat(np.arange(B), me)
    u = (rs.random(len(gid)) * nv[gid]).astype(np.int32)
    v = (rs.random(len(gid)) * nv[gid]).astype(np.int32)
    want = oracle.labels_batch(u, v, vo, eo)
    say("batch scan path", B, int(vo[-1]), int(eo[-1]))
    got = _batch_device(u, v, vo, eo, dev, 5000).cpu().numpy()
    assert np.array_equal(got, want)
    got = cc.labels_batch(to_dev(u, dev), to_dev(v, dev), vo, eo).cpu().numpy()
    assert np.array_equal(got, want)
    # the largest graph above max_n: CC_ERR_ARG, the other graphs' labels written
    big = int(np.argmax(nv))
    out = torch.full((int(vo[-1]),), -1, dtype=torch.int32, device=dev)
    with pytest.raises(cc.CCError) as ei:
        cc.labels_batch_device(to_dev(u, dev), to_dev(v, dev), to_dev64(vo, dev),
                               to_dev64(eo, dev), int(nv[big]) - 1, out)
    assert ei.value.code == cc.CC_ERR_ARG
    got = out.cpu().numpy()
    keep = np.ones(int(vo[-1]), bool)
    keep[vo[big]:vo[big + 1]] = False
    assert np.array_equal(got[keep], want[keep])
    assert (got[~keep] == -1).all()


def test_batch_device_offsets_errors_and_replays(dev):
    import torch
    u = np.array([0, 1, 1, 2], np.int32)
    v = np.array([1, 2, 0, 3], np.int32)
    vo = np.array([0, 3, 7], np.int64)
    eo = np.array([0, 2, 4], np.int64)
    want = oracle.labels_batch(u, v, vo, eo)
    assert np.array_equal(_batch_device(u, v, vo, eo, dev, 4).cpu().numpy(), want)
    # a graph above max_n: CC_ERR_ARG, no label written for it, the others solved
    with pytest.raises(cc.CCError) as ei:
        _batch_device(u, v, vo, eo, dev, 3)
    assert ei.value.code == cc.CC_ERR_ARG
    out = torch.full((7,), -1, dtype=torch.int32, device=dev)
    dvo, deo = to_dev64(vo, dev), to_dev64(eo, dev)
    with pytest.raises(cc.CCError):
        cc.labels_batch_device(to_dev(u, dev), to_dev(v, dev), dvo, deo, 3, out)
    got = out.cpu().numpy()
    assert np.array_equal(got[:3], want[:3]) and (got[3:] == -1).all()
    # offsets that decrease or do not start at 0
    for bad_vo, bad_eo in (([0, 5, 4], [0, 2, 4]), ([1, 3, 7], [0, 2, 4]), ([0, 3, 7], [0, 3, 2])):
        with pytest.raises(cc.CCError) as ei:
            _batch_device(u, v, np.array(bad_vo, np.int64), np.array(bad_eo, np.int64), dev, 8)
        assert ei.value.code == cc.CC_ERR_ARG, (bad_vo, bad_eo)
    # an endpoint outside its graph, and entries in a graph without vertices
    with pytest.raises(cc.CCError) as ei:
        _batch_device(np.array([0, 5], np.int32), np.array([1, 0], np.int32),
                      np.array([0, 3, 7], np.int64), np.array([0, 1, 2], np.int64), dev, 4)
    assert ei.value.code == cc.CC_ERR_RANGE
    with pytest.raises(cc.CCError) as ei:
        _batch_device(u, v, np.array([0, 0, 7], np.int64), eo, dev, 8)
    assert ei.value.code == cc.CC_ERR_RANGE
    # host-side argument checks
    for mx in (0, 65537):
        with pytest.raises(cc.CCError) as ei:
            _batch_device(u, v, vo, eo, dev, mx)
        assert ei.value.code == cc.CC_ERR_ARG
    # a captured launch sequence replayed, with eager calls in between
    bu, bv, bvo, beo = graphgen.batch_er(300, seed=85, lo_exp=6, hi_exp=16)
    bwant = oracle.labels_batch(bu, bv, bvo, beo)
    s = torch.cuda.Stream()
    dbu, dbv, dbvo, dbeo = to_dev(bu, dev), to_dev(bv, dev), to_dev64(bvo, dev), to_dev64(beo, dev)
    bout = torch.empty(int(bvo[-1]), dtype=torch.int32, device=dev)
    for rep in range(4):
        with torch.cuda.stream(s):
            bout.fill_(-1)
            cc.labels_batch_device(dbu, dbv, dbvo, dbeo, 65536, bout,
                                   options=cc.Options(graph=True), stream=s)
            got = bout.cpu().numpy()
        assert np.array_equal(got, bwant), rep
        assert np.array_equal(_batch_device(bu, bv, bvo, beo, dev, 65536).cpu().numpy(), bwant)
        torch.cuda.synchronize()


# ----------------------------------------------------------------------------- full size
def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["er16", "grid4k", "rmat24"])
def test_full_size_workloads_match_oracle_digest(dev, name):
    rec = _golden()[name]
    say("generating", name)
    u, v, n = graphgen.workload(name)
    assert (n, len(u)) == (rec["n"], rec["m"])
    du, dv = to_dev(u, dev), to_dev(v, dev)
    del u, v
    for opt in ("default", "plain", "atomic", "s1", "coherent_giant", "s6_giant_nohot_e4",
                "s12_giant_hotlarge_e16", "s10_giant_hotvertex", "s8_giant_nohalve", "hybrid"):
        if name == "rmat24" and opt == "s1":
            opt = "s9_giant_after3"
        say("full size", name, opt)
        lab = cc.labels(du, dv, n, options=VARIANTS[opt]).cpu().numpy()
        assert int(np.count_nonzero(lab == np.arange(n))) == rec["components"], (name, opt)
        assert digest(lab) == rec["sha256"], (name, opt)


def test_window_round_with_and_without_locality(dev):
    """The hybrid plan's window round on lattices whose entries keep, lose or
    reverse their locality: row-major ids (nearly every entry joined in an
    LDS window), the same lattice with permuted ids or shuffled entries
    (nearly every entry outside the windows: the gated Multi-Jump runs), and
    both orientations of each entry; a lattice wider than a window (rows of
    50,000 vertices), and a graph smaller than one window."""
    rng = np.random.default_rng(23)
    u, v, n = graphgen.grid(1500, 1000, 3, 10, seed=231)
    perm = rng.permutation(n).astype(np.int32)
    order = rng.permutation(len(u))
    wide_u, wide_v, wide_n = graphgen.grid(50000, 40, 3, 10, seed=232)
    cases = {
        "row-major": (u, v, n),
        "permuted ids": (perm[u], perm[v], n),
        "shuffled entries": (u[order], v[order], n),
        "both orientations": (np.concatenate([u, v]), np.concatenate([v, u]), n),
        "reversed pairs": (v, u, n),
        "rows wider than a window": (wide_u, wide_v, wide_n),
        "smaller than a window": (u[u < 20000] % 20000, v[u < 20000] % 20000, 20000),
    }
    for name, (a, b, nn) in cases.items():
        say("window round", name, nn, len(a))
        want = oracle.labels(a, b, nn)
        for opt in (cc.Options(hook="hybrid"), cc.Options(hook="hybrid", path_halving="off")):
            assert np.array_equal(solve(a, b, nn, dev, opt), want), name


def test_repeated_solves_on_deep_trees_stay_exact(dev):
    """Regression: concurrent hooks and path-halving re-points race on the same
    cache lines from different XCDs; on the grid (deep trees, many re-points)
    a lost hook shows up only in some solves, so every one of many solves of
    each Atomic-Hook path (pair list, LDS hot cache, coherent loads, CSR) is
    compared with the oracle's labels."""
    rec = _golden()["grid4k"]
    u, v, n = graphgen.workload("grid4k")
    want_np = oracle.labels(u, v, n)
    assert digest(want_np) == rec["sha256"]
    want = torch.from_numpy(want_np).to(dev)
    du, dv = to_dev(u, dev), to_dev(v, dev)
    del u, v, want_np
    out = torch.empty(n, dtype=torch.int32, device=dev)
    reps = 12
    for opt in ("default", "s1", "s12_giant_hotlarge_e16", "s10_giant_hotvertex",
                "s5_giant_b1024_e16", "coherent_s3",
                "hybrid"):
        say("repeated solves grid4k", opt, reps)
        bad = 0
        for _ in range(reps):
            cc.labels(du, dv, n, out=out, options=VARIANTS[opt])
            bad += not torch.equal(out, want)
        assert bad == 0, (opt, bad, reps)
    say("repeated solves grid4k csr", reps)
    _, order = torch.sort(du.to(torch.int64) * n + dv.to(torch.int64))
    col = dv[order].contiguous()
    rp = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rp[1:] = torch.cumsum(torch.bincount(du, minlength=n), 0)
    del order
    for opt in ("auto", "atomic", "hybrid"):
        bad = 0
        for _ in range(reps):
            cc.labels_csr(rp, col, n, out=out, options=cc.Options(hook=opt))
            bad += not torch.equal(out, want)
        assert bad == 0, ("csr", opt, bad, reps)


def test_full_size_batch_matches_oracle_digest(dev):
    rec = _golden()["batch10k"]
    u, v, vo, eo = graphgen.batch_er(10000, seed=1004)
    assert (int(vo[-1]), len(u)) == (rec["n"], rec["m"])
    say("full size batch10k")
    du, dv = to_dev(u, dev), to_dev(v, dev)
    for cap, halve, block in ((0, "auto", 0), (1, "auto", 0), (3, "auto", 0), (0, "off", 0),
                              (3, "off", 0), (0, "auto", 256), (2, "auto", 512)):
        lab = cc.labels_batch(du, dv, vo, eo,
                              options=cc.Options(segments=cap, path_halving=halve,
                                                 block=block)).cpu().numpy()
        assert digest(lab) == rec["sha256"], (cap, halve, block)
    # the same batch with its offsets in device memory
    dvo, deo = to_dev64(vo, dev), to_dev64(eo, dev)
    out = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    max_n = int(np.diff(vo).max())
    for opt in (cc.Options(), cc.Options(segments=3, path_halving="off")):
        out.fill_(-1)
        lab = cc.labels_batch_device(du, dv, dvo, deo, max_n, out, options=opt).cpu().numpy()
        assert digest(lab) == rec["sha256"], ("device offsets", opt)


# ----------------------------------------------------------------------------- streamed (host edges)
@pytest.mark.parametrize("filt", ["auto", "off", "giant"])
def test_streamed_host_edges_match_oracle(dev, filt):
    """Edges stay in host memory (pinned and pageable) and are streamed in
    chunks; ragged last chunk; labels equal the oracle's."""
    cases = [graphgen.rmat(16, 16, seed=41, symmetrize=True),
             graphgen.grid(300, 200, 3, 10, seed=42),
             graphgen.er_planted(n=1 << 14, m_er=1 << 16, cliques=32, seed=43)[:3]]
    for u, v, n in cases:
        want = oracle.labels(u, v, n)
        for chunk in (4, 1000, 65537, len(u) + 8):
            say("streamed", filt, n, len(u), chunk)
            got = cc.labels_host(u, v, n, chunk=chunk, options=cc.Options(filter=filt)).cpu().numpy()
            assert np.array_equal(got, want), (n, chunk, filt)
        pu = torch.from_numpy(u).pin_memory()
        pv = torch.from_numpy(v).pin_memory()
        got, st = cc.labels_host(pu, pv, n, chunk=1 << 15, options=cc.Options(filter=filt),
                                 return_stats=True)
        assert np.array_equal(got.cpu().numpy(), want)
        assert st["segments"] == (len(u) + (1 << 15) - 1) // (1 << 15)


def test_streamed_range_error_and_full_size(dev):
    with pytest.raises(cc.CCError) as ei:
        cc.labels_host(np.array([0, 7], np.int32), np.array([1, 2], np.int32), 5, chunk=4)
    assert ei.value.code == cc.CC_ERR_RANGE
    rec = _golden()["grid4k"]
    u, v, n = graphgen.workload("grid4k")
    pu = torch.from_numpy(u).pin_memory()
    pv = torch.from_numpy(v).pin_memory()
    lab = cc.labels_host(pu, pv, n, chunk=1 << 22).cpu().numpy()
    assert digest(lab) == rec["sha256"]


# ----------------------------------------------------------------------------- symmetric flag
def test_symmetric_flag_on_symmetrised_lists(dev):
    """cc_options.symmetric hooks only entries with u <= v; on a list that
    holds every pair in both orientations the labels are unchanged."""
    for u, v, n in [graphgen.rmat(16, 8, seed=61, symmetrize=True),
                    graphgen.rmat(12, 4, seed=62, symmetrize=True)]:
        want = oracle.labels(u, v, n)
        for opt in (cc.Options(symmetric=True), cc.Options(symmetric=True, hook="atomic",
                                                           filter="giant", segments=16),
                    cc.Options(symmetric=True, hook="atomic", filter="off", segments=3)):
            assert np.array_equal(solve(u, v, n, dev, opt), want)
        got = cc.labels_host(u, v, n, chunk=10000, options=cc.Options(symmetric=True))
        assert np.array_equal(got.cpu().numpy(), want)
    rec = _golden()["rmat24"]
    u, v, n = graphgen.workload("rmat24")
    du, dv = to_dev(u, dev), to_dev(v, dev)
    del u, v
    lab = cc.labels(du, dv, n, options=cc.Options(symmetric=True)).cpu().numpy()
    assert digest(lab) == rec["sha256"]


# ----------------------------------------------------------------------------- CSR input
def _to_csr(u, v, n):
    """CSR adjacency of the pair list (rows sorted, column order within a row kept)."""
    order = np.argsort(u, kind="stable")
    col = np.ascontiguousarray(v[order].astype(np.int32))
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(u, minlength=n), out=row_ptr[1:])
    return row_ptr, col


def test_csr_input_matches_oracle(dev):
    cases = {
        "rmat_sym": graphgen.rmat(15, 16, seed=71, symmetrize=True),
        "grid": graphgen.grid(200, 150, 3, 10, seed=72),
        "sparse_many_empty_rows": (lambda p: (p[0], p[1], 200000))(graphgen.uniform_pairs(30000, 200000, 73, 0)),
        "hub_rows": (np.concatenate([np.zeros(50000, np.int32), np.arange(1, 4000, dtype=np.int32)]),
                     np.concatenate([np.arange(50000, dtype=np.int32) % 9000, np.arange(1, 4000, dtype=np.int32)]),
                     9000),
        "empty": (np.zeros(0, np.int32), np.zeros(0, np.int32), 17),
    }
    for name, (u, v, n) in cases.items():
        want = oracle.labels(u, v, n)
        rp, col = _to_csr(u, v, n)
        drp = torch.from_numpy(rp).to(dev)
        dcol = to_dev(col, dev)
        for opt in (cc.Options(), cc.Options(filter="giant", segments=8),
                    cc.Options(filter="off", segments=3, path_halving="off"),
                    cc.Options(hook="hybrid"), cc.Options(hook="hybrid", path_halving="off"),
                    cc.Options(filter="giant", segments=6, hot_cache="off"),
                    cc.Options(filter="giant", segments=12, filter_after=2, path_halving="off")):
            say("csr", name, opt.hook, opt.filter, opt.segments, opt.hot_cache)
            got = cc.labels_csr(drp, dcol, n, options=opt).cpu().numpy()
            assert np.array_equal(got, want), (name, opt)
        if name == "rmat_sym":
            for opt in (cc.Options(symmetric=True),
                        cc.Options(symmetric=True, filter="giant", segments=8),
                        cc.Options(symmetric=True, hook="hybrid")):
                got = cc.labels_csr(drp, dcol, n, options=opt).cpu().numpy()
                assert np.array_equal(got, want)
            # the flag hooks exactly the entries with col > row: an adjacency
            # holding only those gives the same labels
            keep = v > u
            rp2, col2 = _to_csr(u[keep], v[keep], n)
            for opt in (cc.Options(symmetric=True), cc.Options(symmetric=True, hook="hybrid")):
                got = cc.labels_csr(torch.from_numpy(rp2).to(dev), to_dev(col2, dev), n,
                                    options=opt).cpu().numpy()
                assert np.array_equal(got, want)


def test_csr_rejects_malformed_input(dev):
    col = to_dev(np.array([1, 2, 0], np.int32), dev)
    for rp in ([0, 2, 1, 3], [1, 2, 3, 3], [0, 1, 2, 4]):
        with pytest.raises(cc.CCError) as ei:
            cc.labels_csr(torch.tensor(rp, dtype=torch.int64, device=dev), col, 3)
        assert ei.value.code == cc.CC_ERR_RANGE
    with pytest.raises(cc.CCError) as ei:
        cc.labels_csr(torch.tensor([0, 1, 2, 3], dtype=torch.int64, device=dev),
                      to_dev(np.array([1, 5, 0], np.int32), dev), 3)
    assert ei.value.code == cc.CC_ERR_RANGE


def test_csr_full_size_rmat24(dev):
    rec = _golden()["rmat24"]
    u, v, n = graphgen.workload("rmat24")
    du, dv = to_dev(u, dev), to_dev(v, dev)
    del u, v
    key, order = torch.sort(du.to(torch.int64) * n + dv.to(torch.int64))
    del key
    col = dv[order].contiguous()
    counts = torch.bincount(du, minlength=n)
    rp = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rp[1:] = torch.cumsum(counts, 0)
    del du, dv, order
    for opt in (cc.Options(), cc.Options(symmetric=True), cc.Options(hook="hybrid"),
                cc.Options(hot_cache="off")):
        lab = cc.labels_csr(rp, col, n, options=opt).cpu().numpy()
        assert digest(lab) == rec["sha256"], opt


def test_vertex_table_past_its_tag_range(dev):
    """The vertex table caches ids below 255 * 81,920 only; forced on a graph
    of 2^25 vertices, the ids above that range (more than a third of them)
    are always tested in the bitmap.  A skewed graph with a giant component,
    so the filter and the table are both used; labels against the oracle."""
    u, v, n = graphgen.rmat(25, 2, seed=77, m=(1 << 24))
    assert n > 255 * 81920
    want = oracle.labels(u, v, n)
    du, dv = to_dev(u, dev), to_dev(v, dev)
    for opt in (cc.Options(hook="atomic", segments=64, filter="giant", hot_cache="vertex"),
                cc.Options(hook="atomic", segments=32, filter="giant", hot_cache="vertex",
                           path_halving="off"),
                cc.Options()):
        say("vertex table past its tag range", opt.segments, opt.hot_cache)
        lab, st = cc.labels(du, dv, n, options=opt, return_stats=True)
        assert np.array_equal(lab.cpu().numpy(), want), opt
        if opt.hot_cache == "vertex":
            assert st["filter_used"] == 1


def test_deep_chains_with_a_ragged_last_block(dev):
    """Two interleaved paths (edges (v, v + 2)) on 2^22 + 5 vertices, in a
    seeded shuffled order: the atomic-free pass leaves chains thousands of
    levels deep, which the block-local jumping (blocks of 16,384 vertices,
    the last one ragged) and the following Multi-Jump must flatten.  Closed
    form: label[v] = v mod 2.  Atomic-free rounds, the hybrid plan and the
    CSR hybrid."""
    n = (1 << 22) + 5
    a = np.arange(n - 2, dtype=np.int32)
    perm = graphgen.permutation(n - 2, seed=81)
    u, v = a[perm], a[perm] + 2
    want = np.arange(n, dtype=np.int32) % 2
    du, dv = to_dev(u, dev), to_dev(v, dev)
    for opt in (cc.Options(hook="plain"), cc.Options(hook="hybrid"), cc.Options()):
        say("deep chains", opt.hook)
        assert np.array_equal(cc.labels(du, dv, n, options=opt).cpu().numpy(), want), opt.hook
    rp, col = _to_csr(u, v, n)
    got = cc.labels_csr(torch.from_numpy(rp).to(dev), to_dev(col, dev), n,
                        options=cc.Options(hook="hybrid")).cpu().numpy()
    assert np.array_equal(got, want)


# ----------------------------------------------------------------------------- maximum sizes
def test_max_vertex_count(dev):
    """n = 2^31 - 1 (the largest int32 vertex count): edges between far-apart
    ids; closed form: {0, n-1, n-2} -> 0, {5, n-3, 2^30} -> 5, the rest alone."""
    n = (1 << 31) - 1
    u = torch.tensor([0, n - 1, 5, 1 << 30], dtype=torch.int32, device=dev)
    v = torch.tensor([n - 1, n - 2, n - 3, n - 3], dtype=torch.int32, device=dev)
    want = torch.arange(n, dtype=torch.int32, device=dev)
    want[n - 1] = 0
    want[n - 2] = 0
    want[n - 3] = 5
    want[1 << 30] = 5
    out = torch.empty(n, dtype=torch.int32, device=dev)
    for name in ("default", "atomic", "plain"):
        say("n = 2^31 - 1", name)
        out.fill_(-1)
        cc.labels(u, v, n, out=out, options=VARIANTS[name])
        assert torch.equal(out, want), name
    del out, want
    torch.cuda.empty_cache()


def test_more_than_2_31_entries(dev):
    """m = 2^31 + 12 entries (64-bit entry indices): a cycle over P = 2^20 ids
    repeated, then four distinctive pairs stored beyond entry 2^31;
    closed form: [0, P) -> 0, {P+5, P+7, P+11} -> P+5, {P+8, P+9} -> P+8,
    {P+20, P+21} -> P+20, the rest alone."""
    P = 1 << 20
    n = (1 << 21) + 64
    m = (1 << 31) + 12
    u = torch.empty(m, dtype=torch.int32, device=dev)
    v = torch.empty(m, dtype=torch.int32, device=dev)
    chunk = 1 << 28
    for start in range(0, m - 4, chunk):
        end = min(m - 4, start + chunk)
        k = torch.arange(start, end, dtype=torch.int64, device=dev)
        u[start:end] = (k % P).to(torch.int32)
        v[start:end] = ((k + 1) % P).to(torch.int32)
        del k
    u[m - 4:] = torch.tensor([P + 5, P + 9, P + 7, P + 20], dtype=torch.int32, device=dev)
    v[m - 4:] = torch.tensor([P + 7, P + 8, P + 11, P + 21], dtype=torch.int32, device=dev)
    want = torch.arange(n, dtype=torch.int32, device=dev)
    want[:P] = 0
    want[P + 7] = P + 5
    want[P + 11] = P + 5
    want[P + 9] = P + 8
    want[P + 21] = P + 20
    out = torch.empty(n, dtype=torch.int32, device=dev)
    for name in ("default", "s1", "s5_giant_b1024_e16", "s3_nohalve"):
        say("m = 2^31 + 12", name)
        out.fill_(-1)
        cc.labels(u, v, n, out=out, options=VARIANTS[name])
        assert torch.equal(out, want), name
    del u, v, out, want
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------- no-sync calls
def test_no_sync_calls_queue_on_the_stream(dev):
    """opts.no_sync enqueues the solve and returns; several solves queued on one
    stream give the oracle's labels once the stream has passed them, and the
    device-detected status is read with cc_stream_status."""
    graphs = [graphgen.rmat(14, 8, seed=500 + i) for i in range(3)]
    graphs.append(graphgen.grid(300, 200, 1, 2, seed=510))
    want = [oracle.labels(u, v, n) for u, v, n in graphs]
    tens = [(to_dev(u, dev), to_dev(v, dev), n) for u, v, n in graphs]
    outs = [torch.empty(n, dtype=torch.int32, device=dev) for _, _, n in graphs]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for opt in (cc.Options(no_sync=True),
                    cc.Options(no_sync=True, filter="giant", segments=8),
                    cc.Options(no_sync=True, graph=True)):
            for o in outs:
                o.fill_(-7)
            torch.cuda.synchronize()
            for (du, dv, n), o in zip(tens, outs):
                cc.labels(du, dv, n, out=o, options=opt, stream=s)
            assert cc.stream_status(s) in (0, cc.CC_PENDING)
            s.synchronize()
            assert cc.stream_status(s) == 0
            for o, w in zip(outs, want):
                assert np.array_equal(o.cpu().numpy(), w)
        # a range error is reported by the status, and the next call clears it
        bad_u = to_dev(np.array([0, 1, 9], np.int32), dev)
        bad_v = to_dev(np.array([1, 2, 3], np.int32), dev)
        o5 = torch.empty(5, dtype=torch.int32, device=dev)
        cc.labels(bad_u, bad_v, 5, out=o5, options=cc.Options(no_sync=True), stream=s)
        s.synchronize()
        with pytest.raises(cc.CCError) as ei:
            cc.stream_status(s)
        assert ei.value.code == cc.CC_ERR_RANGE
        du, dv, n = tens[0]
        cc.labels(du, dv, n, out=outs[0], options=cc.Options(no_sync=True), stream=s)
        s.synchronize()
        assert cc.stream_status(s) == 0
        assert np.array_equal(outs[0].cpu().numpy(), want[0])
        # CSR input
        u, v, n = graphs[0]
        rp, col = _to_csr(u, v, n)
        o = torch.empty(n, dtype=torch.int32, device=dev)
        drp, dcol = torch.from_numpy(rp).to(dev), to_dev(col, dev)  # alive until the sync
        cc.labels_csr(drp, dcol, n, out=o, options=cc.Options(no_sync=True), stream=s)
        s.synchronize()
        assert cc.stream_status(s) == 0
        assert np.array_equal(o.cpu().numpy(), want[0])
        with pytest.raises(cc.CCError):
            cc.labels(du, dv, n, options=cc.Options(no_sync=True, hook="plain"), stream=s)


# ----------------------------------------------------------------------------- hipGraph replay
def test_graph_capture_replays_match_eager(dev):
    """cc_options.graph captures the launch sequence once and replays it; every
    replay (with eager work and synchronisations in between) equals the eager
    result, for single solves (with and without the filter) and for batches."""
    s = torch.cuda.Stream()
    u, v, n = graphgen.rmat(17, 16, seed=81, symmetrize=True)
    want = oracle.labels(u, v, n)
    du, dv = to_dev(u, dev), to_dev(v, dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    for opt in (cc.Options(hook="atomic", graph=True),
                cc.Options(hook="atomic", filter="giant", segments=64, graph=True),
                cc.Options(hook="atomic", filter="giant", segments=64, hot_cache="large", graph=True),
                cc.Options(hook="atomic", filter="off", segments=3, graph=True),
                cc.Options(hook="plain", graph=True),
                cc.Options(hook="plain", graph=True, rounds_per_check=1, compact_threshold=500)):
        for rep in range(4):
            with torch.cuda.stream(s):
                out.fill_(-1)
                cc.labels(du, dv, n, out=out, options=opt, stream=s)
                got = out.cpu().numpy()
            assert np.array_equal(got, want), rep
            # eager work between replays
            assert np.array_equal(cc.labels(du, dv, n).cpu().numpy(), want)
            torch.cuda.synchronize()
    bu, bv, vo, eo = graphgen.batch_er(300, seed=82, lo_exp=6, hi_exp=17)
    bwant = oracle.labels_batch(bu, bv, vo, eo)
    dbu, dbv = to_dev(bu, dev), to_dev(bv, dev)
    bout = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    for rep in range(4):
        with torch.cuda.stream(s):
            bout.fill_(-1)
            cc.labels_batch(dbu, dbv, vo, eo, out=bout, options=cc.Options(graph=True, segments=2),
                            stream=s)
            got = bout.cpu().numpy()
        assert np.array_equal(got, bwant), rep
        assert np.array_equal(cc.labels_batch(dbu, dbv, vo, eo).cpu().numpy(), bwant)
        torch.cuda.synchronize()
    # Two batches of the same shapes (all graphs LDS-solved) but different
    # contents share one captured graph: the descriptors are re-read from the
    # staging buffer at every replay, so alternating them stays exact.
    cu, cv, co, ce = graphgen.batch_er(300, seed=84, lo_exp=6, hi_exp=15)
    ng = np.repeat(np.diff(co), np.diff(ce)).astype(np.int32)
    cu2, cv2 = (ng - 1 - cu).astype(np.int32), (ng - 1 - cv).astype(np.int32)  # mirrored ids
    cwant = oracle.labels_batch(cu, cv, co, ce)
    cwant2 = oracle.labels_batch(cu2, cv2, co, ce)
    assert not np.array_equal(cwant, cwant2)
    cout = torch.empty(int(co[-1]), dtype=torch.int32, device=dev)
    pairs = ((to_dev(cu, dev), to_dev(cv, dev), cwant), (to_dev(cu2, dev), to_dev(cv2, dev), cwant2))
    for rep in range(3):
        for xu, xv, w in pairs:
            with torch.cuda.stream(s):
                cout.fill_(-1)
                cc.labels_batch(xu, xv, co, ce, out=cout, options=cc.Options(graph=True), stream=s)
                got = cout.cpu().numpy()
            assert np.array_equal(got, w), rep
