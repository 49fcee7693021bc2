"""Plan autotuner: the cache and shape keys on the host; on the GPU, a tuned
plan (single graphs and batches) still gives the oracle's labels, and the
search covers the knobs it claims to (segments, filter, tile, block, the
frontier compaction threshold when the atomic-free Hook wins, the LDS table
when the filter does)."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1612_01178_amd as cc
from paper_1612_01178_amd import autotune


def test_shape_key_buckets():
    assert autotune.shape_key(1 << 16, 1 << 19) == "gfx950:n2^16:d2^3"
    # same bucket for nearby shapes, different for another degree
    assert autotune.shape_key(70000, 560000) == autotune.shape_key(1 << 16, 1 << 19)
    assert autotune.shape_key(1 << 16, 1 << 16) != autotune.shape_key(1 << 16, 1 << 19)
    assert autotune.shape_key(1 << 10, 100) == "gfx950:n2^10:d2^-3"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert autotune.options_for(1 << 16, 1 << 19, path=path) == cc.Options()
    opt = cc.Options(hook="plain", edges_per_thread=16, compact_threshold=250)
    autotune._store(path, autotune.shape_key(1 << 16, 1 << 19),
                    {"options": opt.__dict__, "ms": 0.1, "n": 1 << 16, "m": 1 << 19})
    assert autotune.options_for(1 << 16, 1 << 19, path=path) == opt
    assert autotune.options_for(1 << 20, 1 << 19, path=path) == cc.Options()


def test_search_on_a_cost_model(monkeypatch):
    """The coordinate search with the solver replaced by a cost model on the
    host: a filtered plan wins the first coordinate, so the LDS-table
    coordinate is searched too, and every coordinate's best value is kept."""
    torch = pytest.importorskip("torch")

    def cost(u, v, n, out, opt, reps):
        t = 10.0
        if opt.filter == "giant":
            t -= 4.0 - 0.01 * opt.segments  # fewest segments among the filtered plans
        t -= {"large": 1.0, "vertex": 0.5}.get(opt.hot_cache, 0.0)
        t -= 0.25 if opt.block == 512 else 0.0
        t -= 0.125 if opt.edges_per_thread == 16 else 0.0
        return t

    monkeypatch.setattr(autotune, "_time", cost)
    n, m = 1 << 16, 1 << 20
    u = torch.zeros(1, dtype=torch.int32).expand(m)  # only its length is used
    best, table = autotune.tune(u, u, n, reps=1, cache=False)
    assert (best.hook, best.filter, best.segments) == ("atomic", "giant", 4)
    assert (best.hot_cache, best.block, best.edges_per_thread) == ("large", 512, 16)
    assert {o["hot_cache"] for _, o in table} == {"auto", "vertex", "large", "off"}
    assert "compact_threshold" not in {k for _, o in table for k, val in o.items()
                                       if val != getattr(cc.Options(), k)}


@pytest.mark.gpu
def test_tuned_plans_are_exact(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    u, v, n, _ = graphgen.er_planted(1 << 14, 1 << 17, 16, seed=61)
    want = oracle.labels(u, v, n)
    du, dv = torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)
    path = str(tmp_path / "tune.json")
    print("tune er 2^14", flush=True)
    best, table = autotune.tune(du, dv, n, reps=1, path=path)
    fields = {k for _, o in table for k, val in o.items() if val != getattr(cc.Options(), k)}
    assert {"hook", "segments", "filter", "edges_per_thread", "block"} <= fields
    assert {o["hook"] for _, o in table} >= {"auto", "plain", "hybrid", "atomic"}
    if best.hook in ("plain", "auto"):
        assert "compact_threshold" in fields
    assert autotune.options_for(n, len(u), path=path) == best
    for _, o in table:
        got = cc.labels(du, dv, n, options=cc.Options(**o)).cpu().numpy()
        assert np.array_equal(got, want), o
    # batches: halving in the LDS climb and the segment cap
    bu, bv, vo, eo = graphgen.batch_er(60, seed=62, lo_exp=6.0, hi_exp=12.0)
    bwant = oracle.labels_batch(bu, bv, vo, eo)
    dbu, dbv = torch.from_numpy(bu).to(dev), torch.from_numpy(bv).to(dev)
    print("tune batch of 60", flush=True)
    bopt, btable = autotune.tune_batch(dbu, dbv, vo, eo, reps=1)
    default_block = cc.Options().block
    assert sorted((o["path_halving"], o["segments"]) for _, o in btable
                  if o["block"] == default_block) == \
        [("auto", 1), ("auto", 2), ("auto", 4), ("auto", 8), ("off", 0), ("off", 4), ("off", 8)]
    # then the workgroup size, around the best of those
    sized = [o for _, o in btable if o["block"] != default_block]
    assert sorted(o["block"] for o in sized) == [256, 512]
    assert len({(o["path_halving"], o["segments"]) for o in sized}) == 1
    for _, o in btable:
        got = cc.labels_batch(dbu, dbv, vo, eo, options=cc.Options(**o)).cpu().numpy()
        assert np.array_equal(got, bwant), o
