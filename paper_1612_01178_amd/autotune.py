"""Plan autotuner for the solver.

Every plan the library accepts computes exactly the same labels (the
smallest id of each component), so a plan can be chosen purely on speed.
``tune`` times candidate plans on the caller's own graph with the real
solver (cc_labels_ex through the C ABI) and returns the fastest, searching
coordinate by coordinate from the library's default:

1. hook variant and Hook-to-Compress switch: the paper's segment count
   s = round(m / n) (Section 3.B) and multiples of it, with and without the
   giant-component filter, plus the atomic-free Hook and the hybrid plan;
2. edge entries per thread (4, 8, 16);
3. threads per workgroup (256, 512, 1024);
4. when the atomic-free Hook wins, the frontier compaction threshold tau
   (rewrite the frontier every round, or only below a surviving fraction of
   50 %, 25 %, 10 %);
5. when the giant-component filter is in the plan, its LDS table: the
   two-way vertex table, the bitmap-word table, or none.

``tune_batch`` does the same for the batched LDS solver: path halving in
the LDS climb and the per-graph segment cap.

Results are cached in a JSON file keyed by device architecture and a shape
bucket (log2 n, m/n rounded to a power of two), so graphs of a similar shape
reuse a plan without re-timing.  ``options_for(n, m)`` returns the cached
plan, or the library default when there is none.
"""
from __future__ import annotations

import json
import math
import os
import threading
import time

from . import Options, labels, labels_batch

_CACHE_PATH = os.environ.get("HOOKCC_TUNE_CACHE",
                             os.path.join(os.path.expanduser("~"), ".cache", "hookcc", "tune.json"))
_lock = threading.Lock()


def shape_key(n: int, m: int, arch: str = "gfx950") -> str:
    lg_n = int(math.log2(max(n, 1)))
    deg = max(m, 1) / max(n, 1)
    lg_d = int(round(math.log2(deg))) if deg >= 1 else -int(round(math.log2(1.0 / deg)))
    return "%s:n2^%d:d2^%d" % (arch, lg_n, lg_d)


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, value: dict) -> None:
    with _lock:
        data = _load_cache(path)
        data[key] = value
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def options_for(n: int, m: int, path: str | None = None) -> Options:
    """The cached plan for a graph of this shape, else the library default."""
    rec = _load_cache(path or _CACHE_PATH).get(shape_key(n, m))
    return Options(**rec["options"]) if rec else Options()


def _time(u, v, n, out, opt: Options, reps: int) -> float:
    import torch
    labels(u, v, n, out=out, options=opt)  # warm (workspace, code objects)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        labels(u, v, n, out=out, options=opt)
        best = min(best, time.perf_counter() - t)
    return best * 1e3


def tune(u, v, n: int, *, reps: int = 3, cache: bool = True, path: str | None = None,
         log=None):
    """Times candidate plans on (u, v, n) and returns (best Options, table).

    ``table`` lists every candidate tried with its best time in ms."""
    import torch
    m = u.numel()
    out = torch.empty(n, dtype=torch.int32, device=u.device)
    s0 = max(1, round(m / max(n, 1)))
    tried = {}

    def run(opt: Options):
        key = tuple(sorted(opt.__dict__.items()))
        if key not in tried:
            tried[key] = (_time(u, v, n, out, opt, reps), opt)
            if log:
                log("tune %-70s %9.3f ms" % (opt, tried[key][0]))
        return tried[key][0]

    base = Options()
    best_t, best = run(base), base
    # 1. hook variant, segment count, filter
    cands = [Options(hook="plain"), Options(hook="hybrid")]
    for mult in (0.25, 0.5, 1, 2, 4, 8, 16):
        s = max(1, int(round(s0 * mult)))
        cands.append(Options(hook="atomic", segments=s, filter="off"))
        if s >= 4:
            cands.append(Options(hook="atomic", segments=s, filter="giant"))
    for c in cands:
        t = run(c)
        if t < best_t:
            best_t, best = t, c
    # 2. entries per thread, 3. workgroup size, 4. (atomic-free Hook) frontier
    # compaction threshold tau in thousandths (0 = rewrite every round)
    sweeps = [("edges_per_thread", (4, 8, 16)), ("block", (256, 512, 1024))]
    if best.hook == "plain" or (best.hook == "auto" and m < (1 << 22)):
        sweeps.append(("compact_threshold", (0, 500, 250, 100)))
    # the library's own choice for auto plans: the filter on large lists of
    # average degree >= 8 (entries per vertex)
    filtered = best.filter == "giant" or (best.hook == "auto" and m >= (1 << 22) and m >= 8 * n)
    if filtered:
        sweeps.append(("hot_cache", ("vertex", "large", "off")))
    for field, values in sweeps:
        for val in values:
            c = Options(**{**best.__dict__, field: val})
            t = run(c)
            if t < best_t:
                best_t, best = t, c
    table = sorted(((t, o.__dict__) for t, o in tried.values()), key=lambda x: x[0])
    if cache:
        _store(path or _CACHE_PATH, shape_key(n, m),
               {"options": best.__dict__, "ms": best_t, "n": n, "m": m})
    return best, table


def tune_batch(u, v, vtx_off, edge_off, *, reps: int = 3, log=None):
    """Plan of the batched LDS solver: path halving in the LDS climb (on/off),
    the per-graph segment cap S (each graph gets min(S, round(m_g / n_g))
    segments; 0 = the default, 2 with halving and the paper's round(m_g / n_g)
    without) and the workgroup size (256, 512, 1024: with the LDS of the
    largest graph it sets how many workgroups share a CU).  The LDS solver has
    no frontier compaction, so there is no compaction threshold to choose.
    Returns (best Options, table of (ms, options dict))."""
    import torch
    out = torch.empty(int(vtx_off[-1]), dtype=torch.int32, device=u.device)
    cands = [Options(segments=s) for s in (1, 2, 4, 8)]
    cands += [Options(segments=s, path_halving="off") for s in (0, 4, 8)]
    table = []

    def timed(opt):
        labels_batch(u, v, vtx_off, edge_off, out=out, options=opt)
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            labels_batch(u, v, vtx_off, edge_off, out=out, options=opt)
            best = min(best, time.perf_counter() - t)
        return best * 1e3

    for opt in cands:
        t = timed(opt)
        table.append((t, opt))
        if log:
            log("tune batch halving %s, segment cap %d: %.3f ms"
                % (opt.path_halving, opt.segments, t))
    table.sort(key=lambda x: x[0])
    best = table[0][1]
    for block in (256, 512):
        opt = Options(**{**best.__dict__, "block": block})
        t = timed(opt)
        table.append((t, opt))
        if log:
            log("tune batch halving %s, segment cap %d, block %d: %.3f ms"
                % (opt.path_halving, opt.segments, block, t))
    table.sort(key=lambda x: x[0])
    return table[0][1], [(t, o.__dict__) for t, o in table]

