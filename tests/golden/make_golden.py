"""Writes oracle_digests.json: the CPU oracle's labels of the full-size
workloads, as a SHA-256 of the int32 label array plus the component count.

Calls only graphgen (seeded inputs) and oracle/ (the CPU union-find); no
value comes from the GPU library.  The GPU tests compare the digest of the
GPU labels with these, which checks every one of the up to 2^24 labels of
the large workloads bit for bit without rerunning the oracle on the GPU machine.

    python tests/golden/make_golden.py [name ...]
    python tests/golden/make_golden.py serving [mix] [pool]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "oracle_digests.json")


def digest(labels: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()


def entry(name):
    t = time.time()
    if name == "batch10k":
        u, v, vo, eo = graphgen.batch_er(10000, seed=1004)
        lab = oracle.labels_batch(u, v, vo, eo)
        comps = int(np.count_nonzero(lab == (np.arange(len(lab)) - np.repeat(vo[:-1], np.diff(vo)))))
        n, m = int(vo[-1]), int(eo[-1])
    else:
        u, v, n = graphgen.workload(name)
        lab = oracle.labels(u, v, n)
        comps = int(np.count_nonzero(lab == np.arange(n)))
        m = len(u)
    rec = {"n": n, "m": m, "components": comps, "sha256": digest(lab),
           "oracle_seconds": round(time.time() - t, 1)}
    print(name, rec, flush=True)
    return rec


SERVING_OUT = os.path.join(HERE, "serving_digests.json")


def serving_entries(kind):
    """Digests of the oracle's labels for every request of the server test's
    mix ('mix') or of the serving benchmark's pool ('pool')."""
    from tests.golden import cases
    spec, seed = ((cases.serving_mix(), cases.SERVING_MIX_SEED) if kind == "mix"
                  else (cases.serving_pool(), cases.SERVING_POOL_SEED))
    t = time.time()
    reqs = []
    for i, sc, ef in spec:
        u, v, n = graphgen.serving_request(i, sc, ef, seed=seed)
        lab = oracle.labels(u, v, n)
        reqs.append({"index": i, "scale": sc, "edge_factor": ef, "n": n, "m": len(u),
                     "components": int(np.count_nonzero(lab == np.arange(n))),
                     "sha256": digest(lab)})
    rec = {"seed": seed, "requests": reqs, "m_total": sum(r["m"] for r in reqs),
           "oracle_seconds": round(time.time() - t, 1)}
    print(kind, len(reqs), "requests,", rec["m_total"], "entries,", rec["oracle_seconds"], "s",
          flush=True)
    return rec


def main_serving(kinds):
    data = json.load(open(SERVING_OUT)) if os.path.exists(SERVING_OUT) else {}
    data["_about"] = ("SHA-256 of the CPU oracle's int32 labels (little-endian) of every request "
                      "of the server test ('mix') and of the serving benchmark's pool ('pool'); "
                      "written by tests/golden/make_golden.py serving")
    for k in kinds:
        data[k] = serving_entries(k)
        with open(SERVING_OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("SHA-256 of the CPU oracle's int32 labels (little-endian) for the named "
                      "seeded workloads; written by tests/golden/make_golden.py")
    for name in names:
        data[name] = entry(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["serving"]:
        main_serving(sys.argv[2:] or ["mix", "pool"])
    else:
        main(sys.argv[1:] or ["er16", "grid4k", "batch10k", "rmat24"])
