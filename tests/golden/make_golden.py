"""Writes oracle_digests.json: the CPU oracle's labels of the full-size
workloads, as a SHA-256 of the int32 label array plus the component count.

Calls only graphgen (seeded inputs) and oracle/ (the CPU union-find); no
value comes from the GPU library.  The GPU tests compare the digest of the
GPU labels with these, which checks every one of the up to 2^24 labels of
the large workloads bit for bit without rerunning the oracle on the GPU machine.

    python tests/golden/make_golden.py [name ...]
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


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_about"] = ("SHA-256 of the CPU oracle's int32 labels (little-endian) for the named "
                      "seeded workloads; written by tests/golden/make_golden.py")
    for name in names:
        data[name] = entry(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["er16", "grid4k", "batch10k", "rmat24"])
