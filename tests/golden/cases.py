"""Loader for the hand-worked fixtures in hand_cases.txt."""
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def hand_cases():
    """Yield (name, n, u, v, expected_labels) for every fixture row."""
    with open(os.path.join(_HERE, "hand_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, n, edges, labels = [x.strip() for x in line.split(";")]
            n = int(n)
            pairs = [] if edges == "-" else [tuple(map(int, e.split("-"))) for e in edges.split()]
            u = np.array([a for a, _ in pairs], dtype=np.int32)
            v = np.array([b for _, b in pairs], dtype=np.int32)
            want = np.array([int(x) for x in labels.split()], dtype=np.int32)
            assert len(want) == n, name
            yield name, n, u, v, want


# Requests of the server test at the serving workload's sizes: six R-MAT
# requests at scale 19-22 with edge factor 21-32 (the large-request path),
# then 18 more with scale and edge factor drawn from 10-18 and 8-32.  Each is
# graphgen.serving_request(index, scale, ef, seed=SERVING_MIX_SEED).
SERVING_MIX_SEED = 2105
SERVING_MIX_LARGE = ((22, 32), (21, 28), (20, 21), (19, 30), (22, 24), (21, 22))


def serving_mix():
    """[(index, scale, edge_factor)] of the server test's requests."""
    import graphgen
    out = [(i, s, e) for i, (s, e) in enumerate(SERVING_MIX_LARGE)]
    sc, ef = graphgen.serving_request_shapes(18, seed=SERVING_MIX_SEED, scale_lo=10, scale_hi=18)
    for k in range(18):
        out.append((len(SERVING_MIX_LARGE) + k, int(sc[k]), int(ef[k])))
    return out


# The serving benchmark's request pool: graphgen.serving_request_shapes(
# SERVING_POOL_SIZE, seed=SERVING_POOL_SEED) over the full ranges (scale
# 10-22, edge factor 8-32); request i is serving_request(i, scale_i, ef_i,
# seed=SERVING_POOL_SEED).
SERVING_POOL_SEED = 1005
SERVING_POOL_SIZE = 64


def serving_pool():
    """[(index, scale, edge_factor)] of the serving benchmark's pool."""
    import graphgen
    sc, ef = graphgen.serving_request_shapes(SERVING_POOL_SIZE, seed=SERVING_POOL_SEED)
    return [(i, int(sc[i]), int(ef[i])) for i in range(SERVING_POOL_SIZE)]
