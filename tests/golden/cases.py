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
