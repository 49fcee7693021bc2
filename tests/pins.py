"""Independent checks that pin the CPU oracle (and, through it, the GPU path).

None of these shares code with ``oracle/`` or with the GPU library:

* ``closure_labels``   brute-force transitive closure (Warshall) of the
                       adjacency relation, then the minimum of each row --
                       the definition of a min-id component label written out
                       literally (Section 2).  O(n^3): tiny graphs only.
* ``traversal_labels`` the sequential graph-traversal labelling that Section 2
                       describes: scan vertices in increasing id order and
                       flood every unlabelled vertex's component with its id
                       by breadth-first search.  Pure Python: small graphs.
* ``scipy_labels``     scipy.sparse.csgraph.connected_components (a library
                       routine), relabelled to each component's minimum id.
* ``check_invariants`` properties every correct output has.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def closure_labels(u, v, n: int) -> np.ndarray:
    if n == 0:
        return np.zeros(0, dtype=np.int32)
    reach = np.eye(n, dtype=bool)
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        reach[a, b] = True
        reach[b, a] = True
    for k in range(n):
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    # row-wise smallest reachable id
    return np.argmax(reach, axis=1).astype(np.int32)


def traversal_labels(u, v, n: int) -> np.ndarray:
    adj = [[] for _ in range(n)]
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        adj[a].append(b)
        adj[b].append(a)
    label = [-1] * n
    for s in range(n):
        if label[s] != -1:
            continue
        label[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if label[y] == -1:
                    label[y] = s
                    q.append(y)
    return np.asarray(label, dtype=np.int32)


def scipy_labels(u, v, n: int) -> np.ndarray:
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    g = coo_matrix((np.ones(len(u), dtype=np.int8), (u, v)), shape=(n, n)).tocsr()
    ncomp, comp = connected_components(g, directed=False)
    rep = np.full(ncomp, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(rep, comp, np.arange(n, dtype=np.int64))
    return rep[comp].astype(np.int32)


def check_invariants(u, v, n: int, label: np.ndarray) -> None:
    """Raise AssertionError unless ``label`` is a valid min-id labelling shape-wise:
    both ends of every edge agree, label[v] <= v, labels are fixed points."""
    label = np.asarray(label)
    assert label.shape == (n,)
    if n == 0:
        return
    assert label.min() >= 0 and label.max() < n
    ids = np.arange(n)
    assert np.all(label <= ids), "a label exceeds its vertex id"
    assert np.array_equal(label[label], label), "a label is not its own label"
    u = np.asarray(u)
    v = np.asarray(v)
    if len(u):
        assert np.array_equal(label[u], label[v]), "an edge joins two labels"


def component_count(label: np.ndarray) -> int:
    label = np.asarray(label)
    return int(np.count_nonzero(label == np.arange(len(label))))
