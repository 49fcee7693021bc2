"""CPU oracle for connected-component labels -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library (``paper_1612_01178_amd``)
never imports, links or calls it, and the two share no code: the only thing
both sides consume is the seeded input from ``graphgen``.

What the oracle computes (Section 2 of the paper, definition of connected
components, with the smallest vertex id of each component as its
representative -- the root that the high-to-low hooking rule of Figs. 2-3
produces):

    label[v] = min { w : w is joined to v by a path of undirected edges }

``cc_oracle.c`` computes it with a sequential union-find (link the larger
root under the smaller, path halving) and one resolving pass in increasing
id order.  It is pinned, independently of itself, by the ``-m "not gpu"``
tests: brute-force transitive closure on every graph with at most 5 vertices
and on random graphs up to 64 vertices, a breadth-first traversal labeller
(the sequential traversal solution of Section 2), scipy's
``connected_components``, closed forms and output invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libccoracle.so")
_lib = None
_lock = threading.Lock()

OK = 0
ERR_ARG = -1
ERR_RANGE = -2
ERR_NOMEM = -3

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False, src: str | None = None, out: str | None = None) -> str:
    """Compile the oracle with gcc (plain C, -O2).  ``src``/``out`` let a test
    build a deliberately altered copy of the source elsewhere."""
    src = src or _SRC
    out = out or _LIB_PATH
    if force or src != _SRC or not os.path.exists(out) or (
            os.path.getmtime(out) < os.path.getmtime(src)):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, out)
    return out


def _bind(lib):
    lib.cc_oracle_labels.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int64, _i32p]
    lib.cc_oracle_labels.restype = ctypes.c_int32
    lib.cc_oracle_labels_batch.argtypes = [ctypes.c_int32, _i64p, _i64p, _i32p, _i32p, _i32p]
    lib.cc_oracle_labels_batch.restype = ctypes.c_int32
    return lib


def load(path: str | None = None):
    """The oracle library (built on first use); ``path`` loads another build."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _arr32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def labels(u, v, n: int, lib=None) -> np.ndarray:
    """Min-id component labels of the undirected graph with edge entries (u[i], v[i]).

    Raises ValueError on a bad argument or an endpoint outside [0, n).
    """
    lib = lib or load()
    u = _arr32(u)
    v = _arr32(v)
    if u.shape != v.shape or u.ndim != 1:
        raise ValueError("u and v must be 1-D arrays of equal length")
    out = np.empty(max(n, 0), dtype=np.int32)
    rc = lib.cc_oracle_labels(int(n), u.ctypes.data_as(_i32p), v.ctypes.data_as(_i32p),
                              int(u.shape[0]), out.ctypes.data_as(_i32p))
    if rc == ERR_RANGE:
        raise ValueError("endpoint outside [0, n)")
    if rc != OK:
        raise ValueError("oracle status %d" % rc)
    return out


def labels_batch(u, v, vtx_off, edge_off, lib=None) -> np.ndarray:
    """Per-graph local min-id labels of graphs packed back to back."""
    lib = lib or load()
    u = _arr32(u)
    v = _arr32(v)
    vtx_off = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    edge_off = np.ascontiguousarray(np.asarray(edge_off, dtype=np.int64))
    B = len(vtx_off) - 1
    out = np.empty(int(vtx_off[-1]) if B >= 0 else 0, dtype=np.int32)
    rc = lib.cc_oracle_labels_batch(B, vtx_off.ctypes.data_as(_i64p),
                                    edge_off.ctypes.data_as(_i64p), u.ctypes.data_as(_i32p),
                                    v.ctypes.data_as(_i32p), out.ctypes.data_as(_i32p))
    if rc == ERR_RANGE:
        raise ValueError("endpoint outside [0, n_g)")
    if rc != OK:
        raise ValueError("oracle status %d" % rc)
    return out
