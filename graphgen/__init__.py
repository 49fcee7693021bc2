"""Seeded synthetic graph generators for the connected-components workloads.

This module is input plumbing shared by the CPU oracle, the GPU solver, the
tests and the benchmark.  It holds none of the connected-components
arithmetic: it only draws vertex ids.  The heavy loops live in
``graphgen.cpp`` (counter-based SplitMix64 draws, so every slice is
reproducible and thread-count independent); this file composes them into the
five workload families:

* ``er_planted``  Erdos-Renyi pairs plus planted isolated 4-cliques
* ``rmat``        R-MAT (a, b, c, d) pairs, optional id permutation and
                  symmetrisation [E; E^T]
* ``grid``        W x H 4-neighbour lattice with a seeded fraction deleted
* ``batch_er``    many independent ER graphs, log-uniform sizes and degrees,
                  packed back to back with per-graph offsets
* ``serving_pool`` a pool of R-MAT requests of mixed scale / edge factor

Every array is int32 (vertex ids) or int64 (offsets), as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None
_lock = threading.Lock()

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with g++ (host code only)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.gg_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_int64, _u64p]
            lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, _i32p]
            lib.gg_uniform_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                             ctypes.c_uint64, _i32p, _i32p, ctypes.c_int]
            lib.gg_rmat_pairs.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_uint64, _i32p, _i32p, ctypes.c_int]
            lib.gg_apply_map.argtypes = [ctypes.c_int64, _i32p, _i32p, ctypes.c_int]
            lib.gg_grid_edge_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
            lib.gg_grid_edge_count.restype = ctypes.c_int64
            lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_uint64, ctypes.c_uint64, _i32p, _i32p]
            lib.gg_grid.restype = ctypes.c_int64
            lib.gg_batch_uniform_pairs.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_uint64,
                                                   ctypes.c_uint64, _i32p, _i32p, ctypes.c_int]
            _lib = lib
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _p32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_i32p)


def _p64(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_i64p)


# --------------------------------------------------------------------------- raw draws
def draws(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draws(seed, stream, start, count, out.ctypes.data_as(_u64p))
    return out


def uniform01(seed: int, stream: int, count: int) -> np.ndarray:
    """``count`` doubles uniform in [0, 1) (53-bit mantissa of each draw)."""
    return (draws(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def permutation(n: int, seed: int, stream: int = 0) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, stream, _p32(perm))
    return perm


def uniform_pairs(m: int, k: int, seed: int, stream: int):
    u = np.empty(m, dtype=np.int32)
    v = np.empty(m, dtype=np.int32)
    if m:
        _load().gg_uniform_pairs(m, k, seed, stream, _p32(u), _p32(v), _threads())
    return u, v


def _thresholds(a: float, b: float, c: float):
    s = 2.0 ** 32
    tA = min(int(a * s), 2 ** 32 - 1)
    tAB = min(int((a + b) * s), 2 ** 32 - 1)
    tABC = min(int((a + b + c) * s), 2 ** 32 - 1)
    return tA, tAB, tABC


# --------------------------------------------------------------------------- families
def er_planted(n: int = 1 << 16, m_er: int = 1 << 19, cliques: int = 64, clique_size: int = 4,
               seed: int = 1001):
    """Uniform random pairs over the non-clique ids plus planted isolated cliques.

    A seeded permutation of [0, n) is drawn; its first ``cliques*clique_size``
    entries are the clique members (clique c = entries [c*k, (c+1)*k)), the
    rest form the pool that the ``m_er`` uniform pairs (self-loops kept) are
    drawn from.  Clique edges (all k(k-1)/2 pairs, in list order) follow the
    random pairs.  Returns (u, v, n, cliques_ids) with cliques_ids shaped
    (cliques, clique_size).
    """
    planted = cliques * clique_size
    if planted > n:
        raise ValueError("cliques do not fit")
    perm = permutation(n, seed, 0)
    clique_ids = perm[:planted].reshape(cliques, clique_size)
    pool = perm[planted:]
    if m_er and len(pool) == 0:
        raise ValueError("no pool vertices for random pairs")
    iu, iv = uniform_pairs(m_er, max(len(pool), 1), seed, 1)
    er_u = pool[iu] if m_er else np.empty(0, np.int32)
    er_v = pool[iv] if m_er else np.empty(0, np.int32)
    a_idx, b_idx = np.triu_indices(clique_size, k=1)
    cu = clique_ids[:, a_idx].reshape(-1)
    cv = clique_ids[:, b_idx].reshape(-1)
    u = np.ascontiguousarray(np.concatenate([er_u, cu]).astype(np.int32))
    v = np.ascontiguousarray(np.concatenate([er_v, cv]).astype(np.int32))
    return u, v, n, clique_ids


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1002, permute: bool = True, symmetrize: bool = False, m: int | None = None):
    """R-MAT graph on n = 2^scale vertices with m = edge_factor * n pairs.

    With ``permute`` the ids are relabelled by a seeded permutation (stream 0);
    pairs come from stream 1.  With ``symmetrize`` the returned lists are
    [u; v] and [v; u] (2m entries: every pair in both orientations).
    Self-loops and duplicate pairs are kept.  Returns (u, v, n).
    """
    n = 1 << scale
    m_und = edge_factor * n if m is None else m
    tA, tAB, tABC = _thresholds(a, b, c)
    total = 2 * m_und if symmetrize else m_und
    u = np.empty(total, dtype=np.int32)
    v = np.empty(total, dtype=np.int32)
    lib = _load()
    if m_und:
        lib.gg_rmat_pairs(scale, m_und, tA, tAB, tABC, seed, 1, _p32(u), _p32(v), _threads())
    if permute and m_und:
        perm = permutation(n, seed, 0)
        lib.gg_apply_map(m_und, _p32(perm), _p32(u), _threads())
        lib.gg_apply_map(m_und, _p32(perm), _p32(v), _threads())
    if symmetrize and m_und:
        u[m_und:] = v[:m_und]
        v[m_und:] = u[:m_und]
    return u, v, n


def grid_edge_count(W: int, H: int) -> int:
    return int(_load().gg_grid_edge_count(W, H))


def grid(W: int = 4096, H: int = 4096, delete_frac_num: int = 3, delete_frac_den: int = 10,
         seed: int = 1003):
    """W x H 4-neighbour lattice (row-major ids) with floor(E*num/den) edges deleted.

    Returns (u, v, n).
    """
    E = grid_edge_count(W, H)
    ndel = E * delete_frac_num // delete_frac_den
    m = E - ndel
    u = np.empty(m, dtype=np.int32)
    v = np.empty(m, dtype=np.int32)
    got = _load().gg_grid(W, H, ndel, seed, 0, _p32(u), _p32(v))
    assert got == m, (got, m)
    return u, v, W * H


def batch_sizes(num_graphs: int, seed: int, lo_exp: float = 8.0, hi_exp: float = 16.0,
                deg_lo: float = 1.0, deg_hi: float = 16.0):
    """Per-graph vertex and edge counts for ``batch_er``.

    n_g = round(2^(lo + (hi-lo) U)), d_g = deg_lo * (deg_hi/deg_lo)^U' (both
    log-uniform), m_g = round(d_g * n_g / 2) (average degree 2m/n).
    """
    U = uniform01(seed, 0, num_graphs)
    U2 = uniform01(seed, 1, num_graphs)
    nv = np.rint(2.0 ** (lo_exp + (hi_exp - lo_exp) * U)).astype(np.int64)
    deg = deg_lo * (deg_hi / deg_lo) ** U2
    me = np.rint(deg * nv / 2.0).astype(np.int64)
    return nv, me


def batch_er(num_graphs: int = 10000, seed: int = 1004, **size_kw):
    """Independent ER graphs packed back to back (local ids per graph).

    Returns (u, v, vtx_off, edge_off): graph g has vertices
    [vtx_off[g], vtx_off[g+1]) and edge entries [edge_off[g], edge_off[g+1])
    whose endpoints are local ids in [0, n_g).
    """
    nv, me = batch_sizes(num_graphs, seed, **size_kw)
    vtx_off = np.zeros(num_graphs + 1, dtype=np.int64)
    edge_off = np.zeros(num_graphs + 1, dtype=np.int64)
    np.cumsum(nv, out=vtx_off[1:])
    np.cumsum(me, out=edge_off[1:])
    total = int(edge_off[-1])
    u = np.empty(total, dtype=np.int32)
    v = np.empty(total, dtype=np.int32)
    nv32 = np.ascontiguousarray(nv.astype(np.int32))
    _load().gg_batch_uniform_pairs(num_graphs, _p64(edge_off), _p32(nv32), seed, 2, _p32(u),
                                   _p32(v), _threads())
    return u, v, vtx_off, edge_off


def serving_request_shapes(count: int, seed: int, scale_lo: int = 10, scale_hi: int = 22,
                           ef_lo: int = 8, ef_hi: int = 32):
    """(scale, edge_factor) of each request: both uniform integers, inclusive ranges."""
    d = draws(seed, 0, count)
    scales = scale_lo + ((d >> np.uint64(32)) * np.uint64(scale_hi - scale_lo + 1)
                         >> np.uint64(32)).astype(np.int64)
    lo32 = d & np.uint64(0xFFFFFFFF)
    efs = ef_lo + ((lo32 * np.uint64(ef_hi - ef_lo + 1)) >> np.uint64(32)).astype(np.int64)
    return scales, efs


def serving_request(index: int, scale: int, edge_factor: int, seed: int = 1005,
                    a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """Request ``index`` of the serving stream: a permuted, unsymmetrised R-MAT graph."""
    sub_seed = int(draws(seed, 1, 1, start=index)[0])
    return rmat(scale, edge_factor, a, b, c, seed=sub_seed, permute=True, symmetrize=False)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson process of the given rate."""
    U = uniform01(seed, 2, count)
    gaps = -np.log1p(-U) / rate
    return np.cumsum(gaps)


# --------------------------------------------------------------------------- named workloads
def workload(name: str, seed: int | None = None):
    """The named workloads (sizes as in the design doc's input recipe).

    'er16'   : n=2^16, 2^19 uniform pairs + 64 planted 4-cliques (m=524,672)
    'rmat24' : R-MAT scale 24, edge factor 16, permuted, symmetrised (m=2^29)
    'grid4k' : 4096^2 lattice, 30% of edges deleted (m=23,482,368)
    Returns (u, v, n).
    """
    if name == "er16":
        u, v, n, _ = er_planted(seed=1001 if seed is None else seed)
        return u, v, n
    if name == "rmat24":
        return rmat(24, 16, seed=1002 if seed is None else seed, permute=True, symmetrize=True)
    if name == "grid4k":
        return grid(4096, 4096, seed=1003 if seed is None else seed)
    raise KeyError(name)
