"""Adaptive, work-efficient Hook-Compress connected components on MI355X.

Thin Python binding of ``libhookcc.so`` (C ABI in ``include/hookcc.h``):
argument marshalling only.  Every step of a solve runs in the library's HIP
kernels; PyTorch only provides device memory and streams.  There is no CPU
fallback: if the library has not been built, every call raises.

    import paper_1612_01178_amd as cc
    lab = cc.labels(u, v, n)                       # u, v: int32 CUDA tensors
    lab = cc.labels(u, v, n, options=cc.Options(hook="plain"))
    lab = cc.labels_batch(u, v, vtx_off, edge_off) # host int64 offsets

Labels are exact: label[x] is the smallest vertex id of x's component.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhookcc.so")

CC_OK = 0
CC_ERR_ARG = -1
CC_ERR_RANGE = -2
CC_ERR_NOMEM = -3
CC_ERR_HIP = -4
CC_ERR_NOCONVERGE = -5
CC_BATCH_LDS_MAX_N = 65536
CC_NOALLOC_SCRATCH_BYTES = 32 << 20

_HOOKS = {"auto": 0, "atomic": 1, "plain": 2, "hybrid": 3}
_FILTERS = {"off": 0, "giant": 1, "auto": 2}
_HOST_LOOPS = {"off": 0, "jump": 1, "multijump": 2}

# Every symbol include/hookcc.h declares.
EXPORTS = ("cc_options_init", "cc_labels", "cc_labels_ex", "cc_workspace_bytes", "cc_labels_noalloc",
           "cc_labels_batch", "cc_labels_batch_ex", "cc_labels_batch_device", "cc_labels_list", "cc_labels_host", "cc_labels_csr", "cc_probe",
           "cc_last_error", "cc_release", "cc_version", "cc_stream_status", "cc_server_create",
           "cc_server_submit", "cc_server_submit_on", "cc_server_wait", "cc_server_poll", "cc_server_stats",
           "cc_server_destroy", "cc_server_clock")
CC_REQ_HOST_EDGES = 1
CC_REQ_HOST_LABELS = 2


class CCError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("hookcc status %d: %s" % (code, message))
        self.code = code


class _COptions(ctypes.Structure):
    _fields_ = [("hook", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("filter_after", ctypes.c_int32),
                ("block", ctypes.c_int32), ("edges_per_thread", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("rounds_per_check", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("host_loop", ctypes.c_int32),
                ("coherent_loads", ctypes.c_int32), ("hot_cache", ctypes.c_int32),
                ("path_halving", ctypes.c_int32), ("symmetric", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("no_sync", ctypes.c_int32),
                ("compact_threshold", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class _CStats(ctypes.Structure):
    _fields_ = [("hook", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("filter_used", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("active_edges", ctypes.c_int64), ("giant_label", ctypes.c_int32),
                ("host_syncs", ctypes.c_int32), ("hook_launches", ctypes.c_int32),
                ("compress_launches", ctypes.c_int32), ("hook_ms", ctypes.c_float),
                ("compress_ms", ctypes.c_float), ("other_ms", ctypes.c_float),
                ("reserved", ctypes.c_int64 * 4)]


class _CGraph(ctypes.Structure):
    _fields_ = [("edges_u", ctypes.c_void_p), ("edges_v", ctypes.c_void_p),
                ("out_label", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _CServerConfig(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_int64), ("workers", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_batch_edges", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 8)]


class _CRequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_device_done", ctypes.c_double),
                ("t_host_done", ctypes.c_double)]


@dataclasses.dataclass
class Options:
    """Solver options (0 / "auto" = library default).  See cc_options in hookcc.h."""
    hook: str = "auto"
    segments: int = 0
    filter: str = "auto"
    filter_after: int = 0
    block: int = 0
    edges_per_thread: int = 0
    max_rounds: int = 0
    rounds_per_check: int = 0
    profile: bool = False
    host_loop: str = "off"
    coherent_loads: bool = False
    hot_cache: str = "auto"
    path_halving: str = "auto"
    symmetric: bool = False
    graph: bool = False
    no_sync: bool = False
    compact_threshold: int = 0

    def _c(self) -> _COptions:
        o = _COptions()
        o.hook = _HOOKS[self.hook]
        o.segments = self.segments
        o.filter = _FILTERS[self.filter]
        o.filter_after = self.filter_after
        o.block = self.block
        o.edges_per_thread = self.edges_per_thread
        o.max_rounds = self.max_rounds
        o.rounds_per_check = self.rounds_per_check
        o.profile = 1 if self.profile else 0
        o.host_loop = _HOST_LOOPS[self.host_loop]
        o.coherent_loads = 1 if self.coherent_loads else 0
        o.hot_cache = {"auto": 0, "on": 1, "off": 2, "large": 3, "vertex": 4}[self.hot_cache]
        o.path_halving = {"auto": 0, "on": 1, "off": 2}[self.path_halving]
        o.symmetric = 1 if self.symmetric else 0
        o.graph = 1 if self.graph else 0
        o.no_sync = 1 if self.no_sync else 0
        o.compact_threshold = self.compact_threshold
        return o


_lib = None
_lock = threading.Lock()
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def load():
    """The loaded libhookcc.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libhookcc.so is not built (run __graft_entry__.build() or "
                                   "python paper_1612_01178_amd/build.py); there is no fallback")
            lib = ctypes.CDLL(LIB_PATH)
            lib.cc_options_init.argtypes = [ctypes.POINTER(_COptions)]
            lib.cc_options_init.restype = None
            lib.cc_labels.argtypes = [_i32, _vp, _vp, _i64, _vp]
            lib.cc_labels.restype = _i32
            lib.cc_labels_ex.argtypes = [_i32, _vp, _vp, _i64, _vp, ctypes.POINTER(_COptions),
                                         _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_CStats)]
            lib.cc_labels_ex.restype = _i32
            lib.cc_labels_noalloc.argtypes = [_i32, _vp, _vp, _i64, _vp, ctypes.POINTER(_COptions),
                                              _vp, ctypes.POINTER(_CStats)]
            lib.cc_labels_noalloc.restype = _i32
            lib.cc_workspace_bytes.argtypes = [_i32, _i64, ctypes.POINTER(_COptions)]
            lib.cc_workspace_bytes.restype = ctypes.c_size_t
            lib.cc_labels_batch.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp]
            lib.cc_labels_batch.restype = _i32
            lib.cc_labels_batch_ex.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp,
                                               ctypes.POINTER(_COptions), _vp,
                                               ctypes.POINTER(_CStats)]
            lib.cc_labels_batch_ex.restype = _i32
            lib.cc_labels_batch_device.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32,
                                                   ctypes.POINTER(_COptions), _vp,
                                                   ctypes.POINTER(_CStats)]
            lib.cc_labels_batch_device.restype = _i32
            lib.cc_labels_list.argtypes = [_i32, ctypes.POINTER(_CGraph), ctypes.POINTER(_COptions),
                                           _vp, ctypes.POINTER(_CStats)]
            lib.cc_labels_list.restype = _i32
            lib.cc_server_create.argtypes = [ctypes.POINTER(_CServerConfig),
                                             ctypes.POINTER(ctypes.c_void_p)]
            lib.cc_server_create.restype = _i32
            lib.cc_server_submit.argtypes = [_vp, _i32, _vp, _vp, _i64, _vp, _i32,
                                             ctypes.POINTER(_i64)]
            lib.cc_server_submit.restype = _i32
            lib.cc_server_submit_on.argtypes = [_vp, _i32, _vp, _vp, _i64, _vp, _i32, _vp,
                                                ctypes.POINTER(_i64)]
            lib.cc_server_submit_on.restype = _i32
            lib.cc_server_wait.argtypes = [_vp, _i64, ctypes.POINTER(_CRequestInfo)]
            lib.cc_server_wait.restype = _i32
            lib.cc_server_poll.argtypes = [_vp, _i64, ctypes.POINTER(_CRequestInfo)]
            lib.cc_server_poll.restype = _i32
            lib.cc_server_stats.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
            lib.cc_server_stats.restype = _i32
            lib.cc_server_destroy.argtypes = [_vp]
            lib.cc_server_destroy.restype = _i32
            lib.cc_server_clock.argtypes = []
            lib.cc_server_clock.restype = ctypes.c_double
            lib.cc_labels_host.argtypes = [_i32, _vp, _vp, _i64, _vp, _i64,
                                           ctypes.POINTER(_COptions), _vp, ctypes.POINTER(_CStats)]
            lib.cc_labels_host.restype = _i32
            lib.cc_labels_csr.argtypes = [_i32, _vp, _vp, _i64, _vp, ctypes.POINTER(_COptions),
                                          _vp, ctypes.POINTER(_CStats)]
            lib.cc_labels_csr.restype = _i32
            lib.cc_probe.argtypes = [_i32, _vp, _vp, _i64, _vp, _i32, _vp]
            lib.cc_probe.restype = _i32
            lib.cc_last_error.argtypes = []
            lib.cc_last_error.restype = ctypes.c_char_p
            lib.cc_release.argtypes = []
            lib.cc_release.restype = None
            lib.cc_stream_status.argtypes = [_vp]
            lib.cc_stream_status.restype = _i32
            lib.cc_version.argtypes = []
            lib.cc_version.restype = ctypes.c_char_p
            _lib = lib
    return _lib


def last_error() -> str:
    return load().cc_last_error().decode()


def version() -> str:
    return load().cc_version().decode()


def release() -> None:
    load().cc_release()


CC_PENDING = 1


def stream_status(stream=None) -> int:
    """Status of the last ``no_sync`` call on ``stream`` (default: the current
    torch stream): CC_PENDING while its work runs, then 0; raises CCError for
    a device-detected error (CC_ERR_RANGE) or when no such call was made."""
    rc = int(load().cc_stream_status(_stream_handle(stream)))
    if rc == CC_PENDING:
        return rc
    _check(rc)
    return rc


_c_options_cache = {}


def _c_options(options):
    """The C struct of `options` (None = defaults), built once per distinct
    set of field values: the library takes it as const, so calls share it."""
    opts = options if options is not None else Options()
    key = tuple(vars(opts).values())
    c = _c_options_cache.get(key)
    if c is None:
        if len(_c_options_cache) >= 64:
            _c_options_cache.clear()
        c = _c_options_cache[key] = opts._c()
    return c


def _on_device(dev):
    """torch.cuda.device(dev), or nothing when dev is already current (the
    context manager costs several microseconds per call)."""
    import contextlib
    import torch
    dev = torch.device(dev)
    if dev.index is None or dev.index == torch.cuda.current_device():
        return contextlib.nullcontext()
    return torch.cuda.device(dev)


def _check(rc: int) -> None:
    if rc != CC_OK:
        raise CCError(rc, last_error())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _edge_tensor(x, name):
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != torch.int32 or x.device.type != "cuda":
        raise TypeError("%s must be an int32 CUDA tensor" % name)
    if x.dim() != 1 or not x.is_contiguous():
        raise ValueError("%s must be 1-D and contiguous" % name)
    return x


def labels(u, v, n: int, *, out=None, options: Options | None = None, stream=None,
           workspace=None, return_stats: bool = False):
    """Min-id component labels (int32 CUDA tensor of length n) of the graph
    with edge entries (u[i], v[i]).  Synchronous on ``stream`` (default: the
    current torch stream)."""
    import torch
    u = _edge_tensor(u, "u")
    v = _edge_tensor(v, "v")
    if u.numel() != v.numel():
        raise ValueError("u and v differ in length")
    if out is None:
        out = torch.empty(max(int(n), 0), dtype=torch.int32, device=u.device)
    else:
        out = _edge_tensor(out, "out")
        if out.numel() < n:
            raise ValueError("out is shorter than n")
    opts = _c_options(options)
    st = _CStats()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    with _on_device(u.device):
        rc = load().cc_labels_ex(int(n), u.data_ptr(), v.data_ptr(), u.numel(), out.data_ptr(),
                                 ctypes.byref(opts), ws_ptr, ws_bytes, _stream_handle(stream),
                                 ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_noalloc(u, v, n: int, *, out, options: Options | None = None, stream=None,
                   return_stats: bool = False):
    """cc_labels_noalloc: as ``labels`` with the workspace in the library's
    fixed device array, so the call allocates nothing; ``out`` (int32 CUDA
    tensor of at least n entries) must be given."""
    u = _edge_tensor(u, "u")
    v = _edge_tensor(v, "v")
    out = _edge_tensor(out, "out")
    if u.numel() != v.numel():
        raise ValueError("u and v differ in length")
    if out.numel() < n:
        raise ValueError("out is shorter than n")
    opts = _c_options(options)
    st = _CStats()
    import torch
    with _on_device(u.device):
        rc = load().cc_labels_noalloc(int(n), u.data_ptr(), v.data_ptr(), u.numel(),
                                      out.data_ptr(), ctypes.byref(opts), _stream_handle(stream),
                                      ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_raw(n: int, u_ptr: int, v_ptr: int, m: int, out_ptr: int) -> int:
    """cc_labels on raw device pointers (null stream); returns the status."""
    return int(load().cc_labels(int(n), u_ptr, v_ptr, int(m), out_ptr))


def workspace_bytes(n: int, m: int, options: Options | None = None) -> int:
    opts = _c_options(options)
    return int(load().cc_workspace_bytes(int(n), int(m), ctypes.byref(opts)))


def labels_batch(u, v, vtx_off, edge_off, *, out=None, options: Options | None = None,
                 stream=None, return_stats: bool = False):
    """Per-graph local min-id labels of graphs packed back to back.

    ``u``/``v`` are int32 CUDA tensors of local ids; ``vtx_off``/``edge_off``
    are host int64 arrays of length B+1.  Returns an int32 CUDA tensor of
    length vtx_off[-1]."""
    import numpy as np
    import torch
    u = _edge_tensor(u, "u")
    v = _edge_tensor(v, "v")
    vo = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    eo = np.ascontiguousarray(np.asarray(edge_off, dtype=np.int64))
    if vo.ndim != 1 or eo.shape != vo.shape or len(vo) < 1:
        raise ValueError("vtx_off and edge_off must be 1-D of equal length B+1")
    if eo[-1] != u.numel() or u.numel() != v.numel():
        raise ValueError("edge_off[-1] must equal len(u) == len(v)")
    total = int(vo[-1])
    if out is None:
        out = torch.empty(total, dtype=torch.int32, device=u.device)
    st = _CStats()
    with _on_device(u.device):
        opts = _c_options(options)
        rc = load().cc_labels_batch_ex(len(vo) - 1, vo.ctypes.data, eo.ctypes.data, u.data_ptr(),
                                       v.data_ptr(), out.data_ptr(), ctypes.byref(opts),
                                       _stream_handle(stream), ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_batch_device(u, v, vtx_off, edge_off, max_n: int, out, *,
                        options: Options | None = None, stream=None,
                        return_stats: bool = False):
    """labels_batch with the offsets in device memory (int64 CUDA tensors of
    length B+1): the graphs are checked, ordered and described on the device,
    so a call does no host work per graph.  ``max_n`` bounds every graph's
    vertex count (at most CC_BATCH_LDS_MAX_N); ``out`` is the int32 CUDA
    tensor of vtx_off[-1] labels (its length is not checked: reading it
    would need a synchronisation)."""
    import torch
    u = _edge_tensor(u, "u")
    v = _edge_tensor(v, "v")
    for name, t in (("vtx_off", vtx_off), ("edge_off", edge_off)):
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or t.device != u.device
                or t.dim() != 1 or not t.is_contiguous()):
            raise TypeError("%s must be a contiguous 1-D int64 tensor on the edges' device" % name)
    if vtx_off.numel() != edge_off.numel() or vtx_off.numel() < 1:
        raise ValueError("vtx_off and edge_off must be of equal length B+1")
    if u.numel() != v.numel():
        raise ValueError("len(u) must equal len(v)")
    out = _edge_tensor(out, "out")
    st = _CStats()
    with _on_device(u.device):
        rc = load().cc_labels_batch_device(vtx_off.numel() - 1, vtx_off.data_ptr(),
                                           edge_off.data_ptr(), u.data_ptr(), v.data_ptr(),
                                           out.data_ptr(), int(max_n),
                                           ctypes.byref(_c_options(options)),
                                           _stream_handle(stream), ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_host(u, v, n: int, *, chunk: int = 0, out=None, device=None,
                options: Options | None = None, stream=None, return_stats: bool = False):
    """Labels of a graph whose edge lists stay in host memory (numpy int32 or
    CPU torch tensors; pinned memory lets copies overlap the hooks), streamed
    to the device in chunks of ``chunk`` entries.  Returns a CUDA tensor."""
    import numpy as np
    import torch
    if isinstance(u, torch.Tensor):
        if u.dtype != torch.int32 or u.device.type != "cpu" or not u.is_contiguous():
            raise TypeError("u must be a contiguous int32 CPU tensor")
        up, vp, m = u.data_ptr(), v.data_ptr(), u.numel()
    else:
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        up, vp, m = u.ctypes.data, v.ctypes.data, len(u)
    if len(v) != m:
        raise ValueError("u and v differ in length")
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(max(int(n), 0), dtype=torch.int32, device=dev)
    opts = _c_options(options)
    st = _CStats()
    with _on_device(out.device):
        rc = load().cc_labels_host(int(n), up if m else None, vp if m else None, m,
                                   out.data_ptr() if n else None, int(chunk), ctypes.byref(opts),
                                   _stream_handle(stream), ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_csr(row_ptr, col, n: int, *, out=None, options: Options | None = None, stream=None,
               return_stats: bool = False):
    """Labels of a graph given as a CSR adjacency: ``row_ptr`` int64 CUDA
    tensor of n+1 offsets, ``col`` int32 CUDA tensor of m column ids."""
    import torch
    col = _edge_tensor(col, "col")
    if not isinstance(row_ptr, torch.Tensor) or row_ptr.dtype != torch.int64 or \
            row_ptr.device.type != "cuda" or not row_ptr.is_contiguous() or row_ptr.numel() != n + 1:
        raise TypeError("row_ptr must be a contiguous int64 CUDA tensor of length n + 1")
    if out is None:
        out = torch.empty(max(int(n), 0), dtype=torch.int32, device=col.device)
    opts = _c_options(options)
    st = _CStats()
    with _on_device(col.device):
        rc = load().cc_labels_csr(int(n), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                                  col.numel(), out.data_ptr() if n else None, ctypes.byref(opts),
                                  _stream_handle(stream), ctypes.byref(st))
    _check(rc)
    if return_stats:
        return out, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return out


def labels_list(graphs, *, options: Options | None = None, stream=None,
                return_stats: bool = False):
    """Labels of independent graphs, each given as (u, v, n) or (u, v, n, out)
    with its own int32 CUDA tensors.  Returns the list of label tensors."""
    import torch
    descs = (_CGraph * max(len(graphs), 1))()
    outs = []
    dev = None
    for i, g in enumerate(graphs):
        u, v, n = g[0], g[1], int(g[2])
        u = _edge_tensor(u, "u")
        v = _edge_tensor(v, "v")
        if u.numel() != v.numel():
            raise ValueError("u and v differ in length")
        out = g[3] if len(g) > 3 else torch.empty(max(n, 0), dtype=torch.int32, device=u.device)
        outs.append(out)
        dev = u.device
        descs[i].edges_u = u.data_ptr() if u.numel() else None
        descs[i].edges_v = v.data_ptr() if v.numel() else None
        descs[i].out_label = out.data_ptr() if n > 0 else None
        descs[i].m = u.numel()
        descs[i].n = n
        descs[i].reserved = 0
    st = _CStats()
    if dev is None:
        return ([], {}) if return_stats else []
    with _on_device(dev):
        opts = _c_options(options)
        rc = load().cc_labels_list(len(graphs), descs, ctypes.byref(opts), _stream_handle(stream),
                                   ctypes.byref(st))
    _check(rc)
    if return_stats:
        return outs, {f: getattr(st, f) for f, _ in _CStats._fields_ if f != "reserved"}
    return outs


def probe(mode: int, u, v, table=None, n: int = 0, stream=None) -> None:
    """Asynchronous memory-ceiling probe (see cc_probe in hookcc.h)."""
    u = _edge_tensor(u, "u")
    v = _edge_tensor(v, "v")
    tp = table.data_ptr() if table is not None else None
    _check(load().cc_probe(int(mode), u.data_ptr(), v.data_ptr(), u.numel(), tp, int(n),
                           _stream_handle(stream)))


class Server:
    """Continuous-batching request server (cc_server_* in hookcc.h).

    ``submit`` takes either int32 CUDA tensors (device-resident request) or
    numpy int32 arrays (host request: edges copied in at admission, labels
    copied back).  The arrays are kept alive here until ``wait``."""

    def __init__(self, device_bytes: int = 0, workers: int = 0, max_batch: int = 0,
                 max_batch_edges: int = 0):
        cfg = _CServerConfig()
        cfg.device_bytes = device_bytes
        cfg.workers = workers
        cfg.max_batch = max_batch
        cfg.max_batch_edges = max_batch_edges
        h = ctypes.c_void_p()
        _check(load().cc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @staticmethod
    def clock() -> float:
        return float(load().cc_server_clock())

    def submit(self, u, v, n: int, out=None, stream=None) -> int:
        """Queues one request.  Device tensors are read and written on a worker
        stream after the work queued so far on ``stream`` (default: the current
        torch stream), which may still be producing them."""
        import numpy as np
        import torch
        ready = None
        if isinstance(u, torch.Tensor):
            u = _edge_tensor(u, "u")
            v = _edge_tensor(v, "v")
            if out is None:
                out = torch.empty(max(int(n), 0), dtype=torch.int32, device=u.device)
            flags = 0
            up, vp, op = u.data_ptr(), v.data_ptr(), out.data_ptr()
            ready = _stream_handle(stream)
        else:
            u = np.ascontiguousarray(u, dtype=np.int32)
            v = np.ascontiguousarray(v, dtype=np.int32)
            if out is None:
                out = np.empty(max(int(n), 0), dtype=np.int32)
            flags = CC_REQ_HOST_EDGES | CC_REQ_HOST_LABELS
            up, vp, op = u.ctypes.data, v.ctypes.data, out.ctypes.data
        if len(u) != len(v):
            raise ValueError("u and v differ in length")
        t = ctypes.c_int64()
        _check(load().cc_server_submit_on(self._h, int(n), up if len(u) else None,
                                          vp if len(v) else None, len(u), op if n else None,
                                          flags, ready, ctypes.byref(t)))
        self._keep[t.value] = (u, v, out)
        return t.value

    def _info(self, info):
        return {f: getattr(info, f) for f, _ in _CRequestInfo._fields_}

    def wait(self, ticket: int):
        """(labels, info dict) of a finished request; raises CCError on failure."""
        info = _CRequestInfo()
        rc = load().cc_server_wait(self._h, ticket, ctypes.byref(info))
        keep = self._keep.pop(ticket)
        _check(rc)
        return keep[2], self._info(info)

    def poll(self, ticket: int):
        """None while queued or running, else as ``wait``."""
        info = _CRequestInfo()
        rc = load().cc_server_poll(self._h, ticket, ctypes.byref(info))
        if rc == 1:
            return None
        keep = self._keep.pop(ticket)
        _check(rc)
        return keep[2], self._info(info)

    def stats(self):
        p, a = ctypes.c_int64(), ctypes.c_int64()
        _check(load().cc_server_stats(self._h, ctypes.byref(p), ctypes.byref(a)))
        return {"pending": p.value, "arena_used": a.value}

    def close(self) -> None:
        if self._h:
            rc = load().cc_server_destroy(self._h)
            self._h = None
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
