"""cc_labels_noalloc (the entry point that allocates nothing: its workspace
is the library's fixed device array) against cc_labels_ex on the same
inputs, through the C ABI.  Labels are integers with one correct answer, so
every comparison is bit-exact.  Each test makes two calls in a row, the
second on a smaller input, so the second call runs on the array the first
one left behind."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
import paper_1612_01178_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(u, v):
    d = torch.device("cuda:0")
    return torch.from_numpy(u).to(d), torch.from_numpy(v).to(d)


def _noalloc_raw(du, dv, n, out, opts=None, stream=None):
    """cc_labels_noalloc called through ctypes with raw pointers."""
    lib = cc.load()
    o = (opts or cc.Options())._c()
    st = cc._CStats()
    s = ctypes.c_void_p(int(stream.cuda_stream)) if stream is not None else None
    rc = lib.cc_labels_noalloc(int(n), du.data_ptr(), dv.data_ptr(), du.numel(), out.data_ptr(),
                               ctypes.byref(o), s, ctypes.byref(st))
    return int(rc), st


def _pair(u, v, n, opts=None, stream=None, want=None):
    du, dv = _dev(u, v)
    ref = cc.labels(du, dv, n, options=opts, stream=stream)
    out = torch.full((n,), -7, dtype=torch.int32, device=du.device)
    torch.cuda.synchronize()
    rc, st = _noalloc_raw(du, dv, n, out, opts, stream)
    assert rc == cc.CC_OK, cc.last_error()
    got = out.cpu().numpy()
    assert np.array_equal(got, ref.cpu().numpy())
    if want is not None:
        assert np.array_equal(got, want)
    return st


def test_noalloc_filtered_then_smaller():
    # R-MAT scale 19 symmetrised (2^23 entries: the filtered Atomic-Hook with
    # the vertex table, ~22 MiB of workspace), then a small ER graph (the
    # atomic-free rounds)
    u, v, n = graphgen.rmat(19, 8, seed=7101, symmetrize=True)
    print("noalloc rmat19", n, len(u), flush=True)
    st = _pair(u, v, n, want=oracle.labels(u, v, n))
    assert st.hook == 1 and st.filter_used == 1
    u2, v2, n2, _ = graphgen.er_planted(n=1 << 13, m_er=1 << 14, cliques=8, seed=7102)
    print("noalloc er13", n2, len(u2), flush=True)
    st = _pair(u2, v2, n2, want=oracle.labels(u2, v2, n2))
    assert st.hook == 2


def test_noalloc_fallback_then_smaller():
    # percolated 3000^2 grid: the automatic hybrid plan needs 8 B per entry
    # (~100 MB), more than the fixed array, so the call falls back to the
    # Atomic-Hook; then a smaller grid on a side stream
    u, v, n = graphgen.grid(3000, 3000, 3, 10, seed=7103)
    assert cc.workspace_bytes(n, len(u)) > cc.CC_NOALLOC_SCRATCH_BYTES
    print("noalloc grid3000", n, len(u), flush=True)
    st = _pair(u, v, n, want=oracle.labels(u, v, n))
    assert st.hook == 1
    u2, v2, n2 = graphgen.grid(300, 200, 3, 10, seed=7104)
    side = torch.cuda.Stream()
    print("noalloc grid300x200 (side stream)", n2, len(u2), flush=True)
    _pair(u2, v2, n2, stream=side, want=oracle.labels(u2, v2, n2))


def test_noalloc_explicit_plan_too_large_and_bad_options():
    u, v, n = graphgen.grid(2048, 2048, 3, 10, seed=7105)
    du, dv = _dev(u, v)
    out = torch.empty(n, dtype=torch.int32, device=du.device)
    plain = cc.Options(hook="plain")
    assert cc.workspace_bytes(n, len(u), plain) > cc.CC_NOALLOC_SCRATCH_BYTES
    rc, _ = _noalloc_raw(du, dv, n, out, plain)
    assert rc == cc.CC_ERR_NOMEM and "fixed buffer" in cc.last_error()
    for bad in (cc.Options(graph=True), cc.Options(no_sync=True), cc.Options(profile=True)):
        rc, _ = _noalloc_raw(du, dv, n, out, bad)
        assert rc == cc.CC_ERR_ARG
    # an explicit plan that fits still runs, then a smaller one
    print("noalloc grid2048 atomic", n, len(u), flush=True)
    _pair(u, v, n, opts=cc.Options(hook="atomic"), want=oracle.labels(u, v, n))
    u2, v2, n2 = graphgen.rmat(12, 8, seed=7106)
    _pair(u2, v2, n2, opts=cc.Options(hook="hybrid"), want=oracle.labels(u2, v2, n2))


def test_noalloc_range_error_then_valid():
    u = np.array([0, 5, 2], np.int32)
    v = np.array([1, 9, 3], np.int32)
    du, dv = _dev(u, v)
    out = torch.empty(6, dtype=torch.int32, device=du.device)
    rc, _ = _noalloc_raw(du, dv, 6, out)
    assert rc == cc.CC_ERR_RANGE
    u2 = np.array([0, 2], np.int32)
    v2 = np.array([1, 3], np.int32)
    _pair(u2, v2, 4, want=np.array([0, 0, 2, 2], np.int32))
