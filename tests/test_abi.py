"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, its structs match the binding, and argument errors caught on
the host come back as the documented status codes (no device call is made
on these paths)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_1612_01178_amd as cc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hookcc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cc_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cc.LIB_PATH):
        from paper_1612_01178_amd import build
        build.build()
    return cc.load()


def test_library_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert len(declared) >= 10, declared
    out = subprocess.check_output(["nm", "-D", "--defined-only", cc.LIB_PATH]).decode()
    exported = set(re.findall(r" T (cc_[a-z_0-9]+)$", out, flags=re.M))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert set(cc.EXPORTS) == set(declared)
    for f in declared:
        assert hasattr(lib, f)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "hookcc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(cc_options), offsetof(cc_options, profile),
         sizeof(cc_stats), offsetof(cc_stats, hook_ms), offsetof(cc_stats, reserved));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = list(map(int, subprocess.check_output([str(exe)]).split()))
    assert vals == [ctypes.sizeof(cc._COptions), cc._COptions.profile.offset,
                    ctypes.sizeof(cc._CStats), cc._CStats.hook_ms.offset,
                    cc._CStats.reserved.offset]


def test_version_and_options_init(lib):
    assert "gfx950" in cc.version()
    o = cc._COptions()
    lib.cc_options_init(ctypes.byref(o))
    assert o.filter == 2 and o.hook == 0 and o.segments == 0


def test_host_side_argument_errors(lib):
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: these calls fail before any device work
    assert lib.cc_labels(-1, None, None, 0, None) == cc.CC_ERR_ARG
    assert lib.cc_labels(5, None, None, -1, dummy) == cc.CC_ERR_ARG
    assert lib.cc_labels(5, None, None, 3, dummy) == cc.CC_ERR_ARG
    assert lib.cc_labels(5, dummy, dummy, 3, None) == cc.CC_ERR_ARG
    assert "out_label" in cc.last_error()
    # n == 0: nothing to do, unless there are edges (all of them out of range)
    assert lib.cc_labels(0, None, None, 0, None) == cc.CC_OK
    assert lib.cc_labels(0, dummy, dummy, 2, None) == cc.CC_ERR_RANGE
    bad = cc._COptions()
    bad.hook = 7
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    bad = cc._COptions()
    bad.edges_per_thread = 5
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    bad = cc._COptions()
    bad.host_loop = 1  # host loop needs the atomic-free Hook
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    bad = cc._COptions()
    bad.reserved[0] = 1
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    # no_sync: Atomic-Hook only, no profiling, single solves only
    for field, value in (("hook", 2), ("profile", 1)):
        bad = cc._COptions()
        bad.no_sync = 1
        setattr(bad, field, value)
        assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                                None) == cc.CC_ERR_ARG, field
    for tau in (-1, 1001):
        bad = cc._COptions()
        bad.compact_threshold = tau
        assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                                None) == cc.CC_ERR_ARG, tau
    bad = cc._COptions()
    bad.hook = 3  # the hybrid plan starts with the atomic-free Hook: no symmetric flag
    bad.symmetric = 1
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    bad = cc._COptions()
    bad.no_sync = 2
    assert lib.cc_labels_ex(4, dummy, dummy, 1, dummy, ctypes.byref(bad), None, 0, None,
                            None) == cc.CC_ERR_ARG
    bad = cc._COptions()
    bad.no_sync = 1
    assert lib.cc_labels_host(4, dummy, dummy, 1, dummy, 0, ctypes.byref(bad), None,
                              None) == cc.CC_ERR_ARG
    assert lib.cc_labels_list(0, None, ctypes.byref(bad), None, None) == cc.CC_ERR_ARG
    # no no-sync call was made on this stream
    assert lib.cc_stream_status(None) == cc.CC_ERR_ARG
    # batches: offsets are validated on the host
    import numpy as np
    vo = np.array([0, 4, 3], dtype=np.int64)
    eo = np.array([0, 1, 2], dtype=np.int64)
    assert lib.cc_labels_batch(2, vo.ctypes.data, eo.ctypes.data, dummy, dummy,
                               dummy) == cc.CC_ERR_ARG
    vo = np.array([1, 4], dtype=np.int64)
    assert lib.cc_labels_batch(1, vo.ctypes.data, eo.ctypes.data, dummy, dummy,
                               dummy) == cc.CC_ERR_ARG
    assert lib.cc_labels_batch(-1, None, None, None, None, None) == cc.CC_ERR_ARG
    assert lib.cc_labels_batch(0, None, None, None, None, None) == cc.CC_OK
    # the LDS solver's workgroup size is validated before any device work
    vo = np.array([0, 4], dtype=np.int64)
    eo = np.array([0, 1], dtype=np.int64)
    bad_block = cc.Options(block=100)._c()
    assert lib.cc_labels_batch_ex(1, vo.ctypes.data, eo.ctypes.data, dummy, dummy, dummy,
                                  ctypes.byref(bad_block), None, None) == cc.CC_ERR_ARG
    assert lib.cc_probe(3, dummy, dummy, 4, None, 0, None) == cc.CC_ERR_ARG
    # memory-model probes need a table of at least 128 words; unknown modes fail
    assert lib.cc_probe(7, None, None, 0, None, 0, None) == cc.CC_ERR_ARG
    assert lib.cc_probe(10, None, None, 0, dummy, 64, None) == cc.CC_ERR_ARG
    assert lib.cc_probe(12, dummy, dummy, 4, dummy, 128, None) == cc.CC_ERR_ARG


def test_workspace_sizes(lib):
    n, m = 1 << 20, 1 << 24
    base = cc.workspace_bytes(n, m, cc.Options(filter="off"))
    assert base == 256
    giant = cc.workspace_bytes(n, m, cc.Options(filter="giant", hot_cache="off"))
    assert giant == 256 + (n // 32) * 4
    hot = cc.workspace_bytes(n, m, cc.Options(filter="giant", hot_cache="large"))
    assert hot == 256 + 2 * (n // 32) * 4 + 2 * 32768 * 4
    # vertex table: 256 parts x 16,384 sampled endpoints, two 256 x 1,280
    # count/offset tables (parts x buckets of 64 sets), 163,840 one-byte tags
    # and as many member flags
    vert = cc.workspace_bytes(n, m, cc.Options(filter="giant"))
    assert vert == 256 + (n // 32) * 4 + (256 * 16384 + 2 * 256 * 1280) * 4 + 2 * 163840
    assert cc.workspace_bytes(n, m, cc.Options(filter="giant", hot_cache="vertex")) == vert
    big = 255 * 81920 + 1  # ids past the tags' range: the automatic choice is the word table
    assert cc.workspace_bytes(big, m, cc.Options(filter="giant")) == \
        cc.workspace_bytes(big, m, cc.Options(filter="giant", hot_cache="large"))
    plain = cc.workspace_bytes(n, m, cc.Options(hook="plain"))
    assert plain == 256 + 2 * m * 8
    hybrid = cc.workspace_bytes(n, m, cc.Options(hook="hybrid"))
    assert hybrid == 256 + m * 8
    assert cc.workspace_bytes(-1, 5) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(cc, "_lib", None)
    monkeypatch.setattr(cc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        cc.load()
