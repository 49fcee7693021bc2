"""The C ABI used from plain C: tests/c_abi_example (built by
__graft_entry__.build()) solves a graph with cc_labels, a no-sync
cc_labels_ex polled with cc_stream_status, and a two-graph cc_labels_batch,
checks an out-of-range endpoint, and prints the labels, which must equal the
oracle's."""
import os
import subprocess

import numpy as np
import pytest

import graphgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi_example")


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["rmat", "grid", "isolated"])
def test_c_program_uses_the_abi(tmp_path, case):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi_example is not built (run __graft_entry__.build())")
    if case == "rmat":
        u, v, n = graphgen.rmat(12, 8, seed=91)
    elif case == "grid":
        u, v, n = graphgen.grid(64, 48, 3, 10, seed=92)
    else:
        u, v, n = np.array([3], np.int32), np.array([5], np.int32), 9
    path = tmp_path / "graph.txt"
    with open(path, "w") as f:
        f.write("%d %d\n" % (n, len(u)))
        for a, b in zip(u.tolist(), v.tolist()):
            f.write("%d %d\n" % (a, b))
    print("c_abi_example", case, n, len(u), flush=True)
    r = subprocess.run([EXE, str(path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = np.array(r.stdout.split(), dtype=np.int64).astype(np.int32)
    assert np.array_equal(got, oracle.labels(u, v, n))
