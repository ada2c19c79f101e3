"""The C ABI's host code (argument checks, planner, plan cache) built with the
host sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) and driven through
hss_plan_create / hss_plan_query / hss_plan_destroy and hss_factor's checks.

The device parts are replaced by stand-ins that report HSS_EDEVICE
(tests/sanitize/stub_engine.cpp); the driver (tests/sanitize/plan_driver.cpp)
prints every box's sets, which are compared with the oracle's, and exercises the
error paths. Any sanitizer report fails the run (halt_on_error, exit code != 0).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.sets import TreeSets, hss_postorder
from workloads import partition, sipg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1508_07798_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are missing")
    out = str(tmp_path_factory.mktemp("san") / "plan_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-static-libasan", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(SAN, "plan_driver.cpp"), os.path.join(SAN, "stub_engine.cpp"),
           os.path.join(CSRC, "capi.cpp"), os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "tuning.cpp"),
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-ldl", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _write(path, op, tree, heaps, leaf):
    i32 = lambda a: np.asarray(a, dtype="<i4").ravel()
    parts = [i32([op.n_el, op.q, op.row_ptr[-1]]), i32(op.row_ptr), i32(op.col_idx),
             i32([len(tree.leaf_node)]), i32(tree.leaf_node), i32(tree.leaf_ptr), i32(tree.leaf_elems),
             i32(tree.elem_xy), i32([len(heaps)]), i32(heaps), i32([leaf])]
    with open(path, "wb") as f:
        for a in parts:
            f.write(a.tobytes())


def _run(driver, tmp_path, op, tree, leaf):
    T = TreeSets(op.row_ptr, op.col_idx, op.q, tree, hss_leaf_elems=leaf)
    heaps = sorted(T.nodes)
    fn = str(tmp_path / "structure.bin")
    _write(fn, op, tree, heaps, leaf)
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, fn], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert lines[-1] == "ok"
    vec = lambda ln, tag: (ln.split()[0] == tag, np.array([int(x) for x in ln.split()[1:]], dtype=np.int64))
    it = iter(lines[:-1])
    for s in heaps:
        box = next(it).split()
        assert box[0] == "box" and int(box[1]) == s and int(box[2]) == T.height[s]
        ns = T.sets[s]
        ok, I = vec(next(it), "I")
        assert ok and np.array_equal(I, ns.idof), s
        ok, B = vec(next(it), "B")
        assert ok and np.array_equal(B, ns.bdof), s
        ok, H = vec(next(it), "H")
        ref = hss_postorder(ns.hss)
        H = H.reshape(-1, 4)
        assert ok and H.shape[0] == len(ref), s
        for row, t in zip(H, ref):
            assert (row[0], row[1]) == (t.lo, t.hi) and (row[2] < 0) == t.is_leaf
    ok, R = vec(next(it), "R")
    assert ok and np.array_equal(R, T.root_idof)


@pytest.mark.parametrize("n,p,pde,scheme,leaf", [(16, 1, "poisson", "boxes", 4), (21, 2, "helmholtz", "boxes", 4),
                                                  (12, 3, "poisson", "vslabs", 2), (24, 2, "helmholtz", "boxes", 7)])
def test_planner_under_sanitizers(driver, tmp_path, n, p, pde, scheme, leaf):
    op = sipg.assemble(n, p, pde, kappa=10.0)
    tree = partition.build_tree(n, n, 16, scheme=scheme)
    _run(driver, tmp_path, op, tree, leaf)
