"""The host SAH builder's output satisfies what the device traversal relies on: a tree whose
nodes are each reached once, every triangle in exactly one leaf, child boxes inside parent
boxes and around their triangles, leaves of 1..15 triangles, depth <= 24 (the traversal
stack holds 24 references)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2608_24109_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("bvh") / "bvh_check.so")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", "/opt/rocm/include", os.path.join(HERE, "bvh_check.cpp"),
           os.path.join(ROOT, "paper_2608_24109_amd", "csrc", "bvh_build.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    lib = C.CDLL(out)
    lib.bvh_check.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p]
    return lib


def run(checker, pos, tri):
    pos = np.ascontiguousarray(pos, np.float32)
    tri = np.ascontiguousarray(tri, np.int32)
    st = np.zeros(4, np.int32)
    rc = checker.bvh_check(pos.ctypes.data, pos.shape[0], tri.ctypes.data, tri.shape[0], st.ctypes.data)
    return rc, st


@pytest.mark.parametrize("mesh", ["one", "four", "icosphere", "degenerate", "sphere", "tori"])
def test_builder_invariants(checker, mesh):
    if mesh == "one":
        pos, tri = I.quad_mesh(np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]]), 1, 1)
        tri = tri[:1]
    elif mesh == "four":
        pos, tri = I.quad_mesh(np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]]), 2, 1)
    elif mesh == "icosphere":
        pos, tri = I.icosphere(3)
    elif mesh == "degenerate":
        # 5000 copies of the same triangle: centroids coincide, median splits by index
        pos = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
        tri = np.tile(np.array([[0, 1, 2]], np.int32), (5000, 1))
    elif mesh == "sphere":
        pos, tri = I.displaced_cube_sphere(129)
    else:
        pos, tri = I.interlocking_tori(1000, 250)
    rc, st = run(checker, pos, tri)
    assert rc == 0, f"invariant {rc} broken; stats {st}"
    assert st[1] <= 24 and st[2] <= 15
    if mesh == "tori":
        assert st[0] < tri.shape[0]  # internal nodes
        assert st[1] <= 24
