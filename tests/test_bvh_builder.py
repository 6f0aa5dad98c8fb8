"""The host SAH builder's output satisfies what the device traversal relies on: a tree whose
nodes are each reached once, every triangle in exactly one leaf, child boxes inside parent
boxes and around their triangles, leaves of 1..15 triangles, depth <= 24; and the 4-wide tree the
traversal reads, collapsed from it two levels at a time: every wide node reached once, slot boxes
nested and around their triangles, every triangle in one leaf slot, depth <= 12 (the traversal
stack holds three deferred children per wide level)."""
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
    st = np.zeros(6, np.int32)
    rc = checker.bvh_check(pos.ctypes.data, pos.shape[0], tri.ctypes.data, tri.shape[0], st.ctypes.data)
    return rc, st


@pytest.mark.parametrize("mesh", ["one", "four", "icosphere", "degenerate", "sphere", "tori", "stack"])
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
    elif mesh == "stack":
        # a floor and 2^20 coincident copies of one triangle (the GPU deep-stack test's scene)
        floor_p, floor_t = I.quad_mesh(np.array([[-2, 0, 2], [2, 0, 2], [2, 0, -2], [-2, 0, -2]]), 1, 1)
        tv = np.array([[-0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.5, -0.5]], np.float32)
        pos = np.concatenate([floor_p, tv])
        tri = np.concatenate([floor_t, np.tile(np.array([[4, 5, 6]], np.int32), (1 << 20, 1))])
    elif mesh == "sphere":
        pos, tri = I.displaced_cube_sphere(129)
    else:
        pos, tri = I.interlocking_tori(1000, 250)
    rc, st = run(checker, pos, tri)
    assert rc == 0, f"invariant {rc} broken; stats {st}"
    assert st[1] <= 24 and st[2] <= 15
    assert 1 <= st[5] <= 12 and st[4] >= 1  # the 4-wide tree: depth <= 12 (stack of 3 x 12 + 1)
    if mesh == "stack":
        assert st[5] == 9  # a ray through the shared box defers 3 x 9 + 1 = 28 entries (25 in LDS)
    if mesh == "tori":
        assert st[0] < tri.shape[0]  # internal nodes
        assert st[1] <= 24
