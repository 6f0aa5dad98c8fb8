"""The C-ABI library on the CPU: it loads, exports every entry point include/exm.h declares,
and rejects invalid arguments with EXM_E_INVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2608_24109_amd import _lib
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "exm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(exm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L.lib, n), n


def _mesh(L, nV=3, nF=1, nUV=3, ptr=0x1000):
    return L.exm_mesh(nV, nF, nUV, ptr, ptr, ptr, ptr, ptr, ptr)


def _cams(L, n=1, H=8, W=8):
    from paper_2608_24109_amd import inputs as I
    return L.cameras(I.ring_cameras(n, 3.0, H, W))


def _status(L, fn, *args):
    s = fn(*args)
    return s, L.last_error()


def test_raster_validation(L):
    f = L.lib.exm_raster_gbuffer
    m = _mesh(L)
    cams = _cams(L)
    assert _status(L, f, None, cams, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
    assert _status(L, f, C.byref(m), None, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
    assert _status(L, f, C.byref(m), cams, 0, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
    s, msg = _status(L, f, C.byref(m), cams, 1, 0x1000, 0x1004, None)
    assert s == L.EXM_E_INVAL and "aligned" in msg
    bad = _mesh(L, nV=0)
    assert _status(L, f, C.byref(bad), cams, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
    two = _cams(L, 2)
    two[1].H = 9
    s, msg = _status(L, f, C.byref(m), two, 2, 0x1000, 0x1000, None)
    assert s == L.EXM_E_INVAL and "share H and W" in msg
    nan = _cams(L)
    nan[0].mvp[5] = float("nan")
    assert _status(L, f, C.byref(m), nan, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
    huge = _cams(L, 1, H=65536, W=65536)
    assert _status(L, f, C.byref(m), huge, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL


def test_injected_failures_are_counted_and_taken_after_validation(L):
    """exm_inject_failures(n): the next n calls that pass validation return EXM_E_HIP with the
    injected message; invalid calls still return EXM_E_INVAL and leave the count alone. (Every
    call here fails before any launch, so the test never touches a device.)"""
    f = L.lib.exm_raster_gbuffer
    m = _mesh(L)
    cams = _cams(L)
    L.inject_failures(3)
    try:
        assert _status(L, f, None, cams, 1, 0x1000, 0x1000, None)[0] == L.EXM_E_INVAL
        assert _status(L, f, C.byref(m), cams, 1, 0x1000, 0x1004, None)[0] == L.EXM_E_INVAL
        for _ in range(3):
            s, msg = _status(L, f, C.byref(m), cams, 1, 0x1000, 0x1000, None)
            assert s == L.EXM_E_HIP and "injected failure" in msg
        L.inject_failures(1)
        assert L.lib.exm_env_guide_len(4, 8) > 0  # a size query reaches no device, takes nothing
        s, msg = _status(L, f, C.byref(m), cams, 1, 0x1000, 0x1000, None)
        assert s == L.EXM_E_HIP and "injected failure" in msg
        L.inject_failures(-5)  # clears; a negative count injects nothing
        L.inject_failures(1)
    finally:
        L.inject_failures(0)
    s, msg = _status(L, f, None, cams, 1, 0x1000, 0x1000, None)
    assert s == L.EXM_E_INVAL and "injected" not in msg


def test_shade_validation(L):
    m = _mesh(L)
    cams = _cams(L)
    mat = L.exm_material(4, 4, 0x1000)
    env = L.exm_env(4, 8, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    f = L.lib.exm_shade_fwd
    bvh = 0x2000

    def call(p=None, **kw):
        a = dict(m=C.byref(m), bvh=bvh, mat=C.byref(mat), env=C.byref(env), cams=cams, n=1, tri=0x1000,
                 bary=0x1000, p=C.byref(p if p is not None else L.params(8)), L=0x1000, vis=0x1000,
                 ws=0x100000, ws_bytes=1 << 30, stream=None)
        a.update(kw)
        return _status(L, f, *a.values())

    assert call(L.params(65))[0] == L.EXM_E_INVAL
    assert call(L.params(-1))[0] == L.EXM_E_INVAL
    assert call(L.params(8, tmin=float("inf")))[0] == L.EXM_E_INVAL
    assert call(L.params(8, flags=1 << 7))[0] == L.EXM_E_INVAL
    assert call(bvh=None)[0] == L.EXM_E_INVAL
    assert call(L=None)[0] == L.EXM_E_INVAL
    mis = L.exm_material(4, 4, 0x1004)
    assert call(mat=C.byref(mis))[0] == L.EXM_E_INVAL
    e1 = L.exm_env(4, 1, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    assert call(env=C.byref(e1))[0] == L.EXM_E_INVAL
    no_guide = L.exm_env(4, 8, 0x1000, 0x1000, 0x1000, 0x1000, None, 0x1000)
    assert call(env=C.byref(no_guide))[0] == L.EXM_E_INVAL
    rec8 = L.exm_env(4, 8, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1008)
    s, msg = call(env=C.byref(rec8))
    assert s == L.EXM_E_INVAL and "misaligned" in msg
    unprep = L.exm_mesh(3, 1, 3, 0x1000, 0x1000, 0x1000, 0x1000, None, None)
    s, msg = call(m=C.byref(unprep))
    assert s == L.EXM_E_INVAL and "exm_mesh_prepare" in msg
    s, msg = call(ws_bytes=L.exm_shade_fwd_workspace_min(8) - 1)
    assert s == L.EXM_E_INVAL and "workspace" in msg
    assert call(ws=0x100010)[0] == L.EXM_E_INVAL  # not 256-byte aligned
    assert call(ws=None)[0] == L.EXM_E_INVAL


def test_workspace_sizes(L):
    assert L.exm_shade_fwd_workspace_min(64) < L.exm_shade_fwd_workspace_size(1, 128, 128, 64)
    one = L.exm_shade_fwd_workspace_size(1, 1024, 1024, 64)
    assert L.exm_shade_fwd_workspace_size(8, 1024, 1024, 64) > 7 * one
    assert L.exm_shade_fwd_workspace_size(16, 1024, 1024, 64) == L.exm_shade_fwd_workspace_size(8, 1024, 1024, 64)
    assert L.exm_shade_fwd_workspace_size(0, 8, 8, 8) == 0 and L.exm_shade_fwd_workspace_min(65) == 0


def test_adjoint_workspace_sizes(L):
    # one 16-byte record per env sample, twice (as appended and grouped), plus bucket tables
    one = L.exm_shade_bwd_workspace_size(1, 1024, 1024, 64, 512, 1024)
    assert one >= 2 * 16 * 64 * 1024 * 1024
    assert L.exm_shade_bwd_workspace_size(16, 1024, 1024, 64, 512, 1024) == \
        L.exm_shade_bwd_workspace_size(8, 1024, 1024, 64, 512, 1024)
    assert L.exm_shade_bwd_workspace_min(64, 512, 1024) < one
    assert L.exm_trace_bwd_workspace_size(1, 64, 64, 4, 4, 32, 64) >= 2 * 16 * 16 * 64 * 64
    assert L.exm_trace_bwd_workspace_min(8, 16, 32, 64) == 0  # N_b * N_s > 64
    assert L.exm_shade_bwd_workspace_size(1, 8, 8, 65, 32, 64) == 0


def test_indirect_and_backward_validation(L):
    m = _mesh(L)
    cams = _cams(L)
    mat = L.exm_material(4, 4, 0x1000)
    env = L.exm_env(4, 8, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    p = L.params(8, N_b=16, N_s=8)  # 128 light-sample bits do not fit one u64
    s = L.lib.exm_trace_indirect(C.byref(m), 0x2000, C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000,
                                 C.byref(p), 0x1000, 0x1000, 0x1000, 0x100000, 1 << 30, None)
    assert s == L.EXM_E_INVAL
    p = L.params(8, N_b=4, N_s=4)
    small = L.exm_trace_indirect_workspace_min(4, 4) - 1
    s = L.lib.exm_trace_indirect(C.byref(m), 0x2000, C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000,
                                 C.byref(p), 0x1000, 0x1000, 0x1000, 0x100000, small, None)
    assert s == L.EXM_E_INVAL and "workspace" in L.last_error()
    p = L.params(8, N_b=4, N_s=4)
    big = 1 << 30
    s = L.lib.exm_trace_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            float("nan"), 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x100000, big, None)
    assert s == L.EXM_E_INVAL
    s = L.lib.exm_shade_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            0x1000, 0x1000, None, None, 0x1000, 0x100000, big, None)
    assert s == L.EXM_E_INVAL
    small = L.exm_shade_bwd_workspace_min(8, 4, 8) - 1
    s = L.lib.exm_shade_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            0x1000, 0x1000, None, 0x1000, 0x1000, 0x100000, small, None)
    assert s == L.EXM_E_INVAL and "workspace" in L.last_error()
    s = L.lib.exm_shade_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            0x1000, 0x1000, 0x1004, 0x1000, 0x1000, 0x100000, big, None)
    assert s == L.EXM_E_INVAL and "dquery" in L.last_error()
    s = L.lib.exm_shade_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            0x1000, 0x1000, None, 0x1008, 0x1000, 0x100000, big, None)
    assert s == L.EXM_E_INVAL and "dtex" in L.last_error()
    s = L.lib.exm_trace_bwd(C.byref(m), C.byref(mat), C.byref(env), cams, 1, 0x1000, 0x1000, C.byref(p),
                            1.0, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x100010, big, None)
    assert s == L.EXM_E_INVAL and "workspace" in L.last_error()  # not 256-byte aligned


def test_env_sampler_and_bvh_validation(L):
    f = L.lib.exm_build_env_sampler
    a = 0x1000
    assert f(a, 0, 8, a, a, a, a, a, None) == L.EXM_E_INVAL
    assert f(a, 4, 1, a, a, a, a, a, None) == L.EXM_E_INVAL
    assert f(a, 4096, 8192, a, a, a, a, a, None) == L.EXM_E_INVAL
    assert f(a, 4, 8, a, a, 0x1004, a, a, None) == L.EXM_E_INVAL
    assert f(a, 4, 8, a, a, a, None, a, None) == L.EXM_E_INVAL
    assert f(a, 4, 8, a, a, a, a, 0x1008, None) == L.EXM_E_INVAL
    # cutpoint tables: row shift + (He + 1) row entries + He column shifts + He (We + 1) entries
    # cutpoint tables, then for maps narrower than 4096 texels the column CDF in 32 bits, the
    # column entries in 16 and the column CDF's low 16 bits
    assert L.exm_env_guide_len(512, 1024) == 1 + 513 + 512 + 512 * 1025 + 512 * 1024 + 512 * 1025 // 2 + 512 * 512
    assert L.exm_env_guide_len(7, 13) == 1 + 8 + 7 + 7 * 14 + 7 * 13 + (7 * 14 + 1) // 2 + (7 * 13 + 1) // 2
    assert L.exm_env_guide_len(4, 4096) == 1 + 5 + 4 + 4 * 4097
    assert L.exm_env_guide_len(0, 8) == 0
    pos = np.zeros((3, 3), np.float32)
    tri = np.array([[0, 1, 3]], np.int32)
    out = C.c_void_p()
    s = L.lib.exm_build_bvh(pos.ctypes.data, 3, tri.ctypes.data, 1, C.byref(out), None)
    assert s == L.EXM_E_INVAL and "out of range" in L.last_error() and not out.value
    pos[1, 2] = np.inf
    tri[0, 2] = 2
    assert L.lib.exm_build_bvh(pos.ctypes.data, 3, tri.ctypes.data, 1, C.byref(out), None) == L.EXM_E_INVAL
    assert L.lib.exm_free_bvh(None) == L.EXM_OK
    assert L.lib.exm_bvh_device_bytes(None) == 0
    # the depth bound (24 deferred references) holds up to 2 * 2^24 triangles; beyond it the
    # build is refused before the index arrays are read (these hold one triangle only)
    big = (2 << 24) + 1
    assert L.lib.exm_build_bvh(pos.ctypes.data, 3, tri.ctypes.data, big, C.byref(out), None) == L.EXM_E_UNSUPPORTED
    assert "2^25" in L.last_error() and not out.value


def _topo(L, nV=3, nF=1, nUV=3, cap=(4, 3, 5), ptr=0x1000):
    return L.exm_topo_mesh(nV, nF, nUV, cap[0], cap[1], cap[2], ptr, ptr, ptr, ptr, ptr)


def test_topology_validation_and_workspace(L):
    from paper_2608_24109_amd.topology import TopoConfig
    p = TopoConfig().c()
    # workspace: grows with the mesh, needs no device
    small = L.exm_topology_workspace_size(642, 1280, 3840, p)
    big = L.exm_topology_workspace_size(49688, 99372, 298116, p)
    assert 0 < small < big and big > 99372 * 8 * 8
    assert L.lib.exm_topology_workspace_size(-1, 4, 4, C.byref(p)) == 0
    st = L.exm_topo_stats()
    f = L.lib.exm_topology_round
    ws = 0x1000
    m = _topo(L)
    assert _status(L, f, None, None, C.byref(p), ws, 1 << 20, C.byref(st), None)[0] == L.EXM_E_INVAL
    bad = L.exm_topo_params(p.beta_g, p.w_g, p.w_k, p.tau_degen, p.tau_uv, 1.5, p.max_faces, p.flags)
    assert _status(L, f, C.byref(m), None, C.byref(bad), ws, 1 << 20, C.byref(st), None)[0] == L.EXM_E_INVAL
    over = _topo(L, nV=5)
    s, msg = _status(L, f, C.byref(over), None, C.byref(p), ws, 1 << 20, C.byref(st), None)
    assert s == L.EXM_E_INVAL and "capacities" in msg
    # one split needs a vertex, two faces and two UVs of room
    q = TopoConfig(split_fraction=1.0).c()
    tight = _topo(L, cap=(3, 1, 3))
    s, msg = _status(L, f, C.byref(tight), None, C.byref(q), ws, 1 << 20, C.byref(st), None)
    assert s == L.EXM_E_INVAL and "nV + K" in msg
    s, _ = _status(L, f, C.byref(m), None, C.byref(p), ws, 16, C.byref(st), None)
    assert s == L.EXM_E_NOMEM
    g = L.lib.exm_vertex_grad_ema
    assert _status(L, g, 0x1000, 0x1000, 4, 1.5, None)[0] == L.EXM_E_INVAL
    assert _status(L, g, None, 0x1000, 4, 0.9, None)[0] == L.EXM_E_INVAL
    assert _status(L, L.lib.exm_face_render_counts, 0x1000, -1, 4, 0x1000, None)[0] == L.EXM_E_INVAL
