"""ctypes binding of libexm.so: the C ABI of include/exm.h under the same names.

Argument marshalling only: tensors become device pointers, the current torch stream becomes
the HIP stream; every step of the render pass runs in the library's HIP kernels. There is
no fallback: if libexm.so is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexm.so")

EXM_OK = 0
EXM_E_INVAL = -1
EXM_E_HIP = -2
EXM_E_NOMEM = -3
EXM_E_UNSUPPORTED = -4

EXM_METALLIC_OFF = 1 << 0
EXM_DIFFUSE_ONLY = 1 << 1
EXM_SPECULAR_ONLY = 1 << 2
EXM_NO_VIS = 1 << 3
EXM_NO_SECONDARY_MATERIAL = 1 << 4
EXM_MAP_GRAD_ATOMIC = 1 << 5

EXM_TOPO_NO_SPLIT = 1 << 0
EXM_TOPO_NO_MERGE = 1 << 1


class ExmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class exm_mesh(C.Structure):
    _fields_ = [("nV", C.c_int32), ("nF", C.c_int32), ("nUV", C.c_int32), ("pos", C.c_void_p),
                ("tri", C.c_void_p), ("uv", C.c_void_p), ("tri_uv", C.c_void_p), ("vnrm", C.c_void_p),
                ("ftan", C.c_void_p)]


class exm_camera(C.Structure):
    _fields_ = [("mvp", C.c_double * 16), ("eye", C.c_double * 3), ("H", C.c_int32), ("W", C.c_int32),
                ("view_id", C.c_int32)]


class exm_material(C.Structure):
    _fields_ = [("Ht", C.c_int32), ("Wt", C.c_int32), ("tex", C.c_void_p)]


class exm_env(C.Structure):
    _fields_ = [("He", C.c_int32), ("We", C.c_int32), ("env", C.c_void_p), ("cdf_row", C.c_void_p),
                ("cdf_col", C.c_void_p), ("pdf", C.c_void_p), ("guide", C.c_void_p), ("rec", C.c_void_p)]


class exm_params(C.Structure):
    _fields_ = [("N_d", C.c_int32), ("N_b", C.c_int32), ("N_s", C.c_int32), ("seed", C.c_uint64),
                ("iteration", C.c_uint64), ("f_diel", C.c_float), ("eps", C.c_float), ("tmin", C.c_float),
                ("flags", C.c_uint32)]


class exm_request(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("bvh", C.c_void_p), ("mat", C.c_void_p), ("env", C.c_void_p),
                ("cam", exm_camera), ("tmin", C.c_float), ("tri_id", C.c_void_p), ("bary", C.c_void_p),
                ("L_dir", C.c_void_p), ("vis", C.c_void_p)]


SEC_REC_BYTES = 12  # exm_sec_rec {int32 tri; float b1, b2}


class exm_topo_mesh(C.Structure):
    _fields_ = [("nV", C.c_int32), ("nF", C.c_int32), ("nUV", C.c_int32), ("capV", C.c_int32), ("capF", C.c_int32),
                ("capUV", C.c_int32), ("pos", C.c_void_p), ("G", C.c_void_p), ("uv", C.c_void_p),
                ("tri", C.c_void_p), ("tri_uv", C.c_void_p)]


class exm_topo_params(C.Structure):
    _fields_ = [("beta_g", C.c_double), ("w_g", C.c_double), ("w_k", C.c_double), ("tau_degen", C.c_double),
                ("tau_uv", C.c_double), ("split_fraction", C.c_double), ("max_faces", C.c_int32),
                ("flags", C.c_uint32)]


class exm_topo_stats(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("split_selected", "split_invalid", "split_conflict", "splits",
                                         "merge_candidates", "merge_conflict", "merges", "faces_deleted",
                                         "mis_iterations")]

    def as_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_24109_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, st = C.c_void_p, C.c_int32, C.c_int
    sig = {
        "exm_last_error": (C.c_char_p, []),
        "exm_inject_failures": (None, [i32]),
        "exm_mesh_prepare": (st, [vp, vp]),
        "exm_build_bvh": (st, [vp, i32, vp, i32, C.POINTER(vp), vp]),
        "exm_free_bvh": (st, [vp]),
        "exm_bvh_device_bytes": (C.c_size_t, [vp]),
        "exm_env_guide_len": (C.c_size_t, [i32, i32]),
        "exm_build_env_sampler": (st, [vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "exm_raster_gbuffer": (st, [vp, vp, i32, vp, vp, vp]),
        "exm_shade_fwd_workspace_size": (C.c_size_t, [i32, i32, i32, i32]),
        "exm_shade_fwd_workspace_min": (C.c_size_t, [i32]),
        "exm_shade_fwd": (st, [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "exm_trace_indirect_workspace_size": (C.c_size_t, [i32, i32, i32, i32, i32]),
        "exm_trace_indirect_workspace_min": (C.c_size_t, [i32, i32]),
        "exm_trace_indirect": (st, [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "exm_shade_fwd_batch_workspace_size": (C.c_size_t, [vp, i32, i32]),
        "exm_shade_fwd_batch": (st, [vp, i32, vp, vp, C.c_size_t, vp]),
        "exm_shade_fwd_noalloc": (st, [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]),
        "exm_shade_fwd_counted": (st, [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, vp]),
        "exm_trace_indirect_counted": (st, [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp,
                                            vp]),
        "exm_shade_bwd": (st, [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "exm_trace_bwd": (st, [vp, vp, vp, vp, i32, vp, vp, vp, C.c_float, vp, vp, vp, vp, vp, vp, C.c_size_t,
                               vp]),
        "exm_shade_bwd_workspace_size": (C.c_size_t, [i32, i32, i32, i32, i32, i32]),
        "exm_shade_bwd_workspace_min": (C.c_size_t, [i32, i32, i32]),
        "exm_trace_bwd_workspace_size": (C.c_size_t, [i32, i32, i32, i32, i32, i32, i32]),
        "exm_trace_bwd_workspace_min": (C.c_size_t, [i32, i32, i32, i32]),
        "exm_upsample_indirect": (st, [vp, i32, i32, vp, vp, i32, i32, i32, vp, vp]),
        "exm_upsample_indirect_bwd": (st, [vp, i32, i32, vp, i32, i32, i32, C.c_float, vp, vp, vp]),
        "exm_project_maps": (st, [vp, vp, i32, i32, i32, vp, vp, vp, vp]),
        "exm_project_maps_bwd": (st, [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp]),
        "exm_image_loss_workspace_size": (C.c_size_t, [i32, i32]),
        "exm_image_loss": (st, [vp, vp, i32, i32, i32, C.c_float, vp, vp, vp, C.c_size_t, vp]),
        "exm_tv_screen": (st, [vp, vp, i32, i32, i32, i32, C.c_float, vp, vp, vp]),
        "exm_env_regularizers": (st, [vp, i32, i32, C.c_float, C.c_float, vp, vp, vp, vp]),
        "exm_adam_step": (st, [vp, vp, i32, vp, vp, C.c_int64, i32, vp, vp, C.c_double, C.c_double, C.c_double,
                               C.c_double, i32, vp]),
        "exm_vertex_grad_ema": (st, [vp, vp, i32, C.c_double, vp]),
        "exm_face_render_counts": (st, [vp, C.c_int64, i32, vp, vp]),
        "exm_topology_workspace_size": (C.c_size_t, [i32, i32, i32, vp]),
        "exm_topology_scores": (st, [vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
        "exm_topology_round": (st, [vp, vp, vp, vp, C.c_size_t, vp, vp]),
        "exm_timing_enable": (st, [i32]),
        "exm_timing_collect": (st, []),
        "exm_timing_count": (i32, []),
        "exm_timing_name": (C.c_char_p, [i32]),
        "exm_timing_total_ms": (C.c_double, [i32]),
        "exm_timing_launches": (C.c_int64, [i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def last_error() -> str:
    return lib.exm_last_error().decode()


def inject_failures(n: int) -> None:
    """The next n library calls that would reach the device fail with EXM_E_HIP (a test hook for
    error paths); 0 clears."""
    lib.exm_inject_failures(int(n))


def _check(status: int, where: str) -> None:
    if status != EXM_OK:
        raise ExmError(status, where, last_error())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _need(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def cameras(cams, view_ids=None) -> C.Array:
    """Host array of exm_camera from objects with .mvp (4x4), .eye (3), .H, .W."""
    arr = (exm_camera * len(cams))()
    for i, c in enumerate(cams):
        m = np.asarray(c.mvp, dtype=np.float64).ravel()
        for k in range(16):
            arr[i].mvp[k] = float(m[k])
        for k in range(3):
            arr[i].eye[k] = float(c.eye[k])
        arr[i].H, arr[i].W = int(c.H), int(c.W)
        arr[i].view_id = int(view_ids[i] if view_ids is not None else getattr(c, "view_id", i))
    return arr


def params(N_d: int, N_b: int = 0, N_s: int = 0, seed: int = 3, iteration: int = 0, f_diel: float = 0.04,
           eps: float = 1e-6, tmin: float = 0.0, flags: int = 0) -> exm_params:
    return exm_params(N_d, N_b, N_s, seed, iteration, f_diel, eps, tmin, flags)


# ------------------------------------------------------------------------------------------
# the C ABI under the same names
# ------------------------------------------------------------------------------------------

def exm_mesh_prepare(mesh: exm_mesh, stream=None) -> None:
    _check(lib.exm_mesh_prepare(C.byref(mesh), _stream(stream)), "exm_mesh_prepare")


class Bvh:
    """Owner of a device-resident BVH handle."""

    def __init__(self, handle: int):
        self.handle = handle

    @property
    def device_bytes(self) -> int:
        return int(lib.exm_bvh_device_bytes(self.handle))

    def free(self) -> None:
        if self.handle:
            _check(lib.exm_free_bvh(self.handle), "exm_free_bvh")
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def exm_build_bvh(pos: np.ndarray, tri: np.ndarray, stream=None) -> Bvh:
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    out = C.c_void_p()
    _check(lib.exm_build_bvh(pos.ctypes.data, pos.shape[0], tri.ctypes.data, tri.shape[0], C.byref(out),
                             _stream(stream)), "exm_build_bvh")
    return Bvh(out.value)


def exm_env_guide_len(He: int, We: int) -> int:
    return int(lib.exm_env_guide_len(He, We))


def exm_build_env_sampler(env, cdf_row, cdf_col, pdf, guide, rec, stream=None) -> None:
    """`guide` is int32 storage for the uint32 cutpoint tables; `rec` is float32 [He,We,4]."""
    import torch
    He, We = env.shape[0], env.shape[1]
    _need(env, torch.float32, (He, We, 3), "env")
    _need(cdf_row, torch.uint64, (He,), "cdf_row")
    _need(cdf_col, torch.uint64, (He, We), "cdf_col")
    _need(pdf, torch.float32, (He, We), "pdf")
    _need(guide, torch.int32, (exm_env_guide_len(He, We),), "guide")
    _need(rec, torch.float32, (He, We, 4), "rec")
    _check(lib.exm_build_env_sampler(_ptr(env), He, We, _ptr(cdf_row), _ptr(cdf_col), _ptr(pdf), _ptr(guide),
                                     _ptr(rec), _stream(stream)), "exm_build_env_sampler")


def exm_raster_gbuffer(mesh: exm_mesh, cams, tri_id, bary, stream=None) -> None:
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(tri_id, torch.int32, (n, H, W), "tri_id")
    _need(bary, torch.float32, (n, H, W, 2), "bary")
    _check(lib.exm_raster_gbuffer(C.byref(mesh), cams, n, _ptr(tri_id), _ptr(bary), _stream(stream)),
           "exm_raster_gbuffer")


def exm_shade_fwd_workspace_size(nViews: int, H: int, W: int, N_d: int) -> int:
    return int(lib.exm_shade_fwd_workspace_size(nViews, H, W, N_d))


def exm_shade_fwd_workspace_min(N_d: int) -> int:
    return int(lib.exm_shade_fwd_workspace_min(N_d))


def workspace(nbytes: int, device="cuda"):
    """A device byte buffer for the ray workspaces (the caching allocator keeps it 256-B aligned)."""
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def exm_shade_fwd(mesh, bvh: Bvh, mat: exm_material, env: exm_env, cams, tri_id, bary, p: exm_params, L_dir,
                  vis, ws, stream=None) -> None:
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(L_dir, torch.float32, (n, H, W, 3), "L_dir")
    _need(vis, torch.uint64, (n, H, W), "vis")
    _check(lib.exm_shade_fwd(C.byref(mesh), bvh.handle, C.byref(mat), C.byref(env), cams, n, _ptr(tri_id),
                             _ptr(bary), C.byref(p), _ptr(L_dir), _ptr(vis), _ptr(ws), ws.numel(), _stream(stream)),
           "exm_shade_fwd")


def request(mesh, mat, env, cam: exm_camera, tmin: float, tri_id, bary, L_dir, vis) -> exm_request:
    """One request of a batched direct pass: device asset objects (DeviceMesh with its BVH,
    DeviceMaterial, DeviceEnv), its camera, ray start distance and [1,H,W...] buffers. The
    objects must outlive the call."""
    import torch
    H, W = cam.H, cam.W
    _need(tri_id, torch.int32, (1, H, W), "tri_id")
    _need(bary, torch.float32, (1, H, W, 2), "bary")
    _need(L_dir, torch.float32, (1, H, W, 3), "L_dir")
    _need(vis, torch.uint64, (1, H, W), "vis")
    return exm_request(C.addressof(mesh.s), mesh.bvh.handle, C.addressof(mat.s), C.addressof(env.s), cam, float(tmin),
                       _ptr(tri_id), _ptr(bary), _ptr(L_dir), _ptr(vis))


def _requests(reqs) -> C.Array:
    return (exm_request * len(reqs))(*reqs)


def exm_shade_fwd_batch_workspace_size(reqs, N_d: int) -> int:
    return int(lib.exm_shade_fwd_batch_workspace_size(_requests(reqs), len(reqs), N_d))


def exm_shade_fwd_batch(reqs, p: exm_params, ws, stream=None) -> None:
    _check(lib.exm_shade_fwd_batch(_requests(reqs), len(reqs), C.byref(p), _ptr(ws), ws.numel(), _stream(stream)),
           "exm_shade_fwd_batch")


def exm_shade_fwd_noalloc(mesh, bvh: Bvh, mat: exm_material, env: exm_env, cams, tri_id, bary, p: exm_params, L_dir,
                          vis, stream=None) -> None:
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(L_dir, torch.float32, (n, H, W, 3), "L_dir")
    _need(vis, torch.uint64, (n, H, W), "vis")
    _check(lib.exm_shade_fwd_noalloc(C.byref(mesh), bvh.handle, C.byref(mat), C.byref(env), cams, n, _ptr(tri_id),
                                     _ptr(bary), C.byref(p), _ptr(L_dir), _ptr(vis), _stream(stream)),
           "exm_shade_fwd_noalloc")


def exm_trace_indirect_workspace_size(nViews: int, H: int, W: int, N_b: int, N_s: int) -> int:
    return int(lib.exm_trace_indirect_workspace_size(nViews, H, W, N_b, N_s))


def exm_trace_indirect_workspace_min(N_b: int, N_s: int) -> int:
    return int(lib.exm_trace_indirect_workspace_min(N_b, N_s))


def exm_trace_indirect(mesh, bvh: Bvh, mat, env, cams, tri_id, bary, p: exm_params, L_ind, sec_rec, sec_vis, ws,
                       stream=None) -> None:
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(L_ind, torch.float32, (n, H, W, 3), "L_ind")
    _need(sec_rec, torch.int32, (n, H, W, max(p.N_b, 1), 3), "sec_rec")
    _need(sec_vis, torch.uint64, (n, H, W), "sec_vis")
    _check(lib.exm_trace_indirect(C.byref(mesh), bvh.handle, C.byref(mat), C.byref(env), cams, n, _ptr(tri_id),
                                  _ptr(bary), C.byref(p), _ptr(L_ind), _ptr(sec_rec), _ptr(sec_vis), _ptr(ws),
                                  ws.numel(), _stream(stream)), "exm_trace_indirect")


def exm_shade_fwd_counted(mesh, bvh: Bvh, mat, env, cams, tri_id, bary, p: exm_params, L_dir, vis, ws, counters,
                          stream=None) -> None:
    import torch
    _need(counters, torch.uint64, (4,), "counters")
    _check(lib.exm_shade_fwd_counted(C.byref(mesh), bvh.handle, C.byref(mat), C.byref(env), cams, len(cams),
                                     _ptr(tri_id), _ptr(bary), C.byref(p), _ptr(L_dir), _ptr(vis), _ptr(ws),
                                     ws.numel(), _ptr(counters), _stream(stream)), "exm_shade_fwd_counted")


def exm_trace_indirect_counted(mesh, bvh: Bvh, mat, env, cams, tri_id, bary, p: exm_params, L_ind, sec_rec,
                               sec_vis, ws, counters, stream=None) -> None:
    import torch
    _need(counters, torch.uint64, (6,), "counters")
    _check(lib.exm_trace_indirect_counted(C.byref(mesh), bvh.handle, C.byref(mat), C.byref(env), cams, len(cams),
                                          _ptr(tri_id), _ptr(bary), C.byref(p), _ptr(L_ind), _ptr(sec_rec),
                                          _ptr(sec_vis), _ptr(ws), ws.numel(), _ptr(counters), _stream(stream)),
           "exm_trace_indirect_counted")


def exm_shade_bwd_workspace_size(nViews: int, H: int, W: int, N_d: int, He: int, We: int) -> int:
    return int(lib.exm_shade_bwd_workspace_size(nViews, H, W, N_d, He, We))


def exm_shade_bwd_workspace_min(N_d: int, He: int, We: int) -> int:
    return int(lib.exm_shade_bwd_workspace_min(N_d, He, We))


def exm_trace_bwd_workspace_size(nViews: int, H: int, W: int, N_b: int, N_s: int, He: int, We: int) -> int:
    return int(lib.exm_trace_bwd_workspace_size(nViews, H, W, N_b, N_s, He, We))


def exm_trace_bwd_workspace_min(N_b: int, N_s: int, He: int, We: int) -> int:
    return int(lib.exm_trace_bwd_workspace_min(N_b, N_s, He, We))


def exm_shade_bwd(mesh, mat, env, cams, tri_id, bary, p: exm_params, dI, vis, dtex, denv, ws,
                  stream=None, dquery=None) -> None:
    """dquery: optional [n,H,W,8] gradient with respect to the queried map values."""
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(dI, torch.float32, (n, H, W, 3), "dI")
    _need(dtex, torch.float32, (mat.Ht, mat.Wt, 8), "dtex")
    _need(denv, torch.float64, (env.He, env.We, 3), "denv")
    if dquery is not None:
        _need(dquery, torch.float32, (n, H, W, 8), "dquery")
    _check(lib.exm_shade_bwd(C.byref(mesh), C.byref(mat), C.byref(env), cams, n, _ptr(tri_id), _ptr(bary),
                             C.byref(p), _ptr(dI), _ptr(vis), _ptr(dquery), _ptr(dtex), _ptr(denv), _ptr(ws),
                             ws.numel(), _stream(stream)), "exm_shade_bwd")


def exm_trace_bwd(mesh, mat, env, cams, tri_id, bary, p: exm_params, lambda_ind: float, dI, sec_rec, sec_vis,
                  dtex, denv, ws, stream=None) -> None:
    import torch
    n, H, W = len(cams), cams[0].H, cams[0].W
    _need(dI, torch.float32, (n, H, W, 3), "dI")
    _need(dtex, torch.float32, (mat.Ht, mat.Wt, 8), "dtex")
    _need(denv, torch.float64, (env.He, env.We, 3), "denv")
    _check(lib.exm_trace_bwd(C.byref(mesh), C.byref(mat), C.byref(env), cams, n, _ptr(tri_id), _ptr(bary),
                             C.byref(p), float(lambda_ind), _ptr(dI), _ptr(sec_rec), _ptr(sec_vis), _ptr(dtex),
                             _ptr(denv), _ptr(ws), ws.numel(), _stream(stream)), "exm_trace_bwd")


def exm_timing_enable(on: bool) -> None:
    _check(lib.exm_timing_enable(1 if on else 0), "exm_timing_enable")


def exm_timing_collect() -> dict:
    """{kernel name: (total ms, launches)} of the launches recorded since timing was enabled."""
    _check(lib.exm_timing_collect(), "exm_timing_collect")
    return {lib.exm_timing_name(i).decode(): (float(lib.exm_timing_total_ms(i)), int(lib.exm_timing_launches(i)))
            for i in range(lib.exm_timing_count())}


def exm_upsample_indirect(tri_id_half, L_half, tri_id, L_ind, stream=None) -> None:
    import torch
    n, Hh, Wh = tri_id_half.shape
    _, H, W = tri_id.shape
    _need(tri_id_half, torch.int32, (n, Hh, Wh), "tri_id_half")
    _need(L_half, torch.float32, (n, Hh, Wh, 3), "L_half")
    _need(tri_id, torch.int32, (n, H, W), "tri_id")
    _need(L_ind, torch.float32, (n, H, W, 3), "L_ind")
    _check(lib.exm_upsample_indirect(_ptr(tri_id_half), Hh, Wh, _ptr(L_half), _ptr(tri_id), H, W, n, _ptr(L_ind),
                                     _stream(stream)), "exm_upsample_indirect")


def exm_upsample_indirect_bwd(tri_id_half, tri_id, lambda_ind: float, dI, dL_half, stream=None) -> None:
    import torch
    n, Hh, Wh = tri_id_half.shape
    _, H, W = tri_id.shape
    _need(tri_id_half, torch.int32, (n, Hh, Wh), "tri_id_half")
    _need(tri_id, torch.int32, (n, H, W), "tri_id")
    _need(dI, torch.float32, (n, H, W, 3), "dI")
    _need(dL_half, torch.float32, (n, Hh, Wh, 3), "dL_half")
    _check(lib.exm_upsample_indirect_bwd(_ptr(tri_id_half), Hh, Wh, _ptr(tri_id), H, W, n, float(lambda_ind), _ptr(dI),
                                         _ptr(dL_half), _stream(stream)), "exm_upsample_indirect_bwd")


def exm_project_maps(mesh, mat: exm_material, tri_id, bary, P, stream=None) -> None:
    import torch
    n, H, W = tri_id.shape
    _need(P, torch.float32, (n, H, W, 8), "P")
    _check(lib.exm_project_maps(C.byref(mesh), C.byref(mat), n, H, W, _ptr(tri_id), _ptr(bary), _ptr(P),
                                _stream(stream)), "exm_project_maps")


def exm_project_maps_bwd(mesh, mat: exm_material, tri_id, bary, dP, dtex, stream=None) -> None:
    import torch
    n, H, W = tri_id.shape
    _need(dP, torch.float32, (n, H, W, 8), "dP")
    _need(dtex, torch.float32, (mat.Ht, mat.Wt, 8), "dtex")
    _check(lib.exm_project_maps_bwd(C.byref(mesh), C.byref(mat), n, H, W, _ptr(tri_id), _ptr(bary), _ptr(dP),
                                    _ptr(dtex), _stream(stream)), "exm_project_maps_bwd")


def exm_image_loss_workspace_size(H: int, W: int) -> int:
    return int(lib.exm_image_loss_workspace_size(H, W))


def exm_image_loss(I_hat, I, scale: float, loss, dI_hat, ws, stream=None) -> None:
    """loss: device float64 [1] (accumulated); dI_hat written."""
    import torch
    n, H, W = I_hat.shape[:3]
    for t, name in ((I_hat, "I_hat"), (I, "I"), (dI_hat, "dI_hat")):
        _need(t, torch.float32, (n, H, W, 3), name)
    _need(loss, torch.float64, (1,), "loss")
    _check(lib.exm_image_loss(_ptr(I_hat), _ptr(I), n, H, W, float(scale), _ptr(loss), _ptr(dI_hat), _ptr(ws),
                              ws.numel(), _stream(stream)), "exm_image_loss")


def exm_tv_screen(P, tri_id, metallic: bool, scale: float, loss, dP, stream=None) -> None:
    import torch
    n, H, W = tri_id.shape
    _need(P, torch.float32, (n, H, W, 8), "P")
    _need(dP, torch.float32, (n, H, W, 8), "dP")
    _need(loss, torch.float64, (1,), "loss")
    _check(lib.exm_tv_screen(_ptr(P), _ptr(tri_id), n, H, W, 1 if metallic else 0, float(scale), _ptr(loss), _ptr(dP),
                             _stream(stream)), "exm_tv_screen")


def exm_env_regularizers(E, w_tv: float, w_chroma: float, loss, dE, acc3, stream=None) -> None:
    import torch
    He, We = E.shape[:2]
    _need(E, torch.float32, (He, We, 3), "E")
    _need(dE, torch.float64, (He, We, 3), "dE")
    _need(loss, torch.float64, (1,), "loss")
    _need(acc3, torch.float64, (3,), "acc3")
    _check(lib.exm_env_regularizers(_ptr(E), He, We, float(w_tv), float(w_chroma), _ptr(loss), _ptr(dE), _ptr(acc3),
                                    _stream(stream)), "exm_env_regularizers")


def exm_adam_step(param, grad, m, v, lo, hi, lr: float, t: int, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None) -> None:
    """param/m/v float32 of the same shape; grad float32 or float64; lo/hi per trailing channel."""
    import torch
    n_chan = param.shape[-1]
    for x, name in ((m, "m"), (v, "v")):
        _need(x, torch.float32, tuple(param.shape), name)
    if tuple(grad.shape) != tuple(param.shape) or grad.dtype not in (torch.float32, torch.float64):
        raise ValueError("grad must match param in shape, float32 or float64")
    lo_a = (C.c_float * n_chan)(*[float(x) for x in lo])
    hi_a = (C.c_float * n_chan)(*[float(x) for x in hi])
    _check(lib.exm_adam_step(_ptr(param), _ptr(grad), 1 if grad.dtype == torch.float64 else 0, _ptr(m), _ptr(v),
                             param.numel(), n_chan, lo_a, hi_a, float(lr), float(beta1), float(beta2), float(eps),
                             int(t), _stream(stream)), "exm_adam_step")


def exm_vertex_grad_ema(G, grad, beta: float, stream=None) -> None:
    """Eq. 1 in place on G [nV] float32 with grad [nV,3] float32."""
    import torch
    nV = G.shape[0]
    _need(grad, torch.float32, (nV, 3), "grad")
    _check(lib.exm_vertex_grad_ema(_ptr(G), _ptr(grad), nV, float(beta), _stream(stream)), "exm_vertex_grad_ema")


def exm_face_render_counts(tri_id, nF: int, counts, stream=None) -> None:
    """counts [>= nF] int32 += per-face pixel counts of the G-buffer ids tri_id (any shape)."""
    _check(lib.exm_face_render_counts(_ptr(tri_id), tri_id.numel(), int(nF), _ptr(counts), _stream(stream)),
           "exm_face_render_counts")


def exm_topology_workspace_size(nV: int, nF: int, nUV: int, p: exm_topo_params) -> int:
    return int(lib.exm_topology_workspace_size(nV, nF, nUV, C.byref(p)))


def exm_topology_scores(m: exm_topo_mesh, p: exm_topo_params, S, K, D, area, ws, stream=None) -> None:
    _check(lib.exm_topology_scores(C.byref(m), C.byref(p), _ptr(S), _ptr(K), _ptr(D), _ptr(area), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)), "exm_topology_scores")


def exm_topology_round(m: exm_topo_mesh, c_rend, p: exm_topo_params, ws, stream=None) -> dict:
    """One round in place on the arrays of m (its counts are updated); returns the round's counts."""
    st = exm_topo_stats()
    _check(lib.exm_topology_round(C.byref(m), _ptr(c_rend) if c_rend is not None else None, C.byref(p), _ptr(ws),
                                  ws.numel() * ws.element_size(), C.byref(st), _stream(stream)),
           "exm_topology_round")
    return st.as_dict()
