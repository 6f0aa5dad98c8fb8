"""Python access to the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark. The product package never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

METALLIC_OFF = 1 << 0
DIFFUSE_ONLY = 1 << 1
SPECULAR_ONLY = 1 << 2
NO_VIS = 1 << 3
NO_SECONDARY_MATERIAL = 1 << 4  # secondary hits shaded as a grey (0.5) Lambertian with n_g


def build() -> str:
    """Compile oracle.cpp with g++ (FP64, no FMA contraction, OpenMP)."""
    src = os.path.join(HERE, "oracle.cpp")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", LIB_PATH + ".tmp", src]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Mesh(C.Structure):
    _fields_ = [("nV", C.c_int32), ("nF", C.c_int32), ("nUV", C.c_int32),
                ("pos", C.c_void_p), ("tri", C.c_void_p), ("uv", C.c_void_p), ("tri_uv", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("mvp", C.c_double * 16), ("eye", C.c_double * 3), ("H", C.c_int32),
                ("W", C.c_int32), ("view_id", C.c_int32)]


class Tables(C.Structure):
    _fields_ = [("He", C.c_int32), ("We", C.c_int32), ("Q", C.c_uint64), ("cdf_row", C.c_void_p),
                ("cdf_col", C.c_void_p), ("q", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("N_d", C.c_int32), ("N_b", C.c_int32), ("N_s", C.c_int32), ("seed", C.c_uint64),
                ("iteration", C.c_uint64), ("f_diel", C.c_double), ("eps", C.c_double),
                ("tmin", C.c_double), ("flags", C.c_uint32)]


class Theta(C.Structure):
    _fields_ = [("Ht", C.c_int32), ("Wt", C.c_int32), ("tex", C.c_void_p), ("tex_dot", C.c_void_p),
                ("He", C.c_int32), ("We", C.c_int32), ("env", C.c_void_p), ("env_dot", C.c_void_p)]


class Out(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("tri_id", "bary", "L_dir", "L_ind", "dL_dir", "dL_ind", "vis", "sec_tri",
                 "sec_bary", "sec_vis", "n_shadow")]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.ora_bvh_build.restype = vp
        L.ora_bvh_build.argtypes = [vp]
        L.ora_bvh_free.argtypes = [vp]
        L.ora_render.restype = i32
        L.ora_render.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, i32]
        L.ora_trace_closest.argtypes = [vp, vp, i32, vp, vp, dbl, vp, vp, vp, vp]
        L.ora_trace_any.argtypes = [vp, vp, i32, vp, vp, dbl, vp, vp]
        L.ora_ray_margins.argtypes = [vp, vp, vp, dbl, i32, dbl, vp, vp, vp]
        L.ora_raster.argtypes = [vp, vp, vp, vp]
        L.ora_sample_rays.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, vp, vp]
        L.ora_coverage_count.argtypes = [vp, vp, vp]
        L.ora_env_tables.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.ora_env_sample.argtypes = [vp, C.c_uint64, dbl, dbl, vp, vp, vp, vp]
        L.ora_philox4x32_10.argtypes = [vp, vp, vp]
        L.ora_brdf.argtypes = [vp, dbl, dbl, vp, vp, vp, dbl, dbl, C.c_uint32, vp]
        L.ora_ggx_D.restype = dbl
        L.ora_ggx_D.argtypes = [dbl, vp, vp]
        L.ora_smith_G1.restype = dbl
        L.ora_smith_G1.argtypes = [dbl, dbl]
        L.ora_bilinear.argtypes = [i32, i32, vp, i32, dbl, dbl, vp]
        L.ora_shading_normal.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        L.ora_vertex_normals.argtypes = [vp, vp]
        L.ora_face_tangents.argtypes = [vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class OracleMesh:
    """Keeps the numpy arrays alive next to the ctypes struct; owns an oracle BVH."""

    def __init__(self, pos, tri, uv, tri_uv, with_bvh: bool = True):
        self.pos = np.ascontiguousarray(pos, dtype=np.float32)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.uv = np.ascontiguousarray(uv, dtype=np.float32)
        self.tri_uv = np.ascontiguousarray(tri_uv, dtype=np.int32)
        self.s = Mesh(self.pos.shape[0], self.tri.shape[0], self.uv.shape[0], _p(self.pos),
                      _p(self.tri), _p(self.uv), _p(self.tri_uv))
        self.bvh = lib().ora_bvh_build(C.byref(self.s)) if with_bvh else None

    def __del__(self):
        if getattr(self, "bvh", None) and _lib is not None:
            _lib.ora_bvh_free(self.bvh)
            self.bvh = None

    @property
    def ref(self):
        return C.byref(self.s)


def camera(cam, view_id: int = 0) -> Camera:
    c = Camera()
    for i, v in enumerate(np.asarray(cam.mvp, dtype=np.float64).ravel()):
        c.mvp[i] = float(v)
    for i in range(3):
        c.eye[i] = float(cam.eye[i])
    c.H, c.W, c.view_id = int(cam.H), int(cam.W), int(view_id)
    return c


def vertex_normals(m: OracleMesh) -> np.ndarray:
    out = np.zeros((m.pos.shape[0], 3))
    lib().ora_vertex_normals(m.ref, _p(out))
    return out


def face_tangents(m: OracleMesh) -> np.ndarray:
    out = np.zeros((m.tri.shape[0], 4))
    lib().ora_face_tangents(m.ref, _p(out))
    return out


def raster(m: OracleMesh, cam, view_id: int = 0):
    c = camera(cam, view_id)
    ids = np.empty(cam.H * cam.W, dtype=np.int32)
    bary = np.empty((cam.H * cam.W, 3))
    lib().ora_raster(m.ref, C.byref(c), _p(ids), _p(bary))
    return ids.reshape(cam.H, cam.W), bary.reshape(cam.H, cam.W, 3)


def coverage_count(m: OracleMesh, cam) -> np.ndarray:
    c = camera(cam)
    cnt = np.empty(cam.H * cam.W, dtype=np.int32)
    lib().ora_coverage_count(m.ref, C.byref(c), _p(cnt))
    return cnt.reshape(cam.H, cam.W)


class EnvTables:
    def __init__(self, env: np.ndarray):
        env = np.ascontiguousarray(env, dtype=np.float32)
        He, We = env.shape[:2]
        self.He, self.We = He, We
        self.q = np.empty((He, We), dtype=np.uint64)
        self.cdf_row = np.empty(He, dtype=np.uint64)
        self.cdf_col = np.empty((He, We), dtype=np.uint64)
        self.pdf = np.empty((He, We))
        self.w = np.empty((He, We))
        Q = C.c_uint64(0)
        lib().ora_env_tables(He, We, _p(env), _p(self.q), _p(self.cdf_row), _p(self.cdf_col),
                             _p(self.pdf), C.byref(Q), _p(self.w))
        self.Q = Q.value
        self.s = Tables(He, We, self.Q, _p(self.cdf_row), _p(self.cdf_col), _p(self.q))

    @property
    def ref(self):
        return C.byref(self.s)

    def sample(self, x: int, u2: float, u3: float):
        row, col = C.c_int32(), C.c_int32()
        d = np.zeros(3)
        pdf = C.c_double()
        lib().ora_env_sample(self.ref, C.c_uint64(x), u2, u3, C.byref(row), C.byref(col), _p(d),
                             C.byref(pdf))
        return row.value, col.value, d, pdf.value


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def brdf(a, r, m, n, wi, wo, f_diel=0.04, eps=1e-6, flags=0) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    n, wi, wo = (np.ascontiguousarray(x, dtype=np.float64) for x in (n, wi, wo))
    out = np.zeros(3)
    lib().ora_brdf(_p(a), float(r), float(m), _p(n), _p(wi), _p(wo), f_diel, eps, flags, _p(out))
    return out


def ggx_D(r, n, h) -> float:
    n, h = (np.ascontiguousarray(x, dtype=np.float64) for x in (n, h))
    return lib().ora_ggx_D(float(r), _p(n), _p(h))


def smith_G1(r, c) -> float:
    return lib().ora_smith_G1(float(r), float(c))


def bilinear(tex: np.ndarray, u: float, v: float) -> np.ndarray:
    tex = np.ascontiguousarray(tex, dtype=np.float64)
    Ht, Wt, Cc = tex.shape
    out = np.zeros(Cc)
    lib().ora_bilinear(Ht, Wt, _p(tex), Cc, float(u), float(v), _p(out))
    return out


def shading_normal(m: OracleMesh, vnrm, ftan, f: int, b, q):
    b = np.ascontiguousarray(b, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ng, ns = np.zeros(3), np.zeros(3)
    lib().ora_shading_normal(m.ref, _p(vnrm), _p(ftan), int(f), _p(b), _p(q), _p(ng), _p(ns))
    return ng, ns


def trace_closest(m: OracleMesh, o, d, tmin, skip=None, brute=False):
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = o.shape[0]
    hit = np.empty(n, dtype=np.int32)
    t = np.empty(n)
    b2 = np.empty((n, 2))
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
    lib().ora_trace_closest(m.ref, None if brute else m.bvh, n, _p(o), _p(d), float(tmin), _p(sk),
                            _p(hit), _p(t), _p(b2))
    return hit, t, b2


def trace_any(m: OracleMesh, o, d, tmin, skip=None, brute=False):
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = o.shape[0]
    hit = np.empty(n, dtype=np.uint8)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
    lib().ora_trace_any(m.ref, None if brute else m.bvh, n, _p(o), _p(d), float(tmin), _p(sk),
                        _p(hit))
    return hit.astype(bool)


def ray_margins(m: OracleMesh, o, d, tmin, skip, tol):
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    nh, mx, mn = C.c_int32(), C.c_double(), C.c_double()
    lib().ora_ray_margins(m.ref, _p(o), _p(d), float(tmin), int(skip), float(tol), C.byref(nh),
                          C.byref(mx), C.byref(mn))
    return nh.value, mx.value, mn.value


def sample_rays(m: OracleMesh, cam, tables: EnvTables, tex, env, pix, idx, stream: int, N_d: int = 0,
                N_b: int = 0, N_s: int = 0, seed: int = 3, iteration: int = 0, tmin: float = 0.0, flags: int = 0,
                view_id: int = 0):
    """The oracle's ray (origin, direction, cosine argument, skipped triangle) of each listed
    (pixel, sample index) of `stream`; valid = False where the ray does not exist."""
    tex = np.ascontiguousarray(tex, dtype=np.float64)
    env = np.ascontiguousarray(env, dtype=np.float64)
    th = Theta(tex.shape[0], tex.shape[1], _p(tex), None, env.shape[0], env.shape[1], _p(env), None)
    p = Params(N_d, N_b, N_s, seed, iteration, 0.04, 1e-6, tmin, flags)
    c = camera(cam, view_id)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = pix.shape[0]
    o, d, cc = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n)
    sk = np.zeros(n, dtype=np.int32)
    val = np.zeros(n, dtype=np.uint8)
    lib().ora_sample_rays(m.ref, m.bvh, C.byref(c), C.byref(th), tables.ref, C.byref(p), n, _p(pix), _p(idx),
                          int(stream), _p(o), _p(d), _p(cc), _p(sk), _p(val))
    return o, d, cc, sk, val.astype(bool)


class RenderResult(dict):
    __getattr__ = dict.__getitem__


def render(m: OracleMesh, cam, tables: EnvTables, tex: np.ndarray, env: np.ndarray, N_d: int,
           N_b: int = 0, N_s: int = 0, seed: int = 3, iteration: int = 0, tmin: float = 0.0,
           flags: int = 0, view_id: int = 0, pix=None, tex_dot=None, env_dot=None,
           f_diel: float = 0.04, eps: float = 1e-6, n_threads: int = 0, brute: bool = False):
    """Render the listed pixels (linear indices py*W+px; None = the whole view)."""
    tex = np.ascontiguousarray(tex, dtype=np.float64)
    env = np.ascontiguousarray(env, dtype=np.float64)
    tex_dot = None if tex_dot is None else np.ascontiguousarray(tex_dot, dtype=np.float64)
    env_dot = None if env_dot is None else np.ascontiguousarray(env_dot, dtype=np.float64)
    th = Theta(tex.shape[0], tex.shape[1], _p(tex), _p(tex_dot), env.shape[0], env.shape[1],
               _p(env), _p(env_dot))
    p = Params(N_d, N_b, N_s, seed, iteration, f_diel, eps, tmin, flags)
    c = camera(cam, view_id)
    pix_a = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    n = cam.H * cam.W if pix_a is None else pix_a.shape[0]
    nb = max(N_b, 1)
    r = RenderResult(
        tri_id=np.empty(n, dtype=np.int32), bary=np.empty((n, 3)), L_dir=np.empty((n, 3)),
        L_ind=np.empty((n, 3)), dL_dir=np.zeros((n, 3)), dL_ind=np.zeros((n, 3)),
        vis=np.empty(n, dtype=np.uint64), sec_tri=np.full((n, nb), -1, dtype=np.int32),
        sec_bary=np.zeros((n, nb, 2)), sec_vis=np.zeros(n, dtype=np.uint64),
        n_shadow=np.zeros(n, dtype=np.int32))
    o = Out(*[_p(r[k]) for k in ("tri_id", "bary", "L_dir", "L_ind", "dL_dir", "dL_ind", "vis",
                                 "sec_tri", "sec_bary", "sec_vis", "n_shadow")])
    rc = lib().ora_render(m.ref, None if brute else m.bvh, C.byref(c), C.byref(th), tables.ref,
                          C.byref(p), n, _p(pix_a), C.byref(o), n_threads)
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return r


# ------------------------------------------------------------------------------------------
# half-resolution indirect light brought to full resolution (Implementation Details: secondary
# rays at half resolution in both image dimensions, indirect component upsampled). The filter
# is not stated in the paper; the reading: per axis pixel x sits at u = ((x + 1/2) n_half /
# n_full) - 1/2 half-resolution pixels, bilinear over the two edge-clamped taps, only covered
# half-resolution taps count and the weights are renormalised over them; 0 for background
# pixels and pixels with no covered tap. Written out as a plain map over pixels in FP64.
# ------------------------------------------------------------------------------------------

def _up_axis(n_full: int, n_half: int):
    x = np.arange(n_full, dtype=np.float64)
    u = (x + 0.5) * n_half / n_full - 0.5
    i = np.floor(u)
    f = u - i
    i = i.astype(np.int64)
    return np.clip(i, 0, n_half - 1), np.clip(i + 1, 0, n_half - 1), 1.0 - f, f


def _up_taps(tri_half: np.ndarray, tri_full: np.ndarray):
    """Per full-resolution pixel: the 4 half-resolution tap indices and their renormalised
    weights (0 for uncovered taps; all 0 for a background pixel or no covered tap)."""
    Hh, Wh = tri_half.shape
    H, W = tri_full.shape
    y0, y1, wy0, wy1 = _up_axis(H, Hh)
    x0, x1, wx0, wx1 = _up_axis(W, Wh)
    idx, wts = [], []
    for ty, wy in ((y0, wy0), (y1, wy1)):
        for tx, wx in ((x0, wx0), (x1, wx1)):
            k = ty[:, None] * Wh + tx[None, :]
            w = wy[:, None] * wx[None, :]
            w = np.where(tri_half.reshape(-1)[k] >= 0, w, 0.0)
            idx.append(k)
            wts.append(w)
    idx = np.stack(idx, -1)
    wts = np.stack(wts, -1)
    s = wts.sum(-1, keepdims=True)
    ok = (s > 0) & (tri_full[..., None] >= 0)
    wts = np.where(ok, wts / np.where(s > 0, s, 1.0), 0.0)
    return idx, wts


def upsample_indirect(L_half: np.ndarray, tri_half: np.ndarray, tri_full: np.ndarray) -> np.ndarray:
    """[Hh,Wh,3] -> [H,W,3] for one view."""
    idx, wts = _up_taps(tri_half, tri_full)
    Lh = np.asarray(L_half, np.float64).reshape(-1, 3)
    return np.einsum("hwk,hwkc->hwc", wts, Lh[idx])


def upsample_indirect_T(G_full: np.ndarray, tri_half: np.ndarray, tri_full: np.ndarray) -> np.ndarray:
    """The transpose of upsample_indirect: [H,W,3] -> [Hh,Wh,3] for one view."""
    idx, wts = _up_taps(tri_half, tri_full)
    out = np.zeros((tri_half.size, 3))
    G = np.asarray(G_full, np.float64)
    for k in range(4):
        np.add.at(out, idx[..., k].reshape(-1), wts[..., k].reshape(-1, 1) * G.reshape(-1, 3))
    return out.reshape(tri_half.shape + (3,))
