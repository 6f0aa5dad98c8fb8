"""Seeded synthetic inputs for the Stage-II render pass (meshes, UVs, maps, env, cameras).

This module only *constructs inputs*. It holds none of the render pass's arithmetic: no
normals used for shading, no tangent frames, no sampling, no BRDF. Both the HIP path and the
FP64 oracle receive exactly the arrays built here, so the two sides share nothing but inputs.

The paper's datasets (DTU, Synthetic4Relight, Stanford-ORB, NeRF-Synthetic; Experiments,
Experimental Setup) are not available; the meshes, maps and environment maps below stand in
for the fixed mesh-UV carrier and the parameters Theta = {A, R, M_met, N, E} of the
UV-PBR Asset Decomposition section, with the map and env resolutions of the hyperparameter
table where the workload names none.

Texel layout of the packed material map: [Ht, Wt, 8] float32 =
(a.r, a.g, a.b, roughness, metallic, n.x, n.y, n.z), row 0 is v in [0, 1/Ht).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Fixed seeds of the workload recipe.
SEED_MESH_NOISE = 0
SEED_MAPS = 1
SEED_ENV = 2
SEED_RNG_KEY = 3
SEED_UPSTREAM = 4
SEED_RELIGHT_ASSETS = 100   # asset i uses SEED_RELIGHT_ASSETS + i
SEED_RELIGHT_ENVS = 200     # env k uses SEED_RELIGHT_ENVS + k
SEED_RELIGHT_ARRIVALS = 300


# --------------------------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------------------------

def icosphere(subdiv: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit icosphere with welded midpoints; CCW faces seen from outside."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (min(a, b), max(a, b))
            if key not in cache:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    pos = np.array(verts, dtype=np.float64)
    tri = np.array(faces, dtype=np.int32)
    tri = _orient_outward(pos, tri, np.zeros(3))
    return pos.astype(np.float32), tri


def _orient_outward(pos: np.ndarray, tri: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """Flip faces whose (p1-p0)x(p2-p0) points toward `centre` (star-shaped meshes only)."""
    p0, p1, p2 = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    ctr = (p0 + p1 + p2) / 3.0 - centre
    flip = np.einsum("ij,ij->i", nrm, ctr) < 0
    out = tri.copy()
    out[flip, 1], out[flip, 2] = tri[flip, 2], tri[flip, 1]
    return out


class ValueNoise:
    """Periodic 3-D value noise: a seeded 64^3 lattice of U[-1,1] values, trilinear
    interpolation with the 3t^2 - 2t^3 fade, sampled at frequency `freq`."""

    def __init__(self, seed: int, freq: float = 4.0, period: int = 64):
        rng = np.random.default_rng(seed)
        self.lat = rng.uniform(-1.0, 1.0, size=(period, period, period))
        self.freq = freq
        self.period = period

    def __call__(self, p: np.ndarray) -> np.ndarray:
        q = np.asarray(p, dtype=np.float64) * self.freq
        i0 = np.floor(q).astype(np.int64)
        f = q - i0
        w = f * f * (3.0 - 2.0 * f)
        n = self.period
        out = np.zeros(q.shape[0], dtype=np.float64)
        for dx in (0, 1):
            wx = w[:, 0] if dx else 1.0 - w[:, 0]
            for dy in (0, 1):
                wy = w[:, 1] if dy else 1.0 - w[:, 1]
                for dz in (0, 1):
                    wz = w[:, 2] if dz else 1.0 - w[:, 2]
                    v = self.lat[(i0[:, 0] + dx) % n, (i0[:, 1] + dy) % n, (i0[:, 2] + dz) % n]
                    out += wx * wy * wz * v
        return out


def displaced_cube_sphere(n: int = 129, amp: float = 0.05, seed: int = SEED_MESH_NOISE):
    """Cube-sphere: each cube face split into n x n quads (2 triangles each), welded,
    projected to the unit sphere, radius 1 + amp * valuenoise(p)."""
    s = np.linspace(-1.0, 1.0, n + 1)
    A, B = np.meshgrid(s, s, indexing="ij")
    A, B = A.ravel(), B.ravel()
    one = np.ones_like(A)
    faces_xyz = [
        np.stack([one, A, B], 1), np.stack([-one, A, B], 1),
        np.stack([A, one, B], 1), np.stack([A, -one, B], 1),
        np.stack([A, B, one], 1), np.stack([A, B, -one], 1),
    ]
    pts = np.concatenate(faces_xyz, 0)
    # weld identical cube-surface points (edge points are computed identically on both faces)
    key = np.round(pts * (n * 4)).astype(np.int64)
    _, uniq_idx, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    base = pts[uniq_idx]
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    q00, q10 = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    q01, q11 = idx[:-1, 1:].ravel(), idx[1:, 1:].ravel()
    tris = []
    for f in range(6):
        off = f * (n + 1) * (n + 1)
        t1 = np.stack([q00, q10, q11], 1) + off
        t2 = np.stack([q00, q11, q01], 1) + off
        tris.append(np.concatenate([t1, t2], 0))
    tri = inv[np.concatenate(tris, 0)]
    dirs = base / np.linalg.norm(base, axis=1, keepdims=True)
    noise = ValueNoise(seed)
    pos = dirs * (1.0 + amp * noise(dirs))[:, None]
    tri = _orient_outward(pos, tri.astype(np.int32), np.zeros(3))
    return pos.astype(np.float32), tri.astype(np.int32)


def torus(centre, axis: str, n_major: int, n_minor: int, R: float = 1.0, r: float = 0.3,
          amp: float = 0.02, noise: ValueNoise | None = None):
    """Torus around `axis` ('y' or 'z') through `centre`, n_major x n_minor quads,
    displaced along the tube normal by amp * valuenoise(p). CCW seen from outside."""
    u = 2.0 * np.pi * np.arange(n_major) / n_major
    v = 2.0 * np.pi * np.arange(n_minor) / n_minor
    U, Vv = np.meshgrid(u, v, indexing="ij")
    U, Vv = U.ravel(), Vv.ravel()
    if axis == "z":
        e1, e2, ax = np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])
    elif axis == "y":
        e1, e2, ax = np.array([0, 0, 1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    else:
        raise ValueError(axis)
    radial = np.cos(U)[:, None] * e1 + np.sin(U)[:, None] * e2
    tube_n = np.cos(Vv)[:, None] * radial + np.sin(Vv)[:, None] * ax
    p0 = np.asarray(centre, dtype=np.float64) + R * radial + r * tube_n
    d = amp * noise(p0) if noise is not None else 0.0
    pos = p0 + (d * tube_n.T).T if noise is not None else p0
    i = np.arange(n_major)[:, None]
    j = np.arange(n_minor)[None, :]
    a = (i * n_minor + j).ravel()
    b = (((i + 1) % n_major) * n_minor + j).ravel()
    c = (((i + 1) % n_major) * n_minor + (j + 1) % n_minor).ravel()
    dd = (i * n_minor + (j + 1) % n_minor).ravel()
    tri = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, dd], 1)], 0).astype(np.int32)
    # orient outward from the tube centre line
    p_0, p_1, p_2 = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    nrm = np.cross(p_1 - p_0, p_2 - p_0)
    ring = np.asarray(centre) + R * radial[tri[:, 0]]
    inward = np.einsum("ij,ij->i", nrm, (p_0 + p_1 + p_2) / 3.0 - ring) < 0
    tri[inward, 1], tri[inward, 2] = tri[inward, 2].copy(), tri[inward, 1].copy()
    return pos, tri


def interlocking_tori(n_major: int = 1000, n_minor: int = 250, seed: int = SEED_MESH_NOISE):
    """Two interlocking tori (major 1, minor 0.3): A at (-0.5,0,0) around Z, B at (+0.5,0,0)
    around Y; 2 * n_major * n_minor * 2 triangles."""
    noise = ValueNoise(seed)
    pa, ta = torus((-0.5, 0.0, 0.0), "z", n_major, n_minor, noise=noise)
    pb, tb = torus((0.5, 0.0, 0.0), "y", n_major, n_minor, noise=noise)
    pos = np.concatenate([pa, pb], 0)
    tri = np.concatenate([ta, tb + pa.shape[0]], 0)
    return pos.astype(np.float32), tri.astype(np.int32)


def quad_mesh(corners: np.ndarray, nx: int = 1, ny: int = 1):
    """Planar grid between 4 corners (c0,c1,c2,c3 counter-clockwise), nx x ny quads."""
    c = np.asarray(corners, dtype=np.float64)
    s = np.linspace(0, 1, nx + 1)
    t = np.linspace(0, 1, ny + 1)
    S, T = np.meshgrid(s, t, indexing="ij")
    S, T = S.ravel()[:, None], T.ravel()[:, None]
    pos = (1 - S) * (1 - T) * c[0] + S * (1 - T) * c[1] + S * T * c[2] + (1 - S) * T * c[3]
    idx = np.arange((nx + 1) * (ny + 1)).reshape(nx + 1, ny + 1)
    a, b = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    cc, d = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    tri = np.concatenate([np.stack([a, b, cc], 1), np.stack([a, cc, d], 1)], 0)
    return pos.astype(np.float32), tri.astype(np.int32)


def cube_projected_uvs(pos: np.ndarray, tri: np.ndarray, inset: float = 0.01):
    """Cube-projected UV atlas: per face, axis k = argmax |n_f| (ties to the lower axis),
    cell = 2k + (n_f[k] < 0) of a 3 x 2 atlas; corner UV = orthographic projection onto the
    two other axes, normalised by the mesh AABB, placed inside the cell with an inset.
    Every face owns its 3 UV entries (nUV = 3 nF)."""
    p = pos.astype(np.float64)
    p0, p1, p2 = p[tri[:, 0]], p[tri[:, 1]], p[tri[:, 2]]
    nf = np.cross(p1 - p0, p2 - p0)
    k = np.argmax(np.abs(nf), axis=1)  # argmax returns the first maximum -> lower axis
    neg = nf[np.arange(len(k)), k] < 0
    cell = 2 * k + neg.astype(np.int64)
    lo, hi = p.min(0), p.max(0)
    ext = np.maximum(hi - lo, 1e-12)
    others = np.array([[1, 2], [0, 2], [0, 1]])[k]  # (nF, 2)
    cu, cv = (cell % 3).astype(np.float64), (cell // 3).astype(np.float64)
    cw, ch = 1.0 / 3.0, 1.0 / 2.0
    uv = np.zeros((tri.shape[0], 3, 2), dtype=np.float64)
    rows = np.arange(tri.shape[0])
    for c, pc in enumerate((p0, p1, p2)):
        a = (pc[rows, others[:, 0]] - lo[others[:, 0]]) / ext[others[:, 0]]
        b = (pc[rows, others[:, 1]] - lo[others[:, 1]]) / ext[others[:, 1]]
        uv[:, c, 0] = (cu + inset + a * (1 - 2 * inset)) * cw
        uv[:, c, 1] = (cv + inset + b * (1 - 2 * inset)) * ch
    tri_uv = np.arange(3 * tri.shape[0], dtype=np.int32).reshape(-1, 3)
    return uv.reshape(-1, 2).astype(np.float32), tri_uv


# --------------------------------------------------------------------------------------------
# maps, env, cameras, upstream gradients
# --------------------------------------------------------------------------------------------

def pbr_maps(Ht: int, Wt: int, seed: int = SEED_MAPS, chunk_rows: int = 256) -> np.ndarray:
    """Packed material map [Ht,Wt,8] f32: a ~ U[0,1]^3, r ~ U[0.1,1], m ~ U[0,1],
    n = normalize((0,0,1) + N(0, 0.1)^3), i.i.d. per texel (generated in row chunks)."""
    rng = np.random.default_rng(seed)
    tex = np.empty((Ht, Wt, 8), dtype=np.float32)
    for r0 in range(0, Ht, chunk_rows):
        r1 = min(Ht, r0 + chunk_rows)
        n = (r1 - r0) * Wt
        blk = np.empty((n, 8), dtype=np.float64)
        blk[:, 0:3] = rng.random((n, 3))
        blk[:, 3] = rng.uniform(0.1, 1.0, n)
        blk[:, 4] = rng.random(n)
        nn = np.array([0.0, 0.0, 1.0]) + rng.normal(0.0, 0.1, (n, 3))
        blk[:, 5:8] = nn / np.linalg.norm(nn, axis=1, keepdims=True)
        tex[r0:r1] = blk.reshape(r1 - r0, Wt, 8).astype(np.float32)
    return tex


def env_map(He: int, We: int, sigma: float, seed: int = SEED_ENV) -> np.ndarray:
    """Equirect env [He,We,3] f32, E = exp(N(0, sigma)) i.i.d. per texel and channel."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(0.0, sigma, (He, We, 3))).astype(np.float32)


@dataclass
class Camera:
    """OpenGL-convention camera: clip = mvp @ [p, 1] (row-major), eye in world space."""
    mvp: np.ndarray  # (4,4) float64
    eye: np.ndarray  # (3,) float64
    H: int
    W: int


def look_at(eye, target, up) -> np.ndarray:
    eye, target, up = (np.asarray(x, dtype=np.float64) for x in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3], m[1, :3], m[2, :3] = s, u, -f
    m[0, 3], m[1, 3], m[2, 3] = -s @ eye, -u @ eye, f @ eye
    return m


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = (far + near) / (near - far)
    m[2, 3] = 2.0 * far * near / (near - far)
    m[3, 2] = -1.0
    return m


def ring_cameras(n: int, radius: float, H: int, W: int, elev_deg=20.0, fovy: float = 45.0,
                 near: float = 0.1, far: float = 20.0, start: int = 0) -> list[Camera]:
    """n cameras on a ring: eye = R (cos e sin(2 pi k/n), sin e, cos e cos(2 pi k/n)),
    looking at the origin, up +Y. `elev_deg` may be a scalar or a per-view sequence."""
    cams = []
    proj = perspective(fovy, W / H, near, far)
    for k in range(start, start + n):
        e = elev_deg[k - start] if np.ndim(elev_deg) else elev_deg
        e = math.radians(e)
        az = 2.0 * math.pi * k / n
        eye = radius * np.array([math.cos(e) * math.sin(az), math.sin(e), math.cos(e) * math.cos(az)])
        mvp = proj @ look_at(eye, np.zeros(3), np.array([0.0, 1.0, 0.0]))
        cams.append(Camera(mvp=mvp, eye=eye, H=H, W=W))
    return cams


def upstream_grad(V: int, H: int, W: int, seed: int = SEED_UPSTREAM) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, (V, H, W, 3)).astype(np.float32)


def aabb_diagonal(pos: np.ndarray) -> float:
    p = pos.astype(np.float64)
    return float(np.linalg.norm(p.max(0) - p.min(0)))


# --------------------------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------------------------

@dataclass
class Scene:
    name: str
    pos: np.ndarray
    tri: np.ndarray
    uv: np.ndarray
    tri_uv: np.ndarray
    tex: np.ndarray
    env: np.ndarray
    cams: list
    N_d: int
    N_b: int = 0
    N_s: int = 0
    seed: int = SEED_RNG_KEY
    iteration: int = 0
    tmin: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def nV(self):
        return self.pos.shape[0]

    @property
    def nF(self):
        return self.tri.shape[0]


def make_scene(name: str, pos, tri, Ht, Wt, He, We, env_sigma, cams, N_d, N_b=0, N_s=0,
               tex=None, env=None) -> Scene:
    uv, tri_uv = cube_projected_uvs(pos, tri)
    tex = pbr_maps(Ht, Wt) if tex is None else tex
    env = env_map(He, We, env_sigma) if env is None else env
    return Scene(name=name, pos=pos, tri=tri, uv=uv, tri_uv=tri_uv, tex=tex, env=env, cams=cams,
                 N_d=N_d, N_b=N_b, N_s=N_s, tmin=1e-4 * aabb_diagonal(pos))


def config(name: str, views: int | None = None, res: int | None = None) -> Scene:
    """The five workloads. `views`/`res` shrink a workload for parity tests only.

    small:   icosphere subdiv 3 (1280 tris), 256^2 maps, 32x64 env exp(N(0,1)),
             1 view 128^2, 16 env samples/pixel, direct only.
    sphere:  displaced cube-sphere (199,692 tris), 2048^2 maps, 512x1024 env exp(N(0,1.5)),
             8 ring views 1024^2 (R=3), 64 env samples/pixel, direct only.
    tori:    two interlocking displaced tori (1M tris), 2048^2 maps, 512x1024 env,
             8 ring views 1024^2 (R=4.5), 64 env samples + 4 cosine secondary rays x 4 light
             samples.
    tori32:  the tori mesh, 32 ring views 1024^2 (elevations alternating +-20 deg),
             4096^2 maps, env gradients on, G-buffer recomputed in backward.
    paper_shape: cube-sphere n = 91 (99,372 tris, 49,688 vertices), 2048^2 maps, 256x512 env
             exp(N(0,1)), 1 view 1600^2 (R=3), N_d 8, N_b 16 (half resolution), N_s 4.
    """
    if name == "small":
        pos, tri = icosphere(3)
        H = W = res or 128
        cams = ring_cameras(views or 1, 3.0, H, W)
        return make_scene(name, pos, tri, 256, 256, 32, 64, 1.0, cams, N_d=16)
    if name == "sphere":
        pos, tri = displaced_cube_sphere(129)
        H = W = res or 1024
        cams = ring_cameras(views or 8, 3.0, H, W)
        return make_scene(name, pos, tri, 2048, 2048, 512, 1024, 1.5, cams, N_d=64)
    if name == "tori":
        pos, tri = interlocking_tori(1000, 250)
        H = W = res or 1024
        cams = ring_cameras(views or 8, 4.5, H, W)
        return make_scene(name, pos, tri, 2048, 2048, 512, 1024, 1.5, cams, N_d=64, N_b=4, N_s=4)
    if name == "paper_shape":
        # the paper's relighting timing shape: an object of ~100k triangles (52K vertices), one
        # 1600^2 view, 2048^2 maps, a 256x512 env map, N_d 8, N_b 16 at half resolution, N_s 4
        pos, tri = displaced_cube_sphere(91)
        H = W = res or 1600
        cams = ring_cameras(views or 1, 3.0, H, W)
        return make_scene(name, pos, tri, 2048, 2048, 256, 512, 1.0, cams, N_d=8, N_b=16, N_s=4)
    if name == "tori32":
        pos, tri = interlocking_tori(1000, 250)
        H = W = res or 1024
        n = views or 32
        elev = [20.0 if k % 2 == 0 else -20.0 for k in range(n)]
        cams = ring_cameras(n, 4.5, H, W, elev_deg=elev)
        return make_scene(name, pos, tri, 4096, 4096, 512, 1024, 1.5, cams, N_d=64, N_b=4, N_s=4)
    raise KeyError(name)


# --------------------------------------------------------------------------------------------
# relighting service: assets, env maps and a request stream
# --------------------------------------------------------------------------------------------

@dataclass
class RelightAssetSpec:
    index: int
    kind: str       # "sphere" (displaced cube-sphere) or "torus" (one displaced torus around Y)
    n_tris: int     # target triangle count (log-uniform in [10k, 2M])
    tex_res: int    # square material maps of tex_res^2 texels
    seed: int


def relight_asset_specs(n: int = 64, lo: int = 10_000, hi: int = 2_000_000,
                        sizes=(512, 1024, 2048, 4096)) -> list[RelightAssetSpec]:
    out = []
    for i in range(n):
        rng = np.random.default_rng(SEED_RELIGHT_ASSETS + i)
        kind = "sphere" if rng.random() < 0.5 else "torus"
        nt = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        res = int(sizes[int(rng.integers(len(sizes)))])
        out.append(RelightAssetSpec(i, kind, nt, res, SEED_RELIGHT_ASSETS + i))
    return out


def relight_asset_mesh(spec: RelightAssetSpec):
    """(pos, tri, uv, tri_uv) of an asset: about spec.n_tris triangles, cube-projected UVs."""
    if spec.kind == "sphere":
        n = max(2, int(round(math.sqrt(spec.n_tris / 12.0))))
        pos, tri = displaced_cube_sphere(n, seed=spec.seed)
    else:
        nm = max(3, int(round(math.sqrt(spec.n_tris / 8.0))))
        pos, tri = torus((0.0, 0.0, 0.0), "y", 4 * nm, nm, noise=ValueNoise(spec.seed))
        pos, tri = pos.astype(np.float32), tri.astype(np.int32)
    uv, tri_uv = cube_projected_uvs(pos, tri)
    return pos, tri, uv, tri_uv


def pbr_maps_device(Ht: int, Wt: int, seed: int, device="cuda"):
    """Packed material map with the distributions of pbr_maps, drawn on the device from a
    seeded torch generator (a different stream of numbers than pbr_maps' numpy generator)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = Ht * Wt
    tex = torch.empty((n, 8), dtype=torch.float32, device=device)
    tex[:, 0:3] = torch.rand((n, 3), generator=g, device=device)
    tex[:, 3] = 0.1 + 0.9 * torch.rand(n, generator=g, device=device)
    tex[:, 4] = torch.rand(n, generator=g, device=device)
    nn = torch.randn((n, 3), generator=g, device=device, dtype=torch.float64) * 0.1
    nn[:, 2] += 1.0
    tex[:, 5:8] = (nn / nn.norm(dim=1, keepdim=True)).float()
    return tex.view(Ht, Wt, 8)


def relight_envs(n: int = 16, He: int = 256, We: int = 512, sigma: float = 1.0) -> list[np.ndarray]:
    return [env_map(He, We, sigma, seed=SEED_RELIGHT_ENVS + k) for k in range(n)]


@dataclass
class RelightRequestSpec:
    rid: int
    arrival: float      # seconds after the start of the stream
    asset: int
    env: int
    res: int            # square view of res^2 pixels
    azimuth: float      # ring camera azimuth (radians), elevation 20 deg, looking at the origin
    indirect: bool      # direct + one-bounce indirect, else direct only


def relight_stream(rate: float = 200.0, seconds: float = 60.0, n_assets: int = 64, n_envs: int = 16,
                   resolutions=(256, 512, 1024, 2048), seed: int = SEED_RELIGHT_ARRIVALS) -> list[RelightRequestSpec]:
    """Poisson arrivals at `rate` per second over `seconds`; per request a uniform asset, env,
    view resolution and azimuth, direct-only or direct + indirect with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        out.append(RelightRequestSpec(len(out), t, int(rng.integers(n_assets)), int(rng.integers(n_envs)),
                                      int(resolutions[int(rng.integers(len(resolutions)))]),
                                      float(rng.uniform(0.0, 2.0 * math.pi)), bool(rng.random() < 0.5)))
    return out


def relight_camera(pos: np.ndarray, res: int, azimuth: float, elev_deg: float = 20.0) -> Camera:
    """Ring camera at 2.9 x the asset's bounding radius (a unit sphere fills ~ 60% of the view)."""
    R = 2.9 * float(np.sqrt((pos.astype(np.float64) ** 2).sum(1).max()))
    e = math.radians(elev_deg)
    eye = R * np.array([math.cos(e) * math.sin(azimuth), math.sin(e), math.cos(e) * math.cos(azimuth)])
    mvp = perspective(45.0, 1.0, 0.1, 4.0 * R) @ look_at(eye, np.zeros(3), np.array([0.0, 1.0, 0.0]))
    return Camera(mvp=mvp, eye=eye, H=res, W=res)
