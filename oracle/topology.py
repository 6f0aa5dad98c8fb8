"""FP64 reference of the Stage-I topology operations (Vertex Splitting, Vertex Merging, UV
Maintenance; Eq. 1-6).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path; it shares no code with
the HIP library. Plain numpy and Python loops over faces, in the order the paper describes:
one round evaluates every criterion on the mesh as it stands at the start of the round, then
takes the selected splits one by one in score order and the merge candidates one by one, each
skipped when a face it would modify was already modified in the round, and finally compacts
the vertex and UV lists.

Readings of what the paper leaves open (the HIP kernels take the same ones):
  * Eq. 1 is evaluated in FP64 from the float EMA and the float gradient, rounded to float.
  * Face normals, areas and edge lengths in FP64 from the float positions:
    c = (p1 - p0) x (p2 - p0), area = |c| / 2, n = c / |c|. The neighbours N(f) of Eq. 2 are the
    other faces of f's manifold edges (an edge with exactly two faces), once per edge; a face
    with none has K_f = 0. arccos takes the dot product clamped to [-1, 1].
  * G_f = the mean of the three vertex EMAs; S_f = w_g G_f + w_k K_f (Eq. 3).
  * "Relatively large" / "relatively small" faces: area >= / < the mean face area.
  * A splitting round takes the K best-scoring large faces (ties to the lower face index),
    K = min(floor(split_fraction * nF), floor((max_faces - nF) / 2)), so that the face count
    stays within the maximum even if every split is interior.
  * Edge score ties go to the first edge of the face (edge k joins corners k and k+1). The
    new vertex lies at v_a + mu (v_b - v_a) with mu the mean of the projections of v_c and v_d
    onto the edge, mu = ((v_c - v_a).e / e.e + (v_d - v_a).e / e.e) / 2 (for mu >= 0 the paper's
    |v_s - v_a| / |v_b - v_a|; the sign keeps a point beyond v_a from passing the test); a
    boundary edge takes mu = 1/2. A split with mu outside [0.25, 0.75], or on an edge with more
    than two faces, is discarded before the conflict test.
  * New faces keep the orientation of the face they replace: f = (a, b, c) with a->b the split
    edge becomes (a, s, c) in f's slot and (s, b, c) appended; the neighbour (b, a, d) becomes
    (b, s, d) in its slot and (s, a, d) appended. New vertices, faces and UVs are numbered in the
    order the splits are taken. The new vertex's EMA is (1 - mu) G_a + mu G_b.
  * UV seams (Eq. 5-6): tau_uv = half a texel of a 2048^2 map; one shared UV is the mean of the
    two candidates.
  * Merge candidates are taken in ascending D_f, ties to the lower face index. With several
    boundary edges the shortest is collapsed; length ties go to the first edge. Equal degrees
    remove the endpoint with the larger index. v_s keeps its position, and every corner keeps
    its UV index (a merge moves no UV coordinate). The faces a merge modifies are all faces
    incident to v_r; the splits of the same round count as modifications.
  * After the round, vertices and UVs no longer referenced by any face are dropped; the rest keep
    their relative order, and faces keep their order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class TopoParams:
    beta_g: float = 0.95          # EMA coefficient (hyperparameter table)
    w_g: float = 0.6              # split-score weights
    w_k: float = 0.4
    tau_degen: float = 0.05       # degeneracy threshold
    tau_uv: float = 0.5 / 2048.0  # seam threshold in UV units
    max_faces: int = 200_000
    split_fraction: float = 0.05
    do_split: bool = True
    do_merge: bool = True


def grad_ema(G: np.ndarray, grad: np.ndarray, beta: float) -> np.ndarray:
    """Eq. 1 for every vertex: beta G + (1 - beta) |grad|."""
    g = np.asarray(grad, np.float64)
    norm = np.sqrt((g[:, 0] * g[:, 0] + g[:, 1] * g[:, 1]) + g[:, 2] * g[:, 2])
    return (beta * np.asarray(G, np.float64) + (1.0 - beta) * norm).astype(np.float32)


def edge_faces(tri: np.ndarray) -> dict:
    """{(min, max) vertex pair: [faces in index order]} over the face edges k = (v_k, v_k+1)."""
    ef: dict = {}
    for f in range(tri.shape[0]):
        for k in range(3):
            a, b = int(tri[f, k]), int(tri[f, (k + 1) % 3])
            ef.setdefault((min(a, b), max(a, b)), []).append(f)
    return ef


def degrees(nV: int, ef: dict) -> np.ndarray:
    deg = np.zeros(nV, np.int64)
    for a, b in ef:
        deg[a] += 1
        deg[b] += 1
    return deg


def _p(pos, v):
    return [float(pos[v, 0]), float(pos[v, 1]), float(pos[v, 2])]


def _sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def _edge_start(t, x, y):
    """Corner j of face t with (t[j], t[j+1]) = (x, y), or None."""
    for j in range(3):
        if int(t[j]) == x and int(t[(j + 1) % 3]) == y:
            return j
    return None


def face_geometry(pos: np.ndarray, tri: np.ndarray):
    """Per face: unit normal [nF,3], area, edge lengths [nF,3] (edge k = corners k, k+1), D_f."""
    nF = tri.shape[0]
    n = np.zeros((nF, 3))
    area = np.zeros(nF)
    ell = np.zeros((nF, 3))
    D = np.zeros(nF)
    for f in range(nF):
        p = [_p(pos, int(tri[f, k])) for k in range(3)]
        e1, e2 = _sub(p[1], p[0]), _sub(p[2], p[0])
        c = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
        ln = math.sqrt(_dot(c, c))
        area[f] = 0.5 * ln
        if ln > 0.0:
            n[f] = [c[0] / ln, c[1] / ln, c[2] / ln]
        for k in range(3):
            d = _sub(p[(k + 1) % 3], p[k])
            ell[f, k] = math.sqrt(_dot(d, d))
        lmax = max(ell[f, 0], ell[f, 1], ell[f, 2])
        D[f] = area[f] / (lmax * lmax) if lmax > 0.0 else 0.0
    return n, area, ell, D


def face_scores(pos, tri, G, prm: TopoParams, ef: dict | None = None):
    """Eq. 2-4 per face: S_f, K_f, G_f, D_f, area (all FP64)."""
    ef = edge_faces(tri) if ef is None else ef
    n, area, ell, D = face_geometry(pos, tri)
    nF = tri.shape[0]
    K = np.zeros(nF)
    Gf = np.zeros(nF)
    S = np.zeros(nF)
    for f in range(nF):
        s, cnt = 0.0, 0
        for k in range(3):
            a, b = int(tri[f, k]), int(tri[f, (k + 1) % 3])
            fs = ef[(min(a, b), max(a, b))]
            if len(fs) != 2:
                continue
            g = fs[1] if fs[0] == f else fs[0]
            d = _dot(list(n[f]), list(n[g]))
            s += math.acos(min(1.0, max(-1.0, d)))
            cnt += 1
        K[f] = s / cnt if cnt else 0.0
        Gf[f] = ((float(G[tri[f, 0]]) + float(G[tri[f, 1]])) + float(G[tri[f, 2]])) / 3.0
        S[f] = prm.w_g * Gf[f] + prm.w_k * K[f]
    return S, K, Gf, D, area, ell


def split_count(nF: int, prm: TopoParams) -> int:
    return max(0, min(int(math.floor(prm.split_fraction * nF)), (prm.max_faces - nF) // 2))


def topology_round(pos, G, uv, tri, tri_uv, c_rend, prm: TopoParams):
    """One round of splitting then merging with UV maintenance. Returns the new
    (pos, G, uv, tri, tri_uv) and a dict of counts."""
    pos = np.asarray(pos, np.float32)
    G = np.asarray(G, np.float32)
    uv = np.asarray(uv, np.float32)
    tri = np.asarray(tri, np.int64)
    tri_uv = np.asarray(tri_uv, np.int64)
    nV, nF, nUV = pos.shape[0], tri.shape[0], uv.shape[0]
    ef = edge_faces(tri)
    deg = degrees(nV, ef)
    S, K, Gf, D, area, ell = face_scores(pos, tri, G, prm, ef)
    mean_area = float(np.sum(area)) / nF if nF else 0.0
    stats = dict(split_selected=0, split_invalid=0, split_conflict=0, splits=0, merge_candidates=0,
                 merge_conflict=0, merges=0, faces_deleted=0)
    updated = set()
    new_pos, new_G, new_uv = [], [], []
    new_tri, new_tri_uv = [], []
    tri_out = tri.copy()
    tri_uv_out = tri_uv.copy()

    # ---- vertex splitting (Eq. 3, the splitting operation, Eq. 5-6)
    if prm.do_split:
        cand = [f for f in range(nF) if area[f] >= mean_area]
        cand.sort(key=lambda f: (-S[f], f))
        sel = cand[:split_count(nF, prm)]
        stats["split_selected"] = len(sel)
        for f in sel:
            best_k, best = 0, -1.0
            for k in range(3):
                a, b = int(tri[f, k]), int(tri[f, (k + 1) % 3])
                se = ell[f, k] / ((deg[a] + deg[b]) / 2.0)
                if se > best:
                    best_k, best = k, se
            k = best_k
            a, b, c = int(tri[f, k]), int(tri[f, (k + 1) % 3]), int(tri[f, (k + 2) % 3])
            fs = ef[(min(a, b), max(a, b))]
            if len(fs) > 2:
                stats["split_invalid"] += 1
                continue
            pa, pb = _p(pos, a), _p(pos, b)
            e = _sub(pb, pa)
            ee = _dot(e, e)
            g2 = None
            if len(fs) == 2:
                g2 = fs[1] if fs[0] == f else fs[0]
                # the neighbour's corner where its copy of the edge starts: (b, a) when the two
                # faces are oriented alike, (a, b) when not
                j = _edge_start(tri[g2], b, a)
                flip = j is None
                if flip:
                    j = _edge_start(tri[g2], a, b)
                if j is None:  # a neighbour with a repeated vertex: discarded
                    stats["split_invalid"] += 1
                    continue
                d = int(tri[g2, (j + 2) % 3])
                lc = _dot(_sub(_p(pos, c), pa), e) / ee
                ld = _dot(_sub(_p(pos, d), pa), e) / ee
                mu = (lc + ld) * 0.5
            else:
                mu = 0.5
            if not (0.25 <= mu <= 0.75):
                stats["split_invalid"] += 1
                continue
            faces = [f] if g2 is None else [f, g2]
            if any(x in updated for x in faces):
                stats["split_conflict"] += 1
                continue
            updated.update(faces)
            stats["splits"] += 1
            s = nV + len(new_pos)
            new_pos.append([pa[0] + mu * e[0], pa[1] + mu * e[1], pa[2] + mu * e[2]])
            new_G.append((1.0 - mu) * float(G[a]) + mu * float(G[b]))
            ua, ub, uc = int(tri_uv[f, k]), int(tri_uv[f, (k + 1) % 3]), int(tri_uv[f, (k + 2) % 3])
            u1 = [(1.0 - mu) * float(uv[ua, q]) + mu * float(uv[ub, q]) for q in range(2)]
            if g2 is None:
                us1 = us2 = nUV + len(new_uv)
                new_uv.append(u1)
            else:
                if not flip:
                    ub2, ua2, ud2 = int(tri_uv[g2, j]), int(tri_uv[g2, (j + 1) % 3]), int(tri_uv[g2, (j + 2) % 3])
                else:
                    ua2, ub2, ud2 = int(tri_uv[g2, j]), int(tri_uv[g2, (j + 1) % 3]), int(tri_uv[g2, (j + 2) % 3])
                u2 = [(1.0 - mu) * float(uv[ua2, q]) + mu * float(uv[ub2, q]) for q in range(2)]
                dx, dy = u1[0] - u2[0], u1[1] - u2[1]
                if math.sqrt(dx * dx + dy * dy) < prm.tau_uv:
                    us1 = us2 = nUV + len(new_uv)
                    new_uv.append([(u1[0] + u2[0]) * 0.5, (u1[1] + u2[1]) * 0.5])
                else:
                    us1 = nUV + len(new_uv)
                    us2 = us1 + 1
                    new_uv.append(u1)
                    new_uv.append(u2)
            tri_out[f] = (a, s, c)
            tri_uv_out[f] = (ua, us1, uc)
            new_tri.append((s, b, c))
            new_tri_uv.append((us1, ub, uc))
            if g2 is not None:
                if not flip:  # neighbour (b, a, d)
                    tri_out[g2] = (b, s, d)
                    tri_uv_out[g2] = (ub2, us2, ud2)
                    new_tri.append((s, a, d))
                    new_tri_uv.append((us2, ua2, ud2))
                else:         # neighbour (a, b, d)
                    tri_out[g2] = (a, s, d)
                    tri_uv_out[g2] = (ua2, us2, ud2)
                    new_tri.append((s, b, d))
                    new_tri_uv.append((us2, ub2, ud2))

    # ---- vertex merging (Eq. 4, the merging operation)
    deleted = np.zeros(nF + len(new_tri), bool)
    removed_v = set()
    if prm.do_merge:
        vfaces: list = [[] for _ in range(nV)]
        for f in range(nF):
            for k in range(3):
                vfaces[int(tri[f, k])].append(f)
        cand = [f for f in range(nF) if area[f] < mean_area and (int(c_rend[f]) == 0 or D[f] < prm.tau_degen)]
        cand.sort(key=lambda f: (D[f], f))
        stats["merge_candidates"] = len(cand)
        for f in cand:
            bnd = [k for k in range(3)
                   if len(ef[(min(int(tri[f, k]), int(tri[f, (k + 1) % 3])),
                              max(int(tri[f, k]), int(tri[f, (k + 1) % 3])))]) == 1]
            ks = bnd if bnd else [0, 1, 2]
            k = ks[0]
            for kk in ks[1:]:
                if ell[f, kk] < ell[f, k]:
                    k = kk
            i, j = int(tri[f, k]), int(tri[f, (k + 1) % 3])
            if deg[i] < deg[j] or (deg[i] == deg[j] and i > j):
                r, s = i, j
            else:
                r, s = j, i
            faces = sorted(set(vfaces[r]))
            if any(x in updated for x in faces):
                stats["merge_conflict"] += 1
                continue
            updated.update(faces)
            stats["merges"] += 1
            removed_v.add(r)
            for g in faces:
                if s in (int(tri[g, 0]), int(tri[g, 1]), int(tri[g, 2])):
                    deleted[g] = True
                    stats["faces_deleted"] += 1
                else:
                    tri_out[g] = [s if int(x) == r else int(x) for x in tri[g]]

    # ---- compaction (UV maintenance after merging)
    all_pos = np.concatenate([pos, np.asarray(new_pos, np.float64).reshape(-1, 3).astype(np.float32)], 0)
    all_G = np.concatenate([G, np.asarray(new_G, np.float64).astype(np.float32)], 0)
    all_uv = np.concatenate([uv, np.asarray(new_uv, np.float64).reshape(-1, 2).astype(np.float32)], 0)
    all_tri = np.concatenate([tri_out, np.asarray(new_tri, np.int64).reshape(-1, 3)], 0)
    all_tri_uv = np.concatenate([tri_uv_out, np.asarray(new_tri_uv, np.int64).reshape(-1, 3)], 0)
    keep_f = ~deleted
    all_tri, all_tri_uv = all_tri[keep_f], all_tri_uv[keep_f]
    vref = np.zeros(all_pos.shape[0], bool)
    vref[all_tri.ravel()] = True
    uref = np.zeros(all_uv.shape[0], bool)
    uref[all_tri_uv.ravel()] = True
    vmap = np.cumsum(vref) - 1
    umap = np.cumsum(uref) - 1
    out = (all_pos[vref], all_G[vref], all_uv[uref], vmap[all_tri].astype(np.int32),
           umap[all_tri_uv].astype(np.int32))
    return out, stats
