"""Parity helpers: run the HIP path and the FP64 oracle on the same seeded inputs and compare.

Discrete decisions that floating point can flip between an FP32 kernel and an FP64 reference
(a shadow ray grazing an edge, a cosine at zero, a secondary ray hitting next to a seam) are
compared as decisions: every disagreement must be explained by the oracle's own margins
(distance of the ray to a triangle boundary, or |cos| at the clamp). Radiance is compared
element by element on every pixel without a flipped decision."""
from __future__ import annotations

import numpy as np

import oracle as O

RAD_REL = 1e-4   # radiance: |d| <= 1e-4 |L_ref| + 1e-7 max |L_ref|
RAD_ABS = 1e-7
COS_KINK = 1e-5  # |cos| below this at a clamp explains a flip
EDGE_TOL = 1e-5  # ray within 1e-5 * AABB diagonal of a triangle boundary explains a flip


def bits_set(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    c = np.zeros(x.shape, dtype=np.int64)
    for k in range(64):
        c += ((x >> np.uint64(k)) & np.uint64(1)).astype(np.int64)
    return c


def flipped_pairs(a: np.ndarray, b: np.ndarray, nbits: int):
    """(row, bit) of every bit where the u64 arrays a and b differ."""
    if nbits <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    x = (a.astype(np.uint64) ^ b.astype(np.uint64))
    rows, ks = [], []
    for k in range(nbits):
        r = np.nonzero((x >> np.uint64(k)) & np.uint64(1))[0]
        rows.append(r)
        ks.append(np.full(r.shape, k))
    return np.concatenate(rows), np.concatenate(ks)


def explain_flips(om, cam, tab, tex, env, pix, idx, stream, gpu_bit, diag, **kw):
    """For each flipped ray, True if the oracle's margins explain it."""
    if len(pix) == 0:
        return np.zeros(0, dtype=bool)
    o, d, c, sk, valid = O.sample_rays(om, cam, tab, tex, env, pix, idx, stream, **kw)
    tol = EDGE_TOL * diag
    ok = np.zeros(len(pix), dtype=bool)
    for i in range(len(pix)):
        if not valid[i]:
            continue
        if abs(c[i]) < COS_KINK:
            ok[i] = True
            continue
        nh, mx, mn = O.ray_margins(om, o[i], d[i], kw.get("tmin", 0.0), int(sk[i]), tol)
        if gpu_bit[i]:  # GPU saw no occluder: every hit the oracle's ray has must be fragile
            ok[i] = mx < tol if nh > 0 else mn < tol
        else:           # GPU saw an occluder (or another closest hit) the oracle did not: a near miss
            ok[i] = mn < tol
    return ok


def radiance_close(gpu: np.ndarray, ref: np.ndarray, mask: np.ndarray):
    """Element-wise bound on the pixels in `mask`; returns (ok, worst excess, description)."""
    if not mask.any():
        return True, 0.0, ""
    idx = np.nonzero(mask)[0]
    g, r = gpu[mask].astype(np.float64), ref[mask]
    bound = RAD_REL * np.abs(r) + RAD_ABS * max(np.abs(ref).max(), 1e-30)
    excess = np.abs(g - r) / bound
    w = np.unravel_index(np.argmax(excess), excess.shape)
    n_over = int((excess > 1.0).sum())
    desc = (f"row {idx[w[0]]} ch {w[1]}: gpu {g[w]:.9g} ref {r[w]:.9g} rel {abs(g[w] - r[w]) / max(abs(r[w]), 1e-30):.3g}"
            f"; {n_over} of {excess.size} values over the bound; relative error quantiles "
            f"{np.quantile(np.abs(g - r) / np.maximum(np.abs(r), 1e-30), [0.5, 0.99, 0.999])}")
    return bool((excess <= 1.0).all()), float(excess.max()), desc
