"""FP64 reference of the Stage-II objective (Stage-II Optimization, Eq. 21-24).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path; it shares no code with
the HIP library. Plain numpy, one definition per function, written in the paper's terms.

Readings of what the paper leaves open (the HIP kernels take the same ones):
  * L_img = lambda_log * mean |log(1 + I_hat) - log(1 + I)| + lambda_ssim * (1 - mean SSIM) with
    lambda_ssim = 0.2 (hyperparameter table) and lambda_log = 1 - lambda_ssim; the means run over
    pixels and channels of the view.
  * Gamma = the sRGB transfer curve applied to the radiance clamped to [0, 1].
  * SSIM (Wang et al. 2004) per channel with an 11-tap Gaussian window (sigma 1.5, weights
    normalised), zero padding outside the image, C1 = 0.01^2, C2 = 0.03^2.
  * TV(P_hat) over the screen projection of a map group P (the bilinear query of Eq. 10 at each
    visible pixel): sum over right and down neighbour pairs whose two pixels are visible of the
    channel-mean |difference|, divided by the view's pixel count; L_mat sums it over the groups
    A (3 channels), R (1), N (3) and M (1, only when metallic is optimised).
  * TV(E): the same over the env texels, with the pair (i, We-1) - (i, 0) included (phi wraps),
    divided by He * We.
  * Chroma: E_bar = plain mean of E over texels per channel, mu = mean of E_bar,
    L = sum_c (E_bar_c - mu)^2; lambda_chroma(t) = lambda_0 (1 - t / T).
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA_SSIM = 0.2
LAMBDA_LOG = 1.0 - LAMBDA_SSIM
GROUPS = ((0, 3), (3, 4), (5, 8), (4, 5))  # A, R, N, M channel ranges of the packed map


def gauss_taps(n: int = 11, sigma: float = 1.5) -> np.ndarray:
    x = np.arange(n, dtype=np.float64) - (n - 1) / 2
    g = np.exp(-x * x / (2 * sigma * sigma))
    return g / g.sum()


def srgb(v: np.ndarray) -> np.ndarray:
    v = np.clip(v, 0.0, 1.0)
    return np.where(v <= 0.0031308, 12.92 * v, 1.055 * np.power(v, 1 / 2.4) - 0.055)


def srgb_d(v: np.ndarray) -> np.ndarray:
    """d Gamma / dv (0 where the clamp is active)."""
    inside = (v > 0.0) & (v < 1.0)
    vv = np.clip(v, 1e-30, 1.0)
    d = np.where(vv <= 0.0031308, 12.92, 1.055 / 2.4 * np.power(vv, 1 / 2.4 - 1))
    return np.where(inside, d, 0.0)


def blur(x: np.ndarray) -> np.ndarray:
    """Separable Gaussian over the first two axes of [H,W,...], zero padding."""
    g = gauss_taps()
    r = len(g) // 2
    H, W = x.shape[:2]
    out = np.zeros_like(x, dtype=np.float64)
    for k in range(len(g)):
        d = k - r
        lo, hi = max(0, -d), min(W, W - d)
        out[:, lo:hi] += g[k] * x[:, lo + d:hi + d]
    out2 = np.zeros_like(out)
    for k in range(len(g)):
        d = k - r
        lo, hi = max(0, -d), min(H, H - d)
        out2[lo:hi] += g[k] * out[lo + d:hi + d]
    return out2


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def image_loss(I_hat: np.ndarray, I: np.ndarray) -> float:
    """L_img of one view [H,W,3]."""
    a = np.asarray(I_hat, np.float64)
    b = np.asarray(I, np.float64)
    l1 = np.mean(np.abs(np.log1p(a) - np.log1p(b)))
    s = np.mean(ssim_map(srgb(a), srgb(b)))
    return float(LAMBDA_LOG * l1 + LAMBDA_SSIM * (1.0 - s))


def image_loss_grad(I_hat: np.ndarray, I: np.ndarray) -> np.ndarray:
    """dL_img / dI_hat, from the derivatives of SSIM with respect to the local moments
    (mu_x, E[x^2], E[xy]) pulled back through the blur (its own transpose) and the curve."""
    a = np.asarray(I_hat, np.float64)
    b = np.asarray(I, np.float64)
    n = a.size
    d = np.log1p(a) - np.log1p(b)
    g = LAMBDA_LOG * np.sign(d) / (1.0 + a) / n
    x, y = srgb(a), srgb(b)
    mx, my = blur(x), blur(y)
    sxx = blur(x * x) - mx * mx
    syy = blur(y * y) - my * my
    sxy = blur(x * y) - mx * my
    a1, a2 = 2 * mx * my + C1, 2 * sxy + C2
    b1, b2 = mx * mx + my * my + C1, sxx + syy + C2
    S = a1 * a2 / (b1 * b2)
    dm1 = 2 * my * (a2 - a1) / (b1 * b2) - 2 * mx * S * (b2 - b1) / (b1 * b2)
    dm2 = -S / b2
    dm3 = 2 * a1 / (b1 * b2)
    dx = (blur(dm1) + 2 * x * blur(dm2) + y * blur(dm3)) / n
    return g - LAMBDA_SSIM * dx * srgb_d(a)


def project_maps(tri_id: np.ndarray, taps: np.ndarray, weights: np.ndarray, tex: np.ndarray) -> np.ndarray:
    """Screen projection of the packed map: [H,W,8] bilinear queries at visible pixels (taps
    [H,W,4] texel indices and weights [H,W,4] of Eq. 10), 0 elsewhere."""
    t = np.asarray(tex, np.float64).reshape(-1, 8)
    P = np.einsum("hwk,hwkc->hwc", weights, t[taps])
    return np.where((tri_id >= 0)[..., None], P, 0.0)


def tv_screen(P: np.ndarray, tri_id: np.ndarray, metallic: bool) -> float:
    H, W = tri_id.shape
    vis = tri_id >= 0
    tot = 0.0
    groups = GROUPS if metallic else GROUPS[:3]
    for a, b in groups:
        dh = np.abs(P[:, 1:, a:b] - P[:, :-1, a:b]).mean(-1) * (vis[:, 1:] & vis[:, :-1])
        dv = np.abs(P[1:, :, a:b] - P[:-1, :, a:b]).mean(-1) * (vis[1:, :] & vis[:-1, :])
        tot += dh.sum() + dv.sum()
    return float(tot / (H * W))


def tv_screen_grad(P: np.ndarray, tri_id: np.ndarray, metallic: bool) -> np.ndarray:
    H, W = tri_id.shape
    vis = tri_id >= 0
    G = np.zeros_like(P, dtype=np.float64)
    groups = GROUPS if metallic else GROUPS[:3]
    for a, b in groups:
        w = 1.0 / ((b - a) * H * W)
        sh = np.sign(P[:, 1:, a:b] - P[:, :-1, a:b]) * (vis[:, 1:] & vis[:, :-1])[..., None] * w
        sv = np.sign(P[1:, :, a:b] - P[:-1, :, a:b]) * (vis[1:, :] & vis[:-1, :])[..., None] * w
        G[:, 1:, a:b] += sh
        G[:, :-1, a:b] -= sh
        G[1:, :, a:b] += sv
        G[:-1, :, a:b] -= sv
    return G


def tv_env(E: np.ndarray) -> float:
    E = np.asarray(E, np.float64)
    He, We = E.shape[:2]
    dh = np.abs(np.roll(E, -1, axis=1) - E).mean(-1).sum()
    dv = np.abs(E[1:] - E[:-1]).mean(-1).sum()
    return float((dh + dv) / (He * We))


def tv_env_grad(E: np.ndarray) -> np.ndarray:
    E = np.asarray(E, np.float64)
    He, We = E.shape[:2]
    w = 1.0 / (3 * He * We)
    sh = np.sign(np.roll(E, -1, axis=1) - E) * w  # pair (j, j+1): d/dE_{j+1} = +s, d/dE_j = -s
    G = np.roll(sh, 1, axis=1) - sh
    sv = np.sign(E[1:] - E[:-1]) * w
    G[1:] += sv
    G[:-1] -= sv
    return G


def chroma(E: np.ndarray) -> float:
    Eb = np.asarray(E, np.float64).reshape(-1, 3).mean(0)
    return float(np.sum((Eb - Eb.mean()) ** 2))


def chroma_grad(E: np.ndarray) -> np.ndarray:
    E = np.asarray(E, np.float64)
    Eb = E.reshape(-1, 3).mean(0)
    n = E.shape[0] * E.shape[1]
    return np.broadcast_to(2.0 * (Eb - Eb.mean()) / n, E.shape).copy()
