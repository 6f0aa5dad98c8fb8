"""Pins of the FP64 Stage-II objective reference (oracle/losses.py): identities of SSIM and of
the blur it uses, closed forms of the TV and chroma terms, and every analytic gradient against
central finite differences of the loss itself."""
import numpy as np

from oracle import losses as LO


def _fd(f, x, idx, h=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp.flat[idx] += h
    xm.flat[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_ssim_identity_and_blur_properties():
    rng = np.random.default_rng(0)
    x = rng.random((20, 23, 3))
    assert np.allclose(LO.ssim_map(x, x), 1.0, atol=1e-12)
    assert LO.image_loss(x, x) == 0.0
    # the normalised window keeps constants away from the border; the blur is its own transpose
    c = LO.blur(np.ones((30, 30, 1)))
    assert np.allclose(c[5:-5, 5:-5], 1.0, atol=1e-12) and c[0, 0, 0] < 1.0
    y = rng.random((20, 23, 3))
    assert abs(np.sum(LO.blur(x) * y) - np.sum(x * LO.blur(y))) < 1e-10
    assert abs(LO.gauss_taps().sum() - 1.0) < 1e-15


def test_image_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    a = 0.05 + 0.85 * rng.random((9, 11, 3))
    b = 0.05 + 0.85 * rng.random((9, 11, 3))
    g = LO.image_loss_grad(a, b)
    f = lambda z: LO.image_loss(z, b)  # noqa: E731
    for idx in rng.choice(a.size, 40, replace=False):
        assert abs(g.flat[idx] - _fd(f, a, idx)) < 1e-6 * max(1.0, abs(g.flat[idx])) + 1e-9


def test_tv_closed_forms_and_gradients():
    H, W = 6, 7
    tri = np.zeros((H, W), np.int32)
    P = np.zeros((H, W, 8))
    assert LO.tv_screen(P, tri, True) == 0.0
    P[..., 0] = np.arange(W)[None, :]          # a ramp in one base-colour channel
    # (W - 1) horizontal pairs per row, |d| = 1 on one of the group's 3 channels
    assert abs(LO.tv_screen(P, tri, False) - H * (W - 1) / 3 / (H * W)) < 1e-12
    tri[2, 3] = -1                              # an invisible pixel removes its pairs
    assert abs(LO.tv_screen(P, tri, False) - (H * (W - 1) - 2) / 3 / (H * W)) < 1e-12
    rng = np.random.default_rng(2)
    P = rng.random((H, W, 8))
    for metallic in (False, True):
        g = LO.tv_screen_grad(P, tri, metallic)
        f = lambda z: LO.tv_screen(z, tri, metallic)  # noqa: E731
        for idx in rng.choice(P.size, 30, replace=False):
            assert abs(g.flat[idx] - _fd(f, P, idx)) < 1e-7
        if not metallic:
            assert np.all(g[..., 4] == 0.0)


def test_env_tv_and_chroma():
    rng = np.random.default_rng(3)
    E = rng.random((5, 8, 3))
    # phi wraps: a map constant in theta and periodic in phi with one jump of 1 between the
    # last and the first column has TV 1 per row
    Z = np.zeros((5, 8, 3))
    Z[:, -1, :] = 1.0
    assert abs(LO.tv_env(Z) - 2 * 5 / 40) < 1e-12  # jumps (6,7) and (7,0) in every row
    g = LO.tv_env_grad(E)
    for idx in rng.choice(E.size, 30, replace=False):
        assert abs(g.flat[idx] - _fd(LO.tv_env, E, idx)) < 1e-7
    grey = np.ones((4, 6, 3)) * rng.random((4, 6, 1))
    assert LO.chroma(grey) < 1e-30
    cast = np.zeros((4, 6, 3))
    cast[..., 0] = 3.0                          # E_bar = (3, 0, 0), mu = 1
    assert abs(LO.chroma(cast) - (4 + 1 + 1)) < 1e-12
    g = LO.chroma_grad(E)
    for idx in rng.choice(E.size, 30, replace=False):
        assert abs(g.flat[idx] - _fd(LO.chroma, E, idx)) < 1e-8
