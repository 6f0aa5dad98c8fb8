"""Host side of the Stage-II loop: the sRGB-to-linear initialisation of the base colour
(IEC 61966-2-1 values) and the neutral initial parameters (Stage-II initialisation)."""
import numpy as np
import pytest

pytest.importorskip("torch")

from paper_2608_24109_amd.optimize import NEUTRAL_ENV, NEUTRAL_ROUGHNESS, Stage2Config, initial_maps, srgb_to_linear


def test_srgb_to_linear_values():
    assert srgb_to_linear(0.0) == 0.0 and srgb_to_linear(1.0) == 1.0
    # the two branches meet at 0.04045 (to the rounding of the standard's constants)
    lo = 0.04045 / 12.92
    hi = ((0.04045 + 0.055) / 1.055) ** 2.4
    assert abs(lo - hi) < 1e-7
    # sRGB 0.5 is 21.4 % linear; 188/255 is about one half
    assert abs(srgb_to_linear(0.5) - 0.214041140) < 1e-8
    assert abs(srgb_to_linear(188 / 255) - 0.5029) < 1e-3
    x = np.linspace(0, 1, 101)
    assert np.all(np.diff(srgb_to_linear(x)) > 0)


def test_initial_maps():
    rgb = np.random.default_rng(0).random((4, 5, 3))
    tex, env = initial_maps(rgb, 4, 5, 2, 6)
    assert tex.shape == (4, 5, 8) and env.shape == (2, 6, 3)
    assert np.allclose(tex[..., :3], srgb_to_linear(rgb), atol=1e-7)
    assert np.all(tex[..., 3] == NEUTRAL_ROUGHNESS) and np.all(tex[..., 4] == 0.0)
    assert np.all(tex[..., 5:8] == np.array([0, 0, 1], np.float32)) and np.all(env == NEUTRAL_ENV)
    grey, _ = initial_maps(rgb, 4, 5, 2, 6, grey_base=True)
    assert np.all(grey[..., :3] == 0.5)
    with pytest.raises(ValueError):
        initial_maps(rgb, 5, 5, 2, 6)


def test_schedules():
    c = Stage2Config(iters=100, ramp_iters=10, lambda_chroma0=0.1, lambda_ind_max=1.0)
    assert c.lambda_ind(0) == 0.0 and c.lambda_ind(5) == 0.5 and c.lambda_ind(50) == 1.0
    assert c.lambda_chroma(0) == 0.1 and abs(c.lambda_chroma(50) - 0.05) < 1e-15 and c.lambda_chroma(100) == 0.0
