"""Host emulation (float32 with fused multiply-adds) of the short series the direct pass uses for
sin(pi x) and cos(pi x) of the in-texel azimuth, x = u * 2 / W_e with u in [0, 1) and W_e >= 64
(csrc/exm_device.h, sincospi_small): within half a float ulp of 1 of the exact values over the
whole range, so a pick's direction differs from the range-reduced evaluation only by rounding."""
import numpy as np

F = np.float32


def _fma(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def sincospi_small(x):
    t = (x * F(3.14159265358979323846)).astype(np.float32)
    t2 = (t * t).astype(np.float32)
    one = np.ones_like(t2)
    s = (t * _fma(t2, _fma(t2, one * F(1.0 / 120.0), one * F(-1.0 / 6.0)), one)).astype(np.float32)
    c = _fma(t2, _fma(t2, _fma(t2, one * F(-1.0 / 720.0), one * F(1.0 / 24.0)), one * F(-0.5)), one)
    return s, c


def test_series_within_half_an_ulp_on_the_in_texel_range():
    for We in (64, 100, 512, 1024, 4096):
        u = np.linspace(0.0, 1.0, 100001, endpoint=False).astype(np.float32)
        x = (u * F(2.0 / We)).astype(np.float32)
        assert x.max() <= 1.0 / 32.0
        s, c = sincospi_small(x)
        xs = x.astype(np.float64)
        half_ulp = np.spacing(np.float32(1.0)) / 2
        assert np.abs(s - np.sin(np.pi * xs)).max() < half_ulp
        assert np.abs(c - np.cos(np.pi * xs)).max() < half_ulp
        # the direction's azimuth stays on the unit circle
        assert np.abs(s.astype(np.float64) ** 2 + c.astype(np.float64) ** 2 - 1.0).max() < 4 * half_ulp
