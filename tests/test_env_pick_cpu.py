"""The column search's compact compare, emulated on the host: for a row whose column shift s is at
most 16, a probe inside key t's bucket is decided by (cdf - 1) mod 2^16 and t, both masked to s
bits. Over rows of several kinds of env maps (log-normal, nearly constant, one bright texel) the
bucketed search with that compare returns the index a full upper-bound search over the 64-bit row
CDF returns, for every key tried."""
import numpy as np


def _rows(env):
    He, We, _ = env.shape
    lum = (0.2126 * env[..., 0].astype(np.float64) + 0.7152 * env[..., 1]) + 0.0722 * env[..., 2]
    i = np.arange(He)
    om = 2 * np.pi / We * (np.cos(i * np.pi / He) - np.cos((i + 1) * np.pi / He))
    w = lum * om[:, None]
    q = np.maximum(1, np.floor(w / w.max() * 2.0**20)).astype(np.int64) if w.max() > 0 else np.ones_like(w, np.int64)
    return np.cumsum(q, axis=1)


def _shift(T, n):
    s = 0
    while ((T - 1) >> s) > n - 1:
        s += 1
    return s


def _search(cdf, key, s):
    We = len(cdf)
    g = key >> s
    g0 = min(int(np.searchsorted(cdf, g << s, side="right")), We - 1)
    g1 = min(int(np.searchsorted(cdf, (g + 1) << s, side="right")), We - 1)
    mask = (1 << s) - 1
    lo, cnt = g0, max(g1 - g0, 0)
    while cnt > 0:
        step = cnt >> 1
        c = int(cdf[lo + step])
        le = ((c - 1) & 0xFFFF & mask) < (key & mask)
        if le:
            lo += step + 1
            cnt -= step + 1
        else:
            cnt = step
    return lo


def test_sixteen_bit_compare_matches_full_search():
    rng = np.random.default_rng(11)
    envs = [np.exp(rng.normal(0, 1.0, (64, 128, 3))), 1.0 + 0.05 * rng.random((32, 64, 3))]
    bright = np.full((16, 32, 3), 1e-3)
    bright[5, 7] = 1e4
    envs.append(bright)
    tried = 0
    for env in envs:
        cdf = _rows(env)
        We = cdf.shape[1]
        for row in cdf:
            T = int(row[-1])
            s = _shift(T, We)
            if s == 0 or s > 16:
                continue
            keys = np.concatenate([rng.integers(0, T, 200), row[:50] - 1, row[:50] % T, [0, T - 1]])
            for key in keys:
                key = int(key)
                want = min(int(np.searchsorted(row, key, side="right")), We - 1)
                assert _search(row, key, s) == want, (T, s, key)
                tried += 1
    assert tried > 5000
