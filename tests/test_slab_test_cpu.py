"""The traversal's slab test (one FMA per plane with per-axis padded offsets, reciprocals clamped to
+-2^64) emulated in float32 on the host: over random rays — a share with exactly zero or tiny
direction components — and boxes that graze them or have a face through the ray origin, it never
rejects a box the exact slab test (float64, exact reciprocal, a zero component handled as 'inside
the slab or not') accepts. A rejected box would drop every triangle under it, so conservativeness is
what the traversal's answers rest on; the extra boxes it accepts only cost node visits."""
import numpy as np


def _rn(x):
    return np.asarray(x, np.float64).astype(np.float32)


def _fma32(a, b, c):
    # a * b is exact in float64 (24 + 24 bits); one rounding of the sum to float32 after it
    return _rn(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def _fmin(a, b):  # IEEE minimum: a NaN operand yields the other
    return np.where(np.isnan(a), b, np.where(np.isnan(b), a, np.minimum(a, b)))


def _fmax(a, b):
    return np.where(np.isnan(a), b, np.where(np.isnan(b), a, np.maximum(a, b)))


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    o = _rn(rng.uniform(-3, 3, (n, 3)))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[rng.random((n, 3)) < 0.05] = 0.0
    d[rng.random((n, 3)) < 0.05] *= 1e-12
    d = _rn(d)
    d[(d == 0).all(axis=1), 0] = 1.0
    t = rng.uniform(0, 4, n)
    p = o.astype(np.float64) + t[:, None] * d.astype(np.float64)
    half = np.exp(rng.uniform(np.log(1e-7), np.log(0.5), (n, 3)))
    shift = rng.uniform(-1.05, 1.05, (n, 3)) * half
    lo, hi = _rn(p + shift - half), _rn(p + shift + half)
    m = (rng.random((n, 3)) < 0.03) & (o <= hi)
    lo[m] = o[m]
    m = (rng.random((n, 3)) < 0.03) & (o >= lo)
    hi[m] = o[m]
    return o, d, lo, hi


def _exact_hit(o, d, lo, hi):
    dd = d.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        a0 = (lo.astype(np.float64) - o) / dd
        a1 = (hi.astype(np.float64) - o) / dd
    zero = dd == 0
    inside = (lo <= o) & (o <= hi)
    a0 = np.where(zero, np.where(inside, -np.inf, np.inf), a0)
    a1 = np.where(zero, np.inf, a1)
    en = np.maximum(np.max(np.minimum(a0, a1), axis=1), 0.0)
    ex = np.min(np.maximum(a0, a1), axis=1)
    return en <= ex


def _ray(o, d):
    inv = _rn(1.0 / d.astype(np.float64))
    inv = _rn(np.copysign(np.minimum(np.abs(inv), 2.0 ** 64), d))
    oi = _rn(o.astype(np.float64) * inv)
    e = _rn(np.abs(oi).astype(np.float64) * 2.0 ** -21).astype(np.float64)
    pos = inv >= 0
    off_lo = np.where(pos, _rn(oi + e), _rn(oi - e))
    off_hi = np.where(pos, _rn(oi - e), _rn(oi + e))
    return inv, off_lo, off_hi


def _interval(tn3, tf3):
    tn = _fmax(_fmax(tn3[:, 0], tn3[:, 1]), _fmax(tn3[:, 2], np.float32(0)))
    tf = _fmin(_fmin(tf3[:, 0], tf3[:, 1]), tf3[:, 2])
    return tn <= _rn(tf.astype(np.float64) * np.float64(np.float32(1.00000024)))


def _device_hit(o, d, lo, hi):
    """The min/max form: both planes of an axis, then the smaller is the entry."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv, off_lo, off_hi = _ray(o, d)
        t0, t1 = _fma32(lo, inv, -off_lo), _fma32(hi, inv, -off_hi)
        return _interval(_fmin(t0, t1), _fmax(t0, t1))


def _device_hit_signed(o, d, lo, hi):
    """The form the traversal runs: the entry plane of an axis is lo where 1/d >= 0 and hi
    otherwise (chosen per ray), each plane with its own padded offset; no min or max per axis."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv, off_lo, off_hi = _ray(o, d)
        pos = inv >= 0
        near, far = np.where(pos, lo, hi), np.where(pos, hi, lo)
        on, of = np.where(pos, off_lo, off_hi), np.where(pos, off_hi, off_lo)
        return _interval(_fma32(near, inv, -on), _fma32(far, inv, -of))


def test_padded_fma_slab_test_is_conservative():
    o, d, lo, hi = _cases(300_000, 11)
    ex, dev = _exact_hit(o, d, lo, hi), _device_hit(o, d, lo, hi)
    assert ex.sum() > 200_000
    assert not (ex & ~dev).any()
    # and it stays a test: the boxes it accepts beyond the exact ones are few
    assert (dev & ~ex).sum() < 0.03 * ex.sum()


def test_entry_plane_by_ray_sign_equals_min_max():
    """Picking each axis's entry and exit plane by the sign of 1/d gives the same decisions as the
    min/max form on every valid box (the padded offsets already follow the sign), and rejects the
    empty slots of a wide node (lo = +inf, hi = -inf) for every ray, which min/max would accept."""
    o, d, lo, hi = _cases(300_000, 12)
    assert np.array_equal(_device_hit_signed(o, d, lo, hi), _device_hit(o, d, lo, hi))
    inf = np.full(lo.shape, np.inf, np.float32)
    assert not _device_hit_signed(o, d, inf, -inf).any()
    assert _device_hit(o, d, inf, -inf).all()
