"""The close-pair threshold of the Stokeslet P2P (host-side check of the
design; the plan's check itself runs on the GPU, tests/test_gpu_close_pairs.py).

The leaf-relative form rounds the target, moved into the source leaf's
frame, and the source to FP32 relative to the leaf centre, then subtracts
them in FP32.  Emulated here in NumPy exactly as the kernel rounds:
- r's relative error falls like 1/r and stays below 2^-8 for every pair at
  least 1/4096 of a leaf side apart (targets anywhere in the 3x3x3
  neighbourhood of the source leaf);
- pairs far closer than that lose the separation (r = 0 or a relative error
  of order 1), which is what the plan's check guards against;
- the hi/lo form of the same pairs keeps r to FP32 accuracy.
"""
import numpy as np


def split(x):
    hi = x.astype(np.float32)
    lo = (x - hi.astype(np.float64)).astype(np.float32)
    return hi, lo


def rel_form(x, y, c):
    xh, xl = split(x)
    yh, yl = split(y)
    xr = ((xh.astype(np.float64) - c) + xl.astype(np.float64)).astype(np.float32)
    yr = ((yh.astype(np.float64) - c) + yl.astype(np.float64)).astype(np.float32)
    return np.linalg.norm((xr - yr).astype(np.float64), axis=-1)


def hilo_form(x, y):
    xh, xl = split(x)
    yh, yl = split(y)
    d = (xh - yh) + (xl - yl)                    # FP32 arithmetic, as the kernel
    return np.linalg.norm(d.astype(np.float64), axis=-1)


def pairs(rng, n, w, level_origin, gap):
    """n (target, source) pairs gap apart: sources in the leaf of side w
    centred at c, targets in its 3x3x3 neighbourhood (the U list)."""
    c = level_origin + w * (0.5 + rng.integers(0, 8, 3))
    y = c + w * (rng.random((n, 3)) - 0.5)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x = y + gap[:, None] * u
    keep = np.all(np.abs(x - c) <= 1.5 * w, axis=1)
    return x[keep], y[keep], c


def test_error_at_and_above_the_threshold():
    rng = np.random.default_rng(5)
    for w in (1 / 8, 1 / 64, 1 / 1024):
        for scale in (1, 4, 64, 4096):
            gap = w / 4096 * scale * (1 + rng.random(20000))
            x, y, c = pairs(rng, 20000, w, np.zeros(3), gap)
            r = np.linalg.norm(x - y, axis=1)
            e = np.abs(rel_form(x, y, c) - r) / r
            assert e.max() < 2.0 ** -8 / scale, (w, scale, e.max())


def test_far_closer_pairs_are_lost_without_the_check():
    rng = np.random.default_rng(6)
    w = 1 / 16
    gap = np.full(5000, 1e-9)
    x, y, c = pairs(rng, 5000, w, np.zeros(3), gap)
    r = np.linalg.norm(x - y, axis=1)
    e = np.abs(rel_form(x, y, c) - r) / r
    assert np.median(e) > 0.5
    assert np.mean(rel_form(x, y, c) == 0) > 0.05
    # the hi/lo form resolves the same pairs
    eh = np.abs(hilo_form(x, y) - r) / r
    assert eh.max() < 1e-5
