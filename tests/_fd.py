"""Finite differences and sphere quadrature used to pin the oracle's kernels.

These helpers know nothing of any kernel formula: they differentiate or
integrate whatever function they are given.
"""
import numpy as np

# 4th-order central difference weights for the first and second derivative
_D1 = ((-2, 1.0 / 12), (-1, -8.0 / 12), (1, 8.0 / 12), (2, -1.0 / 12))
_D2 = ((-2, -1.0 / 12), (-1, 16.0 / 12), (0, -30.0 / 12), (1, 16.0 / 12), (2, -1.0 / 12))


def grad(fun, x, h=1e-3):
    """d fun / d x_k at points x [n,3]; fun maps [m,3] -> [m,k]. Returns [n, k, 3]."""
    x = np.asarray(x, dtype=np.float64)
    cols = []
    for a in range(3):
        acc = 0.0
        for s, w in _D1:
            xs = x.copy()
            xs[:, a] += s * h
            acc = acc + w * fun(xs)
        cols.append(acc / h)
    return np.stack(cols, axis=-1)


def laplacian(fun, x, h=1e-3):
    x = np.asarray(x, dtype=np.float64)
    acc = 0.0
    for a in range(3):
        for s, w in _D2:
            xs = x.copy()
            xs[:, a] += s * h
            acc = acc + w * fun(xs)
    return acc / (h * h)


def sphere_quadrature(centre, R, n_theta=48, n_phi=96):
    """Gauss-Legendre in cos(theta) x trapezoid in phi; returns points, normals, weights."""
    t, wt = np.polynomial.legendre.leggauss(n_theta)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    ct, PH = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    n = np.stack([st * np.cos(PH), st * np.sin(PH), ct], axis=-1).reshape(-1, 3)
    w = (np.repeat(wt, n_phi) * (2 * np.pi / n_phi)) * R * R
    return np.asarray(centre) + R * n, n, w
