"""Seeded synthetic inputs for the kernel-summation workloads.

This module only draws random numbers and lays out geometry (point clouds,
source values).  It holds none of the method's arithmetic, so both the
FP64 oracle (test infrastructure) and the HIP path may be fed from it.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64).  Points live
in the half-open unit cube [0, 1)^3 unless a box is stated.

Workload recipes (shapes and distributions):

* ``uniform_stokeslet``   N uniform points, SL = targets, f ~ N(0,1)^3.
* ``clustered_rpy``        8-cluster Gaussian mixture (sigma 0.05, centres
  U[0.2,0.8]^3), points outside the cube are redrawn; f ~ N(0,1)^3 and RPY
  radii b ~ U[0.002, 0.005].
* ``periodic_laplace``     N uniform points, charges N(0,1) shifted to zero
  net charge, dipoles N(0,1)^3; SL = DL = targets.
* ``sphere_doublelayer``   non-overlapping spheres of radius 0.01 placed by
  random sequential addition, quasi-uniform (Fibonacci) surface points with
  outward unit normals n, densities v ~ N(0,1)^3 and D = v n^T (row-major).
* ``mixture``              the training mixtures: k ~ U{1..16} clusters,
  sigma ~ U[0.01, 0.1], N log-uniform in a range.
* ``lognormal_points``     the paper's benchmark distribution (Sec. III,
  Eq. ptdist): each coordinate L*(u - floor(u)), u log-normal(m=-1, s=0.5).
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def uniform_points(n, seed, box=1.0):
    rng = _rng(seed)
    return rng.random((n, 3)) * box


def uniform_stokeslet(n=4096, seed=101):
    rng = _rng(seed)
    x = rng.random((n, 3))
    f = rng.standard_normal((n, 3))
    return {"xyz": x, "f": f}


def gaussian_mixture_points(rng, n, centres, sigma):
    """n points from an equal-weight Gaussian mixture, redrawn until inside [0,1)^3."""
    k = len(centres)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (k,))
    counts = np.full(k, n // k, dtype=np.int64)
    counts[: n - counts.sum()] += 1
    out = []
    for c, s, m in zip(centres, sig, counts):
        pts = np.empty((0, 3))
        while len(pts) < m:
            cand = c + s * rng.standard_normal((int(m - len(pts)) + 16, 3))
            ok = np.all((cand >= 0.0) & (cand < 1.0), axis=1)
            pts = np.concatenate([pts, cand[ok]])
        out.append(pts[:m])
    return np.concatenate(out)


def clustered_rpy(n=1_048_576, seed=201, n_clusters=8, sigma=0.05):
    rng = _rng(seed)
    centres = 0.2 + 0.6 * rng.random((n_clusters, 3))
    x = gaussian_mixture_points(rng, n, centres, sigma)
    f = rng.standard_normal((n, 3))
    b = rng.uniform(0.002, 0.005, n)
    return {"xyz": x, "f": f, "b": b, "centres": centres}


def periodic_laplace(n=4_194_304, seed=301):
    rng = _rng(seed)
    x = rng.random((n, 3))
    q = rng.standard_normal(n)
    q -= q.mean()
    d = rng.standard_normal((n, 3))
    return {"xyz": x, "q": q, "d": d}


def fibonacci_sphere(n):
    """Quasi-uniform unit vectors on the sphere (golden-angle spiral)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def rsa_centres(rng, n_spheres, lo, hi, min_dist, max_tries=10_000_000):
    """Random sequential addition of sphere centres with a minimum separation."""
    cells = max(1, int((hi - lo) / min_dist))
    grid = {}
    out = []
    tries = 0
    while len(out) < n_spheres:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        c = lo + (hi - lo) * rng.random(3)
        key = tuple(np.minimum(((c - lo) / min_dist).astype(int), cells - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((out[j] - c) ** 2) < min_dist * min_dist:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault(key, []).append(len(out))
            out.append(c)
    return np.array(out)


def sphere_doublelayer(n_spheres=2000, pts_per_sphere=1000, seed=401, radius=0.01):
    rng = _rng(seed)
    centres = rsa_centres(rng, n_spheres, 0.01, 0.99, 2 * radius + 1e-3)
    nrm = fibonacci_sphere(pts_per_sphere)
    x = (centres[:, None, :] + radius * nrm[None, :, :]).reshape(-1, 3)
    n = np.broadcast_to(nrm, (n_spheres, pts_per_sphere, 3)).reshape(-1, 3).copy()
    v = rng.standard_normal((n_spheres * pts_per_sphere, 3))
    D = (v[:, :, None] * n[:, None, :]).reshape(-1, 9)
    return {"xyz": x, "normal": n, "v": v, "D": D, "centres": centres}


def mixture(seed, n_range=(100_000, 2_000_000)):
    rng = _rng(seed)
    k = int(rng.integers(1, 17))
    sig = rng.uniform(0.01, 0.1, k)
    lo, hi = n_range
    n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    centres = 0.1 + 0.8 * rng.random((k, 3))
    x = gaussian_mixture_points(rng, n, centres, sig)
    f = rng.standard_normal((n, 3))
    return {"xyz": x, "f": f, "k": k, "sigma": sig, "centres": centres}


def lognormal_points(n, seed, box=32.0, m=-1.0, s=0.5):
    rng = _rng(seed)
    u = rng.lognormal(m, s, (n, 3))
    return box * (u - np.floor(u))


def sample_indices(n, k, seed):
    """k distinct indices out of n, sorted (used to sample targets for checks)."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))
