"""Doubly periodic Stokeslet and RPY by Ewald summation (oracle) -- TEST INFRASTRUCTURE ONLY.

Periodic in x and y with period L, open in z (the doubly periodic boundary
of Sec. III and its appendix on periodicity), viscosity 1:

    u(x) = sum_j sum_{n in Z^2} G(x - y_j - n L) f_j,   G = (I/r + r r^T/r^3)/(8 pi)   (Sec. II.B),

defined by its Fourier series in x and y with the k_par = 0 mode the sheet
flow -(1/2A) sum_j f_j,par |z - z_j| (A = L^2, zero net force, no added
constant).  The Ewald split (Hasimoto), the closed forms of the z integrals
and the self terms are stated in ``stokes_dp.c``; RPY adds (b^2/6) lap G f
to the velocity and returns lap u = sum lap G f (Sec. II.B, Eq. RPYkernel).
"""
import ctypes

import numpy as np

from .direct import _p, lib

PI = np.pi
_dp = ctypes.POINTER(ctypes.c_double)


def _setup():
    L = lib()
    if not getattr(L, "_dp_ready", False):
        L.oracle_stokes_dp.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int64, _dp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.oracle_stokes_dp.restype = None
        L._dp_ready = True
    return L


def parameters(L, xi=None, tol=1e-15):
    """(xi, real-space cutoff, spectral mode bound) for relative truncation tol."""
    if xi is None:
        xi = 4.0 / L
    s = np.sqrt(-np.log(tol)) + 0.5
    return xi, s / xi, int(np.ceil(2.0 * xi * s * L / (2.0 * PI)))


def _run(src, f, trg, w, L, xi, tol, want_lap, need_zero_force=True):
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    if need_zero_force and len(y) and np.abs(f.sum(axis=0)).max() > 1e-9 * max(1.0, np.abs(f).sum()):
        raise ValueError("doubly periodic Stokes needs zero net force")
    xi, rc, nk = parameters(L, xi, tol)
    u = np.zeros((len(x), 3))
    lap = np.zeros((len(x), 3)) if want_lap else None
    if len(y) and len(x):
        wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        _setup().oracle_stokes_dp(len(y), _p(y), _p(f), _p(wv), len(x), _p(x), float(L), float(xi), float(rc),
                                  int(nk), _p(u), _p(lap))
    return u, lap


def stokeslet_dp(src, f, trg, L=1.0, xi=None, tol=1e-15):
    """Doubly periodic Stokeslet velocity [m, 3] at trg of forces f [n, 3] at src."""
    return _run(src, f, trg, None, L, xi, tol, False)[0]


def stokeslet_lap_dp(src, f, trg, L=1.0, xi=None, tol=1e-15):
    """(u, sum_j lap G f_j) of the doubly periodic Stokeslet."""
    return _run(src, f, trg, None, L, xi, tol, True)


def lap_g_dp(src, f, trg, L=1.0, xi=None, tol=1e-15):
    """sum_j sum_n lap G(x - y_j - n L) f_j [m, 3]: absolutely convergent (1/r^3),
    any net force."""
    return _run(src, f, trg, None, L, xi, tol, True, need_zero_force=False)[1]


def rpy_dp(src, fb, trg, L=1.0, xi=None, tol=1e-15):
    """Doubly periodic RPY (u, lap u) [m, 6] of (f, b) [n, 4]: u = sum (G + b^2/6 lap G) f."""
    fb = np.asarray(fb, dtype=np.float64).reshape(-1, 4)
    u, lap = _run(src, fb[:, :3], trg, fb[:, 3] ** 2 / 6.0, L, xi, tol, True)
    return np.concatenate([u, lap], axis=1)
