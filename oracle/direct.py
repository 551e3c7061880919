"""FP64 direct sums (oracle) -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrappers over ``direct.c``.  Each function evaluates the plain
O(N_S * N_T) kernel sum of Sec. I, Eq. kernelsumlinear (Eq. kernelsum for
RPY) at the given targets; r = x - y, pairs with r == 0 are skipped.

Value layouts (per point, AoS), following the kernel list of the appendix
table of supported kernels (tab:implement):
  stokeslet  SL f (3)                        -> u (3)
  rpy        SL (f, b) (4)                   -> (u, lap u) (6)
  laplace    SL q (1), DL d (3)              -> (phi, grad phi) (4)
             with hess=True                  -> + (xx,xy,xz,yy,yz,zz) (10)
  pvel       SL (f, q) (4), DL D (9)         -> (p, u) (4)
  traction   SL (f, q) (4), DL D (9)         -> sigma (9), row-major
"""
import ctypes

import numpy as np

from . import build as _build

_lib = None
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        _lib = ctypes.CDLL(path)
        for name in ("oracle_stokeslet", "oracle_rpy", "oracle_stokes_reg", "oracle_stokes_reg_ft"):
            getattr(_lib, name).argtypes = [_i64, _dp, _dp, _i64, _dp, _dp]
        _lib.oracle_laplace.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp, _i64, _dp, _dp, ctypes.c_int]
        _lib.oracle_max_threads.argtypes = []
        _lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib.oracle_set_threads.restype = None
        _lib.oracle_laplace_quad.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp]
        _lib.oracle_pvel_deriv.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp, _i64, _dp, _dp, ctypes.c_int]
        for name in ("oracle_pvel", "oracle_traction"):
            getattr(_lib, name).argtypes = [_i64, _dp, _dp, _i64, _dp, _dp, _i64, _dp, _dp]
        _lib.oracle_ewald_structure.argtypes = [_i64, _dp, _dp, _dp, _dp, ctypes.c_double,
                                                ctypes.c_int, _dp, _dp]
        _lib.oracle_ewald_eval.argtypes = [_i64, _dp, _dp, _dp, _dp, _i64, _dp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           _dp, _dp, _dp, ctypes.c_int]
        _lib.oracle_stokes_ewald_real.argtypes = [_i64, _dp, _dp, _i64, _dp, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, _dp]
        _lib.oracle_stokes_lap_ewald_real.argtypes = [_i64, _dp, _dp, _dp, _i64, _dp, ctypes.c_double,
                                                      ctypes.c_double, ctypes.c_double, _dp]
        _lib.oracle_stokes_dl_ewald_real.argtypes = [_i64, _dp, _dp, _i64, _dp, ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_double, _dp]
    return _lib


def max_threads():
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_max_threads())


def set_threads(n):
    lib().oracle_set_threads(int(n))


def _arr(a, cols=None):
    if a is None:
        return None, 0
    a = np.ascontiguousarray(a, dtype=np.float64)
    if cols is not None:
        a = a.reshape(-1, cols)
    return a, len(a)


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def stokeslet(src, f, trg):
    src, ns = _arr(src, 3)
    f, _ = _arr(f, 3)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 3))
    lib().oracle_stokeslet(ns, _p(src), _p(f), nt, _p(trg), _p(out))
    return out


def rpy(src, fb, trg):
    src, ns = _arr(src, 3)
    fb, _ = _arr(fb, 4)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 6))
    lib().oracle_rpy(ns, _p(src), _p(fb), nt, _p(trg), _p(out))
    return out


def stokes_reg(src, fe, trg):
    """Regularized Stokeslet [f, eps] -> u (Sec. II.B, tab:ktab_reg)."""
    src, ns = _arr(src, 3)
    fe, _ = _arr(fe, 4)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 3))
    lib().oracle_stokes_reg(ns, _p(src), _p(fe), nt, _p(trg), _p(out))
    return out


def stokes_reg_ft(src, fte, trg):
    """Regularized force and torque [f, t, eps] -> [u, omega] (Sec. II.B)."""
    src, ns = _arr(src, 3)
    fte, _ = _arr(fte, 7)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 6))
    lib().oracle_stokes_reg_ft(ns, _p(src), _p(fte), nt, _p(trg), _p(out))
    return out


def laplace(sl=None, q=None, dl=None, d=None, trg=None, hess=False):
    sl, nsl = _arr(sl, 3)
    q, _ = _arr(q)
    dl, ndl = _arr(dl, 3)
    d, _ = _arr(d, 3)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 10 if hess else 4))
    lib().oracle_laplace(nsl, _p(sl), _p(q), ndl, _p(dl), _p(d), nt, _p(trg), _p(out), int(hess))
    return out


def laplace_quad(sl=None, Q=None, trg=None):
    """Quadrupoles Q (9, row-major) -> phi, grad phi, Hessian (xx,xy,xz,yy,yz,zz)."""
    sl, nsl = _arr(sl, 3)
    Q, _ = _arr(Q, 9)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 10))
    lib().oracle_laplace_quad(nsl, _p(sl), _p(Q), nt, _p(trg), _p(out))
    return out


def pvel(sl=None, fq=None, dl=None, D=None, trg=None):
    sl, nsl = _arr(sl, 3)
    fq, _ = _arr(fq, 4)
    dl, ndl = _arr(dl, 3)
    D, _ = _arr(D, 9)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 4))
    lib().oracle_pvel(nsl, _p(sl), _p(fq), ndl, _p(dl), _p(D), nt, _p(trg), _p(out))
    return out


def pvel_grad(sl=None, fq=None, dl=None, D=None, trg=None, lap=False):
    """(p, u, grad p, grad u) (16), or with lap=True (p, u, lap u) (7)."""
    sl, nsl = _arr(sl, 3)
    fq, _ = _arr(fq, 4)
    dl, ndl = _arr(dl, 3)
    D, _ = _arr(D, 9)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 7 if lap else 16))
    lib().oracle_pvel_deriv(nsl, _p(sl), _p(fq), ndl, _p(dl), _p(D), nt, _p(trg), _p(out), int(lap))
    return out


def traction(sl=None, fq=None, dl=None, D=None, trg=None):
    sl, nsl = _arr(sl, 3)
    fq, _ = _arr(fq, 4)
    dl, ndl = _arr(dl, 3)
    D, _ = _arr(D, 9)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 9))
    lib().oracle_traction(nsl, _p(sl), _p(fq), ndl, _p(dl), _p(D), nt, _p(trg), _p(out))
    return out


def evaluate(kernel, sl=None, sl_val=None, dl=None, dl_val=None, trg=None):
    """Dispatch by kernel name (names as in tab:implement)."""
    if kernel == "Stokeslet":
        return stokeslet(sl, sl_val, trg)
    if kernel == "RPY":
        return rpy(sl, sl_val, trg)
    if kernel == "StokesRegVel":
        return stokes_reg(sl, sl_val, trg)
    if kernel == "StokesRegVelOmega":
        return stokes_reg_ft(sl, sl_val, trg)
    if kernel == "LapPGrad":
        return laplace(sl, sl_val, dl, dl_val, trg)
    if kernel == "LapPGradGrad":
        return laplace(sl, sl_val, dl, dl_val, trg, hess=True)
    if kernel == "LapQPGradGrad":
        return laplace_quad(sl, sl_val, trg)
    if kernel == "PVel":
        return pvel(sl, sl_val, dl, dl_val, trg)
    if kernel == "Traction":
        return traction(sl, sl_val, dl, dl_val, trg)
    if kernel == "PVelGrad":
        return pvel_grad(sl, sl_val, dl, dl_val, trg)
    if kernel == "PVelLaplacian":
        return pvel_grad(sl, sl_val, dl, dl_val, trg, lap=True)
    raise ValueError("unknown kernel %r" % kernel)


def rel_l2(got, ref):
    """Relative L2 error ||g - g_ref|| / ||g_ref|| (Sec. III, error metric)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
