"""FP64 Ewald sums for triply periodic Laplace (oracle) -- TEST INFRASTRUCTURE.

Wraps ``ewald.c``.  Evaluates (phi, grad phi[, Hessian]) at targets for charges q and
dipoles d in a periodic cube of side L: the periodic boundary condition of
Sec. III and its appendix on periodicity, with the conventions the paper
leaves open fixed as: zero net charge, k = 0 term dropped, no surface term
("tin-foil").  Coordinates may lie anywhere; the sum is periodic in them.
"""
import math

import numpy as np

from .direct import _arr, _p, lib


def parameters(L, xi=None, tol=1e-13):
    """Split parameter xi, real cutoff rc and reciprocal cube half-width nmax
    such that both truncated tails are below ``tol`` (relative to O(1) terms)."""
    if xi is None:
        xi = 6.0 / L
    s = math.sqrt(-math.log(tol)) + 0.3          # erfc(s) ~ tol
    rc = s / xi
    kc = 2.0 * xi * s                            # exp(-kc^2/(4 xi^2)) ~ tol
    nmax = int(math.ceil(kc * L / (2.0 * math.pi)))
    return xi, rc, nmax


def structure(src, q, d, L, nmax, Q=None):
    src, ns = _arr(src, 3)
    q, _ = _arr(q)
    d, _ = _arr(d, 3)
    Q, _ = _arr(Q, 9)
    w = 2 * nmax + 1
    sr = np.zeros(w ** 3)
    si = np.zeros(w ** 3)
    lib().oracle_ewald_structure(ns, _p(src), _p(q), _p(d), _p(Q), float(L), int(nmax), _p(sr), _p(si))
    return sr, si


def laplace_periodic(src, q, d, trg, L=1.0, xi=None, tol=1e-13, S=None, hess=False, Q=None):
    """(phi, grad phi) [nt, 4] of periodic charges q [ns], dipoles d [ns,3] and
    quadrupoles Q [ns,9] (row-major); with hess=True also the Hessian
    (xx, xy, xz, yy, yz, zz) [nt, 10].

    ``S`` may pass a precomputed structure factor (same src/q/d/L/xi/tol)."""
    if q is not None and abs(float(np.sum(q))) > 1e-9 * max(1.0, float(np.sum(np.abs(q)))):
        raise ValueError("periodic Laplace needs zero net charge")
    xi, rc, nmax = parameters(L, xi, tol)
    if S is None:
        S = structure(src, q, d, L, nmax, Q)
    src, ns = _arr(src, 3)
    q, _ = _arr(q)
    d, _ = _arr(d, 3)
    Q, _ = _arr(Q, 9)
    trg, nt = _arr(trg, 3)
    out = np.zeros((nt, 10 if hess else 4))
    lib().oracle_ewald_eval(ns, _p(src), _p(q), _p(d), _p(Q), nt, _p(trg), float(L), float(xi),
                            float(rc), int(nmax), _p(S[0]), _p(S[1]), _p(out), int(hess))
    return out
