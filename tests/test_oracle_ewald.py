"""Pins for the oracle's FP64 Ewald sum (triply periodic Laplace).

* the rock-salt Madelung constant (a textbook value, independent of Ewald);
* independence of the split parameter xi;
* invariance under a periodic translation of all points (the paper's
  translation test, Sec. III.C);
* grad phi against finite differences of phi;
* a dipole as the limit of a neutral pair of charges;
* a neutral, dipole-free cell summed over growing cubes of images.
"""
import math

import numpy as np
import pytest

from oracle import direct, ewald
from tests import _fd

MADELUNG_NACL = 1.747564594633182  # rock-salt structure, nearest-neighbour units

RNG = np.random.default_rng(777)


@pytest.fixture(autouse=True)
def _fresh_rng():
    # every test draws the same sequence, whatever runs before it
    global RNG
    RNG = np.random.default_rng(777)


def _away(y, k, dmin=0.15, L=1.0):
    """k points at least dmin from every point of y and its periodic images
    (finite differences and limits of point pairs need the distance)."""
    out = []
    while len(out) < k:
        c = RNG.random(3) * L
        d = c - y
        d -= L * np.round(d / L)
        if np.min(np.linalg.norm(d, axis=1)) >= dmin:
            out.append(c)
    return np.array(out)


def _cell(n=12, L=1.0):
    y = RNG.random((n, 3)) * L
    q = RNG.standard_normal(n)
    q -= q.mean()
    d = RNG.standard_normal((n, 3))
    return y, q, d


def test_nacl_madelung():
    a = 0.5
    pos, q = [], []
    for i in range(2):
        for j in range(2):
            for k in range(2):
                pos.append([i * a + 0.1, j * a + 0.2, k * a + 0.05])
                q.append((-1.0) ** (i + j + k))
    pos, q = np.array(pos), np.array(q)
    out = ewald.laplace_periodic(pos, q, None, pos, 1.0)
    # every ion sees -M q / (4 pi a)
    assert np.allclose(out[:, 0] * 4 * math.pi * a / -q, MADELUNG_NACL, rtol=1e-13)
    assert np.max(np.abs(out[:, 1:])) < 1e-13   # cubic symmetry: no field at the ions


def test_xi_independence():
    y, q, d = _cell()
    x = RNG.random((5, 3))
    ref = ewald.laplace_periodic(y, q, d, x, 1.0, xi=4.0)
    for xi in (6.0, 9.0):
        out = ewald.laplace_periodic(y, q, d, x, 1.0, xi=xi)
        assert np.allclose(out, ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))


def test_coincident_targets_xi_independence():
    y, q, d = _cell()
    ref = ewald.laplace_periodic(y, q, d, y, 1.0, xi=4.0)
    out = ewald.laplace_periodic(y, q, d, y, 1.0, xi=8.0)
    assert np.allclose(out, ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))


def test_translation_invariance():
    y, q, d = _cell()
    x = RNG.random((5, 3))
    ref = ewald.laplace_periodic(y, q, d, x, 1.0)
    s = np.array([0.37, -0.81, 0.55])
    out = ewald.laplace_periodic(np.mod(y + s, 1.0), q, d, np.mod(x + s, 1.0), 1.0)
    assert np.allclose(out, ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(ref)))


def test_gradient_is_fd():
    y, q, d = _cell()
    x = _away(y, 4)
    S = ewald.structure(y, q, d, 1.0, ewald.parameters(1.0)[2])
    fun = lambda xx: ewald.laplace_periodic(y, q, d, xx, 1.0, S=S)[:, :1]
    g = _fd.grad(fun, x, h=1e-3)[:, 0, :]
    out = ewald.laplace_periodic(y, q, d, x, 1.0, S=S)
    assert np.allclose(out[:, 1:], g, rtol=1e-7, atol=1e-8)


def test_dipole_is_limit_of_charges():
    y0 = np.array([0.3, 0.6, 0.45])
    dv = np.array([0.2, -0.5, 0.1])
    # targets at least 0.2 from the dipole (and its images): the pair differs
    # from the dipole by O(eps^2 / r^4)
    x = np.array([[0.65, 0.1, 0.8], [0.05, 0.3, 0.2], [0.9, 0.95, 0.5], [0.5, 0.35, 0.1]])
    eps = 1e-4
    pair = ewald.laplace_periodic(np.array([y0 + eps * dv / 2, y0 - eps * dv / 2]),
                                  np.array([1 / eps, -1 / eps]), None, x, 1.0)
    dip = ewald.laplace_periodic(y0[None], None, dv[None], x, 1.0)
    assert np.allclose(dip, pair, rtol=1e-6, atol=1e-7)


def test_image_sum_of_neutral_dipole_free_cell():
    # charges and their mirror images: zero net charge and zero dipole moment.
    # The plain sum over growing cubes of images then converges; it differs
    # from the Ewald value (k = 0 term dropped) by the constant
    # -(1/6V) sum q |y - c|^2 that the cubic summation keeps, and not at all
    # in the gradient.
    y = np.array([[0.2, 0.3, 0.4], [0.7, 0.1, 0.6], [0.45, 0.8, 0.25]])
    q = np.array([1.0, -0.6, 0.9])
    c = np.array([0.5, 0.5, 0.5])
    ys = np.concatenate([y, 2 * c - y, c[None]])
    qs = np.concatenate([q, q, [-2 * q.sum()]])
    assert abs(qs.sum()) < 1e-15
    assert np.allclose(np.sum(qs[:, None] * (ys - c), axis=0), 0, atol=1e-14)
    x = np.array([[0.11, 0.52, 0.93], [0.6, 0.2, 0.3]])
    ref = ewald.laplace_periodic(ys, qs, None, x, 1.0)
    offset = -np.sum(qs * np.sum((ys - c) ** 2, axis=1)) / 6.0
    errs = []
    for K in (8, 16):
        rng = np.arange(-K, K + 1)
        n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)
        img = (ys[None, :, :] + n[:, None, :]).reshape(-1, 3)
        v = direct.laplace(img, np.tile(qs, len(n)), trg=x)
        errs.append(max(np.max(np.abs(v[:, 0] - ref[:, 0] - offset)),
                        np.max(np.abs(v[:, 1:] - ref[:, 1:]))))
    assert errs[1] < errs[0]
    assert errs[1] < 2e-4


def test_rejects_net_charge():
    with pytest.raises(ValueError):
        ewald.laplace_periodic(np.zeros((1, 3)), np.ones(1), None, np.ones((1, 3)) * 0.5)


def test_hessian_is_fd_of_gradient_and_harmonic():
    y, q, d = _cell()
    x = _away(y, 4)
    S = ewald.structure(y, q, d, 1.0, ewald.parameters(1.0)[2])
    out = ewald.laplace_periodic(y, q, d, x, 1.0, S=S, hess=True)
    assert np.allclose(out[:, :4], ewald.laplace_periodic(y, q, d, x, 1.0, S=S), rtol=1e-14, atol=1e-14)
    J = _fd.grad(lambda xx: ewald.laplace_periodic(y, q, d, xx, 1.0, S=S)[:, 1:4], x, h=1e-3)
    H = np.stack([J[:, 0, 0], J[:, 0, 1], J[:, 0, 2], J[:, 1, 1], J[:, 1, 2], J[:, 2, 2]], 1)
    assert np.allclose(out[:, 4:], H, rtol=1e-6, atol=1e-7 * np.abs(H).max())
    # symmetric FD Jacobian, and zero net charge: harmonic between the sources
    assert np.allclose(J[:, 0, 1], J[:, 1, 0], rtol=1e-6, atol=1e-7 * np.abs(H).max())
    assert np.abs(out[:, 4] + out[:, 7] + out[:, 9]).max() < 1e-10 * np.abs(out[:, 4:]).max()


def test_hessian_xi_independence_at_coincident_targets():
    # the self terms: targets on the sources themselves
    y, q, d = _cell()
    ref = ewald.laplace_periodic(y, q, d, y, 1.0, xi=4.0, hess=True)
    out = ewald.laplace_periodic(y, q, d, y, 1.0, xi=8.0, hess=True)
    assert np.allclose(out, ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))


def _quads(n=6):
    y = RNG.random((n, 3))
    Q = RNG.standard_normal((n, 9))
    return y, Q


def test_quadrupole_xi_independence():
    y, Q = _quads()
    for x in (RNG.random((5, 3)), y):      # away from and on the sources (self terms)
        ref = ewald.laplace_periodic(y, None, None, x, 1.0, xi=4.0, hess=True, Q=Q)
        out = ewald.laplace_periodic(y, None, None, x, 1.0, xi=8.0, hess=True, Q=Q)
        assert np.allclose(out, ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))


def test_quadrupole_is_limit_of_dipole_pairs():
    # Q_ab d_a d_b L = d/dy_a d/dy_b L: dipoles (Q_ab/eps) e_b at y +- eps e_a / 2
    _, Q = _quads(2)
    x = np.array([[0.61, 0.12, 0.84], [0.07, 0.33, 0.21], [0.93, 0.95, 0.52]])
    y = _away(x, 2)
    got = ewald.laplace_periodic(y, None, None, x, 1.0, hess=True, Q=Q)
    res = []
    for eps in (2e-3, 4e-3):
        pos, dip = [], []
        for s in range(len(y)):
            for a in range(3):
                for b in range(3):
                    e_a, e_b = np.eye(3)[a], np.eye(3)[b]
                    pos += [y[s] + eps * e_a / 2, y[s] - eps * e_a / 2]
                    dip += [Q[s, 3 * a + b] / eps * e_b, -Q[s, 3 * a + b] / eps * e_b]
        res.append(ewald.laplace_periodic(np.array(pos), None, np.array(dip), x, 1.0, hess=True))
    ref = (4 * res[0] - res[1]) / 3
    assert np.allclose(got, ref, rtol=1e-7, atol=1e-8 * np.max(np.abs(ref)))


def test_quadrupole_gradient_and_hessian_are_fd():
    y, Q = _quads()
    x = _away(y, 4)
    S = ewald.structure(y, None, None, 1.0, ewald.parameters(1.0)[2], Q)
    f = lambda xx: ewald.laplace_periodic(y, None, None, xx, 1.0, S=S, Q=Q)
    out = ewald.laplace_periodic(y, None, None, x, 1.0, S=S, hess=True, Q=Q)
    J = _fd.grad(lambda xx: f(xx)[:, :1], x, h=1e-3)[:, 0, :]
    assert np.allclose(out[:, 1:4], J, rtol=1e-6, atol=1e-7 * np.abs(J).max())
    Jg = _fd.grad(lambda xx: f(xx)[:, 1:4], x, h=1e-3)
    H = np.stack([Jg[:, 0, 0], Jg[:, 0, 1], Jg[:, 0, 2], Jg[:, 1, 1], Jg[:, 1, 2], Jg[:, 2, 2]], 1)
    assert np.allclose(out[:, 4:], H, rtol=1e-6, atol=1e-7 * np.abs(H).max())
