"""Pins for the oracle's no-slip wall image systems (Sec. III, tab:rpywall).

A Stokes flow in the half-space with a given point singularity, vanishing on
the wall and at infinity, is unique; the pins check each of those facts and
the RPY regularisation independently of the image construction:
  * no slip: u = 0 on the wall, for b = 0 and b > 0;
  * incompressibility (finite differences) and lap u = FD Laplacian of u,
    with lap u curl free (it is grad p);
  * far from the wall the image terms vanish: free-space RPY / Stokeslet;
  * the RPY wall tensor is the source-side Faxen operator (1 + b^2/6 lap_y)
    applied to the b = 0 wall tensor (finite differences in y);
  * Lorentz reciprocity: f'.u(x; f at y) = f.u(y; f' at x) for b = 0, and the
    mobility u + (b^2/6) lap u is symmetric for equal radii.
"""
import numpy as np

from oracle import direct, wall
from tests import _fd

RNG = np.random.default_rng(777)


def _src(n, zlo=0.2, zhi=0.6):
    return np.concatenate([RNG.random((n, 2)), RNG.uniform(zlo, zhi, (n, 1))], axis=1)


def _trg(n, zlo=0.05, zhi=0.9):
    return np.concatenate([RNG.uniform(-0.5, 1.5, (n, 2)), RNG.uniform(zlo, zhi, (n, 1))], axis=1)


def test_no_slip_on_the_wall():
    y, f = _src(5), RNG.standard_normal((5, 3))
    b = RNG.uniform(0.01, 0.05, 5)
    xw = np.concatenate([RNG.uniform(-1, 2, (20, 2)), np.zeros((20, 1))], axis=1)
    scale = np.abs(wall.rpy_wall(y, np.c_[f, b], _trg(20))[:, :3]).max()
    assert np.abs(wall.rpy_wall(y, np.c_[f, b], xw)[:, :3]).max() < 1e-13 * scale
    assert np.abs(wall.stokeslet_wall(y, f, xw)).max() < 1e-13 * scale
    # a wall at z_w = 0.3: the same system shifted
    zw = 0.3
    ys = y + [0, 0, zw]
    assert np.abs(wall.rpy_wall(ys, np.c_[f, b], xw + [0, 0, zw], zw=zw)[:, :3]).max() < 1e-13 * scale


def test_stokeslet_is_rpy_with_zero_radius():
    y, f, x = _src(4), RNG.standard_normal((4, 3)), _trg(10)
    got = wall.stokeslet_wall(y, f, x)
    ref = wall.rpy_wall(y, np.c_[f, np.zeros(4)], x)[:, :3]
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-14 * np.abs(ref).max())


def test_incompressible_and_lap_u():
    y, f, b = _src(3), RNG.standard_normal((3, 3)), RNG.uniform(0.02, 0.05, 3)
    x = _trg(6, 0.7, 0.9)
    fb = np.c_[f, b]
    out = wall.rpy_wall(y, fb, x)
    J = _fd.grad(lambda xx: wall.rpy_wall(y, fb, xx)[:, :3], x, h=1e-3)
    assert np.abs(np.trace(J, axis1=1, axis2=2)).max() < 1e-9 * np.abs(J).max()
    L = _fd.laplacian(lambda xx: wall.rpy_wall(y, fb, xx)[:, :3], x, h=2e-3)
    assert np.allclose(out[:, 3:], L, rtol=1e-6, atol=1e-7 * np.abs(L).max())
    # lap u = grad p is curl free
    JL = _fd.grad(lambda xx: wall.rpy_wall(y, fb, xx)[:, 3:], x, h=1e-3)
    curl = np.stack([JL[:, 2, 1] - JL[:, 1, 2], JL[:, 0, 2] - JL[:, 2, 0], JL[:, 1, 0] - JL[:, 0, 1]], 1)
    assert np.abs(curl).max() < 1e-8 * np.abs(JL).max()


def test_far_from_the_wall_is_free_space():
    y, f, b = _src(2), RNG.standard_normal((2, 3)), np.full(2, 0.03)
    x = y[:1] + [0.3, -0.2, 0.25]
    errs = []
    for H in (1e2, 1e3):
        up = np.array([0, 0, H])
        got = wall.rpy_wall(y + up, np.c_[f, b], x + up)
        ref = direct.rpy(y + up, np.c_[f, b], x + up)
        errs.append(np.abs(got[:, :3] - ref[:, :3]).max() / np.abs(ref[:, :3]).max())
    # image terms decay like 1/H
    assert errs[1] < 2e-3 and errs[1] < 0.2 * errs[0]


def test_rpy_wall_is_the_faxen_regularised_wall_tensor():
    y, f, b = _src(1), RNG.standard_normal((1, 3)), 0.05
    x = _trg(5, 0.1, 0.8)
    got = wall.rpy_wall(y, np.c_[f, [b]], x)[:, :3]
    u0 = lambda yy: wall.stokeslet_wall(yy, f, x)
    h = 2e-3
    lap_y = 0.0
    for k in range(3):
        for s, w in ((-2, -1 / 12), (-1, 16 / 12), (0, -30 / 12), (1, 16 / 12), (2, -1 / 12)):
            lap_y = lap_y + w * u0(y + s * h * np.eye(3)[k])
    lap_y /= h * h
    ref = u0(y) + b * b / 6.0 * lap_y
    assert np.allclose(got, ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())


def test_reciprocity():
    ya, yb = _src(1), _src(1)
    fa, fb = RNG.standard_normal(3), RNG.standard_normal(3)
    # b = 0: the wall Green's function is symmetric
    uab = wall.stokeslet_wall(ya, fa[None], yb)[0]
    uba = wall.stokeslet_wall(yb, fb[None], ya)[0]
    assert abs(fb @ uab - fa @ uba) < 1e-13 * (abs(fb @ uab) + 1e-300)
    # equal radii: u + (b^2/6) lap u (Faxen at the target) is symmetric
    b = 0.04
    oa = wall.rpy_wall(ya, np.r_[fa, b][None], yb)[0]
    ob = wall.rpy_wall(yb, np.r_[fb, b][None], ya)[0]
    ma = oa[:3] + b * b / 6.0 * oa[3:]
    mb = ob[:3] + b * b / 6.0 * ob[3:]
    assert abs(fb @ ma - fa @ mb) < 1e-12 * abs(fb @ ma)
