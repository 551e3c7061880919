"""Pins for the oracle's FP64 direct sums.

Each kernel is checked against facts the mathematics fixes, not against a
retyped copy of its formula: finite-difference derivatives, Gauss's law,
the force balance of a point force, the Stokes equations, the DL net-flux
identity (Sec. II.C), the traction identity sigma = 2 T f (Sec. II.C), the
RPY special cases (Sec. II.B) and symmetry.
"""
import numpy as np
import pytest

from oracle import direct
from tests import _fd

RNG = np.random.default_rng(12345)
PI = np.pi


def _pts(n, lo=-0.3, hi=0.3):
    return RNG.uniform(lo, hi, (n, 3))


def _probe(n=6):
    # targets well away from sources placed in [-0.3,0.3]^3
    d = RNG.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return 1.2 * d


# ---------------------------------------------------------------- Laplace
def test_laplace_unit_charge_value():
    # q = 4 pi at unit distance gives phi = 1; at distance 2 gives 1/2
    out = direct.laplace(np.zeros((1, 3)), [4 * PI], trg=[[1.0, 0, 0], [0, 2.0, 0]])
    assert np.allclose(out[:, 0], [1.0, 0.5], rtol=0, atol=1e-15)


def test_laplace_gradient_is_fd_of_potential():
    y, q = _pts(5), RNG.standard_normal(5)
    yd, d = _pts(4), RNG.standard_normal((4, 3))
    x = _probe()
    fun = lambda xx: direct.laplace(y, q, yd, d, xx)[:, :1]
    g = _fd.grad(fun, x)[:, 0, :]
    out = direct.laplace(y, q, yd, d, x)
    assert np.allclose(out[:, 1:], g, rtol=1e-9, atol=1e-11)


def test_laplace_hessian_is_fd_of_gradient_and_traceless():
    y, q = _pts(5), RNG.standard_normal(5)
    yd, d = _pts(4), RNG.standard_normal((4, 3))
    x = _probe()
    fun = lambda xx: direct.laplace(y, q, yd, d, xx)[:, 1:4]
    J = _fd.grad(fun, x)                       # [n, i, j] = d_j (d_i phi)
    out = direct.laplace(y, q, yd, d, x, hess=True)
    H = out[:, 4:]
    full = np.stack([H[:, 0], H[:, 1], H[:, 2], H[:, 1], H[:, 3], H[:, 4],
                     H[:, 2], H[:, 4], H[:, 5]], axis=1).reshape(-1, 3, 3)
    assert np.allclose(full, J, rtol=1e-8, atol=1e-10)
    assert np.allclose(np.trace(full, axis1=1, axis2=2), 0, atol=1e-10)


def test_laplace_gauss_law():
    # flux of grad phi out of a sphere = -(enclosed charge); a dipole adds 0
    y = np.array([[0.1, -0.2, 0.05], [2.0, 0.0, 0.0]])
    q = np.array([0.7, 5.0])                   # second charge is outside
    yd, d = np.array([[-0.1, 0.1, 0.0]]), np.array([[0.3, -0.4, 0.2]])
    pts, n, w = _fd.sphere_quadrature([0, 0, 0], 1.0)
    out = direct.laplace(y, q, yd, d, pts)
    flux = np.sum(w * np.sum(out[:, 1:4] * n, axis=1))
    assert abs(flux - (-0.7)) < 1e-10


def test_laplace_dipole_is_limit_of_two_charges():
    y = np.array([[0.05, 0.02, -0.03]])
    dvec = np.array([0.4, -0.1, 0.3])
    x = _probe()
    eps = 1e-4
    # +q at y + eps d/2, -q at y - eps d/2, q = 1/eps  ->  dipole d
    two = direct.laplace(np.array([y[0] + eps * dvec / 2, y[0] - eps * dvec / 2]),
                         [1 / eps, -1 / eps], trg=x)
    dip = direct.laplace(None, None, y, dvec[None], x)
    assert np.allclose(dip, two, rtol=1e-7, atol=1e-9)


def test_laplace_skips_coincident_points():
    y = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    out = direct.laplace(y, [1.0, 1.0], y, [[1.0, 0, 0], [0, 1.0, 0]], y)
    assert np.all(np.isfinite(out))


# ---------------------------------------------------------------- Stokeslet
def test_stokeslet_force_balance():
    # integral of sigma . n over a sphere enclosing a point force f equals -f
    y = np.array([[0.1, -0.05, 0.2]])
    f = np.array([[0.3, -1.2, 0.7]])
    fq = np.concatenate([f, [[0.0]]], axis=1)
    pts, n, w = _fd.sphere_quadrature([0, 0, 0], 1.0)
    sig = direct.traction(y, fq, None, None, pts).reshape(-1, 3, 3)
    tot = np.einsum("k,kij,kj->i", w, sig, n)
    assert np.allclose(tot, -f[0], atol=1e-10)


def test_stokeslet_divergence_free_and_stokes_equation():
    y, f = _pts(6), RNG.standard_normal((6, 3))
    fq = np.concatenate([f, np.zeros((6, 1))], axis=1)
    x = _probe()
    u = lambda xx: direct.stokeslet(y, f, xx)
    J = _fd.grad(u, x)
    div = np.trace(J, axis1=1, axis2=2)
    assert np.max(np.abs(div)) < 1e-9 * np.max(np.abs(J))
    # lap u = grad p (mu = 1) away from the sources
    lap = _fd.laplacian(u, x, h=2e-3)
    gp = _fd.grad(lambda xx: direct.pvel(y, fq, None, None, xx)[:, :1], x)[:, 0, :]
    assert np.allclose(lap, gp, rtol=1e-6, atol=1e-8)


def test_stokeslet_equals_pvel_velocity():
    y, f = _pts(7), RNG.standard_normal((7, 3))
    fq = np.concatenate([f, np.zeros((7, 1))], axis=1)
    x = _probe()
    assert np.allclose(direct.stokeslet(y, f, x), direct.pvel(y, fq, None, None, x)[:, 1:],
                       rtol=1e-14, atol=1e-15)


def test_stokeslet_reciprocity():
    # G symmetric and even in r: f'.U(f) = f.U(f')
    ya, fa = _pts(5), RNG.standard_normal((5, 3))
    yb, fb = _pts(4, 0.5, 0.9), RNG.standard_normal((4, 3))
    lhs = np.sum(fb * direct.stokeslet(ya, fa, yb))
    rhs = np.sum(fa * direct.stokeslet(yb, fb, ya))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# ---------------------------------------------------------------- RPY
def test_rpy_b0_is_stokeslet_and_laplacian_is_fd():
    y, f = _pts(5), RNG.standard_normal((5, 3))
    x = _probe()
    out = direct.rpy(y, np.concatenate([f, np.zeros((5, 1))], 1), x)
    assert np.allclose(out[:, :3], direct.stokeslet(y, f, x), rtol=1e-14, atol=1e-15)
    lap = _fd.laplacian(lambda xx: direct.stokeslet(y, f, xx), x, h=2e-3)
    assert np.allclose(out[:, 3:], lap, rtol=1e-6, atol=1e-8)


def test_rpy_operator_identity_and_far_field():
    # G^RPY f = G f + (b^2/6) lap G f, and lap of the RPY field is lap G f
    y, f = _pts(5), RNG.standard_normal((5, 3))
    b = RNG.uniform(0.01, 0.05, 5)
    x = _probe()
    out = direct.rpy(y, np.concatenate([f, b[:, None]], 1), x)
    u0 = direct.stokeslet(y, f, x)
    lap_each = np.stack([direct.rpy(y[i:i + 1], np.concatenate([f[i:i + 1], [[0.0]]], 1), x)[:, 3:]
                         for i in range(5)])
    expect = u0 + np.einsum("i,ink->nk", b ** 2 / 6, lap_each)
    assert np.allclose(out[:, :3], expect, rtol=1e-13, atol=1e-15)
    assert np.allclose(out[:, 3:], lap_each.sum(0), rtol=1e-13, atol=1e-15)
    # relative RPY correction decays like (b/r)^2
    one = np.array([[0.0, 0, 0]])
    fb = np.array([[1.0, 0.5, -0.3, 0.05]])
    errs = []
    for R in (1.0, 2.0, 4.0):
        xr = np.array([[R, 0.3 * R, -0.2 * R]])
        a = direct.rpy(one, fb, xr)[:, :3]
        s = direct.stokeslet(one, fb[:, :3], xr)
        errs.append(np.linalg.norm(a - s) / np.linalg.norm(s))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=1e-6)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=1e-6)


# ---------------------------------------------------------------- regularized Stokeslet
def test_stokes_reg_eps0_is_stokeslet():
    y, f = _pts(6), RNG.standard_normal((6, 3))
    x = _probe()
    out = direct.stokes_reg(y, np.concatenate([f, np.zeros((6, 1))], 1), x)
    assert np.allclose(out, direct.stokeslet(y, f, x), rtol=1e-14, atol=1e-15)


def test_stokes_reg_far_field_is_rpy_with_matching_radius():
    # for r >> eps: G^eps = G + (eps^2/2) (delta/r^3 - 3 r r/r^5)/(8 pi) + O(eps^4/r^5),
    # i.e. the RPY far field with b^2 = 3 eps^2/2
    one = np.array([[0.0, 0, 0]])
    f = np.array([[0.4, -1.0, 0.6]])
    eps = 0.01
    fe = np.concatenate([f, [[eps]]], 1)
    fb = np.concatenate([f, [[np.sqrt(1.5) * eps]]], 1)
    rel = []
    for R in (0.1, 0.2, 0.4):
        x = np.array([[R, -0.4 * R, 0.7 * R]])
        ue = direct.stokes_reg(one, fe, x)
        rest = ue - direct.rpy(one, fb, x)[:, :3]
        rel.append(np.linalg.norm(rest) / np.linalg.norm(ue - direct.stokeslet(one, f, x)))
    # the remainder relative to the eps^2 term falls like (eps/r)^2
    assert rel[0] < 0.05
    assert rel[0] / rel[1] == pytest.approx(4.0, rel=2e-2)
    assert rel[1] / rel[2] == pytest.approx(4.0, rel=2e-2)


def test_stokes_reg_solves_stokes_with_the_blob_force():
    # u = G^eps f is the Stokes flow of the force density psi^eps f with the
    # blob psi^eps = 15 eps^4 / (8 pi (r^2+eps^2)^(7/2)) (Sec. II.B): div u = 0
    # and lap u - grad p + psi^eps f = 0, with the pressure of this blob
    # p = (f.r)(2 r^2 + 5 eps^2) / (8 pi (r^2+eps^2)^(5/2)), checked inside the blob core
    y = np.array([[0.05, -0.02, 0.03]])
    f = np.array([[0.3, 0.8, -0.5]])
    eps = 0.2
    fe = np.concatenate([f, [[eps]]], 1)
    x = y + np.array([[0.1, 0.05, -0.08], [-0.15, 0.2, 0.1], [0.3, -0.1, 0.25], [0.02, 0.01, -0.03]])
    u = lambda xx: direct.stokes_reg(y, fe, xx)

    def p(xx):
        r = xx - y
        rr = np.sum(r * r, axis=1)
        return ((r @ f[0]) * (2 * rr + 5 * eps ** 2) / (8 * np.pi * (rr + eps ** 2) ** 2.5))[:, None]

    J = _fd.grad(u, x, h=1e-3)
    # the 4th-order difference error here is ~h^4 |u^(5)| ~ 1e-9 of |grad u|
    assert np.max(np.abs(np.trace(J, axis1=1, axis2=2))) < 1e-8 * np.max(np.abs(J))
    lap = _fd.laplacian(u, x, h=1e-3)
    gp = _fd.grad(p, x, h=1e-3)[:, 0, :]
    rr = np.sum((x - y) ** 2, axis=1)
    psi = 15 * eps ** 4 / (8 * np.pi * (rr + eps ** 2) ** 3.5)
    resid = lap - gp + psi[:, None] * f
    assert np.max(np.abs(resid)) < 1e-7 * np.max(np.abs(psi[:, None] * f))


def test_stokes_reg_reciprocity_and_bounded_self_term():
    ya, fa = _pts(5), RNG.standard_normal((5, 3))
    yb, fb = _pts(4, 0.5, 0.9), RNG.standard_normal((4, 3))
    e = 0.05
    ea = np.concatenate([fa, np.full((5, 1), e)], 1)
    eb = np.concatenate([fb, np.full((4, 1), e)], 1)
    lhs = np.sum(fb * direct.stokes_reg(ya, ea, yb))
    rhs = np.sum(fa * direct.stokes_reg(yb, eb, ya))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # a coincident pair with eps > 0 is finite: u = f / (4 pi eps)
    one = np.array([[0.2, 0.3, 0.4]])
    got = direct.stokes_reg(one, np.array([[1.0, -2.0, 0.5, e]]), one)
    assert np.allclose(got, np.array([[1.0, -2.0, 0.5]]) / (4 * np.pi * e), rtol=1e-14)


def _curl(fun, x, h=1e-3):
    J = _fd.grad(fun, x, h=h)            # J[n, i, l] = d u_i / d x_l
    return np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)


def test_stokes_reg_ft_parts():
    # force part = regularized Stokeslet; torque velocity = (1/2) curl of the
    # regularized Stokeslet of the torque (the regularized rotlet); angular
    # velocity = (1/2) curl u of the whole field (force and torque parts)
    y = _pts(4)
    f, t = RNG.standard_normal((4, 3)), RNG.standard_normal((4, 3))
    eps = RNG.uniform(0.05, 0.2, 4)
    x = _probe()
    fe = np.concatenate([f, eps[:, None]], 1)
    te = np.concatenate([t, eps[:, None]], 1)
    only_f = direct.stokes_reg_ft(y, np.concatenate([f, 0 * t, eps[:, None]], 1), x)
    assert np.allclose(only_f[:, :3], direct.stokes_reg(y, fe, x), rtol=1e-14, atol=1e-15)
    only_t = direct.stokes_reg_ft(y, np.concatenate([0 * f, t, eps[:, None]], 1), x)
    rot = 0.5 * _curl(lambda xx: direct.stokes_reg(y, te, xx), x)
    assert np.allclose(only_t[:, :3], rot, rtol=1e-7, atol=1e-9 * np.abs(rot).max())
    fte = np.concatenate([f, t, eps[:, None]], 1)
    both = direct.stokes_reg_ft(y, fte, x)
    w = 0.5 * _curl(lambda xx: direct.stokes_reg_ft(y, fte, xx)[:, :3], x)
    assert np.allclose(both[:, 3:], w, rtol=1e-7, atol=1e-9 * np.abs(w).max())
    assert np.allclose(both, only_f + only_t, rtol=1e-13, atol=1e-15)


def test_stokes_reg_ft_eps0_rotlet():
    y, t = _pts(3), RNG.standard_normal((3, 3))
    x = _probe()
    out = direct.stokes_reg_ft(y, np.concatenate([0 * t, t, np.zeros((3, 1))], 1), x)
    r = x[:, None, :] - y[None, :, :]
    rn = np.linalg.norm(r, axis=2)
    expect = np.sum(np.cross(t[None, :, :], r) / rn[:, :, None] ** 3, axis=1) / (8 * np.pi)
    assert np.allclose(out[:, :3], expect, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- double layer / PVel
def test_double_layer_net_flux():
    # flux of u out of any sphere around a double-layer source = -tr(D)/2 (Sec. II.C)
    y = np.array([[0.05, -0.1, 0.02]])
    D = RNG.standard_normal((1, 9))
    for R in (0.5, 1.0, 2.0):
        pts, n, w = _fd.sphere_quadrature([0, 0, 0], R, 64, 128)
        u = direct.pvel(None, None, y, D, pts)[:, 1:]
        flux = np.sum(w * np.sum(u * n, axis=1))
        assert abs(flux - (-0.5 * (D[0, 0] + D[0, 4] + D[0, 8]))) < 1e-9


def test_source_flux_and_no_pressure():
    # q is twice the physical source: flux of the q-flow is -q/2, no pressure
    y = np.array([[0.0, 0.1, -0.1]])
    fq = np.array([[0.0, 0.0, 0.0, 1.3]])
    pts, n, w = _fd.sphere_quadrature([0, 0, 0], 1.0)
    out = direct.pvel(y, fq, None, None, pts)
    assert np.max(np.abs(out[:, 0])) == 0.0
    flux = np.sum(w * np.sum(out[:, 1:] * n, axis=1))
    assert abs(flux - (-0.65)) < 1e-10


def test_double_layer_velocity_is_stokeslet_traction():
    # sigma_ij(f) = 2 T_ijk f_k: the Stokeslet's stress (by finite differences
    # of its p and u) equals twice the DL velocity with D = e_j f^T
    y = np.zeros((1, 3))
    f = np.array([0.4, -0.7, 0.2])
    fq = np.concatenate([f, [0.0]])[None]
    x = _probe()
    pu = lambda xx: direct.pvel(y, fq, None, None, xx)
    J = _fd.grad(lambda xx: pu(xx)[:, 1:], x)
    p = pu(x)[:, 0]
    sig = -p[:, None, None] * np.eye(3) + J + np.transpose(J, (0, 2, 1))
    for j in range(3):
        D = np.zeros((3, 3))
        D[j, :] = f
        u = direct.pvel(None, None, y, D.reshape(1, 9), x)[:, 1:]
        assert np.allclose(sig[:, :, j], 2 * u, rtol=1e-8, atol=1e-10)


def test_double_layer_stokes_equations():
    y, D = _pts(4), RNG.standard_normal((4, 9))
    x = _probe()
    fun = lambda xx: direct.pvel(None, None, y, D, xx)
    J = _fd.grad(lambda xx: fun(xx)[:, 1:], x)
    assert np.max(np.abs(np.trace(J, axis1=1, axis2=2))) < 1e-9 * np.max(np.abs(J))
    lap = _fd.laplacian(lambda xx: fun(xx)[:, 1:], x, h=2e-3)
    gp = _fd.grad(lambda xx: fun(xx)[:, :1], x)[:, 0, :]
    assert np.allclose(lap, gp, rtol=1e-6, atol=1e-8)
    lapp = _fd.laplacian(lambda xx: fun(xx)[:, :1], x, h=2e-3)
    assert np.max(np.abs(lapp)) < 1e-6 * np.max(np.abs(gp))


# ---------------------------------------------------------------- traction
@pytest.mark.parametrize("which", ["sl", "dl"])
def test_traction_is_stress_of_pvel_flow(which):
    y = _pts(4)
    fq = RNG.standard_normal((4, 4))
    D = RNG.standard_normal((4, 9))
    args = (y, fq, None, None) if which == "sl" else (None, None, y, D)
    x = _probe()
    pu = lambda xx: direct.pvel(*args, xx)
    J = _fd.grad(lambda xx: pu(xx)[:, 1:], x)
    p = pu(x)[:, 0]
    sig = -p[:, None, None] * np.eye(3) + J + np.transpose(J, (0, 2, 1))
    out = direct.traction(*args, x).reshape(-1, 3, 3)
    assert np.allclose(out, sig, rtol=1e-8, atol=1e-10)


def test_stresslet_special_case_pressure():
    # a trace-free symmetric D (stresslet) has p = -3 r.S.r/(4 pi r^5): the
    # trace term of the DL pressure vanishes, and u is unchanged by D -> D^T
    A = RNG.standard_normal((3, 3))
    S = 0.5 * (A + A.T)
    S -= np.trace(S) / 3 * np.eye(3)
    y = np.zeros((1, 3))
    x = _probe()
    a = direct.pvel(None, None, y, S.reshape(1, 9), x)
    b = direct.pvel(None, None, y, S.T.reshape(1, 9), x)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-15)
    # D = I is a pure source: no pressure
    c = direct.pvel(None, None, y, np.eye(3).reshape(1, 9), x)
    assert np.allclose(c[:, 0], 0, atol=1e-14)


def test_pvel_derivatives_are_fd_of_pvel():
    # grad p, grad u and lap u of the (p, u) field, SL (f, q) and DL D together
    y, fq = _pts(4), RNG.standard_normal((4, 4))
    yd, D = _pts(3, 0.4, 0.8), RNG.standard_normal((3, 9))
    x = _probe()
    pu = lambda xx: direct.pvel(y, fq, yd, D, xx)
    g = direct.pvel_grad(y, fq, yd, D, x)
    lap = direct.pvel_grad(y, fq, yd, D, x, lap=True)
    assert np.allclose(g[:, :4], pu(x), rtol=1e-13, atol=1e-15)
    assert np.allclose(lap[:, :4], pu(x), rtol=1e-13, atol=1e-15)
    J = _fd.grad(pu, x, h=1e-3)                    # [n, k, j] = d (p,u)_k / dx_j
    assert np.allclose(g[:, 4:7], J[:, 0, :], rtol=1e-7, atol=1e-9 * np.abs(J).max())
    assert np.allclose(g[:, 7:].reshape(-1, 3, 3), J[:, 1:, :], rtol=1e-7, atol=1e-9 * np.abs(J).max())
    L = _fd.laplacian(lambda xx: pu(xx)[:, 1:], x, h=2e-3)
    assert np.allclose(lap[:, 4:], L, rtol=1e-6, atol=1e-8 * np.abs(L).max())
    # Stokes equations (mu = 1): lap u = grad p, div u = 0 (q = 0 here)
    fq0 = fq.copy()
    fq0[:, 3] = 0
    g0 = direct.pvel_grad(y, fq0, yd, D, x)
    l0 = direct.pvel_grad(y, fq0, yd, D, x, lap=True)
    assert np.allclose(l0[:, 4:], g0[:, 4:7], rtol=1e-10, atol=1e-12 * np.abs(g0[:, 4:7]).max())
    assert np.allclose(np.trace(g0[:, 7:].reshape(-1, 3, 3), axis1=1, axis2=2), 0, atol=1e-10 * np.abs(g0).max())


def _quad_as_charges(y, Q, h):
    # Q_jk d_j d_k L(x - y) = Q_jk d/dy_j d/dy_k L(x - y): the central difference
    # in y puts charges Q_jk/(4 h^2) (+, -, -, +) at y +- h e_j +- h e_k
    pos, q = [], []
    for s in range(len(y)):
        for j in range(3):
            for k in range(3):
                for sj, sk, sg in ((1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)):
                    p = y[s].copy()
                    p[j] += sj * h
                    p[k] += sk * h
                    pos.append(p)
                    q.append(sg * Q[s, 3 * j + k] / (4 * h * h))
    return np.array(pos), np.array(q)


def test_quadrupole_is_the_limit_of_charges():
    # every output (phi, grad phi, Hessian) against the charge kernel applied
    # to the finite-difference charges, Richardson-extrapolated (error O(h^4))
    y, Q = _pts(3), RNG.standard_normal((3, 9))
    x = _probe()
    got = direct.laplace_quad(y, Q, x)
    ref = []
    for h in (2e-3, 4e-3):
        pos, q = _quad_as_charges(y, Q, h)
        ref.append(direct.laplace(pos, q, None, None, x, hess=True))
    ref = (4 * ref[0] - ref[1]) / 3
    assert np.allclose(got, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_quadrupole_invariants():
    y, x = _pts(4), _probe()
    # the isotropic and the antisymmetric parts of Q make no field
    assert np.abs(direct.laplace_quad(y, np.tile(np.eye(3).ravel(), (4, 1)), x)).max() < 1e-13
    A = RNG.standard_normal((4, 3, 3))
    assert np.abs(direct.laplace_quad(y, (A - A.transpose(0, 2, 1)).reshape(4, 9), x)).max() < 1e-13
    # harmonic: zero Hessian trace; grad phi = FD of phi
    Q = RNG.standard_normal((4, 9))
    g = direct.laplace_quad(y, Q, x)
    assert np.allclose(g[:, 4] + g[:, 7] + g[:, 9], 0, atol=1e-12 * np.abs(g).max())
    J = _fd.grad(lambda xx: direct.laplace_quad(y, Q, xx)[:, :1], x, h=1e-3)
    assert np.allclose(g[:, 1:4], J[:, 0, :], rtol=1e-7, atol=1e-9 * np.abs(J).max())


def test_rel_l2():
    assert direct.rel_l2([1.0, 0.0], [1.0, 0.0]) == 0.0
    assert direct.rel_l2([2.0, 0.0], [1.0, 0.0]) == 1.0
