"""Pins for the oracle's triply periodic Stokeslet (Ewald, Hasimoto split).

* the sum does not depend on the split parameter xi (real and reciprocal
  parts trade places), at targets off the sources and on them (self term);
* it is periodic in the targets and invariant when sources and targets move
  together;
* next to a source it is the free-space Stokeslet (the normalisation
  1/(8 pi)): r u(y + r e) -> (I + e e^T) f / (8 pi) as r -> 0;
* it is divergence free (central differences).
"""
import numpy as np
import pytest

from oracle.stokes_periodic import stokeslet_periodic


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    y = rng.random((n, 3))
    f = rng.standard_normal((n, 3))
    f -= f.mean(axis=0)                      # zero net force
    return rng, y, f


def test_split_parameter_independence():
    rng, y, f = _problem(40, 1)
    x = np.concatenate([rng.random((30, 3)), y[:6]])
    u = [stokeslet_periodic(y, f, x, xi=xi) for xi in (3.0, 5.0, 8.0)]
    scale = np.abs(u[0]).max()
    assert np.abs(u[1] - u[0]).max() < 1e-13 * scale
    assert np.abs(u[2] - u[0]).max() < 1e-13 * scale


def test_periodic_and_translation_invariant():
    rng, y, f = _problem(30, 2)
    x = rng.random((20, 3))
    # keep targets away from sources so that rounding of shifted positions is harmless
    d = np.min(np.linalg.norm(x[:, None] - y[None], axis=2), axis=1)
    x = x[d > 0.05]
    u = stokeslet_periodic(y, f, x)
    up = stokeslet_periodic(y, f, x + np.array([1.0, -2.0, 1.0]))
    assert np.abs(up - u).max() < 1e-12 * np.abs(u).max()
    s = np.array([0.37, 0.81, 0.13])
    ut = stokeslet_periodic((y + s) % 1.0, f, (x + s) % 1.0)
    assert np.abs(ut - u).max() < 1e-12 * np.abs(u).max()


def test_free_space_limit_next_to_a_source():
    rng, y, f = _problem(20, 3)
    e = np.array([0.6, 0.0, 0.8])
    want = (f[0] + e * (e @ f[0])) / (8 * np.pi)
    for r in (1e-5, 1e-6):
        got = stokeslet_periodic(y, f, (y[0] + r * e)[None])[0] * r
        assert np.abs(got - want).max() < 30 * r * np.abs(want).max()


def test_divergence_free():
    rng, y, f = _problem(25, 4)
    x = rng.random((6, 3))
    h = 1e-4
    div = np.zeros(len(x))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        div += (stokeslet_periodic(y, f, x + e)[:, k] - stokeslet_periodic(y, f, x - e)[:, k]) / (2 * h)
    grad_scale = np.abs(stokeslet_periodic(y, f, x)).max() / 0.05
    assert np.abs(div).max() < 1e-6 * grad_scale


def test_laplacian_split_parameter_independence():
    from oracle.stokes_periodic import stokes_lap_periodic
    rng, y, f = _problem(40, 7)
    x = np.concatenate([rng.random((20, 3)), y[:5]])
    w = rng.uniform(0.5, 2.0, len(y))
    a = [stokes_lap_periodic(y, f, w, x, xi=xi) for xi in (3.0, 5.0, 8.0)]
    scale = np.abs(a[0]).max()
    assert np.abs(a[1] - a[0]).max() < 1e-13 * scale
    assert np.abs(a[2] - a[0]).max() < 1e-13 * scale


def test_laplacian_is_the_laplacian_of_the_flow():
    # Richardson-extrapolated central second differences of the periodic
    # Stokeslet sum, at targets away from the sources
    from oracle.stokes_periodic import stokes_lap_periodic
    rng, y, f = _problem(30, 8)
    x = rng.random((40, 3))
    x = x[np.min(np.linalg.norm(((x[:, None] - y[None]) + 0.5) % 1.0 - 0.5, axis=2), axis=1) > 0.1][:6]

    def fd(h):
        lap = -6.0 * stokeslet_periodic(y, f, x)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            lap += stokeslet_periodic(y, f, x + e) + stokeslet_periodic(y, f, x - e)
        return lap / h ** 2

    lap = (4.0 * fd(1e-3) - fd(2e-3)) / 3.0
    ref = stokes_lap_periodic(y, f, np.ones(len(y)), x)
    assert np.abs(lap - ref).max() < 1e-5 * np.abs(ref).max()


def test_rpy_without_radii_is_the_stokeslet():
    from oracle.stokes_periodic import rpy_periodic, stokes_lap_periodic
    rng, y, f = _problem(30, 9)
    x = np.concatenate([rng.random((10, 3)), y[:4]])
    out = rpy_periodic(y, np.concatenate([f, np.zeros((len(f), 1))], 1), x)
    assert np.allclose(out[:, :3], stokeslet_periodic(y, f, x), rtol=0, atol=1e-14 * np.abs(out[:, :3]).max())
    assert np.allclose(out[:, 3:], stokes_lap_periodic(y, f, np.ones(len(y)), x), rtol=0, atol=0)


def _dl_problem(seed):
    rng = np.random.default_rng(seed)
    sl = rng.random((15, 3))
    fq = rng.standard_normal((15, 4))
    fq -= fq.mean(axis=0)                       # zero net force and net source
    dl = rng.random((10, 3))
    D = rng.standard_normal((10, 9))
    D[:, [0, 4, 8]] -= (D[:, 0] + D[:, 4] + D[:, 8]).mean() / 3.0   # zero net tr D
    return rng, sl, fq, dl, D


def test_double_layer_split_parameter_independence():
    from oracle.stokes_periodic import stokes_dl_periodic
    rng, _, _, dl, D = _dl_problem(21)
    x = np.concatenate([rng.random((10, 3)), dl[:3]])
    a = [stokes_dl_periodic(dl, D, x, xi=xi) for xi in (3.0, 5.0, 8.0)]
    scale = np.abs(a[0]).max()
    assert np.abs(a[1] - a[0]).max() < 1e-13 * scale
    assert np.abs(a[2] - a[0]).max() < 1e-13 * scale


def test_double_layer_is_the_limit_of_force_pairs():
    # grad G : D^s = sum_k d_k G D^s_{.k}: pairs -D^s_{.k} at y + h e_k and
    # +D^s_{.k} at y - h e_k of the (pinned) periodic Stokeslet, over 2h
    from oracle.stokes_periodic import stokes_dl_periodic
    rng, _, _, y, D = _dl_problem(22)
    Ds = 0.5 * (D + D.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9))
    x = rng.random((5, 3))
    h = 1e-5
    u = np.zeros((5, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        F = np.concatenate([-Ds.reshape(-1, 3, 3)[:, :, k], Ds.reshape(-1, 3, 3)[:, :, k]])
        u += stokeslet_periodic(np.concatenate([y + e, y - e]), F, x) / (2 * h)
    ref = stokes_dl_periodic(y, D, x)
    assert np.abs(u - ref).max() < 1e-6 * np.abs(ref).max()


def test_pvel_next_to_sources():
    from oracle.stokes_periodic import pvel_periodic
    rng, sl, fq, dl, D = _dl_problem(23)
    e = np.array([0.6, 0.0, 0.8])
    r = 1e-5
    Dm = 0.5 * (D[0].reshape(3, 3) + D[0].reshape(3, 3).T)
    out = pvel_periodic(sl, fq, dl, D, (dl[0] + r * e)[None])[0]
    want_u = -(3.0 / (8 * np.pi)) * e * (e @ Dm @ e)
    want_p = (-3.0 * (e @ Dm @ e) + np.trace(Dm)) / (4 * np.pi)
    assert np.abs(out[1:] * r ** 2 - want_u).max() < 1e-4 * np.abs(want_u).max()
    assert abs(out[0] * r ** 3 - want_p) < 1e-4 * abs(want_p)
    out = pvel_periodic(sl, fq, dl, D, (sl[0] + r * e)[None])[0]
    f, q = fq[0, :3], fq[0, 3]
    assert abs(out[0] * r ** 2 - (e @ f) / (4 * np.pi)) < 1e-3 * abs(e @ f) / (4 * np.pi)
    want = (f + e * (e @ f) - q * e / r) / (8 * np.pi)     # G f / r and the source term
    assert np.abs(out[1:] * r - want).max() < 1e-3 * np.abs(want).max()


def test_pvel_divergence_free():
    from oracle.stokes_periodic import pvel_periodic
    rng, sl, fq, dl, D = _dl_problem(24)
    x = rng.random((4, 3))
    h = 1e-4
    div = np.zeros(len(x))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        div += (pvel_periodic(sl, fq, dl, D, x + e)[:, 1 + k] - pvel_periodic(sl, fq, dl, D, x - e)[:, 1 + k]) / (2 * h)
    grad_scale = np.abs(pvel_periodic(sl, fq, dl, D, x)[:, 1:]).max() / 0.05
    assert np.abs(div).max() < 1e-6 * grad_scale


def _away_from(sources, k, rng, dmin=0.1):
    """k points at least dmin from every source image."""
    out = []
    while len(out) < k:
        c = rng.random(3)
        d = c - sources
        d -= np.round(d)
        if np.min(np.linalg.norm(d, axis=1)) >= dmin:
            out.append(c)
    return np.array(out)


def test_pvel_derivatives_satisfy_the_stokes_equations():
    # lap u (second differences of u) = grad p (first differences of p): the
    # velocity's and the pressure's Ewald sums are separate, so this ties
    # them together; and div u = tr grad u = 0 between the sources
    from oracle.stokes_periodic import pvel_derivs_periodic
    rng, sl, fq, dl, D = _dl_problem(25)
    x = _away_from(np.concatenate([sl, dl]), 4, rng)
    g = pvel_derivs_periodic(sl, fq, dl, D, x, kind="PVelGrad")
    lap = pvel_derivs_periodic(sl, fq, dl, D, x, kind="PVelLaplacian")
    assert np.allclose(g[:, :4], lap[:, :4], rtol=1e-13, atol=0)
    scale = np.abs(g[:, 4:7]).max()
    assert np.abs(lap[:, 4:7] - g[:, 4:7]).max() < 1e-6 * scale
    gu = g[:, 7:].reshape(-1, 3, 3)
    assert np.abs(np.trace(gu, axis1=1, axis2=2)).max() < 1e-8 * np.abs(gu).max()
    sig = pvel_derivs_periodic(sl, fq, dl, D, x, kind="Traction").reshape(-1, 3, 3)
    assert np.allclose(sig, sig.transpose(0, 2, 1), rtol=0, atol=1e-12 * np.abs(sig).max())
    # tr sigma = -3 p + 2 div u
    assert np.abs(np.trace(sig, axis1=1, axis2=2) + 3 * g[:, 0]).max() < 1e-7 * np.abs(gu).max()


def test_pvel_derivatives_converge_at_fourth_order():
    # halving the step divides the change by about 16 (five-point formulas),
    # and at h = 5e-4, 0.1 from every source, the derivatives are settled to
    # a few 1e-8
    from oracle.stokes_periodic import pvel_derivs_periodic
    rng, sl, fq, dl, D = _dl_problem(26)
    x = _away_from(np.concatenate([sl, dl]), 3, rng)
    a, b, c = (pvel_derivs_periodic(sl, fq, dl, D, x, h=h, kind="PVelGrad")[:, 4:] for h in (2e-3, 1e-3, 5e-4))
    d1, d2 = np.abs(a - b).max(), np.abs(b - c).max()
    assert 10.0 < d1 / d2 < 25.0
    assert d2 < 5e-8 * np.abs(c).max()


@pytest.mark.parametrize("layer", ["sl", "dl"])
def test_pvel_derivatives_next_to_a_source(layer):
    # 1e-3 from one source its own free-space term (the oracle's direct
    # PVelGrad and Traction kernels) dominates by 1e5 : 1 or more; the rest
    # of the periodic sum is smooth there (a wrong sign, index or layout
    # would leave an O(1) relative difference)
    from oracle import direct
    from oracle.stokes_periodic import pvel_derivs_periodic
    rng, sl, fq, dl, D = _dl_problem(27)
    r, e = 1e-3, np.array([0.48, -0.6, 0.64])
    y = (sl if layer == "sl" else dl)[0]
    x = (y + r * e)[None]
    one = dict(sl=sl[:1], fq=fq[:1]) if layer == "sl" else dict(dl=dl[:1], D=D[:1])
    for kind in ("PVelGrad", "Traction"):
        got = pvel_derivs_periodic(sl, fq, dl, D, x, h=1e-5, kind=kind)
        if kind == "PVelGrad":
            want = direct.pvel_grad(one.get("sl"), one.get("fq"), one.get("dl"), one.get("D"), x)
            got, want = got[:, 4:], want[:, 4:]            # the derivatives
        else:
            want = direct.traction(one.get("sl"), one.get("fq"), one.get("dl"), one.get("D"), x)
        assert np.abs(got - want).max() < 1e-5 * np.abs(want).max(), kind


def _reg_problem(n, seed, eps=(1e-3, 3e-3)):
    rng = np.random.default_rng(seed)
    y = rng.random((n, 3))
    f = rng.standard_normal((n, 3))
    f -= f.mean(axis=0)
    return rng, y, np.concatenate([f, rng.uniform(*eps, (n, 1))], 1)


def test_regularized_without_blobs_is_the_stokeslet():
    from oracle.stokes_periodic import stokes_reg_periodic
    rng, y, fe = _reg_problem(30, 41)
    x = np.concatenate([rng.random((10, 3)), y[:4]])
    fe[:, 3] = 0.0
    x = x[np.min(np.linalg.norm((x[:, None] - y[None] + 0.5) % 1.0 - 0.5, axis=2), axis=1) > 0]
    got = stokes_reg_periodic(y[:], fe, x[:10])
    assert np.allclose(got, stokeslet_periodic(y, fe[:, :3], x[:10]), rtol=0, atol=1e-13 * np.abs(got).max())


def test_regularized_remainder_converges_absolutely():
    # the remainder's images beyond the nearest 27 change nothing at FP64
    from oracle.stokes_periodic import stokes_reg_periodic
    rng, y, fe = _reg_problem(40, 42)
    x = np.concatenate([rng.random((10, 3)), y[:5]])
    a = stokes_reg_periodic(y, fe, x, images=1)
    b = stokes_reg_periodic(y, fe, x, images=2)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_regularized_far_from_blobs_is_rpy_with_matching_radius():
    # b^2 = 3 eps^2 / 2 gives (1 + b^2/6 lap) G = G + (eps^2/4) lap G: the two
    # periodic sums (one through the RPY oracle) differ by O(eps^4/r^5) at
    # targets 0.1 from every blob: below 1e-5 per unit force for eps <= 3e-3,
    # while a wrong eps^2 term would leave O(eps^2/r^3), about 1e-2
    from oracle.stokes_periodic import rpy_periodic, stokes_reg_periodic
    rng, y, fe = _reg_problem(40, 43)
    x = []
    while len(x) < 6:
        c = rng.random(3)
        d = c - y
        d -= np.round(d)
        if np.min(np.linalg.norm(d, axis=1)) > 0.1:
            x.append(c)
    x = np.array(x)
    fb = np.concatenate([fe[:, :3], np.sqrt(1.5) * fe[:, 3:]], 1)
    got = stokes_reg_periodic(y, fe, x)
    assert np.abs(got - rpy_periodic(y, fb, x)[:, :3]).max() < 1e-6 * np.abs(got).max()


def test_regularized_on_a_blob():
    # a target on a blob: its own G^eps(0) f = 2 f/(8 pi eps) plus the smooth
    # rest, which the target 1e-7 off the blob shares to O(1e-7 / eps)
    from oracle import direct
    from oracle.stokes_periodic import stokes_reg_periodic
    rng, y, fe = _reg_problem(30, 44)
    on = stokes_reg_periodic(y, fe, y[:1])[0]
    near = stokes_reg_periodic(y, fe, y[:1] + 1e-7)[0]
    assert np.allclose(direct.stokes_reg(y[:1], fe[:1], y[:1])[0], 2 * fe[0, :3] / (8 * np.pi * fe[0, 3]))
    assert np.abs(on - near).max() < 1e-3 * np.abs(on).max()


def _curl_fd(fun, x, h=1e-3):
    """Curl of fun [m, 3] at x by five-point central differences."""
    J = np.zeros((len(x), 3, 3))                        # J[:, i, j] = d_j u_i
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, :, j] = (8 * (fun(x + e) - fun(x - e)) - (fun(x + 2 * e) - fun(x - 2 * e))) / (12 * h)
    return np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)


def test_rotlet_split_parameter_independence():
    from oracle.stokes_periodic import rotlet_periodic
    rng, y, t = _problem(30, 51)
    x = np.concatenate([rng.random((10, 3)), y[:4]])
    u = [rotlet_periodic(y, t, x, xi=xi) for xi in (4.0, 6.0, 9.0)]
    assert np.abs(u[1] - u[0]).max() < 1e-12 * np.abs(u[0]).max()
    assert np.abs(u[2] - u[0]).max() < 1e-12 * np.abs(u[0]).max()


def test_rotlet_is_half_the_curl_of_the_stokeslet_sum():
    from oracle.stokes_periodic import rotlet_periodic
    rng, y, t = _problem(30, 52)
    x = _away_from(y, 4, rng)
    want = 0.5 * _curl_fd(lambda p: stokeslet_periodic(y, t, p), x)
    got = rotlet_periodic(y, t, x)
    assert np.abs(got - want).max() < 1e-7 * np.abs(got).max()


def _ft_problem(n, seed):
    rng = np.random.default_rng(seed)
    y = rng.random((n, 3))
    ft = rng.standard_normal((n, 6))
    ft -= ft.mean(axis=0)
    return rng, y, np.concatenate([ft, rng.uniform(1e-3, 3e-3, (n, 1))], 1)


def test_regularized_ft_omega_is_half_the_curl_of_u():
    from oracle.stokes_periodic import stokes_reg_ft_periodic
    rng, y, fte = _ft_problem(25, 53)
    x = _away_from(y, 3, rng)
    got = stokes_reg_ft_periodic(y, fte, x)
    want = 0.5 * _curl_fd(lambda p: stokes_reg_ft_periodic(y, fte, p)[:, :3], x)
    assert np.abs(got[:, 3:] - want).max() < 1e-7 * np.abs(got[:, 3:]).max()


def test_regularized_ft_remainder_and_blob_value():
    from oracle import direct
    from oracle.stokes_periodic import stokes_reg_ft_periodic
    rng, y, fte = _ft_problem(25, 54)
    x = np.concatenate([rng.random((6, 3)), y[:3]])
    a = stokes_reg_ft_periodic(y, fte, x, images=1)
    b = stokes_reg_ft_periodic(y, fte, x, images=2)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    # on a blob: its own regularized value plus a smooth rest
    near = stokes_reg_ft_periodic(y, fte, y[:1] + 1e-7)[0]
    assert np.abs(a[6] - near).max() < 1e-3 * np.abs(a[6]).max()
    own = direct.stokes_reg_ft(y[:1], fte[:1], y[:1])[0]
    assert np.abs(own).max() > 0.1 * np.abs(a[6]).max()
