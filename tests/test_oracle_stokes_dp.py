"""Pins of the doubly periodic Stokes oracle (oracle/stokes_dp.*) against
facts that do not come from it:

* split independence: the Ewald parameter moves work between the real and
  spectral sums, the total must not change (on and off the sources);
* the plain image sum: for cells whose forces have zero sum and zero first
  moment the lattice sum converges absolutely (the far field is a force
  quadrupole, 1/r^3 over a plane); its Richardson-extrapolated square
  partial sums must equal the oracle;
* the sheet flow far from the sources: u_par -> +-(1/2A) sum_j f_j,par z_j
  above / below, u_z -> 0 (the k_par = 0 mode, independent of the split);
* incompressibility and the Laplacian output by central differences;
* periodicity in x and y, in-plane translation invariance, box scaling;
* the free-space Stokeslet next to a source (normalisation);
* RPY: b = 0 gives the Stokeslet; the net force is rejected.
"""
import numpy as np
import pytest

from oracle.stokes_dp import lap_g_dp, rpy_dp, stokeslet_dp, stokeslet_lap_dp

PI = np.pi


def G(r, f):
    """Free-space Stokeslet (I/r + r r^T/r^3)/(8 pi) f for rows of r [m, 3]."""
    rr = np.sqrt(np.sum(r * r, axis=1))
    rf = np.sum(r * f, axis=1)
    return (f / rr[:, None] + r * (rf / rr ** 3)[:, None]) / (8 * PI)


def cell(seed, n=24, L=1.0, zspan=1.0):
    rng = np.random.default_rng(seed)
    y = rng.random((n, 3)) * np.array([L, L, zspan])
    f = rng.standard_normal((n, 3))
    f -= f.mean(axis=0)
    return y, f


def quadrupole_cell(seed, L=1.0):
    """Forces with zero sum and zero first moment: pairs of opposite force
    pairs, f at y, -f at y + a, -f at y + b, f at y + a + b."""
    rng = np.random.default_rng(seed)
    ys, fs = [], []
    for _ in range(3):
        y0 = rng.random(3) * 0.5 * L
        a, b = 0.25 * L * rng.random(3), 0.25 * L * rng.random(3)
        f = rng.standard_normal(3)
        ys += [y0, y0 + a, y0 + b, y0 + a + b]
        fs += [f, -f, -f, f]
    return np.array(ys), np.array(fs)


def plain_sum(y, f, x, R, L=1.0):
    """sum_j sum_{|n_x|, |n_y| <= R} G(x - y_j - n L) f_j."""
    n = np.arange(-R, R + 1) * L
    shifts = np.stack(np.meshgrid(n, n, indexing="ij"), axis=-1).reshape(-1, 2)
    out = np.zeros((len(x), 3))
    for i, xi in enumerate(x):
        for yj, fj in zip(y, f):
            r = np.empty((len(shifts), 3))
            r[:, :2] = xi[:2] - yj[:2] - shifts
            r[:, 2] = xi[2] - yj[2]
            out[i] += np.sum(G(r, np.broadcast_to(fj, r.shape)), axis=0)
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_split_independence():
    y, f = cell(1)
    x = np.concatenate([y[:5], np.random.default_rng(2).random((6, 3))])
    ref = stokeslet_lap_dp(y, f, x, xi=4.0)
    for xi in (2.5, 7.0):
        got = stokeslet_lap_dp(y, f, x, xi=xi)
        assert rel(got[0], ref[0]) < 1e-13
        assert rel(got[1], ref[1]) < 1e-12


def test_plain_lattice_sum():
    # a force-quadrupole cell: the square partial sums converge like
    # 1/R + 1/R^2 + 1/R^3 + ...; Richardson over four sizes removes the first
    # three (measured: 2.4e-3 at R = 96, 1e-8 extrapolated)
    y, f = quadrupole_cell(3)
    x = np.random.default_rng(4).random((4, 3)) * np.array([1.0, 1.0, 0.8])
    s = [plain_sum(y, f, x, R) for R in (24, 48, 96, 192)]
    for order in (1, 2, 3):
        s = [(2 ** order * s[i + 1] - s[i]) / (2 ** order - 1) for i in range(len(s) - 1)]
    ref = stokeslet_dp(y, f, x)
    assert rel(s[0], ref) < 1e-7


def test_sheet_flow_far_from_the_sources():
    y, f = cell(5, zspan=0.6)
    A = 1.0
    m = np.sum(f[:, :2] * y[:, 2:3], axis=0) / (2 * A)      # (1/2A) sum f_par z_j
    # the in-plane modes decay like exp(-2 pi |dz|/L): 1e-15 beyond dz = 5.5
    up = stokeslet_dp(y, f, np.array([[0.3, 0.7, 6.5], [0.9, 0.1, 8.0]]))
    dn = stokeslet_dp(y, f, np.array([[0.3, 0.7, -6.0], [0.6, 0.2, -8.5]]))
    for u, sgn in ((up, 1.0), (dn, -1.0)):
        assert np.allclose(u[:, :2], sgn * m, rtol=1e-9, atol=1e-12 * np.abs(m).max())
        assert np.abs(u[:, 2]).max() < 1e-10 * np.abs(m).max()


def test_divergence_free_and_laplacian():
    y, f = cell(6)
    x0 = np.array([[0.51, 0.43, 0.37], [0.12, 0.88, 0.71]])
    for x in x0:
        assert np.min(np.linalg.norm(np.mod(y - x + 0.5, 1.0) - 0.5, axis=1)) > 0.02
    # central differences at steps h and h/2, Richardson-combined (O(h^4))
    def fd(h):
        div = np.zeros(len(x0))
        lap_fd = np.zeros((len(x0), 3))
        u0 = stokeslet_dp(y, f, x0)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            up, um = stokeslet_dp(y, f, x0 + e), stokeslet_dp(y, f, x0 - e)
            div += (up[:, k] - um[:, k]) / (2 * h)
            lap_fd += (up - 2 * u0 + um) / h ** 2
        return div, lap_fd
    (d1, l1), (d2, l2) = fd(1e-3), fd(5e-4)
    div, lap_fd = (4 * d2 - d1) / 3, (4 * l2 - l1) / 3
    grad_scale = np.abs(stokeslet_dp(y, f, x0)).max() / 0.02
    assert np.abs(div).max() < 1e-8 * grad_scale
    lap = stokeslet_lap_dp(y, f, x0)[1]
    assert rel(lap_fd, lap) < 1e-6


def test_periodicity_translation_and_scaling():
    y, f = cell(7)
    x = np.random.default_rng(8).random((5, 3))
    u = stokeslet_dp(y, f, x)
    assert rel(stokeslet_dp(y, f, x + np.array([1.0, -2.0, 0.0])), u) < 1e-13
    s = np.array([0.37, 0.81, 0.0])
    assert rel(stokeslet_dp(np.mod(y + s, 1.0), f, np.mod(x + s, 1.0)), u) < 1e-13
    # box of side 2.5: u_L(L x) = u_1(x) / L
    Ls = 2.5
    assert rel(stokeslet_dp(Ls * y, f, Ls * x, L=Ls), u / Ls) < 1e-13


def test_free_space_limit_next_to_a_source():
    y, f = cell(9)
    e = np.array([0.6, -0.3, 0.74])
    e /= np.linalg.norm(e)
    rest = []
    for d in (1e-3, 2e-3):
        x = y[:1] + d * e
        rest.append(stokeslet_dp(y, f, x)[0] - G((d * e)[None], f[:1])[0])
    # the remainder is smooth in d: it changes by O(d), while G itself is ~1/d
    assert np.abs(rest[0] - rest[1]).max() < 1e-2 * np.abs(G((1e-3 * e)[None], f[:1])).max() * 1e-2


def test_rpy_reduces_and_adds_the_laplacian():
    y, f = cell(10)
    x = np.random.default_rng(11).random((4, 3))
    b = np.random.default_rng(12).uniform(0.002, 0.005, len(y))
    out0 = rpy_dp(y, np.concatenate([f, 0 * b[:, None]], 1), x)
    u, lap = stokeslet_lap_dp(y, f, x)
    assert rel(out0[:, :3], u) < 1e-14 and rel(out0[:, 3:], lap) < 1e-14
    out = rpy_dp(y, np.concatenate([f, b[:, None]], 1), x)
    # u = sum (G + b^2/6 lap G) f: the Laplacian sum is linear in its forces
    # (and absolutely convergent: no net-force condition)
    lap_w = lap_g_dp(y, f * (b ** 2 / 6.0)[:, None], x)
    assert rel(out[:, :3], u + lap_w) < 1e-13
    assert rel(lap_g_dp(y, f, x), lap) < 1e-14


def test_rejects_net_force():
    y, f = cell(13)
    with pytest.raises(ValueError):
        stokeslet_dp(y, f + 1.0, y[:2])
