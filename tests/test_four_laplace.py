"""FP64 check of the 4-Laplace representation used on the GPU ML tree.

Stokes fields from four Laplace fields (Phi_1..3, Psi) of charges and
dipoles, with Psi carried relative to an origin c, must reproduce the oracle's
direct sums (Sec. II.B-C kernels) to round-off, for any origin:
  u_i = 1/2 [Phi_i - (x-c)_j d_i Phi_j + d_i Psi],  p = -d_j Phi_j,
  lap u_i = -d_i d_j Phi_j,  sigma_ij = -p delta_ij + d_i d_j [Psi - (x-c).Phi].
Sources: force f -> Phi_j charge f_j, Psi charge (y-c).f; source q -> Psi
charge q; RPY radius b -> Psi dipole (b^2/3) f; double layer D -> Phi_j
dipole -D^s_j., Psi dipole -D^s (y-c).
"""
import numpy as np
import pytest

from oracle import direct

RNG = np.random.default_rng(4242)


def laplace_fields(x, y, q, d):
    """Potential, gradient and Hessian of Laplace charges q [n] and dipoles
    d [n,3] at y, at targets x (FP64, L = 1/(4 pi r), dipole phi = d.r/(4 pi r^3))."""
    r = x[:, None, :] - y[None, :, :]
    rr = np.sum(r * r, axis=2)
    i1 = 1 / np.sqrt(rr)
    i3, i5, i7 = i1 ** 3, i1 ** 5, i1 ** 7
    c = 1 / (4 * np.pi)
    I = np.eye(3)
    dr = np.einsum("mni,ni->mn", r, d)
    phi = c * (i1 @ q + np.sum(dr * i3, axis=1))
    grad = c * (-np.einsum("mn,mni,n->mi", i3, r, q)
                + np.einsum("mn,ni->mi", i3, d) - 3 * np.einsum("mn,mni->mi", dr * i5, r))
    hess = c * (np.einsum("mn,mni,mnj,n->mij", 3 * i5, r, r, q) - np.einsum("mn,n,ij->mij", i3, q, I)
                - 3 * (np.einsum("mn,nj,mni->mij", i5, d, r) + np.einsum("mn,ni,mnj->mij", i5, d, r)
                       + np.einsum("mn,ij->mij", dr * i5, I))
                + 15 * np.einsum("mn,mni,mnj->mij", dr * i7, r, r))
    return phi, grad, hess


def stokes_from_4lap(x, y, c, f=None, q=None, b=None, D=None):
    n = len(y)
    qs = np.zeros((4, n))
    ds = np.zeros((4, n, 3))
    yc = y - c
    if f is not None:
        qs[:3] += f.T
        qs[3] += np.sum(yc * f, axis=1)
    if q is not None:
        qs[3] += q
    if b is not None:
        ds[3] += (b[:, None] ** 2 / 3) * f
    if D is not None:
        Ds = 0.5 * (D + np.transpose(D, (0, 2, 1)))
        for j in range(3):
            ds[j] -= Ds[:, j, :]
        ds[3] -= np.einsum("njk,nk->nj", Ds, yc)
    F = [laplace_fields(x, y, qs[k], ds[k]) for k in range(4)]
    Phi = np.stack([F[j][0] for j in range(3)], 1)            # [m, j]
    gPhi = np.stack([F[j][1] for j in range(3)], 2)           # [m, i, j] = d_i Phi_j
    hPhi = np.stack([F[j][2] for j in range(3)], 3)           # [m, i, k, j]
    gPsi, hPsi = F[3][1], F[3][2]
    X = x - c
    u = 0.5 * (Phi - np.einsum("mj,mij->mi", X, gPhi) + gPsi)
    p = -np.trace(gPhi, axis1=1, axis2=2)
    lap = -np.einsum("mijj->mi", hPhi)
    sig = -p[:, None, None] * np.eye(3) + hPsi - np.einsum("ml,mijl->mij", X, hPhi)
    return u, p, lap, sig


def _setup(n=6):
    y = RNG.uniform(-0.2, 0.2, (n, 3))
    d = RNG.standard_normal((5, 3))
    x = d / np.linalg.norm(d, axis=1)[:, None] * RNG.uniform(0.7, 1.5, (5, 1))
    return x, y


@pytest.mark.parametrize("origin", [np.zeros(3), np.array([0.3, -0.5, 0.8])])
def test_stokeslet_and_rpy(origin):
    x, y = _setup()
    f = RNG.standard_normal((6, 3))
    b = RNG.uniform(0.01, 0.05, 6)
    u, p, lap, _ = stokes_from_4lap(x, y, origin, f=f, b=b)
    ref = direct.rpy(y, np.concatenate([f, b[:, None]], 1), x)
    assert np.allclose(u, ref[:, :3], rtol=1e-12, atol=1e-14)
    assert np.allclose(lap, ref[:, 3:], rtol=1e-12, atol=1e-14)
    u0, p0, _, _ = stokes_from_4lap(x, y, origin, f=f)
    assert np.allclose(u0, direct.stokeslet(y, f, x), rtol=1e-12, atol=1e-14)
    pv = direct.pvel(y, np.concatenate([f, np.zeros((6, 1))], 1), None, None, x)
    assert np.allclose(p0, pv[:, 0], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("origin", [np.zeros(3), np.array([-0.4, 0.2, 0.1])])
def test_pvel_and_traction(origin):
    x, y = _setup()
    fq = RNG.standard_normal((6, 4))
    D = RNG.standard_normal((6, 3, 3))
    for sl, dl in ((True, False), (False, True), (True, True)):
        u, p, _, sig = stokes_from_4lap(x, y, origin, f=fq[:, :3] if sl else None,
                                        q=fq[:, 3] if sl else None, D=D if dl else None)
        args = (y if sl else None, fq if sl else None, y if dl else None, D.reshape(6, 9) if dl else None)
        pv = direct.pvel(*args, x)
        tr = direct.traction(*args, x).reshape(-1, 3, 3)
        assert np.allclose(p, pv[:, 0], rtol=1e-11, atol=1e-13)
        assert np.allclose(u, pv[:, 1:], rtol=1e-11, atol=1e-13)
        assert np.allclose(sig, tr, rtol=1e-11, atol=1e-13)


def test_origin_shift_rule():
    # Psi_B = Psi_A - (c_B - c_A).Phi: densities moved between origins give
    # the same velocity
    x, y = _setup()
    f = RNG.standard_normal((6, 3))
    cA, cB = np.array([0.1, 0.2, -0.3]), np.array([-0.2, 0.4, 0.05])
    psiA = np.sum((y - cA) * f, axis=1)
    psiB = psiA - f @ (cB - cA)
    assert np.allclose(psiB, np.sum((y - cB) * f, axis=1), rtol=1e-14, atol=1e-14)
