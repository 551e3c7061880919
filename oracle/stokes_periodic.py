"""Triply periodic Stokeslet by Ewald summation (oracle) -- TEST INFRASTRUCTURE ONLY.

The periodic boundary condition of Sec. III (and its appendix on
periodicity) for the Stokeslet of Sec. II.B (viscosity 1):

    u(x) = sum_j sum_n G(x - y_j - n L) f_j,   G(r) = (I/r + r r^T/r^3) / (8 pi).

The lattice sum does not converge absolutely; the oracle fixes the usual
definition through the Fourier series of the periodic Stokes equations,
u_hat(k) = (I - k k^T/k^2) f_hat(k) / k^2: the net force must vanish and
the k = 0 term is dropped (the mean velocity over the cell is zero).

Ewald split with the Hasimoto factor phi(k) = (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)}:
  reciprocal  (1/V) sum_{k != 0} phi(k)/k^2 (I - k k^T/k^2) Re[S(k) e^{i k.x}],
              S(k) = sum_j f_j e^{-i k.y_j},  k = 2 pi m / L;
  real        the remaining part, G = (I lap - grad grad) B / (8 pi) with
              B'(r) = erfc(xi r) (the biharmonic generator of the split-off
              part, whose transform is -8 pi (1 - phi)/k^4):
              8 pi G_R(r) = (erfc(xi r)/r - c e) I + (erfc(xi r)/r + c e) r r^T/r^2,
              c = 2 xi / sqrt(pi), e = exp(-xi^2 r^2);
  self        a target on source j drops the smooth part of its own term,
              lim_{r->0} (G - G_R) f_j = 4 xi/(8 pi sqrt(pi)) f_j:
              u -= xi / (2 pi^{3/2}) f_j.
The real part's integral vanishes (1 - phi = O(k^4)), so no constant term
arises.  FP64: the real part by plain loops in ewald.c, the reciprocal part
with NumPy.

The same module holds the RPY sum (with lap G), the double layer
(grad G : D^s), PVel's (p, u) built from these and the Laplace Ewald sums,
and PVel's derivative outputs by central differences of (p, u).
"""
import numpy as np

from .direct import _p, lib

PI = np.pi


def parameters(L, xi=None, tol=1e-15):
    """(xi, real cutoff, reciprocal cutoff index) for relative truncation tol."""
    if xi is None:
        xi = 4.0 / L
    s = np.sqrt(-np.log(tol)) + 0.5
    rc = s / xi
    nmax = int(np.ceil(2.0 * xi * s * L / (2.0 * PI)))
    return xi, rc, nmax


def stokeslet_periodic(src, f, trg, L=1.0, xi=None, tol=1e-15):
    """Periodic Stokeslet velocity [m, 3] at trg [m, 3] of forces f [n, 3] at src [n, 3]."""
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    xi, rc, nmax = parameters(L, xi, tol)
    u = np.zeros((len(x), 3))
    if len(y) == 0 or len(x) == 0:
        return u
    # real space and self terms (ewald.c, plain loops over targets, sources
    # and the images within rc)
    lib().oracle_stokes_ewald_real(len(y), _p(y), _p(f), len(x), _p(x), float(L), float(xi), float(rc), _p(u))
    # reciprocal space: every k != 0 in the cube [-nmax, nmax]^3
    m = np.arange(-nmax, nmax + 1)
    K = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    K = K[np.any(K != 0, axis=1)] * (2.0 * PI / L)
    k2 = np.sum(K * K, axis=1)
    g = (1.0 + k2 / (4.0 * xi * xi)) * np.exp(-k2 / (4.0 * xi * xi)) / k2
    S = np.zeros((len(K), 3), dtype=np.complex128)        # S(k), summed over source blocks
    for j0 in range(0, len(y), 1024):
        S += np.exp(-1j * (K @ y[j0:j0 + 1024].T)) @ f[j0:j0 + 1024]
    PS = S - K * (np.sum(K * S, axis=1) / k2)[:, None]    # (I - k k^T/k^2) S
    W = g[:, None] * PS / L ** 3
    for i0 in range(0, len(x), 1024):
        u[i0:i0 + 1024] += np.real(np.exp(1j * (x[i0:i0 + 1024] @ K.T)) @ W)
    return u


def _reciprocal(y, fw, x, L, xi, nmax, lap):
    """(1/V) sum_{k != 0} a(k) (I - k k^T/k^2) Re[S(k) e^{i k.x}], S = sum_j fw_j e^{-i k.y_j},
    a = phi/k^2 (the Stokeslet) or -phi (its Laplacian)."""
    m = np.arange(-nmax, nmax + 1)
    K = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    K = K[np.any(K != 0, axis=1)] * (2.0 * PI / L)
    k2 = np.sum(K * K, axis=1)
    phi = (1.0 + k2 / (4.0 * xi * xi)) * np.exp(-k2 / (4.0 * xi * xi))
    a = -phi if lap else phi / k2
    S = np.zeros((len(K), 3), dtype=np.complex128)
    for j0 in range(0, len(y), 1024):
        S += np.exp(-1j * (K @ y[j0:j0 + 1024].T)) @ fw[j0:j0 + 1024]
    PS = S - K * (np.sum(K * S, axis=1) / k2)[:, None]
    Wk = a[:, None] * PS / L ** 3
    u = np.zeros((len(x), 3))
    for i0 in range(0, len(x), 1024):
        u[i0:i0 + 1024] = np.real(np.exp(1j * (x[i0:i0 + 1024] @ K.T)) @ Wk)
    return u


def stokes_lap_periodic(src, f, w, trg, L=1.0, xi=None, tol=1e-15):
    """Periodic sum of the Stokeslet's Laplacian, lap G = (2 I/r^3 - 6 r r^T/r^5)/(8 pi),
    applied to w_j f_j [m, 3] (same convention: zero net force, k = 0 dropped;
    pairs with r = 0 left out).  Reciprocal amplitude -phi(k) (I - k k^T/k^2);
    real part and self term in ewald.c."""
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    xi, rc, nmax = parameters(L, xi, tol)
    nmax += 2                      # phi(k) k^2 decays more slowly than phi(k)/k^2
    u = np.zeros((len(x), 3))
    if len(y) == 0 or len(x) == 0:
        return u
    lib().oracle_stokes_lap_ewald_real(len(y), _p(y), _p(f), _p(w), len(x), _p(x), float(L), float(xi), float(rc),
                                       _p(u))
    return u + _reciprocal(y, w[:, None] * f, x, L, xi, nmax, True)


def rpy_periodic(src, fb, trg, L=1.0, xi=None, tol=1e-15):
    """Periodic RPY (Sec. II.B: u = (1 + b^2/6 lap) G f for r > 0) with its
    Laplacian: [m, 6] = (u, lap u).  Off the sources lap^2 G = 0, so
    lap u is the periodic sum of lap G f; f must sum to zero."""
    fb = np.ascontiguousarray(fb, dtype=np.float64).reshape(-1, 4)
    f, b2 = fb[:, :3], fb[:, 3] ** 2
    u = stokeslet_periodic(src, f, trg, L, xi, tol) + stokes_lap_periodic(src, f, b2 / 6.0, trg, L, xi, tol)
    lap = stokes_lap_periodic(src, f, np.ones(len(f)), trg, L, xi, tol)
    return np.concatenate([u, lap], axis=1)


def stokes_dl_periodic(src, D, trg, L=1.0, xi=None, tol=1e-15):
    """Periodic sum of grad G : D^s [m, 3], (grad G : D)_i = sum_jk d_k G_ij D_jk,
    D [n, 9] row-major (its symmetric part acts).  Reciprocal amplitude
    i phi(k)/k^2 (I - k k^T/k^2) D^s k; real part in ewald.c; no self term
    (the smooth part is odd)."""
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1, 9)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    xi, rc, nmax = parameters(L, xi, tol)
    nmax += 1                      # phi(k)/k decays more slowly than phi(k)/k^2
    u = np.zeros((len(x), 3))
    if len(y) == 0 or len(x) == 0:
        return u
    lib().oracle_stokes_dl_ewald_real(len(y), _p(y), _p(D), len(x), _p(x), float(L), float(xi), float(rc), _p(u))
    m = np.arange(-nmax, nmax + 1)
    K = np.stack(np.meshgrid(m, m, m, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    K = K[np.any(K != 0, axis=1)] * (2.0 * PI / L)
    k2 = np.sum(K * K, axis=1)
    phi = (1.0 + k2 / (4.0 * xi * xi)) * np.exp(-k2 / (4.0 * xi * xi))
    Ds = 0.5 * (D + D.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9))
    S = np.zeros((len(K), 3), dtype=np.complex128)     # sum_j (D_j k) e^{-i k.y_j}
    for j0 in range(0, len(y), 512):
        E = np.exp(-1j * (K @ y[j0:j0 + 512].T))                          # [nk, nb]
        Dk = np.einsum("bij,kj->kbi", Ds[j0:j0 + 512].reshape(-1, 3, 3), K)  # [nk, nb, 3]
        S += np.einsum("kb,kbi->ki", E, Dk)
    PS = S - K * (np.sum(K * S, axis=1) / k2)[:, None]
    Wk = 1j * (phi / k2)[:, None] * PS / L ** 3
    for i0 in range(0, len(x), 1024):
        u[i0:i0 + 1024] += np.real(np.exp(1j * (x[i0:i0 + 1024] @ K.T)) @ Wk)
    return u


def pvel_periodic(sl, fq, dl, D, trg, L=1.0, tol=1e-13):
    """Periodic PVel [m, 4] = (p, u) of single-layer sources (f, q) [n, 4] at sl
    and double-layer sources D [n, 9] at dl (Sec. II.B's pressure-velocity
    kernels): sum f, sum q and sum tr D must vanish.  Written with the Laplace
    Ewald sums (``ewald``) and the periodic Stokeslet and its gradient:
      u = G f + (q/2) grad L + grad G : D^s + (tr D/2) grad L,
      p = -sum_j d_j (L f_j) - D^s : grad grad L  (L = 1/(4 pi r))."""
    from . import ewald
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((len(x), 4))
    if sl is not None and len(sl):
        sl = np.ascontiguousarray(sl, dtype=np.float64).reshape(-1, 3)
        fq = np.ascontiguousarray(fq, dtype=np.float64).reshape(-1, 4)
        out[:, 1:] += stokeslet_periodic(sl, fq[:, :3], x, L)
        out[:, 1:] += ewald.laplace_periodic(sl, 0.5 * fq[:, 3], None, x, L, tol=tol)[:, 1:]
        for j in range(3):
            out[:, 0] -= ewald.laplace_periodic(sl, fq[:, j], None, x, L, tol=tol)[:, 1 + j]
    if dl is not None and len(dl):
        dl = np.ascontiguousarray(dl, dtype=np.float64).reshape(-1, 3)
        D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1, 9)
        tr = D[:, 0] + D[:, 4] + D[:, 8]
        out[:, 1:] += stokes_dl_periodic(dl, D, x, L)
        out[:, 1:] += ewald.laplace_periodic(dl, 0.5 * tr, None, x, L, tol=tol)[:, 1:]
        Ds = 0.5 * (D + D.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9))
        out[:, 0] += ewald.laplace_periodic(dl, None, None, x, L, tol=tol, Q=-Ds)[:, 0]
    return out



def _stencil(x, h):
    """The target and its four neighbours at +-h, +-2h along each axis:
    [13 m, 3] (x first, then axis j, offsets h, -h, 2h, -2h)."""
    pts = [x]
    for j in range(3):
        for s in (h, -h, 2.0 * h, -2.0 * h):
            y = x.copy()
            y[:, j] += s
            pts.append(y)
    return np.concatenate(pts)


def _derivatives(v, m, h):
    """From values on the stencil [13 m, c]: the centre value [m, c], the
    first derivatives [m, c, 3] and the second derivatives along each axis
    [m, c, 3], by the five-point central formulas (error O(h^4))."""
    v = v.reshape(13, m, -1)
    d1 = np.empty(v.shape[1:] + (3,))
    d2 = np.empty(v.shape[1:] + (3,))
    for j in range(3):
        a, b, c, d = v[1 + 4 * j], v[2 + 4 * j], v[3 + 4 * j], v[4 + 4 * j]
        d1[..., j] = (8.0 * (a - b) - (c - d)) / (12.0 * h)
        d2[..., j] = (16.0 * (a + b) - (c + d) - 30.0 * v[0]) / (12.0 * h * h)
    return v[0], d1, d2


def pvel_derivs_periodic(sl, fq, dl, D, trg, L=1.0, h=None, kind="PVelGrad"):
    """Periodic PVel with derivative outputs (the pressure-velocity kernels'
    gradient, Laplacian and stress outputs of the paper's table of supported
    kernels) at targets away from every source: the derivatives of
    pvel_periodic by five-point central differences (step h, default
    L/1000; the targets must lie much farther than 2h from every source
    image).  kind
      "PVelGrad"      -> [m, 16]: p, u, grad p, grad u (d_j u_i row-major),
      "PVelLaplacian" -> [m, 7]:  p, u, lap u (sum of second differences),
      "Traction"      -> [m, 9]:  sigma = -p I + grad u + grad u^T (row-major).
    The pressure (and so sigma's isotropic part) is that of pvel_periodic:
    zero mean over the cell."""
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    m = len(x)
    h = 1e-3 * L if h is None else h
    v = pvel_periodic(sl, fq, dl, D, _stencil(x, h), L)
    c, d1, d2 = _derivatives(v, m, h)
    p, u = c[:, 0], c[:, 1:]
    gp, gu = d1[:, 0, :], d1[:, 1:, :]                  # gu[:, i, j] = d_j u_i
    if kind == "PVelGrad":
        return np.concatenate([p[:, None], u, gp, gu.reshape(m, 9)], 1)
    if kind == "PVelLaplacian":
        return np.concatenate([p[:, None], u, d2[:, 1:, :].sum(axis=2)], 1)
    if kind == "Traction":
        sig = -p[:, None, None] * np.eye(3)[None] + gu + gu.transpose(0, 2, 1)
        return sig.reshape(m, 9)
    raise ValueError(kind)


def _lap_g(src, wf, trg):
    """Free-space lap G applied to wf [n, 3]: (2 wf/r^3 - 6 r (r.wf)/r^5)/(8 pi)
    summed over the sources, pairs at r = 0 left out."""
    u = np.zeros((len(trg), 3))
    for i0 in range(0, len(trg), 256):
        r = trg[i0:i0 + 256, None, :] - src[None, :, :]
        rr = np.sum(r * r, axis=2)
        ok = rr > 0
        ri = np.where(ok, 1.0 / np.sqrt(np.where(ok, rr, 1.0)), 0.0)
        ri3 = ri ** 3
        rw = np.sum(r * wf[None], axis=2)
        u[i0:i0 + 256] = np.sum(2.0 * wf[None] * ri3[..., None] - 6.0 * r * (rw * ri3 * ri * ri)[..., None], axis=1)
    return u / (8.0 * PI)


def stokes_reg_periodic(src, fe, trg, L=1.0, images=1, tol=1e-15):
    """Periodic regularized Stokeslet [f, eps] -> u [m, 3] (Sec. II.B's
    regularized kernel, tab:ktab_reg; zero net force).  Away from a blob
    G^eps = G + (eps^2/4) lap G + O(eps^4/r^5), so the lattice sum is the
    Ewald sum of that far-field form (the Stokeslet and lap G sums above,
    same convention) plus the absolutely convergent sum of the remainder
    G^eps - G - (eps^2/4) lap G over the images with max|n_k| <= images.  A
    target on a source takes G^eps(0) f from its own blob (the Ewald sums
    leave r = 0 out)."""
    from . import direct
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    fe = np.ascontiguousarray(fe, dtype=np.float64).reshape(-1, 4)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    f, w = fe[:, :3], 0.25 * fe[:, 3] ** 2
    u = stokeslet_periodic(y, f, x, L, tol=tol) + stokes_lap_periodic(y, f, w, x, L, tol=tol)
    m = np.arange(-images, images + 1)
    for n in np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3):
        yn = y + L * n
        u += direct.stokes_reg(yn, fe, x) - direct.stokeslet(yn, f, x) - _lap_g(yn, w[:, None] * f, x)
    return u


def rotlet_periodic(src, t, trg, L=1.0, xi=None, tol=1e-15):
    """Periodic rotlet sum [m, 3]: u = sum (t_j x r)/(8 pi r^3) over the
    lattice, i.e. half the curl of the periodic Stokeslet sum with forces t
    (curl G t = 2 (t x r)/(8 pi r^3)); k = 0 dropped, pairs at r = 0 left
    out (the smooth part is odd).  Ewald split of the Stokeslet's:
      real        (erfc(xi r)/r^3 + c e/r^2 - c xi^2 e) (t x r)/(8 pi),
                  c = 2 xi/sqrt(pi), e = exp(-xi^2 r^2)  (half the curl of G_R t);
      reciprocal  (1/(2V)) sum_{k != 0} phi(k)/k^2 Re[i k x S(k) e^{i k.x}]."""
    from scipy.special import erfc
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    xi, rc, nmax = parameters(L, xi, tol)
    nmax += 1
    u = np.zeros((len(x), 3))
    if len(y) == 0 or len(x) == 0:
        return u
    c = 2.0 * xi / np.sqrt(PI)
    nimg = int(np.ceil(rc / L))
    m = np.arange(-nimg, nimg + 1)
    imgs = np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3) * L
    for i0 in range(0, len(x), 64):
        d0 = x[i0:i0 + 64, None, :] - y[None, :, :]
        d0 -= L * np.round(d0 / L)
        for n in imgs:
            r = d0 + n
            rr = np.sum(r * r, axis=2)
            ok = (rr > 0) & (rr < rc * rc)
            rs = np.sqrt(np.where(ok, rr, 1.0))
            e = np.exp(-xi * xi * rs * rs)
            g = np.where(ok, erfc(xi * rs) / rs ** 3 + c * e / rs ** 2 - c * xi * xi * e, 0.0)
            u[i0:i0 + 64] += np.sum(g[..., None] * np.cross(t[None, :, :], r), axis=1)
    u /= 8.0 * PI
    mm = np.arange(-nmax, nmax + 1)
    K = np.stack(np.meshgrid(mm, mm, mm, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    K = K[np.any(K != 0, axis=1)] * (2.0 * PI / L)
    k2 = np.sum(K * K, axis=1)
    phi = (1.0 + k2 / (4.0 * xi * xi)) * np.exp(-k2 / (4.0 * xi * xi))
    S = np.zeros((len(K), 3), dtype=np.complex128)
    for j0 in range(0, len(y), 512):
        S += np.exp(-1j * (K @ y[j0:j0 + 512].T)) @ t[j0:j0 + 512]
    Wk = 1j * np.cross(K, S) * (phi / k2)[:, None] / (2.0 * L ** 3)
    for i0 in range(0, len(x), 1024):
        u[i0:i0 + 1024] += np.real(np.exp(1j * (x[i0:i0 + 1024] @ K.T)) @ Wk)
    return u


def _rotlet(src, t, trg):
    """Free-space rotlet sum (t x r)/(8 pi r^3), pairs at r = 0 left out."""
    u = np.zeros((len(trg), 3))
    for i0 in range(0, len(trg), 256):
        r = trg[i0:i0 + 256, None, :] - src[None, :, :]
        rr = np.sum(r * r, axis=2)
        ok = rr > 0
        ri3 = np.where(ok, 1.0 / np.sqrt(np.where(ok, rr, 1.0)) ** 3, 0.0)
        u[i0:i0 + 256] = np.sum(ri3[..., None] * np.cross(t[None, :, :], r), axis=1)
    return u / (8.0 * PI)


def stokes_reg_ft_periodic(src, fte, trg, L=1.0, images=1, tol=1e-15):
    """Periodic regularized force and torque [f, t, eps] -> [u, omega] [m, 6]
    (Sec. II.B's force-torque extension; zero net force and torque).  Far
    from a blob the kernels become
      u     = G f + (eps^2/4) lap G f + rotlet(t),
      omega = curl(u)/2 = rotlet(f) - (1/4) lap G t
    (the rotlet is harmonic, so its eps^2 term vanishes, as does curl lap G f),
    each summed by Ewald (same convention as above); the remainder of the
    exact kernels is summed over the images with max|n_k| <= images."""
    from . import direct
    y = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    fte = np.ascontiguousarray(fte, dtype=np.float64).reshape(-1, 7)
    x = np.ascontiguousarray(trg, dtype=np.float64).reshape(-1, 3)
    f, t, w = fte[:, :3], fte[:, 3:6], 0.25 * fte[:, 6] ** 2
    q = -0.25 * np.ones(len(y))
    out = np.zeros((len(x), 6))
    out[:, :3] = (stokeslet_periodic(y, f, x, L, tol=tol) + stokes_lap_periodic(y, f, w, x, L, tol=tol)
                  + rotlet_periodic(y, t, x, L, tol=tol))
    out[:, 3:] = rotlet_periodic(y, f, x, L, tol=tol) + stokes_lap_periodic(y, t, q, x, L, tol=tol)
    m = np.arange(-images, images + 1)
    for n in np.stack(np.meshgrid(m, m, m, indexing="ij"), -1).reshape(-1, 3):
        yn = y + L * n
        far = np.zeros((len(x), 6))
        far[:, :3] = direct.stokeslet(yn, f, x) + _lap_g(yn, w[:, None] * f, x) + _rotlet(yn, t, x)
        far[:, 3:] = _rotlet(yn, f, x) + _lap_g(yn, q[:, None] * t, x)
        out += direct.stokes_reg_ft(yn, fte, x) - far
    return out
