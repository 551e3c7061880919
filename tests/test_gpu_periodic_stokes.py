"""Triply periodic Stokeslet on the GPU against the oracle's Ewald sum
(Hasimoto split, zero net force, zero mean velocity).

* a single leaf: the near images through the shifted U list, the far images
  through the root operator;
* the FMM at p = 8 on uniform and clustered points, and at p = 10;
* the translation test (moving all points together changes nothing);
* a non-zero net force is rejected;
* RPY (u and lap u) on the same path: the root's check-surface flow takes
  the (b^2/6) lap G term, the targets the far images' lap u;
* PVel (p, u) of single-layer (f, q) and double-layer D sources (zero net
  force, flux and tr D), on the unit box and on a shifted box of side 2.5:
  u against the oracle's Ewald sums, p up to an additive constant (the far
  images' pressure is fitted through their flow, which fixes it only up to
  one); non-zero net flux or tr D is rejected;
* PVelGrad, PVelLaplacian and Traction on the same sources, at targets
  kept 0.02 from every source image (their oracle takes central differences
  of the periodic (p, u)); p and the isotropic part of sigma up to a
  constant;
* the regularized Stokeslet (blobs eps in [1e-4, 1e-3]): its far field is
  RPY's with b^2 = 3 eps^2/2, at separate targets and on the blobs;
* the regularized force and torque (u, omega), with and without a net
  torque (only the net force must vanish).
"""
import numpy as np
import pytest
import torch

from oracle.stokes_periodic import (pvel_derivs_periodic, pvel_periodic, rpy_periodic, stokeslet_periodic,
                                    stokes_reg_ft_periodic, stokes_reg_periodic)
from paper_2010_15155_amd import FMM, StkfmmError, workloads as W

pytestmark = pytest.mark.gpu


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _problem(n, seed, clustered=False):
    rng = np.random.default_rng(seed)
    if clustered:
        x = np.mod(W.gaussian_mixture_points(rng, n, rng.uniform(0.0, 1.0, (4, 3)), 0.06), 1.0)
    else:
        x = rng.random((n, 3))
    f = rng.standard_normal((n, 3))
    f -= f.mean(axis=0)
    return x, f


@pytest.fixture(scope="module")
def fmm():
    f = FMM()
    yield f
    f.close()


def test_single_leaf(fmm):
    x, f = _problem(600, 1)
    print("periodic Stokeslet, one leaf, 600 points", flush=True)
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=8, leaf_cap=1000,
                       bc="PXYZ").cpu().numpy()
    assert fmm.stats()["boxes"] == 1
    ref = stokeslet_periodic(x, f, x)
    e = rel(out, ref)
    print("  rel L2", e, flush=True)
    assert e < 1e-5


# the tree's own error: a few 1e-6 at p = 8, lower at p = 10 (the far-image
# operator, of order 10, stays below both)
@pytest.mark.parametrize("clustered,p,tol", [(False, 8, 1e-5), (True, 8, 1e-5), (False, 10, 5e-6)])
def test_fmm(fmm, clustered, p, tol):
    x, f = _problem(8192, 2 + clustered, clustered)
    print("periodic Stokeslet, 8192 points, clustered", clustered, "p", p, flush=True)
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=p, leaf_cap=64,
                       bc="PXYZ").cpu().numpy()
    assert fmm.stats()["depth"] >= 3
    idx = W.sample_indices(len(x), 300, 4)
    ref = stokeslet_periodic(x, f, x[idx])
    e = rel(out[idx], ref)
    print("  rel L2", e, flush=True)
    assert e < tol


def test_translation(fmm):
    x, f = _problem(20000, 5)
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(x), p=8, leaf_cap=100,
                       bc="PXYZ").cpu().numpy()
    s = np.array([0.27, 0.64, 0.91])
    xs = np.mod(x + s, 1.0)
    out2 = fmm.evaluate("Stokeslet", sl_xyz=cu(xs), sl_val=cu(f), trg_xyz=cu(xs), p=8, leaf_cap=100,
                        bc="PXYZ").cpu().numpy()
    e = rel(out2, out)
    print("periodic Stokeslet translation test", e, flush=True)
    assert e < 2e-5          # two p = 8 evaluations, each within 1e-5 of the sum (measured 1.15e-5)


def test_rejects_net_force(fmm):
    x, f = _problem(3000, 6)
    fmm.set_points("Stokeslet", cu(x), None, cu(x), p=6, leaf_cap=100, bc="PXYZ")
    with pytest.raises(StkfmmError) as ei:
        fmm.run(cu(f + np.array([0.0, 1e-3, 0.0])))
    assert ei.value.status == "E_DOMAIN"


def _rpy(n, seed, clustered=False):
    x, f = _problem(n, seed, clustered)
    b = np.random.default_rng(seed + 100).uniform(0.002, 0.005, n)
    return x, np.concatenate([f, b[:, None]], 1)


@pytest.mark.parametrize("n,cap,p,tol_u,tol_lap", [(600, 1000, 8, 1e-5, 2e-6), (8192, 64, 8, 1e-5, 2e-6),
                                                   (8192, 64, 10, 5e-6, 2e-6)])
def test_rpy(fmm, n, cap, p, tol_u, tol_lap):
    x, fb = _rpy(n, 11)
    print("periodic RPY", n, "points, p", p, flush=True)
    out = fmm.evaluate("RPY", sl_xyz=cu(x), sl_val=cu(fb), trg_xyz=cu(x), p=p, leaf_cap=cap,
                       bc="PXYZ").cpu().numpy()
    idx = W.sample_indices(len(x), min(n, 300), 5)
    ref = rpy_periodic(x, fb, x[idx])
    e_u, e_lap = rel(out[idx, :3], ref[:, :3]), rel(out[idx, 3:], ref[:, 3:])
    print("  rel L2 u", e_u, "lap u", e_lap, flush=True)
    assert e_u < tol_u and e_lap < tol_lap


def test_rpy_rejects_net_force(fmm):
    x, fb = _rpy(2000, 12)
    fb[:, 0] += 1e-3
    fmm.set_points("RPY", cu(x), None, cu(x), p=6, leaf_cap=100, bc="PXYZ")
    with pytest.raises(StkfmmError) as ei:
        fmm.run(cu(fb))
    assert ei.value.status == "E_DOMAIN"


def test_separate_targets(fmm):
    x, f = _problem(4096, 13)
    t = np.random.default_rng(14).uniform(-0.3, 1.3, (700, 3))   # wrapped by the plan
    out = fmm.evaluate("Stokeslet", sl_xyz=cu(x), sl_val=cu(f), trg_xyz=cu(t), p=8, leaf_cap=64,
                       bc="PXYZ").cpu().numpy()
    e = rel(out, stokeslet_periodic(x, f, t))
    print("periodic Stokeslet, separate targets", e, flush=True)
    assert e < 1e-5



def _pvel(n_sl, n_dl, seed, clustered=False):
    y, f = _problem(n_sl, seed, clustered)
    rng = np.random.default_rng(seed + 200)
    q = rng.standard_normal(n_sl)
    q -= q.mean()
    x = rng.random((n_dl, 3))
    D = rng.standard_normal((n_dl, 9))
    D[:, [0, 4, 8]] -= (D[:, 0] + D[:, 4] + D[:, 8]).mean() / 3.0
    return y, np.concatenate([f, q[:, None]], 1), x, D


def _pvel_errors(out, ref):
    d = out[:, 0] - ref[:, 0]
    p0 = ref[:, 0] - ref[:, 0].mean()
    return rel(out[:, 1:], ref[:, 1:]), float(np.linalg.norm(d - d.mean()) / np.linalg.norm(p0))


@pytest.mark.parametrize("n,cap,p,tol_u,tol_p", [(600, 2000, 8, 1e-5, 1e-5), (6000, 64, 8, 1e-5, 2e-5),
                                                 (6000, 64, 10, 5e-6, 1e-5)])
def test_pvel(fmm, n, cap, p, tol_u, tol_p):
    y, fq, x, D = _pvel(n // 2, n // 2, 21)
    t = np.concatenate([y, x])
    print("periodic PVel", n, "sources, p", p, flush=True)
    out = fmm.evaluate("PVel", sl_xyz=cu(y), sl_val=cu(fq), dl_xyz=cu(x), dl_val=cu(D), trg_xyz=cu(t), p=p,
                       leaf_cap=cap, bc="PXYZ").cpu().numpy()
    idx = W.sample_indices(len(t), min(len(t), 300), 6)
    ref = pvel_periodic(y, fq, x, D, t[idx])
    e_u, e_p = _pvel_errors(out[idx], ref)
    print("  rel L2 u", e_u, "p (up to a constant)", e_p, flush=True)
    assert e_u < tol_u and e_p < tol_p


@pytest.mark.parametrize("layers", ["sl", "dl"])
def test_pvel_one_layer_scaled_box(layers):
    # a box of side 2.5 away from the origin: the flux q and D enter with
    # their own powers of the box size
    L, org = 2.5, np.array([-1.0, 0.4, 2.0])
    y, fq, x, D = _pvel(3000, 3000, 22)
    y, x = org + L * y, org + L * x
    t = np.concatenate([y, x]) if layers == "sl" else x
    kw = dict(sl_xyz=cu(y), sl_val=cu(fq)) if layers == "sl" else dict(dl_xyz=cu(x), dl_val=cu(D))
    print("periodic PVel, box of side 2.5,", layers, flush=True)
    f = FMM(origin=tuple(org), box_len=L)
    try:
        out = f.evaluate("PVel", trg_xyz=cu(t), p=8, leaf_cap=64, bc="PXYZ", **kw).cpu().numpy()
    finally:
        f.close()
    idx = W.sample_indices(len(t), 300, 7)
    ref = pvel_periodic(y if layers == "sl" else None, fq, x if layers == "dl" else None, D, t[idx], L=L)
    e_u, e_p = _pvel_errors(out[idx], ref)
    print("  rel L2 u", e_u, "p (up to a constant)", e_p, flush=True)
    assert e_u < 1e-5 and e_p < 2e-5


def test_pvel_rejects_net_flux(fmm):
    y, fq, x, D = _pvel(2000, 2000, 23)
    t = np.concatenate([y, x])
    fmm.set_points("PVel", cu(y), cu(x), cu(t), p=6, leaf_cap=100, bc="PXYZ")
    bad = fq.copy()
    bad[:, 3] += 1e-3
    with pytest.raises(StkfmmError) as ei:
        fmm.run(cu(bad), cu(D))
    assert ei.value.status == "E_DOMAIN" and "flux" in str(ei.value)
    bad = D.copy()
    bad[:, 4] += 1e-3
    with pytest.raises(StkfmmError) as ei:
        fmm.run(cu(fq), cu(bad))
    assert ei.value.status == "E_DOMAIN" and "tr D" in str(ei.value)
    bad = fq.copy()
    bad[:, 1] += 1e-3
    with pytest.raises(StkfmmError) as ei:
        fmm.run(cu(bad), cu(D))
    assert ei.value.status == "E_DOMAIN" and "force" in str(ei.value)


def test_pvel_translation(fmm):
    # moving every point by the same shift (wrapped into the box) changes
    # which image of each source the plan holds, and so the flux moment;
    # the result must not change
    y, fq, x, D = _pvel(6000, 6000, 24)
    t = np.concatenate([y, x])
    outs = []
    for s in (np.zeros(3), np.array([0.31, 0.77, 0.58])):
        w = lambda a: np.mod(a + s, 1.0)
        outs.append(fmm.evaluate("PVel", sl_xyz=cu(w(y)), sl_val=cu(fq), dl_xyz=cu(w(x)), dl_val=cu(D),
                                 trg_xyz=cu(w(t)), p=8, leaf_cap=64, bc="PXYZ").cpu().numpy())
    e_u, e_p = _pvel_errors(outs[1], outs[0])
    print("periodic PVel translation: u", e_u, "p", e_p, flush=True)
    # two p = 8 evaluations, each within 1e-5 (u) of the sum (measured
    # 7.0e-6 for u and 1.3e-7 for p)
    assert e_u < 2e-5 and e_p < 2e-5


def _targets_away(sources, k, seed, dmin=0.02):
    from scipy.spatial import cKDTree
    tree = cKDTree(np.mod(sources, 1.0), boxsize=1.0)
    rng = np.random.default_rng(seed)
    out = np.zeros((0, 3))
    while len(out) < k:
        c = rng.random((4 * k, 3))
        out = np.concatenate([out, c[tree.query(c)[0] >= dmin]])
    return out[:k]


DERIV_FIELDS = {"PVelGrad": [("p", 0, 1), ("u", 1, 4), ("grad p", 4, 7), ("grad u", 7, 16)],
                "PVelLaplacian": [("p", 0, 1), ("u", 1, 4), ("lap u", 4, 7)],
                "Traction": [("sigma", 0, 9)]}


def _deriv_errors(kernel, got, ref):
    errs = {}
    for name, a, b in DERIV_FIELDS[kernel]:
        d, r = got[:, a:b] - ref[:, a:b], ref[:, a:b].copy()
        if name == "p":                       # up to a constant
            d, r = d - d.mean(), r - r.mean()
        if name == "sigma":                   # up to a constant times I
            for x in (d, r):
                x[:, [0, 4, 8]] -= x[:, [0, 4, 8]].mean()
        errs[name] = float(np.linalg.norm(d) / np.linalg.norm(r))
    return errs


@pytest.mark.parametrize("kernel,p,tol", [("PVelGrad", 8, 2e-5), ("PVelLaplacian", 8, 2e-5), ("Traction", 8, 2e-5),
                                          ("PVelGrad", 10, 5e-6)])
def test_pvel_derivative_kernels(fmm, kernel, p, tol):
    y, fq, x, D = _pvel(3000, 3000, 31)
    t = _targets_away(np.concatenate([y, x]), 2000, 32)
    print("periodic", kernel, "6000 sources, 2000 targets, p", p, flush=True)
    out = fmm.evaluate(kernel, sl_xyz=cu(y), sl_val=cu(fq), dl_xyz=cu(x), dl_val=cu(D), trg_xyz=cu(t), p=p,
                       leaf_cap=64, bc="PXYZ").cpu().numpy()
    idx = W.sample_indices(len(t), 60, 33)
    ref = pvel_derivs_periodic(y, fq, x, D, t[idx], h=2e-4, kind=kernel)
    errs = _deriv_errors(kernel, out[idx], ref)
    print("  rel L2", errs, flush=True)
    for e in errs.values():
        assert e < tol


def test_traction_shifted_box():
    # a box of side 2.5 away from the origin: sigma scales as 1/L^2
    L, org = 2.5, np.array([-1.0, 0.4, 2.0])
    y, fq, x, D = _pvel(3000, 3000, 34)
    t = _targets_away(np.concatenate([y, x]), 1000, 35)
    f = FMM(origin=tuple(org), box_len=L)
    print("periodic Traction, box of side 2.5", flush=True)
    try:
        out = f.evaluate("Traction", sl_xyz=cu(org + L * y), sl_val=cu(fq), dl_xyz=cu(org + L * x), dl_val=cu(D),
                         trg_xyz=cu(org + L * t), p=8, leaf_cap=64, bc="PXYZ").cpu().numpy()
    finally:
        f.close()
    idx = W.sample_indices(len(t), 40, 36)
    ref = pvel_derivs_periodic(org + L * y, fq, org + L * x, D, org + L * t[idx], L=L, h=2e-4 * L, kind="Traction")
    errs = _deriv_errors("Traction", out[idx], ref)
    print("  rel L2", errs, flush=True)
    assert errs["sigma"] < 2e-5


# p = 10 gains little here (8.1e-6 -> 5.9e-6 at separate targets): on these
# 8192 points the periodic plans keep a floor of a few 1e-6 whatever the
# order (the Stokeslet too), hence one bound for both
@pytest.mark.parametrize("on_blobs,p,tol", [(False, 8, 1e-5), (True, 8, 1e-5), (False, 10, 1e-5)])
def test_regularized(fmm, on_blobs, p, tol):
    x, f = _problem(8192, 41)
    fe = np.concatenate([f, np.random.default_rng(42).uniform(1e-4, 1e-3, (len(x), 1))], 1)
    t = x if on_blobs else np.random.default_rng(43).random((2000, 3))
    print("periodic StokesRegVel, 8192 blobs, on blobs", on_blobs, "p", p, flush=True)
    out = fmm.evaluate("StokesRegVel", sl_xyz=cu(x), sl_val=cu(fe), trg_xyz=cu(t), p=p, leaf_cap=64,
                       bc="PXYZ").cpu().numpy()
    idx = W.sample_indices(len(t), 300, 44)
    ref = stokes_reg_periodic(x, fe, t[idx])
    e = rel(out[idx], ref)
    print("  rel L2", e, flush=True)
    assert e < tol


@pytest.mark.parametrize("on_blobs,net_torque", [(False, False), (True, False), (False, True)])
def test_regularized_force_torque(fmm, on_blobs, net_torque):
    rng = np.random.default_rng(51)
    x = rng.random((4096, 3))
    ft = rng.standard_normal((len(x), 6))
    ft[:, :3] -= ft[:, :3].mean(axis=0)
    if not net_torque:
        ft[:, 3:] -= ft[:, 3:].mean(axis=0)
    fte = np.concatenate([ft, rng.uniform(1e-4, 1e-3, (len(x), 1))], 1)
    t = x if on_blobs else rng.random((2000, 3))
    print("periodic StokesRegVelOmega, 4096 blobs, on blobs", on_blobs, "net torque", net_torque, flush=True)
    out = fmm.evaluate("StokesRegVelOmega", sl_xyz=cu(x), sl_val=cu(fte), trg_xyz=cu(t), p=8, leaf_cap=64,
                       bc="PXYZ").cpu().numpy()
    idx = W.sample_indices(len(t), 200, 52)
    ref = stokes_reg_ft_periodic(x, fte, t[idx])
    e_u, e_w = rel(out[idx, :3], ref[:, :3]), rel(out[idx, 3:], ref[:, 3:])
    print("  rel L2 u", e_u, "omega", e_w, flush=True)
    assert e_u < 1e-5 and e_w < 1e-5


@pytest.mark.parametrize("kernel", ["Stokeslet", "RPY", "StokesRegVel", "StokesRegVelOmega", "PVel", "PVelGrad",
                                    "PVelLaplacian", "Traction"])
def test_no_sources(fmm, kernel):
    # targets only: no source chunks reach the root's check surface
    t = np.random.default_rng(61).random((100, 3))
    out = fmm.evaluate(kernel, trg_xyz=cu(t), p=6, leaf_cap=20, bc="PXYZ").cpu().numpy()
    assert np.array_equal(out, np.zeros_like(out))


def test_single_torque_blob(fmm):
    # one blob with a torque and no force: a net torque, one source record.
    # Its images reach the targets mostly through the tree's expansions, which
    # a lone rotlet stresses: u 1.7e-5 at p = 8, 3.8e-6 at p = 10 (one leaf:
    # 3e-7; open boundary at p = 8: 2.1e-6)
    y = np.array([[0.3, 0.6, 0.45]])
    fte = np.array([[0.0, 0.0, 0.0, 0.4, -1.0, 0.7, 5e-4]])
    t = np.random.default_rng(62).random((200, 3))
    out = fmm.evaluate("StokesRegVelOmega", sl_xyz=cu(y), sl_val=cu(fte), trg_xyz=cu(t), p=10, leaf_cap=20,
                       bc="PXYZ").cpu().numpy()
    ref = stokes_reg_ft_periodic(y, fte, t)
    e_u, e_w = rel(out[:, :3], ref[:, :3]), rel(out[:, 3:], ref[:, 3:])
    print("periodic single torque blob: u", e_u, "omega", e_w, flush=True)
    assert e_u < 1e-5 and e_w < 1e-5
