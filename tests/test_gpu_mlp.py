"""GPU predictor kernels against the FP64 reference network (oracle/mlp.py),
and the learned mode's accuracy check / fallback path."""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(31)


def _data(b=300):
    X = RNG.standard_normal((b, mlp.F)) * 1.5 + 0.5
    y = np.stack([RNG.integers(0, 4, b), RNG.integers(0, 4, b)], 1).astype(np.int32)
    theta = mlp.init(5, mean=X.mean(0), std=X.std(0) + 0.1)
    return X, y, theta


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def test_nparam_matches_reference():
    import paper_2010_15155_amd as pkg
    assert pkg.mlp_nparam() == mlp.nparam()


def test_forward_matches_reference():
    import paper_2010_15155_amd as pkg
    X, y, theta = _data()
    got = pkg.mlp_forward(_t(theta), _t(X)).cpu().numpy()
    ref, _ = mlp.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_gradient_matches_reference():
    import paper_2010_15155_amd as pkg
    X, y, theta = _data()
    loss, g = pkg.mlp_loss_grad(_t(theta), _t(X), _t(y, torch.int32))
    th64 = theta.astype(np.float32).astype(np.float64)
    rl, rg = mlp.loss_and_grad(th64, X.astype(np.float32).astype(np.float64), y)
    assert abs(float(loss.cpu()) - rl) < 1e-5 * max(1.0, abs(rl))
    g = g.cpu().numpy()
    assert np.linalg.norm(g - rg) < 2e-4 * np.linalg.norm(rg)


def test_adam_step_matches_reference():
    import paper_2010_15155_amd as pkg
    X, y, theta = _data()
    p = _t(theta)
    _, g = pkg.mlp_loss_grad(p, _t(X), _t(y, torch.int32))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    gref = g.cpu().numpy().astype(np.float64)
    th = theta.astype(np.float32).astype(np.float64)
    mr, vr = np.zeros_like(th), np.zeros_like(th)
    for step in (1, 2, 3):
        pkg.mlp_adam(p, g, m, v, step, 1e-3)
        th, mr, vr = mlp.adam(th, gref, mr, vr, step, 1e-3)
    assert np.allclose(p.cpu().numpy(), th, rtol=0, atol=2e-6)


def test_training_reduces_loss():
    import paper_2010_15155_amd as pkg
    # a learnable rule: class = quartile of the first feature
    X = RNG.standard_normal((2048, mlp.F))
    q = np.digitize(X[:, 0], np.quantile(X[:, 0], [0.25, 0.5, 0.75]))
    y = np.stack([q, 3 - q], 1).astype(np.int32)
    p = _t(mlp.init(9, mean=X.mean(0), std=X.std(0)))
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    Xt, yt = _t(X), _t(y, torch.int32)
    first = None
    for step in range(1, 301):
        loss, g = pkg.mlp_loss_grad(p, Xt, yt)
        if first is None:
            first = float(loss.cpu())
        pkg.mlp_adam(p, g, m, v, step, 3e-3)
    last = float(loss.cpu())
    acc = (pkg.mlp_forward(p, Xt).cpu().numpy()[:, :4].argmax(1) == q).mean()
    assert last < 0.3 * first and acc > 0.9


def test_learned_mode_falls_back_with_bad_weights():
    # weights that always predict order 6 and capacity 250: the sampled check
    # must catch the error and re-plan with p = 10, leaf_cap = 2000
    from oracle import direct
    from paper_2010_15155_amd import FMM, workloads as W
    theta = mlp.init(1)
    theta[-mlp.C:] = np.array([50, 0, 0, 0, 50, 0, 0, 0])
    d = W.clustered_rpy(60000, 12)
    x, f = d["xyz"], d["f"]
    fmm = FMM()
    fmm.set_option("tol", "1e-9")                 # unreachable at p = 6: forces the fallback
    table = np.full(16, 1e-9)          # claims every order meets any tolerance
    fmm.set_predictor(np.concatenate([theta, table]).astype(np.float32))
    out = None
    from paper_2010_15155_amd import StkfmmError
    with pytest.raises(StkfmmError) as ei:
        fmm.evaluate("Stokeslet", _t(x, torch.float64), _t(f, torch.float64), None, None, _t(x, torch.float64),
                     p=0, leaf_cap=0)
    assert ei.value.status == "E_ACCURACY"
    info = fmm.learned_info()
    assert info["fell_back"] and info["p"] == 10 and info["order_hist"][0] > 0
    fmm.set_option("tol", "1e-5")
    out = fmm.evaluate("Stokeslet", _t(x, torch.float64), _t(f, torch.float64), None, None,
                       _t(x, torch.float64), p=0, leaf_cap=0).cpu().numpy()
    info = fmm.learned_info()
    print("learned (bad weights)", info, flush=True)
    assert info["validated"]
    err = direct.rel_l2(out, direct.stokeslet(x, f, x))
    assert err < 1e-5
    fmm.close()
