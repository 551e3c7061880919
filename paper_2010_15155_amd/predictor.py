"""Training driver of the learned order / leaf-capacity predictor.

Labels come from runs of the method itself (not in the paper, which fixes one
global order and leaf size, Sec. III):
  order class     smallest p in {6, 8, 10, 12} whose FMM result on the leaf's
                  sampled targets has an RMS error, against the FP64 direct
                  sum computed on the GPU (stkfmm_direct), within
                  max(safety * tol * (RMS of the field over all sampled
                  targets), FLOOR * the leaf's smallest error over the orders);
  capacity class  the capacity in {250, 500, 1000, 2000} whose plan, built
                  with that capacity everywhere, gives the leaf's targets the
                  smallest cost: the plan's work attributed to its targets
                  (stkfmm_get_plan_work: P2P lane pairs and wave entries, M2L
                  flops, surface evaluations, boxes) priced by unit costs that
                  `fit_costs` fits to measured stage times on this GPU.
Features: 12 per leaf of the reference tree (leaf_cap 2000), computed by the
library.  Training runs the library's HIP kernels (forward, loss gradient,
Adam).  Weights are saved as a float32 .npy (load with allow_pickle=False).

Plans are priced with the translation compression the learned mode uses
(m2l_tol = tol / 50), since the M2L work and its speed depend on it.

  python -m paper_2010_15155_amd.predictor label --seeds 501:601 --out a.npz   (fits the costs first)
  python -m paper_2010_15155_amd.predictor relabel-caps --data a.npz --out b.npz   (new costs, same order labels)
  python -m paper_2010_15155_amd.predictor train --data a.npz b.npz --out w.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import CAP_CLASSES, FMM, ORDER_CLASSES, mlp_adam, mlp_loss_grad, mlp_nparam, workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "predictor_weights.npy")
N_RANGE = (100_000, 2_000_000)


FLOOR = 1.25      # a leaf's order target: max(safety * tol, FLOOR * its best error over orders)
SAFETY = 0.5


def load_weights(path=WEIGHTS):
    """Network parameters followed by the 4x4 order calibration table."""
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.size != mlp_nparam() + 16:
        raise ValueError("bad predictor weights file %s" % path)
    return w


def order_labels(E, tol=1e-5):
    """Order class per leaf from its errors at the four orders: the smallest
    order within max(SAFETY * tol, FLOOR * best error), so leaves whose error
    floor (FP32 round-off) is above the target do not ask for more order."""
    target = np.maximum(SAFETY * tol, FLOOR * E.min(axis=1))
    return (E <= target[:, None]).argmax(axis=1).astype(np.int32)


def calibration_table(E, cls):
    """table[c][q] = RMS over leaves of class c of their error at order class q."""
    t = np.zeros((4, 4))
    for c in range(4):
        m = cls == c
        t[c] = np.sqrt(np.mean(E[m] ** 2, axis=0)) if m.any() else E.max()
    return t


def learned_compression(fmm, tol=1e-5):
    """Price plans with the V-list compression of learned plans."""
    fmm.set_option("m2l_tol", repr(tol / 50.0))


def cap_costs(fmm, torch, x, costs, n_leaf, leaf_of, p_cap=8):
    """[n_leaf, 4] cost of each leaf's targets under the plan built with each
    capacity class everywhere: the plan's work on them priced by `costs`."""
    price = np.asarray(costs, dtype=np.float64)
    out = np.zeros((n_leaf, len(CAP_CLASSES)))
    for q, cap in enumerate(CAP_CLASSES):
        fmm.set_points("Stokeslet", x, None, x, p=p_cap, leaf_cap=cap)
        out[:, q] = np.bincount(leaf_of, weights=fmm.plan_work() @ price, minlength=n_leaf)
    return out


def fit_costs(fmm, torch, p=8, caps=(250, 500, 1000, 2000), seeds=(201, 911, 912)):
    """Unit costs (seconds) of the five plan-work components, least-squares fits
    of serial stage times over plans at several uniform capacities: P2P time on
    lane pairs and wave entries, M2L time on flops, S2M + S2L + L2T time on
    surface evaluations, the remaining stages on boxes (plus a constant)."""
    rows, times = [], []
    learned_compression(fmm)
    fmm.set_option("overlap", "0")
    for seed in seeds:
        d = W.clustered_rpy(1_048_576, seed) if seed == 201 else W.mixture(seed, (500_000, 2_000_000))
        x = torch.from_numpy(d["xyz"]).cuda()
        f = torch.from_numpy(d["f"]).cuda()
        for cap in caps:
            fmm.set_points("Stokeslet", x, None, x, p=p, leaf_cap=cap)
            for _ in range(3):
                fmm.run(f)
            tm = fmm.timings()["stages_ms"]
            rows.append(fmm.plan_work().sum(axis=0))
            times.append([tm["p2p"], tm["m2l"], tm["s2m"] + tm["s2l"] + tm["l2t"],
                          tm["upward"] + tm["downward"] + tm["pack"] + tm["combine"]])
    fmm.set_option("overlap", "1")
    A, T = np.array(rows), np.array(times) * 1e-3
    lane, entry = np.linalg.lstsq(A[:, :2], T[:, 0], rcond=None)[0]
    flop = np.linalg.lstsq(A[:, 2:3], T[:, 1], rcond=None)[0][0]
    ev = np.linalg.lstsq(A[:, 3:4], T[:, 2], rcond=None)[0][0]
    box = np.linalg.lstsq(np.c_[A[:, 4], np.ones(len(A))], T[:, 3], rcond=None)[0][0]
    return [float(max(v, 0.0)) for v in (lane, entry, flop, ev, box)]


def label_set(fmm, torch, seed, costs, tol=1e-5, per_leaf=4, p_cap=8):
    """Features and (order, capacity) labels of every leaf with targets of one mixture."""
    d = W.mixture(seed, N_RANGE)
    x = torch.from_numpy(d["xyz"]).cuda()
    f = torch.from_numpy(d["f"]).cuda()
    outs = {}
    for p in ORDER_CLASSES:
        fmm.set_points("Stokeslet", x, None, x, p=p, leaf_cap=2000)
        outs[p] = fmm.run(f).clone()
    feat, leaf_of = fmm.leaf_features()
    # capacity: each uniform-capacity plan's work on the leaf's targets, priced
    learned_compression(fmm, tol)
    cap_cost = cap_costs(fmm, torch, x, costs, len(feat), leaf_of, p_cap)
    # sampled targets: up to per_leaf per leaf, spread over the leaf
    rng = np.random.default_rng(seed)
    order = np.argsort(leaf_of, kind="stable")
    bounds = np.searchsorted(leaf_of[order], np.arange(len(feat) + 1))
    sidx, sleaf = [], []
    for L in range(len(feat)):
        members = order[bounds[L]:bounds[L + 1]]
        if len(members) == 0:
            continue
        take = rng.choice(members, size=min(per_leaf, len(members)), replace=False)
        sidx.append(take)
        sleaf.append(np.full(len(take), L))
    sidx = np.concatenate(sidx)
    sleaf = np.concatenate(sleaf)
    ti = torch.from_numpy(sidx).cuda()
    ref = fmm.direct("Stokeslet", x, f, None, None, x[ti].contiguous()).cpu().numpy()
    keep = np.unique(sleaf)
    labels = np.zeros((len(keep), 2), dtype=np.int32)
    errs = np.zeros((len(keep), len(ORDER_CLASSES)))
    rms_all = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
    cnt = np.bincount(sleaf, minlength=len(feat)).astype(np.float64)
    for k, p in enumerate(ORDER_CLASSES):
        got = outs[p][ti].cpu().numpy()
        num = np.zeros(len(feat))
        np.add.at(num, sleaf, np.sum((got - ref) ** 2, axis=1))
        errs[:, k] = np.sqrt(num[keep] / cnt[keep]) / rms_all      # leaf RMS error / global RMS field
    labels[:, 0] = order_labels(errs, tol)
    labels[:, 1] = cap_cost[keep].argmin(axis=1)
    return feat[keep], labels, errs, {"seed": seed, "n": len(d["xyz"]), "leaves": len(feat), "k": d["k"]}


def relabel_caps(fmm, torch, seed, costs, p_cap=8):
    """Capacity labels of one mixture's leaves (the rows `label_set` kept: every
    leaf of the leaf_cap 2000 tree, all of which hold targets) under new unit
    costs; the order labels do not depend on them."""
    d = W.mixture(seed, N_RANGE)
    x = torch.from_numpy(d["xyz"]).cuda()
    fmm.set_points("Stokeslet", x, None, x, p=p_cap, leaf_cap=2000)
    feat, leaf_of = fmm.leaf_features()
    learned_compression(fmm)
    cost = cap_costs(fmm, torch, x, costs, len(feat), leaf_of, p_cap)
    keep = np.unique(leaf_of)
    return feat[keep], cost[keep].argmin(axis=1).astype(np.int32)


def train(X, Y, epochs=60, batch=1024, lr=2e-3, seed=0, log=None):
    """Train on the GPU with the library's kernels; returns float32 parameters."""
    import torch
    mean = X.mean(0)
    std = X.std(0) + 1e-3
    theta = init_params(seed, mean, std)
    p = torch.from_numpy(theta).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    rng = np.random.default_rng(seed)
    Xt = torch.from_numpy(X.astype(np.float32)).cuda()
    Yt = torch.from_numpy(Y.astype(np.int32)).cuda()
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(X))).cuda()
        tot = 0.0
        nb = 0
        for s in range(0, len(X) - batch + 1, batch):
            idx = perm[s:s + batch]
            step += 1
            loss, g = mlp_loss_grad(p, Xt[idx].contiguous(), Yt[idx].contiguous())
            mlp_adam(p, g, m, v, step, lr)
            tot += float(loss.cpu())
            nb += 1
        if log is not None:
            log.append({"epoch": ep, "loss": tot / max(nb, 1)})
    return p.cpu().numpy()


def init_params(seed, mean, std):
    """He-initialised parameters in the library's layout (mean, std, W1, b1, W2, b2, W3, b3)."""
    rng = np.random.default_rng(seed)
    F, H, C = 12, 64, 8
    parts = [np.asarray(mean, np.float64), np.asarray(std, np.float64)]
    for fi, fo in ((F, H), (H, H), (H, C)):
        parts.append(rng.standard_normal(fi * fo) * np.sqrt(2.0 / fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--seeds", default="501:701")
    a.add_argument("--out", required=True)
    a.add_argument("--costs", default="", help="five unit costs (default: fit them first)")
    r = sub.add_parser("relabel-caps")
    r.add_argument("--data", required=True)
    r.add_argument("--out", required=True)
    r.add_argument("--costs", default="", help="five unit costs (default: fit them first)")
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--epochs", type=int, default=60)
    args = ap.parse_args(argv)
    import torch
    if args.cmd == "label":
        fmm = FMM()
        costs = [float(r) for r in args.costs.split(",")] if args.costs else fit_costs(fmm, torch)
        print(json.dumps({"costs": costs}), flush=True)
        lo, hi = (int(s) for s in args.seeds.split(":"))
        Xs, Ys, Es, meta = [], [], [], []
        for seed in range(lo, hi):
            t0 = time.time()
            X, Y, E, info = label_set(fmm, torch, seed, costs)
            Xs.append(X)
            Ys.append(Y)
            Es.append(E)
            info.update(secs=time.time() - t0, order_hist=np.bincount(Y[:, 0], minlength=4).tolist(),
                        cap_hist=np.bincount(Y[:, 1], minlength=4).tolist())
            meta.append(info)
            print(json.dumps(info), flush=True)
            np.savez(args.out, X=np.concatenate(Xs), Y=np.concatenate(Ys), E=np.concatenate(Es),
                     costs=np.array(costs), seeds=np.array([m["seed"] for m in meta]))
    elif args.cmd == "relabel-caps":
        fmm = FMM()
        costs = [float(r) for r in args.costs.split(",")] if args.costs else fit_costs(fmm, torch)
        print(json.dumps({"costs": costs}), flush=True)
        old = np.load(args.data, allow_pickle=False)
        X, Y = old["X"].copy(), old["Y"].copy()
        row = 0
        for seed in old["seeds"]:
            t0 = time.time()
            feat, cap = relabel_caps(fmm, torch, int(seed), costs)
            n = len(feat)
            if not np.allclose(feat, X[row:row + n], rtol=1e-5, atol=1e-6):
                raise RuntimeError("seed %d: leaves differ from the stored rows" % seed)
            changed = int((Y[row:row + n, 1] != cap).sum())
            Y[row:row + n, 1] = cap
            row += n
            print(json.dumps({"seed": int(seed), "leaves": n, "changed": changed,
                              "cap_hist": np.bincount(cap, minlength=4).tolist(),
                              "secs": time.time() - t0}), flush=True)
        if row != len(X):
            raise RuntimeError("stored rows %d, relabelled %d" % (len(X), row))
        np.savez(args.out, X=X, Y=Y, E=old["E"], costs=np.array(costs), seeds=old["seeds"])
    else:
        data = [np.load(f, allow_pickle=False) for f in args.data]
        X = np.concatenate([d["X"] for d in data])
        Y = np.concatenate([d["Y"] for d in data])
        E = np.concatenate([d["E"] for d in data])
        Y[:, 0] = order_labels(E)
        log = []
        w = train(X, Y, epochs=args.epochs, log=log)
        # calibration table on the network's own predicted classes
        import torch
        from . import mlp_forward
        logits = mlp_forward(torch.from_numpy(w).cuda(), torch.from_numpy(X.astype(np.float32)).cuda()).cpu().numpy()
        pred = logits[:, :4].argmax(axis=1)
        table = calibration_table(E, pred)
        np.save(args.out, np.concatenate([w, table.reshape(-1)]).astype(np.float32), allow_pickle=False)
        acc = [float((pred == Y[:, 0]).mean()), float((logits[:, 4:].argmax(axis=1) == Y[:, 1]).mean())]
        print(json.dumps({"table": table.tolist(), "train_accuracy": acc}), flush=True)
        print(json.dumps({"rows": len(X), "final_loss": log[-1]["loss"], "first_loss": log[0]["loss"],
                          "order_hist": np.bincount(Y[:, 0], minlength=4).tolist(),
                          "cap_hist": np.bincount(Y[:, 1], minlength=4).tolist()}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
