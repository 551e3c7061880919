"""Benchmark of the kernel aggregated FMM evaluation pass on one MI355X.

Workload: 1,048,576 points from an 8-cluster Gaussian mixture (sigma 0.05)
in the unit cube, forces N(0,1)^3, RPY radii U[0.002, 0.005]; sources =
targets, open boundary.  A step is one evaluation pass (stkfmm_run: pack,
S2M, upward sweep, M2L, S2L, downward sweep, L2T/M2T, P2P, combine) of the
Stokeslet with the tree already built and every input resident in HBM.  The
plan (tree build, operators and, in learned mode, the prediction and its
one-time sampled FP64 accuracy check) is timed separately, as the paper
times the tree build separately.

The headline value is the learned mode: order p and per-leaf leaf_cap
predicted by the trained network for a relative L2 tolerance of 1e-5, with
the fixed p = 10 plan as fallback.  The fixed p = 10, leaf_cap = 2000 plan
is measured beside it, and every variant reports its relative L2 error
against the FP64 direct sum on 4096 sampled targets.  Prints one JSON line.
Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 flops per P2P pair (FMA = 2, rsqrt = 1), counted on the
# kernel formulas without the hi/lo coordinate refinement: r, r^2 and rsqrt
# 9, then Stokeslet +19, RPY +41, Laplace charge +11 and dipole +24 (the
# periodic Laplace row has as many dipole as charge pairs: 26.5 on average),
# double-layer PVel +37 and Traction +72
P2P_FLOPS = {"Stokeslet": 28, "RPY": 50, "LapPGrad": 26.5, "PVel": 46, "Traction": 81}
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_MFMA_PEAK_TFLOPS = 157.3      # dense MFMA, MI355X
BF16_MFMA_PEAK_TFLOPS = 2500.0
PROFILE = os.path.join(ROOT, "profiles", "p2p_stokeslet_1M_clustered_learned.md")
PROFILE_M2L = os.path.join(ROOT, "profiles", "m2l_gemm_1M_clustered_learned.md")
# the sources that decide a launch's work and traffic: the kernels and the
# plan that sizes their tasks
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2010_15155_amd", "csrc", f) for f in ("kernels.hip", "kernel_math.hpp", "api.hip")]


def measured_traffic(profile=PROFILE):
    """HBM bytes per launch of a kernel of the learned-mode plan from its
    committed PMC summary (P2P by default), or None when the kernel sources
    changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(l.split(": ", 1) for l in open(profile).read().splitlines() if ": " in l
                      and l.split(": ", 1)[0] in ("traffic_bytes_per_launch", "source_sha256"))
        h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
        if fields.get("source_sha256", "").strip() != h:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--samples", type=int, default=4096, help="targets checked by the FP64 GPU direct sum")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="measure the learned Stokeslet plan only (for profiler runs)")
    ap.add_argument("--only-variant", choices=["fixed_p10", "learned_split_bf16"], default=None,
                    help="measure one other 1M Stokeslet plan only (for profiler runs)")
    ap.add_argument("--only-plan", action="store_true",
                    help="measure the plan time with the GPU and the host tree builders only")
    ap.add_argument("--only-periodic", action="store_true",
                    help="measure the triply periodic Stokeslet row only")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the measurement, copy a MIB-sized device buffer once (reference "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    return args


FIELDS = {"Stokeslet": [("u", 0, 3)], "StokesRegVel": [("u", 0, 3)], "RPY": [("u", 0, 3), ("lap_u", 3, 6)],
          "PVel": [("p", 0, 1), ("u", 1, 4)]}


def wall_direct(fmm, torch, y, fb, xt):
    """(u, lap u) of RPY above the wall z = 0 at targets xt: the image
    summations of the paper's wall table (with the SD charges -f3/2, +f3/2
    and the quadrupole at the image), each by the library's FP64 direct sum,
    assembled in FP64 -- the reference for the wall plan's error."""
    f, b = fb[:, :3], fb[:, 3]
    h = y[:, 2]
    yi = y * torch.tensor([1.0, 1.0, -1.0], dtype=y.dtype, device=y.device)
    y2 = torch.cat([y, yi]).contiguous()
    z = torch.zeros_like(h)
    vs = torch.cat([torch.stack([f[:, 0], f[:, 1], z, b], 1), torch.stack([-f[:, 0], -f[:, 1], z, b], 1)])
    S = fmm.direct("RPY", y2, vs.contiguous(), None, None, xt)
    sd_q = torch.cat([-0.5 * f[:, 2], 0.5 * f[:, 2]])[:, None].contiguous()
    sd_d = (h[:, None] * torch.stack([-f[:, 0], -f[:, 1], f[:, 2]], 1)).contiguous()
    SD = fmm.direct("LapPGradGrad", y2, sd_q, yi.contiguous(), sd_d, xt)
    dz = torch.stack([z, z, b * b / 6.0 * f[:, 2]], 1)
    Z = fmm.direct("LapPGrad", y2, torch.cat([0.5 * h * f[:, 2], -0.5 * h * f[:, 2]])[:, None].contiguous(),
                   y2, torch.cat([dz, dz]).contiguous(), xt)
    Q = torch.zeros((len(y), 9), dtype=y.dtype, device=y.device)
    Q[:, 0] = f[:, 2]
    Q[:, 4] = f[:, 2]
    Q[:, 6] = f[:, 0]
    Q[:, 7] = f[:, 1]
    Q *= (b * b / 3.0)[:, None]
    QP = fmm.direct("LapQPGradGrad", yi.contiguous(), Q, None, None, xt)
    x3 = xt[:, 2:3]
    u = S[:, :3] + Z[:, 1:4] + x3 * (SD[:, 1:4] + QP[:, 1:4])
    u[:, 2] -= SD[:, 0] + QP[:, 0]
    col3 = lambda H: torch.stack([H[:, 6], H[:, 8], H[:, 9]], 1)
    return torch.cat([u, S[:, 3:] + 2.0 * (col3(SD) + col3(QP))], 1)


def measure(fmm, torch, W, kernel, x, val, p, cap, args, precision="fp32", bc="open"):
    """Plan once, then time `steps` evaluation passes after `warmup`; error on
    sampled targets against the FP64 GPU direct sum."""
    learned = p == 0 or cap == 0
    fmm.set_option("precision", precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fmm.set_points(kernel, x, None, x, p=p, leaf_cap=cap, bc=bc)
    t_tree = fmm.timings()["t_tree_ms"]
    if learned:
        fmm.run(val)                  # the first run of a learned plan carries its accuracy check
    torch.cuda.synchronize()
    t_plan = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        fmm.run(val)
    torch.cuda.synchronize()
    p2p_ms, run_ms, gemm_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = fmm.run(val)
        tm = fmm.timings()
        p2p_ms.append(tm["stages_ms"]["p2p"])
        gemm_ms.append(tm["stages_ms"]["m2l_gemm"])
        run_ms.append(tm["t_run_ms"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    st = fmm.stats()
    info = fmm.learned_info() if learned else None
    # one serial pass (P2P before the far field) for standalone stage times
    fmm.set_option("overlap", "0")
    fmm.run(val)
    serial = fmm.timings()
    fmm.set_option("overlap", "1")
    idx = torch.from_numpy(W.sample_indices(len(x), args.samples, 7)).cuda()
    # the FP64 GPU direct sum on sampled targets (the library's own judge);
    # the error against the CPU oracle is added by the cpu_baseline leg
    if bc == "wall":
        ref = wall_direct(fmm, torch, x, val, x[idx].contiguous())
    else:
        ref = fmm.direct(kernel, x, val, None, None, x[idx].contiguous())
    got = out[idx]
    fields = FIELDS[kernel]
    errs = {n: float(torch.linalg.norm(got[:, a:b] - ref[:, a:b]) / torch.linalg.norm(ref[:, a:b]))
            for n, a, b in fields}
    fmm.set_option("precision", "fp32")
    r = {"_out": out, "ms_per_step": wall * 1e3, "targets_per_s": len(x) / wall, "run_ms_median": float(np.median(run_ms)),
         "p2p_ms": float(np.mean(p2p_ms)), "p2p_pairs_per_s": st["p2p_pairs"] / (np.mean(p2p_ms) * 1e-3),
         "m2l_gemm_ms": float(np.mean(gemm_ms)),
         "rel_l2_gpu_fp64_direct": errs, "t_tree_ms": t_tree, "t_plan_ms": t_plan, "stages_ms": tm["stages_ms"],
         "stages_serial_ms": serial["stages_ms"], "run_serial_ms": serial["t_run_ms"], "plan": st,
         "p": info["p"] if info else p, "leaf_cap": "per leaf" if cap == 0 else cap, "precision": precision,
         "bc": bc}
    if info:
        r["learned"] = info
    return r


def periodic_stokeslet(FMM, torch, n, args, p=8, cap=500, kernel="Stokeslet"):
    """Triply periodic Stokeslet (or RPY, radii U[0.002, 0.005]; or PVel, half
    the points single-layer (f, q), half double-layer D, every point a
    target) on n uniform points (zero net force, flux and tr D): time per
    pass, and as accuracy the translation test, the relative difference
    between the pass and the pass on all points moved together (PVel's
    pressure up to a constant; a sampled Ewald reference at this size is
    beyond the CPU oracle's budget)."""
    rng = np.random.default_rng(501)
    x = rng.random((n, 3))
    ns = n // 2 if kernel == "PVel" else n
    f = rng.standard_normal((ns, 3))
    f -= f.mean(axis=0)
    dl = dd = None
    if kernel == "RPY":
        f = np.concatenate([f, rng.uniform(0.002, 0.005, (n, 1))], 1)
    elif kernel == "PVel":
        q = rng.standard_normal(ns)
        f = np.concatenate([f, (q - q.mean())[:, None]], 1)
        D = rng.standard_normal((n - ns, 9))
        D[:, [0, 4, 8]] -= (D[:, 0] + D[:, 4] + D[:, 8]).mean() / 3.0
        dd = torch.from_numpy(D).cuda()
    fmm = FMM()

    def plan(shift):
        xs = torch.from_numpy(np.mod(x + shift, 1.0)).cuda()
        sl = xs[:ns]
        dl = xs[ns:] if kernel == "PVel" else None
        fmm.set_points(kernel, sl, dl, xs, p=p, leaf_cap=cap, bc="PXYZ")

    fd = torch.from_numpy(f).cuda()
    plan(np.zeros(3))
    for _ in range(args.warmup):
        fmm.run(fd, dd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = fmm.run(fd, dd)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    out = out.clone()
    stages = fmm.timings()["stages_ms"]
    plan(np.array([0.31, 0.57, 0.89]))
    out2 = fmm.run(fd, dd)
    diff = {}
    for name, a, b in FIELDS[kernel]:
        d = out2[:, a:b] - out[:, a:b]
        ref = out[:, a:b]
        if kernel == "PVel" and name == "p":
            d, ref = d - d.mean(), ref - ref.mean()
        diff[name] = float(torch.linalg.norm(d) / torch.linalg.norm(ref))
    fmm.close()
    what = {"PVel": "%d single-layer and %d double-layer sources, every point a target" % (ns, n - ns)}
    return {"ms_per_step": wall * 1e3, "targets_per_s": n / wall, "p": p, "leaf_cap": cap,
            "translation_rel_diff": diff, "stages_ms": stages,
            "workload": "%d uniform points in the unit cube, %s, PXYZ, zero net force%s%s" % (
                n, kernel, ", flux and tr D" if kernel == "PVel" else "",
                "; " + what[kernel] if kernel in what else "")}


def tree_build(FMM, x):
    """Plan time (stkfmm_set_points: octree, lists and plan arrays; operators
    cached) with the octree and lists built by the GPU kernels or on the host,
    at fixed leaf capacities and for the learned plan (two trees, the leaf
    features and the network)."""
    from paper_2010_15155_amd.predictor import load_weights
    out = {}
    row = {}
    for how in ("gpu", "host"):
        f = FMM()
        f.set_option("tree", how)
        f.set_predictor(load_weights())
        ts = []
        for _ in range(4):
            f.set_points("Stokeslet", x, None, x, p=0, leaf_cap=0)
            ts.append(f.timings()["t_tree_ms"])
        row[how + "_ms"] = float(np.median(ts[1:]))
        f.close()
    out["learned"] = row
    for cap in (2000, 500):
        row = {}
        for how in ("gpu", "host"):
            f = FMM()
            f.set_option("tree", how)
            ts = []
            for _ in range(4):
                f.set_points("Stokeslet", x, None, x, p=8, leaf_cap=cap)
                ts.append(f.timings()["t_tree_ms"])
            row[how + "_ms"] = float(np.median(ts[1:]))
            row["boxes"] = f.stats()["boxes"]
            f.close()
        out["leaf_cap_%d" % cap] = row
    return out


def periodic_laplace_4m(FMM, torch, W, args, n=4_194_304, p=12, caps=(2000, 500)):
    """Triply periodic Laplace charges + dipoles (zero net charge) on n uniform
    points, SL = DL = targets, p = 12: at leaf_cap 2000 (the paper's leaf
    size) and at 500 (eight times fewer P2P pairs on uniform points), each
    with time per pass, P2P rate, the translation test of the periodic
    boundary (all points moved by one vector, wrapped) and the sampled
    outputs that the cpu_baseline leg checks against the Ewald oracle."""
    d = W.periodic_laplace(n, 301)
    x = torch.from_numpy(d["xyz"]).cuda()
    q = torch.from_numpy(d["q"][:, None].copy()).cuda()
    dp = torch.from_numpy(d["d"]).cuda()
    idx = W.sample_indices(n, 24, 9)
    s = np.array([0.37, 0.61, 0.18])
    xs = torch.from_numpy(np.mod(d["xyz"] + s, 1.0)).cuda()
    rows = {}
    fmm = FMM()
    for cap in caps:
        fmm.set_points("LapPGrad", x, x, x, p=p, leaf_cap=cap, bc="PXYZ")
        r = timed_runs(fmm, torch, args, q, dp)
        out = r.pop("_out")
        r["_sample"] = {"idx": idx, "got": out[torch.from_numpy(idx).cuda()].cpu().numpy()}
        fmm.set_points("LapPGrad", xs, xs, xs, p=p, leaf_cap=cap, bc="PXYZ")
        out2 = fmm.run(q, dp)
        dphi = out2[:, 0] - out[:, 0]
        r["translation_rel_diff"] = {
            "phi": float(torch.linalg.norm(dphi - dphi.mean()) / torch.linalg.norm(out[:, 0] - out[:, 0].mean())),
            "grad_phi": float(torch.linalg.norm(out2[:, 1:] - out[:, 1:]) / torch.linalg.norm(out[:, 1:]))}
        del out, out2
        r.update({"p": p, "leaf_cap": cap, "roofline": p2p_roofline("LapPGrad", r)})
        rows["leaf_cap_%d" % cap] = r
    fmm.close()
    rows["_d"] = d
    rows["workload"] = ("%d uniform points in the unit cube, Laplace charges N(0,1) minus their mean and "
                        "dipoles N(0,1)^3, SL = DL = targets, PXYZ" % n)
    return rows


def sphere_doublelayer_2m(FMM, torch, W, args, p=10, cap=2000):
    """Stokes double layer on the surfaces of 2000 spheres (radius 0.01, 1000
    Fibonacci points each, N = 2,000,000), D = v n^T, DL = targets, p = 10,
    leaf_cap 2000: PVel -> (p, u) and Traction -> sigma, each timed, with
    sampled outputs for the cpu_baseline leg's oracle check."""
    d = W.sphere_doublelayer(n_spheres=2000, pts_per_sphere=1000, seed=401)
    x = torch.from_numpy(d["xyz"]).cuda()
    D = torch.from_numpy(d["D"]).cuda()
    idx = W.sample_indices(len(d["xyz"]), 1500, 4)
    rows = {}
    fmm = FMM()
    for kernel in ("PVel", "Traction"):
        fmm.set_points(kernel, None, x, x, p=p, leaf_cap=cap)
        r = timed_runs(fmm, torch, args, None, D)
        out = r.pop("_out")
        r["_sample"] = {"idx": idx, "got": out[torch.from_numpy(idx).cuda()].cpu().numpy()}
        r.update({"p": p, "leaf_cap": cap, "roofline": p2p_roofline(kernel, r)})
        rows[kernel] = r
    fmm.close()
    rows["_d"] = d
    rows["workload"] = ("%d points on 2000 spheres of radius 0.01 (1000 Fibonacci points each), Stokes "
                        "double layer D = v n^T, v ~ N(0,1)^3, DL = targets, open BC" % len(d["xyz"]))
    return rows


def uniform_4096(FMM, torch, W, args, p=8, cap=64):
    """The small configuration (4096 uniform points, seed 101; the case the
    plain FP64 oracle KIFMM also runs): the GPU pass here, while the CPU leg
    times that oracle KIFMM on the same points and judges both against the
    oracle's direct sum over all 4096 targets."""
    d = W.uniform_stokeslet()
    fmm = FMM()
    r = measure(fmm, torch, W, "Stokeslet", torch.from_numpy(d["xyz"]).cuda(), torch.from_numpy(d["f"]).cuda(),
                p, cap, args)
    fmm.close()
    r["_sample"] = {"got": r.pop("_out").cpu().numpy()}
    r["_d"] = d
    return r


def timed_runs(fmm, torch, args, sl, dl):
    """Warm-up and timed passes of the current plan, with P2P launch times."""
    for _ in range(args.warmup):
        fmm.run(sl, dl)
    torch.cuda.synchronize()
    p2p_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = fmm.run(sl, dl)
        p2p_ms.append(fmm.timings()["stages_ms"]["p2p"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    st = fmm.stats()
    fmm.set_option("overlap", "0")
    fmm.run(sl, dl)
    serial = fmm.timings()
    fmm.set_option("overlap", "1")
    n_trg = st["n_trg"]
    return {"_out": out, "ms_per_step": wall * 1e3, "targets_per_s": n_trg / wall, "p2p_ms": float(np.mean(p2p_ms)),
            "p2p_pairs_per_s": st["p2p_pairs"] / (np.mean(p2p_ms) * 1e-3), "stages_serial_ms": serial["stages_ms"],
            "run_serial_ms": serial["t_run_ms"], "plan": st}


def m2l_roofline(r, ncomp=4, learned_fp32=False):
    """Roofline entry of the V-list GEMM (compressed translations) of a row:
    2 kc^2 ncomp flops per V pair over the launch's live time (HIP events
    around that launch on the far-field stream) against the MFMA peak of its
    arithmetic: FP32, or BF16 for the three-pass split (3x the flops)."""
    kc, npairs = r["plan"]["m2l_rank"], r["plan"]["v_pairs"]
    if kc == 0 or r["m2l_gemm_ms"] <= 0:
        return None
    passes, peak = (3, BF16_MFMA_PEAK_TFLOPS) if r["precision"] == "split_bf16" else (1, FP32_MFMA_PEAK_TFLOPS)
    flops = passes * 2.0 * kc * kc * ncomp * npairs
    f = flops / (r["m2l_gemm_ms"] * 1e-3) / 1e12
    # the committed counters cover the learned FP32 plan's launch only
    traffic = measured_traffic(PROFILE_M2L) if learned_fp32 else None
    name = ("gemm_bf16x3_" if passes == 3 else "gemm_f32_") + ("strip<5>" if kc == 160 else "mfma")
    return {"kernel": name, "bound": "mfma", "achieved": f,
            "peak": peak, "unit": "TFLOP/s", "frac": f / peak, "traffic": traffic,
            "flops_per_launch": flops, "rank": kc, "v_pairs": npairs, "avg_launch_ms": r["m2l_gemm_ms"]}


def p2p_roofline(kernel, r):
    """Roofline entry of the P2P kernel of a row: algorithmic FP32 flops
    (P2P_FLOPS per pair) over its live launch time against the FP32 vector peak."""
    f = P2P_FLOPS[kernel] * r["plan"]["p2p_pairs"] / (r["p2p_ms"] * 1e-3) / 1e12
    return {"kernel": "p2p_kernel", "bound": "alu", "achieved": f, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": f / FP32_VECTOR_PEAK_TFLOPS, "flops_per_pair": P2P_FLOPS[kernel],
            "pairs_per_launch": r["plan"]["p2p_pairs"], "avg_launch_ms": r["p2p_ms"]}


def uniform_capacities(FMM, torch, W, x, f, args, p=8, m2l_tol="2e-7"):
    """Fixed order p with one leaf capacity everywhere, at the translation
    rank the learned plan uses (m2l_tol = tol/50), on a context of its own:
    the best of these is what the network's per-leaf capacities are measured
    against."""
    rows = {}
    fmm = FMM()
    fmm.set_option("m2l_tol", m2l_tol)
    for cap in (250, 500, 1000, 2000):
        rows["cap_%d" % cap] = measure(fmm, torch, W, "Stokeslet", x, f, p, cap, args)
    fmm.close()
    return rows


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the evaluation pass is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2010_15155_amd import FMM, workloads as W
    from paper_2010_15155_amd.predictor import load_weights

    d = W.clustered_rpy(args.n, 201)
    x = torch.from_numpy(d["xyz"]).cuda()
    f = torch.from_numpy(d["f"]).cuda()
    if args.only_plan:
        print(json.dumps({"plan_ms": tree_build(FMM, x)}), flush=True)
        return
    if args.only_periodic:
        print(json.dumps({k.lower() + "_pxyz_p8": periodic_stokeslet(FMM, torch, args.n, args, kernel=k)
                          for k in ("Stokeslet", "RPY", "PVel")}), flush=True)
        return
    fmm = FMM()
    fmm.set_predictor(load_weights())
    if args.only_variant:
        p, cap, prec = (10, 2000, "fp32") if args.only_variant == "fixed_p10" else (0, 0, "split_bf16")
        r = measure(fmm, torch, W, "Stokeslet", x, f, p, cap, args, prec)
        r.pop("_out")
        r["roofline_m2l"] = m2l_roofline(r)
        fmm.close()
        print(json.dumps({args.only_variant: r}), flush=True)
        return
    L = measure(fmm, torch, W, "Stokeslet", x, f, 0, 0, args)
    n = args.n
    flops = P2P_FLOPS["Stokeslet"] * L["plan"]["p2p_pairs"]
    achieved = flops / (L["p2p_ms"] * 1e-3) / 1e12
    line = {
        "metric": "targets/sec (Stokeslet N=1M, rel L2 err <=1e-5) learned-p vs fixed p=10; P2P pairs/s",
        "value": L["targets_per_s"],
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": L["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Stokeslet evaluation pass, N=%d points (8-cluster Gaussian mixture, "
                               "sigma 0.05), sources = targets, open BC" % n,
                   "order_mode": "learned (order and per-leaf leaf_cap predicted for tol 1e-5, "
                                 "fallback fixed p=10, leaf_cap 2000)"},
        "rel_l2_gpu_fp64_direct": L["rel_l2_gpu_fp64_direct"],
        "p2p_pairs_per_s": L["p2p_pairs_per_s"],
        "learned": L,
        "roofline": {"kernel": "p2p_kernel<DStokeslet>", "bound": "alu", "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(),
                     "flops_per_pair": P2P_FLOPS["Stokeslet"], "pairs_per_launch": L["plan"]["p2p_pairs"],
                     "avg_launch_ms": L["p2p_ms"]},
        "roofline_m2l": m2l_roofline(L, learned_fp32=True),
    }
    checked = {"learned": L}          # rows whose outputs the cpu_baseline leg checks against the oracle
    configs = {}
    if not args.only_headline:
        F = measure(fmm, torch, W, "Stokeslet", x, f, 10, 2000, args)
        line["fixed_p10"] = checked["fixed_p10"] = F
        line["learned_speedup_vs_fixed_p10"] = F["ms_per_step"] / L["ms_per_step"]
        line["learned_split_bf16"] = checked["learned_split_bf16"] = measure(
            fmm, torch, W, "Stokeslet", x, f, 0, 0, args, "split_bf16")
        F["roofline_m2l"] = m2l_roofline(F)
        line["learned_split_bf16"]["roofline_m2l"] = m2l_roofline(line["learned_split_bf16"])
        fb = torch.from_numpy(np.concatenate([d["f"], d["b"][:, None]], 1)).cuda()
        line["rpy_fixed_p10"] = checked["rpy_fixed_p10"] = measure(fmm, torch, W, "RPY", x, fb, 10, 2000, args)
        U = uniform_capacities(FMM, torch, W, x, f, args)
        best = min(U, key=lambda k: U[k]["ms_per_step"])
        line["uniform_capacities_p8"] = {k: {"ms_per_step": v["ms_per_step"], "rel_l2_gpu_fp64_direct":
                                             v["rel_l2_gpu_fp64_direct"], "leaf_cap": v["leaf_cap"]}
                                         for k, v in U.items()}
        line["learned_speedup_vs_best_uniform_p8"] = U[best]["ms_per_step"] / L["ms_per_step"]
        for v in U.values():
            v.pop("_out")
        # the widened rows on the same points: regularized Stokeslet (blob
        # sizes well below the smallest leaves) and RPY above a no-slip wall
        # at z = 0 (the points lie above it)
        rng = np.random.default_rng(202)
        fe = torch.from_numpy(np.concatenate([d["f"], rng.uniform(5e-5, 1e-4, (n, 1))], 1)).cuda()
        line["widened"] = {
            "stokes_reg_vel_p8": measure(fmm, torch, W, "StokesRegVel", x, fe, 8, 1000, args),
            "rpy_wall_p10": measure(fmm, torch, W, "RPY", x, fb, 10, 1000, args, bc="wall"),
            "stokeslet_pxyz_p8": periodic_stokeslet(FMM, torch, n, args),
            "rpy_pxyz_p8": periodic_stokeslet(FMM, torch, n, args, kernel="RPY"),
            "pvel_pxyz_p8": periodic_stokeslet(FMM, torch, n, args, kernel="PVel"),
        }
        for k in ("stokes_reg_vel_p8", "rpy_wall_p10"):
            line["widened"][k].pop("_out")
        configs["uniform_4096_p8"] = uniform_4096(FMM, torch, W, args)
        configs["periodic_laplace_4M_p12"] = periodic_laplace_4m(FMM, torch, W, args)
        configs["sphere_doublelayer_2M_p10"] = sphere_doublelayer_2m(FMM, torch, W, args)
        line["plan_ms"] = tree_build(FMM, x)
    fmm.close()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(d, args.cpu_seconds, checked, configs)
        line["rel_l2"] = line["cpu_baseline"]["rel_l2_vs_oracle"]["learned"]
    for r in checked.values():
        r.pop("_out", None)
    if configs:
        line["configs"] = configs
        for c in configs.values():
            c.pop("_d", None)
            for r in [c] + [v for v in c.values() if isinstance(v, dict)]:
                r.pop("_sample", None)
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibrate_copy_bytes"] = args.calibrate_copy * (1 << 20)
    print(json.dumps(line), flush=True)


def rel_fields(got, ref, fields):
    return {name: float(np.linalg.norm(got[:, a:b] - ref[:, a:b]) / np.linalg.norm(ref[:, a:b]))
            for name, a, b in fields}


def cpu_baseline(d, budget_s, checked, configs):
    """The CPU leg.  Times the FP64 oracle direct sum on the host cores on a
    bounded sample of targets (all sources), scaled to targets/s, with all its
    OpenMP threads and with one; then judges the GPU rows by the oracle: the
    1M Stokeslet / RPY plans on those sampled targets, the periodic Laplace
    row against the Ewald oracle on 24 sampled targets and the sphere double
    layer rows against the direct sums on 1500 sampled targets."""
    import platform
    from oracle import direct, ewald
    from paper_2010_15155_amd import workloads as W
    x, f = d["xyz"], d["f"]
    n = len(x)
    threads = direct.max_threads()
    # calibrate on a small sample, then size the timed sample to the budget
    t0 = time.perf_counter()
    direct.stokeslet(x, f, x[:512])
    per_target = (time.perf_counter() - t0) / 512
    k = int(max(512, min(n, budget_s / max(per_target, 1e-9))))
    idx = W.sample_indices(n, k, 11)
    t0 = time.perf_counter()
    ref = direct.stokeslet(x, f, x[idx])
    dt = time.perf_counter() - t0
    # one thread, on a sample sized to about a tenth of the budget
    k1 = int(max(16, min(k, 0.1 * budget_s / max(per_target * threads, 1e-9))))
    direct.set_threads(1)
    try:
        t0 = time.perf_counter()
        direct.stokeslet(x, f, x[idx[:k1]])
        dt1 = time.perf_counter() - t0
    finally:
        direct.set_threads(threads)
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        model = platform.processor()
    out = {"value": k / dt, "unit": "targets/s", "cores": threads, "kind": "oracle",
           "sample": "%d sampled targets x %d sources, FP64 direct Stokeslet sum (C, OpenMP, %d threads)"
                     % (k, n, threads),
           "seconds": dt, "pairs_per_s": k * n / dt, "cpu_model": model, "host_cpus": os.cpu_count(),
           "one_thread": {"value": k1 / dt1, "unit": "targets/s", "targets": k1, "seconds": dt1,
                          "pairs_per_s": k1 * n / dt1}}
    # the GPU rows judged by the oracle on the same sampled targets
    errs = {}
    fb = np.concatenate([f, d["b"][:, None]], 1)
    ref_rpy = None
    for name, r in checked.items():
        got = r["_out"][torch_index(r["_out"], idx)].cpu().numpy()
        if name.startswith("rpy"):
            if ref_rpy is None:
                kr = min(k, 4096)
                ref_rpy = direct.rpy(x, fb, x[idx[:kr]])
            errs[name] = rel_fields(got[:len(ref_rpy)], ref_rpy, FIELDS["RPY"])
        else:
            errs[name] = rel_fields(got, ref, FIELDS["Stokeslet"])
    out["rel_l2_vs_oracle"] = errs
    c1 = configs.get("uniform_4096_p8")
    if c1:
        from oracle import kifmm
        dd = c1["_d"]
        ref1 = direct.stokeslet(dd["xyz"], dd["f"], dd["xyz"])
        c1["rel_l2_vs_oracle"] = rel_fields(c1["_sample"]["got"], ref1, FIELDS["Stokeslet"])
        t0 = time.perf_counter()
        uk = kifmm.evaluate("Stokeslet", dd["xyz"], dd["f"], None, None, dd["xyz"], p=c1["p"], leaf_cap=c1["leaf_cap"])
        dtk = time.perf_counter() - t0
        out["kifmm_oracle_4096"] = {
            "value": len(dd["xyz"]) / dtk, "unit": "targets/s", "seconds": dtk, "p": c1["p"],
            "leaf_cap": c1["leaf_cap"], "rel_l2_vs_direct": rel_fields(uk, ref1, FIELDS["Stokeslet"]),
            "kind": "plain FP64 KIFMM oracle (NumPy, the paper's kernel tables)",
            "gpu_ms_per_step_same_points": c1["ms_per_step"]}
    c3 = configs.get("periodic_laplace_4M_p12")
    if c3:
        dd = c3["_d"]
        rows = [v for v in c3.values() if isinstance(v, dict) and "_sample" in v]
        idx3 = rows[0]["_sample"]["idx"]
        refp = ewald.laplace_periodic(dd["xyz"], dd["q"], dd["d"], dd["xyz"][idx3], 1.0, xi=4.0, tol=1e-12)
        for r in rows:
            got = r["_sample"]["got"]
            dphi = got[:, 0] - refp[:, 0]
            r["rel_l2_vs_oracle"] = {
                "phi": float(np.linalg.norm(dphi - dphi.mean()) / np.linalg.norm(refp[:, 0] - refp[:, 0].mean())),
                "grad_phi": float(np.linalg.norm(got[:, 1:] - refp[:, 1:]) / np.linalg.norm(refp[:, 1:])),
                "targets": len(idx3), "oracle": "Ewald sum (FP64, tin-foil, k = 0 term dropped)"}
    c4 = configs.get("sphere_doublelayer_2M_p10")
    if c4:
        dd = c4["_d"]
        for kernel, fields in (("PVel", [("p", 0, 1), ("u", 1, 4)]), ("Traction", [("sigma", 0, 9)])):
            sm = c4[kernel]["_sample"]
            refd = direct.evaluate(kernel, None, None, dd["xyz"], dd["D"], dd["xyz"][sm["idx"]])
            c4[kernel]["rel_l2_vs_oracle"] = dict(rel_fields(sm["got"], refd, fields), targets=len(sm["idx"]))
    return out


def torch_index(t, idx):
    import torch
    return torch.from_numpy(np.asarray(idx)).to(t.device)


if __name__ == "__main__":
    main()
