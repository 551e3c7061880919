"""Benchmark of the kernel aggregated FMM evaluation pass on one MI355X.

Workload: 1,048,576 points from an 8-cluster Gaussian mixture (sigma 0.05)
in the unit cube, forces N(0,1)^3, RPY radii U[0.002, 0.005]; order p = 10,
leaf_cap = 2000.  A step is one evaluation pass (stkfmm_run: pack, S2M,
upward sweep, M2L, S2L, downward sweep, L2T/M2T, P2P, combine) of the
Stokeslet with the tree already built and every input resident in HBM; the
tree build (t_tree) is timed separately, as the paper does.

Prints one JSON line (see the keys below).  Only one GPU is supported.
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
# kernel formulas without the hi/lo coordinate refinement
P2P_FLOPS = {"Stokeslet": 28, "RPY": 50}
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILE = os.path.join(ROOT, "profiles", "p2p_stokeslet_1M_clustered_p10.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2010_15155_amd", "csrc", f) for f in ("kernels.hip", "kernel_math.hpp")]


def measured_traffic():
    """HBM bytes per P2P launch from the committed PMC summary, or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(l.split(": ", 1) for l in open(PROFILE).read().splitlines() if ": " in l
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
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--leaf-cap", type=int, default=2000)
    ap.add_argument("--samples", type=int, default=4096, help="targets checked by the FP64 GPU direct sum")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the measurement, copy a MIB-sized device buffer once (reference "
                         "kernel for scaling hardware byte counters)")
    return ap.parse_args()


def timed_steps(fmm, torch, sl_val, steps, warmup):
    for _ in range(warmup):
        out = fmm.run(sl_val)
    torch.cuda.synchronize()
    p2p_ms, run_ms = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fmm.run(sl_val)
        tm = fmm.timings()
        p2p_ms.append(tm["stages_ms"]["p2p"])
        run_ms.append(tm["t_run_ms"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    return out, wall, float(np.mean(p2p_ms)), float(np.median(run_ms)), tm


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the evaluation pass is not sharded across GPUs "
              "in this build (see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2010_15155_amd import FMM, workloads as W

    d = W.clustered_rpy(args.n, 201)
    x = torch.from_numpy(d["xyz"]).cuda()
    f = torch.from_numpy(d["f"]).cuda()
    fb = torch.from_numpy(np.concatenate([d["f"], d["b"][:, None]], 1)).cuda()
    fmm = FMM()
    res = {}
    for kernel, val in (("Stokeslet", f), ("RPY", fb)):
        t0 = time.perf_counter()
        fmm.set_points(kernel, x, None, x, p=args.p, leaf_cap=args.leaf_cap)
        torch.cuda.synchronize()
        t_plan = (time.perf_counter() - t0) * 1e3
        t_tree = fmm.timings()["t_tree_ms"]
        out, wall, p2p_ms, run_ms, tm = timed_steps(fmm, torch, val, args.steps, args.warmup)
        st = fmm.stats()
        # one serial pass (P2P before the far field) for standalone stage times
        fmm.set_option("overlap", "0")
        fmm.run(val)
        serial = fmm.timings()
        fmm.set_option("overlap", "1")
        # accuracy on sampled targets against the FP64 GPU direct sum
        idx = W.sample_indices(args.n, args.samples, 7)
        ti = torch.from_numpy(idx).cuda()
        ref = fmm.direct(kernel, x, val, None, None, x[ti].contiguous())
        got = out[ti]
        kt = out.shape[1]
        fields = {"Stokeslet": [("u", 0, 3)], "RPY": [("u", 0, 3), ("lap_u", 3, 6)]}[kernel]
        errs = {n: float(torch.linalg.norm(got[:, a:b] - ref[:, a:b]) / torch.linalg.norm(ref[:, a:b]))
                for n, a, b in fields}
        res[kernel] = dict(ms_per_step=wall * 1e3, run_ms=run_ms, p2p_ms=p2p_ms, t_tree_ms=t_tree,
                           t_plan_ms=t_plan, stats=st, rel_l2=errs, stages_ms=tm["stages_ms"],
                           stages_serial_ms=serial["stages_ms"], run_serial_ms=serial["t_run_ms"],
                           p2p_pairs_per_s=st["p2p_pairs"] / (p2p_ms * 1e-3), kt=kt)
        fmm.set_option("precision", "fp32")
    S = res["Stokeslet"]
    n = args.n
    value = n / (S["ms_per_step"] * 1e-3)
    flops = P2P_FLOPS["Stokeslet"] * S["stats"]["p2p_pairs"]
    achieved = flops / (S["p2p_ms"] * 1e-3) / 1e12
    line = {
        "metric": "targets/sec (Stokeslet N=1M, rel L2 err <=1e-5) learned-p vs fixed p=10; P2P pairs/s",
        "value": value,
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": S["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Stokeslet evaluation pass, N=%d points (8-cluster Gaussian mixture, "
                               "sigma 0.05), sources = targets, open BC" % n,
                   "p": args.p, "leaf_cap": args.leaf_cap, "order_mode": "fixed"},
        "rel_l2": S["rel_l2"],
        "p2p_pairs_per_s": S["p2p_pairs_per_s"],
        "t_tree_ms": S["t_tree_ms"],
        "stages_ms": S["stages_ms"],
        "stages_serial_ms": S["stages_serial_ms"],
        "run_serial_ms": S["run_serial_ms"],
        "plan": S["stats"],
        "rpy": {"ms_per_step": res["RPY"]["ms_per_step"], "rel_l2": res["RPY"]["rel_l2"],
                "targets_per_s": n / (res["RPY"]["ms_per_step"] * 1e-3),
                "p2p_pairs_per_s": res["RPY"]["p2p_pairs_per_s"], "stages_ms": res["RPY"]["stages_ms"],
                "stages_serial_ms": res["RPY"]["stages_serial_ms"]},
        "roofline": {"kernel": "p2p_kernel<DStokeslet>", "bound": "alu", "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(),
                     "flops_per_pair": P2P_FLOPS["Stokeslet"], "pairs_per_launch": S["stats"]["p2p_pairs"],
                     "avg_launch_ms": S["p2p_ms"]},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(d, args.cpu_seconds)
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibrate_copy_bytes"] = args.calibrate_copy * (1 << 20)
    print(json.dumps(line), flush=True)


def cpu_baseline(d, budget_s):
    """The FP64 oracle direct sum on the host cores, on a bounded sample of
    targets (all sources), scaled to targets/s."""
    from oracle import direct
    x, f = d["xyz"], d["f"]
    n = len(x)
    # calibrate on a small sample, then size the timed sample to the budget
    t0 = time.perf_counter()
    direct.stokeslet(x, f, x[:64])
    per_target = (time.perf_counter() - t0) / 64
    k = int(max(64, min(n, budget_s / max(per_target, 1e-9))))
    from paper_2010_15155_amd import workloads as W
    idx = W.sample_indices(n, k, 11)
    t0 = time.perf_counter()
    direct.stokeslet(x, f, x[idx])
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": k / dt, "unit": "targets/s", "cores": cores, "kind": "oracle",
            "sample": "%d sampled targets x %d sources, FP64 direct Stokeslet sum (C, OpenMP)" % (k, n),
            "seconds": dt, "pairs_per_s": k * n / dt}


if __name__ == "__main__":
    main()
