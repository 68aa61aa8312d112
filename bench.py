"""Benchmark of the treecode hot path on one MI355X.

One step = one kick-drift-kick leapfrog step through the C ABI: tree build
(root cube, keys, radix sort, gather, topology), FP64 moments, opening radii,
the fused walk + force kernel, the kicks, and the FP64 diagnostics.  Each
step holds exactly one force evaluation, so force-evals/s = steps/s.

Default workload: 3D Plummer sphere, N = 1,048,576, a = 1, M = 1, G = 1,
eps = 1e-2, theta = 0.5, leaf_cap = 16, dt = 1e-3; FP32 state and forces.

Prints ONE JSON line on stdout.  Extra progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32, published
FLOPS_PER_INTERACTION = {3: 20, 2: 15}
METRIC = "force-evals/s & interactions/s at fixed rel. force error, learned vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, n: int | None):
    from paper_1211_2293_amd import workloads
    gen = workloads.BY_NAME[name]
    return gen() if n is None else gen(n)


def force_kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("force.hip", "tc_internal.h"):
        with open(os.path.join(ROOT, "paper_1211_2293_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(per_launch_interactions: int):
    """HBM bytes per launch of the force kernel from the committed counter
    summary, when it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "walk_force_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != force_kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w, sample_groups: int):
    """The FP64 oracle timed on this host: full tree build plus the walk and
    forces of a seeded sample of groups, scaled to one force evaluation."""
    import oracle
    n = w.n
    t0 = time.perf_counter()
    tree = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    t_build = time.perf_counter() - t0
    G = (n + 63) // 64
    rng = np.random.default_rng(1234)
    k = min(sample_groups, G)
    sel = np.sort(rng.choice(G, size=k, replace=False))
    t1 = time.perf_counter()
    tree.forces(w.theta, G=w.G, eps=w.eps, gs=64, groups=sel)
    t_force = time.perf_counter() - t1
    t_eval = t_build + t_force * (G / k)
    return {
        "value": 1.0 / t_eval,
        "unit": "force-evals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: full tree build of all {n} bodies ({t_build:.2f} s) + walk and "
                   f"forces of {k} of {G} seeded 64-body groups ({t_force:.2f} s), scaled to one "
                   f"force evaluation ({t_eval:.2f} s)"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer-3d")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-groups", type=int, default=256)
    ap.add_argument("--no-diag", action="store_true", help="leave the diagnostics out of the step")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): this build has no "
              "multi-GPU path; the sharding design is described in DESIGN.md.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1211_2293_amd import treecode

    w = make_workload(args.workload, args.n)
    theta = w.theta if args.theta is None else args.theta
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pos = torch.from_numpy(w.pos).to(dev)
    vel = torch.from_numpy(w.vel).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    tc = treecode.Treecode(w.dim, leaf_cap=w.leaf_cap)
    log(f"workload {w.name}: n={w.n} dim={w.dim} theta={theta} eps={w.eps} leaf_cap={w.leaf_cap}")

    # initial force evaluation (part of set-up, not timed)
    tc.build(pos, mass)
    tc.moments()
    tc.walk(theta)
    tc.forces(w.G, w.eps)
    torch.cuda.synchronize()

    def step():
        tc.leapfrog(w.dt, pos, vel)
        if not args.no_diag:
            tc.diag(vel)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if tc.status() != treecode.TC_OK:
        raise RuntimeError("device status not ok after warm-up")

    tc.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = tc.timing()
    tc.set_timing(False)
    if tc.status() != treecode.TC_OK:
        raise RuntimeError("device status not ok after the timed steps")

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    inter = tc.interactions()                       # of the last evaluation
    flops = FLOPS_PER_INTERACTION[w.dim] * inter
    kern_avg_ms = kern_ms / max(launches, 1)
    achieved_tflops = flops / (kern_avg_ms * 1e-3) / 1e12
    evals_per_s = 1e3 / ms_per_step
    log(f"{ms_per_step:.3f} ms/step, force kernel {kern_avg_ms:.3f} ms/launch ({launches} launches), "
        f"{inter / w.n:.0f} interactions/body, {achieved_tflops:.1f} TFLOP/s in the force kernel")

    result = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "force-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name} N={w.n} dim={w.dim} theta={theta} eps={w.eps} leaf_cap={w.leaf_cap} "
                        f"dt={w.dt} KDK leapfrog step (build+moments+walk+forces+kicks"
                        f"{'' if args.no_diag else '+diagnostics'})",
            "n": w.n, "dim": w.dim, "theta": theta, "eps": w.eps, "leaf_cap": w.leaf_cap,
            "group": 64,
        },
        "interactions_per_s": inter / (ms_per_step * 1e-3),
        "interactions_per_eval": inter,
        "force_kernel_interactions_per_s": inter / (kern_avg_ms * 1e-3),
        "roofline": {
            "bound": "alu",
            "kernel": "k_walk_force",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": traffic_from_profile(inter),
            "kernel_ms": kern_avg_ms,
            "flops_per_interaction": FLOPS_PER_INTERACTION[w.dim],
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_groups)
        log(result["cpu_baseline"]["sample"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
