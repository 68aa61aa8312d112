"""Benchmark of the treecode hot path on one MI355X.

One step = one kick-drift-kick leapfrog step through the C ABI: tree build
(root cube, keys, radix sort, gather, topology), FP64 moments, opening radii,
the fused walk + force kernel, the kicks, and the FP64 diagnostics.  Each
step holds exactly one force evaluation, so force-evals/s = steps/s.

Default workload: 3D Plummer sphere, N = 1,048,576, a = 1, M = 1, G = 1,
eps = 1e-2, theta = 0.5, leaf_cap = 16, dt = 1e-3; FP32 state and forces.

After the timed steps (outside the timed region):
  * the relative force error E = sqrt(sum |a - a_ref|^2 / sum |a_ref|^2) of
    a fresh evaluation against the FP64 direct sum (computed on the GPU by
    tc_direct) on 8,192 seeded sample bodies;
  * the plain walk with every accepted cell's quadrupole term added, over a
    theta sweep (the analytic control for the learned closure);
  * the same evaluations with per-body lists written to memory and summed
    by a separate kernel (tc_lists_count / tc_lists_forces), over a theta
    sweep;
  * for 3D workloads, the fast multipole method over a theta sweep on a
    tree of its own leaf size (64 by default; dual tree traversal, M2L, L2L,
    L2P and direct sums; each timed evaluation includes the tree build and
    the traversal), with the plain rate at the same E;
  * for 3D workloads, the learned-vs-plain study on the initial positions:
    plain evaluations over a theta sweep (time per evaluation and E), the
    closure network trained on residuals generated at theta = 0.9 for 4,096
    training and 1,024 validation targets, then learned evaluations at
    theta_L = 0.8 over theta_P = 0.5, and the plain evaluation rate at the
    learned E interpolated from the sweep;
  * the CPU oracle timed on whole force evaluations of the same workload.

Prints ONE JSON line on stdout.  Extra progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32, published
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E, published
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 matrix cores, published
MLP_FLOPS_PER_SAMPLE = 2 * (10 * 64 + 64 * 64 + 64 * 3)    # 9,856: the network's products
FLOPS_PER_INTERACTION = {3: 20, 2: 15}
METRIC = "force-evals/s & interactions/s at fixed rel. force error, learned vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, n: int | None):
    import workloads
    gen = workloads.BY_NAME[name]
    return gen() if n is None else gen(n)


def code_only(text: str) -> str:
    """A source's code without its comments and blank lines, so that a
    change of comments alone does not mark a counter profile stale."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def sources_hash(files, read=None) -> str:
    """Hash of the code of the given csrc files (read(f) supplies another
    version of a file's text)."""
    h = hashlib.sha256()
    for f in files:
        if read is None:
            with open(os.path.join(ROOT, "paper_1211_2293_amd", "csrc", f), encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


FORCE_SOURCES = ("force.hip", "walk_common.h", "tc_internal.h")
BUILD_SOURCES = ("build.hip", "tc_internal.h")


def force_kernel_source_hash() -> str:
    return sources_hash(FORCE_SOURCES)


def traffic_from_profile(w, theta: float):
    """HBM bytes per launch of the force kernel from the committed counter
    summary, when it was taken on the current kernel source and on this
    workload; else None."""
    p = os.path.join(ROOT, "profiles", "walk_force_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != force_kernel_source_hash():
        return None
    if d.get("workload") != f"{w.name} N={w.n} theta={theta} eps={w.eps} leaf_cap={w.leaf_cap}":
        return None
    return d.get("bytes_per_launch")


def build_source_hash() -> str:
    return sources_hash(BUILD_SOURCES)


def build_traffic_from_profile(w, theta: float):
    """Calibrated HBM bytes per stage of one step from the committed counter
    summary, when taken on the current build source and on this workload;
    else None."""
    p = os.path.join(ROOT, "profiles", "build_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f).get(f"{w.name} N={w.n} theta={theta} eps={w.eps} leaf_cap={w.leaf_cap}")
    if not d or d.get("source_hash") != build_source_hash():
        return None
    return d


def cpu_model() -> str | None:
    """The host CPU's model name from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, theta: float, min_seconds: float, sample=None):
    """The FP64 oracle timed on this host: whole force evaluations of the
    same workload (tree build, walk groups, walk and forces of every body),
    repeated until min_seconds have passed, with the split between the build
    (tree and moments) and the walk + force summation; the FP64 direct sum
    on the error sample is timed once."""
    import oracle
    n = w.n
    times, t_builds, t_walks = [], [], []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        tree = oracle.Tree(w.pos, w.mass, w.leaf_cap)
        t1 = time.perf_counter()
        tree.walk_forces(theta, G=w.G, eps=w.eps)
        t2 = time.perf_counter()
        times.append(t2 - t0)
        t_builds.append(t1 - t0)
        t_walks.append(t2 - t1)
        del tree
        if time.perf_counter() - t_start >= min_seconds or len(times) >= 50:
            break
    t_eval = float(np.median(times))
    t_build, t_walk = float(np.median(t_builds)), float(np.median(t_walks))
    direct = None
    if sample is not None:
        t0 = time.perf_counter()
        oracle.direct(w.pos, w.mass, G=w.G, eps=w.eps, targets=sample)
        td = time.perf_counter() - t0
        direct = {"seconds": td, "pair_terms": int(len(sample)) * n,
                  "pair_terms_per_s": len(sample) * n / td,
                  "sample": f"{len(sample)} seeded bodies (seed 104) against all {n}"}
    cores = oracle.num_threads()
    # one core: the tree build plus a seeded sample of 1/32 of the walk groups,
    # scaled to the whole evaluation
    tree = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    gb, gc = tree.groups(64, 1024)
    sel = np.sort(np.random.default_rng(1234).choice(len(gb), size=max(1, len(gb) // 32), replace=False))
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        t1_tree = oracle.Tree(w.pos, w.mass, w.leaf_cap)
        t_b = time.perf_counter() - t0
        t0 = time.perf_counter()
        t1_tree.forces_groups(theta, gb[sel], gc[sel], G=w.G, eps=w.eps)
        t_f = (time.perf_counter() - t0) * len(gb) / len(sel)
    finally:
        oracle.set_num_threads(cores)
    return {
        "value": 1.0 / t_eval,
        "unit": "force-evals/s",
        "cores": cores,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"FP64 oracle, {len(times)} whole force evaluation(s) of all {n} bodies (build + walk + "
                   f"forces, theta={theta}, OpenMP over walk groups), median {t_eval:.2f} s each"),
        "stages": {"build_and_moments_s": t_build, "walk_and_forces_s": t_walk,
                   "force_share": t_walk / (t_build + t_walk),
                   "note": "share of the walk + force summation in the oracle's evaluation; the paper puts "
                           "the force step at upwards of 90% of the cycles (§1, §3.2)"},
        "direct_sum": direct,
        "single_core": {"value": 1.0 / (t_b + t_f), "unit": "force-evals/s", "cores": 1,
                        "sample": f"build of all bodies ({t_b:.2f} s) + walk and forces of {len(sel)} of "
                                  f"{len(gb)} seeded walk groups, scaled ({t_f:.2f} s)"},
    }


def _clock_mhz():
    """Peak shader clock reported by the HIP runtime (MHz), or None."""
    try:
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        # hipDeviceAttributeClockRate: kHz
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0 and v.value > 0:
            return v.value / 1000.0
    except OSError:
        pass
    return None


BUILD_STAGES = ("bbox", "keys", "sort", "gather", "topology", "levels", "groups", "moments", "radii")


def build_bytes(n, dim, f64, ncells, ngroups):
    """Algorithmic HBM bytes of each stage of the build (what the stage has
    to read and write at least) for n bodies of the given input dtype,
    ncells cells and ngroups walk groups."""
    e = 8 if f64 else 4                              # input element size
    pos = dim * e
    passes = (dim * (21 if dim == 3 else 31) + 7) // 8   # 8-bit digits of the keys
    return {
        "bbox": n * (pos + e),                          # positions and masses read
        "keys": n * (pos + 12),                         # positions read; key and index written
        "sort": passes * n * 24,                        # each pass: key + index read and written
        "gather": n * (4 + pos + e + 32 + (0 if f64 else 16)),   # index, position, mass in; FP64 body (+ FP32 copy) out
        "topology": n * 8 + ncells * 32,                # sorted keys read, cells written
        "levels": ncells * 12,                          # levels read, level-order maps written
        "groups": ncells * 12 + ngroups * 8,            # counts and flags read, groups written
        "moments": n * 32 + ncells * (112 + 48 + 112),  # bodies read; moments and walk records written, children read
        "radii": ncells * 72,                           # cell and centre of mass read, squared radius written
    }


def stage_breakdown(tc, step, steps, n, dim, f64, traffic=None):
    """Per-stage device time of `steps` further steps (HIP events around every
    stage on the context's stream; outside the timed region), and the build
    stages' achieved bandwidth against their algorithmic bytes."""
    tc.set_stage_timing(True)
    for _ in range(steps):
        step()
    st = tc.stage_timing()
    tc.set_stage_timing(False)
    ncells, ngroups = tc.num_cells(), tc.num_groups()
    per = {k: {"ms_per_step": v[0] / steps, "per_step": v[1] / steps} for k, v in st.items()}
    total = sum(v["ms_per_step"] for v in per.values())
    for v in per.values():
        v["share"] = v["ms_per_step"] / total if total > 0 else None
    nbytes = build_bytes(n, dim, f64, ncells, ngroups)
    rows, b_sum, t_sum, hbm_sum = {}, 0, 0.0, 0.0
    for k in BUILD_STAGES:
        ms = per[k]["ms_per_step"]
        gbs = nbytes[k] / (ms * 1e-3) / 1e9 if ms > 0 else None
        rows[k] = {"algorithmic_bytes": nbytes[k], "ms": ms, "GB/s": gbs,
                   "frac": None if gbs is None else gbs / PEAK_HBM_GBS}
        if traffic is not None and k in traffic["stages"]:
            tb = traffic["stages"][k]["bytes"]
            rows[k]["traffic"] = tb
            rows[k]["traffic_GB/s"] = tb / (ms * 1e-3) / 1e9 if ms > 0 else None
            hbm_sum += tb
        b_sum += nbytes[k]
        t_sum += ms
    build = {"bound": "hbm", "achieved": b_sum / (t_sum * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": b_sum / (t_sum * 1e-3) / 1e9 / PEAK_HBM_GBS,
             "traffic": hbm_sum if traffic is not None else None,
             "traffic_summary": traffic.get("summary") if traffic is not None else None,
             "algorithmic_bytes": b_sum, "ms": t_sum, "cells": ncells, "groups": ngroups, "stages": rows}
    return {"steps": steps, "total_ms_per_step": total, "stages": per}, build


def rel_error(acc, ref):
    """E = sqrt(sum |a - a_ref|^2 / sum |a_ref|^2) with the median and 99th
    percentile of the per-body |a - a_ref| / |a_ref|."""
    acc = np.asarray(acc, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(acc - ref, axis=1)
    r = np.linalg.norm(ref, axis=1)
    per = d / np.where(r > 0, r, 1.0)
    return {"E": float(np.sqrt((d * d).sum() / (r * r).sum())), "median": float(np.median(per)),
            "p99": float(np.percentile(per, 99))}


def time_evals(fn, reps=5, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)) * 1e3


def interp_ms_at_error(sweep, E):
    """Plain ms/eval at error E, piecewise linear in (log E, log ms) over
    the theta sweep; None outside the swept range."""
    pts = sorted((r["E"], r["ms_per_eval"]) for r in sweep)
    for (e0, m0), (e1, m1) in zip(pts, pts[1:]):
        if e0 <= E <= e1 and e1 > e0:
            f = (np.log(E) - np.log(e0)) / (np.log(e1) - np.log(e0))
            return float(np.exp(np.log(m0) + f * (np.log(m1) - np.log(m0))))
    return None


def train_closure(tc, w, args, pos, mass):
    """Residual pairs of the method itself at theta = 0.9 for the seeded
    training and validation targets (tc_residuals), then training on the
    GPU (tc_mlp_step); returns the training statistics with the validation
    MSE of the analytic quadrupole term beside the network's."""
    import torch

    import workloads
    from paper_1211_2293_amd import closure
    tc.build(pos, mass)
    tc.moments()
    t0 = time.perf_counter()
    tr = workloads.sample_indices(w.n, args.train_targets, seed=203)
    va = workloads.sample_indices(w.n, args.val_targets, seed=204)
    f_tr, y_tr = closure.residual_pairs(tc, 0.9, w.eps, tr)
    f_va, y_va = closure.residual_pairs(tc, 0.9, w.eps, va)
    torch.cuda.synchronize()
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    p0, order = workloads.training_draws(f_tr.shape[0], args.epochs, 4096)
    stats = closure.train(tc, f_tr, y_tr, p0, order, epochs=args.epochs, batch=4096, lr=args.lr,
                          lr_final=args.lr_final, val=(f_va, y_va), log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    stats["val_mse_quadrupole"] = float(((closure.quadrupole_prediction(f_va) - y_va) ** 2).mean())
    stats.update({"residual_seconds": t_res, "train_seconds": t_train, "theta": 0.9,
                  "targets": [len(tr), len(va)], "lr": [args.lr, args.lr_final]})
    log(f"  closure: {stats['pairs']} pairs in {t_res:.2f} s; {stats['steps']} steps in {t_train:.2f} s; "
        f"validation MSE {stats['val_mse']:.3e} vs {stats['val_mse_quadrupole']:.3e} for the analytic "
        f"quadrupole term and {stats['val_mse_zero']:.3e} predicting zero")
    return stats


def learned_study(w, args):
    """Plain theta sweep vs the learned closure at matched error, on the
    workload's initial positions; every timed evaluation includes the tree
    build.  Errors are against the FP64 direct sum on the seeded sample."""
    import torch

    import workloads
    from paper_1211_2293_amd import closure, treecode
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(w.pos).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    tc = treecode.Treecode(w.dim, leaf_cap=w.leaf_cap)
    tc.build(pos, mass)
    tc.moments()
    sample = workloads.sample_indices(w.n, args.sample, seed=104)
    ref, _ = tc.direct(torch.from_numpy(sample.astype(np.int32)).to(dev), G=w.G, eps=w.eps)
    ref = ref.cpu().numpy()[:, :w.dim]

    def plain(theta):
        tc.build(pos, mass)
        tc.moments()
        tc.walk(theta)
        return tc.forces(w.G, w.eps, want_pot=False)[0]

    sweep = []
    for th in args.sweep:
        ms = time_evals(lambda: plain(th))
        acc = plain(th).cpu().numpy()[sample]
        e = rel_error(acc, ref)
        inter = tc.interactions()
        sweep.append({"theta": th, "ms_per_eval": ms, "evals_per_s": 1e3 / ms, "E": e["E"],
                      "p99": e["p99"], "interactions_per_body": inter / w.n})
        log(f"  plain theta={th}: {ms:.3f} ms/eval, E={e['E']:.3e}, {inter / w.n:.0f} interactions/body")
    out = {"sample": f"{len(sample)} seeded bodies (seed 104), FP64 direct sum on the GPU", "plain": sweep}

    # quadrupole terms on every accepted cell (the analytic control for the closure)
    if w.dim == 3:
        quad = []
        tc.set_multipole(2)
        for th in args.quad_sweep:
            ms = time_evals(lambda: plain(th))
            acc = plain(th).cpu().numpy()[sample]
            e = rel_error(acc, ref)
            pm = interp_ms_at_error(sweep, e["E"])
            quad.append({"theta": th, "ms_per_eval": ms, "evals_per_s": 1e3 / ms, "E": e["E"], "p99": e["p99"],
                         "interactions_per_body": tc.interactions() / w.n,
                         "plain_evals_per_s_at_same_E": None if pm is None else 1e3 / pm,
                         "speedup_vs_plain_at_same_E": None if pm is None else pm / ms})
            log(f"  quadrupole theta={th}: {ms:.3f} ms/eval, E={e['E']:.3e}, speedup at same E "
                f"{quad[-1]['speedup_vs_plain_at_same_E']}")
        tc.set_multipole(1)
        out["quadrupole"] = quad

    # per-body lists written to HBM and summed (the treecode as the paper states it)
    per_body = []
    buf = None
    for th in args.per_body_sweep:
        tc.build(pos, mass)
        tc.moments()
        tc.walk(th)
        total, _ = tc.lists_count()
        if 4 * total > args.list_gb_max * 1e9:
            log(f"  per-body theta={th}: lists of {4 * total / 1e9:.1f} GB exceed --list-gb-max, skipped")
            per_body.append({"theta": th, "skipped": f"lists of {4 * total / 1e9:.1f} GB"})
            continue
        if buf is None or buf.numel() < total:
            buf = None
            torch.cuda.empty_cache()
            buf = torch.empty(int(total * 1.05) + 1, dtype=torch.int32, device=dev)

        def run_pb():
            tc.build(pos, mass)
            tc.moments()
            tc.walk(th)
            tc.lists_count()
            return tc.lists_forces(w.G, w.eps, lists=buf, want_pot=False)[0]

        ms = time_evals(run_pb)
        acc = run_pb().cpu().numpy()[sample]
        e = rel_error(acc, ref)
        per_body.append({"theta": th, "ms_per_eval": ms, "evals_per_s": 1e3 / ms, "E": e["E"],
                         "entries_per_body": total / w.n, "list_bytes": 4 * total,
                         "grouped_evals_per_s_at_same_E": (None if interp_ms_at_error(sweep, e["E"]) is None
                                                           else 1e3 / interp_ms_at_error(sweep, e["E"]))})
        log(f"  per-body theta={th}: {ms:.3f} ms/eval, E={e['E']:.3e}, {total / w.n:.0f} entries/body, "
            f"lists {4 * total / 1e9:.2f} GB")
    del buf
    torch.cuda.empty_cache()
    out["per_body"] = per_body
    if w.dim != 3:
        return out

    # the fast multipole method (cell-cell expansions), on a tree of its own
    # leaf size
    fmm = []
    tf = treecode.Treecode(w.dim, leaf_cap=args.fmm_leaf_cap) if args.fmm_sweep else None
    for th in args.fmm_sweep:
        def run_fmm():
            tf.build(pos, mass)
            tf.moments()
            tf.fmm_plan(th)
            return tf.fmm_forces(w.G, w.eps, want_pot=False)[0]

        def run_plan():
            tf.build(pos, mass)
            tf.moments()
            return tf.fmm_plan(th)

        ms = time_evals(run_fmm)
        ms_plan = time_evals(run_plan)
        sizes = run_plan()
        acc = tf.fmm_forces(w.G, w.eps, want_pot=False)[0].cpu().numpy()[sample]
        e = rel_error(acc, ref)
        pm = interp_ms_at_error(sweep, e["E"])
        fmm.append({"theta": th, "leaf_cap": args.fmm_leaf_cap, "ms_per_eval": ms, "evals_per_s": 1e3 / ms,
                    "ms_build_and_traversal": ms_plan,
                    "E": e["E"], "p99": e["p99"], "m2l_pairs": sizes[1], "p2p_leaf_pairs": sizes[2],
                    "plain_evals_per_s_at_same_E": None if pm is None else 1e3 / pm,
                    "speedup_vs_plain_at_same_E": None if pm is None else pm / ms})
        log(f"  fmm theta={th}: {ms:.3f} ms/eval ({ms_plan:.3f} build + traversal), E={e['E']:.3e}, "
            f"{sizes[1]} M2L / {sizes[2]} P2P pairs, speedup at same E {fmm[-1]['speedup_vs_plain_at_same_E']}")
    out["fmm"] = fmm
    del tf
    torch.cuda.empty_cache()

    stats = train_closure(tc, w, args, pos, mass)

    learned = []
    for th_l, th_p, tau in args.learned:
        def run():
            tc.build(pos, mass)
            tc.moments()
            return tc.forces_learned(th_l, th_p, tau, G=w.G, eps=w.eps, want_pot=False)[0]
        ms = time_evals(run)
        acc = run().cpu().numpy()[sample]
        e = rel_error(acc, ref)
        kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
        _, gcnt = tc.groups()
        samples = int(((kept + fell) * gcnt.cpu().numpy().astype(np.int64)).sum())
        inter = tc.interactions()
        plain_ms = interp_ms_at_error(sweep, e["E"])
        at_l = [r["ms_per_eval"] for r in sweep if abs(r["theta"] - th_l) < 1e-9]
        # a learned evaluation costs at least the plain walk at theta_l (a free
        # network), and its network at least its BF16 products at the matrix
        # cores' peak on top
        floor_mfma_ms = samples * MLP_FLOPS_PER_SAMPLE / (PEAK_BF16_TFLOPS * 1e12) * 1e3
        row = {"theta_l": th_l, "theta_p": th_p, "tau": tau if np.isfinite(tau) else "inf",
               "ms_per_eval": ms, "evals_per_s": 1e3 / ms, "E": e["E"], "p99": e["p99"],
               "interactions_per_body": inter / w.n, "learned_cells": int(kept.sum()),
               "fallback_cells": int(fell.sum()), "network_samples": samples,
               "plain_evals_per_s_at_same_E": None if plain_ms is None else 1e3 / plain_ms,
               "speedup_vs_plain_at_same_E": None if plain_ms is None else plain_ms / ms,
               "plain_ms_at_theta_l": at_l[0] if at_l else None,
               "network_mfma_floor_ms": floor_mfma_ms}
        if plain_ms and at_l and fell.sum() == 0:
            # with every learned cell kept the walk is the plain walk at theta_l
            row["ceiling_speedup_free_network"] = plain_ms / at_l[0]
            row["ceiling_speedup_at_mfma_peak"] = plain_ms / (at_l[0] + floor_mfma_ms)
        learned.append(row)
        log(f"  learned theta_l={th_l} theta_p={th_p} tau={tau}: {ms:.3f} ms/eval, E={e['E']:.3e}, "
            f"kept {row['learned_cells']} fell back {row['fallback_cells']}, speedup at same E "
            f"{row['speedup_vs_plain_at_same_E']}")
    out["closure_training"] = stats
    out["learned"] = learned
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="plummer-3d")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="least wall time of whole oracle evaluations for the CPU baseline")
    ap.add_argument("--no-study", action="store_true", help="skip the error and learned-vs-plain study")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run 3 plain device copies of MIB MiB (a known-size reference for "
                         "hardware byte counters)")
    ap.add_argument("--sample", type=int, default=8192)
    ap.add_argument("--sweep", type=float, nargs="*", default=[0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9])
    ap.add_argument("--per-body-sweep", type=float, nargs="*", default=[0.3, 0.4, 0.5, 0.6, 0.7])
    ap.add_argument("--list-gb-max", type=float, default=64.0, help="largest per-body list buffer to allocate")
    ap.add_argument("--quad-sweep", type=float, nargs="*", default=[0.5, 0.6, 0.7, 0.8, 0.9, 1.0])
    ap.add_argument("--fmm-sweep", type=float, nargs="*", default=[0.4, 0.5, 0.6, 0.7, 0.8, 0.9])
    ap.add_argument("--fmm-leaf-cap", type=int, default=64, help="leaf size of the FMM's own tree")
    ap.add_argument("--train-targets", type=int, default=4096)
    ap.add_argument("--val-targets", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--lr-final", type=float, default=1e-5)
    ap.add_argument("--learned", type=lambda v: tuple(float(x) for x in v.split(",")), nargs="*",
                    default=[(0.8, 0.5, float("inf")), (0.8, 0.5, 1e-3), (0.8, 0.5, 1e-2), (0.8, 0.5, 3e-2),
                             (0.7, 0.5, float("inf")), (0.7, 0.5, 1e-2)],
                    help="theta_l,theta_p,tau triples")
    ap.add_argument("--no-diag", action="store_true", help="leave the diagnostics out of the step")
    ap.add_argument("--sync-diag", action="store_true",
                    help="copy each step's diagnostics to the host and wait (default: into a device record, "
                         "read after the timed steps)")
    ap.add_argument("--no-split", action="store_true", help="one wave per walk group at every n")
    ap.add_argument("--graph", action="store_true",
                    help="replay the pre-force part of each step as a HIP graph")
    ap.add_argument("--stage-steps", type=int, default=10,
                    help="further steps with HIP events around every stage (after the timed steps)")
    ap.add_argument("--closure", type=lambda v: tuple(float(x) for x in v.split(",")), default=None,
                    metavar="THETA_L,THETA_P,TAU",
                    help="every step uses the learned walk (trained first on the workload's own residuals)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs on a single GPU "
              "and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_1211_2293_amd import treecode

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst

    w = make_workload(args.workload, args.n)
    theta = w.theta if args.theta is None else args.theta
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # a created stream (default priority): graph replay can record on it
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        return run(args, w, theta, dev, treecode, workloads, torch)


def run(args, w, theta, dev, treecode, workloads, torch):
    pos = torch.from_numpy(w.pos).to(dev)
    vel = torch.from_numpy(w.vel).to(dev)
    mass = torch.from_numpy(w.mass).to(dev)
    tc = treecode.Treecode(w.dim, leaf_cap=w.leaf_cap)
    tc.set_graph(args.graph)
    tc.set_split(not args.no_split)
    log(f"workload {w.name}: n={w.n} dim={w.dim} theta={theta} eps={w.eps} leaf_cap={w.leaf_cap}")

    # initial force evaluation (part of set-up, not timed)
    tc.build(pos, mass)
    tc.moments()
    tc.walk(theta)
    tc.forces(w.G, w.eps)
    closure_info = None
    if args.closure is not None:
        # the learned walk in every step: train on the workload's own residuals first
        closure_info = train_closure(tc, w, args, pos, mass)
        tl, tp, tau = args.closure
        tc.set_closure(tl, tp, tau)
        tc.build(pos, mass)
        tc.moments()
        tc.forces_learned(tl, tp, tau, G=w.G, eps=w.eps, want_pot=False)
    torch.cuda.synchronize()

    diags = []
    # one row of 8 FP64 diagnostics per step, written on the device
    record = torch.empty((args.warmup + args.steps + args.stage_steps, 8), dtype=torch.float64, device="cuda:0")

    def step():
        tc.leapfrog(w.dt, pos, vel)
        if args.no_diag:
            return
        if args.sync_diag:
            diags.append(tc.diag(vel))
        else:
            tc.diag_async(vel, record[len(diags)])
            diags.append(None)

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
    try:                                            # cells whose opening test ran in the walk
        tested = int(tc.tests().sum().item())
    except treecode.TcError:                        # learned or split walks keep no count
        tested = None
    if tested is not None:
        log(f"walk: {tested} cells tested per evaluation, {tested / (kern_avg_ms * 1e-3):.3e} per second of the "
            f"force kernel")
    learned_stats = None
    if args.closure is not None:
        kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
        _, gcnt = tc.groups()
        gcnt = gcnt.cpu().numpy().astype(np.int64)
        samples = int(((kept + fell) * gcnt).sum())
        mfma_tflops = samples * MLP_FLOPS_PER_SAMPLE / (kern_avg_ms * 1e-3) / 1e12
        learned_stats = {"learned_cells": int(kept.sum()), "fallback_cells": int(fell.sum()),
                         "fallback_fraction": float(fell.sum() / max(kept.sum() + fell.sum(), 1)),
                         "network_samples": samples, "network_tflops": mfma_tflops,
                         "network_frac_of_bf16_peak": mfma_tflops / PEAK_BF16_TFLOPS}
        log(f"learned walk: {learned_stats}")

    if args.stage_steps > 0:
        stages, build_roof = stage_breakdown(tc, step, args.stage_steps, w.n, w.dim, w.pos.dtype == np.float64,
                                             traffic=build_traffic_from_profile(w, theta))
        log("stages (ms/step): " + ", ".join(f"{k} {v['ms_per_step']:.3f}" for k, v in stages["stages"].items()))
        log(f"build: {build_roof['achieved']:.0f} GB/s of algorithmic bytes ({build_roof['frac']:.3f} of HBM)")
    else:
        stages = build_roof = None

    if diags and diags[0] is None:
        diags = list(record[:len(diags)].cpu().numpy())
    drift = None
    if len(diags) >= 2:
        d0, d1 = diags[0], diags[-1]
        e0, e1 = d0[0] + d0[1], d1[0] + d1[1]
        drift = {"steps": len(diags) - 1, "energy_rel": float((e1 - e0) / abs(e0)),
                 "momentum": float(np.linalg.norm(d1[2:2 + w.dim] - d0[2:2 + w.dim])),
                 "note": "FP64 diagnostics of the warm-up and timed steps: total energy E_kin + E_pot and "
                         "momentum sum(m v), first to last step"}
    props = torch.cuda.get_device_properties(dev)
    gpu = {"name": props.name, "arch": getattr(props, "gcnArchName", None),
           "compute_units": props.multi_processor_count, "memory_gb": props.total_memory / 2 ** 30,
           "hip": torch.version.hip, "clock_mhz": _clock_mhz()}
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
        "diagnostics_drift": drift,
        "gpu": gpu,
        "stages": stages,
        "roofline": {
            "bound": "alu",
            "kernel": "k_walk_force",
            "achieved": achieved_tflops,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP32_TFLOPS,
            "traffic": traffic_from_profile(w, theta),
            "kernel_ms": kern_avg_ms,
            "flops_per_interaction": FLOPS_PER_INTERACTION[w.dim],
            "walk": None if tested is None else {
                "cells_tested": tested,
                "cells_tested_per_s": tested / (kern_avg_ms * 1e-3),
                "note": "cells whose opening test ran (the root and every child of an opened cell) in one "
                        "force evaluation, over all groups, and their rate over the force kernel's time; the "
                        "walk shares the kernel with the force loop"},
            "build": build_roof,
        },
    }
    if args.closure is not None:
        tl, tp, tau = args.closure
        result["config"]["workload"] = (f"{w.name} N={w.n} dim={w.dim} learned walk theta_L={tl} theta_P={tp} "
                                        f"tau={tau} eps={w.eps} leaf_cap={w.leaf_cap} dt={w.dt} KDK leapfrog step "
                                        f"(build+moments+radii+learned walk and forces+kicks"
                                        f"{'' if args.no_diag else '+diagnostics'})")
        result["config"]["closure"] = {"theta_l": tl, "theta_p": tp, "tau": tau if np.isfinite(tau) else "inf"}
        result["closure_training"] = closure_info
        result["learned"] = learned_stats
        result["roofline"].update({"kernel": "k_walk_force_learned", "bound": "alu",
                                   "note": "interactions of the walk's monopole and body entries; the network's "
                                           "BF16 products are in learned.network_tflops"})
    sample = workloads.sample_indices(w.n, args.sample, seed=104)
    if not args.no_study or args.closure is not None:
        # error of a fresh evaluation at the final positions
        st = torch.from_numpy(sample.astype(np.int32)).to(dev)
        tc.build(pos, mass)
        tc.moments()
        if args.closure is not None:
            acc, _ = tc.forces_learned(*args.closure, G=w.G, eps=w.eps, want_pot=False)
        else:
            tc.walk(theta)
            acc, _ = tc.forces(w.G, w.eps, want_pot=False)
        ref, _ = tc.direct(st, G=w.G, eps=w.eps)
        result["rel_force_error"] = dict(rel_error(acc.cpu().numpy()[sample], ref.cpu().numpy()[:, :w.dim]),
                                         sample=f"{len(sample)} seeded bodies vs the FP64 direct sum")
        log(f"relative force error E = {result['rel_force_error']['E']:.3e}")
    if not args.no_study:
        log("learned-vs-plain study ...")
        result["study"] = learned_study(w, args)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on whole force evaluations ...")
        result["cpu_baseline"] = cpu_baseline(w, theta, args.cpu_seconds, sample=sample)
        log(result["cpu_baseline"]["sample"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
