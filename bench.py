#!/usr/bin/env python3
"""Throughput of the batched one-centre WP-CCC propagation on one MI355X.

Workload: proton + hydrogen, single-centre expansion with bound n <= 6 plus 20
Coulomb wave-packet bins per l (l <= 4, all m; N = 580 states, 120 radial
functions), 4000-point r-grid to 100 a.u.; 32 impact parameters log-spaced
0.05..20 a.u., v = 1 a.u., z from -40 to 40 with dz = 0.1 (800 RK4 steps per
path).  All 32 paths advance together.

A "step" is one RK4 step of Algorithm 1 for every path of the batch
(couplings at z_mid and z_new, four stages, the amplitude update).  The
metric is trajectory-steps/s = paths x steps / wall time.

Printed: one JSON line with the metric, a roofline entry for the dominant
kernel (device time from HIP events recorded by the library on its stream),
the oracle timed on this host's cores on a bounded sample, and the
probability error of the GPU path against that oracle sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "RK4 steps/s over batched b (plain FP64 vs mixed) at stated prob. error"
P_FLOOR = 1e-6
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def stage_work(n_l, l_max):
    """Algorithmic flops of one k_stage pass for one path (block-factored Eq. D1
    matvec): V^lam_{l' m', l}[n] = sum_m c P x (complex x real), then
    y[l' m' n'] = sum_{l, lam, n} F V (real x complex): 4 flops per term."""
    fl = 0
    for lp in range(l_max + 1):
        nV = 0
        vterms = 0
        for l in range(l_max + 1):
            for lam in range(abs(l - lp), l + lp + 1, 2):
                nV += n_l[l]
                for mp in range(-lp, lp + 1):
                    nm = sum(1 for m in range(-l, l + 1) if abs(mp - m) <= lam)
                    vterms += n_l[l] * nm
        fl += (2 * lp + 1) * n_l[lp] * nV * 4 + vterms * 4
    return fl


def n_triples(n_l, l_max):
    t = 0
    for la in range(l_max + 1):
        for lb in range(la, l_max + 1):
            for lam in range(lb - la, la + lb + 1, 2):
                t += n_l[la] * n_l[lb]
    return t


def run_propagation(W, plan, X, zgrid, K):
    """Advance every path by K RK4 steps along the grid (wrapping to the start)."""
    done = 0
    n = zgrid.size - 1
    while done < K:
        k = min(K - done, n)
        W.wpccc_propagate(plan, zgrid[: k + 1], X)
        done += k


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=800, help="timed RK4 steps (each over all paths)")
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(paths shard across GPUs without communication; see DESIGN.md). "
              f"--gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2403_04252_amd as W
    from paper_2403_04252_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WL.single_centre_batched()
    rec = w.basis
    lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
    n_states, n_radial, n_r = W.wpccc_basis_info(lb)
    n_l = [rec.n_max - l + rec.n_bins for l in range(rec.l_max + 1)]
    plan = W.wpccc_plan_create(lb, w.b, w.v)
    n_traj = plan.n_traj
    X = torch.zeros((n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X[:, 0] = 1.0

    # warmup
    run_propagation(W, plan, X, w.zgrid, args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps of the whole batch
    X.zero_()
    X[:, 0] = 1.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_propagation(W, plan, X, w.zgrid, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    W.wpccc_plan_status(plan)
    wall = t1 - t0
    value = n_traj * args.steps / wall

    # the same K steps again with per-kernel HIP events on the library's stream
    X.zero_()
    X[:, 0] = 1.0
    W.wpccc_plan_timing(plan, True)
    run_propagation(W, plan, X, w.zgrid, args.steps)
    st_ms, st_n = W.wpccc_plan_kernel_time(plan, "k_stage")
    su_ms, su_n = W.wpccc_plan_kernel_time(plan, "k_prologue")
    W.wpccc_plan_timing(plan, False)
    torch.cuda.synchronize()

    stage_flops = stage_work(n_l, rec.l_max) * n_traj
    stage_avg_s = st_ms / max(st_n, 1) * 1e-3
    trip = n_triples(n_l, rec.l_max)
    setup_avg_s = su_ms / max(su_n, 1) * 1e-3
    dominant = "k_stage"
    if dominant == "k_stage":
        achieved = stage_flops / stage_avg_s / 1e12
        roof = {"kernel": "k_stage", "bound": "alu", "achieved": achieved,
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                "avg_launch_us": stage_avg_s * 1e6, "launches": st_n,
                "algorithmic_flops_per_launch": stage_flops}
    kernel_times = {"k_stage": {"total_ms": st_ms, "launches": st_n},
                    "k_prologue": {"total_ms": su_ms, "launches": su_n}}

    # plain FP64 form: the same paths one after another
    seq_steps = min(args.steps, 100)
    plan_seq = W.wpccc_plan_create(lb, w.b, w.v, batched=False)
    X.zero_()
    X[:, 0] = 1.0
    run_propagation(W, plan_seq, X, w.zgrid, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_propagation(W, plan_seq, X, w.zgrid, seq_steps)
    torch.cuda.synchronize()
    seq_value = n_traj * seq_steps / (time.perf_counter() - t0)
    del plan_seq

    cpu = None
    prob_err = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info
        from oracle.propagate import probabilities, propagate_one_centre
        from oracle.radial import BasisSpec as OSpec, build_basis
        ob = build_basis(OSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
        from oracle.direct import direct_matrix
        t0 = time.perf_counter()
        direct_matrix(ob, w.b[0], w.zgrid[0], w.v[0])
        per_eval = time.perf_counter() - t0
        S = max(2, min(400, int(args.cpu_seconds / (2.0 * per_eval))))
        zs = w.zgrid[: S + 1]
        t0 = time.perf_counter()
        Xo = propagate_one_centre(ob, w.b[0], w.v[0], zs)
        dt = time.perf_counter() - t0
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        cpu = {"value": S / dt, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"path b={w.b[0]:.4g} of the workload, first {S} of its 800 RK4 steps "
                         f"(numpy FP64, {threads} BLAS threads), basis setup excluded"}
        # probability error of the GPU path on the same sample
        plan1 = W.wpccc_plan_create(lb, w.b[:1], w.v[:1])
        X1 = torch.zeros((1, plan1.n_pad), dtype=torch.complex128, device="cuda")
        X1[:, 0] = 1.0
        W.wpccc_propagate(plan1, zs, X1)
        torch.cuda.synchronize()
        Pg = (X1.abs() ** 2).cpu().numpy()[0, :n_states]
        Po = probabilities(Xo)
        dP = np.abs(Pg - Po)
        prob_err = {"max_abs": float(dP.max()),
                    "max_rel_floored": float((dP / np.maximum(Po, P_FLOOR)).max()),
                    "floor": P_FLOOR, "sample": cpu["sample"]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "p+H single-centre N=580 (n<=6 + 20 bins/l, l<=4), 4000-pt grid, "
                               "32 b log-spaced 0.05-20, v=1, z -40..40 dz=0.1",
                   "form": "batched FP64", "n_paths": n_traj, "n_states": n_states,
                   "n_radial": n_radial, "n_r": n_r, "parallelism": "1 GPU, paths batched"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "prob_error": prob_err,
        "plain_fp64_sequential": {"value": seq_value, "unit": "trajectory-steps/s", "steps": seq_steps},
        "kernel_times": kernel_times,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
