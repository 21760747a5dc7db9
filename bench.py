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
FP32_MFMA_PEAK_TFLOPS = 157.3
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


def n_frow_entries(n_l, l_max):
    """Radial-integral entries of the row layout: for every output l' and input
    l, N_l' x N_l entries per multipole lambda = |l-l'|..l+l' step 2."""
    return sum(n_l[lp] * n_l[l] * (min(l, lp) + 1) for lp in range(l_max + 1) for l in range(l_max + 1))


def profiled_traffic(summary, source, field="traffic_bytes_per_launch"):
    """HBM bytes (per launch, or the given field) recorded in profiles/<summary>
    by the FETCH_SIZE and WRITE_SIZE counter runs, or None when the kernel
    source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_2403_04252_amd", "csrc", source)
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line:
            k, _, v = line.strip().partition(":")
            fields[k.strip()] = v.strip()
    key = source.replace(".hip", "").replace("kernels_", "kernels_") + "_sha256"
    if fields.get(key) != digest or field not in fields:
        return None
    return float(fields[field])


def copy_calibration(torch, mib):
    """One elementwise kernel that reads and writes mib MiB each (reference for
    the FETCH_SIZE / WRITE_SIZE counters of a profiled run)."""
    if mib <= 0:
        return
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


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
    ap.add_argument("--steps", type=int, default=None,
                    help="timed RK4 steps, each over all paths (default 800; 20 for c3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 40; 2 for c3)")
    ap.add_argument("--workload", choices=["c2", "c3", "sweep", "sweep2c", "paper"], default="c2",
                    help="c2: batched one-centre N=580 (the headline); c3: batched two-centre; "
                         "sweep: one-centre throughput against basis size (paper shape N_l = 42 - l); "
                         "paper: the paper's trajectory (v = 2, z -300..300 on 6001 points, 8 paths) "
                         "with exact-R and interpolated radial integrals; sweep2c: two-centre throughput "
                         "against basis size (paper shape N_l = 30 - l per centre, N = 60..1910)")
    ap.add_argument("--lmax", type=int, default=6, help="paper: l_max of the paper-shape basis (<= 7)")
    ap.add_argument("--v", type=float, default=1.0, help="c3: projectile speed of the batch (a.u.)")
    ap.add_argument("--mixed", action="store_true", help="c3: the reduced-precision contraction")
    ap.add_argument("--graph", action="store_true", help="c3: replay the steps from captured HIP graphs")
    ap.add_argument("--z0", type=float, default=None,
                    help="c3: steps of 0.1 from this z from a seeded random state (default: the workload's "
                         "grid from its start, from the ground state)")
    ap.add_argument("--explicit-m", action="store_true",
                    help="c3: form M = S^-1 H per coupling point (the paper's form) instead of solving per stage")
    ap.add_argument("--no-2c", action="store_true",
                    help="c2: skip the short two-centre measurement added to the output line")
    ap.add_argument("--no-seeded", action="store_true",
                    help="c2: skip the seeded 64-path FP64 / mixed comparison added to the output line")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing line")
    ap.add_argument("--stage-rows", type=int, default=0,
                    help="c2: rows per workgroup of the RK4 stage kernels (0: chosen by timing at plan creation)")
    ap.add_argument("--stage-launch", choices=["auto", "stages", "persistent"], default="auto",
                    help="c2: kernel per stage, persistent chunk kernel, or the faster (timed at plan creation)")
    ap.add_argument("--stage-cache", choices=["auto", "on", "off"], default="auto",
                    help="c2: stage kernels with the radial-integral cache, without, or timed at plan creation")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the one-path-per-launch comparison (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, launch one elementwise copy kernel that reads and writes "
                         "MIB MiB each (reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path "
              f"(paths are independent and would shard across GPUs without communication). "
              f"--gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c3":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_two_centre(args)
    if args.workload == "sweep2c":
        args.steps = 10 if args.steps is None else args.steps
        args.warmup = 2 if args.warmup is None else args.warmup
        return bench_sweep_2c(args)
    if args.workload == "paper":
        args.warmup = 20 if args.warmup is None else args.warmup
        return bench_paper(args)
    if args.workload == "sweep":
        args.steps = 200 if args.steps is None else args.steps
        args.warmup = 20 if args.warmup is None else args.warmup
        return bench_sweep(args)
    args.steps = 800 if args.steps is None else args.steps
    args.warmup = 40 if args.warmup is None else args.warmup

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
    launch = {"auto": W.WPCCC_LAUNCH_AUTO, "stages": W.WPCCC_LAUNCH_STAGES,
              "persistent": W.WPCCC_LAUNCH_PERSISTENT}[args.stage_launch]
    cache = {"auto": W.WPCCC_CACHE_AUTO, "on": W.WPCCC_CACHE_ON, "off": W.WPCCC_CACHE_OFF}[args.stage_cache]
    plan = W.wpccc_plan_create(lb, w.b, w.v, stage_rows=args.stage_rows, stage_launch=launch, stage_cache=cache)
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
    # probability error of the timed run against the oracle's stored full paths
    golden_err = golden_prob_error(torch, X, n_states, w, args.steps, "c2_paths.npz")
    # observables of the timed run (a whole grid: channel probabilities and
    # cross sections of the batch of impact parameters)
    obs = None
    if args.steps == w.zgrid.size - 1:
        Pobs = (X.abs() ** 2).contiguous()
        chan = torch.empty((n_traj, W.WPCCC_N_CHANNELS), dtype=torch.float64, device="cuda")
        sig = torch.empty((W.wpccc_plan_groups(plan)[0], W.WPCCC_N_CHANNELS), dtype=torch.float64, device="cuda")
        W.wpccc_observables(plan, Pobs, chan, sig)
        torch.cuda.synchronize()
        obs = {"cross_sections_au": dict(zip(W.CHANNELS, sig[0].cpu().numpy().tolist())),
               "note": "sigma = 2 pi int P b db (trapezoid over the 32 b, 0 at b = 0) at z = 40"}

    # the same K steps again with per-kernel HIP events on the library's stream
    X.zero_()
    X[:, 0] = 1.0
    persistent = W.wpccc_plan_stage_launch(plan) == W.WPCCC_LAUNCH_PERSISTENT
    W.wpccc_plan_timing(plan, True)
    run_propagation(W, plan, X, w.zgrid, args.steps)
    st_ms, st_n = W.wpccc_plan_kernel_time(plan, "k_stage")
    ch_ms, ch_n = W.wpccc_plan_kernel_time(plan, "k_chunk")
    su_ms, su_n = W.wpccc_plan_kernel_time(plan, "k_prologue")
    W.wpccc_plan_timing(plan, False)
    torch.cuda.synchronize()

    stage_flops = stage_work(n_l, rec.l_max) * n_traj
    # algorithmic bytes of one stage pass over the batch, the average of the
    # four stages of a step: stages 1 and 3 read the moment-table rows of the
    # step's next new point (one (A_k, B_k+1) pair of 16 B per radial-integral
    # entry), read the cached F of their own point (8 B) and write the new
    # point's F (8 B); stages 2 and 4 read the cached F (8 B): 20 B per entry;
    # plus five amplitude vectors (u_in, X, Xacc in and out, u_out)
    n_entries = n_frow_entries(n_l, rec.l_max)
    cached = W.wpccc_plan_stage_cache(plan)
    # without the cache every stage reads its point's table rows (16 B per entry)
    stage_bytes = n_traj * (n_entries * (20 if cached else 16) + 5 * n_states * 16)
    # the method's minimum per step: the table rows at the two new points
    step_min_bytes = n_traj * (2 * n_entries * 16 + 4 * 5 * n_states * 16)
    passes = 4 * args.steps   # stage passes in the timed run
    if persistent:
        # k_chunk runs the four stages of up to 64 steps per launch
        kname, k_ms, k_n = "k_chunk", ch_ms, ch_n
    else:
        kname, k_ms, k_n = "k_stage", st_ms, st_n
    launch_s = k_ms / max(k_n, 1) * 1e-3
    bytes_per_launch = stage_bytes * passes / max(k_n, 1)
    achieved = bytes_per_launch / launch_s / 1e9
    stage_pass_s = k_ms * 1e-3 / passes
    roof = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if persistent else profiled_traffic(
                "k_stage_1c_N580x32.md" if cached else "k_stage_direct_1c_N580x32.md", "kernels_1c.hip"),
            "radial_cache": cached,
            "avg_launch_us": launch_s * 1e6, "launches": k_n,
            "stage_passes_per_launch": passes / max(k_n, 1),
            "algorithmic_bytes_per_stage_pass": stage_bytes,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "flops_per_stage_pass": stage_flops,
            "fp64_alu_frac": stage_flops / stage_pass_s / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
            "stage_rows": W.wpccc_plan_stage_rows(plan),
            "method_min_bytes_per_step": step_min_bytes,
            "method_min_frac": step_min_bytes / (wall / args.steps) / 1e9 / HBM_PEAK_GBS}
    if persistent:
        t = profiled_traffic("k_chunk_1c_N580x32.md", "kernels_1c.hip", "traffic_bytes_per_stage_pass")
        roof["traffic"] = None if t is None else t * passes / max(k_n, 1)
    kernel_times = {"k_stage": {"total_ms": st_ms, "launches": st_n},
                    "k_chunk": {"total_ms": ch_ms, "launches": ch_n},
                    "k_prologue": {"total_ms": su_ms, "launches": su_n}}

    # plain FP64 form: the same paths one after another
    seq = None
    if not args.no_sequential:
        seq_steps = min(args.steps, 100)
        plan_seq = W.wpccc_plan_create(lb, w.b, w.v, batched=False)
        X.zero_()
        X[:, 0] = 1.0
        run_propagation(W, plan_seq, X, w.zgrid, 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_propagation(W, plan_seq, X, w.zgrid, seq_steps)
        torch.cuda.synchronize()
        seq = {"value": n_traj * seq_steps / (time.perf_counter() - t0), "unit": "trajectory-steps/s",
               "steps": seq_steps}
        del plan_seq

    copy_calibration(torch, args.copy_calibration)
    # sustained HBM rate of a plain copy (torch elementwise, 1 GiB read + 1 GiB written)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    roof["measured_copy_GBs"] = 5 * 2 * src.numel() * 8 / (time.perf_counter() - t0) / 1e9
    roof["frac_of_measured_copy"] = roof["achieved"] / roof["measured_copy_GBs"]
    del src, dst

    cpu = None
    prob_err_sample = None
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
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        affinity = len(os.sched_getaffinity(0))
        threads = min(blas, affinity)
        cpu = {"value": S / dt, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
               "affinity_cores": affinity,
               "sample": f"path b={w.b[0]:.4g} of the workload, first {S} of its 800 RK4 steps "
                         f"(numpy FP64, {blas} BLAS threads on {affinity} cores of the affinity mask), "
                         f"basis setup excluded"}
        # probability error of the GPU path on the same sample
        plan1 = W.wpccc_plan_create(lb, w.b[:1], w.v[:1])
        X1 = torch.zeros((1, plan1.n_pad), dtype=torch.complex128, device="cuda")
        X1[:, 0] = 1.0
        W.wpccc_propagate(plan1, zs, X1)
        torch.cuda.synchronize()
        Pg = (X1.abs() ** 2).cpu().numpy()[0, :n_states]
        Po = probabilities(Xo)
        dP = np.abs(Pg - Po)
        prob_err_sample = {"max_abs": float(dP.max()),
                           "max_rel_floored": float((dP / np.maximum(Po, P_FLOOR)).max()),
                           "floor": P_FLOOR, "sample": cpu["sample"]}
    prob_err = golden_err if golden_err is not None else prob_err_sample

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
                   "form": "batched FP64", "n_paths": n_traj,
                   "stage_launch": "persistent" if persistent else "per stage", "n_states": n_states,
                   "n_radial": n_radial, "n_r": n_r, "parallelism": "1 GPU, paths batched"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "prob_error": prob_err,
        "prob_error_cpu_sample": prob_err_sample,
        "observables": obs,
        "plain_fp64_sequential": seq,
        "kernel_times": kernel_times,
    }
    if not args.no_seeded:
        out["seeded_fp64_vs_mixed"] = seeded_measure(torch, W, WL)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_measure(torch, W, WL)
    if not args.no_2c:
        # secondary: batched two-centre steps through closest approach, FP64
        # and mixed, at each of the workload's three speeds
        del plan
        torch.cuda.empty_cache()
        out["two_centre"] = {}
        for v in (0.5, 1.0, 2.0):
            args.v = v
            pair = two_centre_pair(args, 20, 1)
            out["two_centre"][f"v={v:g}"] = pair
    print(json.dumps(out), flush=True)


def golden_prob_error(torch, X, n_states, w, steps, name):
    """max |dP| (absolute and relative with the floor) of the final probabilities
    of a whole-grid run against the oracle's stored paths (tests/golden/),
    or None when the run did not cover the whole grid or nothing is stored."""
    path = os.path.join(ROOT, "tests", "golden", name)
    if steps != w.zgrid.size - 1 or not os.path.exists(path):
        return None
    g = np.load(path)
    Pg = (X.abs() ** 2).cpu().numpy()[:, :n_states]
    dmax = rmax = 0.0
    for k, j in enumerate(g["paths"]):
        d = np.abs(Pg[j] - g["P"][k])
        dmax = max(dmax, float(d.max()))
        rmax = max(rmax, float((d / np.maximum(g["P"][k], P_FLOOR)).max()))
    return {"max_abs": dmax, "max_rel_floored": rmax, "floor": P_FLOOR,
            "sample": f"final probabilities of paths {list(map(int, g['paths']))} after all "
                      f"{steps} steps of the timed run against the FP64 oracle's stored paths"}


def seeded_measure(torch, W, WL, repeats=3):
    """The seeded workload (the N = 580 basis, 64 impact parameters, all 800
    steps) in FP64 and in the reduced-precision form: rates (median of
    `repeats` whole-grid runs after one warm-up) and every probability of the
    mixed run against the FP64 run and against the oracle's stored paths."""
    w = WL.single_centre_seeded()
    rec = w.basis
    lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
    res, Pf = {}, {}
    for mixed in (False, True):
        plan = W.wpccc_plan_create(lb, w.b, w.v, mixed=mixed)
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        times = []
        for rep in range(repeats + 1):
            X.zero_()
            X[:, 0] = 1.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            W.wpccc_propagate(plan, w.zgrid, X)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t0)
        W.wpccc_plan_status(plan)
        wall = float(np.median(times))
        steps = w.zgrid.size - 1
        Pf[mixed] = (X.abs() ** 2).cpu().numpy()[:, :plan.n_states]
        res["mixed" if mixed else "fp64"] = {
            "value": plan.n_traj * steps / wall, "unit": "trajectory-steps/s", "ms_per_step": wall / steps * 1e3,
            "dtype": "f64 (moment tables f32)" if mixed else "f64", "stage_rows": W.wpccc_plan_stage_rows(plan),
            "device_bytes": plan.device_bytes}
        del plan
    d = np.abs(Pf[True] - Pf[False])
    res["mixed"]["prob_error_vs_fp64_gpu"] = {
        "max_abs": float(d.max()), "max_rel": float((d / np.maximum(Pf[False], 1e-300)).max()),
        "within_bar": bool(np.all((d <= 1e-6) | (d <= 1e-4 * Pf[False]))),
        "sample": "every probability of all 64 paths after 800 steps"}
    g = os.path.join(ROOT, "tests", "golden", "c4_paths.npz")
    if os.path.exists(g):
        g = np.load(g)
        for key, P in (("fp64", Pf[False]), ("mixed", Pf[True])):
            dd = np.concatenate([np.abs(P[j] - g["P"][k]) for k, j in enumerate(g["paths"])])
            ref = np.concatenate([g["P"][k] for k in range(len(g["paths"]))])
            res[key]["prob_error_vs_oracle"] = {
                "max_abs": float(dd.max()), "max_rel_floored": float((dd / np.maximum(ref, P_FLOOR)).max()),
                "floor": P_FLOOR, "sample": f"paths {list(map(int, g['paths']))} of 64, oracle's stored run"}
    res["mixed_over_fp64"] = res["mixed"]["value"] / res["fp64"]["value"]
    res["workload"] = ("p+H 1C N=580 (n<=6 + 20 bins/l, l<=4), 4000-pt grid, 64 b log-uniform 0.05-20 "
                       "(default_rng(4)), v=1, z -40..40 dz=0.1")
    return res


def bench_sweep(args):
    """One-centre batched throughput against basis size with the paper's basis
    shape, N_l = 42 - l radial functions per l (bound n <= 10 plus 32 Coulomb
    wave-packet bins per l), l_max = 0..10, on a 2000-point grid; 8 paths with b
    log-spaced 0.2..10, v = 2, dz = 0.1 from z = -40.  Prints one JSON line with
    one entry per l_max (sizes the stage kernel's LDS cannot hold are listed as
    unsupported)."""
    import torch
    import paper_2403_04252_amd as W
    from paper_2403_04252_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    b = 0.2 * 50.0 ** (np.arange(8) / 7.0)
    v = np.full(8, 2.0)
    zg = WL.z_uniform(-40.0, -40.0 + 0.1 * (args.warmup + args.steps), 0.1)
    rows = []
    for l_max in range(11):
        rec = WL.Recipe(10, l_max, 32, 3.0, 2000)
        lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
        n_states = W.wpccc_basis_info(lb)[0]
        entry = {"l_max": l_max, "n_states": n_states}
        print(f"sweep l_max {l_max}: N = {n_states}", file=sys.stderr, flush=True)
        try:
            t0 = time.perf_counter()
            plan = W.wpccc_plan_create(lb, b, v)
            entry["plan_setup_s"] = time.perf_counter() - t0
        except W.WpcccError as e:
            entry["unsupported"] = str(e)
            rows.append(entry)
            continue
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X[:, 0] = 1.0
        W.wpccc_propagate(plan, zg[: args.warmup + 1], X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W.wpccc_propagate(plan, zg[args.warmup:], X)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        W.wpccc_plan_status(plan)
        entry.update({"value": plan.n_traj * args.steps / wall, "unit": "trajectory-steps/s",
                      "us_per_batched_step": wall / args.steps * 1e6,
                      "stage_rows": W.wpccc_plan_stage_rows(plan),
                      "device_bytes": plan.device_bytes})
        rows.append(entry)
        del plan, X
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "RK4 steps/s over batched b against basis size", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                      "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "p+H 1C, N_l = 42 - l (n <= 10 + 32 bins/l), l_max 0..10, "
                                             "2000-pt grid, 8 b log-spaced 0.2-10, v=2, dz=0.1",
                                 "parallelism": "1 GPU, paths batched"},
                      "sweep": rows}), flush=True)


def bench_sweep_2c(args):
    """Two-centre batched throughput against basis size with the paper's
    two-centre basis shape, N_l = 30 - l radial functions per l on each centre
    (bound n <= 6 plus 24 Coulomb bins per l), l_max = 0..5 (N = 60..1910),
    4000-point grids, 256 x 512 spheroidal nodes, prior lower-left block;
    8 paths (b log-spaced 0.2..10) at v = 2, `steps` steps of 0.1 from
    z = -0.5 (through closest approach, where the most nodes are active),
    replayed from HIP graphs (pipelined: the stages of a step beside the
    couplings of the next).  Prints one JSON line with one entry per l_max."""
    import torch
    import paper_2403_04252_amd as W
    from paper_2403_04252_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    b = 0.2 * 50.0 ** (np.arange(8) / 7.0)
    v = np.full(8, 2.0)
    zs = -0.5 + 0.1 * np.arange(args.steps + 1)
    rows = []
    for l_max in range(6):
        rec = WL.Recipe(6, l_max, 24, 3.0, 4000)
        lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
        t0 = time.perf_counter()
        plan = W.wpccc_plan_create_2c([lb], [lb], np.zeros(8, dtype=np.int32), b, v, q_lower=W.WPCCC_Q_PRIOR,
                                      n_eta=256, n_tau=512, graph=True)
        setup = time.perf_counter() - t0
        N = plan.n_states
        print(f"sweep2c l_max {l_max}: N = {N}", file=sys.stderr, flush=True)
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X[:, 0] = 1.0
        # at least six warm-up steps: they capture the five graphs of the slot rotation
        W.wpccc_propagate(plan, zs[: max(args.warmup, 6) + 1], X)
        X.zero_()
        X[:, 0] = 1.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W.wpccc_propagate(plan, zs, X)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        W.wpccc_plan_status(plan)
        rows.append({"l_max": l_max, "n_states": N, "value": plan.n_traj * args.steps / wall,
                     "unit": "trajectory-steps/s", "ms_per_batched_step": wall / args.steps * 1e3,
                     "plan_setup_s": setup, "device_bytes": plan.device_bytes})
        del plan, X
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "two-centre RK4 steps/s over batched b against basis size", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": "p+H 2C paper shape N_l = 30 - l per centre (n <= 6 + 24 bins/l), "
                                             "l_max 0..5, 4000-pt grids, 256x512 nodes, prior lower block, "
                                             "8 b log-spaced 0.2-10, v = 2, z -0.5..0.5",
                                 "form": "steps replayed from pipelined HIP graphs",
                                 "parallelism": "1 GPU, paths batched"},
                      "sweep": rows}), flush=True)


def bench_paper(args):
    """The paper's trajectory (Sec. III): p + H at 100 keV (v = 2 a.u.), z from
    -300 to 300 a.u. on the paper's geometric grid (z_min = 1e-3, n_z = 3000:
    6001 points, 6000 RK4 steps), 8 paths per batch (b log-spaced 0.2..10);
    one-centre basis of the paper's shape, N_l = 42 - l radial functions per l
    (bound n <= 10 plus 32 Coulomb bins per l) up to l_max, on a 10,000-point
    r-grid to 100 a.u.  Both radial forms: the exact-R quadrature (moment
    tables) and the paper's tabulated F with five-point interpolation.  Prints
    one JSON line: rates, setup times, and the difference of the two forms'
    final probabilities and cross sections."""
    import torch
    import paper_2403_04252_amd as W
    from paper_2403_04252_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    b = 0.2 * 50.0 ** (np.arange(8) / 7.0)
    v = np.full(8, 2.0)
    zg = WL.z_geometric(1e-3, 300.0, 3000)
    rec = WL.Recipe(10, args.lmax, 32, 3.0, 10000)
    t0 = time.perf_counter()
    lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
    basis_s = time.perf_counter() - t0
    n_states = W.wpccc_basis_info(lb)[0]
    res, Pf, sig = {}, {}, {}
    for form in ("exact", "interp"):
        print(f"paper trajectory: N = {n_states}, radial form {form}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        plan = W.wpccc_plan_create(lb, b, v, interp=(form == "interp"))
        setup = time.perf_counter() - t0
        X = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X[:, 0] = 1.0
        W.wpccc_propagate(plan, zg[: args.warmup + 1], X)
        X.zero_()
        X[:, 0] = 1.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W.wpccc_propagate(plan, zg, X)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        W.wpccc_plan_status(plan)
        steps = zg.size - 1
        P = (X.abs() ** 2).contiguous()
        chan = torch.empty((plan.n_traj, W.WPCCC_N_CHANNELS), dtype=torch.float64, device="cuda")
        sg = torch.empty((1, W.WPCCC_N_CHANNELS), dtype=torch.float64, device="cuda")
        W.wpccc_observables(plan, P, chan, sg)
        torch.cuda.synchronize()
        Pf[form] = P.cpu().numpy()[:, :n_states]
        sig[form] = sg.cpu().numpy()[0]
        res[form] = {"value": plan.n_traj * steps / wall, "unit": "trajectory-steps/s",
                     "ms_per_step": wall / steps * 1e3, "plan_setup_s": setup,
                     "stage_rows": W.wpccc_plan_stage_rows(plan), "device_bytes": plan.device_bytes,
                     "cross_sections_au": dict(zip(W.CHANNELS, sig[form].tolist()))}
        del plan, X, P
        torch.cuda.empty_cache()
    d = np.abs(Pf["interp"] - Pf["exact"])
    print(json.dumps({"metric": "RK4 steps/s over batched b on the paper's trajectory", "n_gpus": 1,
                      "steps": int(zg.size - 1), "warmup": args.warmup, "higher_is_better": True, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": f"p+H 1C paper shape N_l = 42 - l, l_max {args.lmax} (N = {n_states}), "
                                             "10000-pt r-grid to 100 a.u., 8 b log-spaced 0.2-10, v = 2 (100 keV), "
                                             "geometric z-grid -300..300 (6001 points, z_min 1e-3)",
                                 "parallelism": "1 GPU, paths batched", "basis_setup_s": basis_s},
                      "exact": res["exact"], "interp": res["interp"],
                      "interp_vs_exact": {"max_abs_dP": float(d.max()),
                                          "max_rel_sigma": float(np.max(np.abs(sig["interp"] - sig["exact"])
                                                                        / np.maximum(np.abs(sig["exact"]), 1e-300)))}}),
          flush=True)


def adjoint_measure(torch, W, WL):
    """Gradients of a weighted sum of final probabilities with respect to the
    screened-potential parameters and b (16 paths, N = 86, 800 steps): the
    reverse sweep's wall time against the forward propagation's."""
    wl = WL.adjoint_batch()
    rec = wl.basis
    lb = W.wpccc_basis(W.BasisSpec(rec.n_max, rec.l_max, rec.n_bins, rec.k_max, rec.n_r, rec.r_max, rec.Z))
    plan = W.wpccc_plan_create(lb, wl.b, wl.v, model_a=wl.a, model_c=wl.c)
    N = plan.n_states
    X0 = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    X0[:, 0] = 1.0
    Xf = X0.clone()
    W.wpccc_propagate(plan, wl.zgrid, Xf)        # warm-up and the final state
    torch.cuda.synchronize()
    Xf.copy_(X0)
    t0 = time.perf_counter()
    W.wpccc_propagate(plan, wl.zgrid, Xf)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    gX = torch.zeros_like(X0)
    gX[:, :N] = torch.as_tensor(wl.weights, device="cuda") * Xf[:, :N]
    grad = torch.empty((plan.n_traj, 3), dtype=torch.float64, device="cuda")
    X = torch.empty_like(X0)
    W.wpccc_adjoint(plan, wl.zgrid, X0, gX, grad, X)   # warm-up (workspace allocation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W.wpccc_adjoint(plan, wl.zgrid, X0, gX, grad, X)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    W.wpccc_plan_status(plan)
    steps = wl.zgrid.size - 1
    return {"workload": "p+H 1C N=86 screened potential, 16 b, 800 steps (gradients in a, c, b)",
            "forward_ms": t_fwd * 1e3, "adjoint_ms": t_adj * 1e3, "adjoint_over_forward": t_adj / t_fwd,
            "value": plan.n_traj * steps / t_adj, "unit": "trajectory-steps/s (forward + reverse sweep)"}


def n_per_l(rec):
    """Radial functions per l of a basis recipe: bound n <= n_max (n > l) plus the bins."""
    return [max(0, rec.n_max - l) + rec.n_bins for l in range(rec.l_max + 1)]


def contract_flops(recT, recP, n_w, n_act, mirror=False):
    """Algorithmic flops of the Eq. K2 contraction of one position: for molecular
    |q'| = s, |q| = t, 2 * nk(s, t) * nA[s] * nB[t] per active node, nA[s] = radial
    functions of the target with l >= s; nk = 2 n_w weights (cos, sin) per
    Bessel order, one order when s t = 0 and two (|s-t|, s+t) otherwise.
    mirror (one basis on both centres): the blocks s < t form three weights
    (overlap, target and projectile potential), s = t two, and s > t none
    (they follow from block (t, s)); in a block s = t the overlap is needed
    only for a >= b (the element (a, b) follows from (b, a)), counted here
    element by element although the kernel forms it in whole 32 x 32 tiles."""
    nlT, nlP = n_per_l(recT), n_per_l(recP)
    nA = [sum(nlT[s:]) for s in range(len(nlT))]
    nB = [sum(nlP[t:]) for t in range(len(nlP))]
    tot = 0
    for s in range(len(nA)):
        for t in range(len(nB)):
            nwb = (3 if s < t else (2 if s == t else 0)) if mirror else n_w
            per = (2 if s > 0 and t > 0 else 1) * 2   # (order, trig) pairs
            if mirror and s == t:
                # target potential on the whole block, overlap on a >= b
                tot += 2 * per * (nA[s] * nB[t] + nA[s] * (nA[s] + 1) // 2)
            else:
                tot += 2 * per * nwb * nA[s] * nB[t]
    return tot * n_act


def bench_two_centre(args):
    """Batched two-centre propagation (Eq. 1 with capture) on one GPU: prints its own JSON line."""
    out = two_centre_measure(args, args.steps, args.warmup, mixed=args.mixed, explicit=args.explicit_m,
                             graph=args.graph, z0=args.z0)
    out.pop("P_final", None)
    print(json.dumps(out), flush=True)


def two_centre_pair(args, steps, warmup, z0=-1.0):
    """FP64 and mixed two-centre rates over `steps` steps of 0.1 from z0 (through
    closest approach by default), both from the same seeded random state, and
    the mixed probabilities against the FP64 ones at the end of the stretch;
    steps replayed from HIP graphs, beside the explicit-M form and FP64
    launched kernel by kernel."""
    r64 = two_centre_measure(args, steps, warmup, mixed=False, z0=z0, graph=True)
    rmx = two_centre_measure(args, steps, warmup, mixed=True, z0=z0, graph=True)
    rex = two_centre_measure(args, steps, warmup, mixed=False, z0=z0, explicit=True, graph=True)
    rgr = two_centre_measure(args, steps, warmup, mixed=False, z0=z0, graph=False)
    P64, Pmx, Pex, Pgr = r64.pop("P_final"), rmx.pop("P_final"), rex.pop("P_final"), rgr.pop("P_final")
    d = np.abs(Pmx - P64)
    keep = ("value", "unit", "ms_per_step", "roofline", "lu", "config", "kernel_times")
    out = {"fp64": {k: r64[k] for k in keep}, "mixed": {k: rmx[k] for k in keep},
           "fp64_explicit_m": {k: rex[k] for k in keep + ("rhs",)}}
    out["fp64_explicit_m"]["dtype"] = "f64"
    out["fp64_explicit_m"]["max_abs_dP_vs_factored"] = float(np.abs(Pex - P64).max())
    out["fp64_no_graph"] = {k: rgr[k] for k in ("value", "unit", "ms_per_step")}
    out["fp64_no_graph"]["bitwise_equal_to_graph"] = bool(np.array_equal(Pgr, P64))
    out["fp64"]["dtype"] = "f64"
    out["mixed"]["dtype"] = "f64 (contraction products f32)"
    out["mixed"]["prob_error_vs_fp64_gpu"] = {
        "max_abs": float(d.max()), "max_rel": float((d / np.maximum(P64, 1e-300)).max()),
        "within_bar": bool(np.all((d <= 1e-6) | (d <= 1e-4 * P64))),
        "sample": f"every probability of the 24 paths after the {steps} timed steps from a seeded random state"}
    out["mixed_over_fp64"] = rmx["value"] / r64["value"]
    return out


def two_centre_measure(args, steps, warmup, mixed=False, z0=None, explicit=False, graph=False):
    """Time `steps` RK4 steps of the batched two-centre workload; returns the
    result dict.  z0 None: the workload's grid from its start, amplitudes from
    e_0; else `steps` steps of 0.1 from z0 from a seeded random state (the
    final probabilities are returned as "P_final")."""
    import torch
    from scipy.special import roots_laguerre
    import paper_2403_04252_amd as W
    from paper_2403_04252_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WL.two_centre_batched(args.v)
    bases = [W.wpccc_basis(W.BasisSpec(r.n_max, r.l_max, r.n_bins, r.k_max, r.n_r, r.r_max, r.Z))
             for r in w.targets]
    ql = W.WPCCC_Q_PRIOR if w.q_lower == "prior" else W.WPCCC_Q_DAGGER
    t0 = time.perf_counter()
    plan = W.wpccc_plan_create_2c(bases, bases, w.set_of, w.b, w.v, q_lower=ql, n_eta=w.n_eta, n_tau=w.n_tau,
                                  mixed=mixed, solve=W.WPCCC_SOLVE_EXPLICIT if explicit else W.WPCCC_SOLVE_FACTORED,
                                  graph=graph)
    setup_s = time.perf_counter() - t0
    n_traj = plan.n_traj
    X = torch.zeros((n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
    if z0 is None:
        zs = w.zgrid[: steps + 1]
        X0 = X.clone()
        X0[:, 0] = 1.0
    else:
        zs = z0 + 0.1 * np.arange(steps + 1)
        X0 = X.clone()
        for j in range(n_traj):
            N = W.wpccc_plan_path_info(plan, j)[0]
            X0[j, :N] = torch.from_numpy(WL.random_state(1, N, seed=100 + j)[0]).cuda()
    X.copy_(X0)
    # graph replay: six warm-up steps capture the five graphs of the pipelined
    # slot rotation (three, both per-slot graphs of the explicit form)
    run_propagation(W, plan, X, zs, max(warmup, 6) if graph else warmup)
    torch.cuda.synchronize()
    X.copy_(X0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W.wpccc_propagate(plan, zs, X)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    W.wpccc_plan_status(plan)
    value = n_traj * steps / wall
    P_final = (X.abs() ** 2).cpu().numpy()

    # per-kernel device time over the same steps (events on the library's stream)
    X.copy_(X0)
    W.wpccc_plan_timing(plan, True)
    W.wpccc_propagate(plan, zs, X)
    names = ["k_2c_contract", "k_2c_reduce", "k_2c_interp", "k_2c_nodes", "k_2c_assemble", "k_setup_batch",
             "k_2c_direct", "k_lu_check", "k_lu_panel", "k_lu_swap_trsm", "k_lu_update", "k_2c_hu", "k_2c_solve",
             "k_lu_rhs"]
    kt = {}
    for nm in names:
        ms, n = W.wpccc_plan_kernel_time(plan, nm)
        kt[nm] = {"total_ms": ms, "launches": n}
    W.wpccc_plan_timing(plan, False)
    torch.cuda.synchronize()
    copy_calibration(torch, args.copy_calibration)

    # algorithmic flops of the contraction over the timed steps: the first step
    # computes z, z_mid, z_new, later steps z_mid and z_new
    # the plan is given one basis object per size for both centres, so the
    # prior block comes from Q by symmetry (two weights in the contraction)
    # and the overlap of the blocks s > t from block (t, s)
    n_w, mirror = 2, True
    xl = roots_laguerre(w.n_eta)[0]
    fl = 0
    for i in range(steps):
        pos = [zs[i], 0.5 * (zs[i] + zs[i + 1]), zs[i + 1]] if i == 0 else [0.5 * (zs[i] + zs[i + 1]), zs[i + 1]]
        for j in range(n_traj):
            rec = w.targets[w.set_of[j]]
            for z in pos:
                R = math.hypot(w.b[j], z)
                lim = (2 * rec.r_max - R) * (1.0 + 1e-12) + 1e-12
                n_act = int(np.sum(xl <= lim)) * w.n_tau
                fl += contract_flops(rec, rec, n_w, n_act, mirror)
    c_ms = kt["k_2c_contract"]["total_ms"]
    achieved = fl / (c_ms * 1e-3) / 1e12
    peak = FP32_MFMA_PEAK_TFLOPS if mixed else FP64_VECTOR_PEAK_TFLOPS
    # sustained rate of back-to-back independent 16x16x4 MFMAs on this device
    ceil64, ceil32 = W.wpccc_measure_mfma()
    ceiling = ceil32 if mixed else ceil64
    roof = {"kernel": "k_2c_contract", "bound": "mfma", "achieved": achieved,
            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None, "avg_launch_us": c_ms / max(kt["k_2c_contract"]["launches"], 1) * 1e3,
            "launches": kt["k_2c_contract"]["launches"], "algorithmic_flops_total": fl,
            "measured_mfma_ceiling": ceiling, "frac_of_measured_ceiling": achieved / ceiling}
    lu_fl = rhs_fl = 0
    for j in range(n_traj):
        N = 2 * sum((2 * l + 1) * n for l, n in enumerate(n_per_l(w.targets[w.set_of[j]])))
        lu_fl += (steps * 2 + 1) * 8.0 / 3.0 * N ** 3
        rhs_fl += (steps * 2 + 1) * 8.0 * N ** 3   # two triangular solves with N right-hand sides
    lu_ms = sum(kt[k]["total_ms"] for k in ("k_lu_check", "k_lu_panel", "k_lu_swap_trsm", "k_lu_update"))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + ": same recipe on both centres (n<=6 + 20 bins/l, l<=1/2/3), "
                               "4000-pt grid, 8 b log-spaced 0.2-10 per size, 256x512 nodes, "
                               f"z {zs[0]:.1f}..{zs[-1]:.1f} dz=0.1, lower-left block {w.q_lower}",
                   "form": ("batched mixed (FP32 contraction products)" if mixed else "batched FP64")
                           + (", explicit M = S^-1 H" if explicit else ", per-stage triangular solves")
                           + (", graph replay" if graph else ""),
                   "n_paths": n_traj, "plan_setup_s": setup_s,
                   "parallelism": "1 GPU, paths batched per basis size"},
        "roofline": roof,
        "lu": {"algorithmic_flops": lu_fl, "device_ms": lu_ms,
               "achieved_tflops": lu_fl / max(lu_ms * 1e-3, 1e-12) / 1e12},
        "kernel_times": kt,
        "cpu_baseline": None,
    }
    if explicit:
        rhs_ms = kt["k_lu_rhs"]["total_ms"]
        out["rhs"] = {"algorithmic_flops": rhs_fl, "device_ms": rhs_ms,
                      "achieved_tflops": rhs_fl / max(rhs_ms * 1e-3, 1e-12) / 1e12}
    if z0 is not None:
        out["P_final"] = P_final
    return out


if __name__ == "__main__":
    main()
