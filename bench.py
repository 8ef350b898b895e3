#!/usr/bin/env python3
"""Throughput of the orthonormalization-multigrid solve on one MI355X.

Workload (one "step" = one complete solve): the SIP-DG Poisson problem on
64^3 cells with the P2 basis (2,621,440 DOFs), coefficient 1 inside a sphere
of radius 0.3 centred in the unit cube and 1000 outside, iid N(0,1)
right-hand side (seed 0), 4-level agglomeration hierarchy (64/32/16/8),
multiplicative synchronous cycle (Algorithm 2) with 2 pre- and 2
post-block-Jacobi iterations (omega = 0.7), level criteria of Sec. 4.2,
coarsest level by dense Cholesky, solved to relative residual 1e-10 in FP64
from x0 = 0. Inputs are resident in HBM before the timed region starts;
setup (assembly, hierarchy, factorisations) is outside it.

Prints one JSON line: DOF/s (FP64) with the mixed-precision (FP32 inner,
FP64 iterative refinement) result beside it, the roofline of the dominant
kernel (durations measured with HIP events on its stream during a solve),
and the FP64 CPU oracle timed on a bounded sample of the same solve.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_RM = os.path.join(ROOT, "profiles", "rm_persistent_L0_64cubed_p2.md")
RM_SOURCE = os.path.join(ROOT, "paper_2512_08728_amd", "csrc", "omg_rm.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rm_kernel_sha():
    """Hash of the RM kernel's source: the part of its file before the
    direction-recombination kernels (exchange helpers and the kernel itself)."""
    text = open(RM_SOURCE, "rb").read()
    end = text.find(b"// Coefficients of x = sum_k alpha_k z_k")
    return hashlib.sha256(text[:end] if end > 0 else text).hexdigest()


def profile_traffic(alg_bytes):
    """HBM bytes per launch of the finest-level persistent RM kernel from the
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by what the same counter reads for the plain copy
    kernel of known size). None when the summary is absent or was taken on a
    different kernel source."""
    if not os.path.exists(PROFILE_RM):
        return None
    kv = {}
    for line in open(PROFILE_RM):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            v = v.strip()
            kv[k.strip()] = v.split("`")[1] if v.startswith("`") else v
    sha = rm_kernel_sha()
    if kv.get("source_sha256") != sha:
        return None
    copy = float(kv["copy_bytes_each_way"])
    fetch = float(kv["fetch_kib_per_dispatch"]) * 1024 * copy / (float(kv["copy_fetch_kib"]) * 1024)
    write = float(kv["write_kib_per_dispatch"]) * 1024 * copy / (float(kv["copy_write_kib"]) * 1024)
    kernel = kv.get("kernel", "?")
    return {"bytes": round(fetch + write), "ratio_to_algorithmic": round((fetch + write) / alg_bytes, 4),
            "note": f"counters of {kernel} over {kv.get('dispatches', '?')} dispatches"}


def batched_bench(omg, synth, torch):
    """Batched workloads: 32 right-hand sides on one 32^3 P2 operator in
    lockstep (matrix-core multi-RHS block products) against one single solve,
    and 16 uneven instances (16^3..48^3 P2, FP64 outer / FP32 inner) in one
    batched call against the same solves one after another."""
    out = {}
    prob = synth.make_problem(32, 2)
    nu = synth.nu_sphere(32, 32, 32, prob.h)
    grid = omg.Solver.make_grid(32, 32, 32, 2, prob.n_levels, prob.h)
    s = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), s_pre=2, s_post=2)
    B = torch.tensor(synth.multi_rhs(prob.n_dofs, 32, seed=0), device="cuda")
    omg.solve_batched([s], [B], nrhs=32)  # creates the column solvers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, reps = omg.solve_batched([s], [B], nrhs=32)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    b0 = B[:, 0].contiguous()
    s.solve(b0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve(b0)
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    out["multi_rhs_32x32cubed_p2"] = {
        "value": prob.n_dofs * 32 / tb, "unit": "DOF/s", "ms": round(tb * 1e3, 1),
        "single_solve_ms": round(t1 * 1e3, 1), "speedup_vs_32_single": round(32 * t1 / tb, 2),
        "iters_fine": [r["iters_fine"] for r in reps], "max_rel_res_true": max(r["rel_res_true"] for r in reps)}
    log(f"multi-RHS: {out['multi_rhs_32x32cubed_p2']}")
    s.close()
    insts = synth.instances(16, seed=2)
    solvers, rhs, dofs = [], [], 0
    for inst in insts:
        pr = synth.make_problem(inst.n, 2)
        nu_i = synth.nu_sphere(inst.n, inst.n, inst.n, pr.h, center=inst.center, radius=inst.radius,
                               nu_out=inst.ratio)
        g = omg.Solver.make_grid(inst.n, inst.n, inst.n, 2, pr.n_levels, pr.h)
        solvers.append(omg.Solver.from_sip(g, torch.tensor(nu_i, device="cuda"), s_pre=2, s_post=2,
                                           precision="mixed_ir"))
        rhs.append(torch.tensor(synth.rhs(pr.n_dofs, inst.seed), device="cuda").reshape(-1, 1))
        dofs += pr.n_dofs
    omg.solve_batched(solvers, rhs, nrhs=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, reps = omg.solve_batched(solvers, rhs, nrhs=1)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for sv, r in zip(solvers, rhs):
        sv.solve(r.reshape(-1))
    torch.cuda.synchronize()
    tseq = time.perf_counter() - t0
    out["instances_16_p2_mixed"] = {
        "value": dofs / tb, "unit": "DOF/s", "ms": round(tb * 1e3, 1), "sequential_ms": round(tseq * 1e3, 1),
        "speedup_vs_sequential": round(tseq / tb, 2), "cells_per_side": [i.n for i in insts], "total_dofs": dofs,
        "max_rel_res_true": max(r["rel_res_true"] for r in reps)}
    log(f"instances: {out['instances_16_p2_mixed']}")
    for sv in solvers:
        sv.close()
    return out


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def cpu_full_solve(omg, synth, torch, n=16, p=2, runs=3):
    """Complete solves of a configuration the oracle finishes in seconds
    (16^3 P2, 40,960 DOFs, two levels, the same field, sweeps, cycle and
    tolerance as the headline): the FP64 oracle on all host cores (median of
    `runs`) and on one thread, beside the GPU on the same configuration
    (median of 5 after a warm-up)."""
    import oracle
    prob = synth.make_problem(n, p)
    nu = synth.nu_sphere(n, n, n, prob.h)
    b = synth.rhs(prob.n_dofs, 0)
    cores = os.cpu_count()
    oracle.set_threads(cores)
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2, omega=0.7)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        o.solve(b, tol=1e-10)
        times.append(time.perf_counter() - t0)
    cyc = o.last_report["iters_fine"]
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.solve(b, tol=1e-10)
    t1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    grid = omg.Solver.make_grid(n, n, n, p, prob.n_levels, prob.h)
    g = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), s_pre=2, s_post=2, omega=0.7)
    bd = torch.tensor(b, device="cuda")
    g.solve(bd, tol=1e-10)
    gt = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.solve(bd, tol=1e-10)
        torch.cuda.synchronize()
        gt.append(time.perf_counter() - t0)
    gcyc = g.last_report["iters_fine"]
    g.close()
    return {"workload": f"{n}^3 P{p} ({prob.n_dofs} DOFs), {prob.n_levels} levels, sphere r=0.3 nu 1:1000, "
                        f"2+2 block-Jacobi, Alg. 2, tol 1e-10, b seed 0",
            "nproc": cores, "oracle_cycles": cyc, "gpu_cycles": gcyc,
            "oracle_all_cores": {"value": prob.n_dofs / median(times), "unit": "DOF/s", "cores": cores,
                                 "s_median_of_3": round(median(times), 3)},
            "oracle_1_thread": {"value": prob.n_dofs / t1, "unit": "DOF/s", "cores": 1, "s": round(t1, 3)},
            "gpu": {"value": prob.n_dofs / median(gt), "unit": "DOF/s", "s_median_of_5": round(median(gt), 4)}}


def cycle_sweep(omg, synth, torch):
    """Finest-level cycles and level-1 behaviour of the headline solve's
    configuration (P2, sphere r = 0.3, ratio 1000, 2+2 sweeps, Sec. 4.2
    criteria, levels down to 8^3 or an odd side) over the mesh size."""
    out = []
    for n in (16, 24, 32, 48, 64):
        prob = synth.make_problem(n, 2)
        nu = synth.nu_sphere(n, n, n, prob.h)
        grid = omg.Solver.make_grid(n, n, n, 2, prob.n_levels, prob.h)
        g = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), s_pre=2, s_post=2, omega=0.7)
        g.solve(torch.tensor(synth.rhs(prob.n_dofs, 0), device="cuda"), tol=1e-10)
        v = g.visits()
        l1 = v[v[:, 0] == 1][:, 1]
        row = {"n": n, "levels": prob.n_levels, "dofs": prob.n_dofs, "cycles": g.last_report["iters_fine"],
               "level1_mean_iters": round(float(l1.mean()), 2) if len(l1) else None,
               "level1_at_cap": round(float((l1 == 20).mean()), 3) if len(l1) else None}
        log(f"cycle sweep: {row}")
        out.append(row)
        g.close()
    return out


def cpu_baseline(prob, nu, b, gpu_cycles, cycles=4):
    """The FP64 oracle on the host cores: the first `cycles` cycles of the
    same solve, scaled to DOF/s of the full solve by the GPU's cycle count."""
    import oracle
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2, omega=0.7, max_iter=cycles)
    t0 = time.perf_counter()
    o.solve(b, tol=1e-10, check=False)
    dt = time.perf_counter() - t0
    frac = cycles / max(gpu_cycles, 1)
    return {
        "value": prob.n_dofs * frac / dt,
        "unit": "DOF/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"first {cycles} of the {gpu_cycles} cycles of the same 64^3 P2 FP64 solve "
                   f"({dt:.1f} s); DOF/s = DOFs x {cycles}/{gpu_cycles} / time. Later cycles hold more "
                   f"stored directions, so this overstates the oracle's full-solve rate"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="cells per side")
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision solves and the other Table 1 configurations")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--cycle-sweep", action="store_true",
                    help="also report finest-level cycles over mesh sizes 16..64")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run the library's plain copy kernel on one finest-level vector "
                         "(reference for traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solve is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_08728_amd as omg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = synth.make_problem(args.n, args.p)
    nu = synth.nu_sphere(args.n, args.n, args.n, prob.h)
    b_host = synth.rhs(prob.n_dofs, 0)
    b = torch.tensor(b_host, device="cuda")
    grid = omg.Solver.make_grid(prob.nx, prob.ny, prob.nz, prob.p, prob.n_levels, prob.h)
    opts = dict(s_pre=2, s_post=2, omega=0.7)
    t0 = time.perf_counter()
    s = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), **opts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"setup {t_setup:.2f} s, {prob.n_dofs} DOFs, {prob.n_levels} levels")
    if args.calib_copy:
        ms, by = s.bench_kernel(omg.K_COPY, 0, reps=5)
        log(f"calibration copy: {by / 2:.0f} bytes read + {by / 2:.0f} written per launch, {ms * 1e3:.1f} us")

    for w in range(args.warmup):
        s.solve(b, tol=1e-10)
        log(f"warmup {w}: {s.last_report}")
    s.kernel_counts()  # reset counters
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    reps = []
    for k in range(args.steps):
        x = s.solve(b, tol=1e-10)
        reps.append(s.last_report)
        log(f"step {k}: {s.last_report['t_solve_ms']:.1f} ms, {s.last_report['iters_fine']} cycles")
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = prob.n_dofs / (ms_per_step / 1e3)
    counts = s.kernel_counts() / args.steps
    rep = reps[-1]

    # dominant kernel. The persistent RM kernel's bytes and duration depend on the
    # number of stored directions, so it is measured live over a whole solve; the
    # other kernels are estimated as launches per solve x isolated duration.
    probed = {}

    def probe(kind, level):
        s.probe(kind, level, max_launches=200000)
        s.solve(b, tol=1e-10)
        n_l, avg_ms, alg = s.probe_result()
        probed[(kind, level)] = (n_l, avg_ms, alg)
        return n_l, avg_ms, alg

    cand = []
    for l in range(prob.n_levels):  # the persistent RM of every level, timed live over a solve
        if counts[omg.K_RMP, l] > 0:
            n_l, avg_ms, _ = probe(omg.K_RMP, l)
            cand.append((counts[omg.K_RMP, l] * avg_ms, omg.K_RMP, l, avg_ms))
    for kind in (omg.K_SPMV, omg.K_BJ, omg.K_MGS, omg.K_BJFIRST, omg.K_RMFIN, omg.K_RESTRICT, omg.K_PROLONG,
                 omg.K_COARSE):
        for l in range(prob.n_levels):
            if counts[kind, l] <= 0:
                continue
            try:
                ms, _ = s.bench_kernel(kind, l, reps=10)
            except omg.OmgError:
                continue
            cand.append((counts[kind, l] * ms, kind, l, ms))
    cand.sort(reverse=True)
    breakdown = {f"{omg.K_NAMES[k]}@L{l}": round(float(t), 2) for t, k, l, _ in cand[:14]}
    log(f"estimated ms per solve by kernel: {breakdown}")
    # the roofline is taken on the finest level, whose data stream from HBM
    # (the coarser levels' operators and directions largely sit in the
    # 256 MB last-level cache, where HBM peak is not the bound)
    roof = None
    for _, kind, l, _ in cand:
        if l == 0 and kind in (omg.K_SPMV, omg.K_BJ, omg.K_MGS, omg.K_RMP):
            n_l, avg_ms, alg = probed.get((kind, l)) or probe(kind, l)
            achieved = alg / (avg_ms * 1e-3) / 1e9
            tr = profile_traffic(alg) if (kind == omg.K_RMP and l == 0) else None
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr["bytes"] if tr else None,
                    "traffic_detail": tr,
                    "kernel": f"{omg.K_NAMES[kind]} level {l}", "launches_timed": n_l,
                    "avg_us": round(avg_ms * 1e3, 2), "alg_bytes_per_launch": alg}
            break

    # SpMV and block-Jacobi sweep against the HBM peak (isolated launches,
    # algorithmic bytes: stored blocks, column indices, vectors once)
    hbm_kernels = {}
    for kind in (omg.K_SPMV, omg.K_BJ, omg.K_SPMV32, omg.K_BJ32):
        for l in range(min(2, prob.n_levels - 1)):
            try:
                ms, by = s.bench_kernel(kind, l, reps=10)
            except omg.OmgError:
                continue
            gbs = by / (ms * 1e-3) / 1e9
            hbm_kernels[f"{omg.K_NAMES[kind]}@L{l}"] = {"GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                                       "us": round(ms * 1e3, 2), "alg_bytes": by}
    log(f"SpMV / smoother HBM: {hbm_kernels}")

    mixed = None
    if not args.no_mixed:
        mixed = {}
        for mode in ("mixed_ir", "mixed_flex"):
            sm = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), precision=mode, **opts)
            sm.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xm = sm.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            tm = time.perf_counter() - t0
            r = sm.last_report
            err = float(torch.linalg.norm(xm - x) / torch.linalg.norm(x))
            mixed[mode] = {"value": prob.n_dofs / tm, "unit": "DOF/s", "ms_per_step": round(tm * 1e3, 2),
                           "iters_fine": r["iters_fine"], "outer_iters": r["outer_iters"],
                           "rel_res_true": r["rel_res_true"], "rel_diff_to_fp64": err}
            log(f"{mode}: {mixed[mode]}")
            sm.close()

    # the other configurations of Table 1 on the same workload (FP64):
    # additive task-parallel (deterministic Algorithm 5: the coarse-grid
    # correction on a second stream while the smoother steps run on the
    # caller's stream), hybrid (Algorithm 2 on the finest level, the
    # Algorithm 5 form below, level 1 forking) and additive synchronous (the
    # Algorithm 5 order on one stream)
    variants = None
    if not args.no_mixed:
        variants = {"sync_mult": {"value": value, "unit": "DOF/s", "ms_per_step": round(ms_per_step, 2),
                                  "iters_fine": rep["iters_fine"], "rel_res_true": rep["rel_res_true"]}}
        # the last three: timing-adaptive loops (Sec. 4.3), the smoother side
        # stepping while the coarse path runs (at most 10 steps per cycle),
        # the last of them inside the mixed form with FP32 inner work
        for name, v, nsm, prec in (("overlap_det", "overlap", 0, "fp64"), ("hybrid", "hybrid", 0, "fp64"),
                                   ("add_sync", "add_sync", 0, "fp64"), ("overlap_adaptive", "overlap", 10, "fp64"),
                                   ("hybrid_adaptive", "hybrid", 10, "fp64"),
                                   ("overlap_adaptive_mixed_flex", "overlap", 10, "mixed_flex")):
            so = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), variant=v, n_s_max=nsm, precision=prec,
                                     **opts)
            so.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xo = so.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            to = time.perf_counter() - t0
            r = so.last_report
            variants[name] = {"value": prob.n_dofs / to, "unit": "DOF/s", "ms_per_step": round(to * 1e3, 2),
                              "iters_fine": r["iters_fine"], "rel_res_true": r["rel_res_true"],
                              "rel_diff_to_sync": float(torch.linalg.norm(xo - x) / torch.linalg.norm(x))}
            if nsm:
                sc = so.step_counts()
                variants[name]["steps_per_cycle_mean"] = round(float(sc.mean()), 2) if len(sc) else None
            log(f"{name}: {variants[name]}")
            so.close()
        # the additive Schwarz smoother (Algorithm 3; one subdomain per cell,
        # one-cell overlap, patch inverses formed at setup) in Algorithm 2:
        # one sweep (omega cancels in RM) and two sweeps damped to 0.1 (the
        # overlapping patch inverses give lambda_max(M A) ~ 11, so repeated
        # sweeps need omega below ~0.18); the last with single-precision local
        # solves inside the mixed form
        for sw, om, prec in ((1, 0.7, "fp64"), (2, 0.1, "fp64"), (2, 0.1, "mixed_flex")):
            o2 = dict(opts, s_pre=sw, s_post=sw, omega=om, precision=prec)
            t0 = time.perf_counter()
            so = omg.Solver.from_sip(grid, torch.tensor(nu, device="cuda"), smoother="schwarz", **o2)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            so.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xo = so.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            to = time.perf_counter() - t0
            r = so.last_report
            name = f"schwarz_{sw}+{sw}" + ("" if prec == "fp64" else f"_{prec}")
            variants[name] = {"value": prob.n_dofs / to, "unit": "DOF/s", "ms_per_step": round(to * 1e3, 2),
                              "iters_fine": r["iters_fine"], "rel_res_true": r["rel_res_true"],
                              "setup_s": round(ts, 3),
                              "rel_diff_to_sync": float(torch.linalg.norm(xo - x) / torch.linalg.norm(x))}
            log(f"{name}: {variants[name]}")
            so.close()

    batched = None if args.no_batched else batched_bench(omg, synth, torch)

    cpu = cpu_full = None
    if not args.no_cpu:
        cpu = cpu_baseline(prob, nu, b_host, rep["iters_fine"])
        log(f"cpu: {cpu}")
        cpu_full = cpu_full_solve(omg, synth, torch)
        log(f"cpu full solve: {cpu_full}")
    sweep = cycle_sweep(omg, synth, torch) if args.cycle_sweep else None

    out = {
        "metric": "DOF/s solved to rel. residual 1e-10 (FP64 vs mixed); SpMV/smoother HBM GB/s",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"SIP-DG Poisson {args.n}^3 cells P{args.p} ({prob.n_dofs} DOFs), sphere r=0.3 "
                               f"nu 1:1000, N(0,1) rhs seed 0, {prob.n_levels}-level OrthoMG Alg. 2, 2+2 "
                               f"block-Jacobi omega 0.7, dense Cholesky coarsest, tol 1e-10",
                   "iters_fine": rep["iters_fine"], "n_dirs_fine": rep["n_dirs_fine"],
                   "rel_res_true": rep["rel_res_true"], "setup_s": round(t_setup, 3),
                   "wall_s": round(wall, 3)},
        "hbm_kernels": hbm_kernels,
        "mixed": mixed,
        "table1_variants": variants,
        "batched": batched,
        "roofline": roof,
        "kernel_ms_per_solve": breakdown,
        "rm_configurations": {f"L{l}": {"config": list(s.level_tuning(l)[1]), "tuner_dropped": s.rm_dropped(l)}
                              for l in range(prob.n_levels - 1)},
        "cpu_baseline": cpu,
        "cpu_full_solve": cpu_full,
        "cycle_sweep": sweep,
    }
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
