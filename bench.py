"""Benchmark: PCG+BDDC solves per second on one MI355X.

A solve runs from vb_setup entry (the subdomain matrices already resident in
device memory) through PCG to a 1e-8 relative residual and the interior
recovery of every subdomain.  The default workload (synthetic, seeded) is the
48^3 jittered-cube configuration: divergence-free VEM k=2, nu=1, 216
subdomains of uneven size (cuts at seeded random positions, 4-12 elements
per side), vertex + edge + face primal constraints, deluxe scaling.
By default both paths are timed: FP64, and mixed (FP32 local factors with
FP64 refinement); `value` is the mixed one, and the mixed solution's FP64
interface residual is checked on the FP64 operator.  Each path also reports
warm solves/s (the setup reused: PCG or refinement and recovery only).

Prints one JSON line: the metric, value (mixed solves/s), the per-path runs,
the speedup over the FP64 path, the accuracy of the mixed solution, the
roofline of the dominant kernel (the FP32 rank-1024 trailing update of the
local Dirichlet factorisations, HIP-event timed) and of the Schur GEMV, the
local condensation's flops (dense as executed, and a sparse LU estimate) and
the oracle's CPU baseline.  The timed solves run as in production (per-launch
timing off, the PCG iteration replayed as a HIP graph); the kernel figures
come from one more solve with per-launch HIP-event timing, outside the timed
region.  `--config c1|c2|c4|c4l|c5s|deg2|deg3|deg4` select the other workloads.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    "c2": "32^3 jittered cube (0.15h), VEM k=2, nu=1, 4x4x4 subdomains, vertex+edge+face, deluxe",
    "c1": "8^3 cube, VEM k=2, nu=1, 2x2x2 subdomains, vertex+edge+flux, deluxe",
    "c3": "48^3 jittered cube (0.15h), VEM k=2, nu=1, 216 uneven subdomains (cuts at seeded "
          "random positions, 4-12 elements per side), vertex+edge+face, deluxe",
    "c4": "32^3 cube, VEM k=2, 8 spherical sinkers (radius 0.1, centres seed 0) with nu=1e4 "
          "inside and 1 outside, 4x4x4 subdomains, vertex+edge+face, deluxe, adaptive face "
          "constraints theta=10 through the learned predictor (trained on the exact eigensolves "
          "of sinker seeds 1, 2), FP64",
    "c4l": "36^3 cube, VEM k=2, 8 spherical sinkers (radius 0.1, centres seed 0) with nu=1e4 "
           "inside and 1 outside, 3x3x3 subdomains of 12^3 elements (faces of about 1,500 dual "
           "coordinates), vertex+edge+face, deluxe, adaptive face constraints theta=10 through "
           "the learned predictor (trained on the exact eigensolves of sinker seeds 1, 2), FP64",
    "c5": "32 independent problems, each 24^3 jittered cube (0.15h, one mesh), VEM k=3, 3x3x3 "
          "subdomains of 8^3 elements, nu per subdomain log-uniform in [1e-3, 1e3] (seed = "
          "problem), vertex+edge+face, deluxe, adaptive theta=10 through the learned predictor, "
          "mixed precision; element matrices on the GPU, run in waves of problems per context",
    "c5s": "32 independent problems in one context, each 12^3 jittered cube (0.15h, one mesh), "
           "VEM k=3, 3x3x3 subdomains, nu per subdomain log-uniform in [1e-3, 1e3] (seed = "
           "problem), vertex+edge+face, deluxe, adaptive theta=10 through the learned predictor, "
           "mixed precision",
}
for _k in (2, 3, 4):
    WORKLOADS["deg%d" % _k] = ("8^3 cube, VEM k=%d, nu=1, 4x4x2 subdomains, vertex+edge+flux, deluxe "
                               "(the paper's degree test, Table optDeg1 setting)" % _k)
C4_TRAIN_SEEDS = (1, 2)
C5S_PROBLEMS = 32
C5S_TRAIN_SEEDS = (100, 101)
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by the readings of a 1 GiB device copy: x2.0, x1.0), per
# workload, path and the outer super-panel the autotuner chose for the local
# Dirichlet factorisations (the rank of each launch); to be cleared whenever
# the kernel changes.
TRAFFIC_BYTES = {("c3", "mixed", 1024): 5.0144e10}
TRAFFIC_SOURCE = "profiles/ldl_update_wide_f32_c3_hbm_counters.md"
PRECISION_NAMES = {"fp64": "fp64",
                   "mixed": "mixed: fp32 local factors and Schur operators, fp64 refinement"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def ldl_roofline(ldl, peak, dtype, rank, traffic=None, source=None):
    """Achieved rate of the timed Dirichlet trailing-update launches
    (vb_kernel_stats 0: algorithmic flops and HIP-event durations)."""
    a = ldl["work"] / (ldl["total_ms"] * 1e-3) / 1e12 if ldl["total_ms"] > 0 else None
    return {"bound": "mfma",
            "kernel": "k_ldl_update_wide_%s (rank-%d trailing update of the local "
                      "Dirichlet LDL^T)" % (dtype, rank),
            "achieved": a, "peak": peak, "unit": "TFLOP/s", "frac": (a / peak) if a else None,
            "traffic": traffic, "traffic_source": source,
            "launches": ldl["launches"], "avg_launch_ms": ldl["total_ms"] / max(ldl["launches"], 1)}


def dense_condensation_flops(wl):
    """Flops a dense right-looking LDL^T executes to condense every
    subdomain's interior unknowns (interior velocities and the n_el - 1
    mean-free pressures, e in all) onto its n_Gamma interface unknowns
    (eqs. uipi, firstSchur), m = e + n_Gamma: per eliminated column with t
    rows left (pivot included), t - 1 to scale the column by the pivot and
    t (t - 1) for the rank-1 update of the trailing lower triangle, t^2 - 1
    in all, for t from m - e + 1 to m."""
    tot = 0
    for sd in wl["subs"]:
        kind = np.asarray(sd["kind"])
        e = int(np.sum(kind == 0)) + int(np.sum(kind == 2)) - 1
        m = e + int(np.sum(kind == 1))
        s2 = lambda n: n * (n + 1) * (2 * n + 1) // 6
        tot += (s2(m) - s2(m - e)) - e
    return float(tot)


def _tri_count(m, e):
    """sum of t^2 - 1 for t = m - e + 1 .. m (see dense_condensation_flops)."""
    s2 = lambda n: n * (n + 1) * (2 * n + 1) // 6
    return (s2(m) - s2(m - e)) - e


def nested_condensation_flops(wl):
    """Flops the two-level factorisation executes, counted like
    dense_condensation_flops: per sub-box front (its e interior velocities
    and pressures but one eliminated, m = e + 1 + |B| rows: the kept
    pressure and the separator and interface DoFs it couples to), then per
    subdomain the second level (separator velocities and sub-box constants
    but one eliminated, onto the interface DoFs).  None without sub-box
    labels."""
    import scipy.sparse as sp
    tot = 0
    for sd in wl["subs"]:
        if sd.get("part") is None:
            return None
        kind, part = np.asarray(sd["kind"]), np.asarray(sd["part"])
        n = len(kind)
        K = sp.csr_matrix((np.ones(len(sd["indices"])), sd["indices"], sd["indptr"]), shape=(n, n))
        elim = (kind != 1) & (part >= 0)
        nbox = int(part.max()) + 1
        for b in range(nbox):
            rows = np.nonzero(elim & (part == b))[0]
            cols = np.unique(K[rows].indices)
            nB = int(np.sum(~elim[cols]))
            e = len(rows) - 1
            tot += _tri_count(e + 1 + nB, e)
        e2 = int(np.sum((kind == 0) & (part < 0))) + nbox - 1
        tot += _tri_count(e2 + int(np.sum(kind == 1)), e2)
    return float(tot)


def sparse_lu_flops(lu):
    """Flops of a sparse LU factorisation from its factors' structure:
    sum over pivots of 2 (c_j - 1)(r_j - 1) + (c_j - 1), c_j and r_j the
    entries of column j of L and row j of U (diagonal included)."""
    c = np.diff(lu.L.tocsc().indptr).astype(np.float64)
    r = np.bincount(lu.U.tocsc().indices, minlength=lu.shape[0]).astype(np.float64)
    return float(np.sum(2.0 * (c - 1.0) * (r - 1.0) + (c - 1.0)))


def setup_flops(wl, sparse_sample, setup_ms):
    """The local condensation's work counted three ways: what the two-level
    factorisation executes (when the workload carries sub-box labels), what
    one dense factorisation per subdomain would execute, and the LU flops of
    the oracle's sparse factorisation of the interior matrices (fill-reducing
    COLAMD ordering; sampled subdomains scaled to all, halved for the
    symmetric factorisation it stands for; the dense Schur complement itself
    not included), each per second of the measured setup."""
    try:
        dense = dense_condensation_flops(wl)
        nested = nested_condensation_flops(wl)
        per_s = lambda f: f / (setup_ms * 1e-3) / 1e12 if (setup_ms and f) else None
        out = {"nested_executed": nested, "nested_tflops_per_setup_s": per_s(nested),
               "dense_single_level": dense, "dense_tflops_per_setup_s": per_s(dense),
               "sparse_factor_est": None, "sparse_tflops_per_setup_s": None, "sparse_sample": None}
        if sparse_sample:
            nsub = len(wl["subs"])
            sp_f = 0.5 * float(np.mean(sparse_sample)) * nsub
            out.update(sparse_factor_est=sp_f,
                       sparse_tflops_per_setup_s=sp_f / (setup_ms * 1e-3) / 1e12 if setup_ms else None,
                       sparse_sample="SuperLU (COLAMD) factors of %d of %d subdomains' interior "
                                     "matrices (each scaled to a subdomain of mean n_I^2), mean "
                                     "scaled x%d, halved" % (len(sparse_sample), nsub, nsub))
        return out
    except Exception as ex:  # a report field only: never fail the bench line
        log("setup flop model skipped: %r" % (ex,))
        return None


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(wl, budget_s=20.0):
    """The oracle on a time-bounded sample of the benchmark's own workload:
    its local Schur complements (sparse LU of the Dirichlet problem and one
    solve per interface column: the dominant part of its setup) on the
    subdomains of smallest cost proxy p = n_I^(4/3) n_Gamma (n_I interior
    unknowns: sparse-factor solves of fill ~ n_I^(4/3), one per interface
    column) until `budget_s` seconds have passed (at least one), scaled to
    all subdomains by the ratio sum_all p / sum_sampled p.  The oracle's
    coarse, scaling, PCG and recovery work is left out, so the solves/s it
    implies is an upper bound for the oracle."""
    from oracle.bddc import LocalSchur
    nsub = len(wl["subs"])
    proxy = []
    for sd in wl["subs"]:
        kind = np.asarray(sd["kind"])
        n_i = float(np.sum(kind != 1))
        proxy.append(n_i ** (4.0 / 3.0) * float(np.sum(kind == 1)))
    proxy = np.array(proxy)
    order = np.argsort(proxy, kind="stable")
    t0 = time.perf_counter()
    times, lus, done = [], [], []
    for s in order:
        t1 = time.perf_counter()
        lus.append(LocalSchur(wl["subs"][int(s)]).lu)
        times.append(time.perf_counter() - t1)
        done.append(int(s))
        if time.perf_counter() - t0 > budget_s:
            break
    est = sum(times) / proxy[done].sum() * proxy.sum()
    try:
        sparse = [sparse_lu_flops(lu) for lu in lus]
    except Exception as ex:
        log("sparse flop count skipped: %r" % (ex,))
        sparse = None
    return {"value": 1.0 / est, "unit": "solves/s", "cores": int(_blas_threads()),
            "_sparse_flops": sparse, "_sampled": done,
            "kind": "oracle",
            "sample": "local Schur complements (sparse LU, one solve per interface column) of "
                      "the %d of %d subdomains of smallest cost proxy n_I^(4/3) n_Gamma "
                      "(%.1f s of CPU work), scaled to all by the proxy (%.0f s estimated); the "
                      "oracle's coarse, scaling, PCG and recovery work is not included (its full "
                      "solve is timed at c1 in oracle_full_c1)" % (len(times), nsub, sum(times), est)}


def oracle_full_c1():
    """The whole oracle (setup, PCG to 1e-8, interior recovery) on the 8^3
    workload c1, timed by phase on the host cores."""
    from inputs.workloads import make_workload
    from oracle.bddc import OracleBDDC
    from oracle.pcg import pcg
    wl, _ = make_workload("c1")
    t0 = time.perf_counter()
    o = OracleBDDC(wl)
    t1 = time.perf_counter()
    x, info = pcg(o.apply_S, o.apply_M, o.rhs(), tol=1e-8)
    t2 = time.perf_counter()
    for i, L in enumerate(o.loc):
        L.recover(x[L.gid], x[o.nG + i])
    t3 = time.perf_counter()
    return {"workload": "c1: " + WORKLOADS["c1"], "setup_s": t1 - t0, "pcg_s": t2 - t1,
            "recovery_s": t3 - t2, "iterations": int(info["iters"]),
            "solves_per_s": 1.0 / (t3 - t0), "cores": int(_blas_threads())}


def vem_assembly(vb, config, stream, dev):
    """The workload's element matrices (A^K, B^K, F^K of every element of its
    mesh) by vb_vem_element_matrices, timed on the GPU (second of two calls),
    beside the host generator's element computation on a 256-element sample
    (one process), scaled to all elements."""
    import torch
    from inputs.workloads import RECIPES
    from inputs.mesh import CubeMesh
    from inputs.vem import element_matrices
    r = RECIPES[config]
    mesh = CubeMesh(r["n"], jitter=r["jitter"], seed=0)
    k, E = r["k"], mesh.nK
    N, nP = vb.vb_vem_dofs(k)
    X8 = torch.tensor(np.ascontiguousarray(mesh.verts[mesh.elem_verts].reshape(E, 24)), device=dev)
    A = torch.empty((E, N, N), dtype=torch.float64, device=dev)
    B = torch.empty((E, nP, N), dtype=torch.float64, device=dev)
    F = torch.empty((E, N), dtype=torch.float64, device=dev)
    ctx = vb.vb_create(stream=stream.cuda_stream)
    try:
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vb.vb_vem_element_matrices(ctx, k, X8, None, A, B, F)
            times.append(time.perf_counter() - t0)
    finally:
        vb.vb_destroy(ctx)
    del A, B, F, X8
    torch.cuda.empty_cache()
    el = np.arange(min(E, 256))
    t0 = time.perf_counter()
    element_matrices(mesh, k, el, 1.0)
    th = (time.perf_counter() - t0) / len(el)
    return {"elements": int(E), "k": int(k), "dofs_per_element": int(N), "gpu_s": times[-1],
            "host_s_per_element": th, "host_estimate_s": th * E,
            "note": "A^K, B^K and F^K of every element on the GPU; the host figure is the "
                    "generator's element computation (one process) on 256 elements, scaled"}


def time_path(vb, wl, prec, steps, warmup, warm_steps, stream, dev, nloc):
    """Create a context for one precision, then time `steps` solves (after
    `warmup` untimed ones) with per-launch timing off, so that the PCG
    iteration replays its HIP graph as in production; then `warm_steps`
    solves with the setup reused; then one more solve with per-launch HIP
    event timing on, for the kernels' roofline figures."""
    import torch
    code = vb.VB_PREC_FP64 if prec == "fp64" else vb.VB_PREC_MIXED
    ctx = vb.vb_create(precision=code, tol=1e-8, stream=stream.cuda_stream, profile=0)
    vb.vb_assemble(ctx, wl)
    n = vb.vb_interface_size(ctx)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    u = torch.zeros(nloc, dtype=torch.float64, device=dev)

    def solve():
        vb.vb_setup(ctx)
        x.zero_()
        info = vb.vb_pcg_solve(ctx, x)
        vb.vb_recover_all(ctx, x, u)
        return info

    with torch.cuda.stream(stream):
        for w in range(warmup):
            info = solve()
            stream.synchronize()
            log("%s warmup %d: %d iterations (%d refinement steps), setup %.1f ms, solve %.1f ms"
                % (prec, w, info["iterations"], info["refinement_steps"], info["setup_ms"],
                   info["solve_ms"]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [solve() for _ in range(steps)]
        stream.synchronize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        last = infos[-1]
        log("%s: timed %d solves in %.3f s: %d iterations, residual %.2e"
            % (prec, steps, dt, last["iterations"], last["true_rel_residual"]))
        launch = {vb.VB_PCG_GRAPH: "graph", vb.VB_PCG_PERSISTENT: "persistent"}.get(
            vb.vb_pcg_launch_used(ctx), "eager")
        sym = vb.vb_tuned_tile(ctx, 4) == 1
        phases = vb.vb_setup_phases(ctx)
        tuned = {"gemv_columns_per_workgroup": [vb.vb_tuned_tile(ctx, w) for w in range(4)],
                 "symmetric_kernels": [vb.vb_tuned_tile(ctx, w) for w in (4, 5)],
                 "factor_panel": [vb.vb_tuned_tile(ctx, w) for w in (6, 7, 8)],
                 "factor_superpanel": [vb.vb_tuned_tile(ctx, w) for w in (9, 10, 11)]}
        # warm solves: the setup reused, PCG (or refinement) + recovery only
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k in range(warm_steps):
            x.zero_()
            vb.vb_pcg_solve(ctx, x)
            vb.vb_recover_all(ctx, x, u)
        stream.synchronize()
        torch.cuda.synchronize()
        dtw = time.perf_counter() - t2
        # profiled pass (outside the timed region)
        vb.vb_set_profile(ctx, 1)
        vb.vb_kernel_stats(ctx, 0, reset=True)
        vb.vb_kernel_stats(ctx, 1, reset=True)
        solve()
        stream.synchronize()
        ldl = vb.vb_kernel_stats(ctx, 0)
        gmv = vb.vb_kernel_stats(ctx, 1)
        vb.vb_set_profile(ctx, 0)
        x.zero_()
        solve()  # leave x as the solution of a production-mode solve
        stream.synchronize()
        history = vb.vb_refinement_history(ctx) if prec != "fp64" else None
    del u
    return dict(ctx=ctx, x=x, dt=dt, steps=steps, warmup=warmup, ldl=ldl, gmv=gmv, info=last,
                dtw=dtw, warm_steps=warm_steps, launch=launch, sym=sym, tuned=tuned, phases=phases,
                history=history)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--cache", default=None, help="workload .npz (generated if missing)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-vem", action="store_true",
                    help="skip the GPU element-matrix timing (outside the timed region)")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of oracle work in the CPU baseline's sample")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"],
                    help="both: time the FP64 path and the mixed path; value = mixed")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed solves of the FP64 comparison path when both are timed "
                         "(its warm-up: at most one solve)")
    ap.add_argument("--warm-steps", type=int, default=3,
                    help="solves with the setup reused, per path")
    ap.add_argument("--prepare-only", action="store_true",
                    help="generate and store the workload (--cache) and exit")
    ap.add_argument("--no-sequential", action="store_true",
                    help="c5s: skip the one-context-per-problem comparison")
    ap.add_argument("--c5-wave", type=int, default=4,
                    help="c5: problems per context (the 32 problems run in waves)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy a 1 GiB device buffer three times and exit (reference for the "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_launch": a.numel() * 4,
                          "bytes_written_per_launch": a.numel() * 4, "launches": 3}), flush=True)
        return
    if args.config == "c5s":
        return run_batched(args)
    if args.config == "c5":
        return run_c5(args)
    if args.config in ("c4", "c4l"):
        return run_adaptive(args)
    # ---- workload (before any GPU initialisation)
    from inputs.workloads import make_workload, save_workload, load_workload
    t = time.perf_counter()
    t_ass = None  # seconds to generate the workload (mesh, VEM assembly, decomposition)
    if args.cache and os.path.exists(args.cache):
        wl = load_workload(args.cache)
        log("loaded workload %s (%.1f s)" % (args.cache, time.perf_counter() - t))
    else:
        t00 = time.perf_counter()
        wl, _ = make_workload(args.config, workers=min(16, os.cpu_count() or 1),
                              progress=lambda m: log("workload %s: %s (%.0f s)"
                                                     % (args.config, m, time.perf_counter() - t00)))
        t_ass = time.perf_counter() - t
        log("generated workload %s (%.1f s)" % (args.config, t_ass))
        if args.cache:
            save_workload(args.cache, wl)
    if args.prepare_only:
        return
    nsub = len(wl["subs"])
    # ---- CPU baseline (oracle, bounded sample of this workload; full at c1)
    cpu, sparse_flops, full_c1 = None, None, None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_budget)
        sparse_flops = cpu.pop("_sparse_flops")
        sampled = cpu.pop("_sampled")
        if sparse_flops:  # per sampled subdomain, scaled to a subdomain of mean n_I^2
            n_i2 = np.array([float(np.sum(np.asarray(sd["kind"]) != 1)) ** 2 for sd in wl["subs"]])
            sparse_flops = [f * n_i2.mean() / n_i2[k] for f, k in zip(sparse_flops, sampled)]
        log("cpu baseline: %s" % cpu["sample"])
        full_c1 = oracle_full_c1()
        log("oracle in full at c1: %s" % full_c1)
    # ---- GPU
    import torch
    from paper_2304_09770_amd import binding as vb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    nloc = sum(len(sd["kind"]) for sd in wl["subs"])
    runs = {}
    # mixed first: each context is destroyed after its run except the FP64
    # one, kept for the accuracy check of the mixed solution (both do not
    # fit in memory at once at the largest workloads)
    order = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    for prec in order:
        comparison = args.precision == "both" and prec == "fp64"
        steps = min(args.steps, args.fp64_steps) if comparison else args.steps
        warmup = min(args.warmup, 1) if comparison else args.warmup
        runs[prec] = time_path(vb, wl, prec, steps, warmup, args.warm_steps, stream, dev, nloc)
        if prec != "fp64":
            vb.vb_destroy(runs[prec]["ctx"])
            runs[prec]["ctx"] = None
            torch.cuda.empty_cache()
    n = vb.vb_interface_size(runs[order[-1]]["ctx"]) if runs[order[-1]]["ctx"] else None
    # ---- accuracy of the mixed solution against the FP64 operator and solution
    check = {}
    if "mixed" in runs and "fp64" in runs:
        c64 = runs["fp64"]["ctx"]
        xm, x64 = runs["mixed"]["x"], runs["fp64"]["x"]
        g = torch.zeros(n, dtype=torch.float64, device=dev)
        y = torch.zeros(n, dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            vb.vb_rhs(c64, g)
            vb.vb_schur_apply(c64, xm, y)
        stream.synchronize()
        check = {"fp64_interface_rel_residual": float(torch.linalg.norm(g - y) / torch.linalg.norm(g)),
                 "rel_diff_vs_fp64_solution": float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))}
        log("mixed vs fp64: %s" % check)
        assert check["fp64_interface_rel_residual"] <= 1e-8 * 1.01, check
    for r in runs.values():
        if r["ctx"] is not None:
            vb.vb_destroy(r["ctx"])
    torch.cuda.empty_cache()
    vem = None
    if not args.no_vem:
        vem = vem_assembly(vb, args.config, stream, dev)
        log("element matrices of %d elements on the GPU: %.3f s (host generator: %.1f s estimated)"
            % (vem["elements"], vem["gpu_s"], vem["host_estimate_s"]))
    head = "mixed" if "mixed" in runs else "fp64"
    R = runs[head]
    if head == "fp64":
        assert R["info"]["true_rel_residual"] <= 1e-8 * 1.01, R["info"]
    peak = PEAK_FP64_TFLOPS if head == "fp64" else PEAK_FP32_TFLOPS

    def roof(r, pk, dtype, prec):
        rank = r["tuned"]["factor_superpanel"][0]
        key = (args.config, prec, rank)
        return ldl_roofline(r["ldl"], pk, dtype, rank, TRAFFIC_BYTES.get(key),
                            TRAFFIC_SOURCE if key in TRAFFIC_BYTES else None)

    def gemv(r):
        g = r["gmv"]
        b = g["work"] / (g["total_ms"] * 1e-3) / 1e9 if g["total_ms"] > 0 else None
        name = ("k_symv_tiles + k_symv_reduce (S_hat p through the lower triangle of each "
                "bordered local Schur operator)") if r["sym"] else \
            "k_gemv_t (S_hat p, bordered local Schur GEMV)"
        return {"kernel": name, "bound": "hbm",
                "achieved": b, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": (b / PEAK_HBM_GBS) if b else None, "launches": g["launches"],
                "avg_launch_ms": g["total_ms"] / max(g["launches"], 1)}

    def summary(r):
        i = r["info"]
        return {"solves_per_s": r["steps"] / r["dt"], "ms_per_step": 1e3 * r["dt"] / r["steps"],
                "steps": r["steps"], "warmup": r["warmup"],
                "warm_solves_per_s": (r["warm_steps"] / r["dtw"]) if r["warm_steps"] else None,
                "warm_steps": r["warm_steps"], "pcg_launch": r["launch"], "autotuned": r["tuned"],
                "setup_phases_ms": r["phases"],
                "iterations": i["iterations"], "refinement_steps": i["refinement_steps"],
                "rel_residual": i["true_rel_residual"], "lambda_min": i["lambda_min"],
                "lambda_max": i["lambda_max"],
                "k2": (i["lambda_max"] / i["lambda_min"]) if i["lambda_min"] > 0 else None,
                "n_coarse": i["n_coarse"], "setup_ms": i["setup_ms"], "solve_ms": i["solve_ms"],
                "refinement_history": ({"rel_residual_before_step": r["history"][0],
                                        "inner_iterations": r["history"][1]}
                                       if r["history"] else None)}

    out = {
        "metric": "PCG+BDDC solves/s at 1e-8 rel. residual, mixed/batched vs FP64 GPU",
        "value": args.steps / R["dt"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * R["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.config + ": " + WORKLOADS[args.config],
                   "precision": PRECISION_NAMES[head], "subdomains": nsub,
                   "interface_unknowns": n,
                   "timed_mode": "per-launch timing off, PCG iterations launched as: %s "
                                 "(persistent: one cooperative launch per inner solve; graph: one "
                                 "captured iteration replayed); kernel figures from one extra "
                                 "profiled solve (launch by launch)" % R["launch"]},
        "roofline": roof(R, peak, "f64" if head == "fp64" else "f32", head),
        "iteration_kernel": gemv(R),
        "runs": {k: summary(v) for k, v in runs.items()},
        "speedup_vs_fp64": ((runs["fp64"]["dt"] / runs["fp64"]["steps"]) /
                            (runs["mixed"]["dt"] / runs["mixed"]["steps"])) if len(runs) == 2 else None,
        "mixed_accuracy": check or None,
        "roofline_fp64": roof(runs["fp64"], PEAK_FP64_TFLOPS, "f64", "fp64") if "fp64" in runs else None,
        "setup_flops": setup_flops(wl, sparse_flops, R["info"]["setup_ms"]),
        "outside_timed_region": {"workload_generation_s": t_ass,
                                 "note": "mesh, VEM assembly and decomposition on the host "
                                         "(the paper's T_ass analogue) and vb_assemble's "
                                         "host copies are not in the timed solves",
                                 "vem_element_matrices": vem},
        "cpu_baseline": cpu,
        "oracle_full_c1": full_c1,
    }
    print(json.dumps(out), flush=True)


def run_adaptive(args):
    """C4 (and c4l: the same sinkers with 12^3-element subdomains): the
    adaptive coarse space through the learned predictor against the exact
    adaptive space and the minimal primal space (the plain FP64 GPU method),
    all FP64 (the contrast of 1e4 inside subdomains)."""
    from inputs.workloads import make_workload, mlp_init_params
    t = time.perf_counter()
    nw = min(16, os.cpu_count() or 1)
    cfg = args.config
    wl, _ = make_workload(cfg, seed=0, workers=nw)
    train = [make_workload(cfg, seed=sd, workers=nw)[0] for sd in C4_TRAIN_SEEDS]
    log("generated %s and %d training workloads (%.1f s)" % (cfg, len(train), time.perf_counter() - t))
    import torch
    from paper_2304_09770_amd import binding as vb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    theta = 10.0
    m = vb.vb_mlp_create(mlp_init_params(12, 32, 7), stream.cuda_stream)
    with torch.cuda.stream(stream):
        for w in train:
            c = vb.vb_create(adaptive_theta=theta, stream=stream.cuda_stream)
            vb.vb_assemble(c, w)
            vb.vb_setup(c)
            vb.vb_mlp_add_samples(m, c)
            vb.vb_destroy(c)
        hist = vb.vb_mlp_train(m, 1500, 3e-3)
    log("predictor: %d samples, loss %.3e -> %.3e" % (vb.vb_mlp_num_samples(m), hist[0], hist[-1]))
    nloc = sum(len(sd["kind"]) for sd in wl["subs"])
    spaces = [("minimal", {}), ("exact", dict(adaptive_theta=theta)),
              ("learned", dict(adaptive_theta=theta, predictor=m))]
    runs, xs = {}, {}
    with torch.cuda.stream(stream):
        for name, kw in spaces:
            ctx = vb.vb_create(tol=1e-8, stream=stream.cuda_stream, profile=0, **kw)
            vb.vb_assemble(ctx, wl)
            n = vb.vb_interface_size(ctx)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            u = torch.zeros(nloc, dtype=torch.float64, device=dev)

            def solve():
                t0 = time.perf_counter()
                vb.vb_setup(ctx)
                stream.synchronize()
                t1 = time.perf_counter()
                x.zero_()
                info = vb.vb_pcg_solve(ctx, x)
                stream.synchronize()
                t2 = time.perf_counter()
                vb.vb_recover_all(ctx, x, u)
                stream.synchronize()
                log("%s step: setup %.3f s (device %.1f ms), solve %.3f s, recovery %.3f s"
                    % (name, t1 - t0, info["setup_ms"], t2 - t1, time.perf_counter() - t2))
                return info

            for _ in range(args.warmup):
                solve()
            stream.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                info = solve()
            stream.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            faces = vb.vb_adaptive_info(ctx) if kw else []
            # one profiled solve (per-launch HIP events) for the kernel figures
            vb.vb_set_profile(ctx, 1)
            vb.vb_kernel_stats(ctx, 0, reset=True)
            solve()
            vb.vb_set_profile(ctx, 0)
            runs[name] = {"solves_per_s": 1.0 / dt, "ms_per_step": 1e3 * dt,
                          "iterations": info["iterations"],
                          "kappa": info["lambda_max"] / info["lambda_min"],
                          "n_coarse": info["n_coarse"], "rel_residual": info["true_rel_residual"],
                          "setup_ms": info["setup_ms"], "solve_ms": info["solve_ms"],
                          "faces": len(faces),
                          "predicted_path_faces": sum(f["path"] == 1 for f in faces),
                          "fallback_faces": sum(f["path"] == 2 for f in faces),
                          "selected_rows": sum(f["n_selected"] for f in faces)}
            runs[name]["ldl"] = vb.vb_kernel_stats(ctx, 0)
            runs[name]["ldl_rank"] = vb.vb_tuned_tile(ctx, 9)
            xs[name] = x.cpu().numpy()
            log("%s: %.3f solves/s, %d iterations, kappa %.1f, N_c %d"
                % (name, 1.0 / dt, info["iterations"], runs[name]["kappa"], info["n_coarse"]))
            assert info["true_rel_residual"] <= 1e-8 * 1.01, info
            vb.vb_destroy(ctx)
    vb.vb_mlp_destroy(m)
    ldl = runs["learned"].pop("ldl")
    ldl_rank = runs["learned"].pop("ldl_rank")
    for r in runs.values():
        r.pop("ldl", None)
        r.pop("ldl_rank", None)
    ref = xs["exact"]
    out = {
        "metric": "PCG+BDDC solves/s at 1e-8 rel. residual, mixed/batched vs FP64 GPU",
        "value": runs["learned"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": runs["learned"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg + ": " + WORKLOADS[cfg], "subdomains": len(wl["subs"]),
                   "precision": "fp64"},
        "roofline": ldl_roofline(ldl, PEAK_FP64_TFLOPS, "f64", ldl_rank),
        "runs": runs,
        "speedup_vs_fp64": runs["learned"]["solves_per_s"] / runs["minimal"]["solves_per_s"],
        "speedup_vs_exact_adaptive": runs["learned"]["solves_per_s"] / runs["exact"]["solves_per_s"],
        "rel_diff_learned_vs_exact_solution": float(np.linalg.norm(xs["learned"] - ref) /
                                                    np.linalg.norm(ref)),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_c5(args):
    """C5 at its stated size: 32 problems of 24^3, k = 3, 27 subdomains each.
    The element matrices of the shared mesh come from the GPU (unit
    viscosity; outside the timed region, like the rest of the generation),
    the host decomposes once and scales each problem's subdomains by their
    viscosity.  The problems run in waves of --c5-wave problems per context
    (all 32 do not fit one GPU's memory at once): per wave one untimed solve,
    then one timed (setup, PCG, recovery of every problem of the wave).
    value = 32 / the sum of the timed waves."""
    import torch
    from paper_2304_09770_amd import binding as vb
    from inputs.workloads import RECIPES, scaled_family, mlp_init_params
    from inputs.mesh import CubeMesh
    from inputs.assemble import Problem
    from inputs.decompose import Decomposition, regular_cuts
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    r = RECIPES["c5"]
    mesh = CubeMesh(r["n"], jitter=r["jitter"], seed=0)
    k, E = r["k"], mesh.nK
    N, nP = vb.vb_vem_dofs(k)
    t0 = time.perf_counter()
    X8 = torch.tensor(np.ascontiguousarray(mesh.verts[mesh.elem_verts].reshape(E, 24)), device=dev)
    A = torch.empty((E, N, N), dtype=torch.float64, device=dev)
    B = torch.empty((E, nP, N), dtype=torch.float64, device=dev)
    F = torch.empty((E, N), dtype=torch.float64, device=dev)
    ctx = vb.vb_create(stream=stream.cuda_stream)
    torch.cuda.synchronize()
    te = time.perf_counter()
    vb.vb_vem_element_matrices(ctx, k, X8, None, A, B, F)
    t_elem = time.perf_counter() - te
    vb.vb_destroy(ctx)
    elem = (A.cpu().numpy(), B.cpu().numpy(), F.cpu().numpy())
    del A, B, F, X8
    torch.cuda.empty_cache()
    log("c5: element matrices of %d elements on the GPU in %.2f s" % (E, t_elem))
    th = time.perf_counter()
    pb = Problem(mesh, k, 1.0, element_data=elem)
    del elem
    dec = Decomposition(pb, regular_cuts(r["n"], r["parts"]), r["cons"])
    base = (dec, dec.workload())
    t_host = time.perf_counter() - th
    log("c5: host assembly and decomposition from them: %.1f s" % t_host)
    theta = 10.0
    m = vb.vb_mlp_create(mlp_init_params(12, 32, 7), stream.cuda_stream)
    with torch.cuda.stream(stream):
        for wl in scaled_family("c5", C5S_TRAIN_SEEDS, base=base):
            c = vb.vb_create(adaptive_theta=theta, stream=stream.cuda_stream, tune_factor=2)
            vb.vb_assemble(c, wl)
            vb.vb_setup(c)
            vb.vb_mlp_add_samples(m, c)
            vb.vb_destroy(c)
        hist = vb.vb_mlp_train(m, 1500, 3e-3)
    log("c5: predictor %d samples, loss %.3e -> %.3e" % (vb.vb_mlp_num_samples(m), hist[0], hist[-1]))
    opts = dict(precision=vb.VB_PREC_MIXED, tol=1e-8, adaptive_theta=theta, predictor=m,
                stream=stream.cuda_stream, profile=0, tune_factor=2)
    seeds = list(range(32))
    P = max(1, args.c5_wave)
    waves, per, lat, faces_pred, faces_fb, mem_used = [], [], [], 0, 0, None
    for w0 in range(0, len(seeds), P):
        wls = list(scaled_family("c5", seeds[w0:w0 + P], base=base))
        with torch.cuda.stream(stream):
            ctx = vb.vb_create(**opts)
            for wl in wls:
                vb.vb_assemble(ctx, wl)
            n = vb.vb_interface_size(ctx)
            nloc = sum(sum(len(sd["kind"]) for sd in wl["subs"]) for wl in wls)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            u = torch.zeros(nloc, dtype=torch.float64, device=dev)
            for step in range(2):  # untimed, then timed
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                vb.vb_setup(ctx)
                x.zero_()
                vb.vb_pcg_solve(ctx, x)
                vb.vb_recover_all(ctx, x, u)
                stream.synchronize()
                dt = time.perf_counter() - t1
            waves.append(dt)
            if w0 == 0:
                free, total = torch.cuda.mem_get_info()
                log("c5: device memory in use with a wave's context: %.1f of %.1f GB"
                    % ((total - free) / 1e9, total / 1e9))
                mem_used = (total - free) / 1e9
            for q in range(len(wls)):
                pi = vb.vb_problem_solve_info(ctx, q)
                per.append(pi)
                lat.append(pi["latency_ms"])
            fc = vb.vb_adaptive_info(ctx)
            faces_pred += sum(f["path"] == 1 for f in fc)
            faces_fb += sum(f["path"] == 2 for f in fc)
            vb.vb_destroy(ctx)
            del x, u
            torch.cuda.empty_cache()
        log("c5: wave of %d problems: %.3f s (setup + PCG + recovery)" % (len(wls), dt))
    vb.vb_mlp_destroy(m)
    res = max(p["true_rel_residual"] for p in per)
    assert all(p["status"] == 0 for p in per), per
    assert res <= 1e-8 * 1.01, res
    total = sum(waves)
    lat = np.array(lat)
    out = {
        "metric": "PCG+BDDC solves/s at 1e-8 rel. residual, mixed/batched vs FP64 GPU",
        "value": len(seeds) / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1e3 * total,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "c5: " + WORKLOADS["c5"], "problems": len(seeds),
                   "problems_per_context": P, "precision": PRECISION_NAMES["mixed"],
                   "device_memory_gb_per_wave": mem_used},
        "waves_s": waves,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max()), "note": "from the start of the wave's solve"},
        "inner_iterations": {"min": int(min(p["iterations"] for p in per)),
                             "max": int(max(p["iterations"] for p in per))},
        "refinement_steps_max": max(p["refinement_steps"] for p in per),
        "max_rel_residual": res,
        "predicted_path_faces": int(faces_pred),
        "fallback_faces": int(faces_fb),
        "outside_timed_region": {"element_matrices_gpu_s": t_elem, "elements": int(E),
                                 "host_assembly_and_decomposition_s": t_host},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_batched(args):
    """Several independent problems in one context against one context per
    problem: aggregate solves/s and per-problem latency (device clock from the
    start of the batched solve to each problem's convergence)."""
    from inputs.workloads import make_family, mlp_init_params
    t = time.perf_counter()
    fam = make_family("c5s", list(C5S_TRAIN_SEEDS) + list(range(C5S_PROBLEMS)),
                      workers=min(16, os.cpu_count() or 1))
    train, batch = fam[:len(C5S_TRAIN_SEEDS)], fam[len(C5S_TRAIN_SEEDS):]
    log("generated %d problems (%.1f s)" % (len(fam), time.perf_counter() - t))
    import torch
    from paper_2304_09770_amd import binding as vb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    theta = 10.0
    # predictor trained on the exact eigensolves of two other problems
    m = vb.vb_mlp_create(mlp_init_params(12, 32, 7), stream.cuda_stream)
    with torch.cuda.stream(stream):
        for wl in train:
            c = vb.vb_create(adaptive_theta=theta, stream=stream.cuda_stream)
            vb.vb_assemble(c, wl)
            vb.vb_setup(c)
            vb.vb_mlp_add_samples(m, c)
            vb.vb_destroy(c)
        hist = vb.vb_mlp_train(m, 1500, 3e-3)
    log("predictor: %d samples, loss %.3e -> %.3e" % (vb.vb_mlp_num_samples(m), hist[0], hist[-1]))
    opts = dict(precision=vb.VB_PREC_MIXED, tol=1e-8, adaptive_theta=theta, predictor=m,
                stream=stream.cuda_stream, profile=0)

    def run(ctx, steps):
        n = vb.vb_interface_size(ctx)
        nloc = sum(sum(len(sd["kind"]) for sd in w["subs"]) for w in ctx_wls[id(ctx)])
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        u = torch.zeros(nloc, dtype=torch.float64, device=dev)
        info = None
        for _ in range(steps):
            t0 = time.perf_counter()
            vb.vb_setup(ctx)
            stream.synchronize()
            t1 = time.perf_counter()
            x.zero_()
            info = vb.vb_pcg_solve(ctx, x)
            stream.synchronize()
            t2 = time.perf_counter()
            vb.vb_recover_all(ctx, x, u)
            stream.synchronize()
            t3 = time.perf_counter()
            if len(ctx_wls[id(ctx)]) > 1:
                log("batch step: setup %.3f s (device %.1f ms), solve %.3f s, recovery %.3f s"
                    % (t1 - t0, info["setup_ms"], t2 - t1, t3 - t2))
        stream.synchronize()
        return info

    ctx_wls = {}
    with torch.cuda.stream(stream):
        # batched: all problems in one context
        ctx = vb.vb_create(**opts)
        ctx_wls[id(ctx)] = batch
        for wl in batch:
            vb.vb_assemble(ctx, wl)
        run(ctx, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = run(ctx, args.steps)
        t1 = time.perf_counter()
        per = [vb.vb_problem_solve_info(ctx, k) for k in range(len(batch))]
        # one profiled solve (per-launch HIP events) for the kernel figures
        vb.vb_set_profile(ctx, 1)
        vb.vb_kernel_stats(ctx, 0, reset=True)
        run(ctx, 1)
        ldl = vb.vb_kernel_stats(ctx, 0)
        ldl_rank = vb.vb_tuned_tile(ctx, 9)
        vb.vb_set_profile(ctx, 0)
        faces = vb.vb_adaptive_info(ctx)
        tiles = [vb.vb_tuned_tile(ctx, k) for k in range(5)]
        vb.vb_destroy(ctx)
        dt_batch = (t1 - t0) / args.steps
        # the same batch with the exact adaptive eigensolves (no predictor)
        ex_opts = dict(opts)
        ex_opts["predictor"] = None
        ctx = vb.vb_create(**ex_opts)
        ctx_wls[id(ctx)] = batch
        for wl in batch:
            vb.vb_assemble(ctx, wl)
        run(ctx, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(ctx, args.steps)
        dt_exact = (time.perf_counter() - t0) / args.steps
        vb.vb_destroy(ctx)
        log("exact adaptive batch: %.3f s per step (learned %.3f s)" % (dt_exact, dt_batch))
        # one context per problem, one after the other
        seq = 0.0
        for k, wl in enumerate([] if args.no_sequential else batch):
            c = vb.vb_create(**opts)
            ctx_wls[id(c)] = [wl]
            vb.vb_assemble(c, wl)
            if k == 0:
                run(c, args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(c, 1)
            seq += time.perf_counter() - t0
            vb.vb_destroy(c)
    vb.vb_mlp_destroy(m)
    lat = np.array([p["latency_ms"] for p in per])
    its = np.array([p["iterations"] for p in per])
    res = max(p["true_rel_residual"] for p in per)
    assert all(p["status"] == 0 for p in per), per
    assert res <= 1e-8 * 1.01, res
    out = {
        "metric": "PCG+BDDC solves/s at 1e-8 rel. residual, mixed/batched vs FP64 GPU",
        "value": len(batch) / dt_batch,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "c5s: " + WORKLOADS["c5s"], "problems": len(batch),
                   "precision": PRECISION_NAMES["mixed"]},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "sequential_solves_per_s": (len(batch) / seq) if seq else None,
        "exact_adaptive_solves_per_s": len(batch) / dt_exact,
        "learned_speedup_vs_exact_adaptive": dt_exact / dt_batch,
        "batch_speedup": (seq / dt_batch) if seq else None,
        "inner_iterations": {"min": int(its.min()), "max": int(its.max())},
        "refinement_steps_max": max(p["refinement_steps"] for p in per),
        "max_rel_residual": res,
        "adaptive_faces": len(faces),
        "predicted_path_faces": sum(f["path"] == 1 for f in faces),
        "fallback_faces": sum(f["path"] == 2 for f in faces),
        "gemv_tiles": tiles,
        "roofline": ldl_roofline(ldl, PEAK_FP32_TFLOPS, "f32", ldl_rank),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
