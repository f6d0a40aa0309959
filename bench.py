"""Benchmark of the macro-element HDG hot path on one MI355X.

A step is one pass of the whole hot path over the plain-FP64-at-scale
workload: factor_local (assemble + pivoted LU of every A_K), solve (right-hand
side, then GMRES on the trace system until the relative residual
||f^ - S lam|| / ||f^|| is at most 1e-10, checked exactly at every restart)
and recover_local.  Inputs (mesh metadata, kappa, f and g_D samples) are
resident in HBM before the timed region.

Workload (default): unit square, 64 x 64 squares -> 8192 macro-triangles,
r = 3 (64 sub-triangles each), p = 3, kappa = 1e-2, a = (1, 0.5), tau = 1,
manufactured u = exp(x) sin(2 pi y); N_K = 975, 304,000 trace unknowns.

Prints one JSON line.  `value` is trace-operator applies per second over the
whole timed job (all applies made by the K steps divided by their wall time,
factorisation and orthogonalisation included); the roofline object is for
the dominant kernel, the per-macro streaming solve of the trace operator,
timed live with HIP events on its stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trace-operator applies/s + solve time to 1e-10 res: tuned form vs plain FP64"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: n, r, p, kappa, beta, manufactured solution, factor precision
    "plain_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5), sol="exp_sin",
                                       precision="fp64"),
    # folded form (same mesh and data): T_K = C_K A_K^-1 B_K stored per macro after the LU,
    # GMRES applies read L_K^2 = 75^2 values per macro instead of the 975^2 factors
    # GMRES(40): with cheap applies the Krylov basis work dominates, and restarting
    # at 30-50 columns solves fastest on this mesh (folded full-block factors: 2000,
    # i.e. no restart, 1207 iterations, 2.31 s; 100: 1826, 1.76 s; 50: 1584, 1.67 s;
    # 30: 1572, 1.71 s.  Folded Schur factors: 50: 0.415 s; 40: 1551, 0.399 s;
    # 30: 1572, 0.397 s; 20: 1999, 0.469 s)
    "folded_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                        sol="exp_sin", precision="fp64", form="folded",
                                        restart=40),
    # flux eliminated exactly (same mesh and data): q through the reference mass, only the
    # Q x Q Schur block on u factored and streamed (Q = 325: 8 Q^2 bytes per macro)
    "qelim_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                       sol="exp_sin", precision="qelim"),
    # folded operators built from the Schur-block factors: LU of Q x Q blocks, T_K by
    # many-right-hand-side Schur-block solves, GMRES(50) with folded applies
    "folded_qelim_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                              sol="exp_sin", precision="qelim", form="folded",
                                              restart=40),
    # the matrix-based form (section 6.1): the global trace matrix assembled block-sparse
    # from the operators folded from the Schur-block factors, GMRES(40) on its products
    "assembled_qelim_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                                 sol="exp_sin", precision="qelim",
                                                 form="assembled", restart=40),
    # the boundary-condensed form (same mesh and data): W_K = (A_K^-1)_bb over the 9P = 216
    # boundary unknowns of each macro, built from the FP64 factors; GMRES applies read
    # 8 x 216^2 bytes per macro (3.06 GB) between the factors' 62 GB and T_K's 0.37 GB
    "boundary_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                          sol="exp_sin", precision="fp64", form="boundary",
                                          restart=40),
    # the same blocks built from the flux elimination's Schur-block factors
    "boundary_qelim_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                                sol="exp_sin", precision="qelim",
                                                form="boundary", restart=40),
    # the best tuned form on the uneven-level mesh (instance 0 of the batching configuration)
    "folded_qelim_mixed_r1to4_8192macro_p3_inst0": dict(n=64, r="mixed", p=3, kappa=None,
                                                        beta=None, sol="exp_sin",
                                                        precision="qelim", form="folded",
                                                        instance=0, restart=50),
    # standard HDG (r = 0: every element its own macro, section 3.2's special case) on the
    # same data: 160 x 160 squares give 305,920 trace unknowns, the macro-element job's
    # 304,000 (matched global size); 512 x 512 squares give the macro job's element size
    # (matched resolution, 3.1 million trace unknowns)
    "standard_hdg_160x160_r0_p3": dict(n=160, r=0, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                       sol="exp_sin", precision="fp64"),
    "standard_hdg_512x512_r0_p3": dict(n=512, r=0, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                       sol="exp_sin", precision="fp64", restart=300),
    "plain_fp64_8macro_r1_p2": dict(n=2, r=1, p=2, kappa=1.0, beta=(1.0, 1.0), sol="sin_sin",
                                    precision="fp64"),
    # precision configuration: same mesh, kappa = 1e-3, FP32 factors + FP64 refinement
    "fp32ir_8192macro_r3_p3_kappa1e-3": dict(n=64, r=3, p=3, kappa=1e-3, beta=(1.0, 0.5),
                                             sol="exp_sin", precision="fp32"),
    # BF16 factors (FP32 LU rounded for storage) + FP64 refinement, same mesh and data
    "bf16ir_8192macro_r3_p3_kappa1e-3": dict(n=64, r=3, p=3, kappa=1e-3, beta=(1.0, 0.5),
                                             sol="exp_sin", precision="bf16", inner_rtol=1e-2),
    "plain_fp64_8192macro_r3_p3_kappa1e-3": dict(n=64, r=3, p=3, kappa=1e-3, beta=(1.0, 0.5),
                                                 sol="exp_sin", precision="fp64"),
    # differentiation configuration: 128 x 128 squares (32,768 macros), r = 2, p = 2,
    # kappa_K = exp(0.5 xi_K) (seed 5), a = (1, 1), f fixed (u = sin sin with kappa = 1,
    # a = (1, 1)), g_D = 0; J = ||u_h - u_obs||^2, u_obs for kappa exp(0.1 eta) (seed 55)
    # batching configuration, one coefficient instance at a time: 8192 macros with r drawn
    # from {1,2,3,4} (seed 3), p = 3, instance i of 64 (kappa log-uniform [1e-3, 1],
    # a random direction, |a| in [0.5, 2], seed 33), u = exp(x) sin(2 pi y) data
    "mixed_r1to4_8192macro_p3_inst0": dict(n=64, r="mixed", p=3, kappa=None, beta=None,
                                           sol="exp_sin", precision="fp64", instance=0),
    # batching configuration, all 64 coefficient instances in one handle: one 8 x 8-square
    # block of the mixed-level mesh (128 macros, r from {1,2,3,4}, seed 3) per instance, so
    # the 64 instances hold the same 219 GB of FP64 factors as one instance of the
    # 8192-macro mesh; every launch covers all instances, GMRES runs per instance in
    # lockstep with converged instances masked out of later applies
    "batched_64inst_128macro_r1to4_p3": dict(n=8, r="mixed", p=3, kappa=None, beta=None,
                                             sol="exp_sin", precision="fp64", n_inst=64),
    # GMRES(1000) for the forward and the adjoint solves (about 12,000 iterations each at
    # 1e-9; GMRES(300) stalls on the adjoint, no restart costs 1.8x more basis traffic)
    # the batching configuration with the folded Schur-factor form: all 64 instances
    # factored (Q x Q Schur blocks), folded and solved together, GMRES(50) per instance
    "batched_folded_qelim_64inst_128macro_r1to4_p3": dict(n=8, r="mixed", p=3, kappa=None,
                                                          beta=None, sol="exp_sin",
                                                          precision="qelim", form="folded",
                                                          n_inst=64, restart=50),
    # the default job with SUPG inside the macros (section 3.4; sub-triangle Peclet number
    # 0.15, tau = 2.9e-4): the stabilised local blocks, plain and tuned forms
    "supg_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                      sol="exp_sin", precision="fp64", supg=True),
    # the plain at-scale operator applied to many vectors per call (one factorisation,
    # several right-hand sides): a wavefront carries 4 vectors through the local solve
    "many_rhs_fp64_8192macro_r3_p3": dict(n=64, r=3, p=3, kappa=1e-2, beta=(1.0, 0.5),
                                          precision="fp64", form="many_rhs", n_rhs=32),
    # the batching configuration at full size: all 64 coefficient instances on the
    # 8192-macro mixed-level mesh, one after another on one handle (their factors do not
    # fit together), each with the folded Schur-factor form.  The diffusion-dominated
    # instances need a longer Krylov basis: with GMRES(50) those with kappa >= 0.1 stall
    # at 20000 iterations, with GMRES(150) they converge in 8300..16300 (GMRES(400) and
    # (1000) are no faster there: fewer iterations, each dearer), while for kappa ~ 1e-3
    # GMRES(50) is the fastest (551 ms against 830 ms at 150)
    "all64_folded_qelim_mixed_r1to4_8192macro_p3": dict(n=64, r="mixed", p=3, kappa=None,
                                                        beta=None, sol="exp_sin",
                                                        precision="qelim",
                                                        form="sequential_instances",
                                                        n_inst=64, restart=50,
                                                        restart_diffusive=150,
                                                        kappa_diffusive=0.015),
    "adjoint_32768macro_r2_p2": dict(n=128, r=2, p=2, kappa=None, beta=(1.0, 1.0), sol="sin_sin",
                                     precision="fp64", form="adjoint", restart=1000, rtol=1e-9),
    # the same with folded applies (T_K, forward and transposed)
    "adjoint_folded_32768macro_r2_p2": dict(n=128, r=2, p=2, kappa=None, beta=(1.0, 1.0),
                                            sol="sin_sin", precision="fp64", form="adjoint",
                                            restart=1000, rtol=1e-9, folded=True),
}


def apply_bytes(m, elem_bytes=8, levels=None, p=None, qelim=False) -> float:
    """Algorithmic HBM bytes of one apply's per-macro solves: every stored LU
    entry once (b N_K^2, b = 8 for FP64 factors, 4 for FP32), the pivot vector
    (4 N_K), the gathered trace and the written contribution slots (about
    2 x 8 x 2 n_trace).  With the flux eliminated the stored factor is the
    Q x Q Schur block (Q = N_K / 3); the per-level templates are shared by all
    macros and read from cache, not counted."""
    s = m.sizes
    if levels is None:
        n_e = np.full(s.n_macro, float(s.max_local))
    else:
        P = (2 ** np.asarray(levels, dtype=np.int64)) * p
        n_e = 3.0 * (P + 1) * (P + 2) / 2
    if qelim:
        n_e = n_e / 3.0
    return float(np.sum(elem_bytes * n_e * n_e + 4.0 * n_e)) + 32.0 * s.n_trace


def fold_bytes(tri, r, p, n_trace):
    """Algorithmic bytes of one folded apply: every T_K once (8 L_K^2, L_K = the
    macro's interior-face trace dofs, n_F = 2^{r_F} p + 1 per interior edge with
    r_F the larger level of the two macros), the gathered trace and the written
    slots (2 x 8 x 2 n_trace)."""
    tri = np.asarray(tri)
    r = np.broadcast_to(np.asarray(r, dtype=np.int64), (len(tri),))
    e = np.sort(np.stack([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=1), axis=2)
    keys = e[..., 0].astype(np.int64) * (tri.max() + 1) + e[..., 1]
    _, inv, cnt = np.unique(keys.ravel(), return_inverse=True, return_counts=True)
    flev = np.zeros(len(cnt), dtype=np.int64)
    np.maximum.at(flev, inv, np.repeat(r, 3))
    nF = (2 ** flev[inv] * p + 1).reshape(-1, 3)
    L = np.where((cnt[inv] == 2).reshape(-1, 3), nF, 0).sum(axis=1)
    return 8.0 * float(np.sum(L.astype(np.float64) ** 2)) + 32.0 * n_trace


def boundary_bytes(m, n_trace):
    """Algorithmic bytes of one boundary-condensed apply: every W_K once
    (8 (9P)^2, P = 2^r_K p), the gathered trace and the written slots
    (2 x 8 x 2 n_trace)."""
    P = m.macro_P().astype(np.float64)
    return 8.0 * float(np.sum((9.0 * P) ** 2)) + 32.0 * n_trace


def lu_flops(w, s, qelim=False):
    """(2/3) N_K^3 summed over macros (and coefficient instances); (2/3) Q^3
    for the Schur blocks of the flux-eliminated form (Q = N_K / 3)."""
    f = 1.0 / 27.0 if qelim else 1.0
    if np.ndim(w["r"]) == 0:
        return f * s.n_macro * (2.0 / 3.0) * float(s.max_local) ** 3
    P = (2 ** np.asarray(w["r"], dtype=np.int64)) * w["p"]
    return f * s.n_instances * float(np.sum((2.0 / 3.0) * (3.0 * (P + 1) * (P + 2) / 2) ** 3))


def measured_traffic(workload):
    """HBM bytes per apply launch from the committed PMC summary
    (profiles/traffic.json), or None when there is none for this workload or
    the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[workload]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    if rec.get("traffic_bytes_per_launch") is None:   # counters taken but not usable
        return None
    return rec


def cpu_baseline(xy, tri, w, lam_seed=1, n_sample=16, budget_s=15.0):
    """The oracle (scipy LU + lu_solve per macro) applying the trace operator
    on a bounded sample of macros, scaled to the full mesh."""
    from oracle import hdg
    from paper_2302_10917_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    orc = hdg.Oracle(xy, tri, w["r"], w["p"], w["kappa"], w["beta"], 1.0,
                     supg=bool(w.get("supg")))
    n_macro = orc.topo.n_macro
    sample = np.unique(np.linspace(0, n_macro - 1, min(n_sample, n_macro)).astype(int))
    lam = inputs.random_vector(orc.topo.n_trace, seed=lam_seed)
    t0 = time.perf_counter()
    for K in sample:
        orc.lu(int(K))
    t_setup = time.perf_counter() - t0
    reps = 0
    t0 = time.perf_counter()
    while True:
        for K in sample:
            orc.macro_contribution(int(K), lam)
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 2000:
            break
    t = (time.perf_counter() - t0) / reps
    per_apply = t * n_macro / len(sample)
    o7 = oracle_condensation_time(orc, sample[:4])
    return {"value": 1.0 / per_apply, "unit": "applies/s", "cores": cores, "kind": "oracle",
            "sample": (f"steps 1-3 (x = B lam, lu_solve, C y) on {len(sample)} of {n_macro} "
                       f"macros, {reps} repetitions, scaled by {n_macro / len(sample):.0f}; "
                       f"assembly + lu_factor of the sample took {t_setup:.1f} s and is excluded"),
            "cpu": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "factor_s_whole_mesh": t_setup * n_macro / len(sample),
            "condensation": o7}


def oracle_solve_estimate(cb, applies_per_solve, gpu_time_to_solve_s):
    """The oracle's time to solve the job, added to the cpu_baseline record cb:
    its assembly + LU of every macro (factor_s_whole_mesh, from the sample), then
    the job's GMRES applies (the mean over the timed solves) at the sampled rate;
    the oracle's Krylov vector work is not counted."""
    n_app = float(np.mean(applies_per_solve))
    cb["time_to_solve_s_estimate"] = cb["factor_s_whole_mesh"] + n_app / cb["value"]
    cb["time_to_solve_estimate"] = (
        f"factor_s_whole_mesh + {n_app:.0f} applies / value; the GPU solve of the "
        f"same job: {gpu_time_to_solve_s:.2f} s")
    return cb


def oracle_condensation_time(orc, sample):
    """The oracle's per-macro condensation (assembly of A_K, B_K, C_K, lu_factor,
    S_K = -C_K A_K^-1 B_K on the interior faces and f^_K; the step before its sparse
    direct solve) timed on a few macros with one BLAS thread and with all of them,
    extrapolated to the whole mesh by the macro count."""
    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits, threadpool_info
    f = np.ones(int(orc.topo.node_off[-1]))
    lamD = orc.dirichlet_trace(np.zeros(orc.topo.n_bnd))

    def one_pass():
        t0 = time.perf_counter()
        for K in sample:
            K = int(K)
            orc._cache.clear()
            b = orc.blocks(K)
            lu = orc.lu(K)
            icols = orc._interior_cols(K)
            if icols:
                Bi = np.hstack([b.B[k] for k, _, _ in icols])
                Ci = np.vstack([b.C[k] for k, _, _ in icols])
                _ = -Ci @ sla.lu_solve(lu, Bi)
                _ = -Ci @ sla.lu_solve(lu, orc.local_rhs(K, f, lamD))
        orc._cache.clear()
        return (time.perf_counter() - t0) / len(sample)

    with threadpool_limits(1):
        t1 = one_pass()
    t_all = one_pass()
    threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    n = orc.topo.n_macro
    return {"per_macro_s_1_thread": t1, "per_macro_s_all_threads": t_all,
            "all_threads": threads,
            "whole_mesh_s_1_thread": t1 * n, "whole_mesh_s_all_threads": t_all * n,
            "whole_mesh_s_one_macro_per_core_estimate": t1 * n / (os.cpu_count() or 1),
            "sample": f"{len(sample)} macros, extrapolated by {n / len(sample):.0f}",
            "direct_solve": "the sparse LU of the assembled S (SuperLU) is not timed here: "
                            "it is minutes on the host at the 8192-macro size"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain_fp64_8192macro_r3_p3", choices=list(WORKLOADS))
    ap.add_argument("--folded-restart", type=int, default=40,
                    help="GMRES restart of the folded form run beside the plain one")
    ap.add_argument("--restart", type=int, default=None,
                    help="GMRES Krylov length (default: 2000, 8000 for the differentiation workload)")
    ap.add_argument("--rtol", type=float, default=None,
                    help="GMRES relative tolerance (default 1e-10; 1e-9 for the differentiation "
                         "workload, whose 440,064-unknown trace system stalls near 1e-10)")
    ap.add_argument("--inner-rtol", type=float, default=None,
                    help="inner GMRES tolerance per refinement step (reduced-precision factors; "
                         "default 1e-5 for FP32, 1e-2 for BF16)")
    ap.add_argument("--fd-check", action="store_true",
                    help="differentiation workload: central differences of J on sampled kappa_K "
                         "and on both advection components, against the adjoint gradient")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="after the timed steps, solve again with FP64 factors and report the "
                         "relative differences of lambda, q and u")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--compare-sequential", type=int, default=0, metavar="K",
                    help="batched workload: after the timed steps, solve the first K instances "
                         "one at a time with single-instance handles (the plain form) and "
                         "report their time")
    ap.add_argument("--instances", default=None, metavar="I,J,...",
                    help="sequential-instances workload: solve only these coefficient "
                         "instances (default: all)")
    ap.add_argument("--n-rhs", type=int, default=None,
                    help="many-vector workload: vectors per call (default 32)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="sequential-instances workload: one handle, no overlap of the next "
                         "instance's factorisation with the current solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--folded", action="store_true",
                    help="run the GMRES applies on the folded macro operators (FP64 workloads, "
                         "including the differentiation workload's adjoint solve)")
    ap.add_argument("--no-tuned-forms", action="store_true",
                    help="plain FP64 workloads: skip the folded-operator comparison that follows "
                         "the timed steps")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel shapes (no autotuning before the warmup)")
    ap.add_argument("--stop-norm", choices=["true", "preconditioned"], default="true",
                    help="stopping test of the FP64 and flux-eliminated solves: the "
                         "unpreconditioned relative residual ||f^ - S lam|| / ||f^|| (default) "
                         "or the preconditioned one; reduced-precision factors stop on the "
                         "refined system's residual")
    ap.add_argument("--driver", choices=["device", "host"], default="device",
                    help="GMRES driver: Arnoldi recurrences on the device, one host wait per "
                         "restart cycle (default), or on the host, one wait per iteration")
    ap.add_argument("--no-jitter-control", action="store_true",
                    help="default job: skip the jittered-mesh control (factor + 20 applies)")
    ap.add_argument("--max-iter", type=int, default=20000,
                    help="GMRES iteration cap (a short cap is for counter runs only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain 1 GiB read + 1 GiB write "
                         "elementwise kernel (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_10917_amd import inputs, mhdg

    w = dict(WORKLOADS[args.workload])
    args.restart_override = args.restart is not None
    if args.restart is None:
        args.restart = w.get("restart", 2000)
    if args.rtol is None:
        args.rtol = w.get("rtol", 1e-10)
    if args.inner_rtol is None:
        args.inner_rtol = w.get("inner_rtol", 1e-5)
    if w.get("form") == "adjoint":
        return bench_adjoint(args, w)
    if w.get("form") == "sequential_instances":
        return bench_sequential_instances(args, w)
    if w.get("form") == "many_rhs":
        return bench_many_rhs(args, w)
    assembled = w.get("form") == "assembled"
    boundary = w.get("form") == "boundary"
    folded = (w.get("form") == "folded" or args.folded) and not (assembled or boundary)
    condensed = folded or assembled or boundary
    xy, tri = inputs.structured_mesh(w["n"])
    n_inst = w.get("n_inst", 1)
    if w["r"] == "mixed":
        w["r"] = inputs.random_levels(len(tri), (1, 2, 3, 4), seed=3)
        kap_i, beta_i = inputs.coefficient_instances(64, seed=33)
        if n_inst > 1:
            w["kappa"], w["beta"] = kap_i[:n_inst], beta_i[:n_inst]
        else:
            w["kappa"] = float(kap_i[w["instance"]])
            w["beta"] = tuple(float(x) for x in beta_i[w["instance"]])
    m = mhdg.MacroMesh(xy, tri, w["r"], w["p"])
    if w.get("supg"):
        m.set_supg(True)
    one = m.sizes
    if n_inst > 1:
        m.set_instances(n_inst)
    s = m.sizes
    node, bnd = m.sample_points()
    dev = "cuda"
    kap_inst = np.atleast_1d(np.asarray(w["kappa"], dtype=np.float64))
    beta_inst = np.asarray(w["beta"], dtype=np.float64).reshape(-1, 2)
    fh, gh = np.empty(s.n_nodes), np.empty(s.n_bnd_points)
    for i in range(n_inst):
        ex = getattr(inputs, w["sol"])(float(kap_inst[i]), beta_inst[i])
        a, b_ = i * one.n_nodes, (i + 1) * one.n_nodes
        fh[a:b_] = ex.f(node[a:b_, 0], node[a:b_, 1])
        a, b_ = i * one.n_bnd_points, (i + 1) * one.n_bnd_points
        gh[a:b_] = ex.u(bnd[a:b_, 0], bnd[a:b_, 1])
    f = torch.as_tensor(fh, device=dev)
    g = torch.as_tensor(gh, device=dev)
    kappa = torch.as_tensor(np.repeat(kap_inst, one.n_macro), device=dev)
    beta_arg = beta_inst if n_inst > 1 else tuple(beta_inst[0])
    lam = torch.zeros(s.n_trace, dtype=torch.float64, device=dev)
    qu = torch.empty(s.n_local, dtype=torch.float64, device=dev)
    prec = {"fp32": mhdg.MHDG_FP32, "bf16": mhdg.MHDG_BF16,
            "qelim": mhdg.MHDG_QELIM}.get(w["precision"], mhdg.MHDG_FP64)
    reduced = prec in (mhdg.MHDG_FP32, mhdg.MHDG_BF16)
    print(f"[bench] {args.workload}: {s.n_macro} macros, N_K={s.max_local}, "
          f"n_trace={s.n_trace}, {n_inst} instance(s), factor workspace "
          f"{m.query(prec).factor_ws_bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)

    infos = []
    Q = s.n_nodes // s.n_macro


    inst_infos = []

    stop = (mhdg.MHDG_NORM_TRUE if args.stop_norm == "true" and not reduced
            else mhdg.MHDG_NORM_PRECONDITIONED)
    drv = mhdg.MHDG_DRIVER_DEVICE if args.driver == "device" else mhdg.MHDG_DRIVER_HOST
    if stop == mhdg.MHDG_NORM_TRUE and drv == mhdg.MHDG_DRIVER_HOST:
        stop = mhdg.MHDG_NORM_PRECONDITIONED
    # the plain form's cycles run as direct launches, so that every apply is
    # bracketed by HIP events for the roofline (its 11 ms applies leave no
    # launch overhead to hide); the folded forms replay captured cycles
    sgraph = condensed

    def step():
        m.factor_local(kappa, beta_arg, 1.0, precision=prec)
        if folded or assembled:
            m.fold_operator()
        if assembled:
            m.assemble_trace_matrix()
        if boundary:
            m.condense_boundary()
        info = m.solve(f, g, lam, rtol=args.rtol, restart=args.restart, max_iter=args.max_iter,
                       check=args.max_iter >= 20000, inner_rtol=args.inner_rtol, folded=folded,
                       max_outer=60, graph=sgraph, driver=drv, stop_norm=stop,
                       assembled=assembled, boundary=boundary)
        m.recover_local(lam, qu)
        infos.append(info.as_dict())
        inst_infos.append(m.last_solve_infos)

    tune = None
    if not args.no_autotune and prec != mhdg.MHDG_QELIM:
        m.factor_local(kappa, beta_arg, 1.0, precision=prec)
        tune = m.autotune()
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i}: {infos[-1]['iterations']} iterations, "
              f"{infos[-1]['t_gmres_ms']:.0f} ms GMRES", file=sys.stderr, flush=True)
    infos.clear()
    inst_infos.clear()
    m.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        its = [x["iterations"] for x in inst_infos[-1]]
        print(f"[bench] step {i}: {min(its)}..{max(its)} iterations, worst rel res "
              f"{max(x['rel_res_prec'] for x in inst_infos[-1]):.2e} (true "
              f"{max(x['rel_res_true'] for x in inst_infos[-1]):.2e})",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = m.profile(False)
    elapsed = t1 - t0
    # applies counted per instance (a batched launch is one apply for every
    # instance that takes part in it)
    applies = sum(x["n_applies"] for step_infos in inst_infos for x in step_infos)
    ms_per_step = 1e3 * elapsed / args.steps

    print("[bench] timed steps done; operator-only throughput", file=sys.stderr, flush=True)
    # pure operator throughput (outside the timed steps)
    lam_r = torch.as_tensor(inputs.random_vector(s.n_trace, seed=1), device=dev)
    out = torch.empty_like(lam_r)
    aflags = (mhdg.MHDG_PRECONDITION | (mhdg.MHDG_FOLDED if folded else 0) |
              (mhdg.MHDG_ASSEMBLED if assembled else 0) | (mhdg.MHDG_BOUNDARY if boundary else 0))
    m.apply_trace_operator(lam_r, out, aflags)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(args.apply_reps):
        m.apply_trace_operator(lam_r, out, aflags)
    torch.cuda.synchronize()
    apply_only = args.apply_reps / (time.perf_counter() - ta)
    # the same applies with events around each kernel (used for the roofline when the
    # timed solves replayed captured cycles, which carry no per-apply events)
    m.profile(True)
    for _ in range(args.apply_reps):
        m.apply_trace_operator(lam_r, out, aflags)
    torch.cuda.synchronize()
    kt_apply = m.profile(False)

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # reference: a plain streaming read of 16 GiB on this device (context for the roofline)
    buf = torch.ones(1 << 31, dtype=torch.float64, device=dev)
    torch.sum(buf)
    torch.cuda.synchronize()
    tr = time.perf_counter()
    for _ in range(5):
        torch.sum(buf)
    torch.cuda.synchronize()
    stream_gbs = 5 * buf.numel() * 8 / (time.perf_counter() - tr) / 1e9
    del buf

    tuned = None
    if (not args.no_tuned_forms and not condensed and n_inst == 1 and prec == mhdg.MHDG_FP64
            and np.ndim(w["r"]) == 0):
        # the tuned form of the same job: folded macro operators (timed like the
        # plain steps, same handle, same data; outside the plain timed region)
        print("[bench] folded form of the same job", file=sys.stderr, flush=True)
        lam_plain = lam.clone()
        f_infos = []

        def fstep():
            m.factor_local(kappa, beta_arg, 1.0, precision=prec)
            m.fold_operator()
            inf = m.solve(f, g, lam, rtol=args.rtol, restart=args.folded_restart,
                          max_iter=args.max_iter, folded=True, driver=drv, stop_norm=stop)
            m.recover_local(lam, qu)
            f_infos.append(inf.as_dict())
        fstep()                                  # warm-up (captures the folded graph)
        f_infos.clear()
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        for _ in range(args.steps):
            fstep()
        torch.cuda.synchronize()
        tf = (time.perf_counter() - tf0) / args.steps
        tuned = {"folded_fp64": {
            "time_to_solve_s": tf,
            "applies_per_s": sum(x["n_applies"] for x in f_infos) / (tf * args.steps),
            "iterations": [x["iterations"] for x in f_infos],
            "gmres_restart": args.folded_restart,
            "speedup_vs_plain": (ms_per_step / 1e3) / tf,
            "rel_res_true": max(x["rel_res_true"] for x in f_infos),
            "rel_res_prec": max(x["rel_res_prec"] for x in f_infos),
            "cycles": f_infos[-1]["cycles"], "host_waits": f_infos[-1]["host_waits"],
            "max_rel_diff_lambda_vs_plain":
                float(torch.linalg.norm(lam - lam_plain) / torch.linalg.norm(lam_plain)),
            "what": "T_K = C_K A_K^-1 B_K stored per macro after the LU (built with the "
                    "stored factors), GMRES applies read 8 L_K^2 bytes per macro"}}
        print(f"[bench] folded: {tuned}", file=sys.stderr, flush=True)

        # the same folded form with the flux eliminated: LU of the Q x Q Schur blocks
        # (Q = N_K / 3), T_K built from them
        print("[bench] folded form from the Schur-block factors", file=sys.stderr, flush=True)
        q_infos = []

        def qstep():
            m.factor_local(kappa, beta_arg, 1.0, precision=mhdg.MHDG_QELIM)
            m.fold_operator()
            inf = m.solve(f, g, lam, rtol=args.rtol, restart=args.folded_restart,
                          max_iter=args.max_iter, folded=True, driver=drv, stop_norm=stop)
            m.recover_local(lam, qu)
            q_infos.append(inf.as_dict())
        qstep()
        q_infos.clear()
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        for _ in range(args.steps):
            qstep()
        torch.cuda.synchronize()
        tq = (time.perf_counter() - tq0) / args.steps
        tuned["folded_flux_eliminated_fp64"] = {
            "time_to_solve_s": tq,
            "applies_per_s": sum(x["n_applies"] for x in q_infos) / (tq * args.steps),
            "iterations": [x["iterations"] for x in q_infos],
            "gmres_restart": args.folded_restart,
            "speedup_vs_plain": (ms_per_step / 1e3) / tq,
            "rel_res_true": max(x["rel_res_true"] for x in q_infos),
            "rel_res_prec": max(x["rel_res_prec"] for x in q_infos),
            "cycles": q_infos[-1]["cycles"], "host_waits": q_infos[-1]["host_waits"],
            "max_rel_diff_lambda_vs_plain":
                float(torch.linalg.norm(lam - lam_plain) / torch.linalg.norm(lam_plain)),
            "what": "q eliminated exactly through the reference mass; LU of the Q x Q Schur "
                    "block on u only; T_K = C_K A_K^-1 B_K from it; folded GMRES applies"}
        print(f"[bench] folded from Schur factors: {tuned['folded_flux_eliminated_fp64']}",
              file=sys.stderr, flush=True)

        # the matrix-based form (section 6.1): S assembled from the operators folded
        # from the Schur factors, GMRES on block-sparse products
        print("[bench] assembled trace matrix from the Schur-block factors", file=sys.stderr,
              flush=True)
        a_infos = []

        def astep():
            m.factor_local(kappa, beta_arg, 1.0, precision=mhdg.MHDG_QELIM)
            m.fold_operator()
            m.assemble_trace_matrix()
            inf = m.solve(f, g, lam, rtol=args.rtol, restart=args.folded_restart,
                          max_iter=args.max_iter, assembled=True, driver=drv, stop_norm=stop)
            m.recover_local(lam, qu)
            a_infos.append(inf.as_dict())
        astep()
        a_infos.clear()
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for _ in range(args.steps):
            astep()
        torch.cuda.synchronize()
        tma = (time.perf_counter() - tm0) / args.steps
        tuned["matrix_based_flux_eliminated_fp64"] = {
            "time_to_solve_s": tma,
            "applies_per_s": sum(x["n_applies"] for x in a_infos) / (tma * args.steps),
            "iterations": [x["iterations"] for x in a_infos],
            "gmres_restart": args.folded_restart,
            "speedup_vs_plain": (ms_per_step / 1e3) / tma,
            "rel_res_true": max(x["rel_res_true"] for x in a_infos),
            "rel_res_prec": max(x["rel_res_prec"] for x in a_infos),
            "cycles": a_infos[-1]["cycles"], "host_waits": a_infos[-1]["host_waits"],
            "max_rel_diff_lambda_vs_plain":
                float(torch.linalg.norm(lam - lam_plain) / torch.linalg.norm(lam_plain)),
            "what": "the global trace matrix S = D - sum T_K assembled block-sparse from the "
                    "folded Schur-factor operators; GMRES on its products (matrix-based form)"}
        print(f"[bench] assembled: {tuned['matrix_based_flux_eliminated_fp64']}",
              file=sys.stderr, flush=True)

        # the boundary-condensed form: W_K = (A_K^-1)_bb built from the FP64 factors,
        # GMRES applies through W_K
        print("[bench] boundary-condensed form", file=sys.stderr, flush=True)
        b_infos = []
        b_prec = prec

        def bstep():
            m.factor_local(kappa, beta_arg, 1.0, precision=b_prec)
            m.condense_boundary()
            inf = m.solve(f, g, lam, rtol=args.rtol, restart=args.folded_restart,
                          max_iter=args.max_iter, boundary=True, driver=drv, stop_norm=stop)
            m.recover_local(lam, qu)
            b_infos.append(inf.as_dict())
        bstep()
        b_infos.clear()
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for _ in range(args.steps):
            bstep()
        torch.cuda.synchronize()
        tbc = (time.perf_counter() - tb0) / args.steps
        lam_b = torch.as_tensor(inputs.random_vector(s.n_trace, seed=1), device=dev)
        out_b = torch.empty_like(lam_b)
        m.profile(True)
        for _ in range(args.apply_reps):
            m.apply_trace_operator(lam_b, out_b, mhdg.MHDG_PRECONDITION | mhdg.MHDG_BOUNDARY)
        torch.cuda.synchronize()
        kb = m.profile(False)["folded_apply"]
        b_ms = kb["ms"] / max(kb["count"], 1)
        b_bytes = boundary_bytes(m, s.n_trace)
        tuned["boundary_condensed_fp64"] = {
            "time_to_solve_s": tbc,
            "applies_per_s": sum(x["n_applies"] for x in b_infos) / (tbc * args.steps),
            "iterations": [x["iterations"] for x in b_infos],
            "gmres_restart": args.folded_restart,
            "speedup_vs_plain": (ms_per_step / 1e3) / tbc,
            "rel_res_true": max(x["rel_res_true"] for x in b_infos),
            "rel_res_prec": max(x["rel_res_prec"] for x in b_infos),
            "max_rel_diff_lambda_vs_plain":
                float(torch.linalg.norm(lam - lam_plain) / torch.linalg.norm(lam_plain)),
            "apply_kernel_ms": b_ms,
            "apply_bytes": b_bytes,
            "apply_gbs": b_bytes / (b_ms * 1e-3) / 1e9,
            "apply_frac_hbm": b_bytes / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "what": "W_K = (A_K^-1)_bb over the macro's 9P boundary unknowns (the interior "
                    "condensed out), built by unit-vector solves on the FP64 factors; GMRES "
                    "applies lift with B_K, multiply by W_K, restrict with C_K"}
        print(f"[bench] boundary-condensed: {tuned['boundary_condensed_fp64']}",
              file=sys.stderr, flush=True)
        # the same blocks from the Schur-block factors of the flux elimination
        print("[bench] boundary-condensed form from the Schur-block factors", file=sys.stderr,
              flush=True)
        b_prec = mhdg.MHDG_QELIM
        b_infos.clear()
        bstep()
        b_infos.clear()
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for _ in range(args.steps):
            bstep()
        torch.cuda.synchronize()
        tbq = (time.perf_counter() - tb0) / args.steps
        tuned["boundary_condensed_flux_eliminated_fp64"] = {
            "time_to_solve_s": tbq,
            "applies_per_s": sum(x["n_applies"] for x in b_infos) / (tbq * args.steps),
            "iterations": [x["iterations"] for x in b_infos],
            "gmres_restart": args.folded_restart,
            "speedup_vs_plain": (ms_per_step / 1e3) / tbq,
            "rel_res_true": max(x["rel_res_true"] for x in b_infos),
            "rel_res_prec": max(x["rel_res_prec"] for x in b_infos),
            "max_rel_diff_lambda_vs_plain":
                float(torch.linalg.norm(lam - lam_plain) / torch.linalg.norm(lam_plain)),
            "what": "W_K = (A_K^-1)_bb built by unit-vector solves through the flux "
                    "elimination and the Q x Q Schur-block factors; GMRES applies through W_K"}
        print(f"[bench] boundary-condensed from Schur factors: "
              f"{tuned['boundary_condensed_flux_eliminated_fp64']}", file=sys.stderr, flush=True)

    jitter = None
    if not args.no_jitter_control and args.workload == "plain_fp64_8192macro_r3_p3":
        # control: the same job on a mesh whose interior vertices move by up to 0.15 h in
        # each coordinate (seed 7), so no two macros share a Jacobian: factorisation and
        # applies must cost what they cost on the uniform mesh (nothing is reused between
        # macros that happen to be congruent)
        print("[bench] jittered-mesh control: factor + 20 applies", file=sys.stderr, flush=True)

        def factor_and_applies(mm):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mm.factor_local(kappa, beta_arg, 1.0)
            torch.cuda.synchronize()
            t_f = time.perf_counter() - t0
            o = torch.empty_like(lam_r)
            mm.apply_trace_operator(lam_r, o, mhdg.MHDG_PRECONDITION | mhdg.MHDG_GRAPH)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(20):
                mm.apply_trace_operator(lam_r, o, mhdg.MHDG_PRECONDITION | mhdg.MHDG_GRAPH)
            torch.cuda.synchronize()
            return t_f, (time.perf_counter() - t1) / 20

        uni = factor_and_applies(m)
        xyj, trij = inputs.structured_mesh(w["n"], jitter=0.15, seed=7)
        mj = mhdg.MacroMesh(xyj, trij, w["r"], w["p"])
        jit = factor_and_applies(mj)
        mj.close()
        del mj
        torch.cuda.empty_cache()
        jitter = {"mesh": f"{w['n']} x {w['n']} squares, interior vertices moved by "
                          f"U(-0.15 h, 0.15 h) per coordinate, seed 7",
                  "factor_s": jit[0], "apply_ms": 1e3 * jit[1],
                  "uniform_factor_s": uni[0], "uniform_apply_ms": 1e3 * uni[1],
                  "factor_ratio": jit[0] / uni[0], "apply_ratio": jit[1] / uni[1]}
        print(f"[bench] jittered control: {jitter}", file=sys.stderr, flush=True)

    seq = None
    if args.compare_sequential and n_inst > 1:
        kk = min(args.compare_sequential, n_inst)
        print(f"[bench] plain form: {kk} instances solved one at a time", file=sys.stderr,
              flush=True)
        m1 = mhdg.MacroMesh(xy, tri, w["r"], w["p"])
        lam1 = torch.zeros(one.n_trace, dtype=torch.float64, device=dev)
        qu1 = torch.empty(one.n_local, dtype=torch.float64, device=dev)
        seq_its, seq_applies, diffs = [], 0, []
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for i in range(kk):
            m1.factor_local(kappa[i * one.n_macro:(i + 1) * one.n_macro], tuple(beta_inst[i]), 1.0)
            inf1 = m1.solve(f[i * one.n_nodes:(i + 1) * one.n_nodes],
                            g[i * one.n_bnd_points:(i + 1) * one.n_bnd_points], lam1,
                            rtol=args.rtol, restart=args.restart, max_iter=args.max_iter)
            m1.recover_local(lam1, qu1)
            seq_its.append(inf1.iterations)
            seq_applies += inf1.n_applies
            ref = lam[i * one.n_trace:(i + 1) * one.n_trace]
            diffs.append(float(torch.linalg.norm(lam1 - ref) / torch.linalg.norm(ref)))
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - ts
        del m1
        seq = {"instances": kk, "seconds": t_seq, "seconds_per_instance": t_seq / kk,
               "applies_per_s": seq_applies / t_seq, "iterations": seq_its,
               "max_rel_diff_lambda_vs_batched": max(diffs),
               "batched_seconds_per_instance": elapsed / args.steps / n_inst,
               "speedup_per_instance": (t_seq / kk) / (elapsed / args.steps / n_inst)}
        print(f"[bench] plain form: {seq}", file=sys.stderr, flush=True)

    # discretisation error of the solution against the manufactured one: the largest
    # nodal difference, and the L2 norm of u_h minus the interpolant of u (the macros'
    # mass matrices), relative to the interpolant's
    u_l2 = None
    if np.ndim(w["r"]) == 0 and n_inst == 1:
        u_h = qu.view(s.n_macro, 3, Q)[:, 2, :].reshape(-1).cpu().numpy()
        u_ex = ex.u(node[:, 0], node[:, 1])
        u_err = float(np.abs(u_h - u_ex).max())

        def l2(v):
            d = torch.zeros(s.n_macro, 3, Q, dtype=torch.float64, device=dev)
            d[:, 2, :] = torch.as_tensor(v, device=dev).view(s.n_macro, Q)
            d = d.reshape(-1)
            o = torch.empty_like(d)
            m.mass_apply(d, o)
            return float(torch.sqrt(torch.dot(d, o)))
        u_l2 = l2(u_h - u_ex) / l2(u_ex)
    else:
        u_err = None

    cmp = None
    if args.compare_fp64 and prec != mhdg.MHDG_FP64:
        print("[bench] reference solve with FP64 factors (rtol 1e-12)", file=sys.stderr, flush=True)
        lam_lp, qu_lp = lam.clone(), qu.clone()
        m.factor_local(kappa, w["beta"], 1.0, precision=mhdg.MHDG_FP64)
        ref = m.solve(f, g, lam, rtol=1e-12, restart=args.restart, max_iter=args.max_iter)
        print(f"[bench] reference: {ref.iterations} iterations", file=sys.stderr, flush=True)
        m.recover_local(lam, qu)
        qv, qv_lp = qu.view(s.n_macro, 3, Q), qu_lp.view(s.n_macro, 3, Q)

        def rd(a, b_):
            return float(torch.linalg.norm(a - b_) / torch.linalg.norm(b_))
        cmp = {"reference": "FP64 factors, GMRES rtol 1e-13",
               "lambda": rd(lam_lp, lam), "q": rd(qv_lp[:, :2], qv[:, :2]),
               "u": rd(qv_lp[:, 2], qv[:, 2])}

    ams = kt["folded_apply" if condensed else "apply_macro_solve"]
    # apply launches that did work: GMRES and residual applies (n_applies less the
    # two right-hand-side passes), per solve the largest count over instances.  The
    # event time of launches after every instance converged (the rest of the last
    # restart cycle runs as near-empty kernels) stays in the total, so the average
    # below is a slight overestimate of a working launch's duration
    work_launches = sum(max(x["n_applies"] - 2 for x in si) for si in inst_infos)
    if reduced:
        work_launches = ams["count"]   # refinement: every launch of the kernel is an apply
    apply_timing = "HIP events around every apply kernel of the timed solves"
    if ams["count"] == 0:
        # captured cycles: the apply kernel timed by events in the apply-only loop
        ams = kt_apply["folded_apply" if condensed else "apply_macro_solve"]
        work_launches = ams["count"]
        apply_timing = ("HIP events around the apply kernel in an apply-only loop after the "
                        "timed solves (those replay captured GMRES cycles, without events)")
    avg_ms = ams["ms"] / max(work_launches, 1)
    nbytes = apply_bytes(m, {mhdg.MHDG_FP32: 4, mhdg.MHDG_BF16: 2}.get(prec, 8),
                         None if np.ndim(w["r"]) == 0 else np.tile(w["r"], n_inst), w["p"],
                         qelim=prec == mhdg.MHDG_QELIM)
    if folded:
        # folded apply: T_K read once (8 L_K^2), the gathered trace and the slots, for
        # every instance
        nbytes = n_inst * fold_bytes(tri, w["r"], w["p"], one.n_trace)
    if assembled:
        # assembled product: every stored block once (and its table), the trace read and
        # the result written once
        # (S and D^-1 S are stored side by side, a product reads one of them: the
        # workspace holds row_ptr, the 72-byte block table, then the two value arrays)
        ws = float(mhdg.load_library().mhdg_trace_matrix_ws_bytes(m.h))
        n_int = s.n_interior_faces
        n_blk = int(m.matrix_ws[:4 * (n_int + 1)].view(torch.int32)[n_int].item())
        a256 = lambda b: (b + 255) // 256 * 256
        tables = a256(4 * (n_int + 1)) + a256(72 * n_blk)
        nbytes = tables + (ws - tables) / 2 + 16.0 * s.n_trace
    if boundary:
        nbytes = boundary_bytes(m, s.n_trace)
    if n_inst > 1:
        # converged instances are masked out of later launches: count the
        # instances each launch actually processed (GMRES applies + the
        # true-residual apply of every instance)
        inst_launches = sum(x["n_applies"] - 2 for si in inst_infos for x in si)
        nbytes = nbytes / n_inst * inst_launches / max(work_launches, 1)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    lu = kt["lu"]
    result = {
        "metric": METRIC,
        "value": applies / elapsed,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {mhdg.MHDG_FP64: "f64", mhdg.MHDG_QELIM: "f64",
                  mhdg.MHDG_FP32: "f32 factors, f64 refinement",
                  mhdg.MHDG_BF16: "bf16 factors (f32 LU), f64 refinement"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "n_macro": s.n_macro, "n_instances": n_inst,
                   "r": w["r"] if np.ndim(w["r"]) == 0 else "U{1,2,3,4} seed 3", "p": w["p"],
                   "N_K": s.max_local, "n_trace": s.n_trace,
                   "kappa": w["kappa"] if n_inst == 1 else "10^U(-3,0) per instance, seed 33",
                   "beta": list(w["beta"]) if n_inst == 1 else
                   "|a| U(0.5,2), direction U[0,2pi) per instance, seed 33",
                   "tau": 1.0, "rtol": args.rtol, "gmres_restart": args.restart,
                   "form": ("folded_fp64" if folded else "boundary_condensed_fp64" if boundary
                            else "batched_fp64" if n_inst > 1 else "plain_fp64")
                   if prec == mhdg.MHDG_FP64 else
                   ("matrix_based_flux_eliminated_fp64" if assembled else
                    "folded_flux_eliminated_fp64" if folded else
                    "boundary_condensed_flux_eliminated_fp64" if boundary else
                    "flux_eliminated_fp64")
                   if prec == mhdg.MHDG_QELIM else
                   ("fp32_factors_fp64_ir" if prec == mhdg.MHDG_FP32 else "bf16_factors_fp64_ir"),
                   "supg": bool(w.get("supg")),
                   "inner_rtol": args.inner_rtol if reduced else None,
                   "stop_norm": ("unpreconditioned ||f^ - S lam|| / ||f^||"
                                 if stop == mhdg.MHDG_NORM_TRUE else
                                 "preconditioned ||D^-1 (f^ - S lam)|| / ||D^-1 f^||"),
                   "gmres_driver": args.driver, "cycles_graph_captured": sgraph},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["traffic_bytes_per_launch"] / 1e9 if traffic else None,
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-kernel calibrated; see profiles/)",
                     "traffic_vs_algorithmic": traffic["traffic_bytes_per_launch"] / nbytes
                     if traffic else None,
                     "kernel": ("trace_matrix_apply_kernel (assembled D^-1 S, the preconditioned product)" if assembled else
                                "bc_apply_kernel (boundary-condensed steps 1-3)" if boundary else
                                "fold_apply_kernel (folded steps 1-3)" if folded else
                                "qelim_solve_kernel (apply steps 1-3, flux eliminated)"
                                if prec == mhdg.MHDG_QELIM else
                                "macro_solve_kernel<%s> (apply steps 1-3)"
                                % {mhdg.MHDG_FP64: "double", mhdg.MHDG_FP32: "float",
                                   mhdg.MHDG_BF16: "bf16_t"}[prec]),
                     "bytes_per_launch": nbytes, "avg_launch_ms": avg_ms,
                     "launches": work_launches, "launch_records": ams["count"],
                     "timing": apply_timing},
        "time_to_solve_s": ms_per_step / 1e3,
        "iterations": [i["iterations"] for i in infos] if n_inst == 1 else
        [[x["iterations"] for x in si] for si in inst_infos],
        "sequential_plain": seq,
        "outer_iterations": [i["outer_iterations"] for i in infos],
        "applies_per_solve": [i["n_applies"] for i in infos],
        "second_gs_passes": [i["reorth_passes"] for i in infos],
        "gmres_cycles": [i["cycles"] for i in infos],
        "host_waits_per_solve": [i["host_waits"] for i in infos],
        "vs_fp64": cmp,
        "rel_res_prec": [max(x["rel_res_prec"] for x in si) for si in inst_infos],
        "rel_res_true": [max(x["rel_res_true"] for x in si) for si in inst_infos],
        "apply_only_per_s": apply_only,
        "stream_read_gbs": stream_gbs,
        "kernel_ms": {k: v["ms"] / max(args.steps, 1) for k, v in kt.items()},
        "lu_tflops": lu_flops(w, s, prec == mhdg.MHDG_QELIM) / (lu["ms"] / max(lu["count"], 1) * 1e-3)
        / 1e12
        if lu["count"] else None,
        "u_max_err_vs_exact": u_err,
        "u_rel_l2_err_vs_exact": u_l2,
        "autotune": tune,
        "tuned_forms": tuned,
        "jitter_control": jitter,
    }
    if not args.no_cpu_baseline:
        wc = dict(w)
        if n_inst > 1:   # the oracle applies one instance's operator
            wc["kappa"], wc["beta"] = float(kap_inst[0]), tuple(beta_inst[0])
        cb = cpu_baseline(xy, tri, wc)
        if result.get("applies_per_solve"):
            oracle_solve_estimate(cb, result["applies_per_solve"], result["time_to_solve_s"])
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def bench_many_rhs(args, w):
    """One step = the preconditioned trace operator D^-1 S applied to n_rhs vectors
    by one call of the many-vector apply (FP64 factors of the plain at-scale mesh).
    After the timed steps: the per-vector rate for 1..32 vectors per call and of
    the single-vector apply."""
    import torch
    from paper_2302_10917_amd import inputs, mhdg

    xy, tri = inputs.structured_mesh(w["n"])
    m = mhdg.MacroMesh(xy, tri, w["r"], w["p"])
    s = m.sizes
    dev = "cuda"
    kappa = torch.full((s.n_macro,), w["kappa"], dtype=torch.float64, device=dev)
    m.factor_local(kappa, w["beta"], 1.0)
    n_rhs = args.n_rhs or w["n_rhs"]
    vec = 32.0 * s.n_trace                       # gathered trace + written slots, per vector
    fac = apply_bytes(m) - vec                   # every stored factor entry once
    flags = mhdg.MHDG_PRECONDITION
    lam = torch.as_tensor(np.stack([inputs.random_vector(s.n_trace, seed=1 + v)
                                    for v in range(32)]), device=dev)
    out = torch.empty_like(lam)
    print(f"[bench] {args.workload}: {s.n_macro} macros, N_K={s.max_local}, "
          f"n_trace={s.n_trace}, {n_rhs} vectors per call", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        m.apply_trace_operator_many(lam[:n_rhs], out[:n_rhs], flags)
    torch.cuda.synchronize()
    m.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m.apply_trace_operator_many(lam[:n_rhs], out[:n_rhs], flags)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = m.profile(False)
    k_ms = kt["apply_macro_solve"]["ms"] / max(kt["apply_macro_solve"]["count"], 1)
    nbytes = fac + n_rhs * vec
    # single-vector apply and other group sizes (outside the timed steps)
    one = torch.empty(s.n_trace, dtype=torch.float64, device=dev)
    m.apply_trace_operator(lam[0], one, flags)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        m.apply_trace_operator(lam[0], one, flags)
    torch.cuda.synchronize()
    single = 5 / (time.perf_counter() - t1)
    sweep = {}
    for k in (1, 2, 4, 8, 16, 32):
        m.apply_trace_operator_many(lam[:k], out[:k], flags)
        torch.cuda.synchronize()
        reps = max(2, 32 // k)
        t2 = time.perf_counter()
        for _ in range(reps):
            m.apply_trace_operator_many(lam[:k], out[:k], flags)
        torch.cuda.synchronize()
        sweep[k] = reps * k / (time.perf_counter() - t2)
        print(f"[bench] {k} vectors per call: {sweep[k]:.1f} vector-applies/s",
              file=sys.stderr, flush=True)
    # the same with the folded operators (T_K read once per group of 8 vectors)
    m.fold_operator()
    fsweep = {}
    for k in (1, 8, 32):
        fl = flags | mhdg.MHDG_FOLDED
        m.apply_trace_operator_many(lam[:k], out[:k], fl)
        torch.cuda.synchronize()
        reps = max(4, 128 // k)
        t2 = time.perf_counter()
        for _ in range(reps):
            m.apply_trace_operator_many(lam[:k], out[:k], fl)
        torch.cuda.synchronize()
        fsweep[k] = reps * k / (time.perf_counter() - t2)
        print(f"[bench] folded, {k} vectors per call: {fsweep[k]:.1f} vector-applies/s",
              file=sys.stderr, flush=True)
    result = {
        "metric": METRIC,
        "value": args.steps * n_rhs / elapsed,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_macro": s.n_macro, "r": w["r"], "p": w["p"],
                   "N_K": s.max_local, "n_trace": s.n_trace, "kappa": w["kappa"],
                   "beta": list(w["beta"]), "tau": 1.0, "n_rhs": n_rhs,
                   "form": "plain_fp64, many vectors per apply"},
        "roofline": {"bound": "hbm", "achieved": nbytes / (k_ms * 1e-3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": nbytes / (k_ms * 1e-3) / 1e9 / 8000.0,
                     "traffic": None,
                     "kernel": ("apply_many_mfma_kernel<8, 8, 1> (16 vectors per workgroup, "
                                "sweeps on MFMA)" if n_rhs >= 12 and s.max_local <= 1024 else
                                "apply_many_kernel (per-wavefront sweeps)"),
                     "algorithmic_bytes_per_launch": nbytes,
                     "kernel_ms": k_ms},
        "single_vector_applies_per_s": single,
        "vector_applies_per_s_by_n_rhs": sweep,
        "folded_vector_applies_per_s_by_n_rhs": fsweep,
    }
    print(json.dumps(result), flush=True)


def bench_sequential_instances(args, w):
    """One step = every coefficient instance of the batching configuration on the
    full mixed-level mesh, solved one after another on one handle with the folded
    Schur-factor form (factor_local with the flux eliminated, fold_operator,
    folded GMRES, recover_local), each to rtol."""
    import torch
    from paper_2302_10917_amd import inputs, mhdg

    xy, tri = inputs.structured_mesh(w["n"])
    r = inputs.random_levels(len(tri), (1, 2, 3, 4), seed=3)
    kap_i, beta_i = inputs.coefficient_instances(64, seed=33)
    ids = (list(range(w["n_inst"])) if args.instances is None
           else [int(x) for x in args.instances.split(",")])
    n_inst = len(ids)
    m = mhdg.MacroMesh(xy, tri, r, w["p"])
    s = m.sizes
    node, bnd = m.sample_points()
    dev = "cuda"
    lam = torch.zeros(s.n_trace, dtype=torch.float64, device=dev)
    qu = torch.empty(s.n_local, dtype=torch.float64, device=dev)
    data = {}
    for i in ids:
        ex = getattr(inputs, w["sol"])(float(kap_i[i]), beta_i[i])
        data[i] = (torch.as_tensor(ex.f(node[:, 0], node[:, 1]), device=dev),
                   torch.as_tensor(ex.u(bnd[:, 0], bnd[:, 1]), device=dev),
                   torch.full((s.n_macro,), float(kap_i[i]), dtype=torch.float64, device=dev),
                   tuple(float(x) for x in beta_i[i]))
    print(f"[bench] {args.workload}: {n_inst} instances x {s.n_macro} macros, N_K up to "
          f"{s.max_local}, n_trace={s.n_trace}", file=sys.stderr, flush=True)
    infos = []

    def restart_for(i):
        if args.restart_override:
            return args.restart
        return w["restart_diffusive"] if kap_i[i] >= w["kappa_diffusive"] else w["restart"]

    # Two handles on two streams (default priority): while one instance's GMRES
    # runs, a second host thread factors and folds the next instance on the other
    # handle.  The library calls release the GIL; each handle keeps its own
    # workspaces, graphs and pinned buffers.
    from concurrent.futures import ThreadPoolExecutor
    n_h = 1 if args.no_overlap else 2
    meshes = [m] + [mhdg.MacroMesh(xy, tri, r, w["p"]) for _ in range(n_h - 1)]
    streams = [torch.cuda.Stream() for _ in meshes]
    lams = [lam] + [torch.zeros_like(lam) for _ in range(n_h - 1)]
    qus = [qu] + [torch.empty_like(qu) for _ in range(n_h - 1)]
    torch.cuda.synchronize()

    def prepare(h, i):
        _, _, kap, beta = data[i]
        with torch.cuda.stream(streams[h]):
            meshes[h].factor_local(kap, beta, 1.0, precision=mhdg.MHDG_QELIM)
            meshes[h].fold_operator()

    def finish(h, i):
        f, g, _, _ = data[i]
        with torch.cuda.stream(streams[h]):
            inf = meshes[h].solve(f, g, lams[h], rtol=args.rtol, restart=restart_for(i),
                                  max_iter=args.max_iter, folded=True, check=False)
            meshes[h].recover_local(lams[h], qus[h])
            streams[h].synchronize()
        d = inf.as_dict()
        print(f"[bench] instance {i}: kappa {kap_i[i]:.3e} |beta| {np.hypot(*beta_i[i]):.2f}: "
              f"GMRES({restart_for(i)}) {d['iterations']} iterations, status {d['status']}, rel res "
              f"{d['rel_res_prec']:.2e}, {d['t_gmres_ms']:.0f} ms GMRES", file=sys.stderr,
              flush=True)
        return d

    def run(seq):
        out = []
        if n_h == 1:
            for i in seq:
                prepare(0, i)
                out.append(finish(0, i))
            return out
        with ThreadPoolExecutor(1) as pool:
            prepare(0, seq[0])
            for k, i in enumerate(seq):
                nxt = pool.submit(prepare, (k + 1) % 2, seq[k + 1]) if k + 1 < len(seq) else None
                out.append(finish(k % 2, i))
                if nxt is not None:
                    nxt.result()
        return out

    for _ in range(args.warmup):
        run(ids[:n_h])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        infos.extend(run(ids))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    applies = sum(x["n_applies"] for x in infos)
    its = [x["iterations"] for x in infos]
    worst = max(x["rel_res_prec"] for x in infos)
    result = {
        "metric": METRIC,
        "value": applies / elapsed,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_macro": s.n_macro, "n_instances": n_inst,
                   "r": "U{1,2,3,4} seed 3", "p": w["p"],
                   "kappa": "10^U(-3,0) per instance, seed 33",
                   "beta": "|a| U(0.5,2), direction U[0,2pi) per instance, seed 33",
                   "tau": 1.0, "rtol": args.rtol,
                   "gmres_restart": (args.restart if args.restart_override else
                                     f"{w['restart']} for kappa < {w['kappa_diffusive']}, "
                                     f"else {w['restart_diffusive']}"),
                   "form": "folded_flux_eliminated_fp64, instances in sequence" +
                           ("" if args.no_overlap else
                            ", next instance factored and folded during the current solve")},
        "time_to_solve_s": elapsed / args.steps,
        "per_instance_s": elapsed / (args.steps * n_inst),
        "iterations_min_max": [min(its), max(its)],
        "worst_rel_res_prec": worst,
        "all_converged": all(x["status"] == 0 for x in infos),
    }
    print(json.dumps(result))


def bench_adjoint(args, w):
    """One step = forward solve (factor_local + solve + recover_local) plus the
    objective and its adjoint gradient (mhdg_adjoint behind torch.autograd)."""
    import torch
    from paper_2302_10917_amd import autograd as ad
    from paper_2302_10917_amd import inputs, mhdg

    args.folded = args.folded or w.get("folded", False)

    xy, tri = inputs.structured_mesh(w["n"])
    n_macro = len(tri)
    m = mhdg.MacroMesh(xy, tri, w["r"], w["p"])
    s = m.sizes
    node, bnd = m.sample_points()
    ex = inputs.sin_sin(1.0, (1.0, 1.0))
    dev = "cuda"
    f = torch.as_tensor(ex.f(node[:, 0], node[:, 1]), device=dev)
    g = torch.as_tensor(ex.u(bnd[:, 0], bnd[:, 1]), device=dev)
    kappa = inputs.lognormal_kappa(n_macro, 0.5, seed=5)
    eta = np.random.default_rng(55).standard_normal(n_macro)
    beta = torch.tensor(w["beta"], dtype=torch.float64)
    print(f"[bench] {args.workload}: {n_macro} macros, N_K={s.max_local}, n_trace={s.n_trace}",
          file=sys.stderr, flush=True)
    with torch.no_grad():
        qu_obs = ad.solve(torch.as_tensor(kappa * np.exp(0.1 * eta), device=dev), beta, m, f, g,
                          args.rtol, args.restart, args.folded).clone()
    print(f"[bench] u_obs solved: {m.last_solve_info['iterations']} iterations", file=sys.stderr,
          flush=True)
    infos = []

    def step():
        k = torch.as_tensor(kappa, device=dev).requires_grad_(True)
        b = beta.clone().requires_grad_(True)
        J = ad.l2_misfit(m, ad.solve(k, b, m, f, g, args.rtol, args.restart, args.folded), qu_obs)
        fwd = dict(m.last_solve_info)
        J.backward()
        infos.append((fwd, dict(m.last_adjoint_info)))
        return J.item(), k.grad, b.grad

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
    infos.clear()
    m.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        J, dk, db = step()
        print(f"[bench] step {i}: forward {infos[-1][0]['iterations']} it, adjoint "
              f"{infos[-1][1]['iterations']} it, J = {J:.6e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = m.profile(False)
    applies = sum(a["n_applies"] + b_["n_applies"] for a, b_ in infos)
    fd = None
    if args.fd_check:
        print("[bench] central differences (outside the timed region)", file=sys.stderr, flush=True)

        def Jof(kap, bet):
            with torch.no_grad():
                qu = ad.solve(torch.as_tensor(kap, device=dev), torch.tensor(bet), m, f, g,
                              args.rtol, args.restart, args.folded)
                return ad.l2_misfit(m, qu, qu_obs).item()
        # J is smooth in kappa_K: a relative step of 1e-3 keeps the central-difference
        # truncation small while lifting the J difference above the solve tolerance
        h, hk = 1e-5, 1e-3
        dkh = dk.cpu().numpy()
        fd = {"step_beta": h, "step_kappa_rel": hk, "kappa": [], "beta": []}
        for K in (int(np.argmax(np.abs(dkh))), n_macro // 3):
            kp, km = kappa.copy(), kappa.copy()
            kp[K] *= 1 + hk
            km[K] *= 1 - hk
            v = (Jof(kp, w["beta"]) - Jof(km, w["beta"])) / (2 * hk * kappa[K])
            fd["kappa"].append({"macro": K, "fd": v, "adjoint": float(dkh[K]),
                                "rel_diff": abs(v - dkh[K]) / abs(v)})
            print(f"[bench] fd kappa_{K}: {fd['kappa'][-1]}", file=sys.stderr, flush=True)
        for d in range(2):
            bp, bm = list(w["beta"]), list(w["beta"])
            bp[d] += h
            bm[d] -= h
            v = (Jof(kappa, bp) - Jof(kappa, bm)) / (2 * h)
            fd["beta"].append({"d": d, "fd": v, "adjoint": float(db[d]),
                               "rel_diff": abs(v - float(db[d])) / abs(v)})
            print(f"[bench] fd beta_{d}: {fd['beta'][-1]}", file=sys.stderr, flush=True)
    ams = kt["folded_apply" if args.folded else "apply_macro_solve"]
    # launches that did work: forward GMRES + residual applies (n_applies less the two
    # right-hand-side passes) and adjoint GMRES applies (less its right side and the
    # final A^-T pass); near-empty launches after convergence stay in the event time
    work = sum((a["n_applies"] - 2) + (b_["n_applies"] - 2) for a, b_ in infos)
    apply_timing = "HIP events around every apply kernel of the timed steps"
    if ams["count"] == 0:
        # the GMRES cycles ran as captured graphs, whose applies carry no events:
        # time the forward and transposed applies alone
        lam_r = torch.as_tensor(inputs.random_vector(s.n_trace, seed=1), device=dev)
        out_r = torch.empty_like(lam_r)
        fl = mhdg.MHDG_PRECONDITION | (mhdg.MHDG_FOLDED if args.folded else 0)
        m.profile(True)
        for _ in range(args.apply_reps):
            m.apply_trace_operator(lam_r, out_r, fl)
            m.apply_trace_operator(lam_r, out_r, fl | mhdg.MHDG_TRANSPOSE)
        torch.cuda.synchronize()
        ams = m.profile(False)["folded_apply" if args.folded else "apply_macro_solve"]
        work = ams["count"]
        apply_timing = ("HIP events around the forward and transposed apply kernels in an "
                        "apply-only loop after the timed steps (those replay captured GMRES "
                        "cycles, without events)")
    avg_ms = ams["ms"] / max(work, 1)
    nbytes = fold_bytes(tri, w["r"], w["p"], s.n_trace) if args.folded else apply_bytes(m, 8)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC, "value": applies / elapsed, "unit": "applies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_macro": n_macro, "r": w["r"], "p": w["p"],
                   "N_K": s.max_local, "n_trace": s.n_trace, "kappa": "lognormal sigma 0.5 seed 5",
                   "beta": list(w["beta"]), "tau": 1.0, "rtol": args.rtol,
                   "gmres_restart": args.restart,
                   "form": "forward + adjoint gradient" + (", folded" if args.folded else "")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("fold_apply_kernel (forward and transposed folded applies)"
                                if args.folded else
                                "macro_solve_kernel<double> (forward apply steps 1-3)"),
                     "bytes_per_launch": nbytes, "avg_launch_ms": avg_ms, "launches": work,
                     "launch_records": ams["count"], "timing": apply_timing},
        "forward_iterations": [a["iterations"] for a, _ in infos],
        "adjoint_iterations": [b_["iterations"] for _, b_ in infos],
        "kernel_ms": {k: v["ms"] / max(args.steps, 1) for k, v in kt.items()},
        "J": J, "dJ_dbeta": [float(x) for x in db], "fd_check": fd,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
