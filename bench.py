#!/usr/bin/env python3
"""Benchmark: TPCG solves/s on one MI355X.

One step = one complete TPCG solve (Algorithm 5) of the deformed-geometry
Poisson workload: p = 3, n_el = 128 (129 dofs per direction), 9 weighted
Kronecker terms, rhs of Tucker rank 5, tol 1e-6, FP64.  Every step runs the
whole hot path (operator application, low-rank FD preconditioner, relative
and dynamic truncation, Tucker dots).  Inputs (operator bands, FD setup,
rhs) are resident in HBM before the timed region.

Prints one JSON line (see the "metric" key) with:
  value/ms_per_step    solves/s and mean solve time over the timed steps
  latency_ms           p50/p99 of the per-solve times
  kernels              per-family launches, time, algorithmic GB/s and GFLOP/s
                       measured with HIP events on the library's stream in
                       one extra solve after the timed ones (events around
                       every launch slow the host, so the timed solves run
                       without them)
  roofline             the dominant kernel family against its MI355X peak
  mode_products_hbm    batched standalone runs of the two HBM-bound mode-product
                       kernels (banded operator, FD chain) moving several GB
                       per launch: algorithmic GB/s, fraction of 8 TB/s and of a
                       plain device copy measured in the same run, and the
                       HBM bytes of the big launch from the committed
                       FETCH_SIZE / WRITE_SIZE summary (null once the kernel
                       source has changed since it was taken); the same runs
                       with FP32 arithmetic (band_apply_f32, fd_chain_f32:
                       FP64 data, bytes counted alike)
  matrix_cores         the library's DGEMM at order 4096 (probe of the FP64
                       matrix-core rate it reaches) and the solve's GEMMs as
                       fractions of the 78.6 TFLOP/s spec and of that probe
  boundary_conditions  solves with Neumann ends and non-homogeneous Dirichlet
                       data at n_el = 128 (manufactured u = 1 + 3z: error;
                       the deformed recipe: iterations, time)
  serving              a seeded mix of solves served with several concurrent
                       solves (one stream and library context each) against
                       the plain one-at-a-time path: solves/s and p50/p99
                       latency at Poisson arrival rates of 0.5, 1 and 2 times
                       the plain capacity and with all requests at once
  cpu_baseline         the FP64 oracle on the host cores (bounded sample)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload deformed|small]
                       [--fd approx|exact] [--arith f64|mixed] [--no-hbm] [--no-serve]
                       [--no-bc] [--no-annulus] [--serve-slots S] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

# HIP maps every stream of the process onto this many hardware queues (4 by
# default); a solve uses three streams (the main one and two for the
# speculative ST-HOSVD modes) and the serving runs one solve per slot, so
# with 4 queues independent kernels serialise behind each other.  Read by
# the HIP runtime at initialisation, so it is set before torch is imported.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPCG solves/sec + p50/p99 latency at rel. err 1e-6; HBM GB/s of mode products"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
# source file holding the kernels of each instrumented family
FAMILY_SOURCE = {"sym_eig": "eig.hip", "dgemm": "gemm.hip", "band_apply": "modeprod.hip",
                 "select_rank": "kernels.hip", "fd_forward": "modeprod.hip", "fd_backward": "modeprod.hip",
                 "householder_qr": "kernels.hip", "band_apply_batched": "modeprod.hip",
                 "fd_forward_batched": "modeprod.hip", "fd_backward_batched": "modeprod.hip"}


def measured_traffic(family):
    """HBM bytes per launch of a kernel family from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when none was taken or the
    family's kernel source has changed since (sha256 of the source file)."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(family)
    except (OSError, ValueError):
        return None
    if not rec or family not in FAMILY_SOURCE:
        return None
    src = os.path.join(ROOT, "paper_2306_00632_amd", "csrc", FAMILY_SOURCE[family])
    with open(src, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    return rec["bytes_per_launch"] if digest == rec.get("source_sha256") else None


def workload(name):
    import workloads as W
    return {"deformed": W.config_deformed, "small": W.config_small, "large": W.config_large}[name]()


# Batched standalone mode-product runs.  A single solve moves too few bytes per
# launch to show HBM bandwidth, so each kernel family is driven through its
# C-ABI call on one tall factor: x of ranks (m, 1, 1), m independent columns.
K1_SHAPE = dict(n_el=1024, p=2, R=9, m=40000, seed_op=8101, seed_x=8102)
K2_SHAPE = dict(n_el=1024, p=3, m=25600, seed_x=8202)


def k1_inputs(shape=K1_SHAPE):
    import workloads as W
    w = W.weighted_cp(shape["n_el"], shape["p"], shape["R"], 1, shape["seed_op"], shape["seed_op"] + 1)
    core, U = W.random_tucker(w.n, (shape["m"], 1, 1), shape["seed_x"])
    return w, core, U


def k2_inputs(shape=K2_SHAPE):
    import workloads as W
    n = shape["n_el"] + shape["p"] - 2
    core, U = W.random_tucker(n, (shape["m"], 1, 1), shape["seed_x"])
    return core, U


def mode_products_hbm(ctx, reps=5):
    """Algorithmic GB/s of the banded operator (tucker_apply_op) and of the
    FD chain (fd_precond) on batched inputs.  Bytes follow the unfused
    per-unit definitions: operator, per mode, 8 (n r + R (2p+1) n + R n r);
    FD, per mode, 8 (n r + R_P n r + n n2) (the intermediate Z between the
    forward and the backward transform is not counted).  Times are the
    kernels' own (HIP events on the library's stream), summed over all
    launches of the family, the two one-column modes included."""
    import torch
    from paper_2306_00632_amd import problem, tk
    out = {}
    # reference: a plain device copy of 2 GiB (read + write), torch's copy kernel
    src = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src.numel() * 8 * reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    # write-only reference (the two mode-product kernels are ~90 % writes)
    ev0.record()
    for _ in range(reps):
        dst.fill_(2.0)
    ev1.record()
    torch.cuda.synchronize()
    fill_gbs = dst.numel() * 8 * reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del src, dst
    out["copy_probe"] = {"bytes_per_copy": 2 * (1 << 28) * 8, "GB_s": copy_gbs, "frac": copy_gbs / PEAK_HBM_GBS}
    out["fill_probe"] = {"bytes_per_fill": (1 << 28) * 8, "GB_s": fill_gbs, "frac": fill_gbs / PEAK_HBM_GBS}
    w, core, U = k1_inputs()
    op = problem.operator(ctx, w)
    x = tk.Tucker.from_host(ctx, core, U)
    del U

    def band(arith):
        y = tk.tucker_apply_op(ctx, op, x, arith=arith)   # warm-up
        del y
        ctx.sync()
        ctx.prof(True)
        for _ in range(reps):
            y = tk.tucker_apply_op(ctx, op, x, arith=arith)
            del y
        ctx.sync()
        k = ctx.prof_read()["band_apply"]
        ctx.prof(False)
        gbs = k["bytes"] / (k["ms"] / 1e3) / 1e9
        return {"call": "tucker_apply_op" if arith == "f64" else "tucker_apply_op_arith", "arith": arith,
                "n_el": w.n_el, "p": w.p, "n": w.n, "R": len(w.nnz), "ranks": [K1_SHAPE["m"], 1, 1],
                "GB_per_call": k["bytes"] / reps / 1e9, "ms_per_call": k["ms"] / reps, "GB_s": gbs,
                "frac": gbs / PEAK_HBM_GBS, "frac_of_copy": gbs / copy_gbs}

    tr = measured_traffic("band_apply_batched")
    out["band_apply"] = band("f64")
    out["band_apply"]["traffic_GB_big_launch"] = None if tr is None else tr / 1e9
    out["band_apply_f32"] = band("f32")
    del x, op
    core, U = k2_inputs()
    P = tk.Preconditioner.create(ctx, K2_SHAPE["n_el"], K2_SHAPE["p"], 0.1)
    info = P.info()
    n2 = P.direction(0)["n2"]
    s = tk.Tucker.from_host(ctx, core, U)
    n = U[0].shape[0]
    del U
    Rp = info["R_P"]
    cols = K2_SHAPE["m"] + 2
    by = 8.0 * ((1 + Rp) * n * cols + 3 * n * n2)

    def fd(arith):
        z = tk.fd_precond(ctx, P, s, arith=arith)   # warm-up
        del z
        ctx.sync()
        ctx.prof(True)
        for _ in range(reps):
            z = tk.fd_precond(ctx, P, s, arith=arith)
            del z
        ctx.sync()
        kk = ctx.prof_read()
        ctx.prof(False)
        ms = kk["fd_forward"]["ms"] + kk["fd_backward"]["ms"]
        gbs = by * reps / (ms / 1e3) / 1e9
        return {"call": "fd_precond" if arith == "f64" else "fd_precond_arith", "arith": arith,
                "n_el": K2_SHAPE["n_el"], "p": K2_SHAPE["p"], "n": n, "R_P": Rp, "ranks": [K2_SHAPE["m"], 1, 1],
                "GB_per_call": by / 1e9, "ms_per_call": ms / reps, "ms_forward": kk["fd_forward"]["ms"] / reps,
                "ms_backward": kk["fd_backward"]["ms"] / reps, "GB_s": gbs, "frac": gbs / PEAK_HBM_GBS,
                "frac_of_copy": gbs / copy_gbs}

    out["fd_chain"] = fd("f64")
    tf, tb = measured_traffic("fd_forward_batched"), measured_traffic("fd_backward_batched")
    out["fd_chain"]["traffic_GB_big_launches"] = None if tf is None or tb is None else (tf + tb) / 1e9
    out["fd_chain_f32"] = fd("f32")
    del s, P
    return out


def boundary_conditions(ctx, reps=3):
    """Solves with Neumann ends and non-homogeneous Dirichlet data (Appendix
    B flags; the lifting of the remark closing Sec. 3) at n_el = 128, p = 3:
    Dirichlet at z = 0 and z = 1, Neumann on the four other faces, the FD
    with Appendix B's eigen-approximations on those spaces (dense).  (1) the Laplacian with the data
    of u = 1 + 3z and f = 0, whose discrete solution is u itself: relative
    error of the TPCG solution; (2) the deformed recipe's 9 weighted terms
    with rhs of rank 5 and Dirichlet data of rank 2 (seeded): iterations and
    time.  Times include the lifting (one operator product on the full
    basis and a row restriction) and exclude the setup."""
    import numpy as np
    import torch
    from paper_2306_00632_amd import problem, tk
    import workloads as W
    n_el, p = 128, 3
    bcs = ((1, 1), (1, 1), (0, 0))
    out = {"n_el": n_el, "p": p, "flags": [list(b) for b in bcs], "fd_eigenpairs": "appendix_b_dense"}
    w = W.laplace_cube(n_el, p)
    gcore, gU = W.linear_dirichlet_data(n_el, p, (1.0, 0.0, 0.0, 3.0))
    op, P = problem.operator_bc(ctx, w, bcs), problem.preconditioner_bc(ctx, w, bcs)
    opf = problem.operator_bc(ctx, w, ((1, 1),) * 3)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = problem.lifted_rhs(ctx, w, bcs, gcore, gU, op_full=opf)
        x, info = tk.tpcg_solve(ctx, op, P, f, tol=1e-8)
        ctx.sync()
        ts.append(time.perf_counter() - t0)
    # the exact discrete solution: the data's coefficients at the unknowns
    rng = [problem.dof_range(n_el, p, b) for b in bcs]
    ref = np.einsum("abc,ia,jb,kc->ijk", gcore, *[gU[k][rng[k][0]:rng[k][1]] for k in range(3)])
    core, U = x.plain()
    xf = np.einsum("abc,ia,jb,kc->ijk", core, U[0], U[1], U[2])
    out["manufactured"] = {"u": "1 + 3z", "tol": 1e-8, "iters": info["iters"], "rank": list(info["rank"]),
                           "rel_err": float(np.linalg.norm(xf - ref) / np.linalg.norm(ref)),
                           "ms_per_solve": 1e3 * min(ts)}
    wd = W.weighted_cp(n_el, p, 9, 5, 2002, 2003)
    n = [n_el + p - 2 + sum(b) for b in bcs]
    fc, fU = W.random_tucker(n, (5, 5, 5), 2003)
    gc, gU = W.random_tucker(n_el + p, (2, 2, 2), 2004)
    op, P = problem.operator_bc(ctx, wd, bcs), problem.preconditioner_bc(ctx, wd, bcs)
    opf = problem.operator_bc(ctx, wd, ((1, 1),) * 3)
    fd = tk.Tucker.from_host(ctx, fc, fU)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = problem.lifted_rhs(ctx, wd, bcs, gc, gU, f=fd, op_full=opf)
        x, info = tk.tpcg_solve(ctx, op, P, f, tol=1e-6, eps_min=1e-8)
        ctx.sync()
        ts.append(time.perf_counter() - t0)
    out["deformed"] = {"tol": 1e-6, "iters": info["iters"], "relres": info["relres"], "rank": list(info["rank"]),
                       "ms_per_solve": 1e3 * min(ts), "solves_per_s": 1.0 / min(ts)}
    return out


def mapped_domain(ctx, domain="annulus", p_list=(2, 3, 4, 5), n_el_list=(128, 256, 512, 1024), scaled_p=(3,),
                  manufactured=True, maxit=400):
    """Sec. 5.1-5.2's mapped domains through the Appendix A front end: the
    thick quarter annulus with the manufactured solution, or the stand-in
    spherical shell (a gnomonic patch, radii 1 and 2) with f = 1.  Q and
    omega are sampled on Chebyshev-Lobatto grids (t = 33 and 64 points per
    direction), their coefficient tensors truncated on the device to the
    paper's eps = max(tol / 10, 1e-12), the 1D matrices and moments of the
    factor columns assembled on the host, and TPCG run at tol = 1e-6 with
    eps_prec = 0.1.  Per (p, n_el): the iterations (the paper's tables
    report 12 everywhere for the annulus and 74-106 for its shell; the
    default run takes the shell to n_el = 256, where a solve takes seconds), the
    solution rank, the front-end, FD-setup and solve times, with the FD of
    the parametric Laplacian (eq. FD_prec with unit coefficients) and, for p
    in scaled_p, with the mean of each diagonal entry of Q as direction
    coefficient; a run that reaches maxit iterations is reported with
    converged = false.  For the annulus with manufactured=True, a solve at
    n_el = 128, p = 3, tol = 1e-10 gives the error to the manufactured
    solution on a 9^3 grid of parametric points (max-norm, relative)."""
    import numpy as np
    from paper_2306_00632_amd import geometry, tk
    import workloads as W
    tol, t_q, t_w = 1e-6, 33, 64
    eps = max(0.1 * tol, 1e-12)
    if domain == "annulus":
        q, _, u = W.annulus_samples(t_q)
        _, omega, _ = W.annulus_samples(t_w)
        paper_iters = "12 for every p and n_el"
    else:
        q, _ = W.shell_samples(t_q)
        _, omega = W.shell_samples(t_w)
        paper_iters = "74-106 (the paper's shell map is not given; this one is a stand-in)"
    coef = geometry.fd_coefficients(q)
    out = {"tol": tol, "eps_front_end": eps, "t_q": t_q, "t_omega": t_w, "eps_prec": 0.1,
           "paper_iterations": paper_iters, "scaled_fd_coefficients": list(coef), "runs": []}
    for p in p_list:
        for n_el in n_el_list:
            ctx.sync()
            t0 = time.perf_counter()
            op, ranks = geometry.operator(ctx, n_el, p, q, eps)
            f = geometry.rhs(ctx, n_el, p, omega, eps)
            ctx.sync()
            t1 = time.perf_counter()
            out.setdefault("q_ranks", {f"{k + 1}{l + 1}": list(r) for (k, l), r in ranks.items()})
            for fd, c in (("parametric", (1.0, 1.0, 1.0)), ("scaled", coef)):
                if fd == "scaled" and p not in scaled_p:
                    continue
                ctx.sync()
                t2 = time.perf_counter()
                P = tk.Preconditioner.create(ctx, n_el, p, 0.1, c)
                ctx.sync()
                t3 = time.perf_counter()
                x, info = tk.tpcg_solve(ctx, op, P, f, allow_noconv=True, tol=tol, maxit=maxit)
                ctx.sync()
                t4 = time.perf_counter()
                out["runs"].append({"p": p, "n_el": n_el, "fd": fd, "iters": info["iters"],
                                    "converged": info["converged"],
                                    "relres": info["relres"], "rank": list(info["rank"]),
                                    "rhs_rank": list(f.shape()[1]), "front_end_ms": 1e3 * (t1 - t0),
                                    "fd_setup_ms": 1e3 * (t3 - t2), "solve_ms": 1e3 * (t4 - t3)})
    if manufactured and domain == "annulus":
        n_el, p = 128, 3
        op, _ = geometry.operator(ctx, n_el, p, q, 1e-11)
        f = geometry.rhs(ctx, n_el, p, omega, 1e-11)
        x, info = tk.tpcg_solve(ctx, op, tk.Preconditioner.create(ctx, n_el, p, 0.1, coef), f, tol=1e-10)
        e = np.linspace(0.05, 0.95, 9)
        E1, E2, E3 = np.meshgrid(e, e, e, indexing="ij")
        r, th = 1.0 + E1, 0.5 * np.pi * E2
        ue = u(r * np.cos(th), r * np.sin(th), E3)
        uh = geometry.evaluate(x, n_el, p, e, e, e)
        out["manufactured"] = {"n_el": n_el, "p": p, "tol": 1e-10, "fd": "scaled", "iters": info["iters"],
                               "rank": list(info["rank"]),
                               "max_rel_err": float(np.abs(uh - ue).max() / np.abs(ue).max())}
    return out


def matrix_cores(ctx, solve_kernels, reps=5):
    """FP64 matrix-core rates: a square GEMM of order 4096 through the
    library's own DGEMM (tk_dgemm, the kernel of every dense contraction of
    the truncation) as the probe of what the kernel reaches on this GPU, and
    the solve's GEMMs (algorithmic 2MNK flops over their kernel time, from the
    instrumented solve) as fractions of the spec peak and of that probe."""
    import torch
    from paper_2306_00632_amd import tk
    n = 4096
    g = torch.Generator(device="cuda").manual_seed(5)
    A = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    B = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    C = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    tk.dgemm(ctx, False, False, n, n, n, 1.0, A, n, B, n, 0.0, C, n)   # warm-up
    ctx.sync()
    ctx.prof(True)
    for _ in range(reps):
        tk.dgemm(ctx, False, False, n, n, n, 1.0, A, n, B, n, 0.0, C, n)
    ctx.sync()
    k = ctx.prof_read()["dgemm"]
    ctx.prof(False)
    del A, B, C
    probe = k["flops"] / (k["ms"] / 1e3) / 1e12
    out = {"probe": {"call": "tk_dgemm", "M": n, "N": n, "K": n, "ms_per_call": k["ms"] / reps,
                     "TFLOP_s": probe, "frac": probe / PEAK_FP64_TFLOPS}}
    d = solve_kernels.get("dgemm")
    if d and d["ms_per_solve"] > 0:
        tf = d["GFLOP_s"] / 1e3
        out["solve_dgemm"] = {"launches_per_solve": d["launches_per_solve"], "ms_per_solve": d["ms_per_solve"],
                              "TFLOP_s": tf, "frac": tf / PEAK_FP64_TFLOPS, "frac_of_probe": tf / probe}
    return out


# eps_min 1e-9: the paper's remedy for the stagnation of Sec. 5.3 (one request of
# this mix stalls near 1.4e-6 with 1e-8); maxit 300 bounds a stalled request
SERVE_MIX = dict(count=48, seed=4000, n_els=(64, 128), ps=(2, 3, 4), Rs=(3, 6, 9), ranks=range(1, 11),
                 eps_min=1e-9, maxit=300)


def serving(slots=16):
    """Continuous serving of a seeded mix of solves (the deformed recipe at
    n_el in {64, 128}, p in {2, 3, 4}, 3/6/9 terms, rhs rank 1..10): the plain
    path (one slot, one solve at a time) gives the capacity mu_plain; the
    server with `slots` concurrent solves then runs the same requests with
    Poisson arrivals at 0.5, 1 and 2 mu_plain and with all of them at once.
    Latency = completion - arrival (queueing and per-request setup included).
    The plain path runs every step in FP64; the served requests use the mixed
    arithmetic (TK_ARITH_MIXED) at the same tolerance, whose solutions meet
    the same accuracy bound (relres_max reports the worst final residual)."""
    import dataclasses
    from paper_2306_00632_amd import serve
    reqs = serve.mixed_requests(**SERVE_MIX)
    plain_srv = serve.Server(slots=1)
    plain_srv.run(reqs[:2])  # warm-up (code objects, pools)
    plain = serve.summarize(plain_srv.run(reqs))
    plain_srv.close()
    mu = plain["solves_per_s"]
    out = {"requests": len(reqs),
           "mix": {k: list(v) if isinstance(v, (tuple, range)) else v for k, v in SERVE_MIX.items()},
           "slots": slots, "plain": dict(plain, arith="f64"), "served_arith": "mixed", "served": {}}
    mreqs = [dataclasses.replace(r, arith="mixed") for r in reqs]
    srv = serve.Server(slots=slots)
    srv.run(mreqs[:slots])  # warm-up of every slot
    for name, rate in (("0.5x", 0.5 * mu), ("1x", mu), ("2x", 2.0 * mu), ("all_at_once", 0.0)):
        res = srv.run(serve.poisson_arrivals(mreqs, rate, SERVE_MIX["seed"] + 7))
        out["served"][name] = dict(serve.summarize(res), arrival_rate=rate)
    srv.close()
    out["speedup_all_at_once"] = out["served"]["all_at_once"]["solves_per_s"] / mu
    return out


def cpu_baseline(w, gpu_iters, target_s=12.0, exact=False):
    """The oracle's TPCG (unchanged) on a bounded sample of the same solve:
    the first k TPCG iterations (including the initial preconditioner and
    operator truncations), k chosen from a one-iteration calibration run so
    that the sample takes about `target_s`, extrapolated to a whole solve by
    the GPU run's iteration count.  Later iterations carry higher ranks and
    cost more, so the extrapolation favours the oracle."""
    import math
    from oracle import fd as ofd, problem as oprob, tpcg as otpcg
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    op = oprob.operator(w)
    f = oprob.rhs(w)
    prec = ofd.LowRankFD(w.n_el, w.p, 0.1, exact=exact)
    t0 = time.perf_counter()
    otpcg.tpcg(op, prec, f, tol=w.tol, eps_min=w.eps_min, maxit=1)
    t1 = time.perf_counter() - t0
    k = int(min(max(gpu_iters, 1), max(1, math.ceil(target_s / max(t1, 1e-3)))))
    if k > 1:
        t0 = time.perf_counter()
        _, info = otpcg.tpcg(op, prec, f, tol=w.tol, eps_min=w.eps_min, maxit=k)
        dt = time.perf_counter() - t0
        k = max(info.iters, 1)
    else:
        dt = t1
    per_solve = dt / k * max(gpu_iters, 1)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} TPCG iteration(s) of the same solve ({dt:.1f} s, numpy/scipy FP64), "
                      f"scaled by the GPU solve's {gpu_iters} iterations",
            "sample_seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="deformed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm", action="store_true", help="skip the batched mode-product bandwidth runs and the DGEMM probe")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving runs")
    ap.add_argument("--no-bc", action="store_true",
                    help="skip the solves with Neumann ends and non-homogeneous Dirichlet data")
    ap.add_argument("--no-annulus", action="store_true",
                    help="skip the thick quarter annulus and spherical shell solves through the Appendix A front end")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--fd", choices=("approx", "exact"), default="approx",
                    help="preconditioner eigenpairs: Appendix B approximations applied by sine transforms "
                         "(default) or the exact generalized eigenpairs applied by dense GEMMs")
    ap.add_argument("--arith", choices=("f64", "mixed"), default="f64",
                    help="f64: every step in FP64; mixed: the preconditioner and the direction's operator "
                         "products in FP32 arithmetic where the precision rule allows (TK_ARITH_MIXED)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of MIB MiB (read + write) before the solves, "
                         "as the known-size reference of a rocprofv3 FETCH_SIZE/WRITE_SIZE run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a TPCG solve is not split "
              f"across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2306_00632_amd import problem, tk

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    w = workload(args.workload)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = tk.Context(0)
    op = problem.operator(ctx, w)
    prec = problem.preconditioner(ctx, w, exact=(args.fd == "exact"))
    f = problem.rhs(ctx, w)
    params = dict(tol=w.tol, eps_min=w.eps_min, arith=args.arith)
    prm_used = tk.tpcg_params(**params)  # the solver defaults plus these, for the bench line
    for _ in range(args.warmup):
        x, info = tk.tpcg_solve(ctx, op, prec, f, **params)
        del x
    torch.cuda.synchronize()
    ctx.sync()

    # timed solves, uninstrumented
    times = []
    refinements0 = ctx.truncate_refinements()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        x, info = tk.tpcg_solve(ctx, op, prec, f, **params)
        ctx.sync()
        times.append(time.perf_counter() - t0)
        last_info = info
        del x
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    refinements = (ctx.truncate_refinements() - refinements0) / max(args.steps, 1)
    # one more solve with HIP events around every launch: per-family kernel
    # times for the breakdown and the roofline (not part of the timed value)
    ctx.prof(True)
    x, _ = tk.tpcg_solve(ctx, op, prec, f, **params)
    ctx.sync()
    del x
    kern = ctx.prof_read()
    ctx.prof(False)
    prof_solves = 1

    ms = [1e3 * t for t in times]
    kernels = {}
    for name, d in kern.items():
        if d["launches"] == 0:
            continue
        t = d["ms"] / 1e3
        kernels[name] = {"launches_per_solve": d["launches"] / prof_solves,
                         "ms_per_solve": d["ms"] / prof_solves,
                         "avg_us": 1e3 * d["ms"] / d["launches"],
                         "GB_s": d["bytes"] / t / 1e9 if t > 0 else 0.0,
                         "GFLOP_s": d["flops"] / t / 1e9 if t > 0 else 0.0}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_solve"])
    dk = kern[dom]
    if dom in ("band_apply", "fd_forward", "fd_backward", "select_rank"):
        achieved = dk["bytes"] / dk["launches"] / (dk["ms"] / dk["launches"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(dom)}
    else:
        achieved = dk["flops"] / dk["launches"] / (dk["ms"] / dk["launches"] / 1e3) / 1e12
        roof = {"bound": "alu" if dom != "dgemm" else "mfma", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(dom)}
    roof["kernel"] = dom
    roof["avg_launch_us"] = 1e3 * dk["ms"] / dk["launches"]
    mp = kern["band_apply"]
    mode_gbs = mp["bytes"] / (mp["ms"] / 1e3) / 1e9 if mp["ms"] > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.arith == "f64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "fd_eigenpairs": args.fd, "arith": args.arith,
                   "f32_applications": last_info["f32_applications"], "n_el": w.n_el, "p": w.p,
                   "dofs_per_direction": w.n,
                   "kronecker_terms": len(w.nnz), "rhs_rank": int(np.asarray(problem.rhs_arrays(w)[0]).shape[0]),
                   "tol": w.tol, "iters": last_info["iters"], "relres": last_info["relres"],
                   "solution_rank": list(last_info["rank"]), "trel_calls": last_info["trel_calls"],
                   "tail_refinements_per_solve": refinements, "eps_min": w.eps_min,
                   "refine_below": prm_used.refine_below, "reuse_bases": prm_used.reuse_bases},
        "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)),
                       "min": min(ms), "max": max(ms)},
        "mode_product_GB_s": mode_gbs,
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": None,
    }
    def section(name, fn, *a):
        t0 = time.perf_counter()
        out[name] = fn(*a)
        print(f"bench: {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    print(f"bench: {args.steps} timed solves done, {1e3 * total / max(args.steps, 1):.1f} ms each",
          file=sys.stderr, flush=True)
    if not args.no_hbm:
        section("mode_products_hbm", mode_products_hbm, ctx)
        section("matrix_cores", matrix_cores, ctx, kernels)
    if not args.no_bc:
        section("boundary_conditions", boundary_conditions, ctx)
    if not args.no_annulus:
        section("annulus", mapped_domain, ctx, "annulus")
        section("shell", lambda: mapped_domain(ctx, "shell", n_el_list=(128, 256)))
    if not args.no_serve:
        section("serving", serving, args.serve_slots)
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        section("cpu_baseline", lambda: cpu_baseline(w, last_info["iters"], exact=(args.fd == "exact")))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
