#!/usr/bin/env python3
"""Benchmark: DDG-PCG time to 1e-8 relative residual on one MI355X.

Workload (default): 3D variable-coefficient diffusion, 7-point cell-centred
stencil on 128^3 cells (2,097,152 unknowns), kappa = exp(GRF, correlation
length 8 cells, sigma 1), f ~ U(-1,1); 512 box subdomains of 16^3 cells,
overlap 1, p = 2 (10 monomials, N_c = 5120).  Synthetic, seeded inputs.

A step is one complete DDG-PCG solve (f resident in HBM -> u in HBM) with the
mixed-precision path (FP32 local factors, FP64 Krylov vectors, dots and
coarse inverse).  The FP64 path is timed on the same problem beside it.
Setup (coarse basis, Galerkin product, coarse inverse, local factors) is
reported separately.  The dominant kernel (the local solves, one launch per
colour phase with the library's default schedule) is timed with HIP events
attached to each of its dispatches on the handle's stream
(`hipExtLaunchKernelGGL`: the pair records the kernel's own start and end) in a
second timed pass of the same K solves (`value` comes from the pass without
them), and its algorithmic bytes give the roofline fraction.  The oracle's CPU time is
measured on a bounded sample (see `cpu_baseline`).

Prints one JSON line on stdout; progress goes to stderr.
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

METRIC = "DDG-PCG time-to-1e-8 residual & iters: mixed vs FP64 GPU; fwd+adjoint solves/s"
HBM_PEAK_GBS = 8000.0


# the local-solve kernel, its tile helpers, and the code that lays out what it reads
SWEEP_SOURCES = ["paper_1504_00907_amd/csrc/kernels_sweep.hip", "paper_1504_00907_amd/csrc/symv_tile.hpp",
                 "paper_1504_00907_amd/csrc/device_util.hpp", "paper_1504_00907_amd/csrc/kernels_setup.hip",
                 "paper_1504_00907_amd/csrc/symbolic.cpp"]


def profiled_traffic(kernel: str, precision: str, tile: int):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary.

    Returns None when no summary exists for this precision or when the kernel
    sources changed since the counters were taken (hash mismatch).
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_diffusion3d_128_{precision}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        for tok in line.split():
            if "=" in tok:
                k, v = tok.split("=", 1)
                kv[k] = v
    h = hashlib.sha256()
    for src in SWEEP_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if kv.get("src_sha256_16") != h.hexdigest()[:16] or kv.get("tile") != str(tile):
        return None
    try:
        return float(kv["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def profiled_mfma():
    """Setup GEMM rates on the FP64 matrix cores from the committed rocprofv3 summary
    (128^3 workload), or None when kernels_setup.hip changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "setup_mfma_diffusion3d_128.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        for tok in line.split():
            if "=" in tok:
                k, v = tok.split("=", 1)
                kv[k] = v
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_1504_00907_amd/csrc/kernels_setup.hip"), "rb").read())
    if kv.get("src_sha256_16") != h.hexdigest()[:16]:
        return None
    out = {"peak": 78.6, "unit": "TFLOP/s", "source": "profiles/setup_mfma_diffusion3d_128.md"}
    for name in ("bgemm", "galerkin"):
        fl, t = float(kv[f"{name}_flops"]), float(kv[f"{name}_s"])
        out[f"k_{name}"] = {"flops": fl, "seconds": t, "achieved": round(fl / t / 1e12, 2),
                            "frac": round(fl / t / 1e12 / 78.6, 4)}
    return out


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, iters: int, n_sample: int = 256, seed: int = 5, workers: int = 16):
    """Oracle time per solve on this host, extrapolated from a bounded sample.

    The sample factors `n_sample` of the subdomains with the oracle's banded
    Cholesky and times their pre- and post-sweep local updates twice: on one
    thread (BLAS limited to one thread), and with a thread pool of `workers`
    threads over the subdomains of each colour (independent by the colouring;
    BLAS one thread per worker).  The full coarse setup (per-subdomain QR,
    Galerkin product, dense Cholesky) and its application plus one SpMV are
    timed whole.  Per-iteration time = (sampled local time) * n_parts /
    n_sample + coarse apply + SpMV; the solve time is that times the
    iteration count.  `value` is the thread-pool figure.
    """
    from concurrent.futures import ThreadPoolExecutor

    import scipy.linalg as sla
    from threadpoolctl import threadpool_limits

    from oracle.ddg import _LocalSolver, coarse_basis, conflict_lists, galerkin, greedy_colouring, overlap_sets

    A = P.A.to_scipy()
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    R0, _, _, _, _ = coarse_basis(P.F, P.part, P.n_parts, 1e-10)
    A0 = galerkin(A, R0)
    fac = sla.cho_factor(A0, lower=True)
    t_coarse_setup = time.perf_counter() - t0
    sample = np.sort(rng.choice(P.n_parts, size=min(n_sample, P.n_parts), replace=False))
    sets = overlap_sets(A, P.part, P.n_parts, P.overlap)
    colours = greedy_colouring(conflict_lists(A, sets, P.n))
    t0 = time.perf_counter()
    solvers = {int(i): (_LocalSolver(A[sets[i]][:, sets[i]], int(i)), sets[i], A[sets[i]]) for i in sample}
    t_local_setup = (time.perf_counter() - t0) * P.n_parts / len(sample)
    order = [[int(i) for i in sample if colours[i] == c] for c in range(int(colours.max()) + 1)]
    r = np.random.default_rng(seed + 1).standard_normal(P.n)

    def update(i, e):
        ls, st, rows = solvers[i]
        e[st] += ls.solve(r[st] - rows @ e)

    with threadpool_limits(1):
        e = np.zeros(P.n)
        t0 = time.perf_counter()
        for seq in (order, order[::-1]):  # pre- and post-sweep
            for ids in seq:
                for i in ids:
                    update(i, e)
        t_local_1 = (time.perf_counter() - t0) * P.n_parts / len(sample)
        e = np.zeros(P.n)
        with ThreadPoolExecutor(max_workers=workers) as ex:
            t0 = time.perf_counter()
            for seq in (order, order[::-1]):
                for ids in seq:
                    # same-colour subdomains: no set meets another's neighbourhood
                    list(ex.map(lambda i: update(i, e), ids))
            t_local_w = (time.perf_counter() - t0) * P.n_parts / len(sample)
    t0 = time.perf_counter()
    q = A @ r
    y = R0.T @ sla.cho_solve(fac, R0 @ (r - A @ e))
    t_rest = time.perf_counter() - t0
    del q, y
    per_iter_1 = t_local_1 + t_rest
    per_iter_w = t_local_w + t_rest
    return {
        "value": per_iter_w * iters * 1e3,
        "unit": "ms",
        "cores": int(workers),
        "kind": "oracle",
        "sample": (f"oracle FP64 local solves on {len(sample)} of {P.n_parts} subdomains (banded "
                   f"LAPACK Cholesky), colour by colour with a pool of {workers} threads (BLAS 1 thread each), "
                   f"scaled by {P.n_parts}/{len(sample)}, plus full coarse apply and SpMV, times {iters} "
                   f"iterations; solve only (setup extrapolated separately: "
                   f"{(t_coarse_setup + t_local_setup):.1f} s)"),
        "single_thread_ms": per_iter_1 * iters * 1e3,
        "pool_threads": int(workers),
        "setup_s_extrapolated": t_coarse_setup + t_local_setup,
        "per_iter_ms": per_iter_w * 1e3,
        "per_iter_ms_single_thread": per_iter_1 * 1e3,
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


def cpu_fwd_adjoint(side: int, g_gpu: np.ndarray, tol: float = 1e-11):
    """The oracle's forward + adjoint + gradient on the differentiation workload.

    Two oracle setups (theta_obs, theta) and three PCG solves (u_obs, u,
    lambda) at rtol `tol`, then the oracle gradient formula; timed, and the
    GPU gradient's relative error against it (2-norm).
    """
    from oracle import DDGOracle
    from oracle.gradient import assemble_cc, coeff_grad_cc
    from workloads import box_partition, cell_coords, grf, monomials, seed_rng

    shape = (side,) * 3
    boxes = (side // 12,) * 3
    theta = grf(shape, 8.0, 1.0, seed_rng(4, 1))
    theta_obs = grf(shape, 8.0, 1.0, seed_rng(4, 2))
    fh = seed_rng(4, 0).uniform(-1.0, 1.0, side ** 3)
    part = box_partition(shape, boxes)
    F = monomials(cell_coords(shape), 2)
    nparts = int(np.prod(boxes))
    t0 = time.perf_counter()
    o = DDGOracle(assemble_cc(np.exp(theta_obs)), F, part, nparts, 1)
    uobs, _, _ = o.pcg(fh, tol)
    del o
    o = DDGOracle(assemble_cc(np.exp(theta)), F, part, nparts, 1)
    u, it_u, _ = o.pcg(fh, tol)
    lam, it_l, _ = o.pcg(2.0 * (u - uobs), tol)
    g = coeff_grad_cc(np.exp(theta), u, lam).ravel()
    t = time.perf_counter() - t0
    err = float(np.linalg.norm(g_gpu - g) / np.linalg.norm(g))
    return {"oracle_s": t, "oracle_rtol": tol, "oracle_iters_fwd": it_u, "oracle_iters_adj": it_l,
            "grad_rel_err_vs_oracle": err}


def elasticity(nel: int, steps: int, tile: int = 0, block_target: int = 0):
    """3D clamped Q1 elasticity leg: FP64, FP32 and BF16 local factors on the same system.

    nel^3 trilinear hexahedra (default 64^3: 811,200 free dofs), E = exp(0.5 z)
    per element, nu = 0.3, x = 0 face clamped, f ~ U(-1, 1) per dof; seeded
    graph-growing partition into subdomains of 2000-8000 dofs, overlap 1,
    12 generating vectors ({1, x, y, z} per component), rtol 1e-8.  The
    error of the FP32 and BF16 solutions is stated against the FP64 GPU path
    (the oracle is too slow at this size; the GPU FP64 path matches it on the
    smaller elasticity cases of the test suite).
    """
    import torch

    from paper_1504_00907_amd import DDGSolver
    from workloads.elasticity import elasticity_q1

    t0 = time.perf_counter()
    P = elasticity_q1(nel)
    log(f"elasticity: {nel}^3 elements, n = {P.n}, {P.n_parts} subdomains, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    f = torch.from_numpy(P.f).cuda()
    A = P.A.to_scipy()
    out = {"workload": f"elasticity_q1_{nel}^3_clamped", "n": P.n, "nnz": P.A.nnz, "subdomains": P.n_parts,
           "overlap": 1, "k": 12, "rtol": 1e-8}
    u64 = None
    for prec in ("fp64", "fp32", "bf16"):
        t0 = time.perf_counter()
        s = DDGSolver.from_problem(P, precision=prec, rtol=1e-8, tile=tile, block_target=block_target)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        u = torch.empty_like(f)
        s.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info = s.solve(f, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        uh = u.cpu().numpy()
        true_res = float(np.linalg.norm(P.f - A @ uh) / np.linalg.norm(P.f))
        hinfo = s.info()
        rec = {"ms_per_solve": ms, "iters": info["iters"], "true_rel_res": true_res,
               "setup_s": setup_s, "setup_ms_device": hinfo["setup_ms"], "factor_bytes": hinfo["factor_bytes"],
               "n_coarse": hinfo["n_coarse"], "colours": hinfo["n_colours"],
               "sweep_groups": hinfo["sweep_groups"], "sweep_bytes": hinfo["sweep_bytes"]}
        if prec == "fp64":
            u64 = uh
        else:
            rec["rel_diff_vs_fp64"] = float(np.linalg.norm(uh - u64) / np.linalg.norm(u64))
        out[prec] = rec
        log(f"elasticity {prec}: {ms:.1f} ms/solve, iters {info['iters']}, true res {true_res:.2e}, "
            f"setup {setup_s:.1f} s")
        s.close()
        del s
    return out


def three_level(P, precision: str, steps: int, group: int = 2):
    """Three-level V-cycle on the headline workload (Section 6, three-level paragraph).

    The 8^3 boxes are grouped 2^3 per coarse subdomain (64 coarse subdomains); the
    coarse level applies the two-level method to A0 with F0 = R0 F and overlap 1,
    in FP64.  Iterations and time per solve beside the two-level method's (Table 1
    compares the two: context, parity unpinned).
    """
    import torch

    from paper_1504_00907_amd import DDGSolver
    from workloads import box_groups

    m = round(P.n_parts ** (1 / 3))
    part0, n0 = box_groups((m, m, m), (group, group, group))
    f = torch.from_numpy(P.f).cuda()
    t0 = time.perf_counter()
    s = DDGSolver.from_problem(P, precision=precision, rtol=P.rtol, part0=part0, n_parts0=n0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    u = torch.empty_like(f)
    s.solve(f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = s.solve(f, u)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    uh = u.cpu().numpy()
    true_res = float(np.linalg.norm(P.f - P.A.to_scipy() @ uh) / np.linalg.norm(P.f))
    hi = s.info()
    s.close()
    rec = {"coarse_subdomains": n0, "group": group, "precision": precision, "ms_per_solve": ms,
           "iters": info["iters"], "true_rel_res": true_res, "n_coarse": hi["n_coarse"],
           "n_coarsest": hi["n_coarsest"], "setup_s": setup_s, "setup_ms_device": hi["setup_ms"]}
    log(f"three-level: {ms:.2f} ms/solve, iters {info['iters']}, true res {true_res:.2e}, "
        f"N_c {hi['n_coarse']} -> {hi['n_coarsest']}")
    return rec


def inexact(P, steps: int, omega: float = 1.0, sweeps: int = 1):
    """Section 7's inexact variant on the headline workload, FP64: the subdomains
    smoothed by symmetric SOR (no local factors) instead of solved exactly, first with
    the exact coarse inverse, then also with the incomplete-Cholesky-preconditioned CG
    coarse solve (inner tolerance 1e-6, Polak-Ribiere outer CG) as in the paper's
    timed runs.  Iterations, time per solve and setup beside the exact solves (context
    for Table 2: cheaper setup and memory, more iterations)."""
    import torch

    from paper_1504_00907_amd import DDGSolver

    f = torch.from_numpy(P.f).cuda()
    out = {"local_solver": "ssor", "omega": omega, "sweeps": sweeps, "precision": "fp64"}
    for label, kw in (("", {}), ("ic_cg", dict(coarse_solver="ic_cg", ic_tol=1e-6, ic_maxit=200, cg_variant="pr"))):
        t0 = time.perf_counter()
        s = DDGSolver.from_problem(P, precision="fp64", rtol=P.rtol, local_solver="ssor", ssor_omega=omega,
                                   ssor_sweeps=sweeps, **kw)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        u = torch.empty_like(f)
        s.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info = s.solve(f, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        uh = u.cpu().numpy()
        true_res = float(np.linalg.norm(P.f - P.A.to_scipy() @ uh) / np.linalg.norm(P.f))
        hi = s.info()
        s.close()
        rec = {"ms_per_solve": ms, "iters": info["iters"], "true_rel_res": true_res, "setup_s": setup_s,
               "setup_ms_device": hi["setup_ms"], "factor_bytes": hi["factor_bytes"],
               "coarse_bytes": hi["coarse_bytes"]}
        if label:
            rec.update(coarse_solver="ic_cg", ic_tol=1e-6, cg_variant="pr", inner_iters=info["coarse_iters"])
            log(f"ssor + ic-cg coarse solve: {ms:.2f} ms/solve, iters {info['iters']} ({info['coarse_iters']} inner "
                f"coarse iterations), true res {true_res:.2e}, setup {setup_s:.2f} s")
            out["ic_cg"] = rec
        else:
            log(f"ssor local smoothing: {ms:.2f} ms/solve, iters {info['iters']}, true res {true_res:.2e}, "
                f"setup {setup_s:.2f} s")
            out.update(rec)
    return out


def biharmonic(m: int, boxes: int, overlap: int, ps, steps: int):
    """Biharmonic high-p study (Section 7 problem F; Fig. 5's setting: m = 1000,
    H/h = 125, overlap 2, tolerance 1e-6), FP64 local factors: iterations, time
    and coarse size per degree p.  The iteration counts are context (Fig. 5's
    plotted values are not available)."""
    import torch

    from paper_1504_00907_amd import DDGSolver
    from workloads.biharmonic import biharmonic_problem

    out = {"workload": f"biharmonic13_{m}^2", "n": m * m, "subdomains": boxes * boxes, "overlap": overlap,
           "rtol": 1e-6, "precision": "fp64", "per_p": []}
    for p in ps:
        P = biharmonic_problem(m, boxes, overlap, p, rtol=1e-6)
        f = torch.from_numpy(P.f).cuda()
        t0 = time.perf_counter()
        s = DDGSolver.from_problem(P, precision="fp64", rtol=1e-6)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        u = torch.empty_like(f)
        _, info = s.solve(f, u, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info = s.solve(f, u, raise_on_error=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        uh = u.cpu().numpy()
        true_res = float(np.linalg.norm(P.f - P.A.to_scipy() @ uh) / np.linalg.norm(P.f))
        hi = s.info()
        rep = s.cg_report()
        s.close()
        fin = lambda x: float(x) if np.isfinite(x) else None  # noqa: E731
        rec = {"p": p, "k": int(P.F.shape[1]), "n_coarse": hi["n_coarse"], "iters": info["iters"],
               "frac_iters": fin(rep["frac_iters"]), "kappa_estimate": fin(rep["kappa"]),
               "iter_bound": rep["iter_bound"], "status": info["status_name"],
               "ms_per_solve": ms, "true_rel_res": true_res, "setup_s": setup_s,
               "matrix_format": _lib_format(hi), "coarse_refine": hi["coarse_refine"],
               "coarse_inverse_err": hi["coarse_inverse_err"]}
        out["per_p"].append(rec)
        log(f"biharmonic p={p}: k {rec['k']}, N_c {hi['n_coarse']}, iters {info['iters']}, {ms:.1f} ms/solve, "
            f"true res {true_res:.2e}")
        torch.cuda.empty_cache()
    return out


def materials(L: int, boxes: int, p: int, steps: int):
    """Two-material diffusion (Section 7 problem C) with plain and material-aware
    generating vectors (degree p, tolerance 1e-9, FP32 local factors): the paper
    reports close to half the iterations with the aware cubic basis (context)."""
    import torch

    from paper_1504_00907_amd import DDGSolver
    from workloads.materials import material_problem

    out = {"workload": f"two_material_{L}^2", "n": L * L, "subdomains": boxes * boxes, "p": p, "rtol": 1e-9}
    for aware in (False, True):
        P = material_problem(L, boxes, 1, p, aware)
        f = torch.from_numpy(P.f).cuda()
        s = DDGSolver.from_problem(P, precision="fp32", rtol=1e-9)
        u = torch.empty_like(f)
        s.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info = s.solve(f, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        hi = s.info()
        s.close()
        out["aware" if aware else "plain"] = {"k": int(P.F.shape[1]), "n_coarse": hi["n_coarse"],
                                             "iters": info["iters"], "ms_per_solve": ms}
        log(f"materials {'aware' if aware else 'plain'}: N_c {hi['n_coarse']}, iters {info['iters']}, {ms:.2f} ms")
    return out


def _lib_format(info: dict) -> str:
    return {1: "csr", 2: "dia"}.get(info.get("matrix_format"), "?")


def _batch_instance(arg):
    """Host arrays of one system of the batched workload (runs in a worker process)."""
    from workloads import cfg4_instance
    i, L = arg
    P = cfg4_instance(i, int(L))
    return (P.A.row_ptr, P.A.col_idx, P.A.val, np.asfortranarray(P.F), P.part, P.n_parts), P.f


def batched(count: int, precision: str, steps: int, warmup: int, persistent_leg: bool = True):
    """Batched leg: `count` independent 2D diffusion systems in one handle.

    Side lengths L ~ U{128..512} (seeded), L x L cells, kappa = exp(z) with z
    iid N(0, 1) per cell, f ~ U(-1, 1); near-equal boxes of about 32^2 cells
    (m = round(L/32) per axis), overlap 2, p = 3 (10 monomials), rtol 1e-8.
    The launch shape (tile edge, level merge target) comes from the library's
    autotuner on a sample of the batch.  Reports solves/s over the whole batch
    and the per-system device time to convergence (p50/p99), for the colour
    launches (systems in lockstep) and for the persistent schedule (one launch,
    systems advancing and stopping independently).
    """
    import multiprocessing as mp

    import torch

    from paper_1504_00907_amd import DDGBatchSolver, tune_batched
    from workloads import cfg4_sides

    sides = cfg4_sides(count)
    t0 = time.perf_counter()
    pool = mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1))
    try:
        res = pool.map(_batch_instance, list(enumerate(sides)), chunksize=4)
    finally:
        # let the workers exit on their own (no terminate signal on the way out)
        pool.close()
        pool.join()
    probs = [r[0] for r in res]
    f = torch.from_numpy(np.concatenate([r[1] for r in res])).cuda()
    del res
    gen_s = time.perf_counter() - t0
    log(f"batched: {count} systems, n = {f.numel()}, generated in {gen_s:.1f} s")
    t0 = time.perf_counter()
    tile, bt, cands = tune_batched(probs, 2, precision, max_sample=0)
    tune_s = time.perf_counter() - t0
    log(f"batched: autotuner chose tile {tile}, block_target {bt} in {tune_s:.1f} s")
    t0 = time.perf_counter()
    b = DDGBatchSolver(probs, 2, precision=precision, rtol=1e-8, tile=tile, block_target=bt)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = b.info()
    persist_probs = probs if persistent_leg else None
    del probs
    log(f"batched: setup {setup_s:.1f} s (device numeric {info['setup_ms']:.0f} ms)")
    u = torch.empty_like(f)
    for _ in range(warmup):
        b.solve(f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, infos = b.solve(f, u)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # the same steps again with an event pair on every local-solve dispatch, for the
    # sweep kernel's figures (the time above comes from the pass without events)
    b.profile_enable(True)
    b.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.solve(f, u)
    torch.cuda.synchronize()
    ms_ev = (time.perf_counter() - t0) * 1e3 / steps
    prof = b.profile_read(reset=True)
    b.profile_enable(False)
    # bytes are credited per system only for launches enqueued while it still iterated;
    # launches that ran for no system are counted apart (idle)
    sweep_gbs = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else 0.0
    per = np.array([i["solve_ms"] for i in infos])
    its = np.array([i["iters"] for i in infos])
    tres = np.array([i["true_rel_res"] for i in infos])
    ok = all(i["status"] == 0 for i in infos)
    u_colours = u.clone()
    b.close()
    log(f"batched: {ms:.1f} ms per batch solve, {count * 1e3 / ms:.1f} solves/s, iters {its.min()}..{its.max()}, "
        f"sweep kernel {sweep_gbs:.0f} GB/s")
    # the same batch with the persistent schedule: one launch per batch solve, every
    # system advancing through its own CG steps from a device task ring
    persistent = None
    if persist_probs is not None:
        t0 = time.perf_counter()
        bp = DDGBatchSolver(persist_probs, 2, precision=precision, rtol=1e-8, tile=tile, block_target=bt,
                            schedule="persistent")
        torch.cuda.synchronize()
        psetup_s = time.perf_counter() - t0
        up = torch.empty_like(f)
        for _ in range(warmup):
            bp.solve(f, up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, pinfos = bp.solve(f, up)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / steps
        pper = np.array([i["solve_ms"] for i in pinfos])
        pits = np.array([i["iters"] for i in pinfos])
        same = bool(torch.equal(up, u_colours))
        bp.close()
        log(f"batched persistent: {pms:.1f} ms per batch solve, {count * 1e3 / pms:.1f} solves/s, per-system "
            f"p50 {np.percentile(pper, 50):.1f} ms p99 {np.percentile(pper, 99):.1f} ms, same u as colour launches: {same}")
        persistent = {"ms_per_batch": pms, "solves_per_s": count * 1e3 / pms,
                      "system_ms_p50": float(np.percentile(pper, 50)),
                      "system_ms_p99": float(np.percentile(pper, 99)),
                      "system_ms_min": float(pper.min()), "system_ms_max": float(pper.max()),
                      "iters_min": int(pits.min()), "iters_max": int(pits.max()),
                      "all_converged": all(i["status"] == 0 for i in pinfos),
                      "same_u_as_colour_launches": same, "setup_s": psetup_s}
    return {
        "persistent": persistent,
        "workload": f"batch{count}_diffusion2d_L128-512_kappa_lognormal",
        "systems": count, "n_total": int(f.numel()), "subdomains": int(info["n_parts"]), "overlap": 2, "p": 3,
        "precision": precision, "rtol": 1e-8, "steps": steps,
        "ms_per_batch": ms, "solves_per_s": count * 1e3 / ms,
        "solves_per_s_incl_setup": count / (ms * 1e-3 + setup_s),
        "system_ms_p50": float(np.percentile(per, 50)), "system_ms_p99": float(np.percentile(per, 99)),
        "iters_min": int(its.min()), "iters_median": float(np.median(its)), "iters_max": int(its.max()),
        "max_true_rel_res": float(tres.max()), "all_converged": ok,
        "setup_s": setup_s, "setup_ms_device": info["setup_ms"], "generate_s": gen_s,
        "tuned": {"tile": tile, "block_target": bt, "tune_s": tune_s,
                  "candidates": [{"tile": c[0], "block_target": c[1], "precond_ms": c[2], "factor_bytes": c[3]}
                                 for c in cands]},
        "factor_bytes": info["factor_bytes"], "iter_bytes": info["iter_bytes"],
        "sweep_kernel": {"achieved_GBps": round(sweep_gbs, 1), "frac": round(sweep_gbs / HBM_PEAK_GBS, 4),
                         "launches": prof["launches"],
                         "avg_launch_us": prof["ms"] * 1e3 / prof["launches"] if prof["launches"] else None,
                         "idle_launches": prof["idle_launches"],
                         "idle_avg_us": (prof["idle_ms"] * 1e3 / prof["idle_launches"]
                                         if prof["idle_launches"] else None),
                         "share_of_solve": (prof["ms"] + prof["idle_ms"]) / (ms_ev * steps),
                         "ms_per_batch_with_events": ms_ev},
    }


def fwd_adjoint(side: int, precision: str, steps: int, warmup: int):
    """Forward + adjoint pairs per second on the differentiation workload.

    side^3 cells (default 96^3), kappa = exp(theta) with theta a GRF (length 8,
    sigma 1), 12^3-cell boxes, overlap 1, p = 2, rtol 1e-10; L = ||u - u_obs||^2
    with u_obs solved from a second seeded field.  One pair = device assembly of
    A(exp(theta)) + numeric refactor (Galerkin product, coarse inverse, local
    factors) + forward solve + adjoint solve + coefficient-gradient kernel,
    all through torch.autograd.
    """
    import torch

    from paper_1504_00907_amd import DiffusionSolver, ddg_solve_fn
    from workloads import box_partition, cell_coords, grf, monomials, seed_rng

    shape = (side,) * 3
    boxes = (side // 12,) * 3
    theta = grf(shape, 8.0, 1.0, seed_rng(4, 1))
    theta_obs = grf(shape, 8.0, 1.0, seed_rng(4, 2))
    fh = seed_rng(4, 0).uniform(-1.0, 1.0, side ** 3)
    part = box_partition(shape, boxes)
    F = monomials(cell_coords(shape), 2)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).cuda()
    log(f"fwd+adjoint workload {side}^3, boxes {boxes}")
    ds = DiffusionSolver((side,) * 3, F, part, int(np.prod(boxes)), 1, dev(theta_obs), precision=precision,
                         rtol=1e-10)
    f = dev(fh)
    u_obs = ds.solve(f).clone()
    th = dev(theta)

    def pair():
        t = th.clone().requires_grad_(True)
        u = ddg_solve_fn(t, f, ds)
        fwd = ds.last_info
        L = ((u - u_obs) ** 2).sum()
        L.backward()
        return fwd, ds.last_info, t.grad

    for _ in range(warmup):
        pair()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fwd, adj, g = pair()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps

    # the same pairs on a handle that already holds A(exp(theta)) (no refactor)
    def pair_kept():
        t = th.clone().requires_grad_(True)
        u = ddg_solve_fn(t, f, ds, refactor=False)
        L = ((u - u_obs) ** 2).sum()
        L.backward()
        return t.grad

    pair_kept()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pair_kept()
    torch.cuda.synchronize()
    ms_kept = (time.perf_counter() - t0) * 1e3 / steps
    # refactor alone
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ds.refactor(th)
    torch.cuda.synchronize()
    ref_ms = (time.perf_counter() - t1) * 1e3
    info = ds.solver.info()
    g_host = g.detach().cpu().numpy().copy()
    # central differences of L at the exact perturbed solves (residual correction
    # u+- = u0 + A+-^{-1} (f - A+- u0), each correction solved by the same DDG-PCG)
    t_fd = time.perf_counter()
    u0 = ddg_solve_fn(th, f, ds).detach().clone()
    cells = seed_rng(4, 5).choice(side ** 3, size=32, replace=False)
    h = 1e-6
    fd = []
    for c in cells:
        deltas = []
        for sgn in (1.0, -1.0):
            tp = th.clone()
            tp[int(c)] += sgn * h
            ds.refactor(tp)
            deltas.append(ds.solve(f - ds.solver.spmv(u0)))
        dp, dm = deltas
        fd.append(float(torch.dot(dp - dm, 2.0 * u0 + dp + dm - 2.0 * u_obs)) / (2.0 * h))
    fd = np.array(fd)
    gc = g_host[cells]
    big = np.abs(gc) >= 1e-3 * np.abs(g_host).max()
    fd_rel = np.abs(fd - gc) / np.abs(gc)
    t_fd = time.perf_counter() - t_fd
    ds.solver.close()
    log(f"fwd+adjoint: {ms:.1f} ms/pair (refactor {ref_ms:.1f} ms; {ms_kept:.1f} ms without), "
        f"iters {fwd['iters']} + {adj['iters']}, FD max rel err {fd_rel[big].max():.2e} ({t_fd:.1f} s)")
    return {
        "workload": f"diffusion3d_{side}^3_exp_theta_L2_loss", "n": side ** 3, "subdomains": int(np.prod(boxes)),
        "precision": precision, "rtol": 1e-10, "steps": steps,
        "pairs_per_s": 1e3 / ms, "ms_per_pair": ms, "refactor_ms": ref_ms,
        "pairs_per_s_without_refactor": 1e3 / ms_kept, "ms_per_pair_without_refactor": ms_kept,
        "solve_ms_fwd": fwd["solve_ms"], "solve_ms_adj": adj["solve_ms"],
        "iters_fwd": fwd["iters"], "iters_adj": adj["iters"], "setup_ms_device": info["setup_ms"],
        "grad_norm": float(np.linalg.norm(g_host)),
        "fd_check": {"cells": 32, "step": h, "protocol": "central difference of the exact perturbed solves "
                     "(residual correction)", "max_rel_err": float(fd_rel[big].max()),
                     "cells_relative": int(big.sum()),
                     "max_abs_err_small_cells_over_gmax": (float(np.abs(fd - gc)[~big].max() / np.abs(g_host).max())
                                                           if (~big).any() else None)},
        "_grad": g_host,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--box", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward+adjoint (differentiation) leg")
    ap.add_argument("--adjoint-side", type=int, default=96)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg (256 uneven 2D systems)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--no-elasticity", action="store_true", help="skip the 3D Q1 elasticity leg")
    ap.add_argument("--no-three-level", action="store_true", help="skip the three-level V-cycle leg")
    ap.add_argument("--no-biharmonic", action="store_true", help="skip the biharmonic high-p leg")
    ap.add_argument("--biharmonic-m", type=int, default=1000)
    ap.add_argument("--biharmonic-boxes", type=int, default=8)
    ap.add_argument("--biharmonic-p", default="1,2,3,4,6,8,10")
    ap.add_argument("--no-materials", action="store_true", help="skip the two-material leg")
    ap.add_argument("--no-inexact", action="store_true", help="skip the SSOR local smoothing leg")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the forward+adjoint leg and print its record (for profiling the refactor)")
    ap.add_argument("--elasticity-only", action="store_true",
                    help="run only the 3D elasticity leg and print its record")
    ap.add_argument("--elasticity-nel", type=int, default=64)
    ap.add_argument("--elasticity-tile", type=int, default=0)
    ap.add_argument("--elasticity-block-target", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--tile", type=int, default=0, help="tile edge of the local factors (0: automatic)")
    ap.add_argument("--block-target", type=int, default=0, help="level merge target (0: merge only tiny levels)")
    ap.add_argument("--tune", action="store_true", help="choose tile and merge target with the library's autotuner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "sharding is a design note only.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1504_00907_amd import DDGSolver
    from workloads import cfg2

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            b.copy_(a)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 10
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                          "copy_ms": ms, "copy_GBps": 2 * a.numel() * 8 / ms / 1e6}), flush=True)
        return
    if args.elasticity_only:
        print(json.dumps({"elasticity": elasticity(args.elasticity_nel, max(1, args.steps // 2), args.elasticity_tile,
                                                   args.elasticity_block_target)}), flush=True)
        return
    if args.adjoint_only:
        adj = fwd_adjoint(args.adjoint_side, args.precision, max(1, args.steps), 1)
        adj.pop("_grad", None)
        print(json.dumps({"fwd_adjoint": adj}), flush=True)
        return
    log(f"generating workload {args.side}^3, boxes {args.box}^3")
    P = cfg2(side=args.side, box=args.box)
    f = torch.from_numpy(P.f).cuda()
    A = P.A.to_scipy()

    tile_bt = (args.tile, args.block_target)
    tuned = None
    if args.tune:
        from paper_1504_00907_amd import tune_batched
        t0 = time.perf_counter()
        tt, bt, cands = tune_batched([(P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts)], P.overlap,
                                     args.precision, max_sample=1)
        tile_bt = (tt, bt)
        tuned = {"tile": tt, "block_target": bt, "tune_s": time.perf_counter() - t0,
                 "candidates": [{"tile": c[0], "block_target": c[1], "precond_ms": c[2]} for c in cands]}
        log(f"autotuner: tile {tt}, block_target {bt} ({tuned['tune_s']:.1f} s): {cands}")

    def setup(precision, schedule="auto"):
        t0 = time.perf_counter()
        s = DDGSolver.from_problem(P, precision=precision, rtol=P.rtol, tile=tile_bt[0], block_target=tile_bt[1],
                                   schedule=schedule)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        log(f"setup {precision}: wall {wall:.2f} s, device numeric {s.info()['setup_ms']:.1f} ms")
        return s, wall

    def timed(s, steps, warmup, profile):
        u = torch.empty_like(f)
        for _ in range(warmup):
            s.solve(f, u)
        if profile:
            s.profile_enable(True)
            s.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = None
        for _ in range(steps):
            _, info = s.solve(f, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        prof = s.profile_read(reset=True) if profile else None
        if profile:
            s.profile_enable(False)
        uh = u.cpu().numpy()
        true_res = float(np.linalg.norm(P.f - A @ uh) / np.linalg.norm(P.f))
        return ms, info, prof, uh, true_res

    smx, setup_wall_mx = setup(args.precision)
    log("timing mixed path")
    ms_mx, info_mx, _, u_mx, res_mx = timed(smx, args.steps, args.warmup, profile=False)
    log(f"mixed: {ms_mx:.2f} ms/solve, iters {info_mx['iters']}, true res {res_mx:.2e}")
    # the same K steps again with a HIP event pair on every local-solve dispatch
    # (`value` comes from the pass above, which records no events)
    ms_ev, _, prof, _, _ = timed(smx, args.steps, 0, profile=True)
    log(f"mixed with per-launch events: {ms_ev:.2f} ms/solve")
    hinfo = smx.info()
    smx.close()
    del smx
    torch.cuda.empty_cache()

    # the same solve with the other sweep schedule (the library's automatic choice is
    # one launch per colour phase): one launch per sweep direction over the task queue
    sq, _ = setup(args.precision, "queue")
    ms_q, info_q, _, u_q, _ = timed(sq, max(1, args.steps // 2), 1, profile=False)
    sq.close()
    del sq
    torch.cuda.empty_cache()
    alt = {"schedule": "task queue", "ms_per_solve": ms_q, "iters": info_q["iters"],
           "same_u": bool(np.array_equal(u_q, u_mx)),
           "max_rel_diff_u": float(np.abs(u_q - u_mx).max() / np.abs(u_mx).max())}
    log(f"task-queue schedule: {ms_q:.2f} ms/solve, iters {info_q['iters']}, same u: {alt['same_u']} "
        f"(max rel diff {alt['max_rel_diff_u']:.1e})")

    out64 = {}
    if not args.no_fp64:
        s64, setup_wall_64 = setup("fp64")
        log("timing fp64 path")
        ms_64, info_64, _, u_64, res_64 = timed(s64, max(1, args.steps), args.warmup, profile=False)
        log(f"fp64: {ms_64:.2f} ms/solve, iters {info_64['iters']}, true res {res_64:.2e}")
        out64 = {
            "fp64_ms_per_solve": ms_64, "fp64_iters": info_64["iters"], "fp64_true_rel_res": res_64,
            "fp64_setup_ms": info_64["setup_ms"], "mixed_speedup_vs_fp64": ms_64 / ms_mx,
            "mixed_vs_fp64_rel_diff": float(np.linalg.norm(u_mx - u_64) / np.linalg.norm(u_64)),
        }
        s64.close()
        del s64
        if args.precision != "bf16":
            # BF16 factors on the same system (tried and reported; FP64 Krylov vectors and coarse inverse)
            sbf, _ = setup("bf16")
            log("timing bf16 path")
            ms_bf, info_bf, _, u_bf, res_bf = timed(sbf, max(1, args.steps), args.warmup, profile=False)
            log(f"bf16: {ms_bf:.2f} ms/solve, iters {info_bf['iters']}, true res {res_bf:.2e}")
            out64.update({
                "bf16_ms_per_solve": ms_bf, "bf16_iters": info_bf["iters"], "bf16_true_rel_res": res_bf,
                "bf16_vs_fp64_rel_diff": float(np.linalg.norm(u_bf - u_64) / np.linalg.norm(u_64)),
            })
            sbf.close()
            del sbf

    lvl3 = None
    if not args.no_three_level:
        lvl3 = three_level(P, args.precision, max(1, args.steps // 2))
        lvl3["two_level_ms_per_solve"] = ms_mx
        lvl3["two_level_iters"] = info_mx["iters"]
        torch.cuda.empty_cache()

    inx = None
    if not args.no_inexact:
        inx = inexact(P, max(1, args.steps // 2))
        inx["exact_fp64_ms_per_solve"] = out64.get("fp64_ms_per_solve")
        inx["exact_iters"] = info_mx["iters"]
        torch.cuda.empty_cache()

    bih = None
    if not args.no_biharmonic:
        bih = biharmonic(args.biharmonic_m, args.biharmonic_boxes, 2,
                         [int(x) for x in args.biharmonic_p.split(",") if x], 1)
        torch.cuda.empty_cache()

    mat = None
    if not args.no_materials:
        mat = materials(512, 16, 3, max(1, args.steps // 2))
        torch.cuda.empty_cache()

    ela = None
    if not args.no_elasticity:
        ela = elasticity(args.elasticity_nel, max(1, args.steps // 2), args.elasticity_tile,
                         args.elasticity_block_target)
        torch.cuda.empty_cache()

    bat = None
    if not args.no_batch:
        bat = batched(args.batch_count, args.precision, max(1, args.steps // 2), 1)
        torch.cuda.empty_cache()

    adj = None
    if not args.no_adjoint:
        adj = fwd_adjoint(args.adjoint_side, args.precision, max(1, args.steps // 2), 1)
        torch.cuda.empty_cache()

    achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof and prof["ms"] > 0 else 0.0
    sweep_kernel = "k_sweep_flow" if hinfo["schedule"] == 2 else "k_sweep"
    avg_s = prof["ms"] * 1e-3 / prof["launches"] if prof and prof["launches"] else None
    # the survey's count of the same launches: factors at the envelope size E (every
    # local matrix's envelope, where a banded Cholesky factor's fill stays), two
    # substitutions per launch, plus the gathers (r and e on each set and its one-ring,
    # a symmetric 7-point row of 32 bytes, e read and written): per launch the average
    # over the 2C launches of one application
    s_f = {"fp32": 4, "bf16": 2, "fp64": 8}[args.precision]
    E, Nhat, Srows, C2 = hinfo["envelope_elems"], hinfo["nbhd_rows"], hinfo["set_rows"], 2 * hinfo["n_colours"]
    survey_app = 4 * E * s_f + 2 * (Nhat * 16 + Srows * (32 + 16))
    survey_launch = survey_app / C2
    traffic = (profiled_traffic(sweep_kernel, args.precision, hinfo["tile"])
               if args.side == 128 and args.box == 16 else None)
    roofline = {
        "bound": "hbm",
        "kernel": sweep_kernel + (" (one sweep direction over the task queue)" if sweep_kernel == "k_sweep_flow"
                                  else " (one colour phase)"),
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "frac_counters": (round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic and avg_s else None),
        "frac_survey": round(survey_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4) if avg_s else None,
        "survey_bytes_per_launch": survey_launch,
        "launches": prof["launches"] if prof else 0,
        "idle_launches": prof["idle_launches"] if prof else 0,
        "idle_avg_us": (prof["idle_ms"] * 1e3 / prof["idle_launches"]) if prof and prof["idle_launches"] else None,
        "avg_launch_us": avg_s * 1e6 if avg_s else None,
        "bytes_per_launch": (prof["bytes"] / prof["launches"]) if prof and prof["launches"] else None,
        "kernel_share_of_solve": ((prof["ms"] + prof["idle_ms"]) / (ms_ev * args.steps)) if prof else None,
        "timed_pass": "a second pass of the same K solves with a HIP event pair attached to each launch's dispatch; "
                      "launches enqueued after convergence ran for no system and are counted apart (idle)",
        "ms_per_step_with_events": round(ms_ev, 3),
    }
    whole = hinfo["iter_bytes"] * info_mx["iters"] / (ms_mx * 1e-3) / 1e9
    # the survey's bytes of one whole CG iteration: the sweeps above, the coarse step
    # (residual SpMV, Q^T s, the dense inverse read twice as two triangular solves would,
    # e += Q y) and the CG SpMV and vector updates
    n, k, Nc = P.n, 10, hinfo["n_coarse"]
    survey_iter = (survey_app + P.n * (16 + 32) + 2 * n * k * 8 + 2 * (Nc * (Nc + 1) // 2) * 8 + 16 * n
                   + n * (16 + 32) + 10 * n * 8)
    whole_survey = survey_iter * info_mx["iters"] / (ms_mx * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline (bounded sample)")
        cpu = cpu_baseline(P, info_mx["iters"])
        log(f"oracle estimate {cpu['value']:.0f} ms/solve ({cpu['single_thread_ms']:.0f} ms single-threaded)")
        if adj is not None:
            log("oracle forward + adjoint + gradient on the differentiation workload")
            cf = cpu_fwd_adjoint(args.adjoint_side, adj["_grad"])
            adj["grad_rel_err_vs_oracle"] = cf["grad_rel_err_vs_oracle"]
            cpu["fwd_adjoint"] = cf
            log(f"oracle gradient {cf['oracle_s']:.1f} s; GPU gradient rel err {cf['grad_rel_err_vs_oracle']:.2e}")
    if adj is not None:
        adj.pop("_grad", None)
    rec = {
        "metric": METRIC,
        "value": round(ms_mx, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_mx, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.precision == "fp32" else ("f64+bf16" if args.precision == "bf16" else "f64"),
        "data": "synthetic",
        "config": {
            "workload": f"diffusion3d_{args.side}^3_variable_kappa",
            "n": P.n, "subdomains": P.n_parts, "box": args.box, "overlap": P.overlap, "p": 2,
            "n_coarse": hinfo["n_coarse"], "colours": hinfo["n_colours"], "rtol": P.rtol,
            "precision": args.precision, "schedule": "task queue" if hinfo["schedule"] == 2 else "colour launches",
            "parallelism": "single GPU",
        },
        "iters": info_mx["iters"],
        "true_rel_res": res_mx,
        "solves_per_s": 1e3 / ms_mx,
        "setup_ms": hinfo["setup_ms"],
        "setup_wall_s": setup_wall_mx,
        "factor_bytes": hinfo["factor_bytes"],
        "iter_bytes": hinfo["iter_bytes"],
        "whole_solve_GBps": round(whole, 1),
        "whole_solve_frac": round(whole / HBM_PEAK_GBS, 4),
        "whole_solve_frac_survey": round(whole_survey / HBM_PEAK_GBS, 4),
        "survey_iter_bytes": survey_iter,
        "envelope_elems": E,
        **out64,
        "matrix_format": _lib_format(hinfo),
        "fwd_adjoint": adj,
        "three_level": lvl3,
        "inexact": inx,
        "biharmonic": bih,
        "materials": mat,
        "batched": bat,
        "elasticity": ela,
        "tuned": tuned,
        "other_schedule": alt,
        "roofline": roofline,
        "setup_mfma": profiled_mfma() if args.side == 128 and args.box == 16 else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
