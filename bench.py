#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on one synthetic problem.

Workload (default): 2-D Poisson on the five-armed star r = 0.3 + 0.1 cos(5 phi)
in [-0.5, 0.5]^2 with 2048 x 2048 cells (2049^2 nodes, 1,246,505 unknowns),
manufactured u = exp(x) sin(4 pi y), plain FP64 AMG-PCG to relative residual
1e-8.  psi and f are resident in HBM before timing starts; each step runs
  classification + diagonal + cut records -> boundary data at the crossings
  -> right-hand side -> AMG setup -> PCG solve
entirely in the library's HIP kernels, and frees the hierarchy.

Output: one JSON line (rank 0).  `value` = unknowns x CG iterations per second
of whole-step time for the plain FP64 path.  `roofline` reports the dominant
solve kernel: its algorithmic bytes per launch over its average launch time,
measured with HIP events on the library's stream inside the timed steps.
`solve_roofline` applies the whole-solve byte model to the measured solve
time.  `mixed` repeats the same steps with the single-precision V-cycle
(FP64 outer CG) and reports its difference from the FP64 solution.
`batched` times one backward-Euler heat step on the star 1024^2 for 64 seeded
initial conditions as one batched solve (pcg_solve_batched) and as 64 single
solves on the same hierarchy.  `learned_3d` solves the 3-D ellipsoid 256^3
Poisson problem with the plain and the learned fine smoother (network trained
on the GPU at 96^3), both V-cycle precisions.  `islands` runs the
shape-optimisation batch (256 random stars, N in {256 .. 1024}, 4 sources
each) as one island solve (pcg_solve_islands: one canvas, one hierarchy,
one launch sequence; timed from assembly to solution) and geometry by
geometry.  `qoi` runs the two shape-parameter studies of Sec. 3.6 (61
fixed-area ellipses at 1024^2, 64 rotated ellipses on the 501^2 grid), each
as one island batch from level sets to quantities of interest.
`disk_latency` reports the latency of the 128^2 disk problem (FP64 to 1e-10).
`wave_stencil` times stencil_apply and eb_wave_rhs on Table 1's 1600^2 grid
against the HBM roofline and runs Table 1's leap-frog column there.
`learned_3d` carries the whole-solve byte model's roofline fraction of the
plain 3-D solves.  `cpu_baseline` times the CPU oracle on full steps of the
same workload (BLAS on one thread and on every usable core), and the heat and
island batches over a process pool (it runs before the GPU is first used).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--kernel NAME]
       python bench.py --copy-calib    (plain copy kernel for counter scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per launch of the timed solve kernels (FP64 values, int32
# ids; every array touched once per launch), from the fine unknowns n0, the
# level-1 unknowns n1 and the dimension.  2-D runs the band-tile kernels:
#   pcg_spmv     p = z + beta p_old; q = A p; (p, q): read z, p_old, d; write p, q
#   pcg_xr_down  x += alpha p; r = r - alpha q; ||r||^2; pre-smoothing residual
#                and restriction: read x, p, r_in, q, 1/d; write x, r; per
#                level-0 box (one per coarse unknown) its aggregate count, first
#                aggregate, node map and omega_1/d_1 (20 B); write r_c, omega r_c/d_c
#   fine_post    prolongation + both smoothing halves + (r, z): read aggregate
#                id (4 B), 1/d, r; gather e_c; write z
# 3-D runs the strip kernels (pcg_xr_down: read x, p, r_in, q, d; write x, r,
# res; fine_post: read z_t, r, d; write z).
def kernel_bytes(name, n0, n1, dim):
    if name == "pcg_spmv":
        return 40.0 * n0
    if name == "pcg_xr_down":
        return 56.0 * n0 + 36.0 * n1 if dim == 2 else 64.0 * n0
    if name == "fine_post":
        return 28.0 * n0 + 8.0 * n1 if dim == 2 else 32.0 * n0
    raise KeyError(name)


TIMED_KERNELS = ("pcg_spmv", "pcg_xr_down", "fine_post")
# blocks of the bench line besides the headline steps, by name (filled in
# below their definitions)
BLOCKS = {}
MALL_BYTES = 256 << 20   # the MI355X Infinity Cache


def design_model_bytes(H):
    """Whole-solve bytes per PCG iteration by the design model of the hot-path
    scope table: fine level 40 + 48 + (20 + 8 n1/n0) + (28 + 8 n1/n0) B per
    unknown (p-update + SpMV, x/r update, restriction, prolongation +
    post-smoothing), each coarse level 2 (12 nnz_A + 4 n) + 12 (nnz_P + nnz_R)
    + 60 n, the coarsest its dense inverse."""
    n0 = H.level(0).n
    n1 = H.level(1).n if H.n_levels > 1 else 0
    total = 136.0 * n0 + 16.0 * n1
    for l in range(1, H.n_levels):
        lv = H.level(l)
        if lv.is_coarsest:
            total += 8.0 * lv.n * lv.n + 16.0 * lv.n
        else:
            total += 2 * (12.0 * lv.nnz_a + 4.0 * lv.n) + 12.0 * (lv.nnz_p + lv.nnz_r) + 60.0 * lv.n
    return total


def impl_model_bytes(H, precision, dim):
    """Bytes per PCG iteration of the kernels this library launches, each array
    once per launch: the fine kernels above, then per coarse level the down
    pass (R and R A, rv and sv, rv_c and sv_c) and the up pass (sliced A, P,
    A P; sv, rv, d, e_c; e), the coarsest its dense inverse (FP64 in both
    V-cycle precisions)."""
    vb = 8.0 if precision == "fp64" else 4.0               # coarse values and vectors
    zb = {"fp64": 8.0, "fp32": 4.0, "bf16": 2.0}[precision]  # z, and 1/d of the post-smoothing
    n0 = H.level(0).n
    n1 = H.level(1).n if H.n_levels > 1 else 0
    if dim == 2:
        # p-update: z, p, d read, p, q written; x/r update with restriction:
        # x, p, r, q, 1/d read, x, r written, r_c and sv_c per coarse row; up
        # pass: aggregate id, r, 1/d, e_c read, z written (CG vectors FP64)
        total = (32.0 + zb) * n0 + (56.0 * n0 + (20.0 + 2 * vb) * n1) + (12.0 + 2 * zb) * n0 + vb * n1
    else:
        total = {"fp64": 184.0, "fp32": 148.0, "bf16": 146.0}[precision] * n0
    for l in range(1, H.n_levels):
        lv = H.level(l)
        if lv.is_coarsest:
            total += 8.0 * lv.n * lv.n + 2 * vb * lv.n
            continue
        nc = H.level(l + 1).n
        nap = lv.info.nnz_ap
        down = (vb + 4) * (lv.nnz_r + nap) + 4.0 * 2 * (nc + 1) + 2 * vb * lv.n + 2 * vb * nc
        up = (vb + 4) * (lv.nnz_a + lv.nnz_p + nap) + 4 * vb * lv.n + vb * nc
        total += down + up
    return total


def working_set_bytes(H, dim):
    """Distinct bytes one PCG iteration touches: the fine fields read or written
    (x, two residuals, two search directions, q, z, d, 1/d: 8 B each; aggregate
    ids 4 B) over the active unknowns, every coarse matrix and vector, the
    coarsest inverse."""
    n0 = H.level(0).n
    total = (9 * 8.0 + 4.0) * n0
    for l in range(1, H.n_levels):
        lv = H.level(l)
        if lv.is_coarsest:
            total += 8.0 * lv.n * lv.n + 16.0 * lv.n
        else:
            total += 12.0 * (lv.nnz_a + lv.nnz_p + lv.nnz_r + 2 * lv.info.nnz_ap) + 48.0 * lv.n
    return total


def batched_heat(n=1024, nrhs=64, reps=3):
    """One backward-Euler step of the heat workload for nrhs seeded initial
    conditions: one batched solve vs nrhs single solves (same hierarchy)."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"
    g = W.unit_box_grid(2, n)
    dt = g.h
    psi = torch.as_tensor(W.psi_star(g), device=dev)
    asm = S.assemble_diag(g, psi)
    zero = torch.zeros(asm.n_cuts, dtype=torch.float64, device=dev)
    u0 = W.heat_initial_batch(g, range(nrhs), dev)
    B = torch.stack([S.assemble_rhs(asm, (u0[j] / dt).contiguous(), zero) for j in range(nrhs)]).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = S.Hierarchy(g, asm.kind, asm.a, 1.0 / dt)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    out = {"workload": f"star2d_{n}_heat_backward_euler_dt_h_{nrhs}rhs", "n_unknowns": asm.n_unknowns, "nrhs": nrhs,
           "setup_ms": setup_ms}
    for prec in ("fp32", "fp64"):
        H.solve_batched(B, tol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            X, infos = H.solve_batched(B, tol=1e-8, precision=prec)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        its = [i["iterations"] for i in infos]
        H.solve(B[0].contiguous(), tol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sits = 0
        for j in range(nrhs):
            _, i = H.solve(B[j].contiguous(), tol=1e-8, precision=prec)
            sits += i["iterations"]
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        shape = S.batched_launch_shape(H)
        out[prec] = {"batch_ms": tb * 1e3, "solves_per_s": nrhs / tb, "launch_shape": shape,
                     "unknowns_iters_per_s": asm.n_unknowns * sum(its) / tb,
                     "iterations_min_max": [min(its), max(its)],
                     "rel_res_true_max": max(i["rel_res_true"] for i in infos),
                     "sequential_ms": ts * 1e3, "sequential_solves_per_s": nrhs / ts,
                     "speedup_vs_sequential": ts / tb}
    H.free()
    return out


def heat_steps(n=1024, nrhs=64, nsteps=200):
    """The heat workload as stated: nsteps backward-Euler steps (dt = h) of nrhs
    seeded initial conditions on the star at n^2, every step one batched solve
    of all right-hand sides warm-started from the previous step, in both
    V-cycle precisions; setup once."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"
    g = W.unit_box_grid(2, n)
    dt = g.h
    psi = torch.as_tensor(W.psi_star(g), device=dev)
    asm = S.assemble_diag(g, psi)
    u0 = W.heat_initial_batch(g, range(nrhs), dev)
    H = S.Hierarchy(g, asm.kind, asm.a, 1.0 / dt)
    out = {"workload": f"star2d_{n}_heat_backward_euler_dt_h_{nrhs}rhs_{nsteps}steps_warm_start",
           "n_unknowns": asm.n_unknowns, "nrhs": nrhs, "steps": nsteps}
    finals = {}
    for prec in ("fp32", "fp64"):
        S.heat_backward_euler_batched(asm, H, u0, dt, 2, precision=prec)     # warm-up (tuning, FP32 copies)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, its = S.heat_backward_euler_batched(asm, H, u0, dt, nsteps, precision=prec)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        flat = [i for row in its for i in row]
        finals[prec] = u
        out[prec] = {"seconds": secs, "ms_per_step": secs * 1e3 / nsteps,
                     "solves_per_s": nrhs * nsteps / secs,
                     "unknowns_iters_per_s": asm.n_unknowns * sum(flat) / secs,
                     "iterations_min_mean_max": [min(flat), sum(flat) / len(flat), max(flat)],
                     "launch_shape": S.batched_launch_shape(H)}
    out["rel_diff_fp32_vs_fp64_final"] = (torch.linalg.vector_norm(finals["fp32"] - finals["fp64"]) /
                                          torch.linalg.vector_norm(finals["fp64"])).item()
    out["fp32_speedup"] = out["fp64"]["seconds"] / out["fp32"]["seconds"]
    H.free()
    return out


def learned_ellipsoid(n=256, n_train=96, steps=120, reps=3):
    """The 3-D ellipsoid Poisson problem: plain Jacobi AMG-PCG against the
    learned fine smoother (network trained on the GPU on the same ellipsoid at
    n_train^3 and applied at n^3), FP64 and single-precision V-cycles."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"

    def build(m):
        p = W.ellipsoid_poisson(m)
        psi = torch.as_tensor(p.psi, device=dev)
        f = torch.as_tensor(p.f, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        asm = S.assemble_diag(p.grid, psi)
        b = S.assemble_rhs(asm, f, torch.as_tensor(p.u_dirichlet(*asm.cut_coordinates()), device=dev))
        H = S.Hierarchy(p.grid, asm.kind, asm.a, 0.0)
        torch.cuda.synchronize()
        return p, psi, asm, b, H, (time.perf_counter() - t0) * 1e3

    def timed(H, b, prec):
        H.solve(b, tol=1e-8, precision=prec)
        ms, its = [], 0
        for _ in range(reps):
            _, info = H.solve(b, tol=1e-8, precision=prec)
            ms.append(info["solve_ms"])
            its = info["iterations"]
        return {"iterations": its, "solve_ms": sorted(ms)[len(ms) // 2]}

    pt, psit, asmt, bt, Ht, _ = build(n_train)
    ls = S.LearnedSmoother(Ht, asmt, psit, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ls.fit(steps=steps, samples=4, sweeps=6, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    params, gl = ls.params.cpu().numpy(), dict(ls.g)
    Ht.free()
    p, psi, asm, b, H, setup_ms = build(n)
    out = {"workload": f"ellipsoid3d_{n}_poisson_tol1e-8", "n_unknowns": asm.n_unknowns, "levels": H.n_levels,
           "assembly_rhs_setup_ms": setup_ms,
           "training": {"grid": f"{n_train}^3", "steps": steps, "seconds": train_s,
                        "loss_first": hist[0], "loss_last5_mean": sum(hist[-5:]) / 5,
                        "level_weight_multipliers": {str(k): v for k, v in gl.items()}}}
    sm, wset = design_model_bytes(H), working_set_bytes(H, 3)
    for prec in ("fp64", "fp32"):
        r = timed(H, b, prec)
        gbs = sm * r["iterations"] / (r["solve_ms"] * 1e-3) / 1e9
        r["solve_roofline"] = {"bound": "hbm", "model": "design", "bytes_per_iter": sm, "achieved": gbs,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                               "mall_resident": wset < MALL_BYTES, "working_set_bytes": wset}
        out[f"plain_{prec}"] = r
    la = S.LearnedSmoother(H, asm, psi, params=params)
    la.g = dict(gl)
    la.apply()
    la.apply_levels(gl)
    for prec in ("fp64", "fp32"):
        out[f"learned_{prec}"] = timed(H, b, prec)
    out["selection"] = la.select(b, tol=1e-8)
    out["learned_fp32_vs_plain_fp64_time"] = out["plain_fp64"]["solve_ms"] / out["learned_fp32"]["solve_ms"]
    H.free()
    return out


def shape_opt_islands(count=256, nrhs=4, reps=2):
    """The shape-optimisation batch: `count` random stars (N in {256 .. 1024}),
    `nrhs` seeded heat-type sources each, Dirichlet data 0, tol 1e-8.  One
    island solve (all geometries stacked in one canvas: one assembly, one
    island hierarchy in which each island ends where its own hierarchy
    would, one launch sequence) against the same work geometry by geometry
    (assembly, setup and a batched solve per star)."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"
    params = W.random_star_params(count)
    grids = [W.unit_box_grid(2, n) for n, _, _ in params]
    canvas = S.stack_islands(grids)

    def psi_of(g, c, ph):
        x = torch.as_tensor(g.axis_coords(0), device=dev)
        y = torch.as_tensor(g.axis_coords(1), device=dev)
        X, Y = x[None, :], y[:, None]
        phi = torch.atan2(Y, X)
        r = torch.full_like(phi, 0.3)
        for m in range(5):
            r = r + float(c[m]) * torch.cos((m + 2) * phi + float(ph[m]))
        return torch.sqrt(X * X + Y * Y) - r

    def sources_of(i, g):
        return W.heat_initial_batch(g, range(nrhs * i, nrhs * i + nrhs), dev)

    # inputs in HBM: per-island psi and sources, and their canvas packing
    psis = [psi_of(g, c, ph) for g, (n, c, ph) in zip(grids, params)]
    srcs = [sources_of(i, g) for i, g in enumerate(grids)]
    psi_c = torch.ones(canvas.grid.shape, dtype=torch.float64, device=dev)
    f_c = torch.zeros((nrhs,) + tuple(canvas.grid.shape), dtype=torch.float64, device=dev)
    for i, (g, sh) in enumerate(zip(grids, canvas.shapes)):
        r0 = int(canvas.rows[i])
        psi_c[r0:r0 + sh[0], :sh[1]] = psis[i]
        f_c[:, r0:r0 + sh[0], :sh[1]] = srcs[i]
    n_unk = 0

    def island_run(prec, gl=None):
        asm = S.assemble_diag(canvas.grid, psi_c)
        B = torch.stack([S.assemble_rhs_islands(asm, canvas, f_c[j]) for j in range(nrhs)]).contiguous()
        H = S.Hierarchy(canvas.grid, asm.kind, asm.a, 0.0, islands=canvas.rows)
        if gl:
            # learned per-level smoothing weights (the batched solve takes
            # the coarse levels' weights; the per-point fine weights are for
            # single solves)
            last = 1.0
            for lv in H.smoothed_levels():
                last = gl.get(lv, last)
                H.set_level_weight(lv, last)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, infos = S.solve_islands(H, B, canvas.rows, tol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        lev = H.n_levels
        H.free()
        return asm.n_unknowns, infos, t_solve, lev

    def sequential_run(prec):
        its = []
        for i, g in enumerate(grids):
            asm = S.assemble_diag(g, psis[i])
            zero = torch.zeros(asm.n_cuts, dtype=torch.float64, device=dev)
            B = torch.stack([S.assemble_rhs(asm, srcs[i][j].contiguous(), zero) for j in range(nrhs)]).contiguous()
            H = S.Hierarchy(g, asm.kind, asm.a, 0.0)
            _, infos = H.solve_batched(B, tol=1e-8, precision=prec)
            its += [x["iterations"] for x in infos]
            H.free()
        return its

    out = {"workload": f"random_stars_{count}_n256-1024_{nrhs}rhs_tol1e-8", "geometries": count, "nrhs": nrhs,
           "canvas_nodes": int(canvas.grid.shape[0]) * int(canvas.grid.shape[1])}
    for prec in ("fp32", "fp64"):
        island_run(prec)                          # warm-up (allocator, FP32 copies)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            n_unk, infos, t_solve, lev = island_run(prec)
        torch.cuda.synchronize()
        t_all = (time.perf_counter() - t0) / reps
        its = [x["iterations"] for row in infos for x in row]
        sequential_run(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sits = sequential_run(prec)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        nsys = count * nrhs
        out[prec] = {"ms": t_all * 1e3, "solve_ms": t_solve * 1e3, "solves_per_s": nsys / t_all,
                     "solve_phase_solves_per_s": nsys / t_solve, "levels": lev,
                     "iterations_min_max": [min(its), max(its)],
                     "rel_res_true_max": max(x["rel_res_true"] for row in infos for x in row),
                     "all_converged": all(x["status"] == 0 for row in infos for x in row),
                     "sequential_ms": t_seq * 1e3, "sequential_solves_per_s": nsys / t_seq,
                     "sequential_iterations_min_max": [min(sits), max(sits)],
                     "iteration_diff_vs_sequential_max": max(abs(a - b) for a, b in zip(its, sits)),
                     "speedup_vs_sequential": t_seq / t_all}
    # learned leg: the smoother trained on the GPU on one star that is not in
    # the batch (N = 256), its per-level weights applied to the island
    # hierarchy, single-precision cycle, against plain FP64 above
    n_t, c_t, ph_t = next(q for q in W.random_star_params(40, seed=W.SEED_BASE + 777) if q[0] == 256)
    gt = W.unit_box_grid(2, n_t)
    psi_t = psi_of(gt, c_t, ph_t)
    asm_t = S.assemble_diag(gt, psi_t)
    Ht = S.Hierarchy(gt, asm_t.kind, asm_t.a, 0.0)
    ls = S.LearnedSmoother(Ht, asm_t, psi_t, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ls.fit(steps=40, samples=4, sweeps=6, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    gl = dict(ls.g)
    Ht.free()
    island_run("fp32", gl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos, t_solve, lev = island_run("fp32", gl)
    torch.cuda.synchronize()
    t_all = (time.perf_counter() - t0) / reps
    its = [x["iterations"] for row in infos for x in row]
    nsys = count * nrhs
    out["learned_levels_fp32"] = {
        "training": {"geometry": "random star N=256 not in the batch", "seconds": t_train,
                     "level_weight_multipliers": {str(k): v for k, v in gl.items()}},
        "ms": t_all * 1e3, "solve_ms": t_solve * 1e3, "solves_per_s": nsys / t_all,
        "iterations_min_max": [min(its), max(its)],
        "rel_res_true_max": max(x["rel_res_true"] for row in infos for x in row),
        "all_converged": all(x["status"] == 0 for row in infos for x in row),
        "speedup_vs_plain_fp64": out["fp64"]["ms"] / (t_all * 1e3)}
    out["n_unknowns"] = n_unk
    return out


def qoi_studies(reps=2):
    """The two shape-parameter studies of Sec. 3.6, each one island batch from
    the level sets (in HBM) to the quantities of interest: u(0, 0) on the
    fixed-area ellipses (1024^2 cells on [-2.2, 2.2]^2, 61 values of a in
    [0.5, 2]) and the integral of u over [-1, 1] x [-0.5, 0.5] under the
    rotated ellipse (the paper's 501^2 grid of [-5, 5]^2, 64 angles), with
    the closed form, symmetry and smoothness figures of each."""
    import numpy as np
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    out = {}
    g = W.qoi_ellipse_grid(1024)
    a = W.qoi_ellipse_params(61)
    wc = np.zeros(g.shape)
    wc[g.n[1] // 2, g.n[0] // 2] = 1.0
    studies = {
        "ellipse_u00": (g, [W.psi_area_ellipse(g, x) for x in a], wc, a),
    }
    g2 = W.qoi_rotated_grid()
    th = W.qoi_rotated_params(64)
    studies["rotated_ellipse_rect_integral"] = (g2, [W.psi_rotated_ellipse(g2, x) for x in th],
                                                W.qoi_rectangle_weights(g2), th)
    for name, (grid, psis, w, par) in studies.items():
        f = np.full(grid.shape, W.QOI_SOURCE)
        S.qoi_study(grid, psis, f, w, tol=1e-10)              # warm-up
        best = None
        for _ in range(reps):
            q, infos, t = S.qoi_study(grid, psis, f, w, tol=1e-10)
            best = t if best is None or t["device_ms"] < best["device_ms"] else best
        its = [i["iterations"] for i in infos]
        step = float(par[1] - par[0])
        d = (q[2:] - q[:-2]) / (2.0 * step)
        r = {"grid_nodes": f"{grid.shape[1]}x{grid.shape[0]}", "geometries": len(psis),
             "n_unknowns": best["n_unknowns"], "levels": best["levels"], "device_ms": best["device_ms"],
             "solves_per_s": len(psis) / (best["device_ms"] * 1e-3),
             "iterations_min_max": [min(its), max(its)],
             "all_converged": all(i["status"] == 0 for i in infos),
             "qoi_min_max": [float(q.min()), float(q.max())],
             "derivative_abs_max": float(np.abs(d).max()),
             "second_difference_abs_max": float(np.abs(np.diff(q, 2)).max())}
        if name == "ellipse_u00":
            exact = -3.0 / (2.0 * (a * a + 1.0 / (a * a)))
            r["max_abs_error_vs_closed_form"] = float(np.abs(q - exact).max())
            r["argmin_a"] = float(a[np.argmin(q)])
            r["symmetry_a_inv_a_max_rel"] = float(max(abs(q[i] - q[j]) / abs(q[i])
                                                      for i, j in ((0, 60), (12, 30), (5, 44))))
        else:
            # theta and 2 pi - theta, theta and theta + pi (angles on the lattice excluded)
            m = len(par)
            pairs = [(k, m - k) for k in range(1, m // 2) if k % (m // 8)]
            r["symmetry_theta_minus_theta_max_rel"] = float(max(abs(q[i] - q[j]) / abs(q[i]) for i, j in pairs))
            pairs = [(k, k + m // 2) for k in range(m // 2) if k % (m // 8)]
            r["symmetry_theta_plus_pi_max_rel"] = float(max(abs(q[i] - q[j]) / abs(q[i]) for i, j in pairs))
        out[name] = r
    return out


def disk_latency(n=128, warm=3, reps=10):
    """The 128^2 disk (Poisson, FP64 AMG-PCG to 1e-10): a latency case (about
    8k unknowns, never bandwidth-bound).  Median of `reps` whole steps
    (assembly, RHS, setup, solve, free) and of `reps` solves on one
    hierarchy (HIP events around the solve), after `warm` of each."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"
    p = W.disk_poisson(n)
    psi = torch.as_tensor(p.psi, device=dev)
    f = torch.as_tensor(p.f, device=dev)

    def step(keep=False):
        asm = S.assemble_diag(p.grid, psi)
        b = S.assemble_rhs(asm, f, torch.as_tensor(p.u_dirichlet(*asm.cut_coordinates()), device=dev))
        H = S.Hierarchy(p.grid, asm.kind, asm.a, 0.0)
        x, info = H.solve(b, tol=p.tol)
        if keep:
            return asm, b, H, x, info
        H.free()
        return asm.n_unknowns, info

    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    wall = []
    for _ in range(reps):
        t0 = time.perf_counter()
        n0, info = step()
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
    asm, b, H, x, info = step(keep=True)
    X, Y = p.grid.mesh()
    exact = torch.as_tensor(p.u_exact(X, Y), device=dev)
    inside = asm.kind.reshape(x.shape) == 2
    err = (x - exact).abs()[inside].max().item()
    for _ in range(warm):
        H.solve(b, tol=p.tol)
    solve = []
    for _ in range(reps):
        t0 = time.perf_counter()
        _, i = H.solve(b, tol=p.tol)
        solve.append((i["solve_ms"], (time.perf_counter() - t0) * 1e3))
    levels = H.n_levels
    H.free()
    med = lambda v: sorted(v)[len(v) // 2]
    return {"workload": f"disk2d_{n}_poisson_fp64_amg_pcg_tol1e-10", "n_unknowns": n0, "levels": levels,
            "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
            "max_error_vs_exact": err,
            "step_latency_ms_median": med(wall), "step_latency_ms_min": min(wall),
            "solve_latency_ms_median": med([s[0] for s in solve]),
            "solve_host_latency_ms_median": med([s[1] for s in solve]),
            "timing": f"median of {reps} after {warm} warm-up; step = assembly + RHS + setup + solve + free, "
                      "host clock with a device synchronisation; solve = HIP events around the PCG solve"}


def wave_stencil(n=1600, launches=200):
    """The explicit wave loop's operator passes on Table 1's finest grid (the
    unit disk in [-1.1, 1.1]^2, n^2 cells): stencil_apply and the leap-frog
    right-hand side eb_wave_rhs, timed with HIP events on the library's
    stream around back-to-back launches queued behind a device-side wait (so
    host gaps do not enter), and the whole leap-frog run of Table 1 (dt =
    0.7 h, 10.2 periods) with its max-error."""
    import torch
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W
    dev = "cuda:0"
    g = W.wave_disk_grid(n)
    psi = torch.as_tensor(W.psi_unit_disk(g), device=dev)
    asm = S.assemble_diag(g, psi)
    nu = asm.n_unknowns
    gen = torch.Generator(device=dev).manual_seed(5)
    x = torch.randn(g.shape, dtype=torch.float64, device=dev, generator=gen)
    xm = torch.randn(g.shape, dtype=torch.float64, device=dev, generator=gen)
    y = torch.empty_like(x)
    nbox = x.numel()
    wset = nbox * (8 * 4 + 1)

    def timed(fn, algo_bytes):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(50_000_000)         # keeps the stream busy while the launches are queued
        e0.record()
        for _ in range(launches):
            fn()
        e1.record()
        torch.cuda.synchronize()
        mean = e0.elapsed_time(e1) * 1e3 / launches
        gbs = algo_bytes / (mean * 1e-6) / 1e9
        return {"avg_launch_us": mean, "launches": launches, "algorithmic_bytes_per_launch": algo_bytes,
                "timing": "HIP events around back-to-back launches queued behind a device-side wait",
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS, "mall_resident": wset < MALL_BYTES}}

    out = {"workload": f"wave_disk_{n}_table1_grid", "grid_nodes": f"{n + 1}x{n + 1}", "n_unknowns": nu,
           "box_nodes": nbox, "working_set_bytes": wset,
           "bytes_model": "stencil_apply 24 B per unknown (x, a read, y written); eb_wave_rhs 32 B per "
                          "unknown (u^n, u^{n-1}, a read, out written); kinds and the zeros written off "
                          "the unknowns not counted"}
    out["stencil_apply"] = timed(lambda: S.stencil_apply(g, asm.kind, asm.a, 0.0, x, out=y), 24.0 * nu)
    out["wave_rhs"] = timed(lambda: S.wave_rhs(asm, 0.0, 0.7 * g.h, 1.0, x, xm, out=y), 32.0 * nu)
    # the leap-frog run of Table 1's first column at this h
    X, Y = g.mesh()
    dt, ns = W.wave_schedule(n, 0.7, 10.2)
    u0 = torch.as_tensor(W.standing_mode(X, Y, 0.0), device=dev)
    u1 = torch.as_tensor(W.standing_mode(X, Y, dt), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, _, st = S.wave_theta(asm, u0, u1, dt, 0.0, ns)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ex = torch.as_tensor(W.standing_mode(X, Y, ns * dt), device=dev)
    inside = asm.kind.reshape(u.shape) == 2
    out["leapfrog_table1"] = {"steps": ns - 1, "seconds": secs, "steps_per_s": (ns - 1) / secs,
                              "max_error": (u - ex).abs()[inside].max().item(), "paper_max_error": 1.7e-4,
                              "note": "one eb_wave_rhs launch per step from a host loop"}
    return out


BLOCKS.update({"batched": lambda: batched_heat(), "heat_steps": lambda: heat_steps(),
               "learned_3d": lambda: learned_ellipsoid(), "islands": lambda: shape_opt_islands(),
               "qoi": lambda: qoi_studies(), "disk_latency": lambda: disk_latency(),
               "wave_stencil": lambda: wave_stencil()})


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel", default="pcg_xr_down", choices=list(TIMED_KERNELS),
                    help="kernel of the counter summary (--pmc-summary)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched heat-step measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the 3-D learned-smoother measurement")
    ap.add_argument("--no-islands", action="store_true", help="skip the shape-optimisation island batch")
    ap.add_argument("--no-qoi", action="store_true", help="skip the shape-parameter QOI studies")
    ap.add_argument("--no-heat-steps", action="store_true", help="skip the 200-step batched heat run")
    ap.add_argument("--no-disk", action="store_true", help="skip the 128^2 disk latency case")
    ap.add_argument("--no-wave", action="store_true", help="skip the wave-loop operator passes")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--block", choices=list(BLOCKS),
                    help="run only this block of the bench line and print its JSON (for profiling)")
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--rocprof-summary", metavar="DIR",
                    help="print a markdown summary of a rocprofv3 --stats/--pmc output directory and exit")
    ap.add_argument("--top", type=int, default=25, help="kernels listed by --rocprof-summary")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="summarise FETCH_SIZE / WRITE_SIZE passes of --kernel and of --copy-calib, then exit")
    ap.add_argument("--phases", action="store_true",
                    help="diagnostics: synchronise between phases and report host time per phase")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size (for scaling FETCH_SIZE / WRITE_SIZE)."""
    import torch
    nbytes = 256 << 20
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_bytes_read": nbytes, "copy_calib_bytes_written": nbytes, "launches": 5}))


_POOL = {}


def _pool_init(kind, n, barrier):
    """Process-pool worker set-up: BLAS on one thread; for the heat workload
    the assembly and the oracle's hierarchy of (A + I/dt), built once per
    worker (set-up is amortised over the steps and right-hand sides)."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)
    if kind == "heat":
        from oracle import amg as OA
        from oracle import eb_assembly as E
        from paper_2204_06083_amd import workloads as W
        g = W.unit_box_grid(2, n)
        asm = E.assemble(g, W.psi_star(g))
        A = E.operator_csr(asm, 1.0 / g.h)
        _POOL.update(g=g, asm=asm, A=A, H=OA.build_hierarchy(A, E.unknown_coords(asm)))
    barrier.wait()


def _pool_heat_solve(rhs_id):
    """One backward-Euler step (dt = h, cold start) of one seeded initial condition."""
    import numpy as np

    from oracle import amg as OA
    from oracle import eb_assembly as E
    from oracle import pcg as OP
    from paper_2204_06083_amd import workloads as W
    P = _POOL
    b = E.rhs(P["asm"], W.heat_initial(P["g"], rhs_id) / P["g"].h, np.zeros(P["asm"].n_cuts))
    res = OP.pcg(P["A"], b, precond=lambda r: OA.vcycle(P["H"], r), tol=1e-8)
    return P["asm"].n_unknowns, res.iterations


def _pool_island(task):
    """One shape-optimisation geometry: assembly, hierarchy and its seeded
    sources solved to 1e-8."""
    import numpy as np

    from oracle import amg as OA
    from oracle import eb_assembly as E
    from oracle import pcg as OP
    from paper_2204_06083_amd import workloads as W
    i, n, c, ph, nrhs = task
    prob = W.random_star_poisson(n, c, ph)
    asm = E.assemble(prob.grid, prob.psi)
    A = E.operator_csr(asm)
    H = OA.build_hierarchy(A, E.unknown_coords(asm))
    its = 0
    for j in range(nrhs):
        b = E.rhs(asm, W.heat_initial(prob.grid, nrhs * i + j), np.zeros(asm.n_cuts))
        its += OP.pcg(A, b, precond=lambda r: OA.vcycle(H, r), tol=1e-8).iterations
    return asm.n_unknowns, its


def _pool_run(kind, n, fn, tasks, workers):
    """Map `tasks` over a spawned pool of `workers` processes; timed from the
    moment every worker has finished its set-up to the last result."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(workers + 1)
    with ctx.Pool(workers, initializer=_pool_init, initargs=(kind, n, barrier)) as pool:
        barrier.wait()
        t0 = time.perf_counter()
        res = pool.map(fn, tasks, chunksize=1)
        secs = time.perf_counter() - t0
    return res, secs


def cpu_baseline(n):
    """The oracle, as it stands, on full steps of the same workload: with BLAS
    on one thread (the headline figure) and on every usable core, and the
    batched workloads over a process pool of every usable core."""
    from threadpoolctl import threadpool_limits

    from oracle import eb_assembly as E
    from oracle import pcg as OP
    from paper_2204_06083_amd import workloads as W

    usable = len(os.sched_getaffinity(0))
    prob = W.star_poisson(n)
    reps = 2

    def steps():
        work = 0
        t0 = time.perf_counter()
        for _ in range(reps):
            asm = E.assemble(prob.grid, prob.psi)
            A = E.operator_csr(asm)
            b = E.rhs(asm, prob.f, prob.u_dirichlet(*E.cut_coordinates(asm)))
            res, H = OP.amg_pcg(A, E.unknown_coords(asm), b, tol=prob.tol)
            work += asm.n_unknowns * res.iterations
        return work, time.perf_counter() - t0, res.iterations

    with threadpool_limits(limits=1):
        work, secs, its = steps()
    with threadpool_limits(limits=usable):
        work_all, secs_all, _ = steps()
    out = {
        "value": work / secs,
        "unit": "unknowns·CG-iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{reps} full steps (assemble, RHS, AMG setup, PCG to 1e-8; {its} iterations each) "
                  f"of the {n}^2 star workload in {secs:.2f} s, BLAS limited to 1 thread; host has "
                  f"{usable} usable cores (os.cpu_count() = {os.cpu_count()})",
        "seconds": secs,
        "iterations": its,
        "all_core_blas": {"value": work_all / secs_all, "unit": "unknowns·CG-iters/s", "cores": usable,
                          "seconds": secs_all,
                          "sample": f"the same {reps} steps with BLAS on {usable} threads (the sparse "
                                    "products stay single-threaded; BLAS serves the coarsest solve)"},
    }
    workers = min(16, usable)
    # one task per worker: heat right-hand sides 0 .. workers-1 of the 64
    # (one backward-Euler step each) and the first `workers` of the 256 seeded
    # geometries (4 sources each); whole-batch times extrapolated by count
    res, secs_h = _pool_run("heat", 1024, _pool_heat_solve, list(range(workers)), workers)
    its_h = [r[1] for r in res]
    params = W.random_star_params(256)
    tasks = [(i, nn, c, ph, 4) for i, (nn, c, ph) in enumerate(params[:workers])]
    res_i, secs_i = _pool_run("islands", 0, _pool_island, tasks, workers)
    out["process_pool"] = {
        "kind": "oracle", "cores": workers, "label": f"process pool of {workers} single-threaded workers",
        "heat_1024_64rhs": {"unit": "solves/s", "value": workers / secs_h, "seconds": secs_h,
                            "extrapolated_step_seconds_64rhs": secs_h * 64 / workers,
                            "iterations_min_max": [min(its_h), max(its_h)],
                            "sample": f"one backward-Euler step (dt = h, cold start, tol 1e-8) of {workers} of the "
                                      "64 seeded right-hand sides on the 1024^2 star; each worker builds the "
                                      "assembly and hierarchy once before the timed map"},
        "islands_256x4": {"unit": "solves/s", "value": 4 * len(tasks) / secs_i, "seconds": secs_i,
                          "extrapolated_batch_seconds": secs_i * len(params) / len(tasks),
                          "sample": f"{len(tasks)} of the {len(params)} seeded geometries (assembly, hierarchy and "
                                    "4 sources to 1e-8 each); batch time extrapolated by geometry count"},
    }
    return out


def rocprof_summary(path, top=25):
    """Markdown table of a rocprofv3 kernel_stats.csv (and counters if present)."""
    import csv
    import glob
    out = []
    stats = sorted(glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True))
    for f in stats:
        rows = list(csv.DictReader(open(f)))
        total = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
        out.append(f"kernel stats: {os.path.relpath(f, path)}")
        out.append("| kernel | calls | avg us | min us | max us | total ms | % |")
        out.append("|---|---|---|---|---|---|---|")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
            name = _kernel_symbol(r["Name"])
            out.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                       f"{float(r['TotalDurationNs']) / 1e6:.3f} | {100 * float(r['TotalDurationNs']) / total:.1f} |")
        out.append("")
    for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        agg = {}
        for r in rows:
            key = (_kernel_symbol(r["Kernel_Name"]), r["Counter_Name"])
            a = agg.setdefault(key, [0, 0.0])
            a[0] += 1
            a[1] += float(r["Counter_Value"])
        out.append(f"counters: {os.path.relpath(f, path)}")
        out.append("| kernel | counter | dispatches | mean per dispatch |")
        out.append("|---|---|---|---|")
        for (k, c), (nd, v) in sorted(agg.items()):
            out.append(f"| {k} | {c} | {nd} | {v / nd:.1f} |")
        out.append("")
    print("\n".join(out))


# FP64 instantiations of the bench's headline path (plain smoother weights)
KERNEL_SYMBOLS = {
    "pcg_spmv": "eb::k_t2_pspmv<double>", "pcg_xr_down": "eb::k_t2_xr_restrict<double, false, true>",
    "fine_post": "eb::k_t2_up_post<double, false>"}


def _kernel_symbol(name):
    """Kernel name as rocprofv3 reports it, without arguments or return type."""
    name = name.split("(")[0]
    return name[5:] if name.startswith("void ") else name
SOLVE_SOURCE = os.path.join(ROOT, "paper_2204_06083_amd", "csrc", "solve.hip")
COPY_BYTES = 256 << 20


def _sha256(path):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def _counter_mean(path, kernel_prefix):
    import csv
    import glob
    vals = []
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if _kernel_symbol(r["Kernel_Name"]) == kernel_prefix:
                vals.append(float(r["Counter_Value"]))
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def pmc_summary(args):
    """Per-launch HBM traffic of one kernel from FETCH_SIZE / WRITE_SIZE passes,
    each scaled by what the same counter reads for a plain copy of known size."""
    fdir, wdir, cfdir, cwdir = args.pmc_summary
    sym = KERNEL_SYMBOLS[args.kernel]
    fetch, nf = _counter_mean(fdir, sym)
    write, nw = _counter_mean(wdir, sym)
    cfetch, _ = _counter_mean(cfdir, "__amd_rocclr_copyBuffer")
    cwrite, _ = _counter_mean(cwdir, "__amd_rocclr_copyBuffer")
    f_scale = COPY_BYTES / (cfetch * 1024.0)
    w_scale = COPY_BYTES / (cwrite * 1024.0)
    traffic = fetch * 1024.0 * f_scale + write * 1024.0 * w_scale
    rec = {"kernel": args.kernel, "symbol": sym, "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
           "dispatches": [nf, nw], "copy_fetch_kib": cfetch, "copy_write_kib": cwrite,
           "fetch_scale": f_scale, "write_scale": w_scale, "traffic_bytes_per_launch": traffic,
           "solve_source_sha256": _sha256(SOLVE_SOURCE)}
    print(f"kernel `{sym}`: FETCH_SIZE {fetch:.0f} KiB x {f_scale:.3f}, WRITE_SIZE {write:.0f} KiB x {w_scale:.3f} "
          f"per dispatch -> {traffic / 1e6:.2f} MB per launch")
    print()
    print("traffic-json: " + json.dumps(rec))


def load_traffic(kernel):
    """traffic bytes per launch from the committed counter summary, if the
    solve source is unchanged since the counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_star2d_2048.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec.get("solve_source_sha256") == _sha256(SOLVE_SOURCE) and rec.get("kernel") == kernel:
                return rec["traffic_bytes_per_launch"]
    return None


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.rocprof_summary:
        rocprof_summary(args.rocprof_summary, args.top)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the library solves on one GPU; several-GPU runs are not part of this benchmark)", file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not (args.copy_calib or args.block or args.no_cpu_baseline):
        # before any GPU use: the pool's workers are started as new processes
        cpu = cpu_baseline(args.n)
    import torch
    if args.copy_calib:
        copy_calibration()
        return
    if args.block:
        torch.cuda.set_device(0)
        print(json.dumps({args.block: BLOCKS[args.block]()}))
        return
    from paper_2204_06083_amd import solver as S
    from paper_2204_06083_amd import workloads as W

    torch.cuda.set_device(0)
    dev = "cuda:0"
    prob = W.star_poisson(args.n)
    g = prob.grid
    psi = torch.as_tensor(prob.psi, device=dev)
    f = torch.as_tensor(prob.f, device=dev)
    first = S.assemble_diag(g, psi)
    cuts_cap = first.n_cuts
    del first
    torch.cuda.synchronize()

    phases = {"assemble": [], "rhs": [], "setup": [], "solve": [], "free": []}

    def mark():
        if args.phases:
            torch.cuda.synchronize()
        return time.perf_counter()

    def step(precision, keep=False):
        """One whole step of the hot path, as a user runs it (iteration graphs
        on, no timing hook): assembly, boundary data, RHS, setup, solve, free."""
        ta = mark()
        asm = S.assemble_diag(g, psi, cuts_cap=cuts_cap)
        tb = mark()
        u = W.u_star(*asm.cut_coordinates())
        b = S.assemble_rhs(asm, f, u)
        t_setup0 = mark()
        H = S.Hierarchy(g, asm.kind, asm.a, 0.0)
        t_setup1 = mark()
        x, info = H.solve(b, tol=prob.tol, precision=precision)
        t_solve1 = mark()
        info["setup_ms_host"] = (t_setup1 - t_setup0) * 1e3
        if args.phases:
            phases["assemble"].append((tb - ta) * 1e3)
            phases["rhs"].append((t_setup0 - tb) * 1e3)
            phases["setup"].append((t_setup1 - t_setup0) * 1e3)
            phases["solve"].append((t_solve1 - t_setup1) * 1e3)
        if keep:
            return asm, b, H, x, info
        t_free0 = mark()
        H.free()
        t_free1 = mark()
        if args.phases:
            phases["free"].append((t_free1 - t_free0) * 1e3)
        return asm.n_unknowns, info

    def timed_steps(precision):
        for _ in range(args.warmup):
            step(precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, work = [], 0
        for _ in range(args.steps):
            n0_, info = step(precision)
            infos.append(info)
            work += n0_ * info["iterations"]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, work, infos

    # the single-precision V-cycle, then plain FP64 (the headline), each over
    # whole steps
    m_secs, mixed_work, m_infos = timed_steps("fp32")
    b_secs, b_work, b_infos = timed_steps("bf16")
    secs, total_work, infos = timed_steps("fp64")
    ms_per_step = secs * 1e3 / args.steps

    # one kept hierarchy: difference between the two precisions' solutions,
    # the byte models, and the fine kernels' launch times in separate solves
    # with the timing hook (it records events at every launch of the selected
    # kernel and runs the iterations kernel by kernel)
    asm, b, H, xd, _ = step("fp64", keep=True)
    xm, _ = H.solve(b, tol=prob.tol, precision="fp32")
    mixed_diff = (torch.linalg.vector_norm(xm - xd) / torch.linalg.vector_norm(xd)).item()
    xb, _ = H.solve(b, tol=prob.tol, precision="bf16")
    bf16_diff = (torch.linalg.vector_norm(xb - xd) / torch.linalg.vector_norm(xd)).item()
    del xm, xd, xb
    dim = g.dim
    n0 = asm.n_unknowns
    n1 = H.level(1).n if H.n_levels > 1 else 0
    kern = {}
    for kname in TIMED_KERNELS:
        H.time_kernel(kname)
        for _ in range(3):
            H.solve(b, tol=prob.tol, precision="fp64")
        nl, kms = H.kernel_time()
        H.time_kernel(None)
        avg_us = kms / max(nl, 1) * 1e3
        byt = kernel_bytes(kname, n0, n1, dim)
        kern[kname] = {"avg_launch_us": avg_us, "launches": nl, "algorithmic_bytes_per_launch": byt,
                       "achieved_GBs": byt / (avg_us * 1e-6) / 1e9}
    models = {"design": design_model_bytes(H),
              "impl_fp64": impl_model_bytes(H, "fp64", dim), "impl_fp32": impl_model_bytes(H, "fp32", dim),
              "impl_bf16": impl_model_bytes(H, "bf16", dim)}
    wset = working_set_bytes(H, dim)
    levels = H.n_levels
    H.free()

    mean_iters = sum(i["iterations"] for i in infos) / len(infos)
    mean_solve = sum(i["solve_ms"] for i in infos) / len(infos)
    m_iters = sum(i["iterations"] for i in m_infos) / len(m_infos)
    m_solve = sum(i["solve_ms"] for i in m_infos) / len(m_infos)
    b_iters = sum(i["iterations"] for i in b_infos) / len(b_infos)
    b_solve = sum(i["solve_ms"] for i in b_infos) / len(b_infos)
    # dominant kernel: the largest time per iteration (one launch each)
    dom = max(kern, key=lambda k: kern[k]["avg_launch_us"])

    def solve_roofline(iters, solve_ms, impl_key):
        per_s = iters / (solve_ms * 1e-3)
        out_ = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "mall_resident": wset < MALL_BYTES, "working_set_bytes": wset}
        for key, mkey in (("design_model", "design"), ("implementation", impl_key)):
            gbs = models[mkey] * per_s / 1e9
            out_[key] = {"bytes_per_iter": models[mkey], "achieved": gbs, "frac": gbs / HBM_PEAK_GBS}
        out_["frac"] = out_["design_model"]["frac"]
        out_["achieved"] = out_["design_model"]["achieved"]
        return out_

    ktraffic = load_traffic(dom)
    out = {
        "metric": "unknowns·CG-iters/s & solves/s to 1e-8 rel-res, learned/mixed vs plain FP64",
        "value": total_work / secs,
        "unit": "unknowns·CG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"star2d_{args.n}_poisson_plain_fp64_amg_pcg_tol1e-8",
                   "grid_nodes": f"{args.n + 1}x{args.n + 1}", "n_unknowns": n0, "tol": prob.tol,
                   "precision": "plain FP64 (no mixed precision, no learned smoother)"},
        "solves_per_s": args.steps / secs,
        "iterations": mean_iters,
        "levels": levels,
        "setup_ms_host": sum(i["setup_ms_host"] for i in infos) / len(infos),
        "solve_ms": mean_solve,
        "solve_phase_unknowns_iters_per_s": n0 * mean_iters / (mean_solve * 1e-3),
        "rel_res_true_max": max(i["rel_res_true"] for i in infos),
        "solve_roofline": solve_roofline(mean_iters, mean_solve, "impl_fp64"),
        "mixed": {
            "precision": "FP32 V-cycle, FP64 outer CG, FP64 true residual with restart, FP64 coarsest solve",
            "value": mixed_work / m_secs,
            "unit": "unknowns·CG-iters/s",
            "ms_per_step": m_secs * 1e3 / args.steps,
            "solves_per_s": args.steps / m_secs,
            "iterations": m_iters,
            "solve_ms": m_solve,
            "solve_phase_unknowns_iters_per_s": n0 * m_iters / (m_solve * 1e-3),
            "rel_res_true_max": max(i["rel_res_true"] for i in m_infos),
            "rel_diff_vs_fp64_solution": mixed_diff,
            "solve_speedup_vs_fp64": mean_solve / m_solve,
            "solve_roofline": solve_roofline(m_iters, m_solve, "impl_fp32"),
            "bf16_smoother": {
                "precision": "FP32 V-cycle whose fine smoother stores z and 1/d in BF16; FP64 outer CG",
                "value": b_work / b_secs,
                "unit": "unknowns·CG-iters/s",
                "ms_per_step": b_secs * 1e3 / args.steps,
                "solves_per_s": args.steps / b_secs,
                "iterations": b_iters,
                "solve_ms": b_solve,
                "time_to_tol_ms": b_solve,
                "rel_res_true_max": max(i["rel_res_true"] for i in b_infos),
                "rel_diff_vs_fp64_solution": bf16_diff,
                "solve_speedup_vs_fp64": mean_solve / b_solve,
                "solve_roofline": solve_roofline(b_iters, b_solve, "impl_bf16"),
            },
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": kern[dom]["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": kern[dom]["achieved_GBs"] / HBM_PEAK_GBS,
            "traffic": ktraffic,
            "avg_launch_us": kern[dom]["avg_launch_us"],
            "launches_timed": kern[dom]["launches"],
            "algorithmic_bytes_per_launch": kern[dom]["algorithmic_bytes_per_launch"],
            "mall_resident": wset < MALL_BYTES,
            "timed": "separate solves on one hierarchy with launch events on the kernel's stream "
                     "(the headline steps run without the timing hook)",
        },
        "fine_kernels": kern,
    }
    if args.phases:
        out["phases_ms"] = {k: sum(v) / len(v) for k, v in phases.items() if v}
    if not args.no_batched:
        out["batched"] = batched_heat()
    if not args.no_heat_steps:
        out["heat_steps"] = heat_steps()
    if not args.no_learned:
        out["learned_3d"] = learned_ellipsoid()
    if not args.no_islands:
        out["islands"] = shape_opt_islands()
    if not args.no_qoi:
        out["qoi"] = qoi_studies()
    if not args.no_disk:
        out["disk_latency"] = disk_latency()
    if not args.no_wave:
        out["wave_stencil"] = wave_stencil()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
