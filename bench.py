#!/usr/bin/env python
"""Benchmark of the slab hot path on one MI355X.

Metric: space-time DoF/s of the Jacobian vmult, FP64 (the value) vs FP32;
slab solves/s (Newton-FGMRES with the hp-STMG preconditioner in FP32 and in
FP64); p50/p99 latency of a served request stream.
Workload: 3D unit cube, 16^3 affine hexahedra, Q3/P2disc (r=2) x DG(2),
nu = 1e-2 (Re = 100), tau = 1/32, Newton state = seeded smooth divergence-free
Fourier field (8 modes per axis, max |v| = 1) at every time node, direction
x = U(-1,1); N = 1,181,721 space-time unknowns.  One step = one application
y = J_n(U) x with inputs already resident in HBM; buffers rotate over >= 1 GiB
so the 256 MB Infinity Cache does not hold the working set.

Output: one JSON line (see the keys below) with the roofline of the dominant
kernel (the cell kernel of the FP64 vmult, timed with HIP events on the
stream it runs on) and the oracle timed on the host cores as cpu_baseline.
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

PEAK_FP64_VALU = 78.6e12      # 256 CU * 4 SIMD * 16 FP64 lanes/clk * 2 flop * 2.4 GHz
PEAK_HBM = 8.0e12
# HBM bytes per launch of the FP64 Jacobian volume kernel on this workload come
# from the rocprofv3 counter summary below (FETCH_SIZE x2, the factor a 1 GiB
# device copy shows, plus WRITE_SIZE x1); they count only while the kernel
# source still has the hash the counters were taken with.
COUNTERS = os.path.join(ROOT, "profiles", "cell_kernel_jac_16cube_r2k2.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2602_13841_amd", "csrc", "cell_ops.hip")


def source_sha(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def counter_traffic():
    """(bytes per launch, date) from the committed counter summary when its
    recorded source hash matches the current kernel source, else (None, why)."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None, "no counter summary"
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            key, v = line[2:].split(": ", 1)
            vals[key.strip()] = v.strip()
    if vals.get("source_sha") != source_sha(KERNEL_SOURCE):
        return None, "kernel changed since the counters were taken"
    return int(vals["traffic_bytes_per_launch"]), vals.get("date", "")

WORKLOAD = dict(dim=3, n=(16, 16, 16), r=2, k=2, nu=1e-2, tau=1.0 / 32)


def vmult_flops(dim, n, r, k, nq):
    """Algorithmic floating-point operations of one matrix-free Jacobian
    application (FMA = 2), volume terms only, counted for the leaner of the
    two sum-factorized schemes: time mixing, 1D sweeps of x, state and mixed
    field, pressure sweeps, collocation gradients at the Gauss points,
    quadrature-point physics, transposed collocation and sweeps.  (The 3D
    kernel takes gradients with the nodal derivative table instead, which
    costs more operations; see vmult_flops_performed.)"""
    n1, rp1, nt = r + 2, r + 1, k + 1
    ncell = int(np.prod(n))
    if dim == 3:
        sw = 2 * (n1 ** 3 * nq + n1 ** 2 * nq ** 2 + n1 * nq ** 3)
        swp = 2 * (rp1 ** 3 * nq + rp1 ** 2 * nq ** 2 + rp1 * nq ** 3)
        nqv, nl = nq ** 3, n1 ** 3
    else:
        sw = 2 * (n1 ** 2 * nq + n1 * nq ** 2)
        swp = 2 * (rp1 ** 2 * nq + rp1 * nq ** 2)
        nqv, nl = nq ** 2, n1 ** 2
    mix = dim * nl * nt * 2
    fwd = 3 * dim * sw + swp
    coll = 2 * dim * dim * nqv * nq * 2
    qp = nqv * (2 * dim ** 3 + 5 * dim ** 2 + 2 * dim ** 3 + 4 * dim + 4)
    bwd = dim * sw + swp
    return ncell * nt * (mix + fwd + coll + qp + bwd)


def vmult_flops_performed(n, r, k, nq):
    """Operations the 3D Jacobian volume kernel performs per application (FMA
    = 2): z sweep (x by S and D, state and mixed field by S, time mixing,
    pressure), y sweep (three x variants, state, mixed field, pressure), x
    sweep per quadrature point, point physics, and the transposed x, y, z
    sweeps."""
    n1, rp1, nt = r + 2, r + 1, k + 1
    ncell = int(np.prod(n))
    z = 3 * n1 ** 3 * nq * 4 + 3 * n1 ** 3 * nt + rp1 ** 3 * nq
    y = 15 * nq ** 2 * n1 ** 2 + nq ** 2 * rp1 ** 2
    xp = nq ** 3 * (18 * n1 + rp1)
    bx = 12 * nq ** 3 * n1 + nq ** 3 * rp1
    by = 9 * nq ** 2 * n1 ** 2 + nq ** 2 * rp1 ** 2
    bz = 6 * nq * n1 ** 3 + nq * rp1 ** 3
    qp = nq ** 3 * (2 * 27 + 5 * 9 + 2 * 27 + 4 * 3 + 4)
    return ncell * nt * (2 * (z + y + xp + bx + by + bz) + qp)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_solve_c1():
    """The oracle's Newton-FGMRES-hp-STMG solve of the 2D 4x4 Q2/P1disc x DG(1)
    slab (tau = 0.1, nu = 1, manufactured forcing, 2 levels) on the host:
    solve time and the paper's throughput measure theta = N / W."""
    import oracle
    from oracle import manufactured as MS
    from oracle import solver as S
    prob = oracle.Problem(dim=2, n=(4, 4), r=1, k=1, nu=1.0, tau=0.1)
    slab = oracle.Slab(prob)
    rhs = MS.slab_rhs(slab, 0.0)
    t0 = time.perf_counter()
    _, st = S.newton_solve(slab, S.Hierarchy(prob, max_levels=2), np.zeros(slab.N), rhs, np.zeros(slab.Nv))
    dt = time.perf_counter() - t0
    return {"N": slab.N, "wall_s": dt, "theta_dof_per_s": slab.N / dt, "newton": st.newton_its,
            "fgmres": st.fgmres_its}


def cpu_lu_sample(seconds=6.0, seed=6):
    """FP64 LU with partial pivoting (the oracle's patch factorization routine,
    scipy.linalg.lu_factor) of seeded dense matrices with the sizes of the
    mixed patch batch, on the host, for about `seconds`: GFLOP/s (2/3 m^3)."""
    import scipy.linalg as sla
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(k + 1) * (3 * (r + 2) ** 3 + {1: 4, 2: 10, 3: 20}[r]) for r, k in
             zip(rng.integers(1, 4, 4096), rng.integers(0, 3, 4096))]
    flops, done, t0 = 0.0, 0, time.perf_counter()
    for m in sizes:
        A = rng.uniform(-1, 1, (m, m)) + 0.5 * np.sqrt(m) * np.eye(m)
        sla.lu_factor(A, overwrite_a=True, check_finite=False)
        flops += 2.0 / 3.0 * m ** 3
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"matrices": done, "gflops": flops / dt / 1e9, "wall_s": dt,
            "patches_per_s_scaled_to_4096": done / dt}


def cpu_baseline(U, X, seconds=12.0):
    """The oracle's element-by-element Jacobian action on a bounded sample of
    cells of the same workload, timed on the host cores; scaled to DoF/s.
    Beside it: the CPU model, the oracle's slab solve of the 2D 4x4 problem
    and FP64 LU of a sample of the mixed patch sizes."""
    import oracle
    w = WORKLOAD
    prob = oracle.Problem(dim=w["dim"], n=w["n"], r=w["r"], k=w["k"], nu=w["nu"], tau=w["tau"])
    slab = oracle.Slab(prob)
    V, _ = slab.split(U)
    Xv, Xp = slab.split(X)
    ncell = slab.space.ncell
    rng = np.random.default_rng(0)
    done_cells = 0
    t0 = time.perf_counter()
    chunk = 32
    while time.perf_counter() - t0 < seconds:
        cells = np.sort(rng.choice(ncell, chunk, replace=False))
        for a in range(slab.nt):
            mix = slab.tt.K[a] @ Xv
            Xa = np.concatenate([Xv[a], Xp[a]])
            slab.space.cell_actions(V[a], Xa, mix, cells)
        done_cells += chunk
    dt = time.perf_counter() - t0
    frac = done_cells / ncell
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": slab.N * frac / dt, "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{done_cells} cells x {slab.nt} time nodes of the 16^3 workload "
                      f"({100 * frac:.1f}% of one vmult), element-matrix action, {dt:.1f} s",
            "cpu_model": cpu_model(), "solve_2d_4x4": cpu_solve_c1(), "lu_fp64_patch_sizes": cpu_lu_sample(),
            "residual_16cube": cpu_residual(slab, U)}


def cpu_residual(slab, U):
    """The oracle's slab residual R_n(U) (eq. InAlgNS, element loop) of the
    whole 16^3 workload on the host: wall time and DoF/s."""
    t0 = time.perf_counter()
    slab.residual(U)
    dt = time.perf_counter() - t0
    return {"N": slab.N, "wall_s": dt, "dof_per_s": slab.N / dt}


SOLVE_WORKLOAD = dict(dim=3, n=(32, 32, 32), r=3, k=1, nu=1e-3, tau=1.0 / 64, perturb=0.2, vert_seed=4, v0_seed=5)
TIMER_NAMES = ["vcycle_graph", "vanka_elem", "vanka_patch", "vanka_lu", "vanka_apply", "cell_jac_f64", "cell_jac_f32",
               "face_jac_f64",
               "face_jac_f32", "gather_f64",
               "gather_f32", "cell_res_f64", "cell_mass_f64", "coarse_factor", "coarse_solve", "transfer"]


def bench_solve(prec, warm=True, **opts):
    """One Newton-FGMRES slab solve of the 32^3 perturbed-mesh workload
    (r=3, k=1, Re=1000, tau=1/64), previous-slab velocity = smooth field,
    zero initial guess, stopping at |R|_M <= 1e-8 |R_0|_M.  Returns solves/s,
    DoF/s (N / wall), iteration counts and the kernel-time split."""
    import torch
    from paper_2602_13841_amd import inputs as I
    from paper_2602_13841_amd import stmg
    w = SOLVE_WORKLOAD
    d, n = w["dim"], w["n"]
    if warm:
        # load the code objects of this configuration on a small mesh
        c = stmg.Context(d, (4, 4, 4), w["r"], w["k"], w["nu"], w["tau"], prec_mg=prec, **opts)
        c.set_slab_data(None, torch.tensor(I.smooth_velocity(d, (4, 4, 4), w["r"], 1), device="cuda"))
        c.newton_solve(torch.zeros(c.N, dtype=torch.float64, device="cuda"))
        del c
    vert = I.perturbed_vertices(d, n, w["perturb"], w["vert_seed"])
    ctx = stmg.Context(d, n, w["r"], w["k"], w["nu"], w["tau"], vertices=vert, prec_mg=prec,
                       newton_rtol=1e-8, newton_atol=0.0, **opts)
    ctx.set_slab_data(None, torch.tensor(I.smooth_velocity(d, n, w["r"], w["v0_seed"]), device="cuda"))
    u = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
    ctx.timing_reset()
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, st, rc = ctx.newton_solve(u)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing(False)
    tm = {k: round(ctx.timing_get(k)[0] / 1e3, 4) for k in TIMER_NAMES if ctx.timing_get(k)[1]}
    out = {"prec_mg": "f64" if prec == stmg.STMG_F64 else "f32", "N": ctx.N, "levels": ctx.num_levels(),
           "converged": rc == 0, "newton": st.newton_its, "fgmres": list(st.fgmres_its[: st.newton_its]),
           "rebuilds": st.rebuilds, "res_rel": st.res_M / st.res0_M, "wall_s": wall,
           "solves_per_s": 1.0 / wall, "dof_per_s": ctx.N / wall, "kernel_s": tm}
    del ctx, u
    torch.cuda.empty_cache()
    return out


def bench_batched_lu(npatch=4096, seed=6):
    """Batched Vanka patch factorizations of mixed sizes: `npatch` full
    space-time surrogate patches (eq. LVS, eq. DefTildeHn) of interior cells of
    8^3-cell meshes (h = 1/8, tau = h/2), (r, k, nu) uniform on {1, 2, 3} x
    {0, 1, 2} x {1, 1e-2, 1e-3} (PCG64 seed), nodal states U(-1, 1); the
    patches are assembled by the library.  One stmg_batched_lu call per
    precision (FP64; FP32 with FP32, BF16 or FP16 operands of the
    trailing-update MFMA, FP32 accumulation), then the triangular solves;
    accuracy as the sampled normwise backward error and the relative
    distance of the solutions to the FP64 ones.  Each factorization is timed
    as one persistent launch with the tuned table and, as the untuned
    reference, as one launch per size class.  (The patches come from the
    library: only the cpu_baseline leg runs the oracle.)"""
    import torch
    from paper_2602_13841_amd import inputs as I
    from paper_2602_13841_amd import stmg
    rng = np.random.Generator(np.random.PCG64(seed))
    draws = [(int(rng.choice([1, 2, 3])), int(rng.choice([0, 1, 2])), float(rng.choice([1.0, 1e-2, 1e-3])))
             for _ in range(npatch)]
    combos = sorted(set(draws))
    n = 8
    interior = [c0 + n * (c1 + n * c2) for c2 in range(1, n - 1) for c1 in range(1, n - 1) for c0 in range(1, n - 1)]
    mats = {}
    for ci, (r, k, nu) in enumerate(combos):
        ctx = stmg.Context(3, (n, n, n), r, k, nu, 1.0 / 16, prec_mg=stmg.STMG_F64)
        ctx.smoother_rebuild(torch.tensor(I.uniform(ctx.N, 200 + ci), device="cuda"))
        need = sum(1 for d in draws if d == (r, k, nu))
        mats[(r, k, nu)] = [ctx.level_patch(0, interior[j % len(interior)]).clone().reshape(-1) for j in range(need)]
        del ctx
    used = {key: 0 for key in mats}
    blocks = []
    for dd in draws:
        blocks.append(mats[dd][used[dd]])
        used[dd] += 1
    del mats
    sizes = np.array([int(round(np.sqrt(b.numel()))) for b in blocks], dtype=np.int32)
    a_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)[:-1]])
    p_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))[:-1]])
    A64 = torch.cat(blocks)
    del blocks
    torch.cuda.empty_cache()
    flops = float(np.sum(2.0 / 3.0 * sizes.astype(np.float64) ** 3))
    out = {"patches": npatch, "sizes": [int(sizes.min()), int(sizes.max()), float(sizes.mean())],
           "lu_flops": flops}
    rng2 = np.random.Generator(np.random.PCG64(seed + 1))
    rhs = torch.tensor(rng2.uniform(-1, 1, int(sizes.sum())), device="cuda")
    x64 = None
    for name, dt, prec, peak in (("fp64", torch.float64, None, 78.6e12), ("fp32_mfma", torch.float32, None, 157.3e12),
                                 ("fp32_bf16_mfma", torch.float32, stmg.STMG_F32_BF16, 2.5e15),
                                 ("fp32_f16_mfma", torch.float32, stmg.STMG_F32_F16, 2.5e15)):
        A = A64.to(dt, copy=True)   # A64 stays the unfactored reference
        piv = torch.zeros(int(sizes.sum()), dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        # untuned reference: one launch per size class
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record()
        stmg.batched_lu(A, a_off, sizes, piv, p_off, info, prec=prec, config=(0, None))
        r1.record()
        torch.cuda.synchronize()
        t_ref = r0.elapsed_time(r1) * 1e-3
        A.copy_(A64.to(dt))
        info.zero_()
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        stmg.batched_lu(A, a_off, sizes, piv, p_off, info, prec=prec)
        e1.record()
        b = rhs.to(dt, copy=True)   # rhs stays the right-hand side of the check
        stmg.batched_lu_solve(A, a_off, sizes, piv, p_off, b, p_off)
        e2.record()
        torch.cuda.synchronize()
        t_lu, t_sv = e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2) * 1e-3
        # normwise backward error on a sample of patches (host check)
        x = b.double().cpu().numpy()
        worst = 0.0
        for i in list(range(0, npatch, max(1, npatch // 16))):
            M = A64[a_off[i]: a_off[i] + int(sizes[i]) ** 2].view(int(sizes[i]), -1).cpu().numpy()
            xi = x[p_off[i]: p_off[i] + sizes[i]]
            ri = rhs[p_off[i]: p_off[i] + sizes[i]].cpu().numpy()
            be = np.max(np.abs(M @ xi - ri)) / (np.max(np.abs(M).sum(1)) * np.max(np.abs(xi)) + np.max(np.abs(ri)))
            worst = max(worst, float(be))
        if x64 is None:
            x64 = x
        rel = [float(np.linalg.norm(x[p_off[i]: p_off[i] + sizes[i]] - x64[p_off[i]: p_off[i] + sizes[i]]) /
                     np.linalg.norm(x64[p_off[i]: p_off[i] + sizes[i]])) for i in range(npatch)]
        out[name] = {"lu_s": t_lu, "patches_per_s": npatch / t_lu, "tflops": flops / t_lu / 1e12,
                     "frac_of_peak": flops / t_lu / peak, "one_launch_per_size_class_s": t_ref,
                     "tuned_speedup": t_ref / t_lu, "solve_s": t_sv, "zero_pivots": int(info.item()),
                     "backward_error_sample_max": worst, "rel_err_vs_fp64_median": float(np.median(rel)),
                     "rel_err_vs_fp64_max": float(np.max(rel))}
        del A, piv, b
        torch.cuda.empty_cache()
    return out


def bench_serve(nreq, slots):
    """Serving: the first `nreq` requests of the seeded mixed stream (2D/3D,
    8..24 cells per axis, r in 1..3, k in 0..2, Re in {1, 100, 1000}).  A
    closed-loop run (all requests at t = 0) gives the throughput X; a second
    run with Poisson arrivals at 0.8 X gives the latencies (completion -
    arrival)."""
    import torch
    from paper_2602_13841_amd import inputs as I
    from paper_2602_13841_amd import stmg
    reqs = I.serving_stream(nreq, 7)
    o = stmg.default_options(newton_rtol=1e-8, newton_atol=0.0)
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.85)
    # per-request progress lines of the serving loop on stderr
    os.environ["STMG_VERBOSE"] = "1"
    for q in reqs:
        q["arrival_s"] = 0.0
    _, res, wall = stmg.serve(reqs, o, slots=slots, hbm_budget=budget)
    X = nreq / wall
    lam = 0.8 * X
    arr = I.poisson_arrivals(nreq, lam, 8)
    for q, a in zip(reqs, arr):
        q["arrival_s"] = float(a)
    _, res2, wall2 = stmg.serve(reqs, o, slots=slots, hbm_budget=budget)
    lat = np.array([x.latency_s for x in res2])
    ok = sum(1 for x in res + res2 if x.rc == 0)
    # how often a request shares the device with another of the same
    # discretization (the only case where merging cell-kernel launches across
    # requests could apply): fraction of in-slot time with such a partner
    def same_shape_overlap(rs):
        key = [(q["dim"], tuple(q["n"]), q["r"], q["k"]) for q in reqs]
        tot = shared = 0.0
        for i, x in enumerate(rs):
            tot += x.end_s - x.start_s
            iv = sorted((max(x.start_s, y.start_s), min(x.end_s, y.end_s)) for j, y in enumerate(rs)
                        if j != i and key[j] == key[i] and min(x.end_s, y.end_s) > max(x.start_s, y.start_s))
            cur = None
            for a, b in iv:
                if cur is None or a > cur[1]:
                    if cur:
                        shared += cur[1] - cur[0]
                    cur = [a, b]
                else:
                    cur[1] = max(cur[1], b)
            if cur:
                shared += cur[1] - cur[0]
        return shared / max(tot, 1e-30)
    classes, sizes = {}, {}
    for q, x in zip(reqs, res2):
        classes.setdefault(f"{q['dim']}D", []).append(x.latency_s)
        sizes.setdefault(f"{q['dim']}D n={q['n'][0]}", []).append(x.latency_s)
    return {"requests": nreq, "slots": slots, "hbm_budget_GB": budget / 1e9, "closed_loop_wall_s": wall,
            "solves_per_s": X, "arrival_rate": lam, "poisson_wall_s": wall2,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_by_dim": {k: float(np.percentile(v, 50)) for k, v in classes.items()},
            "p99_by_dim": {k: float(np.percentile(v, 99)) for k, v in classes.items()},
            "p50_p99_by_size": {k: [float(np.percentile(v, 50)), float(np.percentile(v, 99)), len(v)]
                                for k, v in sorted(sizes.items())},
            "converged": ok, "runs": 2 * nreq,
            "shapes": len({(q["dim"], tuple(q["n"]), q["r"], q["k"]) for q in reqs}),
            "pooled_context_reuse": [sum(x.reused_context for x in res), sum(x.reused_context for x in res2)],
            "same_shape_overlap_fraction": [same_shape_overlap(res), same_shape_overlap(res2)]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rotate-bytes", type=float, default=1.1 * 2 ** 30)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-batched-lu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="one 1 GiB device-to-device copy first (reference for the rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the slab solver runs on one GPU; multi-GPU sharding is not implemented, --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2602_13841_amd import inputs as I
    from paper_2602_13841_amd import stmg

    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    w = WORKLOAD
    ctx = stmg.Context(w["dim"], w["n"], w["r"], w["k"], w["nu"], w["tau"])
    N, Nv = ctx.N, ctx.Nv
    nq = (3 * w["r"] + 5) // 2
    U = I.slab_state(w["dim"], w["n"], w["r"], w["k"], 3, kind="smooth")
    X = I.uniform(N, 2)

    def run(dtype, steps, warmup, ctx=ctx):
        per_set = 3 * N * (8 if dtype == torch.float64 else 4)
        nsets = max(2, int(np.ceil(args.rotate_bytes / per_set)))
        Us = [torch.tensor(U, dtype=dtype, device=dev) for _ in range(nsets)]
        Xs = [torch.tensor(X, dtype=dtype, device=dev) for _ in range(nsets)]
        Ys = [torch.empty(N, dtype=dtype, device=dev) for _ in range(nsets)]
        for i in range(warmup):
            ctx.jacobian_vmult(Us[i % nsets], Xs[i % nsets], Ys[i % nsets])
        # pass 1: throughput, no events between the kernels
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            j = i % nsets
            ctx.jacobian_vmult(Us[j], Xs[j], Ys[j])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # pass 2: the same steps with HIP events around every kernel (on the
        # stream the kernels run on) for the per-kernel durations
        ctx.timing_reset()
        ctx.timing(True)
        torch.cuda.synchronize()
        for i in range(steps):
            j = i % nsets
            ctx.jacobian_vmult(Us[j], Xs[j], Ys[j])
        torch.cuda.synchronize()
        ctx.timing(False)
        suffix = "f64" if dtype == torch.float64 else "f32"
        cell_ms, cell_n = ctx.timing_get("cell_jac_" + suffix)
        face_ms, face_n = ctx.timing_get("face_jac_" + suffix)
        gat_ms, gat_n = ctx.timing_get("gather_" + suffix)
        ctx.timing_reset()
        # pass 3: at least 100 applications timed one by one (events on the
        # current stream, which the library launches on): median and spread
        nper = max(steps, 100)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nper)]
        torch.cuda.synchronize()
        for i in range(nper):
            j = i % nsets
            evs[i][0].record()
            ctx.jacobian_vmult(Us[j], Xs[j], Ys[j])
            evs[i][1].record()
        torch.cuda.synchronize()
        per = np.array([a.elapsed_time(b) for a, b in evs])
        del Us, Xs, Ys
        torch.cuda.empty_cache()
        stats = {"timed_one_by_one": nper, "median_ms": float(np.median(per)), "p10_ms": float(np.percentile(per, 10)),
                 "p90_ms": float(np.percentile(per, 90))}
        return ((t1 - t0) / steps, cell_ms / max(cell_n, 1), face_ms / max(face_n, 1), gat_ms / max(gat_n, 1),
                nsets, stats)

    # device copy of 1 GiB each way: the HBM rate a plain copy reaches here
    src_ = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst_ = torch.empty_like(src_)
    for _ in range(2):
        dst_.copy_(src_)
    ce = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    torch.cuda.synchronize()
    for a, b in ce:
        a.record()
        dst_.copy_(src_)
        b.record()
    torch.cuda.synchronize()
    copy_s = min(a.elapsed_time(b) for a, b in ce) * 1e-3
    copy_gbs = 2 * src_.numel() * 8 / copy_s / 1e9
    del src_, dst_
    torch.cuda.empty_cache()

    t64, cell64, face64, gat64, nsets64, per64 = run(torch.float64, args.steps, args.warmup)
    t32, cell32, face32, gat32, nsets32, per32 = run(torch.float32, args.steps, args.warmup)

    # the FP64 slab residual R_n(U) of the same workload (eq. InAlgNS): at least
    # 100 applications timed one by one, input sets rotating as above
    def run_residual(nrep=100, warmup=5):
        per_set = 2 * N * 8
        nsets = max(2, int(np.ceil(args.rotate_bytes / per_set)))
        Us = [torch.tensor(U, device=dev) for _ in range(nsets)]
        Rs = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(nsets)]
        for i in range(warmup):
            ctx.residual(Us[i % nsets], Rs[i % nsets])
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nrep)]
        torch.cuda.synchronize()
        for i in range(nrep):
            evs[i][0].record()
            ctx.residual(Us[i % nsets], Rs[i % nsets])
            evs[i][1].record()
        torch.cuda.synchronize()
        per = np.array([a.elapsed_time(b) for a, b in evs])
        del Us, Rs
        torch.cuda.empty_cache()
        return {"value": N / (np.median(per) * 1e-3), "unit": "DoF/s", "median_ms": float(np.median(per)),
                "p10_ms": float(np.percentile(per, 10)), "p90_ms": float(np.percentile(per, 90)),
                "timed_one_by_one": nrep, "rotating_sets": nsets}

    res64 = run_residual()
    del ctx
    torch.cuda.empty_cache()
    # the same workload with the cheaper spatial quadrature n_q = r + 2
    nq_p = w["r"] + 2
    ctxp = stmg.Context(w["dim"], w["n"], w["r"], w["k"], w["nu"], w["tau"], n_q=nq_p)
    tp64, cellp64, facep64, gatp64, _, perp64 = run(torch.float64, args.steps, args.warmup, ctxp)
    tp32, cellp32, facep32, gatp32, _, perp32 = run(torch.float32, args.steps, args.warmup, ctxp)
    del ctxp
    torch.cuda.empty_cache()

    flops = vmult_flops(w["dim"], w["n"], w["r"], w["k"], nq)
    flops_p = vmult_flops(w["dim"], w["n"], w["r"], w["k"], nq_p)
    bytes64 = (2 * N + Nv) * 8
    achieved = flops / (cell64 * 1e-3)
    traffic, traffic_note = counter_traffic()
    out = {
        "metric": "space-time DoF/s Jacobian vmult FP64 vs FP32; slab solves/s; p50/p99 latency",
        "value": N / t64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "vmult 3D unit cube 16^3 affine hexes Q3/P2disc (r=2) x DG(2), Re=100, "
                               "tau=1/32, smooth divergence-free Fourier state",
                   "N": N, "n_q": nq, "rotating_sets": nsets64},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
                     "traffic_source": traffic_note,
                     "kernel": "jac_cell_kernel<2,5,192,f64> (3D Jacobian volume terms)",
                     "flops_per_launch": flops,
                     "flops_per_launch_performed": vmult_flops_performed(w["n"], w["r"], w["k"], nq),
                     "kernel_ms": cell64},
        "roofline_hbm": {"achieved": bytes64 / ((cell64 + face64 + gat64) * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": bytes64 / ((cell64 + face64 + gat64) * 1e-3) / PEAK_HBM,
                         "algorithmic_bytes": bytes64, "cell_ms": cell64, "face_ms": face64, "gather_ms": gat64,
                         "device_copy_GBps": copy_gbs, "frac_of_device_copy": bytes64 / (t64 * copy_gbs * 1e9)},
        "per_application_fp64": per64,
        "residual_fp64": res64,
        "fp32": {"value": N / t32, "unit": "DoF/s", "ms_per_step": t32 * 1e3, "cell_ms": cell32,
                 "face_ms": face32, "gather_ms": gat32, "speedup_vs_fp64": t64 / t32, "per_application": per32},
        "nq_r_plus_2": {"n_q": nq_p, "fp64": {"value": N / tp64, "ms_per_step": tp64 * 1e3, "cell_ms": cellp64,
                                               "face_ms": facep64, "gather_ms": gatp64, "per_application": perp64,
                                               "alu_frac": flops_p / (cellp64 * 1e-3) / PEAK_FP64_VALU,
                                               "hbm_frac": bytes64 / (tp64 * PEAK_HBM)},
                        "fp32": {"value": N / tp32, "ms_per_step": tp32 * 1e3, "cell_ms": cellp32,
                                 "face_ms": facep32, "gather_ms": gatp32, "per_application": perp32,
                                 "hbm_frac": bytes64 / 2 / (tp32 * PEAK_HBM)}},
    }
    if not args.no_solve:
        print("[bench] slab solve, FP32 multigrid", file=sys.stderr, flush=True)
        s32 = bench_solve(stmg.STMG_F32)
        print("[bench] slab solve, FP32 multigrid, BF16 copy of the patch factors", file=sys.stderr, flush=True)
        s16 = bench_solve(stmg.STMG_F32, vanka_factor_bf16=1)
        print("[bench] slab solve, FP32 multigrid, diagonal Vanka", file=sys.stderr, flush=True)
        sdv = bench_solve(stmg.STMG_F32, vanka_diagonal=1)
        print("[bench] slab solve, FP64 multigrid", file=sys.stderr, flush=True)
        s64 = bench_solve(stmg.STMG_F64)
        out["solve"] = {"workload": "3D 32^3 hexes perturbed by 0.2h, Q4/P3disc (r=3) x DG(1), Re=1000, "
                                    "tau=1/64, smooth previous-slab velocity, |R|_M <= 1e-8 |R_0|_M",
                        "fp32_mg": s32, "fp32_mg_bf16_factors": s16, "fp32_mg_diagonal_vanka": sdv,
                        "fp64_mg": s64,
                        "speedup_fp32_vs_fp64": s64["wall_s"] / s32["wall_s"]}
    if not args.no_batched_lu:
        print("[bench] batched patch factorizations", file=sys.stderr, flush=True)
        out["batched_lu"] = bench_batched_lu()
    if not args.no_serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = bench_serve(args.serve_requests, args.serve_slots)
    if not args.no_cpu_baseline:
        U_, X_ = U, X
        out["cpu_baseline"] = cpu_baseline(U_, X_)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
