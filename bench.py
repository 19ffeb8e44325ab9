#!/usr/bin/env python3
"""Benchmark of the SIS hot path on one MI355X.

Headline workload (default): Poiseuille flow through quarter rectangular ducts
of aspect ratio 1 and 2 (Sec. 2.4, Sec. 5.3), 64 x 64 cells growing by 1.05
from the walls, inverse-power-law gas with viscosity index 0.81, 24^3
velocities on [-6, 6]^3 padded to 48^3, M = 8 (64 solid-angle directions),
delta in {1, 10, 50} per aspect ratio: 6 cases x 4096 = 24 576 spatial cells
in one batch (the largest single-GPU workload of the set).

A step is one SIS outer iteration over the whole batch: collision (fast-spectral
operator contraction + epilogue), transport sweep, moments, velocity equation,
flow rates and convergence test, launched as one captured HIP graph.
value = cells x steps / wall time (cell-updates of L(h) per second, inputs
resident in HBM).

Distributions are stored by parity (default): these flows are odd in v3 (and
even in v2 in the planar geometry), which the discrete operator preserves, so
the plan keeps the v3 > 0 (v2 > 0) part and the operator restricted to it;
the solution is the full-grid one (equal to 1e-12).  --parity 0 runs the
full grid.

Also reported: the collision contraction's roofline (HIP events around each
eager launch), the per-cell fast-spectral transform path (sis_collide_fsm)
timed against the method's own flop count, the transport sweep's bandwidth,
the time-to-residual 1e-8 of FP64 vs mixed-precision collision, smaller
workloads of the same set as extra keys, and the CPU oracle timed on the
host's cores (one process per core) with its extrapolated time-to-residual.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s of L(h) + time-to-residual 1e-8, mixed SIS vs FP64 plain"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}
# HBM bytes per contraction launch from the FETCH_SIZE / WRITE_SIZE counter passes
# (scaled by a 1 GiB copy: FETCH x2.0, WRITE x1.0), recorded for the kernel as it
# stands, keyed by (workload, parity, precision, tile rows, split-K, k-stage), with the
# profile summary that holds the pass; a launch configuration without a recorded pass
# reports null.
TRAFFIC_KIB = {
    ("planar-hs-32v-100cells-8cases", 2, "fp64", 64, 3, 32):
        (1116445.9 * 2.0, 155136.0, "profiles/gemm_f64_planar-hs-32v-808cells-parity.md"),
    ("planar-hs-32v-100cells-8cases", 2, "fp64", 64, 4, 16):
        (1546552.0 * 2.0, 206848.0, "profiles/gemm_f64_planar-hs-32v-808cells-parity.md"),
    ("planar-hs-32v-100cells-8cases", 2, "fp64", 128, 4, 16):
        (1142963.6 * 2.0, 206848.0, "profiles/gemm_f64_planar-hs-32v-808cells-parity.md"),
    ("duct-ipl081-24v-64x64-6cases", 1, "fp64", 128, 1, 16):
        (19409697.6 * 2.0, 1327104.0, "profiles/gemm_f64_duct-ipl-24v-64x64-6cases.md"),
    ("duct-ipl081-24v-64x64-6cases", 1, "bf16x3", 256, 1, 32):
        (3697812.8 * 2.0, 1327104.0, "profiles/gemm_bf16x3_duct-ipl-24v-64x64-6cases_planar-hs-32v-808cells.md"),
    ("duct-ipl081-24v-64x64-6cases", 1, "bf16x3", 256, 2, 32):
        (3711624.7 * 2.0, 2654208.0, "profiles/gemm_bf16x3_duct-ipl-24v-64x64-6cases_planar-hs-32v-808cells.md"),
    ("planar-hs-32v-100cells-8cases", 2, "bf16x3", 256, 2, 32):
        (239174.1 * 2.0, 103424.0, "profiles/gemm_bf16x3_duct-ipl-24v-64x64-6cases_planar-hs-32v-808cells.md")}
# MFMA pipe utilisation of the same configuration from its counter pass:
# SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD x 1024 SIMDs), and the shader clock
# the kernel ran at (GRBM_GUI_ACTIVE per XCD / kernel duration).
MFMA_BUSY = {("planar-hs-32v-100cells-8cases", 2, "fp64", 64, 3, 32): (0.779, 2.22),
             ("planar-hs-32v-100cells-8cases", 2, "fp64", 64, 4, 16): (0.788, 2.09),
             ("planar-hs-32v-100cells-8cases", 2, "fp64", 128, 4, 16): (0.927, 2.08),
             ("duct-ipl081-24v-64x64-6cases", 1, "fp64", 128, 1, 16): (0.932, 2.33),
             ("duct-ipl081-24v-64x64-6cases", 1, "bf16x3", 256, 1, 32): (0.678, 2.28),
             ("duct-ipl081-24v-64x64-6cases", 1, "bf16x3", 256, 2, 32): (0.686, 1.87),
             ("planar-hs-32v-100cells-8cases", 2, "bf16x3", 256, 2, 32): (0.689, 2.09)}
HBM_GBS = 8000.0
# worker processes of the CPU baseline: the host's cores, at most the 16 that a
# one-GPU share of the box holds
MAX_CPU_WORKERS = 16


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def fsm_flops(n_pad, n_dir):
    """The fast spectral method's own flop count per cell update: 1 forward, 2D
    inverse and 1 loss inverse real 3-D FFT of n_pad^3 points (2.5 N log2 N each)
    plus the spectral multiplications and products (6 D n_pad^3)."""
    import math
    n3 = n_pad ** 3
    return (2 * n_dir + 2) * 2.5 * n3 * math.log2(n3) + 6 * n_dir * n3


# ------------------------------------------------------------------ CPU baseline
_CPU = {}


def _cpu_worker(args):
    """Time L(h) of the cells [lo, hi) of the sample with the parent's oracle
    (inherited through fork) on one core."""
    lo, hi = args
    op, h = _CPU["op"], _CPU["h"]
    t0 = time.perf_counter()
    for c in range(lo, hi):
        op.apply(h[c])
    return hi - lo, time.perf_counter() - t0


def cpu_baseline(w, seconds, n_cells_total, per_case, planar):
    """The oracle (NumPy FFT form of L; mixture: its Carleman form) timed on the
    host's cores, one process per core, on a bounded sample of the workload's cells
    (about `seconds` of wall time).  Runs before anything initialises the GPU, so the
    forked workers hold no device state.  Also times the oracle's transport sweep of
    one case, for the extrapolated time-to-residual (see extrapolate_ttr)."""
    import multiprocessing as mp
    from paper_1612_04488_amd import inputs
    from oracle.velocity import VelocityGrid
    t0 = time.perf_counter()
    mix = w.get("mixture")
    if mix:
        from oracle import mixture
        op = mixture.MixtureFSM(VelocityGrid(w["n_v"], w["l_v"]), mix["masses"], mix["diameters"], mix["chi"],
                                n_pad=w["n_pad"], m_angle=w["m_angle"], m_rho=mix["m_rho"])
        for a in range(2):
            for b in range(2):
                op._feq_factors(a, b)
    else:
        from oracle import collision
        alpha = 2.0 * (1.0 - w.get("visc_index", 0.81)) if w["kernel"] == "ipl" else 1.0
        op = collision.FSM(VelocityGrid(w["n_v"], w["l_v"]), n_pad=w["n_pad"], m_angle=w["m_angle"], alpha=alpha)
    t_build = time.perf_counter() - t0
    # one cell first: sets the sample size for the time budget
    gen = inputs.mixture_h if mix else inputs.smooth_h
    h1 = gen(w["n_v"], w["l_v"], 1)
    t0 = time.perf_counter()
    op.apply(h1[0])
    t_one = time.perf_counter() - t0
    workers = max(1, min(os.cpu_count() or 1, MAX_CPU_WORKERS))
    per_worker = max(1, int(seconds / max(t_one, 1e-6)))
    h = gen(w["n_v"], w["l_v"], per_worker * workers)
    _CPU["op"], _CPU["h"] = op, h
    chunks = [(i * per_worker, (i + 1) * per_worker) for i in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    _CPU.clear()
    done = sum(r[0] for r in res)
    rate = done / wall
    out = {"value": rate, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
           "sample": (f"L(h) of {done} smooth cells of the benchmark batch, {workers} processes "
                      f"(one per core, NumPy FFT single-threaded each) for {wall:.1f} s; table build "
                      f"{t_build:.1f} s excluded"),
           "cpu": _cpu_model(), "host_cpu_count": os.cpu_count()}
    t_sweep_case = None
    if not mix and planar:
        from oracle import transport
        x = inputs.workload_nodes(w)[0]
        rhs = inputs.smooth_h(w["n_v"], w["l_v"], len(x))
        t0 = time.perf_counter()
        transport.sweep_1d(rhs, op.nu, x, op.grid)
        t_sweep_case = time.perf_counter() - t0
    elif not mix and w["name"].startswith("duct"):
        from oracle import duct
        f1, f2, _ = inputs.duct_cases(w)[0]
        g = duct.Grid2D(f1, f2, (duct.WALL, duct.SYM, duct.WALL, duct.SYM))
        rhs = inputs.smooth_h(w["n_v"], w["l_v"], len(g.cells))
        t0 = time.perf_counter()
        duct.sweep_2d(rhs, op.nu, g, op.grid, rhs)
        t_sweep_case = time.perf_counter() - t0
    out["_t_sweep_case"] = t_sweep_case
    out["_n_cells"] = n_cells_total
    out["_n_cases"] = len(per_case)
    return out


def extrapolate_ttr(cb, iters_fp64):
    """Oracle time to residual 1e-8: the FP64 solve's iteration count (slowest case;
    all cases run in one batch) x the per-iteration cost, i.e. the collision of every
    cell at the measured multi-core rate plus the oracle's sweep of one case per case,
    the cases spread over the worker processes."""
    t_sweep, n_cells, n_cases = cb.pop("_t_sweep_case"), cb.pop("_n_cells"), cb.pop("_n_cases")
    if not iters_fp64:
        return
    workers = cb["cores"]
    t_iter = n_cells / cb["value"] + (t_sweep or 0.0) * -(-n_cases // workers)
    cb["time_to_residual_1e-8_extrapolated"] = {
        "seconds": t_iter * max(iters_fp64), "per_iteration_seconds": t_iter,
        "iterations": int(max(iters_fp64)),
        "basis": ("extrapolated: the GPU FP64 solve's iteration count (slowest case, all cases in one batch) x "
                  f"(collision of all {n_cells} cells at the measured multi-core rate"
                  + (f" + the oracle's sweep of one case, {t_sweep:.2f} s, for each of the {n_cases} cases "
                     f"spread over {workers} processes" if t_sweep is not None else "")
                  + "); velocity equation and flow rates not included")}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------ one workload
def build_workload(key, args):
    from paper_1612_04488_amd import inputs, sis
    import numpy as np
    w = {"batch": inputs.PLANAR_BATCH, "small": inputs.PLANAR_SMALL, "duct": inputs.DUCT_IPL,
         "porous": inputs.POROUS_HS, "mixture": inputs.MIX_NEAR, "mixture-ragged": inputs.MIX_RAGGED,
         "mixture-duct": inputs.MIX_DUCT, "sierpinski": inputs.SIERPINSKI_HS, "tube": inputs.TUBE_HS}[key]
    mix = w.get("mixture")
    # penalty N of the SIS velocity equations: nubar for one gas, 1.5 for the
    # mixture and the carpets (the values the paper runs them with)
    Npen = 1.5 if mix or key == "sierpinski" else 0.0
    planar = key in ("batch", "small", "mixture", "mixture-ragged")
    tube = key == "tube"
    parity = (2 if planar else (0 if tube else 1)) if args.parity == "auto" else int(args.parity)
    t0 = time.perf_counter()
    plan = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], kernel=w["kernel"],
                    visc_index=w.get("visc_index", 0.81), mixture=mix, parity=parity, polar=w.get("polar"))
    t_plan = time.perf_counter() - t0
    info = plan.info
    log(f"plan {w['name']}: {t_plan:.2f} s (host {info['plan_seconds_host']:.2f} s, device "
        f"{info['plan_seconds_device']:.2f} s), operator {info['operator_bytes'] / 2**30:.2f} GiB")
    t0 = time.perf_counter()
    diff_info = None
    if tube:
        xs = [inputs.tube_radial(w["radial"])] * len(w["deltas"])
        geom = sis.Geometry(plan, xs, w["deltas"], w["flows"], kind="tube")
        per_case = [len(x) for x in xs]
        Npen = 1.0
    elif planar:
        xs = inputs.workload_nodes(w)
        geom = sis.Geometry(plan, xs, w["deltas"], w["flows"])
        per_case = [len(x) for x in xs]
    else:
        cases = {"duct": inputs.duct_cases, "porous": inputs.porous_cases, "mixture-duct": inputs.duct_cases,
                 "sierpinski": inputs.sierpinski_cases}[key](w)
        geom = sis.Geometry2D(plan, "periodic" if key == "porous" else "duct", cases, w["deltas"], w["flows"])
        per_case = np.diff(geom.offsets).tolist()
        if args.diffusion == "cg":
            geom.diffusion_solver("cg")
        n_inv, n_dist, inv_res = geom.diffusion_info()
        diff_info = {"solver": args.diffusion, "cases_on_inverse": n_inv, "distinct_inverses": n_dist,
                     "inverse_residual": inv_res, "sweep_form": geom.sweep_form()}
    t_geom = time.perf_counter() - t0
    log(f"geometry: {t_geom:.2f} s" + (f", velocity equation {diff_info}" if diff_info else ""))
    return dict(key=key, w=w, mix=mix, Npen=Npen, planar=planar, tube=tube, parity=parity, plan=plan,
                info=info, geom=geom, per_case=per_case, t_plan=t_plan, t_geom=t_geom, diff_info=diff_info)


def stored_h(W, nc):
    """Smooth synthetic distributions of the workload, restricted to the stored parity half."""
    import numpy as np
    from paper_1612_04488_amd import inputs
    w, parity = W["w"], W["parity"]
    if W["tube"]:
        return inputs.tube_h(W["plan"].n_dof, nc)
    h0 = inputs.mixture_h(w["n_v"], w["l_v"], nc) if W["mix"] else inputs.smooth_h(w["n_v"], w["l_v"], nc)
    hv = w["n_v"] // 2
    if parity >= 1:
        h0 = h0[..., hv:]
    if parity == 2:
        h0 = h0[..., hv:, :]
    return np.ascontiguousarray(h0).reshape(nc, -1)


def step_rate(W, precision, steps, warmup):
    """Whole-step throughput: `steps` SIS iterations of the batch as graph replays."""
    import torch
    from paper_1612_04488_amd import sis
    plan, geom = W["plan"], W["geom"]
    plan.set_precision(precision)
    state = sis.State(plan, geom, scheme="SIS", N=W["Npen"], eps=0.0, max_it=1 << 30,
                      project=precision != "fp64" and not W["mix"] and not W["tube"])
    state.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    state.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    state.close()
    log(f"{W['w']['name']}: {steps} steps: wall {wall * 1e3:.2f} ms, events {ev_ms:.2f} ms")
    return wall, ev_ms


def contraction_roofline(W, precision, reps):
    """HIP-event duration of the eager contraction launches (the dominant kernel of a step)."""
    import numpy as np
    import torch
    plan, geom = W["plan"], W["geom"]
    nc, n3 = geom.n_cells, plan.n_dof
    plan.set_precision(precision)
    h = torch.tensor(stored_h(W, nc), device="cuda")
    delta = torch.tensor(np.repeat(W["w"]["deltas"], W["per_case"]), dtype=torch.float64, device="cuda")
    rhs = torch.empty_like(h)
    plan.collide(h, delta, rhs)   # warm (and tune)
    torch.cuda.synchronize()
    plan.timing(True)
    for _ in range(reps):
        plan.collide(h, delta, rhs)
    gemm_ms, launches = plan.timing_read()
    plan.timing(False)
    tile_rows, splits, tuned, k_stage = plan.contraction_config(nc, precision, with_depth=True)
    avg_ms = gemm_ms / launches
    flops = 2.0 * n3 * n3 * nc
    executed = flops * (3 if precision == "bf16x3" else 1)
    achieved = executed / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    tile = "256x256" if tile_rows == 256 else f"{tile_rows}x128"
    log(f"contraction ({precision}): {avg_ms:.3f} ms/launch, {achieved:.1f} TFLOP/s of {peak} peak "
        f"(tile {tile}, k-stage {k_stage}, split-K {splits}, autotuned {tuned})")
    ck = (W["w"]["name"], W["parity"], precision, tile_rows, splits, k_stage)
    tk, mb = TRAFFIC_KIB.get(ck), MFMA_BUSY.get(ck)
    info = W["info"]
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": (tk[0] + tk[1]) * 1024.0 if tk else None,
            "mfma_busy": mb[0] if mb else None, "clock_ghz_counters": mb[1] if mb else None,
            "counters_source": tk[2] if tk else None,
            "kernel": f"gemm_{precision}", "avg_launch_ms": round(avg_ms, 4),
            "tile": tile, "k_stage": k_stage, "split_k": splits, "autotuned": tuned,
            "work_per_unit": "2 n_dof^2 flops per cell update (the dense operator of L+ applied to one cell)",
            "flops_per_launch": executed, "flops_per_cell_update": 2.0 * n3 * n3}
    if not W["mix"] and not W["tube"]:
        fa = fsm_flops(info["n_pad"], info["n_dir"])
        roof["fsm_flops_per_cell_update"] = fa
        roof["fsm_equivalent_tflops"] = round(fa * nc / (avg_ms * 1e-3) / 1e12, 1)
    return roof, h, delta, rhs


def sweep_rate(W, rhs, reps):
    import torch
    from paper_1612_04488_amd import sis
    plan, geom = W["plan"], W["geom"]
    nc, n3 = geom.n_cells, plan.n_dof
    hh = torch.zeros_like(rhs)
    mom_s = torch.empty((nc, geom.mom_stride * plan.n_species), dtype=torch.float64, device="cuda")
    sis.transport_sweep(plan, geom, rhs, hh, mom_s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sis.transport_sweep(plan, geom, rhs, hh, mom_s)
    e1.record()
    torch.cuda.synchronize()
    sweep_ms = e0.elapsed_time(e1) / reps
    sweep_bytes = 16.0 * nc * n3          # rhs read + h written per (cell, unknown)
    kern = "sweep_tube" if W["tube"] else ("sweep1d" if W["planar"] else "sweep2d")
    out = {"kernel": kern, "avg_ms_with_moments": round(sweep_ms, 4), "algorithmic_bytes": sweep_bytes,
           "achieved": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9, 1), "peak": HBM_GBS, "unit": "GB/s",
           "frac": round(sweep_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_GBS, 4)}
    log(f"transport sweep + moments: {sweep_ms:.3f} ms, {out['achieved']} GB/s of {HBM_GBS} (algorithmic 16 B "
        f"per (cell, unknown))")
    return out


def fsm_path(W, h, delta, reps):
    """The per-cell fast-spectral transform path (sis_collide_fsm) on the same batch:
    kernel time against the method's own flop count and against what it executes."""
    import torch
    from paper_1612_04488_amd import sis
    plan, geom = W["plan"], W["geom"]
    nc = geom.n_cells
    rhs = torch.empty_like(h)
    plan.collide_fsm(h, delta, rhs)   # warm
    torch.cuda.synchronize()
    plan.timing(True)
    for _ in range(reps):
        plan.collide_fsm(h, delta, rhs)
    ms, launches = plan.timing_read(fsm=True)
    plan.timing(False)
    avg_ms = ms / launches
    fi = plan.fsm_info()
    fa = fsm_flops(W["info"]["n_pad"], W["info"]["n_dir"])
    alg = fa * nc / (avg_ms * 1e-3) / 1e12
    exe = fi["flops_per_cell"] * nc / (avg_ms * 1e-3) / 1e12
    out = {"kernel": "fsm_collide (forward transform, 2D + 1 multiplied inverse transforms, field products)",
           "avg_call_ms": round(avg_ms, 3), "cell_updates_per_s": nc / (avg_ms * 1e-3),
           "roofline": {"bound": "mfma", "achieved": round(alg, 3), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                        "frac": round(alg / PEAK_TFLOPS["fp64"], 4),
                        "work_per_unit": "F_alg = (2D+2) 2.5 N_p^3 log2 N_p^3 + 6 D N_p^3 flops per cell update",
                        "flops_per_cell_update": fa},
           "executed": {"flops_per_cell_update": fi["flops_per_cell"], "achieved": round(exe, 3),
                        "frac": round(exe / PEAK_TFLOPS["fp64"], 4)},
           "vs_dense_contraction": None}
    log(f"fsm path: {avg_ms:.3f} ms per call, {alg:.2f} TFLOP/s of F_alg ({alg / 78.6:.3f} of peak), "
        f"executed {exe:.2f} TFLOP/s")
    return out


def ttr_runs(W, runs, refresh_every):
    import numpy as np
    from paper_1612_04488_amd import sis
    plan, geom = W["plan"], W["geom"]
    ttr, ref = {}, {}
    if W["mix"] or W["tube"]:
        runs = [(prec, proj) for prec, proj in runs if not proj]
    if W["mix"]:
        # one bf16 product is not offered for two-species plans
        runs = [(prec, proj) for prec, proj in runs if prec != "bf16"]
    for prec, proj in runs:
        plan.set_precision(prec)
        r = sis.solve(plan, geom, scheme="SIS", N=W["Npen"], eps=1e-8, max_it=400, project=proj,
                      raise_not_converged=False, refresh_every=refresh_every if prec != "fp64" else 0)
        key = prec + ("+projection" if proj else "")
        e = {"seconds": round(r["seconds"], 4), "iters": r["iters"].tolist(),
             "converged": bool(r["status"] == 0), "M": r["M"].tolist(), "Q": r["Q"].tolist()}
        if prec == "fp64":
            ref[proj] = r
            if proj and False in ref:
                e["projection_effect_M_vs_fp64"] = float(np.max(np.abs(r["M"] - ref[False]["M"]) / np.abs(ref[False]["M"])))
        elif proj in ref or False in ref:
            base = ref[proj] if proj in ref else ref[False]
            e["compared_with"] = "fp64" + ("+projection" if proj in ref and proj else "")
            e["max_rel_dev_M_vs_fp64"] = float(np.max(np.abs(r["M"] - base["M"]) / np.abs(base["M"])))
            e["max_rel_dev_Q_vs_fp64"] = float(np.max(np.abs(r["Q"] - base["Q"]) / np.abs(base["Q"])))
            e["speedup_vs_fp64"] = float(base["seconds"] / r["seconds"])
            e["refresh_every"] = refresh_every
        ttr[key] = e
        log(f"{W['w']['name']}: time-to-residual {key}: {r['seconds']:.4f} s, iters {r['iters'].tolist()}")
    plan.set_precision("fp64")
    return ttr


def ttr_persistent(W, launched):
    """Time to residual 1e-8 of the FP64 solve run as persistent cooperative launches
    (grid barriers between the steps of an iteration, 8 iterations per launch)."""
    from paper_1612_04488_amd import sis
    plan, geom = W["plan"], W["geom"]
    plan.set_precision("fp64")
    sis.solve(plan, geom, scheme="SIS", N=W["Npen"], eps=1e-8, max_it=400, persistent=1, check_every=8,
              raise_not_converged=False)
    r = sis.solve(plan, geom, scheme="SIS", N=W["Npen"], eps=1e-8, max_it=400, persistent=1, check_every=8,
                  raise_not_converged=False)
    import numpy as np
    e = {"seconds": round(r["seconds"], 4), "iters": r["iters"].tolist(), "converged": bool(r["status"] == 0),
         "max_rel_dev_M_vs_launched": float(np.max(np.abs(r["M"] - np.asarray(launched["M"])) / np.abs(launched["M"]))),
         "speedup_vs_launched": round(launched["seconds"] / r["seconds"], 3)}
    log(f"{W['w']['name']}: time-to-residual fp64 persistent: {r['seconds']:.4f} s, iters {r['iters'].tolist()}")
    return e


def library_reference(n_cells, n3, reps):
    """The vendor library's GEMM (torch.matmul: rocBLAS / hipBLASLt) on the contraction's own shape,
    timed back to back with HIP events on random operands: FP64 X[n_cells, n3] @ Op[n3, n3]^T, and
    the BF16 product with K = 3 n3 that the three products of the 3xBF16 contraction amount to
    (FP32 accumulation, BF16 output).  A reference point for the hand-written kernels only: the
    solver never calls it."""
    import torch
    out = {}
    g = torch.Generator(device="cuda").manual_seed(5)
    for name, dt, k, peak in (("fp64", torch.float64, n3, 78.6), ("bf16_k3n", torch.bfloat16, 3 * n3, 2500.0)):
        x = torch.randn(n_cells, k, dtype=dt, device="cuda", generator=g)
        op = torch.randn(n3, k, dtype=dt, device="cuda", generator=g)
        c = torch.empty(n_cells, n3, dtype=dt, device="cuda")
        torch.matmul(x, op.t(), out=c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.matmul(x, op.t(), out=c)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * n_cells * n3 * k / (ms * 1e-3) / 1e12
        out[name] = {"ms": round(ms, 4), "tflops": round(tf, 2), "frac": round(tf / peak, 4)}
        del x, op, c
    torch.cuda.empty_cache()
    out["what"] = ("torch.matmul (rocBLAS/hipBLASLt) on the same shape, back-to-back launches; fp64: X @ Op^T; "
                   "bf16_k3n: one BF16 GEMM with K = 3 n_dof, the work of the three BF16 products")
    return out


def config_of(W, precision):
    w, plan, geom, parity = W["w"], W["plan"], W["geom"], W["parity"]
    c = {"workload": w["name"], "kernel": w["kernel"], "n_v": w["n_v"], "l_v": w["l_v"], "n_pad": w["n_pad"],
         "directions": W["info"]["n_dir"], "cells": geom.n_cells, "cases": geom.n_cases,
         "nodes_per_case": [int(x) for x in W["per_case"]], "deltas": w["deltas"],
         "flows": w["flows"], "scheme": "SIS", "collision_precision": precision,
         "unknowns_per_cell": plan.n_dof, "species": plan.n_species,
         "parity": {0: "full grid", 1: "odd in v3 (v3 > 0 stored)",
                    2: "odd in v3, even in v2 (v2, v3 > 0 stored)"}[parity]}
    if W["diff_info"]:
        c["velocity_equation"] = W["diff_info"]
    if W["tube"]:
        c["n_pad"] = W["info"]["n_pad"]
        c["parity"] = "polar grid: th in [0, pi] (even), v_z > 0 (odd)"
        c["polar"] = w["polar"]
        c["radial_nodes"] = w["radial"]
    return c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "bf16"])
    keys = ["duct", "batch", "small", "porous", "mixture", "mixture-ragged", "mixture-duct", "sierpinski", "tube"]
    ap.add_argument("--workload", default="duct", choices=keys)
    ap.add_argument("--extras", default="batch,small,mixture-ragged",
                    help="smaller workloads of the set measured after the headline (comma list; '' for none): "
                         "whole-step rate, contraction, time-to-residual FP64 vs 3xBF16")
    ap.add_argument("--diffusion", default="inverse", choices=["inverse", "cg"],
                    help="2-D velocity equation: precomputed inverse or conjugate gradients")
    ap.add_argument("--ttr", default="fp64,fp32,bf16x3,fp64+projection,bf16x3+projection",
                    help="time-to-residual runs of the headline workload (comma list)")
    ap.add_argument("--parity", default="auto", choices=["auto", "0", "1", "2"],
                    help="parity storage (auto: 2 for planar workloads, 1 for 2-D cross sections)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall time budget of the CPU baseline's timed sample (all host cores)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--no-ttr", action="store_true", help="skip time-to-residual runs")
    ap.add_argument("--no-fsm", action="store_true", help="skip the per-cell transform path")
    ap.add_argument("--no-library", action="store_true",
                    help="skip timing the vendor library's GEMM on the contraction's shape")
    ap.add_argument("--cis-max-it", type=int, default=0,
                    help="also run the conventional iteration (FP64) with this iteration cap")
    ap.add_argument("--refresh-every", type=int, default=16,
                    help="mixed runs: FP64 anchors of the defect correction at iterations R/2, 3R/2, ...")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU (each box here has one); sharding "
                                   "the cases over several GPUs is not built",
                          "n_gpus": args.gpus}))
        return 2

    # the CPU baseline runs first, before anything touches the GPU, so that its
    # forked worker processes hold no device state
    cb = None
    if args.workload == "tube":
        log("cpu baseline: the tube oracle's dense transform matrices do not fit at the paper's polar grid; skipped")
    elif not args.no_cpu_baseline and not args.calibrate_copy:
        from paper_1612_04488_amd import inputs
        w0 = {"batch": inputs.PLANAR_BATCH, "small": inputs.PLANAR_SMALL, "duct": inputs.DUCT_IPL,
              "porous": inputs.POROUS_HS, "mixture": inputs.MIX_NEAR, "mixture-ragged": inputs.MIX_RAGGED,
              "mixture-duct": inputs.MIX_DUCT, "sierpinski": inputs.SIERPINSKI_HS}[args.workload]
        log("cpu baseline ...")
        planar0 = args.workload in ("batch", "small", "mixture", "mixture-ragged")
        if planar0:
            pc = [len(x) for x in inputs.workload_nodes(w0)]
        elif args.workload in ("duct", "mixture-duct"):
            pc = [w0["cells"] ** 2] * len(w0["deltas"])
        else:
            pc = [0] * len(w0["deltas"])
        cb = cpu_baseline(w0, args.cpu_seconds, sum(pc), pc, planar0)
        log(f"cpu baseline: {cb['value']:.2f} cell-updates/s on {cb['cores']} processes")

    import torch
    from paper_1612_04488_amd import sis  # noqa: F401  (fails loudly without libsis.so)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per copy: the reference for the FETCH_SIZE /
        # WRITE_SIZE counters of the contraction
        src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        for _ in range(5):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src_t.numel() * 8, "copy_bytes_written": dst_t.numel() * 8,
                          "copies": 5}), flush=True)
        return 0

    W = build_workload(args.workload, args)
    nc = W["geom"].n_cells
    wall, _ = step_rate(W, args.precision, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    value = nc * args.steps / wall
    reps = max(args.steps, 5)
    roofline, h, delta, rhs = contraction_roofline(W, args.precision, reps)
    lowp = None
    if args.precision == "fp64" and not W["tube"]:
        # the 3xBF16 contraction of the mixed-precision solves, on the same batch
        lowp, lh, ld, lr = contraction_roofline(W, "bf16x3", reps)
        del lh, ld, lr
        W["plan"].set_precision(args.precision)
    sweep = sweep_rate(W, rhs, reps)
    del rhs
    if not args.no_library and not W["mix"] and not W["tube"]:
        roofline["library_reference"] = library_reference(nc, W["plan"].n_dof, min(reps, 10))
    fsm = None
    if not args.no_fsm and not W["mix"] and not W["tube"] and hasattr(W["plan"], "collide_fsm"):
        W["plan"].set_precision("fp64")
        fsm = fsm_path(W, h, delta, max(3, min(reps, 5)))
        fsm["vs_dense_contraction"] = round(fsm["avg_call_ms"] / roofline["avg_launch_ms"], 2)
    del h, delta
    ttr = {}
    if not args.no_ttr:
        runs = [(r.split("+")[0], r.endswith("+projection")) for r in args.ttr.split(",") if r]
        ttr = ttr_runs(W, runs, args.refresh_every)
    cis = None
    if args.cis_max_it > 0:
        W["plan"].set_precision("fp64")
        r = sis.solve(W["plan"], W["geom"], scheme="CIS", N=W["Npen"], eps=1e-8, max_it=args.cis_max_it,
                      raise_not_converged=False)
        cis = {"seconds": round(r["seconds"], 4), "iters": r["iters"].tolist(), "max_it": args.cis_max_it,
               "converged": [bool(x < 1e-8) for x in r["residual"]], "M": r["M"].tolist()}
        log(f"conventional iteration (FP64, cap {args.cis_max_it}): {r['seconds']:.3f} s, "
            f"iters {r['iters'].tolist()}")

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "bf16": "bf16+f64"}[args.precision],
           "data": "synthetic",
           "config": config_of(W, args.precision),
           "roofline": roofline, "bf16x3_contraction": lowp, "sweep": sweep,
           "plan_seconds": round(W["t_plan"], 3), "geometry_seconds": round(W["t_geom"], 3),
           "time_to_residual_1e-8": ttr}
    if "fp64" in ttr:
        out["plan_plus_time_to_residual_1e-8"] = {
            k: round(W["t_plan"] + W["t_geom"] + v["seconds"], 3) for k, v in ttr.items()}
    if fsm is not None:
        out["fsm_path"] = fsm
    if cis is not None:
        out["conventional_iteration_fp64"] = cis
    iters_fp64 = ttr.get("fp64", {}).get("iters")
    keep = {"plan": W["plan"], "geom": W["geom"]}
    # ---------------------------------------------------------- extra workloads of the set
    extras = {}
    for key in [k for k in args.extras.split(",") if k and k != args.workload]:
        E = build_workload(key, args)
        en = E["geom"].n_cells
        ew, _ = step_rate(E, "fp64", args.steps, args.warmup)
        er, eh, ed, erhs = contraction_roofline(E, "fp64", reps)
        del eh, ed, erhs
        elp = None
        if not E["tube"]:
            elp, eh, ed, erhs = contraction_roofline(E, "bf16x3", reps)
            del eh, ed, erhs
            E["plan"].set_precision("fp64")
        et = ttr_runs(E, [("fp64", False), ("bf16x3", False)], args.refresh_every) if not args.no_ttr else {}
        if et and E["planar"] and not E["mix"] and en <= 64:
            # the persistent launch is meant for small batches (its contraction runs on at most
            # 64 workgroups with 32-row tiles)
            et["fp64_persistent"] = ttr_persistent(E, et["fp64"])
        extras[E["w"]["name"]] = {
            "value": en * args.steps / ew, "unit": "cell-updates/s", "ms_per_step": ew * 1e3 / args.steps,
            "config": config_of(E, "fp64"), "roofline": er, "bf16x3_contraction": elp,
            "plan_seconds": round(E["t_plan"], 3), "time_to_residual_1e-8": et}
        E["plan"].close()
        E["geom"].close()
    if extras:
        out["extra_workloads"] = extras
    if cb is not None:
        if cb["_n_cells"] != nc:   # porous and carpet cell counts are known only after the geometry
            cb["_n_cells"] = nc
            cb["_n_cases"] = len(W["per_case"])
        extrapolate_ttr(cb, iters_fp64)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = value / cb["value"]
    del keep
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
