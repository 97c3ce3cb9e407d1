"""Throughput of the Gaussian-RBF hot path on one MI355X.

One step = one pass of the whole path over the torus workload (200,000
surface points, 600,000 centres, sigma 0.02, cutoff 4 sigma):
  setup      extended centres, Morton sort, cells, source lists;
  solve      one refinement step of the chosen pipeline: a GMRES(30) cycle on
             the float32 operator (30 applications) and the float64 true
             residual of its result (1 application);
  grid       the interpolant on the 256^3 grid around the cloud.
value = useful kernel evaluations (pairs with r <= cutoff) of every operator
application and of the grid, divided by the step time.  Inputs (points,
normals) are resident in device memory before timing starts.

Fields beside the step (all measured after the timed steps):
  roofline      the float32 operator kernel's live launch time (HIP events in
                its dispatches during the timed steps) against the pair peak,
                with its HBM bytes from the committed counter summary;
  phases, pairs setup / cycle / grid split, matvec times, pair counts;
  schwarz, schwarz1024, schwarz_half, schwarz1024_half
                the Schwarz preconditioner with blocks up to 192 and with
                blocks of 64..1024, its local inverses in float32 and in
                float16: setup, local inverses, apply time and its HBM
                fraction;
  solve         the second half of the metric: setup -> solve -> grid to
                relative residual 1e-8 (or 3,000 operator applications) for
                the refinement (float32 and float64 Krylov basis), the same
                with each Schwarz configuration (float32 and float16 local
                inverses), and the plain float64
                method; residual/time histories, stall levels, and time to
                the lowest residual all reach with the speed-up over plain;
  signs         every pipeline's 256^3 grid against the plain method's on the
                nodes with |f| > 1e-6 + 8 u32 sum_j |c_j phi_j| (and the
                torus's signed distance);
  cpu_baseline  the C cell-list oracle (float64, OpenMP) on one thread and on
                every host thread: the operator's rows (all of them, and a
                sample on one thread), band points of the grid, one GMRES(30)
                cycle of the oracle, and the solve's time extrapolated from
                that cycle.
  roofline.measured_rates
                the device's vector-ALU issue rates (FMA, v_exp_f32 and their
                mixes) from register-resident loops: the evidence for the pair
                peak's cost model.

Prints one JSON line.  --gpus above 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RBF kernel evals/s (% FP32 roofline); solve+grid time to resid 1e-8 vs plain"

# Pair roofline of the float32 kernel (alu bound):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-slots/s.  A useful
# pair needs at least four float32 operations (2 t.s as one multiply and two
# FMAs, and the FMA of the weighted sum) and one exponential.  At the
# published vector FP32 peak (packed, two operations per lane-slot) the four
# take 2 slots; v_exp_f32 issues at half the FMA rate on gfx950 (2 slots).
# 4 slots per pair: 9.83e12 pairs/s.
LANE_SLOTS = 256 * 4 * 16 * 2.4e9
PEAK_PAIRS = LANE_SLOTS / 4.0

# HBM bytes per operator launch of the float32 kernel, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a copy of
# known size; valid only for the kernel source they were taken on.
COUNTERS = os.path.join(ROOT, "profiles", "k_pairsum_f32_torus200k_hbm_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1305_5179_amd", "csrc", "pairsum.hip")


def measured_traffic():
    import hashlib
    import re
    if not os.path.exists(COUNTERS):
        return None, "no counter summary"
    text = open(COUNTERS).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"operator_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_b):
        return None, "counter summary unreadable"
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if sha != m_sha.group(1):
        return None, "kernel changed since the counters were taken"
    return float(m_b.group(1)), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["torus", "metaballs"], default="torus",
                    help="torus: 200k points / 600k centres (default); metaballs: 2M points / 6M centres, "
                         "hole and noise, 512^3 grid")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-row-frac", type=float, default=0.08,
                    help="share of the operator rows the one-thread CPU oracle run evaluates")
    ap.add_argument("--cpu-points", type=int, default=800_000,
                    help="band points the CPU oracle evaluates the interpolant at (all threads; 1/10 on one)")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the solves to a common residual (chosen pipelines vs plain float64) and the "
                         "grid-sign comparison")
    ap.add_argument("--solve-iters", type=int, default=3000,
                    help="operator applications each solve may take before it is compared at the common residual")
    ap.add_argument("--cull-samples", type=int, default=1_000_000,
                    help="training positions of the learned narrow-band cull (0: skip that measurement)")
    ap.add_argument("--cull-epochs", type=int, default=60)
    ap.add_argument("--calibrate", action="store_true",
                    help="after the timed steps, run one plain 256 MiB device copy (the reference a "
                         "hardware-counter run scales FETCH_SIZE / WRITE_SIZE by)")
    return ap.parse_args()


def measured_rates(rbf):
    """The device's vector-ALU issue rates (rbf_measure_rates): VOP2 FMA, its
    DPP row-broadcast form, v_exp_f32 and their mixes, and the float32 pair
    kernel's own chunk bodies on register operands.  The clock is the one the
    VOP2 FMA rate implies at 32 lanes per SIMD per cycle; body_pairs_per_s is
    the bodies' rate weighted by the operator's share of inner and masked
    examined pairs (filled in by the caller)."""
    r = rbf.measure_rates()
    simds = r.compute_units * 4
    return {
        "fma_vop2_per_s": r.fma_per_s, "fma_dpp_per_s": r.dpp_fma_per_s, "exp_per_s": r.exp_per_s,
        "exp_3fma_chains_per_s": r.exp_3fma_per_s, "exp_7fma_chains_per_s": r.exp_7fma_per_s,
        "inner_body_pair_steps_per_s": r.inner_pair_steps_per_s,
        "masked_body_pair_steps_per_s": r.masked_pair_steps_per_s,
        "clock_ghz_if_32_lanes": r.fma_per_s / (simds * 32) / 1e9,
    }


def cpu_baseline(cloud, eps, sigma, cutoff, row_frac, eval_points, solve_apps):
    """The C cell-list oracle (float64, oracle/cellsum.c) on the host: one
    operator application over every row on all threads, the same on one
    thread over a seeded sample of the rows, and the interpolant at points of
    the support band (a cloud point plus a uniform offset in the cutoff ball,
    seeded) on all threads and on one, and one GMRES(30) cycle of the oracle
    (oracle GMRES, the C operator on all threads).  The solve to the common
    residual is not run on the host (its thousands of applications would take
    about half an hour): its time is extrapolated as the measured cycle time x
    the cycles the plain float64 method needed to reach that residual."""
    import numpy as np

    from oracle import cells
    from oracle import rbf_oracle as o
    from paper_1305_5179_amd import workloads as w

    X, b = o.extended_centres(cloud.points, cloud.normals, eps)
    t0 = time.perf_counter()
    L = cells.CellOracle(X, cutoff)
    build_s = time.perf_counter() - t0
    nthr = cells.max_threads()
    x = w.random_vector(X.shape[0], seed=4)
    res = {}
    # operator, all threads, every row
    t0 = time.perf_counter()
    L.matvec_rows(x, sigma, threads=nthr)
    dt = time.perf_counter() - t0
    res["matvec_all"] = {"threads": nthr, "rows": X.shape[0], "s": dt, "useful": L.useful,
                         "examined": L.examined, "useful_per_s": L.useful / dt}
    # operator, one thread, a sample of the rows
    rows = np.sort(np.random.default_rng(7).choice(X.shape[0], int(row_frac * X.shape[0]), replace=False))
    t0 = time.perf_counter()
    L.matvec_rows(x, sigma, rows=rows, threads=1)
    dt = time.perf_counter() - t0
    res["matvec_1"] = {"threads": 1, "rows": int(rows.size), "s": dt, "useful": L.useful,
                       "examined": L.examined, "useful_per_s": L.useful / dt}
    # interpolant at band points
    pts = w.band_samples(cloud.points, cutoff, eval_points, seed=21)
    coef = w.random_vector(X.shape[0], seed=22)
    for key, thr, npts in (("eval_all", nthr, eval_points), ("eval_1", 1, eval_points // 10)):
        t0 = time.perf_counter()
        L.evaluate(coef, pts[:npts], sigma, threads=thr)
        dt = time.perf_counter() - t0
        res[key] = {"threads": thr, "points": npts, "s": dt, "useful": L.useful, "examined": L.examined,
                    "useful_per_s": L.useful / dt}
    # one restart cycle of the oracle's GMRES(30) on the C operator (all threads)
    t0 = time.perf_counter()
    g = o.gmres(lambda v: L.matvec_rows(v, sigma, threads=nthr), b, restart=30, max_iters=30, tol=1e-8)
    dt = time.perf_counter() - t0
    res["gmres_cycle_all"] = {"threads": nthr, "restart": 30, "iters": int(g.iters), "s": dt,
                              "rel_resid": float(g.rel_resid)}
    L.close()
    out = {"value": res["matvec_all"]["useful_per_s"], "unit": "evals/s", "cores": nthr, "kind": "oracle",
           "sample": (f"C cell-list float64 oracle: one full operator application ({X.shape[0]} rows) on {nthr} "
                      f"threads; {rows.size} sampled rows on 1 thread; the interpolant at {eval_points} band "
                      f"points on {nthr} threads and {eval_points // 10} on 1; one GMRES(30) cycle of the "
                      f"oracle on the operator on {nthr} threads"),
           "host_cpus": os.cpu_count(), "cell_list_s": build_s, **res}
    if solve_apps:
        cycles = solve_apps / 31
        out["solve_extrapolated_s"] = res["gmres_cycle_all"]["s"] * cycles
        out["solve_extrapolated_note"] = (f"{cycles:.0f} GMRES(30) cycles (the plain float64 method's count to the "
                                          f"common residual, {solve_apps} operator applications) x the measured "
                                          f"all-thread cycle time of the oracle")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1305_5179_amd import rbf
    from paper_1305_5179_amd import workloads as w

    if args.workload == "torus":
        cfg = w.TORUS_200K
        cloud = w.torus(cfg["n"], cfg["seed"])
        wl_name = ("torus R=1 r=0.35, 200000 points, 600000 centres, sigma 0.02, cutoff 0.08; "
                   "setup + IR-GMRES(30) cycle (float32 operator) + float64 residual + 256^3 grid")
    else:
        cfg = w.METABALLS_2M
        cloud = w.metaballs(cfg["n"], cfg["seed"])
        wl_name = ("12 Gaussian metaballs with a hole and N(0,1e-3) noise, 2000000 points, 6000000 centres, "
                   "sigma 0.01, cutoff 0.04; setup + IR-GMRES(30) cycle (float32 operator) + float64 residual "
                   "+ 512^3 grid")
    eps, sigma, cutoff, restart = cfg["eps"], cfg["sigma"], cfg["cutoff"], cfg["restart"]
    g = w.Grid.around(cloud.points, cfg["grid_n"])
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pts = torch.as_tensor(cloud.points, device=dev).contiguous()
    nrm = torch.as_tensor(cloud.normals, device=dev).contiguous()
    grid_out = torch.empty(g.size, dtype=torch.float32, device=dev)
    lib = rbf.load_library()

    def step():
        ctx = rbf.Rbf(pts, nrm, eps, sigma, cutoff)
        coef, info = ctx.solve(tol=1e-8, restart=restart, max_iters=restart, max_outer=1,
                               mode=rbf.RBF_SOLVE_IR_FP32)
        ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=rbf.RBF_FP32, out=grid_out)
        st = ctx.stats()
        ctx.close()
        return info, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps follow the warmup directly; the untimed legs below
    # (pair counts, phases, matvecs, the preconditioner) come after them
    rbf.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step()[0] for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = rbf.profile_end()
    # pair counts of one step (fixed by the geometry)
    ctx = rbf.Rbf(pts, nrm, eps, sigma, cutoff)
    st = ctx.stats()
    grid_useful, grid_examined = ctx.count_grid_pairs(g.origin, g.h, g.dims)
    ctx.close()

    # phase breakdown of one (untimed) step
    phases = {}
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx = rbf.Rbf(pts, nrm, eps, sigma, cutoff)
    torch.cuda.synchronize()
    phases["setup_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    coef, _ = ctx.solve(tol=1e-8, restart=restart, max_iters=restart, max_outer=1, mode=rbf.RBF_SOLVE_IR_FP32)
    torch.cuda.synchronize()
    phases["solve_cycle_ms"] = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=rbf.RBF_FP32, out=grid_out)
    torch.cuda.synchronize()
    phases["grid_ms"] = 1e3 * (time.perf_counter() - t)
    x = torch.as_tensor(w.random_vector(3 * cfg["n"], seed=4), device=dev)
    y = torch.empty_like(x)
    for prec, key in ((rbf.RBF_FP32, "matvec_f32_ms"), (rbf.RBF_FP64, "matvec_f64_ms")):
        ctx.matvec(x, y, prec=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            ctx.matvec(x, y, prec=prec)
        torch.cuda.synchronize()
        phases[key] = 1e3 * (time.perf_counter() - t) / 5
    schwarz = schwarz_measurement(rbf, ctx, torch, x, SCHWARZ_192)
    schwarz1024 = schwarz_measurement(rbf, ctx, torch, x, SCHWARZ_1024)
    schwarz_half = schwarz_measurement(rbf, ctx, torch, x, SCHWARZ_192_HALF)
    schwarz1024_half = schwarz_measurement(rbf, ctx, torch, x, SCHWARZ_1024_HALF)
    dens = ctx.density()
    density = {"q": dens.q, "h_max": dens.h_max, "h": dens.h, "h_from": "sqrt(2) h_max (eq. hmax)",
               "sigma_sep": dens.sigma_sep, "sigma_fill": dens.sigma_fill, "sigma": sigma,
               "sigma_over_h": sigma / dens.h}
    ctx.close()


    applications = infos[0].iters + 1   # cycle + true residual of its result
    useful_step = applications * st.useful_pairs + grid_useful
    value = useful_step * args.steps / dt
    ms_step = 1e3 * dt / args.steps

    # dominant kernel: the float32 pair sum, operator launches (the GMRES cycle)
    OP, EV, F32, F64 = 0, 1, 0, 1
    f32_ms = prof.kernel_ms[OP][F32]
    f32_launch = prof.launches[OP][F32]
    achieved = prof.useful_pairs[OP][F32] / (f32_ms * 1e-3)
    traffic, traffic_src = measured_traffic() if args.workload == "torus" else (None, "not measured")
    roofline = {
        "bound": "alu", "kernel": "k_pairsum_f32 (operator launches)",
        "achieved": achieved / 1e9, "peak": PEAK_PAIRS / 1e9, "unit": "Gpair/s",
        "frac": achieved / PEAK_PAIRS, "traffic": traffic, "traffic_unit": "bytes/launch",
        "traffic_source": traffic_src,
        "launches_timed": f32_launch, "avg_launch_ms": f32_ms / max(f32_launch, 1),
        "useful_pairs_per_launch": prof.useful_pairs[OP][F32] / max(f32_launch, 1),
        "examined_per_useful": prof.examined_pairs[OP][F32] / max(prof.useful_pairs[OP][F32], 1),
        "examined_rate": prof.examined_pairs[OP][F32] / (f32_ms * 1e-3) / 1e9,
        "measured_rates": measured_rates(rbf),
    }
    # the chunk bodies' rate for this operator's mix of inner and masked
    # examined pairs, and the kernel's examined-pair rate against it
    mr = roofline["measured_rates"]
    fin = st.inner_entries / max(st.list_entries, 1)
    body = 1.0 / (fin / mr["inner_body_pair_steps_per_s"] + (1 - fin) / mr["masked_body_pair_steps_per_s"])
    mr["inner_share_of_examined"] = fin
    mr["body_pairs_per_s"] = body
    mr["kernel_examined_rate_over_body"] = roofline["examined_rate"] * 1e9 / body
    ev_ms = prof.kernel_ms[EV][F32]
    # (the grid's launches count no pairs themselves: the pair count of the
    # grid, from the list builder, times the launches)
    evaluation = {"launches": prof.launches[EV][F32], "avg_launch_ms": ev_ms / max(prof.launches[EV][F32], 1),
                  "useful_rate": grid_useful * prof.launches[EV][F32] / max(ev_ms * 1e-3, 1e-30) / 1e9}
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl_name,
                   "n_points": cfg["n"], "n_centres": 3 * cfg["n"], "sigma": sigma, "cutoff": cutoff,
                   "restart": restart, "grid": list(g.dims)},
        "roofline": roofline,
        "phases": phases,
        "pairs": {"operator_useful": st.useful_pairs, "operator_examined": st.examined_pairs,
                  "grid_useful": grid_useful, "grid_examined": grid_examined,
                  "applications_per_step": applications},
        "grid_kernel_f32": evaluation,
        "schwarz": schwarz,
        "schwarz1024": schwarz1024,
        "schwarz_half": schwarz_half,
        "schwarz1024_half": schwarz1024_half,
        "density": density,
        "fp64_kernel": {"launches": prof.launches[OP][F64],
                        "avg_launch_ms": prof.kernel_ms[OP][F64] / max(prof.launches[OP][F64], 1),
                        "useful_rate": prof.useful_pairs[OP][F64] / max(prof.kernel_ms[OP][F64] * 1e-3, 1e-30) / 1e9},
    }
    if args.cull_samples > 0:
        out["cull"] = cull_measurement(rbf, torch, pts, nrm, cloud, cfg, g, args.cull_samples, args.cull_epochs)
    if args.calibrate:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = int(src.numel() * 8)
    if not args.no_solve:
        out["solve"], grids = solve_comparison(rbf, torch, pts, nrm, cfg, g, args.solve_iters)
        radii = (cfg["R"], cfg["r"], 2 * cutoff) if args.workload == "torus" else None
        out["signs"] = sign_comparison(torch, grids, g, args.workload, radii)
        del grids
    if not args.no_cpu:
        apps = None
        if "solve" in out:
            p = out["solve"]["plain_fp64"]
            # operator applications of the plain method up to the common residual (30 per cycle + 1 residual)
            k = next(i for i, h in enumerate(p["history"]) if h <= out["solve"]["common_resid"])
            apps = k * (restart + 1)
        out["cpu_baseline"] = cpu_baseline(cloud, eps, sigma, cutoff, args.cpu_row_frac, args.cpu_points, apps)
    print(json.dumps(out), flush=True)


def schwarz_measurement(rbf, ctx, torch, x, opts):
    """The Schwarz preconditioner with the given options: setup time (the
    local inverses' own device time apart), and the time of one apply
    (gather, local products, sums, scatter) from torch events on the stream
    the library runs on.  The apply streams the local inverses (float32 or
    float16) once:
    its algorithmic bytes are those plus the vector traffic (members
    gathered, local results written and summed, result written), against the
    8 TB/s of HBM."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    info = ctx.schwarz_setup(**opts)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t)
    z = torch.empty_like(x)
    ctx.schwarz_apply(x, z)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.schwarz_apply(x, z)
    e1.record()
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / reps
    m = x.numel()
    alg_bytes = info.inverse_bytes + 8 * (3 * info.n_members + 4 * m)
    return {"form": "additive", "options": opts, "overlap_pct": opts.get("overlap_pct", 10),
            "shift": opts.get("shift", 0.3),
            "n_sub": info.n_sub, "n_members": info.n_members, "min_members": info.min_members,
            "max_members": info.max_members, "inverse_bytes": info.inverse_bytes, "retries": info.retries,
            "setup_ms": setup_ms, "factor_ms": info.factor_ms,
            "apply_shape": {"threads": info.apply_threads, "workgroups": info.apply_blocks},
            "apply_ms": apply_ms,
            "apply_roofline": {"bound": "hbm", "achieved": alg_bytes / (apply_ms * 1e-3) / 1e9, "peak": 8000.0,
                               "unit": "GB/s", "frac": alg_bytes / (apply_ms * 1e-3) / 8e12,
                               "bytes_per_apply": alg_bytes}}


def cull_measurement(rbf, torch, pts, nrm, cloud, cfg, g, n_samples, epochs):
    """The learned narrow-band cull on the workload's grid.  Weights from
    three refinement steps (float32 operator); the network is trained (Adam,
    lr 3e-3, batches of 16384) on positions in the support band (a cloud
    point plus a uniform offset in the cutoff ball, seeded), on f / tau with
    tau the RMS of f there; e_val is its largest error on a held-out set of
    band positions.  Reported: the grid time plain and
    culled (torch events, the network's inference included, training not),
    the bricks kept, and the sign errors against the plain grid on nodes
    with |f| > 1e-6 + 8 u32 |f|max."""
    import numpy as np

    from paper_1305_5179_amd import workloads as w
    eps, sigma, rc = cfg["eps"], cfg["sigma"], cfg["cutoff"]
    ctx = rbf.Rbf(pts, nrm, eps, sigma, rc)
    coef, info = ctx.solve(tol=1e-8, restart=cfg["restart"], max_iters=3 * cfg["restart"], max_outer=3)
    lo = np.asarray(g.origin, dtype=np.float64)
    hi = lo + (np.asarray(g.dims) - 1) * np.asarray(g.h)
    X = w.band_samples(cloud.points, rc, n_samples, seed=3)
    Xh = w.band_samples(cloud.points, rc, 100_000, seed=13)
    Xd = torch.as_tensor(X, device="cuda")
    Xhd = torch.as_tensor(Xh, device="cuda")
    f = ctx.eval_points(coef, Xd, prec=rbf.RBF_FP32)
    fh = ctx.eval_points(coef, Xhd, prec=rbf.RBF_FP32)
    tau = float(torch.sqrt(torch.mean(f * f)))
    centre = 0.5 * (lo + hi)
    scale = 2.0 / float((hi - lo).max())
    ctx.net_set(w.net_init(8), centre, scale, tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = ctx.net_train(Xd, f, 16384, epochs, 3e-3)
    torch.cuda.synchronize()
    train_ms = 1e3 * (time.perf_counter() - t0)
    yh = ctx.net_forward(Xhd).double()
    e_val = float(torch.max(torch.abs(yh - fh / tau)))
    total = g.size
    plain = torch.empty(total, dtype=torch.float32, device="cuda")
    culled = torch.empty_like(plain)
    ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=rbf.RBF_FP32, out=plain)
    ctx.eval_grid_culled(coef, g.origin, g.h, g.dims, e_val, out=culled)
    times = {}
    for name, fn in (("plain", lambda: ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=rbf.RBF_FP32, out=plain)),
                     ("culled", lambda: ctx.eval_grid_culled(coef, g.origin, g.h, g.dims, e_val, out=culled))):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            r = fn()
        torch.cuda.synchronize()
        times[name] = 1e3 * (time.perf_counter() - t) / 3
    st = r[1]
    fmax = float(torch.max(torch.abs(plain)))
    tau_s = 1e-6 + 8 * 2.0 ** -24 * fmax
    signed = torch.abs(plain) > tau_s
    wrong = signed & (torch.sign(plain) != torch.sign(culled))
    ctx.close()
    return {"weights_resid": info.rel_resid, "samples": n_samples, "epochs": epochs, "batch": 16384, "lr": 3e-3,
            "train_ms": train_ms, "final_loss": loss, "tau": tau, "e_val": e_val,
            "support_bricks": st.support_bricks, "kept_bricks": st.kept_bricks,
            "kept_fraction": st.kept_bricks / max(st.support_bricks, 1),
            "grid_ms_plain": times["plain"], "grid_ms_culled": times["culled"],
            "signed_nodes": int(signed.sum()), "sign_errors": int(wrong.sum()),
            "sign_error_rate": float(wrong.sum()) / max(int(signed.sum()), 1)}


# the Schwarz configurations: blocks up to 192 centres (every block inverted
# in LDS; about 9,500 subdomains on the torus), and blocks of 64..1024
# centres (small octree leaves merged; about 2,000 subdomains, the larger
# blocks inverted in global memory), each with the library's default shift
# (0.3) and overlap (10 %)
SCHWARZ_192 = dict(max_block=192)
SCHWARZ_1024 = dict(max_block=1024, min_block=64)
# the same with the local inverses stored in float16
SCHWARZ_192_HALF = dict(max_block=192, half=1)
SCHWARZ_1024_HALF = dict(max_block=1024, min_block=64, half=1)

SOLVE_RUNS = (
    # name, mode, basis, Schwarz options (None: no preconditioner)
    ("ir_fp32", "ir", "fp32", None),
    ("ir_fp32_basis64", "ir", "fp64", None),
    ("ir_fp32_schwarz", "ir", "fp32", SCHWARZ_192),
    ("ir_fp32_schwarz1024", "ir", "fp32", SCHWARZ_1024),
    ("ir_fp32_schwarz_half", "ir", "fp32", SCHWARZ_192_HALF),
    ("ir_fp32_schwarz1024_half", "ir", "fp32", SCHWARZ_1024_HALF),
    ("plain_fp64", "plain", "fp64", None),
)


def solve_comparison(rbf, torch, pts, nrm, cfg, g, iters):
    """Setup -> solve -> grid for the chosen pipeline (float32 operator inside
    float64 refinement; its Krylov basis in float32, and in float64 for
    comparison), the same with the additive Schwarz preconditioner, and the
    plain float64 method (float64 operator, basis and grid), each to relative
    residual 1e-8 or `iters` operator applications.  When one stops above
    1e-8 they are compared at the lowest residual all reach (the common
    residual): time to it = setup (+ preconditioner setup) + solve up to the
    first true residual at or below it + grid.  Returns the summary and the
    grids of the final iterates (for the sign comparison)."""
    res, grids = {}, {}
    for name, mode, basis, pre in SOLVE_RUNS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = rbf.Rbf(pts, nrm, cfg["eps"], cfg["sigma"], cfg["cutoff"])
        sinfo = ctx.schwarz_setup(**pre) if pre is not None else None
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        m = rbf.RBF_SOLVE_IR_FP32 if mode == "ir" else rbf.RBF_SOLVE_PLAIN_FP64
        coef, info = ctx.solve(tol=1e-8, restart=cfg["restart"], max_iters=iters, mode=m,
                               precond=rbf.RBF_PRECOND_SCHWARZ if pre is not None else rbf.RBF_PRECOND_NONE,
                               basis=rbf.RBF_FP32 if basis == "fp32" else rbf.RBF_FP64)
        t1 = time.perf_counter()
        prec = rbf.RBF_FP32 if mode == "ir" else rbf.RBF_FP64
        out = torch.empty(g.size, dtype=torch.float32 if prec == rbf.RBF_FP32 else torch.float64, device="cuda")
        ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=prec, out=out)
        torch.cuda.synchronize()
        grid_ms = 1e3 * (time.perf_counter() - t1)
        if name == "plain_fp64":
            # sum_j |c_j phi_j| per node, for the sign threshold
            grids["abs_sum"] = ctx.eval_grid(torch.abs(coef), g.origin, g.h, g.dims, prec=rbf.RBF_FP64)
        grids[name] = out
        res[name] = {"operator": "float32" if mode == "ir" else "float64", "basis": basis,
                     "precond": "none" if pre is None else
                     {"schwarz": pre, "n_sub": sinfo.n_sub, "block_sizes": [sinfo.min_members, sinfo.max_members],
                      "factor_ms": sinfo.factor_ms},
                     "grid": "float32" if prec == rbf.RBF_FP32 else "float64",
                     "setup_ms": setup_ms, "grid_ms": grid_ms, "status": rbf.STATUS_NAMES[info.status],
                     "iters": info.iters, "rel_resid": info.rel_resid, "stall": min(info.history),
                     "solve_ms": info.history_ms[-1] if info.history_ms else 0.0,
                     "history": info.history, "history_ms": info.history_ms}
        ctx.close()
    common = max(max(r["stall"] for r in res.values()), 1e-8)
    for r in res.values():
        t = next(ms for h, ms in zip(r["history"], r["history_ms"]) if h <= common)
        r["ms_to_common"] = r["setup_ms"] + t + r["grid_ms"]
    plain = res["plain_fp64"]["ms_to_common"]
    summary = {"target": 1e-8, "max_applications": iters, "reached_target": {k: r["stall"] <= 1e-8 for k, r in
                                                                             res.items()},
               "common_resid": common,
               "speedup_at_common": {k: plain / r["ms_to_common"] for k, r in res.items() if k != "plain_fp64"},
               **res}
    return summary, grids


def sign_comparison(torch, grids, g, cloud_kind, torus_radii=None):
    """Grid signs of each pipeline's final iterate against the plain float64
    method's grid.  A node has a sign when |f_plain| > tau = 1e-6 +
    8 u32 sum_j |c_j phi_j| (the float32 evaluation bound on top of the
    absolute 1e-6); the others (zero outside the support, or too small) are
    excluded.  For the torus, the signs are also compared with the signed
    distance to the torus on nodes within 2 cutoffs of it."""
    ref = grids["plain_fp64"]
    tau = 1e-6 + 8 * 2.0 ** -24 * grids["abs_sum"]
    signed = torch.abs(ref) > tau
    n_signed = int(signed.sum())
    zero = int((ref == 0).sum())
    out = {"reference": "plain_fp64", "tau": "1e-6 + 8 u32 sum_j |c_j phi_j(node)|", "nodes": g.size,
           "signed": n_signed, "excluded_zero": zero, "excluded_small": g.size - n_signed - zero,
           "disagree": {}, "agreement": {}}
    sref = torch.sign(ref)
    for name, f in grids.items():
        if name in ("plain_fp64", "abs_sum"):
            continue
        bad = int((signed & (torch.sign(f.double()) != sref)).sum())
        out["disagree"][name] = bad
        out["agreement"][name] = 1.0 - bad / max(n_signed, 1)
    if cloud_kind == "torus" and torus_radii is not None:
        R, r, band = torus_radii
        k = torch.arange(g.size, device=ref.device, dtype=torch.int64)
        nx, ny = g.dims[0], g.dims[1]
        ix, iy, iz = k % nx, (k // nx) % ny, k // (nx * ny)
        x = g.origin[0] + ix.double() * g.h[0]
        y = g.origin[1] + iy.double() * g.h[1]
        z = g.origin[2] + iz.double() * g.h[2]
        sdf = torch.sqrt((torch.sqrt(x * x + y * y) - R) ** 2 + z * z) - r
        near = signed & (torch.abs(sdf) <= band)
        n_near = int(near.sum())
        geo = {"band": band, "nodes": n_near}
        for name in ("plain_fp64", "ir_fp32"):
            f = grids[name].double()
            geo[name] = 1.0 - int((near & (torch.sign(f) != torch.sign(sdf))).sum()) / max(n_near, 1)
        out["torus_sdf_agreement"] = geo
    return out


if __name__ == "__main__":
    main()
