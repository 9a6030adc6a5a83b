"""Benchmark: LOD grid-point-updates/s of the full RE+V solve on one MI355X.

One "step" is one complete solve of the 30000-atom complex (321^3 nodes,
h = 0.35 A, 33 M nodes, ~0.6 GB of FP32 fields: beyond the 256 MB
Infinity Cache, so the sweeps stream from HBM): setup, solvated and vacuum
LODIE2 loops at dt = 0.4 (20 steps) and dt = 0.2 (40 steps), FP64 energy
reductions and the Richardson + vacuum combination.  Inputs are resident in
device memory before the timed region (the solve itself copies the atoms in,
1.2 MB).  Beside the headline: the same solves on the plain FP64 path, and
the 2000-atom globular workload (161^3) as an extra key.

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f32|f32x|f64]
                    [--workload large_complex_321|globular_2000_161] [--no-cpu-baseline]
    python bench.py --batch [--scheme AOSIE2]   64 uneven grids in one batch
    python bench.py --serve                     request loop, p50/p99 latency
    python bench.py --large                     30000 atoms on 321^3: LOD, AOS, FP64, dt 0.2
    python bench.py --direct                    direct vacuum Poisson solve, recovered potential
    python bench.py --sphere                    analytic charged cavity: convergence, stability
    python bench.py --euler                     explicit Euler reference: rate, energy at T = 10
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LOD grid-point-updates/s at ≤1e-3 kcal/mol energy err; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def _sweep_source_sha(source: str = "sweep_kernels.hip"):
    p = os.path.join(ROOT, "paper_1410_2788_amd", "csrc", source)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def _traffic(workload: str, kernel: str, source: str = "sweep_kernels.hip"):
    """HBM bytes per launch of `kernel` (the profiler's name of the template
    instance) on `workload`, from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (profiles/traffic.json), if those counters were taken
    on the current kernel source; else None.  Returns (bytes, label)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None, None
    try:
        d = json.load(open(p))
        e = d.get(workload, {}).get(kernel)
        sha = _sweep_source_sha(source)
        if e and e.get("source_sha") == sha:
            return e.get("bytes_per_launch"), (
                f"profiles/traffic.json: rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of {workload}, "
                f"{e.get('dispatches')} dispatches, calibrated on a plain copy; kernel source "
                f"sha256[:16] {sha}")
    except (OSError, ValueError):
        return None, None
    return None, None


def cpu_baseline(workload, n_steps_meas: int = 2):
    """The FP64 oracle on the host: setup of both media plus a few LODIE2
    steps, extrapolated to the full solve's step count."""
    import threadpoolctl

    import oracle
    w = workload
    p = w.params
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        pb_m = oracle.make_problem(w.molecule, w.grid, p, "solvated")
        pb_v = oracle.make_problem(w.molecule, w.grid, p, "vacuum")
        t_setup = time.perf_counter() - t0
        u = pb_m.u0.copy()
        t1 = time.perf_counter()
        for _ in range(n_steps_meas):
            u = oracle.lod_step(u, pb_m, p.dt, p.alpha, "LODIE2")
        t_step = (time.perf_counter() - t1) / n_steps_meas
    del pb_v
    steps = p.n_steps * (3 if p.richardson else 1) * (2 if p.vacuum else 1)
    pts = w.grid.interior_points
    est = t_setup + steps * t_step
    return {"value": steps * pts / est, "unit": "grid-point-updates/s", "cores": 1,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": (f"{w.name}: setup of both media ({t_setup:.1f} s) + the first "
                       f"{n_steps_meas} solvated LODIE2 steps ({t_step:.2f} s/step), "
                       f"extrapolated to the {steps} steps of one solve; numpy FP64, 1 thread"),
            "seconds_measured": t_setup + n_steps_meas * t_step}


def cpu_baseline_large(workload, n_steps_meas: int = 5):
    """The FP64 oracle on the host, on the full 321^3 grid: the first
    `n_steps_meas` solvated LODIE2 steps, timed and extrapolated to the
    solve's step count.  The oracle's own setup functions build the step's
    data (solute mask, trilinear charges, source density) outside the
    timed steps; its Dirichlet data of 30000 atoms on 6.2e5 shell nodes
    (1.9e10 pair terms, several minutes in NumPy) are left at zero, which
    does not change what a step costs.  The paper also leaves setup out of
    its CPU times."""
    import numpy as np
    import threadpoolctl

    from oracle import npb as O
    w = workload
    p = w.params
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        Q = O.spread_charges(w.grid, w.molecule.xyz, w.molecule.q)
        rho = O.source_density(Q, w.grid.h, p.temperature_K)
        kb2 = O.kappa_bar_sq(p.ionic_molar, p.temperature_K)
        pb = O.problem_from_fields(w.grid, w.molecule, p.eps_in, p.eps_out, kb2, rho,
                                   np.zeros(O.shape_zyx(w.grid)), p.temperature_K)
        t_setup = time.perf_counter() - t0
        u = pb.u0
        t1 = time.perf_counter()
        for _ in range(n_steps_meas):
            u = O.lod_step(u, pb, p.dt, p.alpha, "LODIE2")
        t_step = (time.perf_counter() - t1) / n_steps_meas
    steps = p.n_steps * (3 if p.richardson else 1) * (2 if p.vacuum else 1)
    pts = w.grid.interior_points
    return {"value": pts / t_step, "unit": "grid-point-updates/s", "cores": 1,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": (f"{w.name}: the first {n_steps_meas} solvated LODIE2 steps of the FP64 "
                       f"oracle on the full {w.grid.nx}^3 grid ({t_step:.2f} s/step), "
                       f"extrapolated to the {steps} steps of one RE+V solve "
                       f"({steps * t_step:.0f} s); setup ({t_setup:.1f} s for mask, charges and "
                       f"source; Dirichlet data left at zero) not timed; every step timed as a "
                       f"solvated one (the vacuum steps have no mask and no sinh); "
                       f"numpy FP64, 1 thread"),
            "seconds_measured": n_steps_meas * t_step}


def _energy_tol(ref):
    return max(1e-3, 1e-5 * abs(ref))


def _golden(name):
    p = os.path.join(ROOT, "tests", "golden", name)
    return json.load(open(p)) if os.path.exists(p) else None


def _single_f64(probs, npb):
    """Plain single-solve FP64 GPU path, one problem after another: device
    time per problem (graph replay after a warm-up solve) and the energies."""
    import torch
    out = []
    for w in probs:
        p = dataclasses.replace(w.params, precision="f64")
        s = npb.Solver(w.molecule, w.grid, p, device=0)
        s.run()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        ev0.record(stream)
        r = s.run()
        ev1.record(stream)
        torch.cuda.synchronize()
        out.append((ev0.elapsed_time(ev1), r))
        del s
    return out


def bench_batch(args):
    """64 uneven grids (atom counts log-uniform 200..5000, 79..193 nodes at
    h = 0.5), RE+V, solved together by npb_solve_batch.  Every member's
    energy is checked against the FP64 single-solve GPU path (itself held
    to the FP64 oracle); sampled members also against stored oracle values."""
    import torch

    from paper_1410_2788_amd import inputs, npb
    scheme = args.scheme
    probs = inputs.batch_mix(n_mol=64, seed=3, precision=args.precision, scheme=scheme)
    bs = npb.BatchSolver([(w.molecule, w.grid, w.params) for w in probs])
    print(f"[bench] batch of {len(probs)} grids, {sum(w.grid.nx ** 3 for w in probs) / 1e6:.1f} M nodes, "
          f"{scheme} {args.precision}", file=sys.stderr, flush=True)
    for _ in range(max(1, args.warmup)):
        res = bs.run()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        res = bs.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    del bs
    if args.no_f64:
        # no FP64 reference solves (a profiler pass): every member counted
        single = [(0.0, r) for r in res]
    else:
        print("[bench] FP64 single solves of the same problems", file=sys.stderr, flush=True)
        single = _single_f64(probs, npb)
    single_ms = sum(t for t, _ in single)
    errs = [abs(res[i]["dG"] - single[i][1]["dG"]) for i in range(len(probs))]
    ok = [res[i]["finite"] and errs[i] <= _energy_tol(single[i][1]["dG"]) for i in range(len(probs))]
    pts_all = [r["grid_point_updates"] for r in res]
    pts = sum(pts_all)
    pts_ok = sum(p for p, k in zip(pts_all, ok) if k)
    sampled = {}
    g = _golden("batch_mix_64_samples.json")
    if g:
        for key, ref in g["members"].items():
            sch, i = key.split(":")
            if sch == scheme:
                i = int(i)
                sampled[i] = {"grid": probs[i].grid.nx, "dG": res[i]["dG"], "oracle_dG": ref["dG"],
                              "abs_err": abs(res[i]["dG"] - ref["dG"]), "tolerance": _energy_tol(ref["dG"]),
                              "fp64_gpu_abs_err": abs(single[i][1]["dG"] - ref["dG"])}
    return {"metric": "LOD grid-point-updates/s, batch of uneven grids", "value": pts_ok / (ms * 1e-3),
            "unit": "grid-point-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": args.precision, "data": "synthetic",
            "config": {"workload": "batch_mix_64_seed3", "grids": [w.grid.nx for w in probs],
                       "scheme": scheme, "richardson": True, "vacuum": True,
                       "grid_point_updates_per_batch": pts},
            "accuracy": {"reference": "FP64 single-solve GPU path, same inputs",
                         "within_tolerance": int(sum(ok)), "members": len(probs),
                         "max_abs_err": max(errs), "oracle_samples": sampled},
            "single_f64": ({"ms_total": single_ms,
                            "grid_point_updates_per_s": pts / (single_ms * 1e-3),
                            "speedup_of_batch": single_ms / ms} if not args.no_f64 else None)}


def bench_large(args):
    """The 30000-atom complex on 321^3 nodes (h = 0.35): FP32 LODIE2, FP32
    AOSIE2 and FP64 LODIE2 at dt 0.4 (20 / 40 steps, RE+V), and FP32 LODIE2
    at dt 0.2 (40 / 80 steps); energies against stored oracle values."""
    import torch

    from paper_1410_2788_amd import inputs, npb
    runs = [("f32", "LODIE2", 0.4, 20, "large_complex_321_lodie2_dt04.json"),
            ("f32", "AOSIE2", 0.4, 20, "large_complex_321_aosie2_dt04.json"),
            ("f64", "LODIE2", 0.4, 20, "large_complex_321_lodie2_dt04.json"),
            ("f32", "LODIE2", 0.2, 40, "large_complex_321_lodie2_dt02.json")]
    out_runs = []
    for prec, scheme, dt, n, gname in runs:
        w = inputs.large_complex(precision=prec, scheme=scheme, dt=dt, n_steps=n)
        print(f"[bench] {w.name} {prec} {scheme} dt={dt} n={n}", file=sys.stderr, flush=True)
        s = npb.Solver(w.molecule, w.grid, w.params, device=0)
        if not args.no_autotune:
            s.autotune()
        for _ in range(max(1, args.warmup)):
            s.run()
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        rs = [s.run() for _ in range(args.steps)]
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        ref = _golden(gname)
        rec = {"precision": prec, "scheme": scheme, "dt": [dt, dt / 2], "steps": [n, 2 * n],
               "ms_per_solve": ms, "grid_point_updates_per_solve": rs[0]["grid_point_updates"],
               "dG": rs[0]["dG"], "dG_plain": rs[0]["dG_plain"], "dG_err_est": rs[0]["dG_err_est"]}
        good = len(rs)
        if ref:
            errs = [abs(r["dG"] - ref["dG"]) for r in rs]
            good = sum(e <= _energy_tol(ref["dG"]) for e in errs)
            rec.update(oracle_dG=ref["dG"], abs_err=errs[0], tolerance=_energy_tol(ref["dG"]),
                       within_estimate=bool(errs[0] <= rs[0]["dG_err_est"]))
        # ms is per solve: count the fraction of solves within tolerance
        rec["solves_within_tolerance"] = f"{good}/{len(rs)}" if ref else None
        rec["grid_point_updates_per_s"] = rs[0]["grid_point_updates"] * (good / len(rs)) / (ms * 1e-3)
        out_runs.append(rec)
        del s
    head = out_runs[0]
    return {"metric": "LOD grid-point-updates/s, 321^3 complex", "value": head["grid_point_updates_per_s"],
            "unit": "grid-point-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": head["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "large_complex_321", "grid": [321, 321, 321], "h": 0.35,
                       "atoms": 30000},
            "runs": out_runs}


def bench_sphere(args):
    """The analytic charged-cavity benchmark of Sec. 4.1 (caller-given fields,
    FP64): spatial convergence of every scheme (Delta t = h^2/20, T = 10,
    H = 1, h = 1 .. 0.0625; the paper's Tables LODspat .. MAOSspat), the
    temporal convergence of LODIE2 at h = 0.125 against a Delta t = 2.5e-5
    reference (Table LODtemp), and the stability sweep (Table stab: h = 0.5 and
    0.25, H = 1 and 20, Delta t = 0.001 .. 5, T = 1e4 Delta t) of one scheme
    per family.  Errors are relative L2 and Linf over all nodes but the
    singular centre (Eq. (ErrorMeasure))."""
    import math

    import numpy as np

    from paper_1410_2788_amd import inputs, npb

    def run(b, scheme, dt, n):
        p = npb.make_params_raw(b.eps_in, b.eps_out, b.kbar_sq, 1.0, dt, n, scheme=scheme,
                                face_rule=args.face_rule)
        return npb.FieldsSolver(b.solute, b.grid, p, b.u0, b.rho, graphs=False).run()

    def norms(u, ref, valid):
        e = (u - ref)[valid]
        r = ref[valid]
        return (float(np.sqrt(np.sum(e * e) / np.sum(r * r))),
                float(np.max(np.abs(e)) / np.max(np.abs(r))))

    t0 = time.perf_counter()
    paper = _golden("paper_sphere_spatial.json")
    hs = [1.0, 0.5, 0.25, 0.125, 0.0625]
    schemes = ["LODIE2", "LODCN2", "AOSIE1", "AOSIE2", "AOSCN1", "AOSCN2", "MAOSIE", "MAOSCN"]
    spatial = {}
    ms_total = 0.0
    pts_total = 0.0
    for sc in schemes:
        rows = []
        for h in hs:
            b = inputs.sphere_benchmark(h)
            dt = h * h / 20.0
            n = int(round(10.0 / dt))
            print(f"[bench] sphere spatial {sc} h={h} steps={n}", file=sys.stderr, flush=True)
            r = run(b, sc, dt, n)
            l2, linf = norms(r["u"], b.exact, b.valid)
            ms_total += r["device_ms"]
            pts_total += r["grid_point_updates"]
            rows.append({"h": h, "steps": n, "L2": l2, "Linf": linf, "device_ms": r["device_ms"]})
        for i in range(len(rows) - 1):
            rows[i]["L2_order"] = math.log2(rows[i]["L2"] / rows[i + 1]["L2"])
            rows[i]["Linf_order"] = math.log2(rows[i]["Linf"] / rows[i + 1]["Linf"])
        spatial[sc] = rows
    if args.sphere_spatial_only:
        wall = time.perf_counter() - t0
        return {"metric": "analytic charged-cavity benchmark (Sec. 4.3): spatial errors and "
                          "orders", "value": pts_total / (ms_total * 1e-3),
                "unit": "grid-point-updates/s (spatial study, device time)", "n_gpus": 1,
                "steps": 1, "warmup": 0, "ms_per_step": ms_total, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "analytic",
                "config": {"workload": "charged cavity R=1, eps 1/80, kbar=1, alpha=1, [-3,3]^3",
                           "spatial": "dt = h^2/20, T = 10, H = 1", "face_rule": args.face_rule},
                "spatial": spatial, "paper_LODspat": paper, "wall_s": wall}
    # temporal: LODIE2, h = 0.125, against the dt = 2.5e-5 solution
    b = inputs.sphere_benchmark(0.125)
    print("[bench] sphere temporal reference", file=sys.stderr, flush=True)
    ref = run(b, "LODIE2", 2.5e-5, 400000)["u"]
    temporal = []
    for dt in (8e-4, 4e-4, 2e-4, 1e-4, 5e-5):
        n = int(round(10.0 / dt))
        print(f"[bench] sphere temporal dt={dt} steps={n}", file=sys.stderr, flush=True)
        u = run(b, "LODIE2", dt, n)["u"]
        l2, linf = norms(u, ref, b.valid)
        # against a numerical reference the centre node is finite: also
        # over every node
        l2a, linfa = norms(u, ref, np.ones_like(b.valid))
        temporal.append({"dt": dt, "steps": n, "L2": l2, "Linf": linf, "L2_all_nodes": l2a,
                         "Linf_all_nodes": linfa})
    for i in range(len(temporal) - 1):
        temporal[i]["L2_order"] = math.log2(temporal[i]["L2"] / temporal[i + 1]["L2"])
        temporal[i]["Linf_order"] = math.log2(temporal[i]["Linf"] / temporal[i + 1]["Linf"])
    # stability: one scheme per family, T = 1e4 dt
    dts = [0.001, 0.002, 0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0, 5.0]
    stability = {}
    for fam, sc in (("LOD", "LODIE2"), ("AOS", "AOSIE2"), ("MAOS", "MAOSIE")):
        for H in (1.0, 20.0):
            for h in (0.5, 0.25):
                b = inputs.sphere_benchmark(h, H=H)
                errs = []
                for dt in dts:
                    print(f"[bench] sphere stability {sc} H={H} h={h} dt={dt}", file=sys.stderr,
                          flush=True)
                    errs.append(norms(run(b, sc, dt, 10000)["u"], b.exact, b.valid)[0])
                finite = [dt for dt, e in zip(dts, errs) if math.isfinite(e)]
                stability[f"{fam} H={H:g} h={h:g}"] = {
                    "scheme": sc, "L2": errs,
                    "stable_range": [min(finite), max(finite)] if finite else None}
    wall = time.perf_counter() - t0
    return {"metric": "analytic charged-cavity benchmark (Sec. 4.1-4.4): errors, orders, "
                      "stability range", "value": pts_total / (ms_total * 1e-3),
            "unit": "grid-point-updates/s (spatial study, device time)", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": ms_total, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "analytic",
            "config": {"workload": "charged cavity R=1, eps 1/80, kbar=1, alpha=1, [-3,3]^3",
                       "spatial": "dt = h^2/20, T = 10, H = 1", "temporal": "h = 0.125, T = 10",
                       "stability": "T = 1e4 dt", "face_rule": args.face_rule},
            "spatial": spatial, "temporal_LODIE2": temporal, "stability": stability,
            "paper_LODspat": paper, "wall_s": wall}


FP64_PEAK_TFLOPS = 78.6


def bench_direct(args):
    """The 2000-atom workload with the direct vacuum Poisson solve
    (vacuum_direct): device time of the solve with and without it, the
    transforms' FP64 rate, Eq. (deltaG2) energy and sampled nodes of the
    recovered potential against stored oracle values."""
    import numpy as np
    import torch

    from paper_1410_2788_amd import inputs, npb
    w = inputs.globular_2000(precision=args.precision)
    ref = _golden("globular_2000_161_direct.json")
    X, Y, Z = w.grid.nx - 2, w.grid.ny - 2, w.grid.nz - 2
    # forward and inverse: each line of each axis times an N x N matrix
    flops = 2 * 2 * (Y * Z * X * X + X * Z * Y * Y + X * Y * Z * Z)
    out = {}
    for vd in (False, True):
        s = npb.Solver(w.molecule, w.grid, w.params, device=0, vacuum_direct=vd,
                       want_field=vd, field_select=3 if vd else 0)
        if not args.no_autotune:
            s.autotune()
        for _ in range(max(1, args.warmup)):
            s.run()
        torch.cuda.synchronize()
        rs = [s.run() for _ in range(args.steps)]
        out[vd] = (float(np.median([r["device_ms"] for r in rs])), rs)
        if vd:
            npb.npb_ctx_set_timing(s.ctx, True)
            for _ in range(3):
                s.run()
            torch.cuda.synchronize()
            kt = npb.npb_ctx_get_kernel_times(s.ctx)["direct"]
            npb.npb_ctx_set_timing(s.ctx, False)
            phi = s.field.cpu().numpy().ravel()
        del s
    ms_direct = kt["ms"] / max(kt["count"], 1)
    tf = flops / (ms_direct * 1e-3) / 1e12
    r = out[True][1][0]
    rec = {"metric": "direct vacuum Poisson solve (Sec. 5.1) beside the RE+V solve",
           "value": ms_direct, "unit": "ms per direct solve", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": out[True][0],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 (direct solve); " + args.precision + " (time loops)", "data": "synthetic",
           "config": {"workload": w.name, "grid": [w.grid.nx, w.grid.ny, w.grid.nz],
                      "field_select": "recovered potential"},
           "solve_device_ms": {"without_direct": out[False][0], "with_direct_and_field": out[True][0]},
           "roofline": {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                        "traffic": None, "kernel": "npb::dst_lines_kernel (+ rhs, scale, energy)",
                        "flops_per_direct_solve": flops,
                        "note": "FP64 FMA on the vector units; the launch group's time includes "
                                "the right-hand side, scaling and energy kernels"},
           "energy": {"dG": r["dG"], "dG_direct": r["dG_direct"]}}
    if ref:
        tol = _energy_tol(ref["dG_direct"])
        rec["energy"].update(oracle_dG_direct=ref["dG_direct"],
                             abs_err=abs(r["dG_direct"] - ref["dG_direct"]), tolerance=tol)
        d = np.array([phi[i] for i in ref["field_nodes"]]) - np.array(ref["phi_rec"])
        rec["recovered_field_sampled_rel_err"] = float(np.max(np.abs(d)) / ref["phi_rec_absmax"])
    return rec


def bench_euler(args):
    """The explicit Euler reference solver (FP64) on the 2000-atom workload:
    the step rate over --steps solves of 2000 steps each (vacuum by the
    direct solve), the step kernel's own time from kernel-attached events
    (roofline: 17 algorithmic bytes per interior node and step), parity of
    a 40-step solve against stored oracle values, then reference runs to
    T = euler_t / 2 and euler_t (dt 1e-5) whose Eq. (deltaG2) energy is set
    beside the LODIE2 RE+V and RE energies of the same molecule."""
    import numpy as np
    import torch

    from paper_1410_2788_amd import inputs, npb
    rate_steps = 2000
    w = inputs.globular_2000_euler(n_steps=rate_steps)
    X, Y, Z = w.grid.nx - 2, w.grid.ny - 2, w.grid.nz - 2
    s = npb.Solver(w.molecule, w.grid, w.params, vacuum_direct=True)
    for _ in range(max(1, args.warmup)):
        s.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [s.run() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = float(np.median([r["device_ms"] for r in rs]))
    updates = rs[0]["grid_point_updates"]
    print(f"euler rate: {args.steps} solves of {rate_steps} steps, median {dev_ms:.2f} ms",
          file=sys.stderr, flush=True)
    npb.npb_ctx_set_timing(s.ctx, True)
    s.run()
    torch.cuda.synchronize()
    kt = npb.npb_ctx_get_kernel_times(s.ctx)
    npb.npb_ctx_set_timing(s.ctx, False)
    ke = kt["by_kernel"]["euler"]
    avg_us = 1e3 * ke["ms"] / max(ke["count"], 1)
    bytes_per_launch = ke["bytes"] / max(ke["count"], 1)
    gbps = bytes_per_launch / (avg_us * 1e-6) / 1e9
    del s
    # parity of a short full-size run
    ref = _golden("globular_2000_161_euler40.json")
    g40 = npb.solve(w.molecule, w.grid, inputs.globular_2000_euler(n_steps=40).params,
                    want_field=True, vacuum_direct=True)
    phi = g40["phi"].ravel()
    d = np.array([phi[i] for i in ref["field_nodes"]]) - np.array(ref["phi_m"])
    parity = {"dG_direct": g40["dG_direct"], "oracle_dG_direct": ref["dG_direct"],
              "abs_err": abs(g40["dG_direct"] - ref["dG_direct"]),
              "sampled_field_rel_err": float(np.max(np.abs(d)) / ref["phi_m_absmax"])}
    # reference runs
    refs = []
    for T in (0.5 * args.euler_t, args.euler_t):
        n = max(1, int(round(T / 1e-5)))
        we = inputs.globular_2000_euler(n_steps=n)
        t1 = time.perf_counter()
        r = npb.solve(we.molecule, we.grid, we.params, vacuum_direct=True)
        el = time.perf_counter() - t1
        print(f"euler reference T={T:g} ({n} steps): dG {r['dG_direct']:.4f} kcal/mol, "
              f"{el:.1f} s", file=sys.stderr, flush=True)
        refs.append({"T": T, "steps": n, "dG": r["dG_direct"], "G_m": r["G_m"][0],
                     "device_s": r["device_ms"] * 1e-3, "wall_s": el, "finite": r["finite"]})
    # LODIE2 on the same molecule: the benchmark's own setting (dt 0.2 / 0.1,
    # 20 / 40 steps), then T = euler_t at falling dt (the paper's RE+V runs
    # use T = 10), RE+V (Eq. (deltaG3)) and RE with the direct vacuum
    # potential (Eq. (deltaG2)) beside the Euler energy
    e_ref = refs[-1]["dG"]
    lod = {}
    for prec in ("f64", "f32"):
        wl = inputs.globular_2000(precision=prec)
        r = npb.solve(wl.molecule, wl.grid, wl.params, vacuum_direct=True)
        lod["benchmark_" + prec] = {"dt": wl.params.dt, "steps": wl.params.n_steps,
                                    "RE+V": r["dG"], "RE (phi_0 direct)": r["dG_direct"],
                                    "RE+V minus Euler": r["dG"] - e_ref,
                                    "RE minus Euler": r["dG_direct"] - e_ref,
                                    "device_ms": r["device_ms"]}
    sweep = []
    for dt in (0.4, 0.2, 0.1, 0.05, 0.025):
        wl = inputs.globular_2000(precision="f64")
        wl.params = dataclasses.replace(wl.params, dt=dt,
                                        n_steps=max(1, int(round(args.euler_t / dt))))
        r = npb.solve(wl.molecule, wl.grid, wl.params, vacuum_direct=True)
        sweep.append({"dt": dt, "steps": wl.params.n_steps, "RE+V": r["dG"],
                      "RE (phi_0 direct)": r["dG_direct"], "RE+V minus Euler": r["dG"] - e_ref,
                      "RE minus Euler": r["dG_direct"] - e_ref, "device_ms": r["device_ms"]})
        print(f"LODIE2 T={args.euler_t:g} dt={dt}: RE+V {r['dG']:.3f}, RE {r['dG_direct']:.3f} "
              f"(Euler {e_ref:.3f})", file=sys.stderr, flush=True)
    lod["T_sweep_f64"] = sweep
    rec = {"metric": "explicit Euler grid-point-updates/s (FP64 reference solver)",
            "value": updates / (dev_ms * 1e-3), "unit": "grid-point-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": w.name, "grid": [w.grid.nx, w.grid.ny, w.grid.nz],
                       "dt": 1e-5, "alpha": w.params.alpha, "euler_steps_per_solve": rate_steps,
                       "vacuum": "direct Poisson solve (Eq. (deltaG2))"},
            "device_ms_median": dev_ms,
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4),
                         "traffic": _traffic(w.name, "npb::euler_step_kernel", "euler_kernels.hip")[0],
                         "kernel": "npb::euler_step_kernel", "avg_launch_us": round(avg_us, 2),
                         "algorithmic_bytes_per_launch": bytes_per_launch,
                         "bytes_per_node": 17, "interior_nodes": X * Y * Z,
                         "timing": "kernel-attached HIP events (hipExtLaunchKernelGGL) on every "
                                   "step launch of one solve"},
            "parity_40_steps": parity, "reference": refs, "lodie2": lod}
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    return rec


def bench_serve(args):
    """Serving: requests with atom counts log-uniform 500..20000 (grids
    103..257 at h = 0.5), LODIE2 RE+V 20/40 steps, Poisson arrivals (seed 4)
    at 70 % of the capacity measured with a saturated queue first; the
    request loop batches continuously (requests join the running launches
    every few steps and leave when done).  Latency percentiles are taken
    over the Poisson phase only."""
    import numpy as np

    from paper_1410_2788_amd import inputs, npb
    reqs = inputs.serve_requests(args.requests, seed=4, precision=args.precision)
    budget = int(args.arena_gb * (1 << 30))
    sv = npb.Server(budget, max_batch=args.max_batch, max_queue=4 * len(reqs))

    def drain(tickets):
        lat, done, t_end = {}, set(), None
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = sv.poll(t)
                    if r is not None:
                        done.add(t)
                        lat[t] = (time.perf_counter(), r[0], r[1])
            time.sleep(0.0005)
        return lat

    try:
        # warm-up and capacity: everything submitted at once
        drain([sv.submit(w.molecule, w.grid, w.params) for w in reqs[:4]])
        t0 = time.perf_counter()
        tk = [sv.submit(w.molecule, w.grid, w.params) for w in reqs]
        drain(tk)
        cap = len(reqs) / (time.perf_counter() - t0)
        rate = 0.7 * cap
        arr = inputs.poisson_arrivals(rate, len(reqs), seed=4)
        print(f"[bench] serve: capacity {cap:.2f} req/s, arrivals at {rate:.2f} req/s",
              file=sys.stderr, flush=True)
        # the server's own counters and percentiles cover the Poisson phase only
        sv.reset_stats()
        t0 = time.perf_counter()
        sub = {}
        i = 0
        pending = []
        lat = {}
        while len(lat) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and arr[i] <= now:
                t = sv.submit(reqs[i].molecule, reqs[i].grid, reqs[i].params)
                sub[t] = time.perf_counter()
                pending.append(t)
                i += 1
            for t in list(pending):
                r = sv.poll(t)
                if r is not None:
                    lat[t] = (time.perf_counter() - sub[t], r[0], r[1])
                    pending.remove(t)
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
        after = sv.stats()
    finally:
        sv.close()
    ls = np.array([v[0] for v in lat.values()]) * 1e3
    pts = sum(v[2]["grid_point_updates"] for v in lat.values() if v[1] == npb.NPB_OK)
    return {"metric": "serving: LOD grid-point-updates/s and p50/p99 request latency",
            "value": pts / wall, "unit": "grid-point-updates/s", "n_gpus": 1,
            "steps": len(reqs), "warmup": 4, "ms_per_step": wall * 1e3 / len(reqs),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": args.precision, "data": "synthetic",
            "config": {"workload": f"serve_requests_{len(reqs)}_seed4", "arrival_rate_per_s": rate,
                       "capacity_per_s": cap, "arena_bytes": budget, "max_batch": args.max_batch,
                       "grids": [w.grid.nx for w in reqs]},
            "latency_ms": {"p50": float(np.percentile(ls, 50)), "p99": float(np.percentile(ls, 99)),
                           "max": float(ls.max())},
            "server": after}


_TNAME = {"f32": "float, float", "f32x": "float, double", "f64": "double, double"}


def _kernel_instance(kname, shapes, precision, scheme):
    """The profiler's name of the sweep kernel instance a timing-pass key
    ("x", "yz_plain", "yz_flow", "yz_general") ran as, from the launch
    shapes [rows per chunk, chunks, lines per block or tile width, threads]."""
    tname = _TNAME[precision]
    if kname == "x":
        cn = "true" if "CN" in scheme else "false"
        return f"npb::sweep_x_kernel<{tname}, {shapes[0][0]}, {shapes[0][2]}, {cn}>"
    var = {"yz_plain": 0, "yz_flow": 1, "yz_general": 2}[kname]
    d = 1 if var != 1 else 2
    return f"npb::sweep_yz_kernel<{tname}, {shapes[d][0]}, {var}, {shapes[d][2]}>"


def _measure(w, args, ref, steps, timing, tune, label):
    """Solves of workload w as a caller runs them (graph replay, inputs
    resident): `steps` timed solves between two stream events after the
    warm-up, then optionally a timing pass with kernel-attached events.
    Energies against ref["dG"] under the contract max(1e-3, 1e-5 |dG|)."""
    import numpy as np
    import torch

    from paper_1410_2788_amd import npb
    solver = npb.Solver(w.molecule, w.grid, w.params, device=0)
    print(f"[bench] {label}: {w.name} {w.params.precision} {w.params.scheme} "
          f"warmup={args.warmup} steps={steps}", file=sys.stderr, flush=True)
    tune_ms = solver.autotune() if tune else None
    shapes = npb.npb_launch_shapes(solver.ctx, solver.grid, solver.params)
    for _ in range(max(1, args.warmup)):
        solver.run()
    stream = torch.cuda.current_stream()
    lat, results = [], []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        t = time.perf_counter()
        results.append(solver.run())
        lat.append((time.perf_counter() - t) * 1e3)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ktimes = None
    if timing:
        # the same solves once more with every sweep launch carrying events
        # that record its kernel's own start and stop (direct launches, the
        # two media's launches one after another on the solve's stream)
        print(f"[bench] {label}: per-kernel timing pass", file=sys.stderr, flush=True)
        npb.npb_ctx_set_timing(solver.ctx, True)
        for _ in range(min(steps, 5)):
            solver.run()
        torch.cuda.synchronize()
        ktimes = npb.npb_ctx_get_kernel_times(solver.ctx)
        npb.npb_ctx_set_timing(solver.ctx, False)
    del solver
    tol = _energy_tol(ref["dG"])
    errs = [abs(r["dG"] - ref["dG"]) for r in results]
    good = sum(e <= tol for e in errs)
    per_solve = results[0]["grid_point_updates"]
    return {"results": results, "total_ms": total_ms, "ms_per_solve": total_ms / steps,
            "lat": lat, "ktimes": ktimes, "shapes": shapes, "tuned": tune_ms is not None,
            "tol": tol, "errs": errs, "good": good, "per_solve": per_solve,
            "value": per_solve * good / (total_ms * 1e-3),
            "value_all": per_solve * len(results) / (total_ms * 1e-3)}


def _roofline(m, w, precision, scheme, steps):
    """Roofline of the dominant sweep kernel (largest summed duration in the
    timing pass): its algorithmic bytes per launch over its mean
    kernel-attached-event duration; and the whole solve's sweep bytes over
    its device time."""
    import numpy as np
    ktimes = m["ktimes"]
    bk = ktimes["by_kernel"]
    kname = max(bk, key=lambda k: bk[k]["ms"])
    kt = bk[kname]
    avg_ms = kt["ms"] / max(kt["count"], 1)
    bpl = kt["bytes"] / max(kt["count"], 1)
    ach = bpl / (avg_ms * 1e-3) / 1e9
    full = _kernel_instance(kname, m["shapes"], precision, scheme)
    traffic, tlabel = _traffic(w.name, full)
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": tlabel,
            "kernel": full, "avg_launch_us": round(avg_ms * 1e3, 2),
            "algorithmic_bytes_per_launch": bpl,
            "timing": "timing pass: every sweep launch carries HIP events that record the "
                      "kernel's own start and stop (hipExtLaunchKernelGGL); the two media's "
                      "launches issued one after another on one stream",
            "per_kernel": {_kernel_instance(k, m["shapes"], precision, scheme): {
                "launches": bk[k]["count"],
                "avg_us": round(bk[k]["ms"] / max(bk[k]["count"], 1) * 1e3, 2),
                "GBps": round(bk[k]["bytes"] / max(bk[k]["ms"], 1e-12) / 1e6, 1),
                "frac": round(bk[k]["bytes"] / max(bk[k]["ms"], 1e-12) / 1e6 / HBM_PEAK_GBS, 4)}
                for k in bk if bk[k]["count"] and k != "euler"},
            "per_class": {c: {"launches": ktimes[c]["count"],
                              "avg_us": round(ktimes[c]["ms"] / max(ktimes[c]["count"], 1) * 1e3, 2),
                              "GBps": round(ktimes[c]["bytes"] / max(ktimes[c]["ms"], 1e-12) / 1e6, 1)}
                          for c in ("sweep_x", "sweep_y", "sweep_z", "init", "setup", "energy")}}
    # whole solve, as timed (the two media's sweeps on concurrent streams):
    # algorithmic bytes of every sweep of one solve over its device time
    sweep_bytes = sum(ktimes[c]["bytes"] for c in ("sweep_x", "sweep_y", "sweep_z"))
    nsolves = max(min(steps, 5), 1)
    dev_ms = float(np.median([r["device_ms"] for r in m["results"]]))
    pg = sweep_bytes / nsolves / (dev_ms * 1e-3) / 1e9
    roof["solve_pipeline"] = {"algorithmic_sweep_bytes_per_solve": sweep_bytes / nsolves,
                              "solve_device_ms": dev_ms, "achieved": round(pg, 1),
                              "frac": round(pg / HBM_PEAK_GBS, 4)}
    return roof


def bench_solve(args):
    """The headline line: one RE+V solve per step on the chosen workload
    (default: the 30000-atom complex on 321^3, FP32 LODIE2, dt 0.4 / 0.2 with
    20 / 40 steps), energies held to the stored FP64-oracle values; the plain
    FP64 path on the same workload beside it; the 161^3 globular workload
    as an extra key; the oracle's rate on the host."""
    import numpy as np
    import torch

    from paper_1410_2788_amd import inputs, npb
    large = args.workload == "large_complex_321"
    mk = ((lambda prec: inputs.large_complex(precision=prec, scheme=args.scheme)) if large
          else (lambda prec: inputs.globular_2000(precision=prec, scheme=args.scheme)))
    w = mk(args.precision)
    gname = {("large_complex_321", "LODIE2"): "large_complex_321_lodie2_dt04.json",
             ("large_complex_321", "AOSIE2"): "large_complex_321_aosie2_dt04.json",
             ("globular_2000_161", "LODIE2"): "globular_2000_161.json"}.get((w.name, args.scheme))
    ref = _golden(gname) if gname else None
    ref_kind = "FP64 oracle (stored, tests/golden/" + gname + ")" if ref else None
    if ref is None:
        # other schemes: the FP64 GPU path of the same scheme (held to the
        # oracle by the parity tests) as the reference
        ref = npb.solve(w.molecule, w.grid, dataclasses.replace(w.params, precision="f64"))
        ref_kind = "FP64 GPU path, same scheme"
    m = _measure(w, args, ref, args.steps, not args.no_timing, not args.no_autotune, "headline")
    roof = _roofline(m, w, args.precision, args.scheme, args.steps) if m["ktimes"] else None
    results = m["results"]
    out = {
        "metric": METRIC, "value": m["value"], "unit": "grid-point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f32x": "f32-storage/f64-solve", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.grid.nx, w.grid.ny, w.grid.nz], "h": w.grid.h,
                   "atoms": w.molecule.n_atoms, "scheme": args.scheme, "richardson": True,
                   "vacuum": True, "dt": [w.params.dt, w.params.dt / 2],
                   "steps_per_solve": results[0]["steps_done"],
                   "launch_shapes": {"x": m["shapes"][0], "y": m["shapes"][1],
                                     "z": m["shapes"][2], "autotuned": m["tuned"]},
                   "grid_point_updates_per_solve": m["per_solve"]},
        "latency_ms": {"p50": float(np.percentile(m["lat"], 50)),
                       "p99": float(np.percentile(m["lat"], 99)),
                       "device_ms_median": float(np.median([r["device_ms"] for r in results]))},
        "energy": {"dG": results[0]["dG"], "reference": ref_kind, "oracle_dG": ref["dG"],
                   "abs_err": m["errs"][0], "max_abs_err": max(m["errs"]),
                   "tolerance": m["tol"], "solves_within_tolerance": m["good"],
                   "dG_err_est": results[0].get("dG_err_est"),
                   "within_estimate": m["errs"][0] <= results[0].get("dG_err_est", float("inf"))},
        "roofline": roof,
    }
    if args.precision != "f64" and not args.no_f64:
        # the plain single-solve FP64 GPU path on the same workload
        w64 = mk("f64")
        n64 = max(1, min(args.steps, 5))
        m64 = _measure(w64, args, ref, n64, False, False, "fp64")
        out["fp64_same_workload"] = {
            "value": m64["value"], "ms_per_solve": m64["ms_per_solve"], "solves": n64,
            "abs_err": m64["errs"][0], "solves_within_tolerance": m64["good"],
            "speedup_of_headline": m["value"] / m64["value"] if m64["value"] else None}
    if large and not args.no_extra:
        wg = inputs.globular_2000(precision=args.precision, scheme=args.scheme)
        rg = _golden("globular_2000_161.json") if args.scheme == "LODIE2" else None
        if rg is not None:
            mg = _measure(wg, args, rg, args.steps, False, not args.no_autotune, "extra")
            out["globular_2000_161"] = {
                "value": mg["value"], "ms_per_solve": mg["ms_per_solve"],
                "grid": [wg.grid.nx, wg.grid.ny, wg.grid.nz],
                "abs_err": mg["errs"][0], "solves_within_tolerance": mg["good"],
                "note": "4 FP32 fields of 24 MB: the working set fits the 256 MB Infinity "
                        "Cache, so this rate is not an HBM figure"}
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = (cpu_baseline_large(inputs.large_complex(precision="f64"))
                               if large else cpu_baseline(inputs.globular_2000(precision="f64")))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f32", choices=["f32", "f32x", "f64"])
    ap.add_argument("--scheme", default="LODIE2",
                    choices=["LODIE2", "LODIE1", "AOSIE2", "AOSIE1", "LODCN1", "LODCN2",
                             "AOSCN1", "AOSCN2", "MAOSIE", "MAOSCN"])
    ap.add_argument("--workload", default="large_complex_321",
                    choices=["large_complex_321", "globular_2000_161"],
                    help="headline workload: the 30000-atom complex on 321^3 (default) or the "
                         "2000-atom globular molecule on 161^3")
    ap.add_argument("--no-f64", action="store_true",
                    help="skip the FP64 solves of the same workload beside the headline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 161^3 globular workload beside the 321^3 headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="skip the per-kernel event timing pass")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of tuning them first")
    ap.add_argument("--batch", action="store_true",
                    help="time a batch of 64 uneven grids instead (own JSON line)")
    ap.add_argument("--large", action="store_true",
                    help="time the 30000-atom 321^3 complex in FP32 LOD, FP32 AOS and FP64 LOD (own JSON line)")
    ap.add_argument("--direct", action="store_true",
                    help="time the direct vacuum Poisson solve and the recovered potential "
                         "(own JSON line)")
    ap.add_argument("--sphere", action="store_true",
                    help="the analytic charged-cavity benchmark: spatial / temporal "
                         "convergence and stability of the schemes (own JSON line)")
    ap.add_argument("--face-rule", default="harmonic", choices=["harmonic", "location"],
                    help="eps at the half points for --sphere")
    ap.add_argument("--sphere-spatial-only", action="store_true",
                    help="--sphere: the spatial-convergence study only")
    ap.add_argument("--euler", action="store_true",
                    help="the explicit Euler reference solver: step rate, roofline, and the "
                         "reference energy at T = --euler-t (own JSON line)")
    ap.add_argument("--euler-t", type=float, default=10.0)
    ap.add_argument("--serve", action="store_true",
                    help="time the request loop under Poisson arrivals instead (own JSON line)")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--arena-gb", type=float, default=24.0)
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with plain device copies of 256 MiB (FP32) that calibrate "
                         "the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    if args.batch:
        out = bench_batch(args)
        if args.copy_calibration:
            import torch
            src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        print(json.dumps(out))
        return
    if args.serve:
        print(json.dumps(bench_serve(args)))
        return
    if args.direct:
        print(json.dumps(bench_direct(args)))
        return
    if args.sphere:
        print(json.dumps(bench_sphere(args)))
        return
    if args.euler:
        print(json.dumps(bench_euler(args)))
        return
    if args.large:
        print(json.dumps(bench_large(args)))
        return

    print(json.dumps(bench_solve(args)))


if __name__ == "__main__":
    main()
