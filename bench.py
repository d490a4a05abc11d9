#!/usr/bin/env python3
"""Throughput of the relativistic-beam PIC step on one MI355X.

Default workload (the largest single-GPU configuration): a 3D beam in a
uniform plasma, moving window, grid 512 x 256 x 256, dx = (0.02, 0.05, 0.05)
c/omega_p, dt = dx1/4 (kappa = 4); 2^22 beam electrons in a tri-Gaussian
bunch (sigma_z = 0.1, sigma_r = 0.05, gamma = 1e4, 1% energy spread, 1 mrad
divergence) plus plasma electrons at 8 per cell (2 x 2 x 2 lattice, thermal
u = 1e-4, immobile ions), 2.7e8 particles, injected into the front slab at
every window shift; customized solver (Table 1, M = 16, J1 correction); FP32
fields and particles with cell + offset positions, and the same workload in
FP64.  The vacuum beam alone (the same grid and bunch) is reported beside it.

One step = gather + Boris push + Esirkepov deposit (both species) + J1
correction + field update + window bookkeeping and injection.  The timed
region starts with a particle re-sort (the library re-sorts every 25 steps),
so a window of K <= 25 steps carries at least its share of sorting.  Inputs
are resident on the GPU before the timed region.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
TRAFFIC_FILE_BATCH = os.path.join(ROOT, "profiles", "traffic_counters_batch.json")


def measured_traffic(path, key):
    """HBM bytes per launch of kernel class `key` ("solver/precision/class")
    from a calibrated rocprofv3 counter summary, or None when the summary is
    missing or was taken from other kernel sources."""
    try:
        tf = json.load(open(path))
        from paper_1910_13529_amd.profiling import kernel_source_hash
        if tf.get("source_hash") != kernel_source_hash():
            return None
        ent = tf.get("kernels", {}).get(key)
        return ent["hbm_bytes_per_launch"] if ent else None
    except Exception:
        return None


def algorithmic_bytes(kernel, ncells, npart, esz):
    """Algorithmic HBM bytes of one launch of each kernel class."""
    if kernel == "push_deposit":   # particle state read + written: cell int32 + 3 offsets + 3 momenta
        return npart * 2 * (4 + 6 * esz)
    if kernel == "curl_e":         # E read, B read, B written (B at the next half step)
        return ncells * 9 * esz
    if kernel == "curl_b":         # B read, E read + written
        return ncells * 9 * esz
    if kernel == "leap":           # fused: E and B read once, E and the next B written once
        return ncells * 12 * esz
    return 0


# Vector ALU peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6
# TFLOP/s for FP32 issued one op per lane (the library is built without packed
# FP32, whose 157.3 TFLOP/s it therefore cannot reach) and for FP64.
FP32_VECTOR_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6


def push_flops_per_particle(ndim):
    """Algorithmic floating-point operations of one particle's gather + Boris
    push + move + charge-conserving quadratic deposit (multiply-add = 2),
    counted from the method, not from the kernel's instructions:
      shape weights    3 (2D: 2) axes x 2 staggerings x 3 quadratic weights x 6
      gather           6 components, tensor-product interpolation over 3^d points
                       (3D: 27*2 + 9*2 + 3*2 = 78 per component; 2D: 9*2 + 3*2 = 24)
      Boris            75 (half kicks, gamma, t, s, two cross products, sqrt, divides)
      move             4 per axis
      deposit          1D shapes at x^n and x^{n+1} (2 x axes x 3 x 6), DS and running
                       sums, transverse Esirkepov weights S0a P_b + DSa Q_b over the
                       exact supports, one product and one add per current point
                       (3D: 36 + 30 + 30 points; 2D: 12 + 10 + 15)."""
    if ndim == 3:
        shapes = 3 * 2 * 3 * 6
        gather = 6 * 78
        move = 3 * 4
        deposit = 2 * 3 * 3 * 6 + 3 * 4 + 3 * 3 + 3 * 3 * 2 * 2 + (9 + 15 + 15) * 3 + (36 + 30 + 30) * 2
    else:
        shapes = 2 * 2 * 3 * 6
        gather = 6 * 24
        move = 2 * 4
        deposit = 2 * 2 * 3 * 6 + 2 * 4 + 2 * 3 + 2 * 3 * 2 + (3 + 5 + 15) * 2 + (12 + 10 + 15) * 2
    return shapes + gather + 75 + move + deposit


def make_workload(args):
    from paper_1910_13529_amd import inputs
    n = tuple(int(v) for v in args.grid.split(","))
    w = inputs.config_beam3d(n=n, npart=args.npart)
    cell, off, u = inputs.beam_inputs(w, seed=2)
    Q = inputs.beam_charge(w)
    return w, cell, off, u, Q


# Table 1 of the paper: customized coefficients for kappa = 4, r = 1, M = 16
TABLE1_C = [
    1.248130933469396, -0.125139446419605, 0.040951412341664, -0.018181000724779,
    0.009121734802653, -0.004812019139855, 0.002570175265005, -0.001356670416082,
    0.000694723529383, -0.000339356036052, 0.000155316438379, -0.000065152281459,
    0.000024294488165, -0.000007666519708, 0.000001867004186, -0.000000273002422,
]


def run_gpu(args, w, cell, off, u, Q, solver, precision=None):
    import torch
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=3, n=w.n, dx=w.dx, dt=w.dt, window=True, window_speed=1.0)
    sim = Sim(grid, C=TABLE1_C if solver == "custom" else None, precision=precision or args.precision)
    sid = sim.add_species(-1.0, Q, len(cell))
    sim.load_particles(sid, cell, off, u)
    try:
        fused = sim.set_fused_fields(not args.separate_fields)
    except RuntimeError:
        fused = False
    stream = torch.cuda.current_stream()
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.sort_particles()  # the timed window opens with a re-sort (one per <= 25 steps)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    ev_ms = ev0.elapsed_time(ev1)
    # per-kernel durations from HIP events around each launch, in a separate pass
    sim.profile_enable(True)
    nprof = max(8, min(args.steps, 64))
    sim.step(nprof)
    prof = sim.profile_read()
    sim.profile_enable(False)
    diag = sim.diagnostics()
    sim.close()
    return dict(wall_s=wall, event_ms=ev_ms, prof=prof, diag=diag, nprof=nprof, fused=fused)


def run_batch(args):
    """The batched workload: 256 independent 2D periodic runs (n1 in 128..1024,
    n2 in 64..256, gamma log-uniform 1e1..1e5, dt/dx1 in 0.3..0.99, Yee and
    customized mixed), 4096 particles each, one launch per phase over all
    runs, graph-recorded, tile shapes from the autotuner."""
    import torch
    from paper_1910_13529_amd import workloads
    from paper_1910_13529_amd.relpic import Batch
    runs = workloads.batch_workload(256, solver=args.batch_solver)
    b = Batch([r["grid"] for r in runs], [r["C"] for r in runs], precision=args.precision)
    for br, r in zip(b.runs, runs):
        sid = br.add_species(-1.0, r["Q"], len(r["cell"]))
        br.load_particles(sid, r["cell"], r["offset"], r["u"])
    b.step(1)
    b.sync()
    tune = b.autotune(reps=20)
    stream = torch.cuda.current_stream()
    b.step(args.warmup)
    b.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.sync()
    ev_ms = ev0.elapsed_time(ev1)
    # B update alone, timed again after the run (HIP events on the same stream)
    tune_after = b.autotune(reps=20)
    diag = [b.runs[k].diagnostics() for k in (0, 128, 255)]
    b.close()
    return runs, dict(wall_s=wall, event_ms=ev_ms, tune=tune, tune_after=tune_after, diag=diag)


def batch_cpu_baseline(runs, nsample=8, steps=2):
    """The FP64 oracle on `nsample` of the runs (every 256/nsample-th), `steps` full steps each."""
    import numpy as np
    from oracle.pic import OracleSim
    picks = list(range(0, len(runs), max(1, len(runs) // nsample)))[:nsample]
    tcells = tparts = tsec = 0.0
    for k in picks:
        r = runs[k]
        g = r["grid"]
        o = OracleSim(g["n"][:2], g["dx"][:2], g["dt"], C=[1.0] if r["C"] is None else list(r["C"]), window=False)
        o.add_particles(r["cell"].astype(np.float64) + r["offset"], r["u"], r["Q"], -1.0)
        t0 = time.perf_counter()
        o.step(steps)
        tsec += time.perf_counter() - t0
        tcells += g["n"][0] * g["n"][1] * steps
        tparts += len(r["cell"]) * steps
        o.close()
    return {"value": tcells / tsec, "unit": "cell-updates/s", "particle_steps_per_s": tparts / tsec, "cores": 1,
            "kind": "oracle",
            "sample": "FP64 C oracle, single thread: runs %s of the batched workload, %d full steps each "
                      "(%.1f s in total)" % (picks, steps, tsec)}


def batch_main(args):
    runs, r = run_batch(args)
    ncells = sum(x["grid"]["n"][0] * x["grid"]["n"][1] for x in runs)
    npart = sum(len(x["cell"]) for x in runs)
    esz = 4 if args.precision == "fp32" else 8
    ms = 1e3 * r["wall_s"] / args.steps
    avg_ms = r["tune_after"]["ms_chosen"]
    alg = algorithmic_bytes("curl_e", ncells, npart, esz)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    step_bytes = ncells * 18 * esz + npart * 2 * (4 + 5 * esz)
    out = {
        "metric": "particle-steps/s + field cell-updates/s per PIC step; % HBM peak; FP32 vs FP64",
        "value": ncells * args.steps / r["wall_s"],
        "unit": "cell-updates/s",
        "particle_steps_per_s": npart * args.steps / r["wall_s"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "event_ms_per_step": r["event_ms"] / args.steps,
        "hbm_frac_step": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "batched: 256 independent 2D periodic single-bunch runs (n1 128..1024, n2 64..256, "
                        "gamma log-uniform 1e1..1e5, dt/dx1 0.3..0.99, %s solvers), 4096 particles each, one "
                        "launch per phase over all runs, graph-recorded" % args.batch_solver,
            "cells": ncells,
            "particles": npart,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "batch_curl_e",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(TRAFFIC_FILE_BATCH, "batch/%s/batch_curl_e" % args.precision)
            if args.batch_solver == "mixed" else None,
            "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": alg,
        },
        "autotune": r["tune"],
        "diag": [{k: d[k] for k in ("step", "n_alive", "w_field", "gauss_max", "rho_max", "error_word")}
                 for d in r["diag"]],
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = batch_cpu_baseline(runs)
    print(json.dumps(out), flush=True)


def adjoint_main(args):
    """Gradient of the field loss around a ballistic bunch (2D 1024 x 256,
    2^16 particles, gamma = 1e4, 200 steps, M = 4, checkpoints every 20
    steps): time per gradient (forward + backward) in FP32, and its error
    against the FP64 adjoint."""
    import numpy as np
    import torch
    from paper_1910_13529_amd import workloads
    from paper_1910_13529_amd.relpic import Adjoint
    w = workloads.adjoint_workload()
    adj = {}
    for prec in ("fp32", "fp64"):
        a = Adjoint(w["grid"], w["C0"], w["nsteps"], w["box"], checkpoint_every=20, precision=prec)
        a.load_particles(w["Q"], w["cell"], w["offset"], w["u"])
        adj[prec] = a
    a = adj["fp32"]
    for _ in range(max(1, args.warmup // 10)):
        a.forward(w["C0"])
        a.backward()
    torch.cuda.synchronize()
    reps = max(1, args.steps // 40)
    t0 = time.perf_counter()
    for _ in range(reps):
        L = a.forward(w["C0"])
        g = a.backward()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    L64 = adj["fp64"].forward(w["C0"])
    g64 = adj["fp64"].backward()
    ncells = w["grid"]["n"][0] * w["grid"]["n"][1]
    out = {
        "metric": "time per gradient (forward + adjoint) of the field loss in the axial coefficients",
        "value": ms,
        "unit": "ms",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": w["nsteps"],
        "repetitions": reps,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D 1024x256 periodic, dx=0.05, dt=0.0125, 65536 ballistic particles gamma=1e4, "
                               "M=4 coefficients from the App. C fit, 200 steps, checkpoints every 20", "cells": ncells},
        "cell_steps_per_s": ncells * w["nsteps"] * 3 / (ms * 1e-3),
        "loss_fp32": L,
        "loss_fp64": L64,
        "grad_fp32": [float(v) for v in g],
        "grad_fp64": [float(v) for v in g64],
        "grad_rel_err_fp32_vs_fp64": float(np.abs(g - g64).max() / np.abs(g64).max()),
    }
    for k in adj:
        adj[k].close()
    print(json.dumps(out), flush=True)


# the plasma's launch: tile-sorted, 8 particles per cell, so the wide kernel
# with cell groups and without the wavefront rounds
PUSH_PLASMA_KERNEL = "relpic::k_push_deposit<float, 3, 4, false>"
TRAFFIC_FILE_PLASMA = os.path.join(ROOT, "profiles", "traffic_plasma3d_fp32.json")


def plasma_traffic(kernel):
    """Calibrated HBM bytes per launch of `kernel` in the beam-in-plasma run,
    or None when the counter summary is missing or from other sources."""
    try:
        tf = json.load(open(TRAFFIC_FILE_PLASMA))
        from paper_1910_13529_amd.profiling import kernel_source_hash
        if tf.get("source_hash") != kernel_source_hash():
            return None
        ent = tf.get("kernels", {}).get(kernel)
        return ent["hbm_bytes_per_launch"] if ent else None
    except Exception:
        return None


def run_plasma(args, precision, warmup, steps):
    """One run of the beam-in-plasma workload; returns timings and diagnostics."""
    import torch
    from paper_1910_13529_amd import inputs
    from paper_1910_13529_amd.relpic import Sim
    w, cell, off, u, Q = make_workload(args)
    n1, n2, n3 = w.n
    dV = w.dx[0] * w.dx[1] * w.dx[2]
    Qp = -dV / 8.0  # n0 = 1
    ppc = (2, 2, 2)
    nprof = max(4, min(steps, 12))
    shifts = (warmup + steps + nprof) // 4 + 2
    n_plasma0 = (n1 - 4) * n2 * n3 * 8
    cap = n_plasma0 + shifts * n2 * n3 * 8
    grid = dict(ndim=3, n=w.n, dx=w.dx, dt=w.dt, window=True, window_speed=1.0)
    sim = Sim(grid, C=TABLE1_C, precision=precision)
    try:
        fused = sim.set_fused_fields(not args.separate_fields)
    except RuntimeError:
        fused = False
    sb = sim.add_species(-1.0, Q, len(cell))
    sim.load_particles(sb, cell, off, u)
    sp = sim.add_species(-1.0, Qp, cap)
    print("[bench] plasma %s: %d particles in %d slabs" % (precision, n_plasma0, (n1 - 4 + 31) // 32),
          file=sys.stderr, flush=True)
    for k, lo in enumerate(range(2, n1 - 2, 32)):
        hi = min(lo + 32, n1 - 2)
        c, o, uu = inputs.plasma_lattice(100 + k, (lo, 0, 0), (hi, n2, n3), ppc, 1e-4)
        sim.load_particles(sp, c, o, uu)
        del c, o, uu
    sim.set_injection(sp, ppc, 1e-4, 12345)
    print("[bench] plasma %s: %d warmup + %d timed steps" % (precision, warmup, steps), file=sys.stderr, flush=True)
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sort_particles()  # the timed window opens with a re-sort (one per <= 25 steps)
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # a re-sort alone, for its amortized cost
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.sort_particles()
    torch.cuda.synchronize()
    sort_ms = 1e3 * (time.perf_counter() - t1)
    print("[bench] plasma %s: timing pass (%d steps)" % (precision, nprof), file=sys.stderr, flush=True)
    sim.profile_enable(True)
    sim.step(nprof)
    prof = sim.profile_read()
    push_plasma = sim.profile_read_species(sp)
    push_beam = sim.profile_read_species(sb)
    sim.profile_enable(False)
    diag = sim.diagnostics()
    n_plasma_now = sim.num_slots(sp)
    sim.close()
    return dict(w=w, npart=len(cell) + n_plasma0, nbeam=len(cell), n_plasma_end=n_plasma_now, wall_s=wall,
                sort_ms=sort_ms, prof=prof, nprof=nprof, push_plasma=push_plasma, push_beam=push_beam, diag=diag,
                fused=fused)


def beam_block(args):
    """The vacuum beam alone (same grid and bunch, customized solver, FP32):
    throughput and the fused field update's HBM roofline."""
    w, cell, off, u, Q = make_workload(args)
    ncells = int(math.prod(w.n))
    print("[bench] vacuum beam: %d warmup + %d timed steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    r = run_gpu(args, w, cell, off, u, Q, "custom", precision="fp32")
    prof = r["prof"]
    out = {
        "workload": "3D vacuum beam, moving window, grid 512x256x256, 4194304 macro-electrons, customized solver",
        "ms_per_step": 1e3 * r["wall_s"] / args.steps,
        "cell_updates_per_s": ncells * args.steps / r["wall_s"],
        "particle_steps_per_s": len(cell) * args.steps / r["wall_s"],
        "kernel_ms_per_step": {k: prof[k][1] / r["nprof"] for k in prof if prof[k][0]},
    }
    if prof.get("leap", (0, 0))[0]:
        avg = prof["leap"][1] / prof["leap"][0]
        alg = algorithmic_bytes("leap", ncells, len(cell), 4)
        out["roofline_leap"] = {"bound": "hbm", "kernel": "k_leap (fused E and B update)",
                                "achieved": alg / (avg * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": alg / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "traffic": measured_traffic(TRAFFIC_FILE, "custom/fp32/leap"),
                                "avg_launch_ms": avg, "algorithmic_bytes_per_launch": alg}
    if prof.get("push_deposit", (0, 0))[0]:
        avg = prof["push_deposit"][1] / prof["push_deposit"][0]
        flops = push_flops_per_particle(3) * len(cell)
        out["roofline_push"] = {"bound": "alu", "kernel": "k_push_deposit (beam)",
                                "achieved": flops / (avg * 1e-3) / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": flops / (avg * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                                "avg_launch_ms": avg}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def plasma_cpu_baseline(args, w, cell, off, u, Q):
    """The FP64 oracle on the host cores: a bounded sample of the
    beam-in-plasma workload -- the full 256 x 256 transverse grid over a
    16-cell window slab holding the plasma at 8 per cell and the beam
    particles that fall in it; one field-only and one full step.  The
    per-phase rates are combined at the full workload's cell and particle
    counts."""
    import numpy as np
    from oracle import pic
    from oracle.pic import OracleSim
    from paper_1910_13529_amd import inputs
    n1s = 16
    n = (n1s, w.n[1], w.n[2])
    dV = w.dx[0] * w.dx[1] * w.dx[2]
    centre = int(np.round(np.median(cell[:, 0])))
    shift = centre - n1s // 2
    cs = cell.copy()
    cs[:, 0] -= shift
    keep = (cs[:, 0] >= 2) & (cs[:, 0] <= n1s - 3)
    o = OracleSim(n, w.dx, w.dt, C=TABLE1_C, window=True)
    t0 = time.perf_counter()
    o.field_only(1)
    t_fields = time.perf_counter() - t0
    o2 = OracleSim(n, w.dx, w.dt, C=TABLE1_C, window=True)
    c, of, uu = inputs.plasma_lattice(7, (2, 0, 0), (n1s - 2, n[1], n[2]), (2, 2, 2), 1e-4)
    o2.add_particles(c.astype(np.float64) + of, uu, -dV / 8.0, -1.0)
    o2.add_particles(cs[keep].astype(np.float64) + off[keep], u[keep], Q, -1.0)
    npart_s = len(c) + int(keep.sum())
    del c, of, uu
    t0 = time.perf_counter()
    o2.step(1)
    t_step = time.perf_counter() - t0
    ncell_s = int(np.prod(n))
    rate_c = ncell_s / t_fields
    rate_p = npart_s / max(t_step - t_fields, 1e-9)
    ncells = int(np.prod(w.n))
    npart = len(cell) + (w.n[0] - 4) * w.n[1] * w.n[2] * 8
    t_est = ncells / rate_c + npart / rate_p
    return {
        "value": npart / t_est,
        "unit": "particle-steps/s",
        "cell_updates_per_s": ncells / t_est,
        "cores": pic.threads(),
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "FP64 C oracle (OpenMP over cells and particles' gather+push, deposit serial) on %d threads: "
                  "full 256x256 transverse grid x 16-cell window slab with the plasma at 8 ppc and %d beam "
                  "particles (%d particles), 1 field-only step (%.2f s) + 1 full step (%.2f s); per-phase rates "
                  "(%.3g cell-updates/s, %.3g particle-steps/s) combined at the full workload's %d cells and %d "
                  "particles" % (pic.threads(), int(keep.sum()), npart_s, t_fields, t_step, rate_c, rate_p, ncells,
                                 npart),
    }


def plasma_main(args):
    """The 3D beam in a uniform plasma (the largest single-GPU configuration):
    headline throughput in FP32, the plasma push's ALU roofline, the same
    workload in FP64, the vacuum beam alone, and the oracle on the host."""
    r = run_plasma(args, args.precision, args.warmup, args.steps)
    w, npart, wall, prof, nprof = r["w"], r["npart"], r["wall_s"], r["prof"], r["nprof"]
    ncells = int(math.prod(w.n))
    esz = 4 if args.precision == "fp32" else 8
    ms = 1e3 * wall / args.steps
    # dominant kernel: the plasma species' push+deposit launch (one per step)
    pl_launches, pl_ms = r["push_plasma"]
    avg_ms = pl_ms / max(pl_launches, 1)
    n_pl = npart - r["nbeam"]  # plasma particles at the start of the timing pass (injection adds ~0.2% per shift)
    flops = push_flops_per_particle(3) * n_pl
    alg_bytes = algorithmic_bytes("push_deposit", ncells, n_pl, esz)
    peak_alu = FP64_VECTOR_PEAK_TFLOPS  # non-packed FP32 = FP64 vector rate (packed FP32 is not used)
    traffic = plasma_traffic(PUSH_PLASMA_KERNEL) if args.precision == "fp32" else None
    step_bytes = ncells * (12 if r["fused"] else 18) * esz + npart * 2 * (4 + 6 * esz)
    out = {
        "metric": "particle-steps/s + field cell-updates/s per PIC step; % HBM peak; FP32 vs FP64",
        "value": npart * args.steps / wall,
        "unit": "particle-steps/s",
        "cell_updates_per_s": ncells * args.steps / wall,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "3D beam in uniform plasma, moving window, grid 512x256x256, dx=(0.02,0.05,0.05), "
                               "dt=0.005 (kappa=4); 4194304 beam electrons (sigma_z=0.1, sigma_r=0.05, gamma=1e4, "
                               "1% spread, 1 mrad) + plasma electrons at 8 ppc (2x2x2 lattice, u_th=1e-4, immobile "
                               "ions) injected at each window shift; customized solver (Table 1, M=16, J1 "
                               "correction)",
                   "cells": ncells, "particles": npart, "fused_field_update": r["fused"],
                   "particle_sort_interval": 25,
                   "timed_region": "steps %d..%d after a re-sort at their start (sort included)" %
                                   (args.warmup, args.warmup + args.steps - 1),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": PUSH_PLASMA_KERNEL + " (plasma species)",
                     "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": peak_alu, "unit": "TFLOP/s",
                     "frac": flops / (avg_ms * 1e-3) / 1e12 / peak_alu, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "flops_per_particle": push_flops_per_particle(3),
                     "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": alg_bytes,
                     "hbm_achieved_gbs": alg_bytes / (avg_ms * 1e-3) / 1e9,
                     "hbm_frac": alg_bytes / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "peak_note": "78.6 TFLOP/s = 256 CU x 64 FP32 FMA lanes/clk x 2 x 2.4 GHz (packed FP32, "
                                  "157.3, is not used: the build disables it)"},
        "hbm_frac_step": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "hbm_bytes_step_definition": "%d B/cell (E, B read and written once%s) + %d B/particle (state read and "
                                     "written once)" % ((12 if r["fused"] else 18) * esz,
                                                        ", fused update" if r["fused"] else "", 2 * (4 + 6 * esz)),
        "resort": {"ms_per_sort": r["sort_ms"], "amortized_ms_per_step": r["sort_ms"] / 25.0},
        "push_ms_per_step": {"plasma": avg_ms, "beam": r["push_beam"][1] / max(r["push_beam"][0], 1)},
        "kernel_ms_per_step": {k: prof[k][1] / nprof for k in prof if prof[k][0]},
        "diag": {k: r["diag"][k] for k in ("step", "window_start", "n_alive", "w_field", "w_kin", "error_word")},
    }
    if args.precision == "fp32" and not args.no_fp64 and args.fp64_steps > 0:
        wu = min(args.warmup, 5)
        r64 = run_plasma(args, "fp64", wu, args.fp64_steps)
        p64 = r64["prof"]
        out["fp64"] = {
            "steps": args.fp64_steps, "warmup": wu,
            "ms_per_step": 1e3 * r64["wall_s"] / args.fp64_steps,
            "particle_steps_per_s": npart * args.fp64_steps / r64["wall_s"],
            "cell_updates_per_s": ncells * args.fp64_steps / r64["wall_s"],
            "kernel_ms_per_step": {k: p64[k][1] / r64["nprof"] for k in p64 if p64[k][0]},
            "diag": {k: r64["diag"][k] for k in ("step", "n_alive", "w_field", "w_kin", "error_word")},
        }
        d32, d64 = r["diag"], r64["diag"]
        if d32["step"] == d64["step"]:
            out["fp64"]["fp32_vs_fp64_at_step_%d" % d64["step"]] = {
                "w_field_rel": abs(d32["w_field"] - d64["w_field"]) / abs(d64["w_field"]),
                "w_kin_rel": abs(d32["w_kin"] - d64["w_kin"]) / abs(d64["w_kin"]),
                "charge_rel": abs(d32["charge"] - d64["charge"]) / abs(d64["charge"]),
                "n_alive_fp32": d32["n_alive"], "n_alive_fp64": d64["n_alive"]}
    if not args.no_beam_block:
        out["beam3d"] = beam_block(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        w, cell, off, u, Q = make_workload(args)
        out["cpu_baseline"] = plasma_cpu_baseline(args, w, cell, off, u, Q)
    print(json.dumps(out), flush=True)


def cpu_baseline(args, w, cell, off, u, Q, solver):
    """The FP64 oracle on the host: a bounded sample of the same workload.

    Sample: the full transverse grid with a 64-cell window slab that holds the
    whole bunch (all 2^22 particles), one field-only step and one full step;
    per-phase rates are then combined at the full workload's cell and
    particle counts."""
    import numpy as np
    from oracle.pic import OracleSim
    n1s = 64
    n = (n1s, w.n[1], w.n[2])
    shift = int(np.round(np.median(cell[:, 0]))) - n1s // 2
    cs = cell.copy()
    cs[:, 0] -= shift
    keep = (cs[:, 0] >= 2) & (cs[:, 0] <= n1s - 3)
    C = TABLE1_C if solver == "custom" else (1.0,)
    o = OracleSim(n, w.dx, w.dt, C=C, window=True)
    t0 = time.perf_counter()
    o.field_only(1)
    t_fields = time.perf_counter() - t0
    o2 = OracleSim(n, w.dx, w.dt, C=C, window=True)
    o2.add_particles(cs[keep].astype(np.float64) + off[keep], u[keep], Q, -1.0)
    t0 = time.perf_counter()
    o2.step(1)
    t_step = time.perf_counter() - t0
    ncell_s = int(np.prod(n))
    npart_s = int(keep.sum())
    rate_c = ncell_s / t_fields
    rate_p = npart_s / max(t_step - t_fields, 1e-9)
    ncells = int(np.prod(w.n))
    t_est = ncells / rate_c + len(cell) / rate_p
    return {
        "value": ncells / t_est,
        "unit": "cell-updates/s",
        "particle_steps_per_s": len(cell) / t_est,
        "cores": 1,
        "kind": "oracle",
        "sample": "FP64 C oracle, single thread: full 256x256 transverse grid x 64-cell window slab holding "
                  "all %d particles, 1 field-only step (%.1f s) + 1 full step (%.1f s); per-phase rates "
                  "(%.3g cell-updates/s, %.3g particle-steps/s) combined at the full workload's %d cells and "
                  "%d particles" % (npart_s, t_fields, t_step, rate_c, rate_p, ncells, len(cell)),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--grid", default="512,256,256")
    ap.add_argument("--npart", type=int, default=1 << 22)
    ap.add_argument("--solvers", default="custom,yee")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of the same workload")
    ap.add_argument("--fp64-steps", type=int, default=20, help="timed steps of the plasma workload's FP64 run")
    ap.add_argument("--separate-fields", action="store_true",
                    help="3D beam: separate E and B updates instead of the fused one")
    ap.add_argument("--workload", default="plasma3d", choices=["beam3d", "batch", "adjoint", "plasma3d"],
                    help="plasma3d: the 3D beam in a uniform plasma, 8 ppc, 2.7e8 particles (default); beam3d: "
                         "the vacuum beam alone; batch: the 256-run batched workload; adjoint: time per "
                         "gradient of the differentiable case")
    ap.add_argument("--no-beam-block", action="store_true", help="plasma3d: skip the vacuum-beam block")
    ap.add_argument("--batch-solver", default="mixed", choices=["mixed", "yee", "custom"])
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the PIC step here is a single-GPU build "
              "(multi-GPU sharding along x2/x3 is a design note, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        batch_main(args)
        return
    if args.workload == "adjoint":
        adjoint_main(args)
        return
    if args.workload == "plasma3d":
        plasma_main(args)
        return
    w, cell, off, u, Q = make_workload(args)
    ncells = int(math.prod(w.n))
    npart = len(cell)
    esz = 4 if args.precision == "fp32" else 8
    solvers = args.solvers.split(",")
    results = {}
    for s in solvers:
        print("[bench] %s solver: %d warmup + %d timed steps" % (s, args.warmup, args.steps), file=sys.stderr,
              flush=True)
        results[s] = run_gpu(args, w, cell, off, u, Q, s)
    head = solvers[0]
    r = results[head]
    ms = 1e3 * r["wall_s"] / args.steps
    cell_rate = ncells * args.steps / r["wall_s"]
    part_rate = npart * args.steps / r["wall_s"]
    # E, B read + written once (fused update: 12 words per cell; separate
    # updates: 18, the second one reading E and B again); particle state
    step_bytes = ncells * (12 if r["fused"] else 18) * esz + npart * 2 * (4 + 6 * esz)

    # dominant kernel and its roofline: the push is bound by instruction issue
    # (ALU roofline, algorithmic flops), the field updates by HBM
    prof = r["prof"]
    dom = max((k for k in prof if prof[k][0] > 0), key=lambda k: prof[k][1])
    launches, tot = prof[dom]
    avg_ms = tot / launches
    alg = algorithmic_bytes(dom, ncells, npart, esz)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    flops = push_flops_per_particle(3) * npart
    peak_alu = FP32_VECTOR_PEAK_TFLOPS if args.precision == "fp32" else FP64_VECTOR_PEAK_TFLOPS
    traffic_of = {}
    if os.path.exists(TRAFFIC_FILE) and args.grid == "512,256,256":
        try:
            tf = json.load(open(TRAFFIC_FILE))
            from paper_1910_13529_amd.profiling import kernel_source_hash
            if tf.get("source_hash") == kernel_source_hash():
                for k, ent in tf.get("kernels", {}).items():
                    sol, prec, cls = k.split("/")
                    if sol == head and prec == args.precision:
                        traffic_of[cls] = ent["hbm_bytes_per_launch"]
        except Exception:
            traffic_of = {}
    traffic = traffic_of.get(dom)

    out = {
        "metric": "particle-steps/s + field cell-updates/s per PIC step; % HBM peak; FP32 vs FP64",
        "value": cell_rate,
        "unit": "cell-updates/s",
        "particle_steps_per_s": part_rate,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "event_ms_per_step": r["event_ms"] / args.steps,
        "hbm_frac_step": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D vacuum beam, moving window, grid %s, dx=(0.02,0.05,0.05), dt=0.005 (kappa=4), "
                        "%d macro-electrons sigma_z=0.1 sigma_r=0.05 gamma=1e4 (1%% spread, 1 mrad), "
                        "%s solver" % ("x".join(map(str, w.n)), npart,
                                       "customized (Table 1, M=16, J1 correction)" if head == "custom" else "Yee"),
            "cells": ncells,
            "particles": npart,
            "particle_sort_interval": 25,
            "fused_field_update": r["fused"],
            "parallelism": "single GPU",
        },
        "roofline": ({
            "bound": "alu",
            "kernel": dom,
            "achieved": flops / (avg_ms * 1e-3) / 1e12,
            "peak": peak_alu,
            "unit": "TFLOP/s",
            "frac": flops / (avg_ms * 1e-3) / 1e12 / peak_alu,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "algorithmic_flops_per_launch": flops,
            "flops_per_particle": push_flops_per_particle(3),
            "hbm_achieved_gbs": achieved,
            "algorithmic_bytes_per_launch": alg,
        } if dom == "push_deposit" else {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": alg,
        }),
        "roofline_fields": {
            k: {"bound": "hbm", "achieved": algorithmic_bytes(k, ncells, npart, esz) / (prof[k][1] / prof[k][0] * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": algorithmic_bytes(k, ncells, npart, esz) / (prof[k][1] / prof[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "traffic": traffic_of.get(k),
                "avg_launch_ms": prof[k][1] / prof[k][0],
                "algorithmic_bytes_per_launch": algorithmic_bytes(k, ncells, npart, esz)}
            for k in ("curl_e", "curl_b", "leap") if prof.get(k, (0, 0))[0] > 0},
        # the push against the vector-ALU peak (algorithmic flops), whichever kernel dominates
        "roofline_push": ({
            "bound": "alu", "kernel": "push_deposit",
            "achieved": flops / (prof["push_deposit"][1] / prof["push_deposit"][0] * 1e-3) / 1e12,
            "peak": peak_alu, "unit": "TFLOP/s",
            "frac": flops / (prof["push_deposit"][1] / prof["push_deposit"][0] * 1e-3) / 1e12 / peak_alu,
            "traffic": traffic_of.get("push_deposit"),
            "avg_launch_ms": prof["push_deposit"][1] / prof["push_deposit"][0],
            "algorithmic_flops_per_launch": flops,
            "algorithmic_bytes_per_launch": algorithmic_bytes("push_deposit", ncells, npart, esz),
        } if prof.get("push_deposit", (0, 0))[0] > 0 else None),
        "kernel_ms_per_step": {k: prof[k][1] / r["nprof"] for k in prof if prof[k][0]},
        "diag": {k: r["diag"][k] for k in ("step", "window_start", "n_alive", "w_field", "w_kin", "error_word")},
    }
    for s in solvers[1:]:
        rr = results[s]
        out["other_solvers"] = out.get("other_solvers", {})
        out["other_solvers"][s] = {
            "ms_per_step": 1e3 * rr["wall_s"] / args.steps,
            "cell_updates_per_s": ncells * args.steps / rr["wall_s"],
            "particle_steps_per_s": npart * args.steps / rr["wall_s"],
            "kernel_ms_per_step": {k: rr["prof"][k][1] / rr["nprof"] for k in rr["prof"] if rr["prof"][k][0]},
        }
    if args.precision == "fp32" and not args.no_fp64:
        # the same workload in FP64 (same steps): throughput and how far the
        # FP32 run's FP64 diagnostics are from it at the same step
        print("[bench] %s solver, FP64: %d warmup + %d timed steps" % (head, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        r64 = run_gpu(args, w, cell, off, u, Q, head, precision="fp64")
        p64 = r64["prof"]
        d32, d64 = r["diag"], r64["diag"]
        out["fp64"] = {
            "ms_per_step": 1e3 * r64["wall_s"] / args.steps,
            "cell_updates_per_s": ncells * args.steps / r64["wall_s"],
            "particle_steps_per_s": npart * args.steps / r64["wall_s"],
            "kernel_ms_per_step": {k: p64[k][1] / r64["nprof"] for k in p64 if p64[k][0]},
            "fields_hbm_frac": {
                k: algorithmic_bytes(k, ncells, npart, 8) / (p64[k][1] / p64[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS
                for k in ("curl_e", "curl_b", "leap") if p64.get(k, (0, 0))[0] > 0},
            "fp32_vs_fp64_at_step_%d" % d64["step"]: {
                "w_field_rel": abs(d32["w_field"] - d64["w_field"]) / abs(d64["w_field"]),
                "w_kin_rel": abs(d32["w_kin"] - d64["w_kin"]) / abs(d64["w_kin"]),
                "charge_rel": abs(d32["charge"] - d64["charge"]) / abs(d64["charge"]),
                "gauss_max_fp32": d32["gauss_max"], "gauss_max_fp64": d64["gauss_max"], "rho_max": d64["rho_max"],
            } if d32["step"] == d64["step"] else None,
        }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, w, cell, off, u, Q, head)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
