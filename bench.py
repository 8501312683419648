"""Benchmark of the Eulerian Gaussian beam hot path on one MI355X.

One step = one pass of the whole path over the heterogeneous-VTI workload
(256 x 256 x 256 phase grid, 4 km square, 600 SSP-RK3 steps, beam sum over 32
frequencies 5-60 Hz, first-arrival pick at 128 receivers), inputs resident
in HBM:  medium table + velocity/DRT field, point-source data, the march, the
beam superposition, the pick.

Metric: phase-space cell-updates/s (nx nz nth x RK3 steps / wall time).
The dominant kernel (the RK3 stage) is timed live with HIP events on the
launch stream; its roofline entry counts the scheme's floating-point
operations per cell-stage against the FP32 vector rate.  The oracle (FP64,
C + OpenMP) is timed on the host on one full-size RK3 step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Floating-point operations of the scheme per cell and RK stage, counted from
# its definition (WENO5-JS in Hamilton-Jacobi form on 6 planes x 3 axes,
# convection, sources, stage combine); see the design notes.
FLOP_WENO = 80
FLOP_CELL_STAGE = 18 * FLOP_WENO + 6 * 6 + 3 + 17 + 30
PEAK_FP32_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 excluded
PEAK_HBM_GBPS = 8000.0    # HBM3E spec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid size per axis (256 = the quoted workload)")
    ap.add_argument("--rk-steps", type=int, default=600)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=10,
                    help="RK3 steps for the batched-vs-sequential comparison on the 64-problem uneven workload "
                         "(0 skips it)")
    ap.add_argument("--batched-problems", type=int, default=64)
    ap.add_argument("--adjoint-sources", type=int, default=2,
                    help="sources of the 16-source adjoint workload to time (0 skips it)")
    ap.add_argument("--paraxial-sources", type=int, default=16,
                    help="surface sources picked from the paraxial depth march of the same medium (0 skips it)")
    ap.add_argument("--migration-points", type=int, default=32,
                    help="surface points of the migration leg on the depth march (0: skip it)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape search (profiling runs: keeps every timed launch at the default)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the run, copy a device buffer of this size (a plain copy kernel of known "
                         "size, to scale HBM byte counters)")
    return ap.parse_args()


def batched_vs_sequential(nprob, nsteps, lo=128, hi=384, tune=True):
    """`nprob` independent VTI problems with per-axis sizes uniform in lo..hi:
    one graph-captured batched march of all of them against marching them
    one after another with the single-problem call (same GPU, same steps)."""
    import torch

    import paper_2006_11945_amd as egb
    import workloads as W

    probs = W.batch_uneven(nprob=nprob, nsteps=nsteps, lo=lo, hi=hi)
    solvers = []
    for p in probs:
        s = egb.Solver(p, "cuda:0")
        s.velocity()
        s.init()
        solvers.append(s)
    cells = sum(p.grid.ncell for p in probs)
    arr = egb.make_problem_array(solvers)
    work = egb.alloc_bytes(egb.workspace_size_batched(arr), "cuda:0")
    # launch shape for this batch (results do not depend on it); 0 = the default
    blocks = egb.egb_tune_batched(arr, work, reps=6) if tune else 0
    egb.egb_liouville_step_batched(arr, 1, work)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    egb.egb_liouville_step_batched(arr, nsteps, work)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    del work
    step_work = egb.alloc_bytes(max(egb.workspace_size(s.eg, egb.EGB_OP_STEP) for s in solvers), "cuda:0")
    for s in solvers:
        s.work_step = step_work
    solvers[0].step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(nsteps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    return {"problems": nprob, "sizes": [lo, hi], "cells": cells, "rk3_steps": nsteps, "tuned_blocks": blocks,
            "batched_cell_updates_per_s": cells * nsteps / t_batch,
            "sequential_cell_updates_per_s": cells * nsteps / t_seq,
            "batched_over_sequential": t_seq / t_batch}


def adjoint_vs_forward(nsrc, nsteps, n=256):
    """Traveltime misfit at 128 receivers for `nsrc` of the 16 sources on the
    VTI medium: forward (kinematic march with checkpoints every 16 steps +
    pick) and backward (pick adjoint, recomputation, adjoint steps, medium
    gradient) timed separately, next to the plain full-plane forward march."""
    from dataclasses import replace

    import numpy as np
    import torch

    import paper_2006_11945_amd as egb
    import workloads as W

    probs = W.adjoint_sources(n=n, nsteps=nsteps)
    true = probs[0].extra["true_medium"]
    dev = "cuda:0"
    mk = lambda m, grad=False: [torch.tensor(np.asarray(a, dtype=np.float64), device=dev, requires_grad=grad)
                                for a in (m.vp0, m.eps, m.delta, m.tilt)]
    # one step for every march: within the CFL limits of the model and of the
    # perturbed medium that makes the observed traveltimes
    dt = min(egb.Solver(probs[0], dev).velocity(), egb.Solver(replace(probs[0], medium=true), dev).velocity())
    t_fwd = t_bwd = t_plain = 0.0
    for p in probs[:nsrc]:
        spec = {"grid": p.grid, "source": p.source, "receivers": p.receivers, "nsteps": nsteps, "vs_ratio": 0.5,
                "dtype": "f32", "checkpoint_every": 16, "dt": dt}
        with torch.no_grad():
            t_obs = egb.traveltime(*mk(true), spec)
        ts = mk(p.medium, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = egb.traveltime(*ts, spec)
        ok = ~(torch.isnan(t) | torch.isnan(t_obs))
        J = torch.sum((t[ok] - t_obs[ok]) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_fwd += t1 - t0
        t_bwd += t2 - t1
        s = egb.Solver(p, dev)
        s.velocity()
        s.init()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        s.step(nsteps, dt=dt)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t3
        del s, ts, t, J
        torch.cuda.empty_cache()
    cu = probs[0].grid.ncell * nsteps * nsrc
    return {"sources": nsrc, "rk3_steps": nsteps, "receivers": 128, "checkpoint_every": 16,
            "forward_s": t_fwd, "backward_s": t_bwd, "plain_forward_s": t_plain,
            "backward_cell_updates_per_s": cu / t_bwd, "backward_over_plain_forward": t_bwd / t_plain}


# Paraxial stage: 7 planes x 2 axes of WENO5, convection, sources, the
# stage combine and the coefficient interpolation, per cell and RK stage.
FLOP_PCELL_STAGE = 14 * FLOP_WENO + 7 * 2 * 2 + 17 + 7 * 4 + 7 * 3


def migration_leg(P, p, npoints):
    """Green's-function migration on the march just made: the Green's
    functions of `npoints` surface points at the workload's frequencies (one
    beam sum each), the Born data of a synthetic reflectivity (point
    scatterers and a reflector segment) and its image."""
    import numpy as np
    import torch

    import paper_2006_11945_amd as egb

    g = p.grid
    L = g.nx * g.dx
    xs_list = np.linspace(0.1 * L, 0.9 * L, npoints)
    m = np.zeros((g.nx, g.nz))
    pts = [(g.nx // 2, g.nz // 2), (g.nx // 3, (2 * g.nz) // 3), ((2 * g.nx) // 3, g.nz // 3)]
    for i, k in pts:
        m[i, k] = 1.0
    m[g.nx // 4:(3 * g.nx) // 4, (3 * g.nz) // 4] = 0.5
    md = torch.as_tensor(m, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = P.greens(xs_list, p.omegas)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = egb.egb_born_data(P.eg, G, p.omegas, md)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    img = egb.egb_migrate(P.eg, G, p.omegas, d)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # complex multiply-adds of either contraction: ns^2 per image point and frequency
    flop = 8.0 * npoints ** 2 * g.nx * g.nz * len(p.omegas)
    im = np.abs(img.cpu().numpy())
    bg = float(np.median(im))
    peaks = []
    for i, k in pts:  # the image's peak in a 21 x 21 window around each scatterer: offset, contrast
        i0, k0 = max(i - 10, 0), max(k - 10, 0)
        win = im[i0:i + 11, k0:k + 11]
        a, b = np.unravel_index(np.argmax(win), win.shape)
        peaks.append({"offset_cells": int(max(abs(i0 + a - i), abs(k0 + b - k))),
                      "contrast": float(win.max() / max(bg, 1e-300))})
    kr = (3 * g.nz) // 4
    prof = im[g.nx // 4:(3 * g.nx) // 4].sum(axis=0)
    return {"surface_points": npoints, "frequencies": len(p.omegas), "greens_s": t1 - t0,
            "born_ms": (t2 - t1) * 1e3, "migrate_ms": (t3 - t2) * 1e3,
            "born_fp64_TFLOPs": flop / (t2 - t1) / 1e12, "migrate_fp64_TFLOPs": flop / (t3 - t2) / 1e12,
            "scatterers": peaks, "reflector_depth_error_cells": int(np.argmax(prof) - kr),
            "image_finite": bool(np.isfinite(im).all())}


def paraxial_leg(n, nsrc, nth=256, theta_max=None, migration_points=0):
    """The paraxial depth march (the paper's own formulation) on the same
    medium: 256 x 256 slice of 256 theta nodes in (-60, 60) degrees, all 256
    depth levels, first arrivals of `nsrc` surface sources from the one march,
    and the Green's function of the central surface source (eq. 34, the
    benchmark's 32 frequencies)."""
    from dataclasses import replace

    import numpy as np
    import torch

    import paper_2006_11945_amd as egb
    import workloads as W

    theta_max = np.pi / 3 if theta_max is None else theta_max
    p = W.vti_256(n=n, nsteps=1)
    g = replace(p.grid, nth=nth)
    L = g.nx * g.dx
    P = egb.Paraxial(g, p.medium, theta_max, "cuda:0", "f32")
    P.velocity()
    nsub = P.substeps()
    xs = np.linspace(0.1 * L, 0.9 * L, nsrc)
    P.init(1.0 / (2 * L))
    P.march(nsub)  # warm-up
    P.init(1.0 / (2 * L))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.march(nsub)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = P.pick(xs)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    G = P.beam(0.5 * L, p.omegas)  # Green's function of the central source, all frequencies
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    launches = 3 * nsub * (g.nz - 1)
    cells = g.nx * nth
    stage_ms = (t1 - t0) * 1e3 / launches
    achieved = cells * FLOP_PCELL_STAGE / (stage_ms * 1e-3) / 1e12
    return {"grid": [g.nx, g.nz, nth], "theta_max_deg": float(np.degrees(theta_max)), "substeps_per_level": nsub,
            "stage_launches": launches, "march_s": t1 - t0, "pick_s": t2 - t1, "sources": nsrc,
            "beam_sum_s": t3 - t2, "beam_frequencies": len(p.omegas), "beam_finite": bool(torch.isfinite(G).all()),
            "migration": migration_leg(P, p, migration_points) if migration_points > 0 else None,
            "arrival_fraction": float(torch.isfinite(T).float().mean()),
            "cell_updates_per_s": cells * nsub * (g.nz - 1) / (t1 - t0),
            "roofline": {"bound": "alu", "kernel": "k_pstage (one depth-substep RK3 stage)",
                         "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                         "avg_launch_ms": stage_ms, "flop_per_cell_stage": FLOP_PCELL_STAGE,
                         "note": "march wall time (launch gaps included) divided by the stage launches"}}


# sources the stage kernel is built from (the traffic record names their hash)
STAGE_SOURCES = ("liouville.hip", "stage_common.h", "egb_device.h")


def measured_counters(n):
    """The committed rocprofv3 record of the stage kernel (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE, VALU figures from the SQ counters),
    only while the kernel sources are unchanged since; else None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_stage_vti256_traffic.json")
    if n != 256 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2006_11945_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in STAGE_SOURCES)
    return rec if hashlib.sha256(src).hexdigest() == rec["source_sha256"] else None


def copy_bandwidth(mib=1024, reps=5):
    """Device-to-device copy of `mib` MiB (read + write) timed with HIP
    events: the practical HBM ceiling next to the 8 TB/s spec."""
    import torch

    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbps = 2 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def cpu_baseline(problem):
    """Oracle (as it stands) on one full-size RK3 step of the same workload."""
    import oracle

    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    t0 = time.perf_counter()
    r = oracle.solve(problem, nsteps=0)
    t1 = time.perf_counter()
    oracle.march(problem.grid, r["vel"], problem.source, r["U0"], r["dt"], 1)
    t2 = time.perf_counter()
    g = problem.grid
    return {"value": g.ncell / (t2 - t1), "unit": "cell-updates/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", cores)), "kind": "oracle",
            "sample": f"one SSP-RK3 step of the full {g.nx}x{g.nz}x{g.nth} grid "
                      f"(FP64; setup {t1 - t0:.1f} s not counted, step {t2 - t1:.1f} s)",
            "cpu_model": cpu_model(), "value_1_thread": single_thread_oracle(),
            "sample_1_thread": "one SSP-RK3 step of the same VTI recipe at 128^3, OMP_NUM_THREADS=1"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_thread_oracle():
    """The oracle on one thread (a child process: OpenMP fixes its thread
    count when the library loads), one RK3 step of a 128^3 grid of the same
    recipe; cell-updates/s, None if it did not run."""
    import subprocess
    import sys

    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import oracle, workloads as W\n"
            "p = W.vti_256(n=128)\n"
            "r = oracle.solve(p, nsteps=0)\n"
            "t0 = time.perf_counter()\n"
            "oracle.march(p.grid, r['vel'], p.source, r['U0'], r['dt'], 1)\n"
            "print(p.grid.ncell / (time.perf_counter() - t0))\n") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        return float(out.stdout.strip().splitlines()[-1]) if out.returncode == 0 else None
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a design "
              "note, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2006_11945_amd as egb
    import workloads as W

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = W.vti_256(n=args.n, nsteps=args.rk_steps)
    L = p.grid.nx * p.grid.dx
    rx = np.stack([np.linspace(0.1 * L, 0.9 * L, 128), np.full(128, 0.9 * L)], axis=1)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    s = egb.Solver(p, dev)
    s.velocity()
    dt = s.dt_cfl
    s.init()
    # stage launch shape for this grid (results do not depend on it)
    blocks = egb.egb_get_blocks(s.eg, egb.EGB_TUNE_STEP) if args.no_tune else s.tune(reps=6)
    s.work_beam = egb.alloc_bytes(egb.workspace_size(s.eg, egb.EGB_OP_BEAM), dev)
    out = torch.empty((len(p.omegas), p.grid.nx, p.grid.nz, 2), dtype=torch.float32, device=dev)
    rx_d = torch.as_tensor(rx, device=dev)
    t_pick = torch.empty(128, dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    march_ms = []

    ev2 = torch.cuda.Event(enable_timing=True)
    beam_ms = []

    def one_step(timed):
        s.velocity()
        s.init()
        if timed:
            ev0.record(stream)
        s.step(p.nsteps, dt=dt)
        if timed:
            ev1.record(stream)
        s.beam(p.omegas, out=out)
        if timed:
            ev2.record(stream)
        egb.egb_pick_receivers(s.eg, s.state, rx_d, t_pick)
        if timed:
            ev2.synchronize()
            march_ms.append(ev0.elapsed_time(ev1))
            beam_ms.append(ev1.elapsed_time(ev2))

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cells = p.grid.ncell
    value = cells * p.nsteps / (ms * 1e-3)
    launches = 3 * p.nsteps
    stage_ms = float(np.mean(march_ms)) / launches
    achieved = cells * FLOP_CELL_STAGE / (stage_ms * 1e-3) / 1e12
    rec = measured_counters(args.n)
    copy_gbps = copy_bandwidth()  # after the timed region
    hbm_gbps = None if rec is None else rec["hbm_bytes_per_launch"] / (stage_ms * 1e-3) / 1e9
    res = {
        "metric": "phase-space cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"heterogeneous VTI {p.grid.nx}x{p.grid.nz}x{p.grid.nth}, {p.nsteps} RK3 steps, "
                               f"beam sum {len(p.omegas)} freqs 5-60 Hz, 128 receivers",
                   "grid": [p.grid.nx, p.grid.nz, p.grid.nth], "rk3_steps": p.nsteps,
                   "frequencies": len(p.omegas), "receivers": 128, "psi_dtype": "f64"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None if rec is None else rec["hbm_bytes_per_launch"],
                     "kernel": "k_stage (one SSP-RK3 stage)", "avg_launch_ms": stage_ms, "blocks_per_launch": blocks,
                     "flop_per_cell_stage": FLOP_CELL_STAGE,
                     # HBM side (counters x live launch time) against the spec and a measured device copy
                     "hbm_GBps": hbm_gbps, "hbm_frac_of_8TBps": None if rec is None else hbm_gbps / PEAK_HBM_GBPS,
                     "copy_GBps": copy_gbps, "hbm_frac_of_copy": None if rec is None else hbm_gbps / copy_gbps,
                     "valu_instr_per_cell_stage": None if rec is None else rec.get("valu_instr_per_cell_stage"),
                     "valu_busy": None if rec is None else rec.get("valu_busy")},
        "beam_sum": {"ms": float(np.mean(beam_ms)), "frequencies": len(p.omegas),
                     "output_point_freqs_per_s": p.grid.nx * p.grid.nz * len(p.omegas) / (np.mean(beam_ms) * 1e-3)},
        "march_ms": float(np.mean(march_ms)),
        "march_cell_updates_per_s": cells * p.nsteps / (float(np.mean(march_ms)) * 1e-3),
    }
    del s, out
    torch.cuda.empty_cache()
    if args.batched_steps > 0:
        res["batched"] = batched_vs_sequential(args.batched_problems, args.batched_steps, tune=not args.no_tune)
        # many small problems: one problem alone cannot fill the chip
        res["batched_small"] = batched_vs_sequential(256, 4 * args.batched_steps, lo=32, hi=96,
                                                     tune=not args.no_tune)
        torch.cuda.empty_cache()
    if args.adjoint_sources > 0:
        res["adjoint"] = adjoint_vs_forward(args.adjoint_sources, args.rk_steps, args.n)
        torch.cuda.empty_cache()
    if args.paraxial_sources > 0:
        res["paraxial"] = paraxial_leg(args.n, args.paraxial_sources, migration_points=args.migration_points)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(W.vti_256(n=args.n, nsteps=1))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
