"""Benchmark of the Eulerian Gaussian beam hot path on one MI355X.

One step = one pass of the whole path over the 2D TTI workload (512 x 512 x
512 phase grid on a 4 km square, the VTI blob medium plus a smooth random
tilt in [-45, 45] degrees, 1200 SSP-RK3 steps, beam sum over 64 frequencies
5-60 Hz, first-arrival pick at 128 receivers), inputs resident in HBM:
medium table + velocity/DRT field, point-source data, the march, the beam
superposition, the pick.  FP32 planes, traveltime psi in FP64.

Metric: phase-space cell-updates/s (nx nz nth x RK3 steps / wall time).
The dominant kernel (the RK3 stage) is timed live with HIP events on the
launch stream; its roofline entry counts the scheme's floating-point
operations per cell-stage against the published FP32 vector peak, next to
the issue rate without packed FP32 and the HBM floor of the state traffic.
The oracle (FP64, C + OpenMP) is timed on the host on a window of the same
grid.  Secondary legs: the 256^3 VTI workload, batched and adjoint marches
against the plain solve, the paraxial depth march.
"""
import argparse
import json
import os
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Floating-point operations of the scheme per cell and RK stage, counted from
# its definition: WENO5-JS in Hamilton-Jacobi form on 6 planes (phi1, C, B,
# psi) x 3 axes, the linear fifth-order upwind derivative of the phase plane
# on 3 axes, convection (7 planes x 3 axes, a multiply-add each), sources
# (psi 3, A (C, B) 17, A12 Im(B / C) 9), stage combine (7 planes x 5).
FLOP_WENO = 80
FLOP_UPWIND5 = 15
FLOP_CELL_STAGE = 18 * FLOP_WENO + 3 * FLOP_UPWIND5 + 7 * 6 + 3 + 17 + 9 + 7 * 5
PEAK_FP32_TFLOPS = 157.3           # published MI355X FP32 vector peak (counts packed, dual-lane FP32)
PEAK_FP32_UNPACKED_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz: one FP32 op per lane
PEAK_HBM_GBPS = 8000.0             # HBM3E spec
XCDS = 8                           # accelerator dies (each with its own L2 and cycle counter)
# State bytes per cell (six FP32 planes and psi in FP64); one RK3 step must
# at least read and write the state once: the HBM floor per cell-update.
STATE_BYTES_PER_CELL = 6 * 4 + 8
FLOOR_BYTES_PER_CELL_UPDATE = 2 * STATE_BYTES_PER_CELL

WORKLOADS = {
    "tti512": "2D TTI 512x512x512 (VTI blob medium + smooth tilt in [-45, 45] deg, 4 km square), "
              "1200 RK3 steps, beam sum 64 freqs 5-60 Hz, 128 receivers",
    "vti256": "heterogeneous VTI 256x256x256 (4 km square), 600 RK3 steps, beam sum 32 freqs 5-60 Hz, "
              "128 receivers",
}


def make_workload(name, n=None, rk_steps=None):
    import workloads as W

    if name == "tti512":
        return W.tti_512(n=512 if n is None else n, nsteps=1200 if rk_steps is None else rk_steps)
    return W.vti_256(n=256 if n is None else n, nsteps=600 if rk_steps is None else rk_steps)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="tti512",
                    help="the timed pass: tti512 (the quoted 512^3 TTI workload) or vti256")
    ap.add_argument("--n", type=int, default=None, help="grid size per axis (default: the workload's own)")
    ap.add_argument("--rk-steps", type=int, default=None, help="RK3 steps per pass (default: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--vti-leg", type=int, default=1,
                    help="timed passes of the 256^3 VTI workload as a secondary leg (0 skips it)")
    ap.add_argument("--batched-steps", type=int, default=10,
                    help="RK3 steps for the batched-vs-sequential comparison on the 64-problem uneven workload "
                         "(0 skips it)")
    ap.add_argument("--batched-problems", type=int, default=64)
    ap.add_argument("--adjoint-sources", type=int, default=1,
                    help="sources of the 16-source adjoint workload to time (0 skips it)")
    ap.add_argument("--paraxial-sources", type=int, default=16,
                    help="surface sources picked from the paraxial depth march of the same medium (0 skips it)")
    ap.add_argument("--migration-points", type=int, default=32,
                    help="surface points of the migration leg on the depth march (0: skip it)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape search (profiling runs: keeps every timed launch at the default)")
    ap.add_argument("--time-budget-s", type=float, default=540.0,
                    help="secondary legs that would end later than this many seconds after the start are "
                         "skipped (and named so in the output); 0: no limit")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the run, copy a device buffer of this size (a plain copy kernel of known "
                         "size, to scale HBM byte counters)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "SQ_DIR"), default=None,
                    help="no GPU run: read three rocprofv3 --pmc output folders of a profiling run of this "
                         "bench (FETCH_SIZE; WRITE_SIZE; SQ counters) and print the stage kernel's counter "
                         "record as JSON")
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
    # launch (tile shape and block count) for this batch; results do not depend on it
    blocks = egb.egb_tune_batched(arr, work, reps=3) if tune else 0
    tile_rows, _ = egb.egb_get_launch_batched(arr)
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
            "tuned_tile_rows": tile_rows,
            "batched_cell_updates_per_s": cells * nsteps / t_batch,
            "sequential_cell_updates_per_s": cells * nsteps / t_seq,
            "batched_over_sequential": t_seq / t_batch}


def adjoint_vs_forward(nsrc, nsteps, n=256, tune=True):
    """Traveltime misfit at 128 receivers for `nsrc` of the 16 sources on the
    VTI medium: forward (kinematic march keeping the states the backward
    sweep needs + pick) and backward (pick adjoint, recomputation, adjoint steps, medium
    gradient) timed separately on each source's second call, next to the plain
    full-plane forward march; the first call's forward, which allocates the
    state archive, is reported apart."""
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
    # every step's phi1 and psi resident in HBM (FP32 phi1 + FP64 psi per cell
    # and step) when that takes at most half of the free memory, else a
    # checkpoint every 16 steps and the segments recomputed
    g0 = probs[0].grid
    tuned = None
    if tune:  # launch shapes of the grid's full-plane and kinematic stages (the library keeps them per grid shape)
        s = egb.Solver(probs[0], dev)
        s.velocity()
        s.init()
        tuned = {}
        for name, op in (("full_plane", egb.EGB_TUNE_STEP), ("kinematic", egb.EGB_TUNE_KINEMATIC)):
            s.tune(op=op, reps=2)
            tuned[name] = egb.egb_get_launch(s.eg, op)
        del s
    need = nsteps * g0.nx * g0.nz * g0.nth * (4 + 8)
    K = 0 if need <= 0.5 * torch.cuda.mem_get_info(dev)[0] else 16
    t_fwd = t_bwd = t_plain = t_first = 0.0
    for p in probs[:nsrc]:
        spec = {"grid": p.grid, "source": p.source, "receivers": p.receivers, "nsteps": nsteps, "vs_ratio": 0.5,
                "dtype": "f32", "checkpoint_every": K, "dt": dt}
        with torch.no_grad():
            t_obs = egb.traveltime(*mk(true), spec)
        ts = mk(p.medium, True)
        # two calls: the first allocates the state archive (and pays for the
        # device's first touch of memory that earlier legs released); torch's
        # caching allocator keeps it for the second, which is the one timed,
        # as in an inversion loop over sources and iterations
        for rep in range(2):
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
            if rep == 0:
                t_first += t1 - t0
            else:
                t_fwd += t1 - t0
                t_bwd += t2 - t1
            del t, J
        s = egb.Solver(p, dev)
        s.velocity()
        s.init()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        s.step(nsteps, dt=dt)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t3
        del s, ts
        torch.cuda.empty_cache()
    cu = probs[0].grid.ncell * nsteps * nsrc
    return {"sources": nsrc, "rk3_steps": nsteps, "receivers": 128, "tuned_launch": tuned,
            "states_kept": "every step's phi1 and psi resident" if K == 0 else f"a checkpoint every {K} steps",
            "archive_GB": need / 1e9 if K == 0 else 0.0,
            "forward_s": t_fwd, "backward_s": t_bwd, "plain_forward_s": t_plain, "first_call_forward_s": t_first,
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
    # the two contractions once untimed (buffers, first launches), then timed
    work = egb.alloc_bytes(max(egb.egb_born_workspace_size(P.eg, npoints, len(p.omegas)), 256), "cuda:0")
    d = egb.egb_born_data(P.eg, G, p.omegas, md, work=work)
    img = egb.egb_migrate(P.eg, G, p.omegas, d)
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    egb.egb_born_data(P.eg, G, p.omegas, md, d=d, work=work)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    egb.egb_migrate(P.eg, G, p.omegas, d, image=img)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tg, t1 = t1 - t0, t1b
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
    return {"surface_points": npoints, "frequencies": len(p.omegas), "greens_s": tg,
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


# sources the stage kernel is built from (the counter records name their hash)
STAGE_SOURCES = ("liouville.hip", "stage_common.h", "egb_device.h")


def stage_source_hash():
    import hashlib

    csrc = os.path.join(ROOT, "paper_2006_11945_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in STAGE_SOURCES)).hexdigest()


def measured_counters(workload, n):
    """The committed rocprofv3 record of the stage kernel on this workload
    (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE, VALU figures from the
    SQ counters), only while the kernel sources are unchanged since; else
    None."""
    path = os.path.join(ROOT, "profiles", f"k_stage_{workload}_traffic.json")
    if n is not None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec if stage_source_hash() == rec["source_sha256"] else None


def _counter_rows(folder):
    """Rows of every rocprofv3 counter_collection.csv under `folder`."""
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def summarize_counters(fetch_dir, write_dir, sq_dir):
    """Counter record of the stage kernel from three --pmc runs of a
    profiling pass of this bench (one RK3 step or more, --calibrate-copy-mib
    1024 so that a plain copy of known size scales FETCH_SIZE / WRITE_SIZE).
    Per dispatch the counter values of all reporting instances are summed;
    stage launches are the k_stage dispatches (not the batched ones)."""
    from collections import defaultdict

    def per_dispatch(folder, names):
        acc = defaultdict(lambda: defaultdict(float))
        kern, grid = {}, {}
        for r in _counter_rows(folder):
            if r["Counter_Name"] not in names:
                continue
            d = int(r["Dispatch_Id"])
            acc[d][r["Counter_Name"]] += float(r["Counter_Value"])
            kern[d] = r["Kernel_Name"]
            grid[d] = int(r.get("Grid_Size", 0) or 0)
        return acc, kern, grid

    def is_stage(name):
        return name.startswith("void egb::(anonymous namespace)::k_stage<") or name.startswith("egb::(anonymous namespace)::k_stage<")

    def stage_of(name):  # the template's second argument: the RK stage
        inner = name[name.index("<") + 1:]
        return int(inner.split(",")[1].strip())

    def copy_kib(acc, kern, counter):
        v = [acc[d][counter] for d in acc if "copyBuffer" in kern[d]]
        return max(v) if v else None

    cal = 1024 * 1024  # KiB of the 1 GiB calibration copy, read once and written once
    fa, fk, _ = per_dispatch(fetch_dir, {"FETCH_SIZE"})
    wa, wk, _ = per_dispatch(write_dir, {"WRITE_SIZE"})
    fscale = cal / copy_kib(fa, fk, "FETCH_SIZE")
    wscale = cal / copy_kib(wa, wk, "WRITE_SIZE")
    per_stage = defaultdict(lambda: {"fetch": [], "write": [], "valu": [], "active": [], "gui": [], "waves": []})
    for d, k in fk.items():
        if is_stage(k):
            per_stage[stage_of(k)]["fetch"].append(fa[d]["FETCH_SIZE"] * 1024 * fscale)
    for d, k in wk.items():
        if is_stage(k):
            per_stage[stage_of(k)]["write"].append(wa[d]["WRITE_SIZE"] * 1024 * wscale)
    sa, sk, _ = per_dispatch(sq_dir, {"SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE"})
    # GRBM_GUI_ACTIVE counts the cycles of each XCD: rocprofv3 either lists
    # the 8 instances per dispatch or gives one row with their sum; the
    # device's busy cycles are their mean either way
    inst_counts = defaultdict(int)
    for r in _counter_rows(sq_dir):
        if r["Counter_Name"] == "GRBM_GUI_ACTIVE":
            inst_counts[int(r["Dispatch_Id"])] += 1
    inst_counts = {d: (XCDS if n == 1 else n) for d, n in inst_counts.items()}
    for d, k in sk.items():
        if is_stage(k):
            st = per_stage[stage_of(k)]
            st["valu"].append(sa[d]["SQ_INSTS_VALU"])
            st["active"].append(sa[d]["SQ_ACTIVE_INST_VALU"])
            st["waves"].append(sa[d]["SQ_WAVES"])
            st["gui"].append(sa[d]["GRBM_GUI_ACTIVE"] / max(inst_counts[d], 1))
    mean = lambda v: sum(v) / len(v) if v else None
    stages = {}
    for k in sorted(per_stage):
        st = per_stage[k]
        f, w = mean(st["fetch"]), mean(st["write"])
        stages[k] = {"fetch_bytes": f, "write_bytes": w, "hbm_bytes": None if f is None or w is None else f + w,
                     "valu_instr": mean(st["valu"]), "valu_busy": None if not st["gui"] else
                     mean(st["active"]) * 4 / 1024 / mean(st["gui"]), "waves": mean(st["waves"])}
    hb = [v["hbm_bytes"] for v in stages.values() if v["hbm_bytes"] is not None]
    return {"kernel": "k_stage<float, *, 12, false>", "source_sha256": stage_source_hash(),
            "fetch_scale": fscale, "write_scale": wscale, "stages": stages,
            "hbm_bytes_per_launch": mean(hb),
            "valu_instr_per_launch": mean([v["valu_instr"] for v in stages.values() if v["valu_instr"] is not None]),
            "valu_busy": mean([v["valu_busy"] for v in stages.values() if v["valu_busy"] is not None])}


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


def window_problem(p, n, nsteps):
    """An n x n (x, z) window of problem p around its source over all theta
    nodes, with the same spacing and medium (the cost per cell of the whole
    grid)."""
    import numpy as np

    import workloads as W

    g = p.grid
    i0 = min(max(int(p.source.xs / g.dx) - n // 2, 0), g.nx - n)
    k0 = min(max(int(p.source.zs / g.dz) - n // 2, 0), g.nz - n)
    gw = W.Grid(nx=n, nz=n, nth=g.nth, dx=g.dx, dz=g.dz, x0=g.x0 + i0 * g.dx, z0=g.z0 + k0 * g.dz)
    cut = lambda a: np.ascontiguousarray(a[i0:i0 + n, k0:k0 + n])
    m = p.medium
    mw = W.Medium(vp0=cut(m.vp0), eps=cut(m.eps), delta=cut(m.delta), tilt=cut(m.tilt), vs_ratio=m.vs_ratio)
    return W.Problem(p.name + "-window", gw, mw, p.source, nsteps, p.omegas, dtype=p.dtype)


def cpu_baseline(key, p, window, nsteps):
    """The oracle (as it stands) on `nsteps` RK3 steps of an n x n window of
    the workload's grid over all its theta nodes (the whole grid when the
    window covers it), on the host cores."""
    import oracle

    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    g = p.grid
    pw = p if window >= min(g.nx, g.nz) else window_problem(p, window, nsteps)
    t0 = time.perf_counter()
    r = oracle.solve(pw, nsteps=0)
    t1 = time.perf_counter()
    oracle.march(pw.grid, r["vel"], pw.source, r["U0"], r["dt"], nsteps)
    t2 = time.perf_counter()
    gw = pw.grid
    what = "the full grid" if pw is p else f"a {gw.nx}x{gw.nz} (x, z) window of the {g.nx}x{g.nz} grid around the source"
    return {"value": gw.ncell * nsteps / (t2 - t1), "unit": "cell-updates/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", cores)), "kind": "oracle",
            "sample": f"{nsteps} SSP-RK3 step(s) of {what}, all {gw.nth} theta nodes, same spacing and medium "
                      f"(FP64; setup {t1 - t0:.1f} s not counted, march {t2 - t1:.1f} s)",
            "cpu_model": cpu_model(), "value_1_thread": single_thread_oracle(key, min(window, g.nx) // 4),
            "sample_1_thread": f"one SSP-RK3 step of a {min(window, g.nx) // 4}^2 (x, z) window of the same "
                               "grid, OMP_NUM_THREADS=1"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_thread_oracle(key, window):
    """The oracle on one thread (a child process: OpenMP fixes its thread
    count when the library loads), one RK3 step of a window of the
    workload's grid; cell-updates/s, None if it did not run."""
    import subprocess

    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import bench, oracle\n"
            "p = bench.window_problem(bench.make_workload(%r), %d, 1)\n"
            "r = oracle.solve(p, nsteps=0)\n"
            "t0 = time.perf_counter()\n"
            "oracle.march(p.grid, r['vel'], p.source, r['U0'], r['dt'], 1)\n"
            "print(p.grid.ncell / (time.perf_counter() - t0))\n") % (ROOT, key, window)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        return float(out.stdout.strip().splitlines()[-1]) if out.returncode == 0 else None
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None


def timed_passes(egb, p, steps, warmup, tune, stream):
    """Warm-up then `steps` timed passes of the whole path on problem p:
    medium table and velocity, point-source data, the march, the beam sum,
    the pick at 128 receivers.  The march and the beam sum of each timed
    pass are bracketed by HIP events on the launch stream."""
    import numpy as np
    import torch

    L = p.grid.nx * p.grid.dx
    rx = np.stack([np.linspace(0.1 * L, 0.9 * L, 128), np.full(128, 0.9 * L)], axis=1)
    dev = torch.device("cuda:0")
    s = egb.Solver(p, dev)
    dt = s.velocity()
    s.init()
    # stage launch (tile shape, block count) for this grid; results do not depend on it
    if tune:
        s.tune(reps=6)
    tile_rows, blocks = egb.egb_get_launch(s.eg, egb.EGB_TUNE_STEP)
    s.work_beam = egb.alloc_bytes(egb.workspace_size(s.eg, egb.EGB_OP_BEAM), dev)
    out = torch.empty((len(p.omegas), p.grid.nx, p.grid.nz, 2), dtype=torch.float32, device=dev)
    rx_d = torch.as_tensor(rx, device=dev)
    t_pick = torch.empty(128, dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    march_ms, beam_ms = [], []

    def one_pass(timed):
        s.velocity()
        s.init()
        if timed:
            ev[0].record(stream)
        s.step(p.nsteps, dt=dt)
        if timed:
            ev[1].record(stream)
        s.beam(p.omegas, out=out)
        if timed:
            ev[2].record(stream)
        egb.egb_pick_receivers(s.eg, s.state, rx_d, t_pick)
        if timed:
            ev[2].synchronize()
            march_ms.append(ev[0].elapsed_time(ev[1]))
            beam_ms.append(ev[1].elapsed_time(ev[2]))

    for _ in range(warmup):
        one_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one_pass(True)
        print(f"bench: pass {i + 1}/{steps} {march_ms[-1] + beam_ms[-1]:.0f} ms on the GPU", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    finite = bool(torch.isfinite(out).all()) and bool(torch.isfinite(t_pick).any())
    del s, out
    torch.cuda.empty_cache()
    return {"ms": (t1 - t0) * 1e3 / steps, "march_ms": float(np.mean(march_ms)), "beam_ms": float(np.mean(beam_ms)),
            "blocks": blocks, "tile_rows": tile_rows, "dt": dt, "finite": finite}


def stage_roofline(p, r, rec):
    """Roofline entry of the stage kernel from the live launch time and the
    committed counter record (None fields when there is none)."""
    cells = p.grid.ncell
    stage_ms = r["march_ms"] / (3 * p.nsteps)
    achieved = cells * FLOP_CELL_STAGE / (stage_ms * 1e-3) / 1e12
    traffic = None if rec is None else rec["hbm_bytes_per_launch"]
    hbm = None if traffic is None else traffic / (stage_ms * 1e-3) / 1e9
    # SQ_INSTS_VALU counts wave instructions; a wave updates 64 cells (one per lane)
    valu = None if rec is None or rec.get("valu_instr_per_launch") is None else rec["valu_instr_per_launch"] * 64 / cells
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
            "kernel": "k_stage (one SSP-RK3 stage)", "avg_launch_ms": stage_ms, "blocks_per_launch": r["blocks"],
            "tile_theta_rows": r["tile_rows"],
            "flop_per_cell_stage": FLOP_CELL_STAGE,
            # FP32 arithmetic without packed (dual-lane) instructions, which the library is compiled without
            "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS, "frac_of_unpacked": achieved / PEAK_FP32_UNPACKED_TFLOPS,
            # HBM side: counter bytes over the live launch time
            "hbm_GBps": hbm, "hbm_frac_of_8TBps": None if hbm is None else hbm / PEAK_HBM_GBPS,
            "traffic_bytes_per_cell_stage": None if traffic is None else traffic / cells,
            "valu_instr_per_cell_stage": valu, "valu_busy": None if rec is None else rec.get("valu_busy")}


def main():
    args = parse()
    if args.summarize_counters:
        print(json.dumps(summarize_counters(*args.summarize_counters), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a design "
              "note, not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2006_11945_amd as egb

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    # the oracle on the host cores first (CPU only, ~15 s): it is part of every
    # line, whatever the time the timed passes leave for the secondary legs
    cpu = None
    if not args.no_cpu_baseline:
        print(f"bench: leg cpu_baseline at {time.perf_counter() - T_START:.0f} s", file=sys.stderr, flush=True)
        win = 256 if args.workload == "tti512" and args.n is None else 10 ** 9
        cpu = cpu_baseline(args.workload, make_workload(args.workload, args.n, 2), win, 2 if win < 10 ** 9 else 1)
    p = make_workload(args.workload, args.n, args.rk_steps)
    r = timed_passes(egb, p, args.steps, args.warmup, not args.no_tune, stream)
    cells = p.grid.ncell
    value = cells * p.nsteps / (r["ms"] * 1e-3)
    rec = measured_counters(args.workload, args.n)
    g = p.grid
    desc = WORKLOADS[args.workload] if args.n is None and args.rk_steps is None else (
        f"{p.name} {g.nx}x{g.nz}x{g.nth}, {p.nsteps} RK3 steps, beam sum {len(p.omegas)} freqs 5-60 Hz, "
        "128 receivers")
    res = {
        "metric": "phase-space cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "grid": [g.nx, g.nz, g.nth], "rk3_steps": p.nsteps,
                   "frequencies": len(p.omegas), "receivers": 128, "psi_dtype": "f64", "tilt": args.workload == "tti512"},
        "roofline": stage_roofline(p, r, rec),
        "hbm_floor": {"bytes_per_cell_update": FLOOR_BYTES_PER_CELL_UPDATE,
                      "GBps": value * FLOOR_BYTES_PER_CELL_UPDATE / 1e9,
                      "frac_of_8TBps": value * FLOOR_BYTES_PER_CELL_UPDATE / 1e9 / PEAK_HBM_GBPS,
                      "note": "the state read and written once per RK3 step at the whole pass's rate"},
        "beam_sum": {"ms": r["beam_ms"], "frequencies": len(p.omegas),
                     "output_point_freqs_per_s": g.nx * g.nz * len(p.omegas) / (r["beam_ms"] * 1e-3)},
        "march_ms": r["march_ms"],
        "march_cell_updates_per_s": cells * p.nsteps / (r["march_ms"] * 1e-3),
        "outputs_finite": r["finite"],
    }
    res["roofline"]["copy_GBps"] = copy_bandwidth()  # after the timed region
    hbm = res["roofline"]["hbm_GBps"]
    res["roofline"]["hbm_frac_of_copy"] = None if hbm is None else hbm / res["roofline"]["copy_GBps"]

    def budget_ok(name, est_s):
        if args.time_budget_s > 0 and time.perf_counter() - T_START + est_s > args.time_budget_s:
            res[name] = {"skipped": f"time budget ({args.time_budget_s:.0f} s after the start)"}
            return False
        print(f"bench: leg {name} at {time.perf_counter() - T_START:.0f} s", file=sys.stderr, flush=True)
        return True

    if cpu is not None:
        res["cpu_baseline"] = cpu
    # secondary legs, each skipped when it would end past the time budget
    # (rough duration estimates, seconds)
    if args.batched_steps > 0 and budget_ok("batched", 40):
        res["batched"] = batched_vs_sequential(args.batched_problems, args.batched_steps, tune=not args.no_tune)
        # many small problems: one problem alone cannot fill the chip
        res["batched_small"] = batched_vs_sequential(256, 4 * args.batched_steps, lo=32, hi=96,
                                                     tune=not args.no_tune)
        torch.cuda.empty_cache()
    if args.adjoint_sources > 0 and budget_ok("adjoint", 8 + 16 * args.adjoint_sources):
        res["adjoint"] = adjoint_vs_forward(args.adjoint_sources, 600, 256, tune=not args.no_tune)
        torch.cuda.empty_cache()
    if args.vti_leg > 0 and args.workload != "vti256" and budget_ok("vti256", 6 + 2 * args.vti_leg):
        pv = make_workload("vti256")
        rv = timed_passes(egb, pv, args.vti_leg, 1, not args.no_tune, stream)
        vv = pv.grid.ncell * pv.nsteps / (rv["ms"] * 1e-3)
        res["vti256"] = {"workload": WORKLOADS["vti256"], "passes": args.vti_leg, "ms_per_pass": rv["ms"],
                         "cell_updates_per_s": vv, "march_ms": rv["march_ms"], "beam_ms": rv["beam_ms"],
                         "roofline": stage_roofline(pv, rv, measured_counters("vti256", None)),
                         "outputs_finite": rv["finite"]}
    if args.paraxial_sources > 0 and budget_ok("paraxial", 12):
        res["paraxial"] = paraxial_leg(256, args.paraxial_sources, migration_points=args.migration_points)
        torch.cuda.empty_cache()
    res["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
