"""Write tti96_fp32_velocity_sensitivity.json: how far the FP64 oracle itself
moves when only its Liouville velocity field (V and A) is rounded to FP32,
on the TTI recipe at 96^3 over 1200 SSP-RK3 steps (3.6 s of pseudo-time).
Everything else stays FP64, so the numbers measure the conditioning of the
long march, not any kernel: they bound what an FP32 path can match.

Both marches share the CFL step and the FP64 initial and boundary data.
Recorded: the traveltime psi, max relative difference over the active
cells beyond two source-ball radii of travel (all of them, and those whose
psi has settled: changes by at most 1e-7 relative over 10 further steps of
the exact march); the first arrivals at 128 receivers (max relative
difference over receivers with an arrival in both); the Green's function at
the 64 frequencies 5-60 Hz (relative L2 per frequency).

Run from the repository root (about 25 minutes on 8 cores):
    python tests/golden/make_tti_fp32_sensitivity.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N, STEPS, SETTLE = 96, 1200, 10


def active(g, U):
    """Cells near Gamma (|phi1| / |grad phi1| < 2 dx in rows or columns) with psi > 0."""
    phi, psi = U[0], U[1]
    lam = g.dx / g.dth
    ft = (np.roll(phi, -1, 0) - np.roll(phi, 1, 0)) / (2 * g.dth)
    fx = np.gradient(phi, g.dx, axis=1)
    fz = np.gradient(phi, g.dz, axis=2)
    drow = phi / np.sqrt(fx ** 2 + (ft / lam) ** 2)
    dcol = phi / np.sqrt(fz ** 2 + (ft / lam) ** 2)
    return ((np.abs(drow) < 2 * g.dx) | (np.abs(dcol) < 2 * g.dz)) & (psi > 0)


def main():
    p = W.tti_512(n=N, nsteps=STEPS)
    g = p.grid
    o = oracle.solve(p, nsteps=0)
    dt = o["dt"]
    vel32 = o["vel"].astype(np.float32).astype(np.float64)
    Ua = oracle.march(g, o["vel"], p.source, o["U0"], dt, STEPS, Ub=o["U0"])
    Ub = oracle.march(g, vel32, p.source, o["U0"], dt, STEPS, Ub=o["U0"])
    Us = oracle.march(g, o["vel"], p.source, Ua, dt, SETTLE, Ub=o["U0"])
    vmax = float(np.sqrt(o["vel"][0] ** 2 + o["vel"][1] ** 2).max())
    far = active(g, Ua) & (Ua[1] >= 2 * p.source.r0 / vmax)
    settled = far & (np.abs(Us[1] - Ua[1]) <= 1e-7 * Ua[1])
    rel = np.abs(Ua[1] - Ub[1]) / np.where(far, Ua[1], 1.0)
    L = g.nx * g.dx
    rx = np.stack([np.linspace(0.1 * L, 0.9 * L, 128), np.full(128, 0.9 * L)], axis=1)
    ta, tb = oracle.pick(g, Ua, rx), oracle.pick(g, Ub, rx)
    ok = ~np.isnan(ta) & ~np.isnan(tb)
    Ga = oracle.beam_sum(g, o["vel"], o["vaux"], p.source, Ua, p.omegas)
    Gb = oracle.beam_sum(g, o["vel"], o["vaux"], p.source, Ub, p.omegas)
    wf = [float(np.linalg.norm(Ga[w] - Gb[w]) / np.linalg.norm(Ga[w])) for w in range(len(p.omegas))]
    rec = {
        "workload": f"TTI recipe {N}^3, {STEPS} SSP-RK3 steps",
        "dt": dt, "pseudo_time_s": dt * STEPS,
        "far_active_cells": int(far.sum()), "settled_cells": int(settled.sum()),
        "psi_far_max": float(rel[far].max()), "psi_settled_max": float(rel[settled].max()),
        "picks_max": float((np.abs(ta - tb)[ok] / ta[ok]).max()), "picks_compared": int(ok.sum()),
        "wavefield_hz": [float(w / (2 * np.pi)) for w in p.omegas], "wavefield_rel_l2": wf,
        "command": "python tests/golden/make_tti_fp32_sensitivity.py",
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tti96_fp32_velocity_sensitivity.json")
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k not in ("wavefield_hz", "wavefield_rel_l2")}))
    print("wavefield max", max(wf))


if __name__ == "__main__":
    main()
