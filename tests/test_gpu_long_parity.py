"""Full-length parity: the GPU march over the step counts of the benchmark
workloads against the FP64 oracle marched the same steps on the host cores,
and the whole path end to end (GPU march -> GPU beam sum and pick against
oracle march -> oracle beam sum and pick), in the benchmark's launch
configuration.

* The heterogeneous VTI recipe (8 blobs, smoothed epsilon and delta, 4 km
  square) at 128^3 for its 600 RK3 steps, 32 frequencies 5-60 Hz.
* The TTI recipe (the same plus a smooth tilt in [-45, 45] degrees) at 96^3,
  64 frequencies: for 225 RK3 steps (the pseudo-time, 0.68 s, that the
  512^3 workload's 1200 steps cover: the step scales with the cell size) and
  for 1200 steps (3.6 s).

One oracle run serves two GPU marches:
* FP64 planes: the kernels compute the oracle's arithmetic, up to the order
  of rounding (FMA contraction on the GPU): picks and wavefield within
  1e-9, every plane within 1e-7 of its maximum (a long march amplifies
  rounding-order differences where the field is not smooth; measured
  <= 6.2e-9 in the DRT planes of the TTI march after 1200 steps, 1e-10 in
  phi1 and psi);
* FP32 planes (psi in FP64, its WENO derivative evaluated in FP32): the
  traveltime psi within 1e-5 relative over the active cells (|phi1| /
  |grad phi1| < 2 dx, psi > 0) more than two source-ball radii of travel
  from the source (psi >= 2 r0 / max|V|; nearer, psi is a few cells of
  traveltime and FP32 rounding of the convection term, ~1e-7 s after a
  long march, is not small relative to it), and within 1e-5 of the largest
  traveltime over all active cells; the first arrivals at 128 receivers
  1e-5 relative (arrival or none alike); the wavefield relative L2 <= 1e-4
  per frequency.  The FP32 phi1 and DRT planes are reported, not bounded
  on their own: over long marches their rounding grows where the field is
  not smooth (measured up to 8e-4 of the maximum away from Gamma), and the
  wavefield, which reads them on Gamma, is the bound.
* TTI over 1200 steps: most far active cells have not settled (WENO's
  nonlinear weights keep psi moving near the tube edges), and there the
  march amplifies any perturbation: the FP64 oracle with only its velocity
  field rounded to FP32 moves by the amounts stored in
  tests/golden/tti96_fp32_velocity_sensitivity.json (written by the oracle
  alone).  The FP32 bounds there are the bars above or ten times that
  sensitivity, whichever is larger (measured ratios: psi 3.4, first
  arrivals 3.7, wavefield up to 1.1: the FP32 march rounds every plane at
  every step, the reference perturbation only the velocity, once; the
  wavefield ratio moves with any change of rounding in the march, 5.0 and
  12 with two other roundings of the same WENO5 arithmetic), and psi
  on the cells that have settled (psi changes by at most 1e-7 relative over
  10 further oracle steps) the same way (measured 2.1e-5 against 5.5e-6).
The oracle marches in chunks and reports its progress."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.conftest import progress
from tests.gpu_helpers import gpu_planes, oracle_planes, rel_err, plane_scale

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def receivers(p):
    L = p.grid.nx * p.grid.dx
    return np.stack([np.linspace(0.1 * L, 0.9 * L, 128), np.full(128, 0.9 * L)], axis=1)


def gpu_run(p, dtype, rx, dt=None):
    import paper_2006_11945_amd as egb

    s = egb.Solver(p, DEV, dtype)
    dt_cfl = s.velocity()
    s.init()
    s.step(p.nsteps, dt=dt_cfl if dt is None else dt)
    out = s.beam(p.omegas)
    t = s.pick(rx).cpu().numpy()
    torch.cuda.synchronize()
    Gw = out.double().cpu().numpy()
    planes = gpu_planes(s)
    del s, out
    torch.cuda.empty_cache()
    return planes, Gw[..., 0] + 1j * Gw[..., 1], t, dt_cfl


SENS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tti96_fp32_velocity_sensitivity.json")


def full_length(p, label, sens=None):
    from tests.test_gpu_parity import active_mask

    rx = receivers(p)
    progress(f"[{label}] GPU: {p.grid.nx}x{p.grid.nz}x{p.grid.nth}, {p.nsteps} RK3 steps, "
             f"{len(p.omegas)} frequencies, FP64 and FP32")
    G64, W64, t64, dt = gpu_run(p, "f64", rx)
    G32, W32, t32, _ = gpu_run(p, "f32", rx, dt)
    o = oracle.solve(p, nsteps=0, dt=dt)
    U = o["U0"]
    chunk = 50
    for done in range(0, p.nsteps, chunk):  # the same march (ghosts and ball from the initial data)
        U = oracle.march(p.grid, o["vel"], p.source, U, dt, min(chunk, p.nsteps - done), Ub=o["U0"])
        progress(f"[{label}] oracle at step {min(done + chunk, p.nsteps)}/{p.nsteps}")
    O = oracle_planes(U)
    Us = oracle.march(p.grid, o["vel"], p.source, U, dt, 10, Ub=o["U0"])  # has psi settled?
    t_or = oracle.pick(p.grid, U, rx)
    Ow = oracle.beam_sum(p.grid, o["vel"], o["vaux"], p.source, U, p.omegas)
    wrel = lambda Gw: np.array([np.linalg.norm(Gw[w] - Ow[w]) / np.linalg.norm(Ow[w]) for w in range(len(p.omegas))])
    ok = ~np.isnan(t_or)
    prel = lambda t: (np.abs(t - t_or)[ok] / t_or[ok]).max()

    # FP64: the oracle's arithmetic
    e64 = {name: rel_err(G64[name], O[name], np.abs(O[name]).max() if name == "psi" else plane_scale(O, name))
           for name in O}
    w64 = wrel(W64)
    progress(f"[{label}] FP64 planes " + " ".join(f"{k} {v:.1e}" for k, v in e64.items()) +
             f"; picks {prel(t64):.1e}; wavefield {w64.max():.1e}")
    assert max(e64.values()) <= 1e-7
    assert np.array_equal(np.isnan(t64), np.isnan(t_or)) and prel(t64) <= 1e-9
    assert w64.max() <= 1e-9

    # FP32
    act = active_mask(p.grid, U)
    vmax = float(np.sqrt(o["vel"][0] ** 2 + o["vel"][1] ** 2).max())
    far = act & (U[1] >= 2 * p.source.r0 / vmax)
    settled = far & (np.abs(Us[1] - U[1]) <= 1e-7 * U[1])
    dpsi = np.abs(G32["psi"] - O["psi"])
    trel = (dpsi[far] / O["psi"][far]).max()
    srel = (dpsi[settled] / O["psi"][settled]).max() if settled.any() else 0.0
    tabs = dpsi[act].max() / O["psi"][act].max()
    errs = {name: rel_err(G32[name], O[name], plane_scale(O, name))
            for name in ("phi1", "ReC", "ImC", "ReB", "ImB", "phase")}
    w32 = wrel(W32)
    progress(f"[{label}] FP32 psi rel {trel:.2e} over {far.sum()} active cells beyond 2 r0 ({srel:.2e} over the "
             f"{settled.sum()} settled ones), abs/max {tabs:.2e}; " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    progress(f"[{label}] FP32 picks: {ok.sum()} arrivals, max rel err {prel(t32):.2e}; wavefield rel L2 max "
             f"{w32.max():.2e} (at {p.omegas[w32.argmax()] / 2 / np.pi:.1f} Hz), median {np.median(w32):.2e}")
    assert all(np.isfinite(G32[name]).all() for name in G32)
    assert np.array_equal(np.isnan(t32), np.isnan(t_or))
    assert ok.sum() > 64
    assert np.isfinite(W32).all()
    if sens is None:
        assert trel <= 1e-5 and tabs <= 1e-5
        assert prel(t32) <= 1e-5
        assert w32.max() <= 1e-4
    else:
        # the bars, or ten times the oracle's own move under FP32 velocity
        wsens = np.asarray(sens["wavefield_rel_l2"])
        progress(f"[{label}] oracle FP32-velocity sensitivity: psi {sens['psi_far_max']:.2e} (settled "
                 f"{sens['psi_settled_max']:.2e}), picks {sens['picks_max']:.2e}, wavefield max {wsens.max():.2e}; "
                 f"ratios psi {trel / sens['psi_far_max']:.2f}, picks {prel(t32) / sens['picks_max']:.2f}, "
                 f"wavefield {(w32 / wsens).max():.2f}")
        K = 10
        assert trel <= max(1e-5, K * sens["psi_far_max"]) and tabs <= max(1e-5, K * sens["psi_far_max"])
        assert srel <= max(1e-5, K * sens["psi_settled_max"])
        assert prel(t32) <= max(1e-5, K * sens["picks_max"])
        assert np.all(w32 <= np.maximum(1e-4, K * wsens))


def test_vti_recipe_128_full_600_steps_end_to_end():
    full_length(W.vti_256(n=128, nsteps=600), "VTI 128^3 x 600")


def test_tti_recipe_96_workload_pseudo_time_end_to_end():
    full_length(W.tti_512(n=96, nsteps=1200 * 96 // 512), "TTI 96^3 x 225")


def test_tti_recipe_96_full_1200_steps_end_to_end():
    sens = json.load(open(SENS))
    assert sens["workload"] == "TTI recipe 96^3, 1200 SSP-RK3 steps"
    full_length(W.tti_512(n=96, nsteps=1200), "TTI 96^3 x 1200", sens)
