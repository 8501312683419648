"""The KMAH phase on the GPU.  Behind a low-velocity Gaussian lens the rays
from a point source form a caustic and a triplication zone, and the middle
arrival's C turns past pi, so its beams take the other branch of
sqrt(v / C).  The GPU march carries the phase plane (arg C continued along
the ray, source A12 Im(B / C), linear fifth-order upwind derivative) and the
beam sum picks each beam's branch from it; both against the oracle on the
same grid and pseudo-time step, 0.7 s of pseudo-time (the whole lens and
the zone below it):
* FP64 planes: every plane, the phase included, within 1e-9 of its scale
  (the oracle's arithmetic up to rounding order); FP32: within 1e-4;
* the branch index round((phase - arg C) / 2 pi) equal on the cells of
  Gamma (|phi1| / |grad phi1| < 2 dx, psi > 0) where the oracle's phase is
  more than 0.01 rad from a branch boundary (all but a few cells next to the
  caustic, where |C| is small and the march resolves C poorly: measured
  within 0.12 rad at worst, 3 cells beyond 0.9 pi of 12478), with odd
  indices present (724 cells);
* the Green's function at 5-30 Hz: FP64 within 1e-9 relative L2 of the
  oracle's, FP32 within 1e-4, while the sum with every beam on the principal
  branch (the oracle's, phase set to arg C) is more than 1e-2 away."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.raytrace import GaussianLensMedium
from tests.gpu_helpers import gpu_planes, log, oracle_planes, plane_scale, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PSEUDO_TIME = 0.7


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def lens_problem(dtype):
    med = GaussianLensMedium(2000.0, -700.0, 600.0, 420.0, 110.0)
    dx = 25.0
    g = W.Grid(nx=32, nz=44, nth=96, dx=dx, dz=dx, x0=210.0, z0=-50.0)
    X, Z = np.meshgrid(g.xc(), g.zc(), indexing="ij")
    v = med.vgrad(X, Z)[0]
    zero = np.zeros_like(v)
    m = W.Medium(vp0=v, eps=zero, delta=zero, tilt=zero, vs_ratio=0.5)
    src = W.Source(xs=610.0, zs=100.0, r0=4 * dx, beta=1.0 / 2200.0)
    return W.Problem("lens", g, m, src, 0, W.hz([5.0, 10.0, 20.0, 30.0]), dtype=dtype)


def branch(P):
    """Branch index and the distance of the phase from its branch's centre."""
    r = P["phase"] - np.arctan2(P["ImC"], P["ReC"])
    k = np.rint(r / (2 * np.pi))
    return k, np.abs(r - 2 * np.pi * k)


@pytest.fixture(scope="module")
def lens_runs():
    import paper_2006_11945_amd as egb

    out = {}
    dt = nsteps = None
    for dtype in ("f64", "f32"):
        p = lens_problem(dtype)
        s = egb.Solver(p, DEV, dtype)
        dt_cfl = s.velocity()
        if dt is None:
            dt, nsteps = dt_cfl, int(np.ceil(PSEUDO_TIME / dt_cfl))
        log(f"lens {dtype}: {p.grid.nx}x{p.grid.nz}x{p.grid.nth}, {nsteps} RK3 steps, dt {dt:.4e}")
        s.init()
        s.step(nsteps, dt=dt)
        Gw = s.beam(p.omegas).double().cpu().numpy()
        torch.cuda.synchronize()
        out[dtype] = (gpu_planes(s), Gw[..., 0] + 1j * Gw[..., 1])
        del s
    p = lens_problem("f64")
    o = oracle.solve(p, nsteps=0, dt=dt)
    U = oracle.march(p.grid, o["vel"], p.source, o["U0"], dt, nsteps, Ub=o["U0"])
    Ow = oracle.beam_sum(p.grid, o["vel"], o["vaux"], p.source, U, p.omegas)
    Up = U.copy()
    Up[6] = np.arctan2(U[3], U[2])  # every beam on the principal branch
    Pw = oracle.beam_sum(p.grid, o["vel"], o["vaux"], p.source, Up, p.omegas)
    torch.cuda.empty_cache()
    return p, U, Ow, Pw, out


def gamma_mask(p, U):
    from tests.test_gpu_parity import active_mask

    return active_mask(p.grid, U)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_phase_plane_and_branches_match_the_oracle(lens_runs, dtype):
    p, U, _, _, out = lens_runs
    G, O = out[dtype][0], oracle_planes(U)
    tol = 1e-9 if dtype == "f64" else 1e-4
    errs = {name: rel_err(G[name], O[name], np.abs(O[name]).max() if name == "psi" else plane_scale(O, name))
            for name in O}
    log(f"  {dtype} planes " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert max(errs.values()) <= tol
    act = gamma_mask(p, U)
    kg, ko, off = branch(G)[0][act], branch(O)[0][act], branch(O)[1][act]
    sure = off < np.pi - 1e-2
    log(f"  {dtype} branches on {act.sum()} Gamma cells: odd {int(np.sum(ko % 2 != 0))}, "
        f"mismatches {int(np.sum(kg != ko))} ({int(np.sum((kg != ko) & sure))} away from a branch boundary)")
    assert act.sum() > 1000 and np.sum(ko % 2 != 0) > 20 and np.sum(~sure) <= 3
    assert np.array_equal(kg[sure], ko[sure])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_beam_sum_takes_each_beams_branch(lens_runs, dtype):
    p, _, Ow, Pw, out = lens_runs
    Gw = out[dtype][1]
    rel = lambda A, B: np.array([np.linalg.norm(A[w] - B[w]) / np.linalg.norm(B[w]) for w in range(len(p.omegas))])
    e, d = rel(Gw, Ow), rel(Pw, Ow)
    log(f"  {dtype} wavefield rel L2 {np.array2string(e, precision=2)}; principal-branch sum off by "
        f"{np.array2string(d, precision=2)}")
    assert np.isfinite(Gw).all()
    assert e.max() <= (1e-9 if dtype == "f64" else 1e-4)
    assert d.min() > 1e-2
