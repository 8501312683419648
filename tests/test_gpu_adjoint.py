"""Traveltime-misfit gradients from the HIP adjoint (through the C ABI)
against the oracle's autograd gradient, and a directional-derivative check of
the full-size adjoint workload."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import adjoint as AD
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def adjoint_problem(n=24, nth=24, nsteps=14, tilt=True):
    L = 480.0
    g = W.Grid(nx=n, nz=n + 4, nth=nth, dx=L / n, dz=L / n)
    rng = W.rng_for(4, 900)
    med = W.vti_medium(rng, g, L, tilt=tilt)
    src = W.Source(xs=0.5 * L + 3.0, zs=0.3 * L, r0=4 * g.dx, beta=1.0 / (2 * L))
    rx = np.stack([np.linspace(0.25 * L, 0.75 * L, 9), np.full(9, 0.72 * L)], axis=1)
    return W.Problem("adj", g, med, src, nsteps, W.hz([20.0])), rx


def spec_of(p, rx, dtype, dt, K=5):
    return {"grid": p.grid, "source": p.source, "receivers": rx, "nsteps": p.nsteps,
            "vs_ratio": p.medium.vs_ratio, "dtype": dtype, "checkpoint_every": K, "dt": dt}


def gpu_gradient(p, rx, t_obs, dtype, dt, K=5):
    import paper_2006_11945_amd as egb
    ts = [torch.tensor(np.asarray(a, dtype=np.float64), device=DEV, requires_grad=True)
          for a in (p.medium.vp0, p.medium.eps, p.medium.delta, p.medium.tilt)]
    t = egb.traveltime(*ts, spec_of(p, rx, dtype, dt, K))
    ok = ~torch.isnan(t)
    J = torch.sum((t[ok] - torch.as_tensor(t_obs, device=DEV)[ok]) ** 2)
    J.backward()
    return float(J.detach()), [x.grad.cpu().numpy() for x in ts], t.detach().cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_gradient_matches_oracle(dtype):
    p, rx = adjoint_problem()
    r = oracle.solve(p)
    dt = r["dt"]
    true = replace(p.medium, vp0=p.medium.vp0 * 1.03, eps=p.medium.eps + 0.02)
    rt = oracle.solve(replace(p, medium=true), dt=dt)
    t_obs = oracle.pick(p.grid, rt["U"], rx)
    Jo, go = AD.gradient(p, rx, t_obs, dt, p.nsteps)
    Jg, gg, tg = gpu_gradient(p, rx, t_obs, dtype, dt)
    log(f"adjoint {dtype}: J oracle {Jo:.6e} gpu {Jg:.6e}")
    tol = 1e-9 if dtype == "f64" else 1e-3
    assert Jg == pytest.approx(Jo, rel=1e-9 if dtype == "f64" else 1e-4)
    for name, a, b in zip(("vp0", "eps", "delta", "tilt"), gg, go):
        e = np.abs(a - b).max() / np.abs(b).max()
        log(f"  d/d{name}: max rel err {e:.3e} (scale {np.abs(b).max():.3e})")
        assert e < tol, name


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_gradient_with_receivers_at_the_edges(dtype):
    """Receivers in the first and last cells of x and z: their traveltimes
    depend on the ghost values (the point-source data extended past the
    edges), so the gradient carries the boundary-data sensitivity through
    the source as well."""
    p, _ = adjoint_problem(nsteps=20)
    g = p.grid
    Lx, Lz = g.nx * g.dx, g.nz * g.dz
    rx = np.array([[0.5 * g.dx, 0.35 * Lz], [Lx - 0.5 * g.dx, 0.4 * Lz], [0.45 * Lx, Lz - 0.5 * g.dz],
                   [0.6 * Lx, 0.5 * g.dz], [0.5 * g.dx, Lz - 0.5 * g.dz], [Lx - 1.5 * g.dx, 1.5 * g.dz]])
    r = oracle.solve(p)
    t_obs = oracle.pick(g, oracle.solve(replace(p, medium=replace(p.medium, vp0=p.medium.vp0 * 1.02)),
                                        dt=r["dt"])["U"], rx)
    Jo, go = AD.gradient(p, rx, t_obs, r["dt"], p.nsteps)
    Jg, gg, _ = gpu_gradient(p, rx, t_obs, dtype, r["dt"])
    log(f"adjoint edges {dtype}: J oracle {Jo:.6e} gpu {Jg:.6e}")
    assert Jo > 0
    assert Jg == pytest.approx(Jo, rel=1e-9 if dtype == "f64" else 1e-4)
    tol = 1e-9 if dtype == "f64" else 1e-3
    for name, a, b in zip(("vp0", "eps", "delta", "tilt"), gg, go):
        e = np.abs(a - b).max() / np.abs(b).max()
        log(f"  d/d{name}: max rel err {e:.3e}")
        assert e < tol, name


def test_adjoint_checkpoint_interval_does_not_change_gradient():
    p, rx = adjoint_problem(nsteps=11)
    r = oracle.solve(p)
    t_obs = oracle.pick(p.grid, oracle.solve(replace(p, medium=replace(p.medium, vp0=p.medium.vp0 * 0.98)),
                                                 dt=r["dt"])["U"], rx)
    _, g1, _ = gpu_gradient(p, rx, t_obs, "f64", r["dt"], K=1)
    _, g2, _ = gpu_gradient(p, rx, t_obs, "f64", r["dt"], K=4)
    _, g0, _ = gpu_gradient(p, rx, t_obs, "f64", r["dt"], K=0)  # every step's phi1 and psi resident
    _, g32a, _ = gpu_gradient(p, rx, t_obs, "f32", r["dt"], K=0)
    _, g32b, _ = gpu_gradient(p, rx, t_obs, "f32", r["dt"], K=3)
    for a, b, c in zip(g1, g2, g0):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    for a, b in zip(g32a, g32b):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("src_index", [3, 12])
def test_adjoint_full_size_directional_derivative(src_index):
    """256^3 VTI medium, 600 RK3 steps, 128 receivers, one of the 16 sources
    of the adjoint workload each: <grad J, d> against a central difference
    of J along a smooth direction d of each parameter (vp0, eps, delta,
    tilt).  Every step's phi1 and psi stay resident for the backward sweep
    (121 GB at this size)."""
    import paper_2006_11945_amd as egb
    probs = W.adjoint_sources(nsteps=600)
    p = probs[src_index]
    rx = p.receivers
    true = p.extra["true_medium"]
    log(f"adjoint full size 256^3, 600 steps, source {src_index}")
    spec = {"grid": p.grid, "source": p.source, "receivers": rx, "nsteps": p.nsteps, "vs_ratio": 0.5,
            "dtype": "f32"}
    mk = lambda m: [torch.tensor(np.asarray(a, dtype=np.float64), device=DEV) for a in (m.vp0, m.eps, m.delta, m.tilt)]
    # every evaluation uses one step, within the CFL limits of the base and
    # the observed media and of the finite-difference perturbations (the
    # library refuses a step above the limit of the medium it marches)
    spec["dt"] = 0.95 * min(egb.Solver(p, DEV).velocity(), egb.Solver(replace(p, medium=true), DEV).velocity())
    t_obs = torch.as_tensor(egb.traveltime(*mk(true), spec).cpu().numpy(), device=DEV)
    ts = mk(p.medium)
    for x in ts:
        x.requires_grad_(True)
    t = egb.traveltime(*ts, spec)
    ok = ~(torch.isnan(t) | torch.isnan(t_obs))
    J = torch.sum((t[ok] - t_obs[ok]) ** 2)
    J.backward()
    base = [p.medium.vp0, p.medium.eps, p.medium.delta, p.medium.tilt]
    # smooth directions of each parameter's own scale
    dirs = [W.smooth_field(np.random.default_rng(11 + q), p.grid, 400.0) * sc
            for q, sc in enumerate((p.medium.vp0, 0.05, 0.05, 0.1))]
    for q, name in enumerate(("vp0", "eps", "delta", "tilt")):
        d = np.asarray(dirs[q], dtype=np.float64)
        gd = float(np.sum(ts[q].grad.cpu().numpy() * d))
        # eps, delta and tilt move J a thousand times less than vp0: a larger
        # step keeps the difference above the FP32 march's rounding
        h = 2e-4 if q == 0 else 2e-3
        Js = []
        for sgn in (1, -1):
            pert = [np.asarray(b, dtype=np.float64) for b in base]
            pert[q] = pert[q] + sgn * h * d
            with torch.no_grad():
                tt = egb.traveltime(*[torch.tensor(a, device=DEV) for a in pert], spec)
            Js.append(float(torch.sum((tt[ok] - t_obs[ok]) ** 2)))
        fd = (Js[0] - Js[1]) / (2 * h)
        log(f"  d/d{name}: <g,d> {gd:.6e}  FD {fd:.6e}  rel {abs(fd - gd) / abs(fd):.1e}")
        assert fd == pytest.approx(gd, rel=1e-3)
