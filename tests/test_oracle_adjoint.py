"""Pins of the autograd traveltime-misfit gradient (oracle/adjoint.py):
its forward equals the C oracle's phi1 / psi, and its gradient equals central
differences of the misfit computed by the C oracle at a fixed time step."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import adjoint as AD


def adjoint_problem(n=24, nth=24, nsteps=14, tilt=True):
    L = 480.0
    g = W.Grid(nx=n, nz=n + 4, nth=nth, dx=L / n, dz=L / n)
    rng = W.rng_for(4, 900)
    med = W.vti_medium(rng, g, L, tilt=tilt)
    src = W.Source(xs=0.5 * L + 3.0, zs=0.3 * L, r0=4 * g.dx, beta=1.0 / (2 * L))
    rx = np.stack([np.linspace(0.25 * L, 0.75 * L, 9), np.full(9, 0.72 * L)], axis=1)
    return W.Problem("adj", g, med, src, nsteps, W.hz([20.0])), rx


def c_oracle_misfit(p, rx, t_obs, dt):
    r = oracle.solve(p, dt=dt)
    t = oracle.pick(p.grid, r["U"], rx)
    ok = ~np.isnan(t)
    return float(np.sum((t[ok] - t_obs[ok]) ** 2)), t


def test_torch_forward_equals_c_oracle():
    p, rx = adjoint_problem()
    r = oracle.solve(p)
    m = p.medium
    ts = [torch.tensor(a, dtype=torch.float64) for a in (m.vp0, m.eps, m.delta, m.tilt)]
    J, t, valid, (phi, psi) = AD.misfit(p, ts, rx, np.zeros(len(rx)), r["dt"], p.nsteps)
    assert np.abs(phi.numpy() - r["U"][0]).max() <= 1e-9 * np.abs(r["U"][0]).max()
    assert np.abs(psi.numpy() - r["U"][1]).max() <= 1e-12 * np.abs(r["U"][1]).max()
    to = oracle.pick(p.grid, r["U"], rx)
    assert np.array_equal(valid, ~np.isnan(to))
    assert np.allclose(t.numpy()[valid], to[valid], rtol=1e-12)


def test_gradient_matches_central_differences():
    p, rx = adjoint_problem()
    r = oracle.solve(p)
    dt = r["dt"]
    # observed data from a perturbed model (as the adjoint workload does)
    rng = np.random.default_rng(5)
    true = replace(p.medium, vp0=p.medium.vp0 * 1.03, eps=p.medium.eps + 0.02)
    _, t_obs = c_oracle_misfit(replace(p, medium=true), rx, np.zeros(len(rx)), dt)
    J, grads = AD.gradient(p, rx, t_obs, dt, p.nsteps)
    J0, _ = c_oracle_misfit(p, rx, t_obs, dt)
    assert J == pytest.approx(J0, rel=1e-9)
    names = ("vp0", "eps", "delta", "tilt")
    steps = {"vp0": 1e-3, "eps": 1e-6, "delta": 1e-6, "tilt": 1e-6}
    checked = 0
    for fi, name in enumerate(names):
        gfield = grads[fi]
        # the nodes with the largest sensitivity, plus one in the source region
        idx = np.dstack(np.unravel_index(np.argsort(-np.abs(gfield).ravel())[:3], gfield.shape))[0]
        for (i, j) in idx:
            h = steps[name]
            fd = []
            for sgn in (1, -1):
                arr = getattr(p.medium, name).copy()
                arr[i, j] += sgn * h
                Jp, _ = c_oracle_misfit(replace(p, medium=replace(p.medium, **{name: arr})), rx, t_obs, dt)
                fd.append(Jp)
            fdg = (fd[0] - fd[1]) / (2 * h)
            assert fdg == pytest.approx(gfield[i, j], rel=2e-4, abs=1e-6 * np.abs(gfield).max()), (name, i, j)
            checked += 1
    assert checked == 12
