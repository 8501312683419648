"""Batched march (one persistent, graph-captured launch per stage over a tile
queue spanning uneven grids) against the single-problem march and the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import gpu_planes, log, oracle_planes, rel_err, plane_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_batch(dtype="f32", seeds=(0, 1, 2, 3)):
    probs = []
    for s in seeds:
        rng = W.rng_for(3, 500 + s)
        nx, nz, nth = (int(v) for v in rng.integers(24, 80, size=3))
        L = 1200.0
        g = W.Grid(nx=nx, nz=nz, nth=nth, dx=L / nx, dz=L / nz)
        med = W.vti_medium(rng, g, L, tilt=bool(s % 2))
        src = W.Source(xs=0.5 * L + 7.0 * s, zs=0.45 * L, r0=4 * max(g.dx, g.dz), beta=1.0 / (2 * L))
        probs.append(W.Problem(f"batch{s}", g, med, src, 12, W.hz([20.0]), dtype=dtype))
    return probs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_equals_single_and_oracle(dtype):
    import paper_2006_11945_amd as egb

    probs = small_batch(dtype)
    log("batched " + dtype + ": " + ", ".join(f"{p.grid.nx}x{p.grid.nz}x{p.grid.nth}" for p in probs))
    single, batch = [], []
    for p in probs:
        for lst in (single, batch):
            s = egb.Solver(p, "cuda:0", dtype)
            s.velocity()
            s.init()
            lst.append(s)
    nsteps = probs[0].nsteps
    for s in single:
        s.step(nsteps)
    arr = egb.make_problem_array(batch)
    work = egb.alloc_bytes(egb.workspace_size_batched(arr), "cuda:0")
    egb.egb_liouville_step_batched(arr, nsteps, work)
    torch.cuda.synchronize()
    for a, b in zip(single, batch):
        A, B = gpu_planes(a), gpu_planes(b)
        for k in A:
            assert np.array_equal(A[k], B[k]), k
    # and the first problem against the oracle at its own dt
    o = oracle.solve(probs[0], nsteps=nsteps)
    assert batch[0].dt_cfl == pytest.approx(o["dt"], rel=1e-10)
    G, O = gpu_planes(batch[0]), oracle_planes(o["U"])
    tol = 1e-10 if dtype == "f64" else 1e-5
    for name in O:
        sc = plane_scale(O, name)
        assert rel_err(G[name], O[name], sc) < tol, name


def test_full_size_batch_equals_single_problems():
    """The benchmark's batch (64 independent VTI problems, every axis drawn
    from 128..384, 1.1e9 cells) in its launch configuration: two steps of the
    batched march, then each problem must equal its own single-problem march
    bit for bit (compared on the GPU, one problem at a time), and the
    smallest problem the oracle."""
    import paper_2006_11945_amd as egb

    probs = W.batch_uneven(nprob=64, nsteps=2)
    log("full-size batch: %d problems, %.3g cells" % (len(probs), sum(p.grid.ncell for p in probs)))
    batch = []
    for p in probs:
        s = egb.Solver(p, "cuda:0")
        s.work_step = None  # the batched march brings its own workspace
        s.velocity()
        s.init()
        batch.append(s)
    arr = egb.make_problem_array(batch)
    work = egb.alloc_bytes(egb.workspace_size_batched(arr), "cuda:0")
    egb.egb_liouville_step_batched(arr, 2, work)
    torch.cuda.synchronize()
    del work
    torch.cuda.empty_cache()
    for i, (p, b) in enumerate(zip(probs, batch)):
        s = egb.Solver(p, "cuda:0")
        s.velocity()
        assert s.dt_cfl == b.dt_cfl
        s.init()
        s.step(2)
        torch.cuda.synchronize()
        for k, v in s.planes().items():
            assert torch.equal(v, b.planes()[k]), (i, k)
        del s
    small = min(range(len(probs)), key=lambda i: probs[i].grid.ncell)
    p = probs[small]
    log(f"  oracle on problem {small}: {p.grid.nx}x{p.grid.nz}x{p.grid.nth}")
    o = oracle.solve(p, nsteps=2, dt=batch[small].dt_cfl)
    G, O = gpu_planes(batch[small]), oracle_planes(o["U"])
    for name in O:
        sc = plane_scale(O, name)
        assert rel_err(G[name], O[name], sc) < 1e-5, name
