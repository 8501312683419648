"""The allocation-free beam sum (egb_beam_sum_noalloc, fixed per-device
scratch) against egb_beam_sum with a caller workspace, through the C ABI:
two calls in a row, the second on a smaller grid (the scratch keeps the
first call's contents), each within the wavefield bar of 1e-4 relative L2
per frequency (the same kernels; the record order inside a line list may
differ between calls, which moves FP32 sums by rounding only); a grid too
large for the fixed scratch is refused before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def marched(nx, nz, nth, nsteps, seed):
    import paper_2006_11945_amd as egb

    dx = 15.625
    g = W.Grid(nx=nx, nz=nz, nth=nth, dx=dx, dz=dx)
    L = max(nx, nz) * dx
    med = W.vti_medium(W.rng_for(1, 500 + seed), g, L, tilt=True)
    src = W.Source(xs=0.5 * nx * dx, zs=0.5 * nz * dx, r0=4 * dx, beta=1.0 / (2 * L))
    p = W.Problem("noalloc", g, med, src, nsteps, W.hz([8.0, 20.0, 35.0, 50.0]), dtype="f32")
    s = egb.Solver(p, DEV)
    s.velocity()
    s.init()
    s.step(nsteps)
    return p, s


def test_noalloc_beam_sum_matches_the_workspace_call_twice():
    import paper_2006_11945_amd as egb

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for nx, nz, nth, nsteps, seed in ((56, 80, 48, 30, 0), (36, 44, 32, 20, 1)):
        p, s = marched(nx, nz, nth, nsteps, seed)
        ref = s.beam(p.omegas).double().cpu().numpy()
        out = torch.full((len(p.omegas), nx, nz, 2), float("nan"), dtype=torch.float32, device=DEV)
        egb.egb_beam_sum_noalloc(s.eg, s.coeff2d, s.vel3d, s.src, s.state, p.omegas, out)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        assert np.isfinite(got).all()
        R, Gg = ref[..., 0] + 1j * ref[..., 1], got[..., 0] + 1j * got[..., 1]
        err = [np.linalg.norm(Gg[w] - R[w]) / np.linalg.norm(R[w]) for w in range(len(p.omegas))]
        print(f"{nx}x{nz}x{nth}: rel L2 per frequency {np.array(err)}")
        assert max(err) <= 1e-4
        del s


def test_noalloc_beam_sum_refuses_grids_beyond_its_scratch():
    import paper_2006_11945_amd as egb

    g = W.Grid(nx=5000, nz=5000, nth=8, dx=1.0, dz=1.0)
    eg = egb.make_grid(g, "f32")
    src = egb.EgbSource(10.0, 10.0, 4.0, 1e-4)
    om = (ctypes.c_double * 1)(100.0)
    P = ctypes.c_void_p
    assert egb.lib().egb_beam_scratch_bytes() == 128 << 20
    rc = egb.lib().egb_beam_sum_noalloc(ctypes.byref(eg), P(256), P(256), ctypes.byref(src), P(256), om, 1, P(256),
                                        None)
    assert rc == egb.EGB_EUNSUPPORTED
