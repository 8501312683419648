"""The forward stage and the reverse (adjoint) stage split the (tile, x) work
of a grid into one contiguous range per block, and a range may start or end
anywhere inside a tile.  The results must not depend on that split: the same
march and the same misfit gradient computed with different block counts are
bit-identical (block counts forced through the tuning overrides)."""
import os

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import gpu_planes, log
from tests.test_gpu_adjoint import adjoint_problem, gpu_gradient
from tests.test_gpu_parity import ragged_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def with_env(name, value, fn):
    old = os.environ.get(name)
    os.environ[name] = str(value)
    try:
        return fn()
    finally:
        if old is None:
            del os.environ[name]
        else:
            os.environ[name] = old


def forward_planes(p, dtype, nsteps):
    import paper_2006_11945_amd as egb
    s = egb.Solver(p, DEV, dtype)
    s.velocity()
    s.init()
    s.step(nsteps)
    torch.cuda.synchronize()
    return gpu_planes(s)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_forward_independent_of_block_split(dtype):
    # 42 x 72 x 36: two z tiles (one ragged), ragged theta tiles, 42 x steps
    p = ragged_problem(dtype=dtype, tilt=True)
    ref = forward_planes(p, dtype, 6)
    for G in (1, 3, 17, 64, 10000):
        log(f"forward {dtype}: {G} blocks")
        got = with_env("EGB_STAGE_GRID", G, lambda: forward_planes(p, dtype, 6))
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (G, k)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adjoint_independent_of_block_split(dtype):
    p, rx = adjoint_problem(nsteps=8)
    r = oracle.solve(p)
    t_obs = oracle.pick(p.grid, r["U"], rx) * 1.01
    J0, g0, _ = gpu_gradient(p, rx, t_obs, dtype, r["dt"])
    assert J0 > 0
    for G in (1, 5, 144, 10000):
        log(f"adjoint {dtype}: {G} blocks")
        J, g, _ = with_env("EGB_ADJ_GRID", G, lambda: gpu_gradient(p, rx, t_obs, dtype, r["dt"]))
        assert J == J0
        for a, b in zip(g0, g):
            assert np.array_equal(a, b), G
