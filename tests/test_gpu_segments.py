"""The forward stage and the reverse (adjoint) stage split the (tile, x) work
of a grid into one contiguous range per block, and a range may start or end
anywhere inside a tile.  The results must not depend on that split: the same
march and the same misfit gradient computed with different block counts are
bit-identical (block counts fixed through egb_set_blocks).  The autotuner
picks one of those counts by timing: tuning leaves the state unchanged and
a tuned march equals the default one bit for bit."""
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


def with_blocks(grid, dtype, ops, blocks, fn):
    """Run fn with `blocks` per launch for the given operations on grids of
    this shape, then restore the default."""
    import paper_2006_11945_amd as egb
    eg = egb.make_grid(grid, dtype)
    for op in ops:
        egb.egb_set_blocks(eg, op, blocks)
        assert egb.egb_get_blocks(eg, op) == blocks
    try:
        return fn()
    finally:
        for op in ops:
            egb.egb_set_blocks(eg, op, 0)


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
        got = with_blocks(p.grid, dtype, (0,), G, lambda: forward_planes(p, dtype, 6))
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
        J, g, _ = with_blocks(p.grid, dtype, (1, 2), G, lambda: gpu_gradient(p, rx, t_obs, dtype, r["dt"]))
        assert J == J0
        for a, b in zip(g0, g):
            assert np.array_equal(a, b), G


@pytest.mark.parametrize("dtype,op", [("f32", 0), ("f64", 0), ("f32", 1)])
def test_autotuned_march_equals_default(dtype, op):
    import paper_2006_11945_amd as egb
    p = ragged_problem(dtype=dtype, tilt=True)
    ref = egb.Solver(p, DEV, dtype)
    ref.velocity()
    ref.init()
    s = egb.Solver(p, DEV, dtype)
    s.velocity()
    s.init()
    before = {k: v.clone() for k, v in s.planes().items()}
    try:
        b = s.tune(op=op, reps=2)
        torch.cuda.synchronize()
        log(f"tuned {dtype} op {op}: {b} blocks")
        assert b >= 1 and egb.egb_get_blocks(s.eg, op) == b
        for k, v in s.planes().items():  # tuning leaves the state as it was
            assert torch.equal(v, before[k]), k
        step = s.step if op == 0 else s.step_kinematic
        step(5)
    finally:
        egb.egb_set_blocks(s.eg, op, 0)
    (ref.step if op == 0 else ref.step_kinematic)(5)
    torch.cuda.synchronize()
    A, B = gpu_planes(ref), gpu_planes(s)
    for k in A:
        assert np.array_equal(A[k], B[k]), k


def test_autotuned_batch_equals_default():
    import paper_2006_11945_amd as egb
    from tests.test_gpu_batched import small_batch
    probs = small_batch("f32", seeds=(4, 5, 6))
    runs = []
    for tuned in (False, True):
        ss = []
        for p in probs:
            s = egb.Solver(p, DEV, "f32")
            s.velocity()
            s.init()
            ss.append(s)
        arr = egb.make_problem_array(ss)
        work = egb.alloc_bytes(egb.workspace_size_batched(arr), DEV)
        if tuned:
            before = [gpu_planes(s) for s in ss]
            b = egb.egb_tune_batched(arr, work, reps=2)
            log(f"tuned batch: {b} blocks")
            assert b >= 1
            for s, bp in zip(ss, before):
                after = gpu_planes(s)
                assert all(np.array_equal(after[k], bp[k]) for k in bp)
        try:
            egb.egb_liouville_step_batched(arr, 6, work)
        finally:
            egb.egb_set_blocks_batched(arr, 0)
        torch.cuda.synchronize()
        runs.append([gpu_planes(s) for s in ss])
    for A, B in zip(*runs):
        for k in A:
            assert np.array_equal(A[k], B[k]), k


def with_launch(grid, dtype, op, tile_rows, blocks, fn):
    """Run fn with a fixed launch (tile shape, blocks) for op, then restore the default."""
    import paper_2006_11945_amd as egb
    eg = egb.make_grid(grid, dtype)
    egb.egb_set_launch(eg, op, tile_rows, blocks)
    assert egb.egb_get_launch(eg, op) == (tile_rows, blocks)
    try:
        return fn()
    finally:
        egb.egb_set_launch(eg, op, 0, 0)


@pytest.mark.parametrize("op", [0, 1])
def test_march_independent_of_tile_shape(op):
    """Every tile shape the autotuner may pick (theta rows per tile, with its
    LDS slice, halo and waves per SIMD) gives the default march bit for bit,
    at the default block count and at an odd one."""
    import paper_2006_11945_amd as egb
    p = ragged_problem(dtype="f32", tilt=True)
    eg = egb.make_grid(p.grid, "f32")
    rows = egb.egb_tile_rows(eg, op)
    assert len(rows) >= 2

    def march():
        s = egb.Solver(p, DEV, "f32")
        s.velocity()
        s.init()
        (s.step if op == 0 else s.step_kinematic)(6)
        torch.cuda.synchronize()
        return gpu_planes(s)

    ref = march()
    for tk in rows:
        for G in (0, 19):
            log(f"op {op}: {tk} theta rows per tile, blocks {G or 'default'}")
            got = with_launch(p.grid, "f32", op, tk, G, march)
            for k in ref:
                assert np.array_equal(ref[k], got[k]), (tk, G, k)


def test_batch_independent_of_tile_shape():
    import paper_2006_11945_amd as egb
    from tests.test_gpu_batched import small_batch
    probs = small_batch("f32", seeds=(7, 8, 9))
    runs = []
    rows = None
    for tk in (None, 12, 8, 16):
        ss = []
        for p in probs:
            s = egb.Solver(p, DEV, "f32")
            s.velocity()
            s.init()
            ss.append(s)
        arr = egb.make_problem_array(ss)
        work = egb.alloc_bytes(egb.workspace_size_batched(arr), DEV)
        if rows is None:
            rows = egb.egb_tile_rows(ss[0].eg, 0)
        if tk is not None:
            assert tk in rows
            egb.egb_set_launch_batched(arr, tk, 0)
            assert egb.egb_get_launch_batched(arr) == (tk, 0)
        try:
            egb.egb_liouville_step_batched(arr, 5, work)
        finally:
            egb.egb_set_launch_batched(arr, 0, 0)
        torch.cuda.synchronize()
        runs.append([gpu_planes(s) for s in ss])
        log(f"batch with {tk or 'default'} theta rows per tile")
    for other in runs[1:]:
        for A, B in zip(runs[0], other):
            for k in A:
                assert np.array_equal(A[k], B[k]), k


def test_tuned_launch_shape_is_reported():
    import paper_2006_11945_amd as egb
    p = ragged_problem(dtype="f32", tilt=True)
    s = egb.Solver(p, DEV, "f32")
    s.velocity()
    s.init()
    try:
        b = s.tune(op=0, reps=2)
        tk, blocks = egb.egb_get_launch(s.eg, 0)
        log(f"tuned: {tk} theta rows per tile, {blocks} blocks")
        assert blocks == b and tk in egb.egb_tile_rows(s.eg, 0)
    finally:
        egb.egb_set_launch(s.eg, 0, 0, 0)


def test_tti_512_full_size_march_independent_of_launch_shape():
    """At the 512^3 TTI workload's full size: the launch shape the autotuner
    picks (as the benchmark does), and other tile shapes and block counts,
    give bit-identical states after 3 RK3 steps (all seven planes), with
    every value finite."""
    import paper_2006_11945_amd as egb
    import workloads as W
    p = W.tti_512(nsteps=3)
    eg = egb.make_grid(p.grid, "f32")
    rows = egb.egb_tile_rows(eg, 0)

    def march(shape):
        s = egb.Solver(p, DEV, "f32")
        s.velocity()
        s.init()
        try:
            if shape == "tuned":
                s.tune(op=0, reps=1)
            else:
                egb.egb_set_launch(s.eg, 0, *shape)
            used = egb.egb_get_launch(s.eg, 0)
            s.step(p.nsteps)
        finally:
            egb.egb_set_launch(s.eg, 0, 0, 0)
        torch.cuda.synchronize()
        out = {k: v.clone() for k, v in s.planes().items()}
        del s
        torch.cuda.empty_cache()
        return used, out

    used, ref = march("tuned")
    log(f"TTI 512^3: tuned launch {used[0]} theta rows per tile, {used[1]} blocks")
    for k, v in ref.items():
        assert bool(torch.isfinite(v).all()), k
    shapes = [(r, b) for r, b in ((rows[0], 97), (rows[-1], 4096)) if (r, b) != tuple(used)]
    for shape in shapes:
        got_used, got = march(shape)
        log(f"  {got_used[0]} theta rows per tile, {got_used[1]} blocks")
        for k in ref:
            assert torch.equal(ref[k], got[k]), (shape, k)
        del got
