"""The C-ABI library loads and exports every symbol include/egb.h declares.

CPU only: only host-side size queries and argument validation are called
(they return before any HIP call).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "egb.h")
LIB = os.path.join(ROOT, "paper_2006_11945_amd", "libegb.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(egb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libegb.so not built (run python paper_2006_11945_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 10
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_sizes_and_validation_without_gpu():
    import numpy as np
    import paper_2006_11945_amd as egb
    import workloads as W

    g = W.Grid(nx=40, nz=72, nth=36, dx=10.0, dz=10.0)
    eg = egb.make_grid(g, "f32")
    n = 40 * 72 * 36
    st = egb.plane_stride(eg)
    assert st >= n and st % 64 == 0
    assert egb.state_bytes(eg) == 6 * st * 4 + st * 8
    assert egb.state_plane_offset(eg, egb.EGB_PHASE) == 5 * st * 4
    assert egb.state_plane_offset(eg, egb.EGB_PSI) == 6 * st * 4
    assert egb.vel3d_bytes(eg) == 7 * st * 4
    assert egb.coeff2d_bytes(eg) == 30 * 40 * 72 * 8
    assert egb.workspace_size(eg, egb.EGB_OP_STEP) >= 2 * egb.state_bytes(eg)
    eg64 = egb.make_grid(g, "f64")
    assert egb.state_bytes(eg64) == 7 * st * 8
    # invalid grids give zero sizes and EINVAL before any device work
    bad = egb.EgbGrid(4, 72, 36, 0, 0.0, 0.0, 10.0, 10.0)
    assert egb.state_bytes(bad) == 0
    L = egb.lib()
    src = egb.EgbSource(1.0, 1.0, 1.0, 1e-4)
    assert L.egb_init_state(ctypes.byref(bad), None, ctypes.byref(src), None, None) == egb.EGB_EINVAL
    assert L.egb_init_state(None, None, None, None, None) == egb.EGB_EINVAL
    P = ctypes.c_void_p
    # the fake velocity buffer at 256 gets a CFL limit (as egb_hamiltonian_velocity would record it)
    assert L.egb_declare_velocity(ctypes.byref(eg), P(256), 1e-3) == egb.EGB_OK
    assert L.egb_liouville_step(ctypes.byref(eg), P(256), ctypes.byref(src), P(256), P(256), P(256), 1 << 30, -1.0,
                                1, None) == egb.EGB_ECFL
    assert L.egb_liouville_step(ctypes.byref(eg), P(256), ctypes.byref(src), P(256), P(256), P(256), 16, 1e-3, 1,
                                None) == egb.EGB_EWORKSPACE
    assert L.egb_liouville_step(ctypes.byref(eg), P(258), ctypes.byref(src), P(256), P(256), P(256), 1 << 30, 1e-3,
                                1, None) == egb.EGB_EINVAL
    # the boundary data is required and aligned
    assert L.egb_liouville_step(ctypes.byref(eg), P(256), ctypes.byref(src), None, P(256), P(256), 1 << 30, 1e-3, 1,
                                None) == egb.EGB_EINVAL
    assert L.egb_liouville_step(ctypes.byref(eg), P(256), ctypes.byref(src), P(264), P(256), P(256), 1 << 30, 1e-3,
                                1, None) == egb.EGB_EINVAL
    assert L.egb_boundary_data(ctypes.byref(eg), None, P(256), None) == egb.EGB_EINVAL
    bs = egb.bdata_plane_stride(eg)
    assert bs >= 36 * 6 * (40 + 72) and bs % 64 == 0
    assert egb.bdata_bytes(eg) == 6 * bs * 4 + bs * 8
    assert egb.bdata_bytes(eg64) == 7 * bs * 8
    assert egb.bfold_bytes(eg) == 2 * 36 * 12 * (40 + 72) * 8
    badlin = egb.EgbSource(1.0, 1.0, 1.0, 1e-4, 7)  # no such linear-phase variant
    assert L.egb_init_state(ctypes.byref(eg), ctypes.c_void_p(256), ctypes.byref(badlin), ctypes.c_void_p(256),
                            None) == egb.EGB_EINVAL
    nosrc = egb.EgbSource(1.0, 1.0, 1.0, 0.0)  # beta must be > 0
    assert L.egb_init_state(ctypes.byref(eg), ctypes.c_void_p(256), ctypes.byref(nosrc), ctypes.c_void_p(256),
                            None) == egb.EGB_EINVAL
    om = np.array([-1.0])
    assert L.egb_beam_sum(ctypes.byref(eg), ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.byref(src),
                          ctypes.c_void_p(256), om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1,
                          ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 30, None) == egb.EGB_EINVAL
    assert L.egb_pick_receivers(ctypes.byref(eg), ctypes.c_void_p(256), None, 0, None, None) == egb.EGB_OK
    assert egb.lib().egb_status_string(-3) == b"workspace too small"


def test_time_step_above_the_cfl_limit_is_refused_before_any_launch():
    """A step above the CFL limit recorded for the velocity buffer
    (dt > dt_cfl (1 + 1e-12)) returns EGB_ECFL from every marching call,
    a buffer without a record (or recorded for another grid) EGB_EINVAL;
    both before any device call, so they run here without a GPU (a call
    that passed the checks would fail at its first launch with EGB_EHIP,
    or at the workspace check with EGB_EWORKSPACE)."""
    import paper_2006_11945_amd as egb
    import workloads as W

    L = egb.lib()
    P = ctypes.c_void_p
    eg = egb.make_grid(W.Grid(nx=40, nz=72, nth=36, dx=10.0, dz=10.0), "f32")
    other = egb.make_grid(W.Grid(nx=40, nz=72, nth=40, dx=10.0, dz=10.0), "f32")
    src = egb.EgbSource(200.0, 300.0, 40.0, 1e-4)
    vel, unknown = 4096 * 1024, 4096 * 2048
    lim = 2.5e-3
    assert L.egb_declare_velocity(ctypes.byref(eg), P(vel), lim) == egb.EGB_OK
    out = ctypes.c_double(0.0)
    assert L.egb_velocity_dt_cfl(ctypes.byref(eg), P(vel), ctypes.byref(out)) == egb.EGB_OK and out.value == lim
    assert L.egb_velocity_dt_cfl(ctypes.byref(other), P(vel), ctypes.byref(out)) == egb.EGB_EINVAL
    assert L.egb_declare_velocity(ctypes.byref(eg), P(vel + 4), lim) == egb.EGB_EINVAL  # misaligned
    assert L.egb_declare_velocity(ctypes.byref(eg), P(vel), -1.0) == egb.EGB_EINVAL
    over, ok_dt = lim * (1 + 1e-9), lim * (1 + 1e-13)

    def step(fn, g, v, dt, work_bytes=16):
        return fn(ctypes.byref(g), P(v), ctypes.byref(src), P(256), P(256), P(256), work_bytes, dt, 1, None)

    for fn in (L.egb_liouville_step, L.egb_liouville_step_kinematic):
        assert step(fn, eg, vel, over) == egb.EGB_ECFL
        assert step(fn, eg, vel, ok_dt) == egb.EGB_EWORKSPACE  # the CFL check passed
        assert step(fn, eg, unknown, ok_dt) == egb.EGB_EINVAL
        assert step(fn, other, vel, ok_dt) == egb.EGB_EINVAL
    adj = lambda v, dt: L.egb_adjoint_step(ctypes.byref(eg), P(v), ctypes.byref(src), P(256), P(512), P(768),
                                           P(1024), P(1280), P(1536), 16, dt, None)
    assert adj(vel, over) == egb.EGB_ECFL
    assert adj(vel, ok_dt) == egb.EGB_EWORKSPACE
    assert adj(unknown, ok_dt) == egb.EGB_EINVAL
    b = ctypes.c_int32(0)
    tune = lambda dt: L.egb_tune_step(ctypes.byref(eg), P(vel), ctypes.byref(src), P(256), P(256), P(256), 16, dt,
                                      egb.EGB_TUNE_STEP, 3, None, ctypes.byref(b))
    assert tune(over) == egb.EGB_ECFL
    assert tune(ok_dt) == egb.EGB_EWORKSPACE
    probs = (egb.EgbProblem * 2)()
    probs[0] = egb.EgbProblem(eg, vel, src, 256, 256, ok_dt)
    probs[1] = egb.EgbProblem(eg, vel, src, 256, 256, over)
    assert L.egb_liouville_step_batched(probs, 2, 1, P(256), 16, None) == egb.EGB_ECFL
    probs[1] = egb.EgbProblem(eg, unknown, src, 256, 256, ok_dt)
    assert L.egb_liouville_step_batched(probs, 2, 1, P(256), 16, None) == egb.EGB_EINVAL
    probs[1] = egb.EgbProblem(eg, vel, src, 256, 256, ok_dt)
    assert L.egb_liouville_step_batched(probs, 2, 1, P(256), 16, None) == egb.EGB_EWORKSPACE


def test_grids_beyond_32_bit_offsets_are_refused_before_any_launch():
    """The stage kernels address every array with 32-bit byte offsets: a
    1024^3 FP32 grid (a 30 GB state) is a valid request the library does not
    implement.  Host-side validation only (fake aligned device pointers)."""
    import paper_2006_11945_amd as egb
    import workloads as W

    g = W.Grid(nx=1024, nz=1024, nth=1024, dx=10.0, dz=10.0)
    eg = egb.make_grid(g, "f32")
    assert egb.state_bytes(eg) > 1 << 32
    src = egb.EgbSource(5000.0, 5000.0, 40.0, 1e-4)
    P = ctypes.c_void_p
    assert egb.lib().egb_declare_velocity(ctypes.byref(eg), P(256), 1e-3) == egb.EGB_OK
    rc = egb.lib().egb_liouville_step(ctypes.byref(eg), P(256), ctypes.byref(src), P(256), P(256), P(256),
                                      1 << 62, 1e-3, 1, None)
    assert rc == egb.EGB_EUNSUPPORTED


def test_paraxial_levels_beyond_32_bit_offsets_are_refused():
    """The paraxial stage kernel uses 32-bit element offsets within a level:
    a slice whose level reaches 2 GiB is refused before any launch."""
    import paper_2006_11945_amd as egb
    import workloads as W

    g = W.Grid(nx=8192, nz=8, nth=8192, dx=10.0, dz=10.0)
    eg = egb.make_grid(g, "f32")
    assert egb.paraxial_level_bytes(eg) >= 1 << 31
    P = ctypes.c_void_p
    rc = egb.lib().egb_paraxial_march(ctypes.byref(eg), P(256), 1.0, 2, P(256), P(256), 1 << 62, None)
    assert rc == egb.EGB_EUNSUPPORTED


def test_launch_tuning_arguments_are_validated_before_any_device_call():
    import paper_2006_11945_amd as egb
    import workloads as W

    g = W.Grid(nx=40, nz=72, nth=36, dx=10.0, dz=10.0)
    eg = egb.make_grid(g, "f32")
    bad = egb.EgbGrid(4, 72, 36, 0, 0.0, 0.0, 10.0, 10.0)
    L = egb.lib()
    P = ctypes.c_void_p
    for op, blocks in ((3, 1), (-1, 1), (egb.EGB_TUNE_STEP, -1)):
        assert L.egb_set_blocks(ctypes.byref(eg), op, blocks) == egb.EGB_EINVAL
    assert L.egb_set_blocks(ctypes.byref(bad), egb.EGB_TUNE_STEP, 8) == egb.EGB_EINVAL
    assert L.egb_get_blocks(ctypes.byref(bad), egb.EGB_TUNE_STEP) == 0
    assert L.egb_get_blocks(ctypes.byref(eg), 9) == 0
    src = egb.EgbSource(1.0, 1.0, 1.0, 1e-4)
    out = ctypes.c_int32(0)
    assert L.egb_declare_velocity(ctypes.byref(eg), P(256), 1e-3) == egb.EGB_OK
    args = (ctypes.byref(eg), P(256), ctypes.byref(src), P(256), P(256), P(256), 1 << 30, 1e-3)
    # the reverse stages cannot be timed without side effects: set only
    assert L.egb_tune_step(*args, egb.EGB_TUNE_ADJOINT, 3, None, ctypes.byref(out)) == egb.EGB_EINVAL
    assert L.egb_tune_step(*args, egb.EGB_TUNE_STEP, 0, None, ctypes.byref(out)) == egb.EGB_EINVAL
    assert L.egb_tune_step(*args, egb.EGB_TUNE_STEP, 3, None, None) == egb.EGB_EINVAL
    assert L.egb_tune_step(ctypes.byref(eg), P(256), ctypes.byref(src), P(256), P(256), P(256), 16, 1e-3,
                           egb.EGB_TUNE_STEP, 3, None, ctypes.byref(out)) == egb.EGB_EWORKSPACE
    assert L.egb_tune_batched(None, 0, P(256), 1 << 30, 3, None, ctypes.byref(out)) == egb.EGB_EINVAL
    assert L.egb_set_blocks_batched(None, 1, 4) == egb.EGB_EINVAL


def test_launch_shapes_are_listed_and_validated_without_gpu():
    """Tile heights per operation and dtype; a tile height the operation
    does not have, or a negative count, is refused before any device call."""
    import paper_2006_11945_amd as egb
    import workloads as W

    g = W.Grid(nx=40, nz=72, nth=36, dx=10.0, dz=10.0)
    e32, e64 = egb.make_grid(g, "f32"), egb.make_grid(g, "f64")
    assert egb.egb_tile_rows(e32, egb.EGB_TUNE_STEP) == [12, 8, 16]
    assert egb.egb_tile_rows(e32, egb.EGB_TUNE_KINEMATIC) == [16, 8, 12]
    assert egb.egb_tile_rows(e64, egb.EGB_TUNE_STEP) == [8]
    assert egb.egb_tile_rows(e32, egb.EGB_TUNE_ADJOINT) == [8]
    assert egb.egb_tile_rows(e32, 7) == []
    L = egb.lib()
    for rows, blocks in ((10, 0), (12, -1), (16, 0)):
        eg = e64 if rows == 16 else e32
        l = egb.EgbLaunch(rows, blocks)
        assert L.egb_set_launch(ctypes.byref(eg), egb.EGB_TUNE_STEP, ctypes.byref(l)) == egb.EGB_EINVAL
    assert L.egb_get_launch(ctypes.byref(e32), egb.EGB_TUNE_STEP, None) == egb.EGB_EINVAL


def test_header_compiles_as_c(tmp_path):
    """include/egb.h is a C header: a C99 translation unit that includes it
    (and calls nothing) compiles without a warning from the header."""
    import shutil
    import subprocess

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "uses_egb.c"
    src.write_text('#include "egb.h"\nint main(void) { egb_grid g; (void)g; return (int)EGB_TUNE_STEP; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-fsyntax-only", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "egb.h" not in r.stderr, r.stderr


def test_paraxial_drt_variant_is_validated():
    import paper_2006_11945_amd as egb
    import workloads as W

    eg = egb.make_grid(W.Grid(nx=40, nz=16, nth=36, dx=10.0, dz=10.0), "f32")
    P = ctypes.c_void_p
    L = egb.lib()
    rate = ctypes.c_double(0.0)
    assert L.egb_paraxial_velocity(ctypes.byref(eg), P(256), 1.0, 2, P(256), ctypes.byref(rate), P(256), 1 << 30,
                                   None) == egb.EGB_EINVAL
    assert L.egb_paraxial_init(ctypes.byref(eg), P(256), 1.0, 1e-4, -1, P(256), None) == egb.EGB_EINVAL
    om = (ctypes.c_double * 1)(100.0)
    assert L.egb_paraxial_beam_sum(ctypes.byref(eg), P(256), P(256), 1.0, 200.0, 0, 5, -1, om, 1, P(256), P(256),
                                   1 << 30, None) == egb.EGB_EINVAL


def test_migration_arguments_are_validated():
    import paper_2006_11945_amd as egb
    import workloads as W

    eg = egb.make_grid(W.Grid(nx=40, nz=16, nth=36, dx=10.0, dz=10.0), "f32")
    P = ctypes.c_void_p
    L = egb.lib()
    om = (ctypes.c_double * 2)(100.0, 200.0)
    bad = (ctypes.c_double * 2)(100.0, -1.0)
    big = 1 << 40
    assert L.egb_born_data(ctypes.byref(eg), P(256), 65, om, 2, P(256), P(256), P(256), big, None) == egb.EGB_EUNSUPPORTED
    assert L.egb_born_data(ctypes.byref(eg), P(256), 0, om, 2, P(256), P(256), P(256), big, None) == egb.EGB_EINVAL
    assert L.egb_born_data(ctypes.byref(eg), P(256), 4, bad, 2, P(256), P(256), P(256), big, None) == egb.EGB_EINVAL
    assert L.egb_born_data(ctypes.byref(eg), P(256), 4, om, 2, P(256), P(256), None, big, None) == egb.EGB_EINVAL
    # frequencies are a grid dimension of the split kernel: at most 65535
    assert L.egb_born_data(ctypes.byref(eg), P(256), 4, om, 70000, P(256), P(256), P(256), big, None) == egb.EGB_EUNSUPPORTED
    # the workspace: partial sums of the split over image points
    nb = egb.egb_born_workspace_size(eg, 4, 2)
    assert nb > 0 and nb % (4 * 4 * 2 * 2 * 8) == 0
    assert egb.egb_born_workspace_size(eg, 65, 2) == 0 and egb.egb_born_workspace_size(eg, 4, 0) == 0
    assert L.egb_born_data(ctypes.byref(eg), P(256), 4, om, 2, P(256), P(256), P(256), nb - 1, None) == egb.EGB_EWORKSPACE
    assert L.egb_migrate(ctypes.byref(eg), P(256), 4, om, 2, P(256), None, None) == egb.EGB_EINVAL
    assert L.egb_migrate(ctypes.byref(eg), P(260), 4, om, 2, P(256), P(256), None) == egb.EGB_EINVAL
