"""Python binding of libegb, the MI355X Eulerian Gaussian beam library.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/egb.h``.  PyTorch supplies device
memory and streams.  Importing this package fails loudly when ``libegb.so``
has not been built; there is no CPU fallback.

The functions named ``egb_*`` mirror the C entry points one to one.  The
``Solver`` helper strings them together for one source: medium table and
velocity, point-source data, the march, the beam sum and the receiver pick.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libegb.so")

EGB_OK, EGB_EINVAL, EGB_ECFL, EGB_EWORKSPACE, EGB_EHIP, EGB_ENONFINITE, EGB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
EGB_F32, EGB_F64 = 0, 1
EGB_PHI1, EGB_RE_C, EGB_IM_C, EGB_RE_B, EGB_IM_B, EGB_PHASE, EGB_PSI = range(7)
EGB_OP_VELOCITY, EGB_OP_STEP, EGB_OP_BEAM, EGB_OP_ADJOINT, EGB_OP_PARAXIAL, EGB_OP_PBEAM = range(6)
STATE_PLANES = ("phi1", "ReC", "ImC", "ReB", "ImB", "phase", "psi")
VEL_PLANES = ("Vx", "Vz", "Vt", "A11", "A12", "A21", "A22")
PAR_PLANES = ("X", "vartheta", "ReC", "ImC", "ReB", "ImB", "phase", "tau")   # paraxial level planes, in memory order
PVEL_PLANES = ("u", "w", "Stau", "A11", "A12", "A21", "A22")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2006_11945_amd/build.py`; "
                      "there is no CPU fallback")


class EgbGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nz", ctypes.c_int32), ("nth", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("x0", ctypes.c_double), ("z0", ctypes.c_double), ("dx", ctypes.c_double), ("dz", ctypes.c_double)]


class EgbMedium(ctypes.Structure):
    _fields_ = [("vp0", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("delta", ctypes.c_void_p),
                ("tilt", ctypes.c_void_p), ("vs_ratio", ctypes.c_double)]


class EgbSource(ctypes.Structure):
    _fields_ = [("xs", ctypes.c_double), ("zs", ctypes.c_double), ("r0", ctypes.c_double), ("beta", ctypes.c_double),
                ("lin_variant", ctypes.c_int32)]


class EgbProblem(ctypes.Structure):
    _fields_ = [("grid", EgbGrid), ("vel3d", ctypes.c_void_p), ("src", EgbSource), ("bdata", ctypes.c_void_p),
                ("state", ctypes.c_void_p), ("dt", ctypes.c_double)]


class EgbLaunch(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("blocks", ctypes.c_int32)]


class EgbError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status} ({_lib.egb_status_string(status).decode()})")
        self.status = status


def _load():
    L = ctypes.CDLL(LIB_PATH)
    G, M, S = ctypes.POINTER(EgbGrid), ctypes.POINTER(EgbMedium), ctypes.POINTER(EgbSource)
    vp, sz, i32, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("egb_plane_stride", "egb_coeff2d_bytes", "egb_vel3d_bytes", "egb_state_bytes", "egb_bdata_bytes",
                 "egb_bdata_plane_stride", "egb_bfold_bytes", "egb_paraxial_plane_stride", "egb_paraxial_level_bytes",
                 "egb_paraxial_vel_bytes"):
        getattr(L, name).argtypes = [G]
        getattr(L, name).restype = sz
    L.egb_state_plane_offset.argtypes = [G, i32]; L.egb_state_plane_offset.restype = sz
    L.egb_workspace_size.argtypes = [G, i32]; L.egb_workspace_size.restype = sz
    L.egb_hamiltonian_velocity.argtypes = [G, M, vp, vp, dp, vp, sz, vp]
    L.egb_init_state.argtypes = [G, vp, S, vp, vp]
    L.egb_velocity_dt_cfl.argtypes = [G, vp, dp]
    L.egb_declare_velocity.argtypes = [G, vp, d]
    L.egb_boundary_data.argtypes = [G, vp, vp, vp]
    L.egb_liouville_step.argtypes = [G, vp, S, vp, vp, vp, sz, d, i32, vp]
    L.egb_beam_sum.argtypes = [G, vp, vp, S, vp, dp, i32, vp, vp, sz, vp]
    L.egb_beam_sum_noalloc.argtypes = [G, vp, vp, S, vp, dp, i32, vp, vp]
    L.egb_beam_sum_noalloc.restype = ctypes.c_int
    L.egb_beam_scratch_bytes.argtypes = []
    L.egb_beam_scratch_bytes.restype = sz
    L.egb_pick_receivers.argtypes = [G, vp, vp, i32, vp, vp]
    L.egb_gvel_bytes.argtypes = [G]; L.egb_gvel_bytes.restype = sz
    L.egb_liouville_step_kinematic.argtypes = [G, vp, S, vp, vp, vp, sz, d, i32, vp]
    L.egb_pick_adjoint.argtypes = [G, vp, vp, i32, vp, vp, vp]
    L.egb_adjoint_step.argtypes = [G, vp, S, vp, vp, vp, vp, vp, vp, sz, d, vp]
    L.egb_adjoint_medium.argtypes = [G, M, vp, S, vp, vp, vp, vp, vp, sz, vp]
    for name in ("egb_liouville_step_kinematic", "egb_pick_adjoint", "egb_adjoint_step", "egb_adjoint_medium"):
        getattr(L, name).restype = ctypes.c_int
    P = ctypes.POINTER(EgbProblem)
    L.egb_workspace_size_batched.argtypes = [P, i32]; L.egb_workspace_size_batched.restype = sz
    L.egb_liouville_step_batched.argtypes = [P, i32, i32, vp, sz, vp]
    L.egb_liouville_step_batched.restype = ctypes.c_int
    for name in ("egb_hamiltonian_velocity", "egb_init_state", "egb_boundary_data", "egb_liouville_step",
                 "egb_beam_sum", "egb_pick_receivers", "egb_velocity_dt_cfl", "egb_declare_velocity"):
        getattr(L, name).restype = ctypes.c_int
    L.egb_medium_table.argtypes = [G, M, vp, vp]
    L.egb_paraxial_velocity.argtypes = [G, vp, d, i32, vp, dp, vp, sz, vp]
    L.egb_paraxial_init.argtypes = [G, vp, d, d, i32, vp, vp]
    L.egb_paraxial_march.argtypes = [G, vp, d, i32, vp, vp, sz, vp]
    L.egb_paraxial_pick.argtypes = [G, vp, d, vp, i32, vp, vp]
    L.egb_paraxial_beam_sum.argtypes = [G, vp, vp, d, d, i32, i32, i32, dp, i32, vp, vp, sz, vp]
    for name in ("egb_medium_table", "egb_paraxial_velocity", "egb_paraxial_init", "egb_paraxial_march",
                 "egb_paraxial_pick", "egb_paraxial_beam_sum"):
        getattr(L, name).restype = ctypes.c_int
    L.egb_born_data.argtypes = [G, vp, i32, dp, i32, vp, vp, vp, sz, vp]
    L.egb_born_workspace_size.argtypes = [G, i32, i32]
    L.egb_born_workspace_size.restype = ctypes.c_size_t
    L.egb_migrate.argtypes = [G, vp, i32, dp, i32, vp, vp, vp]
    L.egb_born_data.restype = ctypes.c_int
    L.egb_migrate.restype = ctypes.c_int
    L.egb_get_blocks.argtypes = [G, i32]; L.egb_get_blocks.restype = i32
    L.egb_set_blocks.argtypes = [G, i32, i32]
    L.egb_tune_step.argtypes = [G, vp, S, vp, vp, vp, sz, d, i32, i32, vp, ctypes.POINTER(i32)]
    L.egb_tune_batched.argtypes = [P, i32, vp, sz, i32, vp, ctypes.POINTER(i32)]
    L.egb_set_blocks_batched.argtypes = [P, i32, i32]
    LP = ctypes.POINTER(EgbLaunch)
    L.egb_tile_rows.argtypes = [G, i32, ctypes.POINTER(i32)]
    L.egb_tile_rows.restype = i32
    L.egb_get_launch.argtypes = [G, i32, LP]
    L.egb_set_launch.argtypes = [G, i32, LP]
    L.egb_get_launch_batched.argtypes = [P, i32, LP]
    L.egb_set_launch_batched.argtypes = [P, i32, LP]
    for name in ("egb_set_blocks", "egb_tune_step", "egb_tune_batched", "egb_set_blocks_batched", "egb_get_launch",
                 "egb_set_launch", "egb_get_launch_batched", "egb_set_launch_batched"):
        getattr(L, name).restype = ctypes.c_int
    L.egb_status_string.argtypes = [i32]; L.egb_status_string.restype = ctypes.c_char_p
    return L


_lib = _load()


def lib():
    return _lib


def _check(fn: str, rc: int):
    if rc != EGB_OK:
        raise EgbError(fn, rc)


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ structs
def make_grid(g, dtype: str = "f32") -> EgbGrid:
    """egb_grid from a workloads.Grid-like object (nx, nz, nth, x0, z0, dx, dz)."""
    return EgbGrid(g.nx, g.nz, g.nth, EGB_F64 if dtype == "f64" else EGB_F32, g.x0, g.z0, g.dx, g.dz)


EGB_LIN_EXACT, EGB_LIN_PAPER28 = 0, 1


def make_source(s, lin_variant: int = EGB_LIN_EXACT) -> EgbSource:
    return EgbSource(s.xs, s.zs, s.r0, s.beta, int(lin_variant))


def real_dtype(eg: EgbGrid):
    return torch.float64 if eg.dtype == EGB_F64 else torch.float32


# ------------------------------------------------------------------ sizes
def plane_stride(eg) -> int: return _lib.egb_plane_stride(ctypes.byref(eg))
def coeff2d_bytes(eg) -> int: return _lib.egb_coeff2d_bytes(ctypes.byref(eg))
def vel3d_bytes(eg) -> int: return _lib.egb_vel3d_bytes(ctypes.byref(eg))
def state_bytes(eg) -> int: return _lib.egb_state_bytes(ctypes.byref(eg))
def state_plane_offset(eg, p: int) -> int: return _lib.egb_state_plane_offset(ctypes.byref(eg), p)
def workspace_size(eg, op: int) -> int: return _lib.egb_workspace_size(ctypes.byref(eg), op)
def bdata_bytes(eg) -> int: return _lib.egb_bdata_bytes(ctypes.byref(eg))
def bdata_plane_stride(eg) -> int: return _lib.egb_bdata_plane_stride(ctypes.byref(eg))
def bfold_bytes(eg) -> int: return _lib.egb_bfold_bytes(ctypes.byref(eg))


def alloc_bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 16), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ calls
def egb_hamiltonian_velocity(eg, medium: "DeviceMedium", coeff2d, vel3d, work, stream=None) -> float:
    dt = ctypes.c_double(0.0)
    rc = _lib.egb_hamiltonian_velocity(ctypes.byref(eg), ctypes.byref(medium.struct()), _ptr(coeff2d), _ptr(vel3d),
                                       ctypes.byref(dt), _ptr(work), work.numel(), _stream(stream))
    _check("egb_hamiltonian_velocity", rc)
    return dt.value


def egb_velocity_dt_cfl(eg, vel3d) -> float:
    """The CFL limit the library recorded for vel3d on this grid."""
    dt = ctypes.c_double(0.0)
    _check("egb_velocity_dt_cfl", _lib.egb_velocity_dt_cfl(ctypes.byref(eg), _ptr(vel3d), ctypes.byref(dt)))
    return dt.value


def egb_declare_velocity(eg, vel3d, dt_cfl: float):
    _check("egb_declare_velocity", _lib.egb_declare_velocity(ctypes.byref(eg), _ptr(vel3d), float(dt_cfl)))


def egb_init_state(eg, coeff2d, src: EgbSource, state, stream=None):
    _check("egb_init_state", _lib.egb_init_state(ctypes.byref(eg), _ptr(coeff2d), ctypes.byref(src), _ptr(state),
                                                 _stream(stream)))


def egb_boundary_data(eg, state, bdata, stream=None):
    _check("egb_boundary_data", _lib.egb_boundary_data(ctypes.byref(eg), _ptr(state), _ptr(bdata), _stream(stream)))


def egb_liouville_step(eg, vel3d, src: EgbSource, bdata, state, work, dt: float, nsteps: int, stream=None):
    rc = _lib.egb_liouville_step(ctypes.byref(eg), _ptr(vel3d), ctypes.byref(src), _ptr(bdata), _ptr(state),
                                 _ptr(work), 0 if work is None else work.numel(), float(dt), int(nsteps),
                                 _stream(stream))
    _check("egb_liouville_step", rc)


def egb_beam_sum(eg, coeff2d, vel3d, src: EgbSource, state, omegas, out, work, stream=None):
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
    rc = _lib.egb_beam_sum(ctypes.byref(eg), _ptr(coeff2d), _ptr(vel3d), ctypes.byref(src), _ptr(state),
                           om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(om), _ptr(out), _ptr(work),
                           work.numel(), _stream(stream))
    _check("egb_beam_sum", rc)


def egb_beam_sum_noalloc(eg, coeff2d, vel3d, src: EgbSource, state, omegas, out, stream=None):
    """egb_beam_sum with the library's fixed per-device scratch (no workspace)."""
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
    rc = _lib.egb_beam_sum_noalloc(ctypes.byref(eg), _ptr(coeff2d), _ptr(vel3d), ctypes.byref(src), _ptr(state),
                                   om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(om), _ptr(out),
                                   _stream(stream))
    _check("egb_beam_sum_noalloc", rc)


def egb_pick_receivers(eg, state, rx, t_out, stream=None):
    n = 0 if rx is None else rx.shape[0]
    rc = _lib.egb_pick_receivers(ctypes.byref(eg), _ptr(state), _ptr(rx), n, _ptr(t_out), _stream(stream))
    _check("egb_pick_receivers", rc)


def gvel_bytes(eg) -> int: return _lib.egb_gvel_bytes(ctypes.byref(eg))


def egb_liouville_step_kinematic(eg, vel3d, src: EgbSource, bdata, state, work, dt: float, nsteps: int,
                                 stream=None):
    rc = _lib.egb_liouville_step_kinematic(ctypes.byref(eg), _ptr(vel3d), ctypes.byref(src), _ptr(bdata),
                                           _ptr(state), _ptr(work), work.numel(), float(dt), int(nsteps),
                                           _stream(stream))
    _check("egb_liouville_step_kinematic", rc)


def egb_pick_adjoint(eg, state, rx, tbar, lam, stream=None):
    rc = _lib.egb_pick_adjoint(ctypes.byref(eg), _ptr(state), _ptr(rx), rx.shape[0], _ptr(tbar), _ptr(lam),
                               _stream(stream))
    _check("egb_pick_adjoint", rc)


def egb_adjoint_step(eg, vel3d, src: EgbSource, bdata, state_n, lam, gvel, bfold, work, dt: float, stream=None):
    rc = _lib.egb_adjoint_step(ctypes.byref(eg), _ptr(vel3d), ctypes.byref(src), _ptr(bdata), _ptr(state_n),
                               _ptr(lam), _ptr(gvel), _ptr(bfold), _ptr(work), work.numel(), float(dt),
                               _stream(stream))
    _check("egb_adjoint_step", rc)


def egb_adjoint_medium(eg, medium: "DeviceMedium", coeff2d, src: EgbSource, gvel, lam0, bfold, grad, work,
                       stream=None):
    rc = _lib.egb_adjoint_medium(ctypes.byref(eg), ctypes.byref(medium.struct()), _ptr(coeff2d), ctypes.byref(src),
                                 _ptr(gvel), _ptr(lam0), _ptr(bfold), _ptr(grad), _ptr(work), work.numel(),
                                 _stream(stream))
    _check("egb_adjoint_medium", rc)


def paraxial_plane_stride(eg) -> int: return _lib.egb_paraxial_plane_stride(ctypes.byref(eg))
def paraxial_level_bytes(eg) -> int: return _lib.egb_paraxial_level_bytes(ctypes.byref(eg))
def paraxial_vel_bytes(eg) -> int: return _lib.egb_paraxial_vel_bytes(ctypes.byref(eg))


def egb_medium_table(eg, medium: "DeviceMedium", coeff2d, stream=None):
    _check("egb_medium_table", _lib.egb_medium_table(ctypes.byref(eg), ctypes.byref(medium.struct()), _ptr(coeff2d),
                                                     _stream(stream)))


EGB_DRT_EXACT, EGB_DRT_PAPER23 = 0, 1


def egb_paraxial_velocity(eg, coeff2d, theta_max: float, pvel, work, stream=None, drt: int = EGB_DRT_EXACT) -> float:
    rate = ctypes.c_double(0.0)
    rc = _lib.egb_paraxial_velocity(ctypes.byref(eg), _ptr(coeff2d), float(theta_max), int(drt), _ptr(pvel),
                                    ctypes.byref(rate), _ptr(work), work.numel(), _stream(stream))
    _check("egb_paraxial_velocity", rc)
    return rate.value


def egb_paraxial_init(eg, pvel, theta_max: float, beta: float, levels, stream=None, drt: int = EGB_DRT_EXACT):
    _check("egb_paraxial_init", _lib.egb_paraxial_init(ctypes.byref(eg), _ptr(pvel), float(theta_max), float(beta),
                                                       int(drt), _ptr(levels), _stream(stream)))


def egb_paraxial_march(eg, pvel, theta_max: float, nsub: int, levels, work, stream=None):
    rc = _lib.egb_paraxial_march(ctypes.byref(eg), _ptr(pvel), float(theta_max), int(nsub), _ptr(levels), _ptr(work),
                                 work.numel(), _stream(stream))
    _check("egb_paraxial_march", rc)


def egb_paraxial_pick(eg, levels, theta_max: float, xs, T, stream=None):
    n = 0 if xs is None else xs.numel()
    _check("egb_paraxial_pick", _lib.egb_paraxial_pick(ctypes.byref(eg), _ptr(levels), float(theta_max), _ptr(xs), n,
                                                       _ptr(T), _stream(stream)))


def egb_paraxial_beam_sum(eg, coeff2d, levels, theta_max: float, xs: float, lin: int, comp: int, omegas, out, work,
                          stream=None, drt: int = EGB_DRT_EXACT):
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
    rc = _lib.egb_paraxial_beam_sum(ctypes.byref(eg), _ptr(coeff2d), _ptr(levels), float(theta_max), float(xs),
                                    int(lin), int(drt), int(comp), om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    len(om), _ptr(out), _ptr(work), work.numel(), _stream(stream))
    _check("egb_paraxial_beam_sum", rc)


def make_problem_array(solvers, dts=None):
    """ctypes array of egb_problem from Solver objects (their own dt_cfl unless given)."""
    arr = (EgbProblem * len(solvers))()
    for i, s in enumerate(solvers):
        dt = s.dt_cfl if dts is None else dts[i]
        arr[i] = EgbProblem(s.eg, s.vel3d.data_ptr(), s.src, s.bdata.data_ptr(), s.state.data_ptr(), float(dt))
    return arr


def workspace_size_batched(arr) -> int:
    return _lib.egb_workspace_size_batched(arr, len(arr))


def egb_liouville_step_batched(arr, nsteps: int, work, stream=None):
    rc = _lib.egb_liouville_step_batched(arr, len(arr), int(nsteps), _ptr(work), work.numel(), _stream(stream))
    _check("egb_liouville_step_batched", rc)


# ------------------------------------------------- Green's-function migration
def _host_omegas(omegas):
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
    return om, om.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def egb_born_workspace_size(eg, ns: int, nw: int) -> int:
    return int(_lib.egb_born_workspace_size(ctypes.byref(eg), int(ns), int(nw)))


def egb_born_data(eg, G, omegas, m, d=None, work=None, stream=None) -> torch.Tensor:
    """Born data d [nw][ns][ns][re, im] (float64) of the reflectivity m
    (float64 [nx][nz]) from the Green's functions G [ns][nw][nx][nz][re, im];
    `work` (bytes, egb_born_workspace_size) is allocated when not given."""
    om, omp = _host_omegas(omegas)
    ns = G.shape[0]
    if d is None:
        d = torch.empty((len(om), ns, ns, 2), dtype=torch.float64, device=G.device)
    nb = egb_born_workspace_size(eg, ns, len(om))
    if work is None:
        work = alloc_bytes(max(nb, 256), G.device)
    _check("egb_born_data", _lib.egb_born_data(ctypes.byref(eg), _ptr(G), ns, omp, len(om), _ptr(m), _ptr(d),
                                               _ptr(work), work.numel() * work.element_size(), _stream(stream)))
    return d


def egb_migrate(eg, G, omegas, d, image=None, stream=None) -> torch.Tensor:
    """Image [nx][nz] (float64), the adjoint of egb_born_data."""
    om, omp = _host_omegas(omegas)
    if image is None:
        image = torch.empty((eg.nx, eg.nz), dtype=torch.float64, device=G.device)
    _check("egb_migrate", _lib.egb_migrate(ctypes.byref(eg), _ptr(G), G.shape[0], omp, len(om), _ptr(d),
                                           _ptr(image), _stream(stream)))
    return image


# ----------------------------------------------------------- launch tuning
EGB_TUNE_STEP, EGB_TUNE_KINEMATIC, EGB_TUNE_ADJOINT = 0, 1, 2


def egb_get_blocks(eg, op: int) -> int:
    return int(_lib.egb_get_blocks(ctypes.byref(eg), int(op)))


def egb_set_blocks(eg, op: int, blocks: int):
    _check("egb_set_blocks", _lib.egb_set_blocks(ctypes.byref(eg), int(op), int(blocks)))


def egb_tune_step(eg, vel3d, src: EgbSource, bdata, state, work, dt: float, op: int = EGB_TUNE_STEP, reps: int = 3,
                  stream=None) -> int:
    b = ctypes.c_int32(0)
    rc = _lib.egb_tune_step(ctypes.byref(eg), _ptr(vel3d), ctypes.byref(src), _ptr(bdata), _ptr(state), _ptr(work),
                            work.numel(), float(dt), int(op), int(reps), _stream(stream), ctypes.byref(b))
    _check("egb_tune_step", rc)
    return b.value


def egb_tune_batched(arr, work, reps: int = 3, stream=None) -> int:
    b = ctypes.c_int32(0)
    rc = _lib.egb_tune_batched(arr, len(arr), _ptr(work), work.numel(), int(reps), _stream(stream), ctypes.byref(b))
    _check("egb_tune_batched", rc)
    return b.value


def egb_set_blocks_batched(arr, blocks: int):
    _check("egb_set_blocks_batched", _lib.egb_set_blocks_batched(arr, len(arr), int(blocks)))


def egb_tile_rows(eg, op: int) -> list:
    """Tile heights (theta rows per tile) `op` supports on this grid's dtype, the default first."""
    rows = (ctypes.c_int32 * 8)()
    n = _lib.egb_tile_rows(ctypes.byref(eg), int(op), rows)
    return [rows[i] for i in range(n)]


def egb_get_launch(eg, op: int) -> tuple:
    """(tile_rows, blocks) in use for `op` on this grid shape (blocks 0: the default)."""
    l = EgbLaunch()
    _check("egb_get_launch", _lib.egb_get_launch(ctypes.byref(eg), int(op), ctypes.byref(l)))
    return l.tile_rows, l.blocks


def egb_set_launch(eg, op: int, tile_rows: int, blocks: int = 0):
    l = EgbLaunch(int(tile_rows), int(blocks))
    _check("egb_set_launch", _lib.egb_set_launch(ctypes.byref(eg), int(op), ctypes.byref(l)))


def egb_get_launch_batched(arr) -> tuple:
    l = EgbLaunch()
    _check("egb_get_launch_batched", _lib.egb_get_launch_batched(arr, len(arr), ctypes.byref(l)))
    return l.tile_rows, l.blocks


def egb_set_launch_batched(arr, tile_rows: int, blocks: int = 0):
    l = EgbLaunch(int(tile_rows), int(blocks))
    _check("egb_set_launch_batched", _lib.egb_set_launch_batched(arr, len(arr), ctypes.byref(l)))


# ------------------------------------------------------------------ views
def state_views(eg, state: torch.Tensor) -> dict:
    """Named [nth][nx][nz] views of the planes of a state byte buffer."""
    n = eg.nth * eg.nx * eg.nz
    out = {}
    for p, name in enumerate(STATE_PLANES):
        dt = torch.float64 if p == EGB_PSI else real_dtype(eg)
        off = state_plane_offset(eg, p)
        es = torch.empty((), dtype=dt).element_size()
        out[name] = state[off:off + n * es].view(dt).view(eg.nth, eg.nx, eg.nz)
    return out


def vel_views(eg, vel3d: torch.Tensor) -> dict:
    n = eg.nth * eg.nx * eg.nz
    dt = real_dtype(eg)
    flat = vel3d.view(dt)
    st = plane_stride(eg)
    return {name: flat[q * st:q * st + n].view(eg.nth, eg.nx, eg.nz) for q, name in enumerate(VEL_PLANES)}


def coeff2d_view(eg, coeff2d: torch.Tensor) -> torch.Tensor:
    """[field][taylor][nx][nz] float64 view."""
    return coeff2d.view(torch.float64).view(5, 6, eg.nx, eg.nz)


def write_state(eg, state: torch.Tensor, planes: dict):
    """Copy named host/device arrays into a state buffer (marshalling for tests)."""
    v = state_views(eg, state)
    for name, arr in planes.items():
        v[name].copy_(torch.as_tensor(np.asarray(arr)).to(v[name].dtype))


@dataclass
class DeviceMedium:
    vp0: torch.Tensor
    eps: torch.Tensor
    delta: torch.Tensor
    tilt: Optional[torch.Tensor]
    vs_ratio: float

    @staticmethod
    def from_numpy(m, device) -> "DeviceMedium":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
        return DeviceMedium(f(m.vp0), f(m.eps), f(m.delta), None if m.tilt is None else f(m.tilt), float(m.vs_ratio))

    def struct(self) -> EgbMedium:
        return EgbMedium(self.vp0.data_ptr(), self.eps.data_ptr(), self.delta.data_ptr(),
                         None if self.tilt is None else self.tilt.data_ptr(), self.vs_ratio)


class Solver:
    """Buffers and call sequence for one problem (one source) on one device."""

    def __init__(self, problem, device="cuda", dtype: Optional[str] = None):
        self.p = problem
        self.device = torch.device(device)
        self.eg = make_grid(problem.grid, dtype or problem.dtype)
        self.src = make_source(problem.source)
        self.medium = DeviceMedium.from_numpy(problem.medium, self.device)
        eg = self.eg
        self.coeff2d = alloc_bytes(coeff2d_bytes(eg), self.device)
        self.vel3d = alloc_bytes(vel3d_bytes(eg), self.device)
        self.state = alloc_bytes(state_bytes(eg), self.device)
        self.bdata = alloc_bytes(bdata_bytes(eg), self.device)
        self.work_vel = alloc_bytes(workspace_size(eg, EGB_OP_VELOCITY), self.device)
        self.work_step = alloc_bytes(workspace_size(eg, EGB_OP_STEP), self.device)
        self.work_beam = None
        self.dt_cfl = None

    def tune(self, op: int = EGB_TUNE_STEP, reps: int = 3, dt: Optional[float] = None, stream=None) -> int:
        """Autotune the stage launch shape for this grid (after velocity() and
        init()); the state is left unchanged."""
        return egb_tune_step(self.eg, self.vel3d, self.src, self.bdata, self.state, self.work_step,
                             self.dt_cfl if dt is None else dt, op, reps, stream)

    def velocity(self, stream=None) -> float:
        self.dt_cfl = egb_hamiltonian_velocity(self.eg, self.medium, self.coeff2d, self.vel3d, self.work_vel, stream)
        return self.dt_cfl

    def init(self, stream=None):
        """Point-source data, and the boundary data of the march taken from it."""
        egb_init_state(self.eg, self.coeff2d, self.src, self.state, stream)
        egb_boundary_data(self.eg, self.state, self.bdata, stream)

    def step(self, nsteps: int, dt: Optional[float] = None, stream=None):
        egb_liouville_step(self.eg, self.vel3d, self.src, self.bdata, self.state, self.work_step,
                           self.dt_cfl if dt is None else dt, nsteps, stream)

    def step_kinematic(self, nsteps: int, dt: Optional[float] = None, stream=None):
        """March phi1 and psi only (the other planes are left as they are)."""
        egb_liouville_step_kinematic(self.eg, self.vel3d, self.src, self.bdata, self.state, self.work_step,
                                     self.dt_cfl if dt is None else dt, nsteps, stream)

    def beam(self, omegas, out: Optional[torch.Tensor] = None, stream=None, lin: int = EGB_LIN_EXACT) -> torch.Tensor:
        """Green's function [nw][nx][nz][re, im]; lin selects the linear phase
        coefficient (EGB_LIN_EXACT or EGB_LIN_PAPER28)."""
        om = np.atleast_1d(np.asarray(omegas, dtype=np.float64))
        if self.work_beam is None:
            self.work_beam = alloc_bytes(workspace_size(self.eg, EGB_OP_BEAM), self.device)
        if out is None:
            out = torch.empty((len(om), self.eg.nx, self.eg.nz, 2), dtype=real_dtype(self.eg), device=self.device)
        src = self.src if lin == EGB_LIN_EXACT else make_source(self.p.source, lin)
        egb_beam_sum(self.eg, self.coeff2d, self.vel3d, src, self.state, om, out, self.work_beam, stream)
        return out

    def pick(self, receivers, stream=None) -> torch.Tensor:
        rx = torch.as_tensor(np.ascontiguousarray(receivers, dtype=np.float64), device=self.device).reshape(-1, 2)
        t = torch.empty(rx.shape[0], dtype=torch.float64, device=self.device)
        egb_pick_receivers(self.eg, self.state, rx, t, stream)
        return t

    def planes(self) -> dict:
        return state_views(self.eg, self.state)

    def vel_planes(self) -> dict:
        return vel_views(self.eg, self.vel3d)


def paraxial_level_views(eg, levels: torch.Tensor, n: int) -> dict:
    """Named [nth][nx] views of level n of a paraxial levels buffer."""
    lb, st = paraxial_level_bytes(eg), paraxial_plane_stride(eg)
    rd = real_dtype(eg)
    es = torch.empty((), dtype=rd).element_size()
    base = levels[n * lb:(n + 1) * lb]
    out = {}
    for q, name in enumerate(PAR_PLANES):
        dt, off = (torch.float64, 7 * st * es) if name == "tau" else (rd, q * st * es)
        e = torch.empty((), dtype=dt).element_size()
        out[name] = base[off:off + eg.nth * eg.nx * e].view(dt).view(eg.nth, eg.nx)
    return out


class Paraxial:
    """Buffers and call sequence of the paraxial depth march for one medium:
    medium table, coefficients, surface data, march, first-arrival picks of
    any number of surface sources.  theta_max: half aperture (rad); drt: the
    DRT frame (EGB_DRT_EXACT, or EGB_DRT_PAPER23 for eqs. 21-23)."""

    def __init__(self, grid, medium, theta_max: float, device="cuda", dtype: str = "f32",
                 drt: int = EGB_DRT_EXACT):
        self.device = torch.device(device)
        self.eg = make_grid(grid, dtype)
        self.theta_max = float(theta_max)
        self.drt = int(drt)
        self.medium = DeviceMedium.from_numpy(medium, self.device)
        eg = self.eg
        self.coeff2d = alloc_bytes(coeff2d_bytes(eg), self.device)
        self.pvel = alloc_bytes(paraxial_vel_bytes(eg), self.device)
        self.levels = alloc_bytes(eg.nz * paraxial_level_bytes(eg), self.device)
        self.work_vel = alloc_bytes(workspace_size(eg, EGB_OP_VELOCITY), self.device)
        self.work = alloc_bytes(workspace_size(eg, EGB_OP_PARAXIAL), self.device)
        self.work_beam = None
        self.rate = None

    def velocity(self, stream=None) -> float:
        egb_medium_table(self.eg, self.medium, self.coeff2d, stream)
        self.rate = egb_paraxial_velocity(self.eg, self.coeff2d, self.theta_max, self.pvel, self.work_vel, stream,
                                          self.drt)
        return self.rate

    def substeps(self, cfl: float = 0.5) -> int:
        """RK3 substeps per depth interval: dz / nsub * rate <= cfl."""
        return max(1, int(np.ceil(self.eg.dz * self.rate / cfl - 1e-12)))

    def init(self, beta: float, stream=None):
        egb_paraxial_init(self.eg, self.pvel, self.theta_max, beta, self.levels, stream, self.drt)

    def march(self, nsub: Optional[int] = None, stream=None):
        egb_paraxial_march(self.eg, self.pvel, self.theta_max, self.substeps() if nsub is None else nsub,
                           self.levels, self.work, stream)

    def pick(self, xs, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        x = torch.as_tensor(np.ascontiguousarray(np.atleast_1d(xs), dtype=np.float64), device=self.device)
        if out is None:
            out = torch.empty((x.numel(), self.eg.nz, self.eg.nx), dtype=torch.float64, device=self.device)
        egb_paraxial_pick(self.eg, self.levels, self.theta_max, x, out, stream)
        return out

    def beam(self, xs: float, omegas, lin: int = EGB_LIN_EXACT, out: Optional[torch.Tensor] = None,
             stream=None, comp: int = -1) -> torch.Tensor:
        """Green's function [nw][nx][nz][re, im] of a surface source at xs
        (row n = depth level n); comp = 2 i + k: component G_ik of the qP
        Green's tensor (x = 0, z = 1), -1: the scalar sum."""
        om = np.atleast_1d(np.asarray(omegas, dtype=np.float64))
        if self.work_beam is None:
            self.work_beam = alloc_bytes(workspace_size(self.eg, EGB_OP_PBEAM), self.device)
        if out is None:
            out = torch.empty((len(om), self.eg.nx, self.eg.nz, 2), dtype=real_dtype(self.eg), device=self.device)
        egb_paraxial_beam_sum(self.eg, self.coeff2d, self.levels, self.theta_max, xs, lin, comp, om, out,
                              self.work_beam, stream, self.drt)
        return out

    def greens(self, xs_list, omegas, lin: int = EGB_LIN_EXACT, stream=None) -> torch.Tensor:
        """Green's functions [ns][nw][nx][nz][re, im] of the surface points
        xs_list from the one march (the input of egb_born_data / egb_migrate)."""
        om = np.atleast_1d(np.asarray(omegas, dtype=np.float64))
        xs_list = np.atleast_1d(np.asarray(xs_list, dtype=np.float64))
        G = torch.empty((len(xs_list), len(om), self.eg.nx, self.eg.nz, 2), dtype=real_dtype(self.eg),
                        device=self.device)
        for i, xs in enumerate(xs_list):
            self.beam(float(xs), om, lin=lin, out=G[i], stream=stream)
        return G

    def level(self, n: int) -> dict:
        return paraxial_level_views(self.eg, self.levels, n)

    def pvel_level(self, n: int) -> dict:
        st = paraxial_plane_stride(self.eg)
        flat = self.pvel.view(real_dtype(self.eg))[n * 7 * st:(n + 1) * 7 * st]
        m = self.eg.nth * self.eg.nx
        return {name: flat[q * st:q * st + m].view(self.eg.nth, self.eg.nx) for q, name in enumerate(PVEL_PLANES)}


class TravelTime(torch.autograd.Function):
    """First-arrival traveltimes at receivers as a differentiable function of
    the gridded medium (vp0, eps, delta, tilt; float64 device tensors [nx][nz]).

    forward: medium table and velocity, point-source data, ``nsteps``
    kinematic RK3 steps (phi1, psi), then the pick.  The states the backward
    sweep needs are kept in one of two ways:
    * ``checkpoint_every`` = K > 0: a whole state every K steps; the backward
      sweep recomputes each segment from its checkpoint;
    * K = 0: the two planes the adjoint reads (phi1, psi) of every step's
      state, resident in device memory (12 B per cell and step in FP32:
      121 GB for 600 steps at 256^3, which HBM of 288 GB holds), so nothing
      is recomputed but the two inner stages of each step;
    * K = "auto" (the default): 0 when the archive takes at most half of the
      free device memory, else 16.
    backward: the pick adjoint, then step by step in reverse the adjoint
    step, and finally the medium gradient.  The gradient is the same bit for
    bit for every K.  The time step is fixed (the CFL step of the forward
    medium unless ``spec['dt']`` is set).

    spec: grid (nx, nz, nth, x0, z0, dx, dz), source (xs, zs, r0, beta),
    receivers (numpy [nr][2]), nsteps, vs_ratio, dtype ("f32" / "f64"),
    checkpoint_every (default "auto"), dt (optional).
    """

    @staticmethod
    def forward(ctx, vp0, eps, delta, tilt, spec):
        dev = vp0.device
        eg = make_grid(spec["grid"], spec.get("dtype", "f32"))
        src = make_source(spec["source"])
        med = DeviceMedium(vp0.contiguous(), eps.contiguous(), delta.contiguous(), tilt.contiguous(),
                           float(spec.get("vs_ratio", 0.5)))
        coeff2d = alloc_bytes(coeff2d_bytes(eg), dev)
        vel3d = alloc_bytes(vel3d_bytes(eg), dev)
        wv = alloc_bytes(workspace_size(eg, EGB_OP_VELOCITY), dev)
        dt = egb_hamiltonian_velocity(eg, med, coeff2d, vel3d, wv)
        dt = float(spec["dt"]) if spec.get("dt") is not None else dt
        state = alloc_bytes(state_bytes(eg), dev)
        egb_init_state(eg, coeff2d, src, state)
        bdata = alloc_bytes(bdata_bytes(eg), dev)
        egb_boundary_data(eg, state, bdata)
        work = alloc_bytes(workspace_size(eg, EGB_OP_STEP), dev)
        nsteps = int(spec["nsteps"])
        views = state_views(eg, state)
        K = spec.get("checkpoint_every", "auto")
        if not any(ctx.needs_input_grad[:4]):
            K = nsteps  # no backward sweep will run: only the start is kept
        elif K == "auto":
            need = nsteps * (views["phi1"].numel() * views["phi1"].element_size() +
                             views["psi"].numel() * views["psi"].element_size())
            K = 0 if need <= 0.5 * torch.cuda.mem_get_info(dev)[0] else 16
        K = int(K)
        ckpts, arch = [], None
        if K == 0:  # phi1 and psi of every step's state, resident
            arch = (torch.empty((nsteps,) + tuple(views["phi1"].shape), dtype=views["phi1"].dtype, device=dev),
                    torch.empty((nsteps,) + tuple(views["psi"].shape), dtype=views["psi"].dtype, device=dev))
            for i in range(nsteps):
                arch[0][i].copy_(views["phi1"])
                arch[1][i].copy_(views["psi"])
                egb_liouville_step_kinematic(eg, vel3d, src, bdata, state, work, dt, 1)
        done = 0
        while K > 0 and done < nsteps:
            ckpts.append((done, state.clone()))
            n = min(K, nsteps - done)
            egb_liouville_step_kinematic(eg, vel3d, src, bdata, state, work, dt, n)
            done += n
        rx = torch.as_tensor(np.ascontiguousarray(spec["receivers"], dtype=np.float64), device=dev).reshape(-1, 2)
        t = torch.empty(rx.shape[0], dtype=torch.float64, device=dev)
        egb_pick_receivers(eg, state, rx, t)
        ctx.egb = dict(eg=eg, src=src, med=med, coeff2d=coeff2d, vel3d=vel3d, bdata=bdata, dt=dt, K=K, nsteps=nsteps,
                       ckpts=ckpts, arch=arch, final=state, rx=rx, work=work)
        return t

    @staticmethod
    def backward(ctx, tbar):
        d = ctx.egb
        eg, src, dev = d["eg"], d["src"], d["final"].device
        lam = torch.zeros(state_bytes(eg), dtype=torch.uint8, device=dev)
        gvel = torch.zeros(gvel_bytes(eg), dtype=torch.uint8, device=dev)
        bfold = torch.zeros(bfold_bytes(eg), dtype=torch.uint8, device=dev)
        tb = torch.nan_to_num(tbar.detach().to(torch.float64).contiguous(), nan=0.0)
        egb_pick_adjoint(eg, d["final"], d["rx"], tb, lam)
        wadj = alloc_bytes(workspace_size(eg, EGB_OP_ADJOINT), dev)
        if d["arch"] is not None:  # every step's phi1 and psi are resident
            # two state buffers: step i - 1's planes are copied into one on a
            # side stream while the adjoint step of i reads the other
            main = torch.cuda.current_stream(dev)
            side = torch.cuda.Stream(dev)
            st = [d["final"].clone(), d["final"].clone()]
            views = [state_views(eg, b) for b in st]
            ready = [torch.cuda.Event(), torch.cuda.Event()]
            done = [torch.cuda.Event(), torch.cuda.Event()]

            def stage(i, b):
                side.wait_event(done[b])  # the step that last read buffer b has ended
                with torch.cuda.stream(side):
                    views[b]["phi1"].copy_(d["arch"][0][i])
                    views[b]["psi"].copy_(d["arch"][1][i])
                ready[b].record(side)

            n = d["nsteps"]
            if n > 0:
                stage(n - 1, 0)
            for k, i in enumerate(reversed(range(n))):
                b = k % 2
                if i > 0:
                    stage(i - 1, 1 - b)
                main.wait_event(ready[b])
                egb_adjoint_step(eg, d["vel3d"], src, d["bdata"], st[b], lam, gvel, bfold, wadj, d["dt"])
                done[b].record(main)
        for start, ck in reversed(d["ckpts"]):
            n = min(d["K"], d["nsteps"] - start)
            states = [ck]
            cur = ck.clone()
            for _ in range(n - 1):
                egb_liouville_step_kinematic(eg, d["vel3d"], src, d["bdata"], cur, d["work"], d["dt"], 1)
                states.append(cur.clone())
            for st in reversed(states):
                egb_adjoint_step(eg, d["vel3d"], src, d["bdata"], st, lam, gvel, bfold, wadj, d["dt"])
        grad = torch.empty((4, eg.nx, eg.nz), dtype=torch.float64, device=dev)
        egb_adjoint_medium(eg, d["med"], d["coeff2d"], src, gvel, lam, bfold, grad, wadj)
        d["arch"], d["ckpts"] = None, []  # the kept states are not needed again
        return grad[0], grad[1], grad[2], grad[3], None


def traveltime(vp0, eps, delta, tilt, spec):
    """Differentiable first-arrival traveltimes (see TravelTime)."""
    return TravelTime.apply(vp0, eps, delta, tilt, spec)
