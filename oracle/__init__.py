"""FP64 CPU oracle for the Eulerian Gaussian beam hot path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (``paper_2006_11945_amd``) and never imports it.

The arithmetic lives in ``egb_oracle.c`` (plain double-precision loops, built
with gcc by :func:`build`); this module only marshals numpy arrays.  The
migration operators (plain sums over the Green's functions) are numpy, in
``migration.py``.  Plane
order of the oracle state: phi1, psi, Re C, Im C, Re B, Im B, and the
continuous phase of C (the KMAH phase, which decides the branch of
sqrt(1/C) in the beam sum).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "egb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PLANES = ("phi1", "psi", "ReC", "ImC", "ReB", "ImB", "phase")
PAR_PLANES = ("X", "vt", "tau", "ReC", "ImC", "ReB", "ImB", "phase")  # paraxial depth march
VEL_PLANES = ("Vx", "Vz", "Vt", "A11", "A12", "A21", "A22")
NFLD, NTAY = 5, 6

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-D_DEFAULT_SOURCE", "-Wall", "-Wno-unused-function",
                               SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.oc_fd1.argtypes = [P, i, i, d]; L.oc_fd1.restype = d
        L.oc_fd2.argtypes = [P, i, i, d]; L.oc_fd2.restype = d
        L.oc_medium_table.argtypes = [i, i, d, d, P, P, P, P, d, P]
        L.oc_vjet.argtypes = [P, d, P]; L.oc_vjet.restype = None
        L.oc_va.argtypes = [P, d, P, P]; L.oc_va.restype = None
        L.oc_velocity.argtypes = [i, i, i, d, d, P, P, P, P]
        L.oc_init_state.argtypes = [i, i, i, d, d, d, d, P, d, d, d, P]
        L.oc_weno.argtypes = [P, i]; L.oc_weno.restype = d
        L.oc_upwind5.argtypes = [P, i]; L.oc_upwind5.restype = d
        L.oc_march.argtypes = [i, i, i, d, d, d, d, P, d, d, d, P, P, d, i]
        L.oc_beam_sum.argtypes = [i, i, i, d, d, d, d, P, P, d, i, P, P, i, P]
        L.oc_beam_sum_at.argtypes = [i, i, i, d, d, d, d, P, P, d, i, P, P, i, ctypes.POINTER(i), i, P]
        L.oc_pbeam_sum.argtypes = [i, i, i, d, d, d, d, d, P, P, d, i, i, i, P, i, P]
        L.oc_paper23_drt.argtypes = [P, d, d, P]
        L.oc_qp_polarization.argtypes = [P, d, P]
        L.oc_qp_polarization.restype = None
        L.oc_lin28.argtypes = [d, d, d, d]
        L.oc_lin28.restype = d
        L.oc_pick.argtypes = [i, i, i, d, d, d, d, P, P, i, P]
        L.oc_pvelocity.argtypes = [i, i, i, d, d, d, i, P, P, P]
        L.oc_pinit.argtypes = [i, i, d, d, d, P, d, i, P]
        L.oc_pmarch.argtypes = [i, i, i, d, d, d, P, i, P, P]
        L.oc_ppick.argtypes = [i, i, i, d, P, P, i, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def fd1(f, i: int, h: float) -> float:
    f = _c(f)
    return lib().oc_fd1(_p(f), len(f), i, h)


def fd2(f, i: int, h: float) -> float:
    f = _c(f)
    return lib().oc_fd2(_p(f), len(f), i, h)


def medium_table(grid, medium) -> np.ndarray:
    """Table [nx][nz][5 fields (a11, a33, b, a55, nu)][6 (f, fx, fz, fxx, fxz, fzz)]."""
    tab = np.zeros((grid.nx, grid.nz, NFLD, NTAY))
    rc = lib().oc_medium_table(grid.nx, grid.nz, grid.dx, grid.dz, _p(_c(medium.vp0)), _p(_c(medium.eps)),
                               _p(_c(medium.delta)), _p(_c(medium.tilt)), float(medium.vs_ratio), _p(tab))
    if rc != 0:
        raise ValueError(f"oc_medium_table failed ({rc})")
    return tab


def vjet(t: np.ndarray, theta: float) -> np.ndarray:
    """Jet of v at one point: v, v_x, v_z, v_t, v_xx, v_xz, v_zz, v_xt, v_zt, v_tt."""
    t = _c(t).reshape(NFLD * NTAY)
    o = np.zeros(10)
    lib().oc_vjet(_p(t), float(theta), _p(o))
    return o


def va(vj: np.ndarray, theta: float):
    """(V[3], A[4]) from a v-jet."""
    vj = _c(vj)
    V, A = np.zeros(3), np.zeros(4)
    lib().oc_va(_p(vj), float(theta), _p(V), _p(A))
    return V, A


def velocity(grid, tab: np.ndarray):
    """Returns (vel[7][nth][nx][nz], vaux[4][nth][nx][nz] = v, v_x, v_z, v_t, dt_cfl)."""
    sh = (grid.nth, grid.nx, grid.nz)
    vel = np.zeros((7,) + sh)
    vaux = np.zeros((4,) + sh)
    dt = np.zeros(1)
    lib().oc_velocity(grid.nx, grid.nz, grid.nth, grid.dx, grid.dz, _p(_c(tab)), _p(vel), _p(vaux), _p(dt))
    return vel, vaux, float(dt[0])


def init_state(grid, tab: np.ndarray, source) -> np.ndarray:
    U = np.zeros((len(PLANES), grid.nth, grid.nx, grid.nz))
    lib().oc_init_state(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, _p(_c(tab)),
                        source.xs, source.zs, source.beta, _p(U))
    return U


def weno(u7, minus: bool) -> float:
    u7 = _c(u7)
    return lib().oc_weno(_p(u7), int(bool(minus)))


def march(grid, vel: np.ndarray, source, U: np.ndarray, dt: float, nsteps: int, Ub=None) -> np.ndarray:
    """nsteps SSP-RK3 steps from U.  Ub: the point-source data (boundary
    values outside the grid and in the ball); U itself when None."""
    U = _c(U).copy()
    Ub = U.copy() if Ub is None else _c(Ub)
    rc = lib().oc_march(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, _p(_c(vel)),
                        source.xs, source.zs, source.r0, _p(Ub), _p(U), float(dt), int(nsteps))
    if rc != 0:
        raise MemoryError("oc_march")
    return U


def beam_sum(grid, vel, vaux, source, U, omegas, lin: int = 0) -> np.ndarray:
    """Complex Green's function [nw][nx][nz]; lin = 1: eq. 28's linear
    phase coefficient instead of eq. 7's p1."""
    om = _c(np.atleast_1d(omegas))
    out = np.zeros((len(om), grid.nx, grid.nz, 2))
    rc = lib().oc_beam_sum(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, _p(_c(vel)),
                           _p(_c(vaux)), source.beta, int(lin), _p(_c(U)), _p(om), len(om), _p(out))
    if rc == -3:
        raise RuntimeError("oracle beam list overflow")
    return out[..., 0] + 1j * out[..., 1]


def beam_sum_at(grid, vel, vaux, source, U, omegas, points, lin: int = 0) -> np.ndarray:
    """The same Green's function at the output cells points[j] = (ix, iz)
    only: complex [nw][npts] (the beams are those of the whole state)."""
    om = _c(np.atleast_1d(omegas))
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 2))
    out = np.zeros((len(om), len(pts), 2))
    rc = lib().oc_beam_sum_at(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, _p(_c(vel)),
                              _p(_c(vaux)), source.beta, int(lin), _p(_c(U)), _p(om), len(om),
                              pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(pts), _p(out))
    if rc == -1:
        raise ValueError("output cell outside the grid")
    if rc == -3:
        raise RuntimeError("oracle beam list overflow")
    return out[..., 0] + 1j * out[..., 1]


def pick(grid, U, receivers) -> np.ndarray:
    rx = _c(receivers).reshape(-1, 2)
    out = np.zeros(len(rx))
    lib().oc_pick(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, _p(_c(U)), _p(rx),
                  len(rx), _p(out))
    return out


def solve(problem, nsteps=None, dt=None):
    """Full oracle pipeline: table, velocity, data, march (at the CFL step of
    this medium unless ``dt`` is given).  Returns a dict."""
    g = problem.grid
    tab = medium_table(g, problem.medium)
    vel, vaux, dt_cfl = velocity(g, tab)
    dt = dt_cfl if dt is None else float(dt)
    U0 = init_state(g, tab, problem.source)
    ns = problem.nsteps if nsteps is None else nsteps
    U = march(g, vel, problem.source, U0, dt, ns) if ns > 0 else U0
    return {"tab": tab, "vel": vel, "vaux": vaux, "dt": dt, "dt_cfl": dt_cfl, "U0": U0, "U": U, "nsteps": ns}


# ---------------------------------------------------------------- paraxial
# Depth march on (x, theta) slices, theta in (-theta_max, theta_max); see the
# paraxial section of egb_oracle.c.  Arrays: pvel[nz][7][nth][nx],
# states [nz][8][nth][nx] (planes PAR_PLANES), T[source][nz][nx].

def ptheta(grid, theta_max: float) -> np.ndarray:
    dth = 2.0 * theta_max / grid.nth
    return -theta_max + (np.arange(grid.nth) + 0.5) * dth


def pvelocity(grid, tab: np.ndarray, theta_max: float, drt: int = 0):
    """(pvel, rate) with rate = max(|u|/dx + |w|/dtheta); raises if V_z <= 0.
    drt = 1: the DRT coefficients of eqs. 21-23 (lateral frame, corrected)."""
    pvel = np.zeros((grid.nz, 7, grid.nth, grid.nx))
    rate = np.zeros(1)
    rc = lib().oc_pvelocity(grid.nx, grid.nz, grid.nth, grid.dx, grid.dz, float(theta_max), int(drt), _p(_c(tab)),
                            _p(pvel), _p(rate))
    if rc != 0:
        raise ValueError("paraxial velocity: V_z <= 0 inside (-theta_max, theta_max)")
    return pvel, float(rate[0])


def psubsteps(grid, rate: float, cfl: float = 0.5) -> int:
    """SSP-RK3 steps per depth interval dz: dz / nsub * rate <= cfl."""
    return max(1, int(np.ceil(grid.dz * rate / cfl - 1e-12)))


def pinit(grid, pvel: np.ndarray, theta_max: float, beta: float, drt: int = 0) -> np.ndarray:
    U = np.zeros((len(PAR_PLANES), grid.nth, grid.nx))
    lib().oc_pinit(grid.nx, grid.nth, grid.x0, grid.dx, float(theta_max), _p(_c(pvel[0])), float(beta), int(drt),
                   _p(U))
    return U


def pmarch(grid, pvel: np.ndarray, theta_max: float, U0: np.ndarray, nsub: int, Ub=None) -> np.ndarray:
    """Levels [nz][8][nth][nx] from U0 on level 0; Ub: the surface data held
    in the ghosts (U0 itself when None)."""
    Uall = np.zeros((grid.nz, len(PAR_PLANES), grid.nth, grid.nx))
    Uall[0] = U0
    Ub = _c(U0 if Ub is None else Ub)
    rc = lib().oc_pmarch(grid.nx, grid.nz, grid.nth, grid.dx, grid.dz, float(theta_max), _p(_c(pvel)), int(nsub),
                         _p(Ub), _p(Uall))
    if rc != 0:
        raise MemoryError("oc_pmarch")
    return Uall


def pbeam_sum(grid, tab, Uall, theta_max: float, xs: float, omegas, lin: int = 0, comp: int = -1,
              drt: int = 0) -> np.ndarray:
    """Green's function [nw][nx][nz] of a surface source at xs from the
    depth-march levels (row n = depth level n; row 0 left zero); comp =
    2 i + k >= 0: the (i, k) component of the qP Green's tensor (x = 0, z = 1);
    drt = 1 for levels marched with the lateral-frame DRT of eqs. 21-23."""
    om = _c(np.atleast_1d(omegas))
    out = np.zeros((len(om), grid.nx, grid.nz, 2))
    rc = lib().oc_pbeam_sum(grid.nx, grid.nz, grid.nth, grid.x0, grid.z0, grid.dx, grid.dz, float(theta_max),
                            _p(_c(tab)), _p(_c(Uall)), float(xs), int(lin), int(drt), int(comp), _p(om), len(om),
                            _p(out))
    if rc == -3:
        raise RuntimeError("oracle beam list overflow")
    if rc != 0:
        raise MemoryError("oc_pbeam_sum")
    return out[..., 0] + 1j * out[..., 1]


def paper23_drt(vj: np.ndarray, theta: float, u: float) -> np.ndarray:
    """(a11, a12, a21, a22) of the lateral-frame DRT of eqs. 21-23 (per unit
    depth) from a v-jet, the phase angle and u = dx/dz."""
    a = np.zeros(4)
    lib().oc_paper23_drt(_p(_c(vj)), float(theta), float(u), _p(a))
    return a


def qp_polarization(ms, theta: float) -> np.ndarray:
    """qP polarisation (g_x, g_z) for medium values (a11, a33, a13 + a55, a55, nu)."""
    g = np.zeros(2)
    lib().oc_qp_polarization(_p(_c(ms)), float(theta), _p(g))
    return g


def lin28(s: float, c: float, u: float, v: float) -> float:
    """Eq. 28's linear phase coefficient (see oc_lin28)."""
    return lib().oc_lin28(float(s), float(c), float(u), float(v))


def ppick(grid, Uall: np.ndarray, xs, theta_max: float) -> np.ndarray:
    xs = _c(np.atleast_1d(xs))
    T = np.zeros((len(xs), grid.nz, grid.nx))
    lib().oc_ppick(grid.nx, grid.nz, grid.nth, float(theta_max), _p(_c(Uall)), _p(xs), len(xs), _p(T))
    return T


def psolve(grid, medium, theta_max: float, beta: float, xs=(), cfl: float = 0.5, drt: int = 0):
    """Table, paraxial velocity, surface data, depth march, picks."""
    tab = medium_table(grid, medium)
    pvel, rate = pvelocity(grid, tab, theta_max, drt)
    nsub = psubsteps(grid, rate, cfl)
    U0 = pinit(grid, pvel, theta_max, beta, drt)
    Uall = pmarch(grid, pvel, theta_max, U0, nsub)
    T = ppick(grid, Uall, xs, theta_max) if len(np.atleast_1d(xs)) else None
    return {"tab": tab, "pvel": pvel, "rate": rate, "nsub": nsub, "U": Uall, "T": T, "drt": drt}
