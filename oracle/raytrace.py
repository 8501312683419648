"""Lagrangian ray tracing along bicharacteristics (test infrastructure only).

The continuum counterpart of the Eulerian fields: a single ray of the
phase-space flow dx/dtau, dz/dtau (eqs. 8-9) and dtheta/dtau (eq. 12) is
integrated with an adaptive Runge-Kutta method (scipy's DOP853, a library
primitive), optionally together with the linearised perturbation
d(dn, dth_perp)/dtau = A (dn, dth_perp) of the ray-normal frame.  The medium
is analytic: a callable returning, at (x, z), the five fields
(a11, a33, a13 + a55, a55, nu) with their first and second derivatives, so
the ray tracer sees no grid.

Used to pin the dynamic-ray-tracing matrix A (finite differences of ray
pairs) and traveltimes in heterogeneous media.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp

from . import vjet, va


def thomsen_fields(vp0, eps, delta, nu, fs=0.5):
    """Field values (a11, a33, b, a55, nu) from Thomsen parameters (scalars)."""
    a33 = vp0 ** 2
    a55 = (fs * vp0) ** 2
    a11 = a33 * (1 + 2 * eps)
    b = np.sqrt((a33 - a55) * (a33 * (1 + 2 * delta) - a55))
    return np.array([a11, a33, b, a55, nu])


class QuadraticMedium:
    """Each of the five fields is an exact quadratic in (x - xc, z - zc)."""

    def __init__(self, centre, f0, fx, fz, fxx, fxz, fzz):
        self.c = np.asarray(centre, dtype=np.float64)
        self.f0, self.fx, self.fz = map(np.asarray, (f0, fx, fz))
        self.fxx, self.fxz, self.fzz = map(np.asarray, (fxx, fxz, fzz))

    def table(self, x, z):
        dx, dz = x - self.c[0], z - self.c[1]
        t = np.zeros((5, 6))
        t[:, 0] = self.f0 + self.fx * dx + self.fz * dz + 0.5 * (self.fxx * dx * dx + 2 * self.fxz * dx * dz + self.fzz * dz * dz)
        t[:, 1] = self.fx + self.fxx * dx + self.fxz * dz
        t[:, 2] = self.fz + self.fxz * dx + self.fzz * dz
        t[:, 3] = self.fxx
        t[:, 4] = self.fxz
        t[:, 5] = self.fzz
        return t


class GradientIsoMedium:
    """Isotropic v = v0 + g (z - zref), shear ratio fs."""

    def __init__(self, v0, g, zref, fs=0.5):
        self.v0, self.g, self.zref, self.fs = v0, g, zref, fs

    def table(self, x, z):
        v = self.v0 + self.g * (z - self.zref)
        k = np.array([1.0, 1.0, 1.0 - self.fs ** 2, self.fs ** 2])  # a11, a33, b, a55 over v^2
        t = np.zeros((5, 6))
        t[:4, 0] = k * v * v
        t[:4, 2] = k * 2 * self.g * v
        t[:4, 5] = k * 2 * self.g * self.g
        return t


def velocity_at(medium, x, z, th):
    vj = vjet(medium.table(x, z), th)
    V, A = va(vj, th)
    return V, A, vj


def frame(V):
    nv = np.hypot(V[0], V[1])
    g = V[:2] / nv
    return g, np.array([g[1], -g[0]]), nv


def trace(medium, y0, tau, with_drt=False, d0=None, rtol=1e-11, atol=1e-12, dense=False):
    """Integrate one ray from phase point y0 = (x, z, theta) for time tau
    (negative tau traces backward).  With ``with_drt`` also integrates the
    ray-normal perturbation (dn, dth_perp) from d0."""

    def rhs(t, y):
        V, A, _ = velocity_at(medium, y[0], y[1], y[2])
        out = [V[0], V[1], V[2]]
        if with_drt:
            out += [A[0] * y[3] + A[1] * y[4], A[2] * y[3] + A[3] * y[4]]
        return out

    y = list(y0) + (list(d0) if with_drt else [])
    sol = solve_ivp(rhs, (0.0, tau), y, method="DOP853", rtol=rtol, atol=atol, dense_output=dense)
    if not sol.success:
        raise RuntimeError(sol.message)
    return sol


def normal_components(medium, y_ref, y_pert):
    """(dn, dth_perp) of the phase-space difference y_pert - y_ref in the
    ray-normal frame at y_ref: dn = g_perp.dx, dth_perp = dth - (g.dx) V_t/|V|."""
    V, _, _ = velocity_at(medium, *y_ref)
    g, gp, nv = frame(V)
    d = np.asarray(y_pert) - np.asarray(y_ref)
    dn = gp @ d[:2]
    dtp = d[2] - (g @ d[:2]) * V[2] / nv
    return np.array([dn, dtp])
