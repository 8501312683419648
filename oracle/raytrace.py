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


# ---------------------------------------------------------------------------
# Vectorised rays in an analytic TTI medium, and the continuum point-source
# fields (phi1, psi) they define.

class LinearThomsenMedium:
    """A smooth heterogeneous TTI medium whose medium table is exact under
    4th-order differences: vp0 = v0 + gx (x - xc) + gz (z - zc), constant
    eps, delta and shear ratio fs, tilt nu = nu0 + kx (x - xc) + kz (z - zc).
    Every modulus is vp0^2 times a constant, so all five table fields are
    polynomials of degree <= 2 in position.

    The qP phase velocity is v(x, z, theta) = vp0(x, z) s(theta - nu(x, z))
    with s^2 the larger eigenvalue of the Christoffel matrix (eq. 4) of the
    moduli divided by vp0^2:
      s^2 = (P + sqrt(Q^2 + R^2)) / 2,  P = (c11 + c55) S^2 + (c33 + c55) C^2,
      Q = (c11 - c55) S^2 - (c33 - c55) C^2,  R = 2 c13' S C
    (S, C = sin, cos of the angle from the symmetry axis, c13' = c13 + c55).
    Everything is numpy and elementwise, for many points at once."""

    def __init__(self, centre, v0, gx, gz, eps, delta, nu0=0.0, kx=0.0, kz=0.0, fs=0.5):
        self.xc, self.zc = float(centre[0]), float(centre[1])
        self.v0, self.gx, self.gz = float(v0), float(gx), float(gz)
        self.eps, self.delta, self.fs = float(eps), float(delta), float(fs)
        self.nu0, self.kx, self.kz = float(nu0), float(kx), float(kz)
        c33, c55 = 1.0, fs * fs
        self.c = (c33 * (1 + 2 * eps), c33, np.sqrt((c33 - c55) * (c33 * (1 + 2 * delta) - c55)), c55)

    def vp0(self, x, z):
        return self.v0 + self.gx * (np.asarray(x) - self.xc) + self.gz * (np.asarray(z) - self.zc)

    def nu(self, x, z):
        return self.nu0 + self.kx * (np.asarray(x) - self.xc) + self.kz * (np.asarray(z) - self.zc)

    def gridded(self, xc, zc):
        """(vp0, eps, delta, tilt) sampled on the cell centres xc[i], zc[j]: arrays [nx][nz]."""
        X, Z = np.meshgrid(xc, zc, indexing="ij")
        return self.vp0(X, Z), np.full(X.shape, self.eps), np.full(X.shape, self.delta), self.nu(X, Z)

    def table(self, x, z):
        """The five fields and their derivatives at one point (for trace())."""
        c11, c33, b, c55 = self.c
        vp, nu = float(self.vp0(x, z)), float(self.nu(x, z))
        t = np.zeros((5, 6))
        for f, k in enumerate((c11, c33, b, c55)):
            t[f] = k * np.array([vp * vp, 2 * self.gx * vp, 2 * self.gz * vp, 2 * self.gx ** 2,
                                 2 * self.gx * self.gz, 2 * self.gz ** 2])
        t[4] = [nu, self.kx, self.kz, 0.0, 0.0, 0.0]
        return t

    def shape(self, phi):
        """s(phi) and s'(phi)."""
        c11, c33, b, c55 = self.c
        S, C = np.sin(phi), np.cos(phi)
        S2, C2, s2, c2 = S * S, C * C, 2 * S * C, C * C - S * S
        P = (c11 + c55) * S2 + (c33 + c55) * C2
        Q = (c11 - c55) * S2 - (c33 - c55) * C2
        R = b * s2
        D = np.sqrt(Q * Q + R * R)
        g = 0.5 * (P + D)
        dP, dQ, dR = (c11 - c33) * s2, (c11 + c33 - 2 * c55) * s2, 2 * b * c2
        dg = 0.5 * (dP + (Q * dQ + R * dR) / D)
        s = np.sqrt(g)
        return s, dg / (2 * s)

    def velocity(self, x, z, th):
        """Liouville velocity (V_x, V_z, V_theta) of eqs. 8-9 and 12 and the
        phase velocity v at phase points (arrays)."""
        vp = self.vp0(x, z)
        s, ds = self.shape(th - self.nu(x, z))
        v, vt = vp * s, vp * ds
        vx = self.gx * s - vt * self.kx
        vz = self.gz * s - vt * self.kz
        sn, cs = np.sin(th), np.cos(th)
        return np.stack([v * sn + vt * cs, v * cs - vt * sn, -(vx * cs - vz * sn)]), v


def _rk4(f, y, h):
    k1 = f(y)
    k2 = f(y + 0.5 * h * k1)
    k3 = f(y + 0.5 * h * k2)
    k4 = f(y + h * k3)
    return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def closest_approach_fields(medium, xs, zs, x, z, th, dtau=1e-3, tmax=1.0):
    """The continuum point-source fields at phase points (x, z, theta):
    follow each ray (eqs. 8-9, 12) to the point x_c where it passes closest
    to the source, i.e. where f = (x - x_s).V_xz changes sign, and return
      phi1 = (x_c - x_s).g_perp(x_c)            (signed miss distance),
      psi  = p(theta_c).(x_c - x_s) + tau_c     (traveltime, dpsi/dtau = 1),
    tau_c the ray time from x_c to the point, g_perp = (g_z, -g_x) with g the
    unit ray direction, p = (sin, cos)(theta)/v (eq. 7).  In a homogeneous
    medium this is the point-source data phi1 = (x - x_s).g_perp,
    psi = p.(x - x_s) exactly; in general phi1 is constant along rays and psi
    grows with unit rate, so (phi1, psi) solve the transport equations of
    eqs. 16 and 19, with Gamma = {phi1 = 0} the rays through the source.

    Classical 4th-order Runge-Kutta steps of dtau (toward the closest point:
    backward where f > 0, forward otherwise) until f changes sign, then the
    root within that step by the Illinois variant of regula falsi on single
    Runge-Kutta steps of the trial length from the step's start."""
    y = np.stack([np.asarray(x, dtype=np.float64).ravel(), np.asarray(z, dtype=np.float64).ravel(),
                  np.asarray(th, dtype=np.float64).ravel()])
    n = y.shape[1]
    F = lambda q: medium.velocity(q[0], q[1], q[2])[0]

    def fval(q):
        V = F(q)
        return (q[0] - xs) * V[0] + (q[1] - zs) * V[1]

    f0 = fval(y)
    h = np.where(f0 > 0, -dtau, dtau)
    h[f0 == 0] = 0.0
    start = y.copy()      # state at the start of the bracketing step
    f_end = np.zeros(n)   # f at its end
    t_start = np.zeros(n)
    done = f0 == 0
    cur, t = y.copy(), np.zeros(n)
    for _ in range(int(np.ceil(tmax / dtau))):
        if done.all():
            break
        idx = np.flatnonzero(~done)
        nxt = _rk4(F, cur[:, idx], h[idx])
        fn = fval(nxt)
        crossed = np.sign(fn) != np.sign(f0[idx])
        hit = idx[crossed]
        start[:, hit] = cur[:, hit]
        t_start[hit] = t[hit]
        f_end[hit] = fn[crossed]
        done[hit] = True
        go = idx[~crossed]
        cur[:, go] = nxt[:, ~crossed]
        t[go] += h[go]
    if not done.all():
        raise RuntimeError("closest approach not reached within tmax")
    # Illinois regula falsi on s in [0, h]: f(0) = fa, f(h) = fb of opposite signs
    a, b = np.zeros(n), h.copy()
    fa, fb = fval(start), f_end.copy()
    fb[h == 0] = 1.0
    side = np.zeros(n)
    for _ in range(40):
        den = fb - fa
        c = np.where(den != 0, (a * fb - b * fa) / np.where(den != 0, den, 1.0), a)
        fc = fval(_rk4(F, start, c))
        same_a = np.sign(fc) == np.sign(fa)
        # replace the endpoint of fc's sign; halve the other's value if it was kept twice
        a_new, fa_new = np.where(same_a, c, a), np.where(same_a, fc, fa)
        b_new, fb_new = np.where(same_a, b, c), np.where(same_a, fb, fc)
        fb_new = np.where(same_a & (side == 1), 0.5 * fb_new, fb_new)
        fa_new = np.where(~same_a & (side == -1), 0.5 * fa_new, fa_new)
        side = np.where(same_a, 1, -1)
        a, fa, b, fb = a_new, fa_new, b_new, fb_new
        if np.all(np.abs(b - a) <= 1e-15 + 1e-13 * np.abs(h)):
            break
    s = np.where(np.abs(fa) <= np.abs(fb), a, b)
    s[h == 0] = 0.0
    yc = _rk4(F, start, s)
    tc = t_start + s                       # ray time of x_c relative to the point (<= 0 backward)
    V, v = medium.velocity(yc[0], yc[1], yc[2])
    nv = np.hypot(V[0], V[1])
    gx, gz = V[0] / nv, V[1] / nv
    dxc, dzc = yc[0] - xs, yc[1] - zs
    phi1 = dxc * gz - dzc * gx
    psi = (np.sin(yc[2]) * dxc + np.cos(yc[2]) * dzc) / v - tc
    shape = np.shape(x)
    return phi1.reshape(shape), psi.reshape(shape)


class GaussianLensMedium:
    """Isotropic v(x, z) = v0 + a exp(-|x - c|^2 / (2 sigma^2)) (a < 0: a
    low-velocity lens that focuses rays and makes caustics behind it), with
    the Liouville velocity of eqs. 8-9 and 12 in closed form:
    V = (v sin, v cos, -(v_x cos - v_z sin))."""

    def __init__(self, v0, a, cx, cz, sigma):
        self.v0, self.a, self.cx, self.cz, self.sig = float(v0), float(a), float(cx), float(cz), float(sigma)

    def vgrad(self, x, z):
        e = self.a * np.exp(-((x - self.cx) ** 2 + (z - self.cz) ** 2) / (2 * self.sig ** 2))
        return self.v0 + e, -e * (x - self.cx) / self.sig ** 2, -e * (z - self.cz) / self.sig ** 2

    def velocity(self, x, z, th):
        v, vx, vz = self.vgrad(x, z)
        sn, cs = np.sin(th), np.cos(th)
        return np.stack([v * sn, v * cs, -(vx * cs - vz * sn)]), v

    def table(self, x, z, fs=0.5):
        """The five fields and their derivatives at one point (for trace()):
        isotropic, a11 = a33 = v^2, a55 = (fs v)^2, a13 + a55 = a33 - a55."""
        v, vx, vz = self.vgrad(x, z)
        e = self.a * np.exp(-((x - self.cx) ** 2 + (z - self.cz) ** 2) / (2 * self.sig ** 2))
        s2 = self.sig ** 2
        vxx = e * ((x - self.cx) ** 2 / s2 - 1.0) / s2
        vzz = e * ((z - self.cz) ** 2 / s2 - 1.0) / s2
        vxz = e * (x - self.cx) * (z - self.cz) / s2 ** 2
        sq = np.array([v * v, 2 * v * vx, 2 * v * vz, 2 * (vx * vx + v * vxx), 2 * (vx * vz + v * vxz),
                       2 * (vz * vz + v * vzz)])
        t = np.zeros((5, 6))
        for f, k in enumerate((1.0, 1.0, 1.0 - fs * fs, fs * fs)):
            t[f] = k * sq
        return t


def continuous_phase_of_c(medium, y0, tau, beta, s=1.0, n=400):
    """The continuous phase of the ray-normal DRT amplitude C along the ray
    from the source point y0 = (x_s, z_s, take-off angle) for time tau:
    (C, B)(0) = (s, i beta s) (the point-source data at the source), carried
    by d(C, B)/dtau = A (C, B) (real A, so the propagator of the two real
    unit starts gives C), arg C unwrapped over n samples."""
    sol1 = trace(medium, y0, tau, with_drt=True, d0=(1.0, 0.0), dense=True)
    sol2 = trace(medium, y0, tau, with_drt=True, d0=(0.0, 1.0), dense=True)
    t = np.linspace(0.0, tau, n)
    C = s * (sol1.sol(t)[3] + 1j * beta * sol2.sol(t)[3])
    return float(np.unwrap(np.angle(C))[-1])


def fan_crossings(medium, xs, zs, take_off, z_line, dtau=1e-3, tmax=5.0):
    """Shoot rays from the source (x_s, z_s) at the phase angles `take_off`
    (classical Runge-Kutta steps of dtau) and return, per ray, where it
    first crosses the depth z_line going down: x, the phase angle theta and
    the traveltime (linear between the two steps around the crossing); NaN
    for rays that have not crossed within tmax."""
    th0 = np.asarray(take_off, dtype=np.float64)
    y = np.stack([np.full_like(th0, xs), np.full_like(th0, zs), th0])
    F = lambda q: medium.velocity(q[0], q[1], q[2])[0]
    out = np.full((3, th0.size), np.nan)
    done = np.zeros(th0.size, bool)
    t = 0.0
    for _ in range(int(np.ceil(tmax / dtau))):
        yn = _rk4(F, y, dtau)
        cr = (~done) & (yn[1] >= z_line) & (y[1] < z_line)
        f = (z_line - y[1][cr]) / (yn[1][cr] - y[1][cr])
        out[0, cr] = y[0][cr] + f * (yn[0][cr] - y[0][cr])
        out[1, cr] = y[2][cr] + f * (yn[2][cr] - y[2][cr])
        out[2, cr] = t + f * dtau
        done |= cr
        y, t = yn, t + dtau
        if done.all():
            break
    return out
