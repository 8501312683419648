"""Traveltime-misfit gradients by automatic differentiation (test
infrastructure only).

The kinematic part of the oracle's scheme -- medium table (values and first
derivatives), the Liouville velocity V (eqs. 8-9, 12), the point-source data
for phi1 and psi, the WENO5 / SSP-RK3 march of phi1 and psi, the receiver pick
(eq. 35) -- written again with PyTorch float64 CPU tensors, so that autograd
returns the exact gradient of the discrete misfit
    J = sum_r (psi_pick,r - psi_obs,r)^2
with respect to the gridded vp0, eps, delta and tilt.  phi1 and psi do not
depend on the dynamic-ray-tracing pair (C, B), so those planes are left out.
The time step is an input (held fixed under perturbations of the medium).

Checked against the C oracle (same fields to rounding) and against central
differences of J computed by the C oracle.
"""
from __future__ import annotations

import numpy as np
import torch

T = torch.float64

# 4th-order first-derivative weights: central (-2..2); one-sided at the first
# two points (offsets 0..4 and -1..3); mirrored with a sign change at the end.
W1C = [1.0, -8.0, 0.0, 8.0, -1.0]
W1E0 = [-25.0, 48.0, -36.0, 16.0, -3.0]
W1E1 = [-3.0, -10.0, 18.0, -6.0, 1.0]


def d1_matrix(n: int, h: float) -> torch.Tensor:
    D = torch.zeros((n, n), dtype=T)
    for i in range(n):
        if 2 <= i <= n - 3:
            for m, w in enumerate(W1C):
                D[i, i - 2 + m] = w
        else:
            lo = i < 2
            e = i if lo else n - 1 - i
            w = W1E0 if e == 0 else W1E1
            sgn = 1.0 if lo else -1.0
            for m in range(5):
                off = -e + m
                j = i + off if lo else i - off
                D[i, j] = sgn * w[m]
    return D / (12.0 * h)


def medium_fields(vp0, eps, delta, tilt, fs):
    a33 = vp0 * vp0
    a55 = fs * fs * a33
    a11 = a33 * (1 + 2 * eps)
    b = torch.sqrt((a33 - a55) * (a33 * (1 + 2 * delta) - a55))
    return [a11, a33, b, a55, tilt]


def table1(fields, dx, dz):
    """Values and first derivatives (f, f_x, f_z) of each field, [nx][nz]."""
    nx, nz = fields[0].shape
    Dx, Dz = d1_matrix(nx, dx), d1_matrix(nz, dz)
    return [(f, Dx @ f, f @ Dz.T) for f in fields]


class J1:
    """First-order jet in (x, z, theta): value and gradient."""

    def __init__(self, f, g):
        self.f, self.g = f, g

    def __add__(self, o):
        return J1(self.f + o.f, [a + b for a, b in zip(self.g, o.g)])

    def __sub__(self, o):
        return J1(self.f - o.f, [a - b for a, b in zip(self.g, o.g)])

    def __mul__(self, o):
        return J1(self.f * o.f, [self.f * b + o.f * a for a, b in zip(self.g, o.g)])

    def scale(self, s):
        return J1(self.f * s, [a * s for a in self.g])

    def chain(self, f0, f1):
        return J1(f0, [f1 * a for a in self.g])


def jsqrt(a: J1):
    r = torch.sqrt(a.f)
    return a.chain(r, 0.5 / r)


def phase_velocity_j1(tab, theta):
    """v and its gradient (v_x, v_z, v_theta) from the Christoffel qP eigenvalue
    (eqs. 3-4) for every cell; theta broadcasts as [nth][1][1]."""
    zero = torch.zeros_like(tab[0][0])
    fj = [J1(f, [fx, fz, zero]) for (f, fx, fz) in tab]
    a11, a33, b, a55, nu = fj
    phi = J1(theta - nu.f, [-nu.g[0], -nu.g[1], torch.ones_like(theta - nu.f)])
    n1 = phi.chain(torch.sin(phi.f), torch.cos(phi.f))
    n3 = phi.chain(torch.cos(phi.f), -torch.sin(phi.f))
    g11 = a11 * (n1 * n1) + a55 * (n3 * n3)
    g33 = a55 * (n1 * n1) + a33 * (n3 * n3)
    g13 = b * (n1 * n3)
    d = g11 - g33
    G = (g11 + g33 + jsqrt(d * d + (g13 * g13).scale(4.0))).scale(0.5)
    return jsqrt(G)


def velocity(tab, nth):
    th = (torch.arange(nth, dtype=T) * (2 * np.pi / nth))[:, None, None]
    v = phase_velocity_j1(tab, th)
    s, c = torch.sin(th), torch.cos(th)
    Vx = v.f * s + v.g[2] * c
    Vz = v.f * c - v.g[2] * s
    Vt = -(v.g[0] * c - v.g[1] * s)
    return Vx, Vz, Vt


def bilinear_at(f, g, x, z):
    fx = (x - g.x0) / g.dx - 0.5
    fz = (z - g.z0) / g.dz - 0.5
    ix = int(np.clip(np.floor(fx), 0, g.nx - 2))
    iz = int(np.clip(np.floor(fz), 0, g.nz - 2))
    tx = float(np.clip(fx - ix, 0.0, 1.0))
    tz = float(np.clip(fz - iz, 0.0, 1.0))
    return ((1 - tx) * (1 - tz) * f[ix, iz] + tx * (1 - tz) * f[ix + 1, iz] + (1 - tx) * tz * f[ix, iz + 1]
            + tx * tz * f[ix + 1, iz + 1])


def init_kinematic(tab, g, src):
    """phi1 = (x - xs).g_perp(theta), psi = p(theta).(x - xs) with the medium
    frozen (bilinear) at the source."""
    ms = [bilinear_at(f, g, src.xs, src.zs) for (f, _, _) in tab]
    th = (torch.arange(g.nth, dtype=T) * (2 * np.pi / g.nth))
    zero = torch.zeros_like(th)
    tab_s = [(m + zero, zero, zero) for m in ms]
    v = phase_velocity_j1(tab_s, th)
    s, c = torch.sin(th), torch.cos(th)
    Vx = v.f * s + v.g[2] * c
    Vz = v.f * c - v.g[2] * s
    nv = torch.sqrt(Vx * Vx + Vz * Vz)
    gpx, gpz = Vz / nv, -Vx / nv
    px, pz = s / v.f, c / v.f
    X = torch.as_tensor(g.xc() - src.xs, dtype=T)[None, :, None]
    Z = torch.as_tensor(g.zc() - src.zs, dtype=T)[None, None, :]
    phi = X * gpx[:, None, None] + Z * gpz[:, None, None]
    psi = X * px[:, None, None] + Z * pz[:, None, None]
    return phi, psi


def weno(u7, minus):
    """WENO5 HJ undivided derivative from u7 = [7, ...] at offsets -3..3;
    `minus` (bool tensor) selects D-.  0 where all differences vanish."""
    dm = [u7[m + 1] - u7[m] for m in range(5)]          # D- differences v1..v5
    dp = [u7[6 - m] - u7[5 - m] for m in range(5)]      # D+ differences v1..v5
    v = [torch.where(minus, a, b) for a, b in zip(dm, dp)]
    # evaluated on v / max|v| and scaled back (W is 1-homogeneous): the same
    # value without overflow of 1 / (e + s)^2 for tiny differences
    am = torch.stack([x.abs() for x in v]).amax(0)
    ok = am > 0
    ams = torch.where(ok, am, torch.ones_like(am))
    v = [torch.where(ok, x / ams, torch.ones_like(x)) for x in v]
    v1, v2, v3, v4, v5 = v
    mxs = torch.stack([x * x for x in v]).amax(0)
    q0 = v1 / 3 - 7 * v2 / 6 + 11 * v3 / 6
    q1 = -v2 / 6 + 5 * v3 / 6 + v4 / 3
    q2 = v3 / 3 + 5 * v4 / 6 - v5 / 6
    s0 = 13 / 12 * (v1 - 2 * v2 + v3) ** 2 + 0.25 * (v1 - 4 * v2 + 3 * v3) ** 2
    s1 = 13 / 12 * (v2 - 2 * v3 + v4) ** 2 + 0.25 * (v2 - v4) ** 2
    s2 = 13 / 12 * (v3 - 2 * v4 + v5) ** 2 + 0.25 * (3 * v3 - 4 * v4 + v5) ** 2
    e = 1e-6 * mxs
    a0, a1, a2 = 0.1 / (e + s0) ** 2, 0.6 / (e + s1) ** 2, 0.3 / (e + s2) ** 2
    w = ams * ((a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2))
    return torch.where(ok, w, torch.zeros_like(w))


def _stencil_xz(u, b, axis):
    """[7, ...] values at offsets -3..3 along axis 1 (x) or 2 (z); ghosts are
    the point-source data b of the plane extended by linear extrapolation
    b_{-m} = (m+1) b_0 - m b_1 (fixed in time)."""
    n = u.shape[axis]
    sl = lambda i: b.narrow(axis, i, 1)
    lo = [(m + 1) * sl(0) - m * sl(1) for m in (3, 2, 1)]
    hi = [(m + 1) * sl(n - 1) - m * sl(n - 2) for m in (1, 2, 3)]
    ext = torch.cat(lo + [u] + hi, dim=axis)
    return torch.stack([ext.narrow(axis, 3 + o, n) for o in range(-3, 4)])


def _stencil_t(u):
    return torch.stack([torch.roll(u, -o, dims=0) for o in range(-3, 4)])


def rhs(phi, psi, V, g, bc):
    Vx, Vz, Vt = V
    cx, cz, ct = Vx / g.dx, Vz / g.dz, Vt / g.dth
    out = []
    for u, b in zip((phi, psi), bc):
        L = -(cx * weno(_stencil_xz(u, b, 1), cx >= 0) + cz * weno(_stencil_xz(u, b, 2), cz >= 0)
              + ct * weno(_stencil_t(u), ct >= 0))
        out.append(L)
    out[1] = out[1] + 1.0
    return out


def march(phi, psi, V, g, src, dt, nsteps, bc=None):
    """bc: the point-source data (phi1, psi) that the ghosts extend; the
    starting state when None."""
    bc = (phi, psi) if bc is None else bc
    X = torch.as_tensor(g.xc() - src.xs, dtype=T)[:, None]
    Z = torch.as_tensor(g.zc() - src.zs, dtype=T)[None, :]
    ball = (X * X + Z * Z <= src.r0 ** 2)[None, :, :]
    ca, cb = (0.0, 0.75, 1.0 / 3.0), (1.0, 0.25, 2.0 / 3.0)
    for _ in range(nsteps):
        u0 = (phi, psi)
        ui = u0
        for st in range(3):
            L = rhs(ui[0], ui[1], V, g, bc)
            new = []
            for f in range(2):
                y = ca[st] * u0[f] + cb[st] * (ui[f] + dt * L[f])
                new.append(torch.where(ball, u0[f], y))
            ui = tuple(new)
        phi, psi = ui
    return phi, psi


def pick(phi, psi, g, rx):
    """First-arrival pick (see the C oracle); returns (t [nr], valid [nr])."""
    out, valid = [], []
    for (x, z) in np.asarray(rx, dtype=np.float64).reshape(-1, 2):
        ph = torch.stack([bilinear_at(phi[k], g, x, z) for k in range(g.nth)])
        ps = torch.stack([bilinear_at(psi[k], g, x, z) for k in range(g.nth)])
        ph1, ps1 = torch.roll(ph, -1), torch.roll(ps, -1)
        root = (ph == 0) | (ph * ph1 < 0)
        den = torch.where(root, ph - ph1, torch.ones_like(ph))
        t = torch.where(root, ph / den, torch.zeros_like(ph))
        val = ps + t * (ps1 - ps)
        cand = root & (val > 0)
        if not bool(cand.any()):
            out.append(torch.zeros((), dtype=T))
            valid.append(False)
            continue
        masked = torch.where(cand, val, torch.full_like(val, float("inf")))
        k = int(torch.argmin(masked))
        out.append(val[k])
        valid.append(True)
    return torch.stack(out), np.array(valid)


def misfit(problem, medium_tensors, rx, t_obs, dt, nsteps):
    """J and the picked times for the given (vp0, eps, delta, tilt) tensors."""
    g, src = problem.grid, problem.source
    vp0, eps, dlt, tilt = medium_tensors
    tab = table1(medium_fields(vp0, eps, dlt, tilt, problem.medium.vs_ratio), g.dx, g.dz)
    V = velocity(tab, g.nth)
    phi, psi = init_kinematic(tab, g, src)
    phi, psi = march(phi, psi, V, g, src, dt, nsteps)
    t, valid = pick(phi, psi, g, rx)
    tv = t[torch.as_tensor(valid)]
    ov = torch.as_tensor(np.asarray(t_obs)[valid], dtype=T)
    return torch.sum((tv - ov) ** 2), t, valid, (phi, psi)


def gradient(problem, rx, t_obs, dt, nsteps):
    """(J, dJ/dvp0, dJ/deps, dJ/ddelta, dJ/dtilt) as numpy arrays."""
    m = problem.medium
    ts = [torch.tensor(np.asarray(a, dtype=np.float64), dtype=T, requires_grad=True)
          for a in (m.vp0, m.eps, m.delta, m.tilt)]
    J, _, _, _ = misfit(problem, ts, rx, t_obs, dt, nsteps)
    grads = torch.autograd.grad(J, ts)
    return float(J.detach()), [gr.numpy() for gr in grads]
