"""Closed-form results that pin the oracle (test infrastructure only).

These are textbook results, independent of the Eulerian scheme:

* straight-ray traveltime |x - xs| / v in a homogeneous isotropic medium;
* elliptic (eps = delta) traveltime sqrt(x'^2/v_h^2 + z'^2/v_z^2) with the
  coordinates rotated into the symmetry frame by the tilt nu (measured from
  +z toward +x), v_h = v_z sqrt(1 + 2 eps);
* the constant-gradient traveltime T = arccosh(1 + g^2 r^2 / (2 v_s v_r)) / g
  for v = v0 + g z (circular rays);
* the 2D Green's functions with time dependence exp(-i omega t) (paper eq. 2):
  (i/4) H0^(1)(omega r / v) for (Laplacian + omega^2/v^2) G = -delta, and
  (i/4)(v_z/v_h) H0^(1)(omega T_ell) for the elliptic operator
  ((v_h^2 d_xx + v_z^2 d_zz) / v_z^2 + omega^2 / v_z^2) G = -delta (tilted by nu);
* the far-field of the same normalisation for a general homogeneous
  anisotropic medium with slowness curve G(p) = 1 (stationary phase of the
  plane-wave integral):
  G ~ (i/4pi) a33 sqrt(2 pi / (omega R phi_g' v^2 |V|)) exp(i(omega T - pi/4)),
  where the ray with phase angle theta points at the receiver, phi_g' is the
  derivative of the ray angle with respect to the phase angle, v the phase and
  |V| the group speed.
"""
from __future__ import annotations

import numpy as np
from scipy.special import hankel1


def t_straight(x, z, xs, zs, v):
    return np.hypot(np.asarray(x) - xs, np.asarray(z) - zs) / v


def t_elliptic(x, z, xs, zs, vz, eps, tilt=0.0):
    vh = vz * np.sqrt(1.0 + 2.0 * eps)
    dx, dz = np.asarray(x) - xs, np.asarray(z) - zs
    xr = dx * np.cos(tilt) - dz * np.sin(tilt)
    zr = dx * np.sin(tilt) + dz * np.cos(tilt)
    return np.sqrt(xr ** 2 / vh ** 2 + zr ** 2 / vz ** 2)


def t_gradient(x, z, xs, zs, v0, g, zref):
    """First-arrival traveltime for v(z) = v0 + g (z - zref)."""
    vs = v0 + g * (zs - zref)
    vr = v0 + g * (np.asarray(z) - zref)
    r2 = (np.asarray(x) - xs) ** 2 + (np.asarray(z) - zs) ** 2
    return np.arccosh(1.0 + g * g * r2 / (2.0 * vs * vr)) / g


def green_iso(x, z, xs, zs, v, omega):
    r = np.hypot(np.asarray(x) - xs, np.asarray(z) - zs)
    return 0.25j * hankel1(0, omega * r / v)


def green_elliptic(x, z, xs, zs, vz, eps, omega, tilt=0.0):
    vh = vz * np.sqrt(1.0 + 2.0 * eps)
    return 0.25j * (vz / vh) * hankel1(0, omega * t_elliptic(x, z, xs, zs, vz, eps, tilt))


def thomsen_phase_velocity(theta, vp0, eps, delta, fs=0.5, tilt=0.0):
    """qP phase velocity of a 2D TTI medium from the largest eigenvalue of the
    Christoffel matrix, computed with numpy's symmetric eigen-solver (a library
    routine independent of the oracle's closed-form root)."""
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64)) - tilt
    a33 = vp0 ** 2
    a55 = (fs * vp0) ** 2
    a11 = a33 * (1 + 2 * eps)
    a13 = np.sqrt((a33 - a55) * (a33 * (1 + 2 * delta) - a55)) - a55
    n1, n3 = np.sin(th), np.cos(th)
    M = np.empty(th.shape + (2, 2))
    M[..., 0, 0] = a11 * n1 ** 2 + a55 * n3 ** 2
    M[..., 1, 1] = a55 * n1 ** 2 + a33 * n3 ** 2
    M[..., 0, 1] = M[..., 1, 0] = (a13 + a55) * n1 * n3
    return np.sqrt(np.linalg.eigvalsh(M)[..., -1])


def green_aniso_far(R_dir_theta, R, omega, vp0, eps, delta, fs=0.5, tilt=0.0, h=1e-5):
    """Far-field Green's function along the ray of phase angle theta at distance R
    (see module docstring).  Returns (x, z) of the receiver relative to the
    source and the complex value."""
    th = float(R_dir_theta)

    def vel(t):
        return float(thomsen_phase_velocity(t, vp0, eps, delta, fs, tilt)[0])

    def group(t):
        v = vel(t)
        vt = (vel(t + h) - vel(t - h)) / (2 * h)
        return np.array([v * np.sin(t) + vt * np.cos(t), v * np.cos(t) - vt * np.sin(t)])

    Vg = group(th)
    phig = lambda t: np.arctan2(*group(t))
    dphig = (phig(th + h) - phig(th - h)) / (2 * h)
    v = vel(th)
    nV = np.linalg.norm(Vg)
    x = R * Vg / nV
    T = R / nV * 1.0  # along the ray tau = R / |V| and p.V = 1
    p = np.array([np.sin(th), np.cos(th)]) / v
    T = float(p @ x)
    a33 = vp0 ** 2
    amp = a33 / (4 * np.pi) * np.sqrt(2 * np.pi / (omega * R * dphig * v * v * nV))
    return x, 1j * amp * np.exp(1j * (omega * T - np.pi / 4))


def qp_polarization(theta, vp0, eps, delta, fs=0.5, tilt=0.0):
    """qP polarisation vector (g_x, g_z) of a 2D TTI medium: the eigenvector of
    the lab-frame Christoffel matrix Gamma_ik = c_ijkl n_j n_l for its largest
    eigenvalue (numpy's symmetric eigen-solver), the stiffness rotated from
    the symmetry frame by the tilt, signed along the phase direction n."""
    a33 = vp0 ** 2
    a55 = (fs * vp0) ** 2
    a11 = a33 * (1 + 2 * eps)
    a13 = np.sqrt((a33 - a55) * (a33 * (1 + 2 * delta) - a55)) - a55
    n = np.array([np.sin(theta), np.cos(theta)])
    # rotation taking symmetry-frame vectors (angle from z toward x) to the lab frame
    c, s = np.cos(tilt), np.sin(tilt)
    Rm = np.array([[c, s], [-s, c]])
    npr = Rm.T @ n
    G = np.array([[a11 * npr[0] ** 2 + a55 * npr[1] ** 2, (a13 + a55) * npr[0] * npr[1]],
                  [(a13 + a55) * npr[0] * npr[1], a55 * npr[0] ** 2 + a33 * npr[1] ** 2]])
    w, V = np.linalg.eigh(Rm @ G @ Rm.T)
    g = V[:, -1]
    return g if g @ n >= 0 else -g
