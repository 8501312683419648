"""Green's-function migration on the depth march's wavefields: single-
scattering (Born) data of a reflectivity and its adjoint, the image.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper ends with migration as the application of its Green's functions
(section 6) but fixes no imaging condition.  Here, with G(x; y, omega) the
Green's function of a surface point y (one depth march serves every y,
eqs. 34-35):

  Born data    d[w][s][r] = omega_w^2 dA sum_x G[s][w][x] m[x] G[r][w][x]
  image        I[x] = Re sum_w omega_w^2 dA sum_{s,r} conj(G[s][w][x])
                      conj(G[r][w][x]) d[w][s][r]

(sources s and receivers r on the same surface points, dA = dx dz), so that
the image is the exact adjoint of the data for a real reflectivity:
Re <B m, d> = <m, I(d)>.  Written as plain sums (einsum), no blocking.
"""
from __future__ import annotations

import numpy as np


def born_data(G: np.ndarray, m: np.ndarray, omegas, dA: float) -> np.ndarray:
    """G [ns][nw][nx][nz] complex, m [nx][nz] real -> d [nw][ns][ns] complex."""
    om = np.asarray(omegas, dtype=np.float64)
    Gm = G * m[None, None]
    d = np.einsum("swxz,rwxz->wsr", Gm, G)
    return (om ** 2)[:, None, None] * dA * d


def migrate(G: np.ndarray, d: np.ndarray, omegas, dA: float) -> np.ndarray:
    """G [ns][nw][nx][nz], d [nw][ns][ns] -> image [nx][nz] (real)."""
    om = np.asarray(omegas, dtype=np.float64)
    Gc = np.conj(G)
    q = np.einsum("wsr,rwxz->swxz", d, Gc)          # sum over receivers
    img = np.einsum("swxz,swxz->wxz", Gc, q)        # then over sources
    return np.real(np.einsum("w,wxz->xz", om ** 2 * dA, img))
