"""Seeded synthetic inputs for the Eulerian Gaussian beam hot path.

This module only draws random media, grids, sources and receiver sets. It holds
none of the method's arithmetic (no Christoffel matrix, no velocities, no
scheme), so both the FP64 oracle and the HIP path can take their inputs from
here without sharing any computation.

The paper (theory only, Sec. 1) measures nothing, so every workload is
synthetic:

* ``homog_iso_64``: homogeneous isotropic medium, v = 2000 m/s, 1 km square,
  64^3 phase grid, 100 SSP-RK3 steps, one frequency (20 Hz), FP64 end to end.
* ``vti_256``: heterogeneous VTI, vp0 = 3000 m/s + 8 Gaussian blobs
  (+-1000 m/s, sigma 100-300 m), smoothed random epsilon in [0, 0.3] and delta
  in [-0.1, 0.2], 4 km square, 256^3, 600 steps, 32 frequencies 5-60 Hz, FP32.
* ``tti_512``: the VTI recipe at 512^2 plus a smoothed random tilt in
  [-45, 45] deg, 512^3, 1200 steps, 64 frequencies.
* ``batch_uneven``: 64 independent VTI-recipe problems with per-axis sizes
  drawn uniformly from 128..384, 400 steps each.
* ``adjoint_sources``: VTI medium, 16 sources at z = 0.1 L and 128 receivers
  at z = 0.9 L; observed traveltimes come from a perturbed model
  (vp0 +-5 %, eps +-0.05).

Units: metres, seconds, radians.  Arrays are float64, indexed [ix][iz]
(z fastest), sampled at cell centres x_i = x0 + (i + 1/2) dx.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter

SEED_BASE = 20061194


def rng_for(kind: int, src: int = 0) -> np.random.Generator:
    """Seeded generator for workload family ``kind`` (0 homogeneous, 1 VTI,
    2 TTI, 3 batched, 4 adjoint) and source ``src``."""
    return np.random.default_rng(SEED_BASE + 1000 * kind + src)


@dataclass
class Grid:
    nx: int
    nz: int
    nth: int
    dx: float
    dz: float
    x0: float = 0.0
    z0: float = 0.0

    @property
    def dth(self) -> float:
        return 2.0 * np.pi / self.nth

    def xc(self) -> np.ndarray:
        return self.x0 + (np.arange(self.nx) + 0.5) * self.dx

    def zc(self) -> np.ndarray:
        return self.z0 + (np.arange(self.nz) + 0.5) * self.dz

    def th(self) -> np.ndarray:
        return np.arange(self.nth) * self.dth

    @property
    def ncell(self) -> int:
        return self.nx * self.nz * self.nth


@dataclass
class Medium:
    vp0: np.ndarray
    eps: np.ndarray
    delta: np.ndarray
    tilt: np.ndarray
    vs_ratio: float = 0.5


@dataclass
class Source:
    xs: float
    zs: float
    r0: float
    beta: float


@dataclass
class Problem:
    name: str
    grid: Grid
    medium: Medium
    source: Source
    nsteps: int
    omegas: np.ndarray
    dtype: str = "f32"           # "f32" (psi kept in f64) or "f64"
    receivers: Optional[np.ndarray] = None   # [nr][2] (x, z)
    extra: dict = field(default_factory=dict)


def square_grid(n: int, L: float, nth: Optional[int] = None) -> Grid:
    return Grid(nx=n, nz=n, nth=n if nth is None else nth, dx=L / n, dz=L / n)


def _rescale(f: np.ndarray, lo: float, hi: float) -> np.ndarray:
    mn, mx = float(f.min()), float(f.max())
    if mx == mn:
        return np.full_like(f, 0.5 * (lo + hi))
    return lo + (f - mn) / (mx - mn) * (hi - lo)


def _smoothed_uniform(rng: np.random.Generator, g: Grid, sigma_m: float,
                      lo: float, hi: float) -> np.ndarray:
    raw = rng.uniform(0.0, 1.0, size=(g.nx, g.nz))
    sm = gaussian_filter(raw, sigma=(sigma_m / g.dx, sigma_m / g.dz), mode="reflect")
    return _rescale(sm, lo, hi)


def blob_velocity(rng: np.random.Generator, g: Grid, L: float, nblob: int = 8,
                  base: float = 3000.0, amp: float = 1000.0,
                  sig_lo: float = 100.0, sig_hi: float = 300.0,
                  vmin: float = 1000.0) -> np.ndarray:
    """vp0 = base + sum of Gaussian blobs, clamped at vmin."""
    X, Z = np.meshgrid(g.xc(), g.zc(), indexing="ij")
    v = np.full((g.nx, g.nz), base)
    for _ in range(nblob):
        cx, cz = rng.uniform(g.x0, g.x0 + L), rng.uniform(g.z0, g.z0 + L)
        a = rng.uniform(-amp, amp)
        s = rng.uniform(sig_lo, sig_hi)
        v += a * np.exp(-((X - cx) ** 2 + (Z - cz) ** 2) / (2.0 * s * s))
    return np.maximum(v, vmin)


def vti_medium(rng: np.random.Generator, g: Grid, L: float, tilt: bool = False,
               smooth_m: float = 200.0, vs_ratio: float = 0.5) -> Medium:
    """The heterogeneous VTI recipe (optionally with a smooth random tilt)."""
    vp0 = blob_velocity(rng, g, L)
    eps = _smoothed_uniform(rng, g, smooth_m, 0.0, 0.3)
    dlt = _smoothed_uniform(rng, g, smooth_m, -0.1, 0.2)
    if tilt:
        nu = _smoothed_uniform(rng, g, smooth_m, -np.pi / 4, np.pi / 4)
    else:
        nu = np.zeros((g.nx, g.nz))
    return Medium(vp0=vp0, eps=eps, delta=dlt, tilt=nu, vs_ratio=vs_ratio)


def homogeneous(g: Grid, v: float, eps: float = 0.0, delta: float = 0.0,
                tilt: float = 0.0, vs_ratio: float = 0.5) -> Medium:
    s = (g.nx, g.nz)
    return Medium(vp0=np.full(s, v), eps=np.full(s, eps), delta=np.full(s, delta),
                  tilt=np.full(s, tilt), vs_ratio=vs_ratio)


def gradient_medium(g: Grid, v0: float, grad: float, zref: float) -> Medium:
    """Isotropic v(z) = v0 + grad * (z - zref)."""
    Z = np.broadcast_to(g.zc()[None, :], (g.nx, g.nz))
    v = v0 + grad * (Z - zref)
    s = (g.nx, g.nz)
    return Medium(vp0=np.array(v, dtype=np.float64), eps=np.zeros(s), delta=np.zeros(s),
                  tilt=np.zeros(s), vs_ratio=0.5)


def centre_source(g: Grid, L: float, r0_cells: float = 4.0) -> Source:
    return Source(xs=g.x0 + 0.5 * L, zs=g.z0 + 0.5 * L, r0=r0_cells * g.dx,
                  beta=1.0 / (2.0 * L))


def hz(f) -> np.ndarray:
    return 2.0 * np.pi * np.asarray(f, dtype=np.float64)


# ---------------------------------------------------------------- workloads

def homog_iso_64(n: int = 64, nsteps: int = 100) -> Problem:
    L = 1000.0
    g = square_grid(n, L)
    return Problem("homog-iso-64", g, homogeneous(g, 2000.0), centre_source(g, L),
                   nsteps, hz([20.0]), dtype="f64")


def vti_256(n: int = 256, nsteps: int = 600, L: Optional[float] = None, nw: int = 32,
            src: int = 0, nth: Optional[int] = None) -> Problem:
    """Heterogeneous VTI.  ``n``/``L`` can be shrunk for parity-size runs."""
    L = 4000.0 if L is None else L
    g = square_grid(n, L, nth)
    rng = rng_for(1, src)
    med = vti_medium(rng, g, L)
    return Problem(f"vti-{n}", g, med, centre_source(g, L), nsteps,
                   hz(np.linspace(5.0, 60.0, nw)), dtype="f32")


def tti_512(n: int = 512, nsteps: int = 1200, L: Optional[float] = None, nw: int = 64,
            nth: Optional[int] = None) -> Problem:
    L = 4000.0 if L is None else L
    g = square_grid(n, L, nth)
    rng = rng_for(2, 0)
    med = vti_medium(rng, g, L, tilt=True)
    return Problem(f"tti-{n}", g, med, centre_source(g, L), nsteps,
                   hz(np.linspace(5.0, 60.0, nw)), dtype="f32")


def batch_uneven(nprob: int = 64, nsteps: int = 400, lo: int = 128, hi: int = 384,
                 L: float = 4000.0) -> List[Problem]:
    """Independent VTI-recipe problems with per-axis sizes drawn from lo..hi."""
    out = []
    for s in range(nprob):
        rng = rng_for(3, s)
        nx, nz, nth = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        g = Grid(nx=nx, nz=nz, nth=nth, dx=L / nx, dz=L / nz)
        med = vti_medium(rng, g, L)
        src = Source(xs=0.5 * L, zs=0.5 * L, r0=4.0 * max(g.dx, g.dz), beta=1.0 / (2.0 * L))
        out.append(Problem(f"batch-{s}", g, med, src, nsteps, hz([20.0]), dtype="f32"))
    return out


def smooth_field(rng: np.random.Generator, g: Grid, sigma_m: float = 300.0) -> np.ndarray:
    """Smooth seeded field in [-1, 1]."""
    return _smoothed_uniform(rng, g, sigma_m, -1.0, 1.0)


def adjoint_sources(n: int = 256, nsteps: int = 600, L: float = 4000.0, nsrc: int = 16, nrec: int = 128,
       nth: Optional[int] = None) -> List[Problem]:
    """Adjoint workload: shared medium, many sources, receivers at depth.

    ``extra['true_medium']`` holds the perturbed model that produces the
    observed traveltimes.
    """
    g = square_grid(n, L, nth)
    rng = rng_for(4, 0)
    med = vti_medium(rng, g, L)
    q1, q2 = smooth_field(rng, g), smooth_field(rng, g)
    true = replace(med, vp0=med.vp0 * (1.0 + 0.05 * q1), eps=med.eps + 0.05 * q2)
    xs = np.linspace(0.1 * L, 0.9 * L, nsrc)
    rx = np.stack([np.linspace(0.1 * L, 0.9 * L, nrec), np.full(nrec, 0.9 * L)], axis=1)
    out = []
    for s in range(nsrc):
        src = Source(xs=float(xs[s]), zs=0.1 * L, r0=4.0 * g.dx, beta=1.0 / (2.0 * L))
        out.append(Problem(f"adjoint-src-{s}", g, med, src, nsteps, hz([20.0]), dtype="f32",
                           receivers=rx, extra={"true_medium": true}))
    return out
