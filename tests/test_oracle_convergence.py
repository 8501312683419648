"""The march converges to the continuum solution at the scheme's order.

Continuum (the definition): in a smooth heterogeneous TTI medium the
point-source fields phi1 (signed miss distance of the ray from the source)
and psi (traveltime) are carried along the rays of eqs. 8-9 and 12; at a
phase point they follow from the ray's closest approach to the source
(oracle/raytrace.py, closest_approach_fields: classical Runge-Kutta rays in
an analytic medium, pinned below against the closed forms of a homogeneous
medium and against adaptive DOP853 rays of the oracle's own Hamiltonian).

Discrete: the oracle's steady march (WENO5 + SSP-RK3, eqs. 16 and 19 times
dz/dtau).  The source-ball and edge data are the continuum fields
themselves (not the frozen-medium point-source data, whose O(h^2) error
would hide the scheme's), and so is the initial state; the march runs one
and a half transit times from the ball to the measured cells.  Measured:
cells outside the ball whose ray comes from it (outgoing, |phi1| at most half
the ball radius), clear of the edges.

The medium: vp0 linear in x and z, constant eps and delta, tilt linear in x
and z, so that every table field is a quadratic in position and the table's
4th-order differences are exact (the velocity carries no discretisation
error of its own).

Orders (measured when fixed: x-z refinement 5.73 / 5.42, theta refinement
4.68 / 4.02 for psi / phi1):
* x and z refined at a fine, fixed theta spacing: >= 4.5 for psi and phi1;
* theta refined at a fixed x-z spacing: >= 4.5 for psi; >= 3.5 for phi1.  On
  Gamma, phi1 is odd in theta about its root (an inflection), where the
  WENO5-JS weights depart from the linear ones at O(1) and the local order
  of the theta derivative drops (a known property of those weights); psi
  has no such point there."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.raytrace import LinearThomsenMedium, closest_approach_fields, trace, velocity_at

L, XS, ZS, R0 = 300.0, 150.0, 150.0, 50.0
RMIN, RMAX, PHIMAX = 62.5, 87.5, 25.0


def medium():
    return LinearThomsenMedium((XS, ZS), 2000.0, 0.4, 0.7, 0.15, 0.05, nu0=0.3, kx=1.5e-3, kz=-1.0e-3)


def march_error(N, nth):
    """Max |psi - psi*| and |phi1 - phi1*| over the measured cells after the
    march on an N x N x nth grid of the 300 m square (source at its centre)."""
    med = medium()
    g = W.Grid(nx=N, nz=N, nth=nth, dx=L / N, dz=L / N)
    vp, ep, de, nu = med.gridded(g.xc(), g.zc())
    m = W.Medium(vp0=vp, eps=ep, delta=de, tilt=nu, vs_ratio=0.5)
    src = W.Source(xs=XS, zs=ZS, r0=R0, beta=1.0 / (2 * L))
    tab = oracle.medium_table(g, m)
    vel, _, dt = oracle.velocity(g, tab)
    Ub = oracle.init_state(g, tab, src)
    TH, X, Z = np.meshgrid(g.th(), g.xc(), g.zc(), indexing="ij")
    phs, pss = closest_approach_fields(med, XS, ZS, X, Z, TH, dtau=2e-3)
    Ub[0], Ub[1] = phs, pss
    nsteps = int(np.ceil(1.5 * (RMAX - R0) / 1800.0 / dt))
    U = oracle.march(g, vel, src, Ub, dt, nsteps, Ub=Ub)
    V, _ = med.velocity(X, Z, TH)
    out = (X - XS) * V[0] + (Z - ZS) * V[1] > 0
    R = np.hypot(X - XS, Z - ZS)
    sel = (R >= RMIN) & (R <= RMAX) & (np.abs(phs) <= PHIMAX) & out
    assert sel.sum() > 100
    return np.abs(U[1] - pss)[sel].max(), np.abs(U[0] - phs)[sel].max()


def test_continuum_fields_are_the_point_source_data_in_a_homogeneous_medium():
    med = LinearThomsenMedium((0.0, 0.0), 2000.0, 0.0, 0.0, 0.15, 0.05, nu0=0.3)
    rng = np.random.default_rng(3)
    x, z, th = rng.uniform(-100, 100, 400), rng.uniform(-100, 100, 400), rng.uniform(0, 2 * np.pi, 400)
    phi, psi = closest_approach_fields(med, 0.0, 0.0, x, z, th)
    V, v = med.velocity(x, z, th)
    nv = np.hypot(V[0], V[1])
    assert np.abs(phi - (x * V[1] - z * V[0]) / nv).max() < 1e-10
    assert np.abs(psi - (np.sin(th) * x + np.cos(th) * z) / v).max() < 1e-14


def test_continuum_fields_follow_the_oracle_rays():
    """phi1 is constant and psi grows at unit rate along rays traced with
    DOP853 through the oracle's own Hamiltonian (medium table -> qP jet ->
    Liouville velocity); the analytic medium and the table agree."""
    med = medium()
    rng = np.random.default_rng(4)
    for _ in range(4):
        y0 = (rng.uniform(60, 240), rng.uniform(60, 240), rng.uniform(0, 2 * np.pi))
        sol = trace(med, y0, -0.03)
        y1 = sol.y[:, -1]
        a = closest_approach_fields(med, XS, ZS, np.array([y0[0]]), np.array([y0[1]]), np.array([y0[2]]))
        b = closest_approach_fields(med, XS, ZS, np.array([y1[0]]), np.array([y1[1]]), np.array([y1[2]]))
        assert abs(a[0][0] - b[0][0]) < 1e-9
        assert abs((a[1][0] - b[1][0]) - 0.03) < 1e-12
        # the two Hamiltonians: V from the table (oracle) and from the analytic medium
        Va, _ = med.velocity(np.array(y0[0]), np.array(y0[1]), np.array(y0[2]))
        Vo, _, _ = velocity_at(med, *y0)
        assert np.allclose(Vo, Va.ravel(), rtol=1e-13, atol=1e-12)


def test_march_order_under_x_z_refinement():
    e1 = march_error(24, 192)
    e2 = march_error(48, 192)
    orders = np.log2(np.array(e1) / np.array(e2))
    print(f"x-z refinement: psi {e1[0]:.3e} -> {e2[0]:.3e}, phi1 {e1[1]:.3e} -> {e2[1]:.3e}, orders {orders}")
    assert orders[0] >= 4.5 and orders[1] >= 4.5


def test_march_order_under_theta_refinement():
    e1 = march_error(64, 48)
    e2 = march_error(64, 96)
    orders = np.log2(np.array(e1) / np.array(e2))
    print(f"theta refinement: psi {e1[0]:.3e} -> {e2[0]:.3e}, phi1 {e1[1]:.3e} -> {e2[1]:.3e}, orders {orders}")
    assert orders[0] >= 4.5 and orders[1] >= 3.5
