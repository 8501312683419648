"""Reciprocity of the heterogeneous beam sum: G(a; b) = G(b; a).

The Green's function of a self-adjoint operator is symmetric in source and
receiver.  For the isotropic operator the beam sum targets
((Laplacian + omega^2 / v^2) G = -delta, the isotropic case of the target
of eqs. 29-34 as read here), the beam sum of a source at b evaluated at a
must equal the beam sum of a source at a evaluated at b, to within the
asymptotic error of the method (a beam sum is a high-frequency
approximation; the Eulerian quadrature adds O(h^2)).

Medium: v = 3000 m/s with three weak Gaussian inclusions (-200, +150,
-120 m/s) between the two points, so that the rays from a to b and back
cross the heterogeneity while the source neighbourhoods and the edges of
the 2.4 km square are homogeneous (the point-source data, frozen at the
source and used as ball and edge data, is then the exact solution there).
Points at cell centres (no interpolation of G), 1345 m apart (6.7 to 13
wavelengths at 15-30 Hz).  Budget: 8 % at 20-30 Hz (measured 1.4-5.9 % at
64^3); at 10 Hz (4.5 wavelengths) the asymptotic error is larger
(measured 19 %) and the test checks that the mismatch shrinks with
frequency.

Outside this setting the frozen-medium data are not the exact solution at
the edges: in a medium with a background gradient, rays entering through
an edge carry data that do not match the rays from the source ball, and
far from the source the rays from the ball form a tube only ~2 r0 / r wide
in angle (2-3 theta cells for r0 = 4 cells and nth = nx), across which the
WENO stencils reach.  The traveltimes near Gamma there carry errors of
~1 ms that do not shrink under refinement, and reciprocity fails by tens of
percent (measured: v = 2600 + 0.4 z m/s, 3 ms phase asymmetry at 64^3 and
96^3).  That is a property of the source and edge data this project
chose, and it is not what this test is about."""
import numpy as np

import oracle
import workloads as W

L, N = 2400.0, 64
INCLUSIONS = ((1100.0, 1050.0, -200.0, 170.0), (1300.0, 1250.0, 150.0, 150.0), (1250.0, 900.0, -120.0, 140.0))


def test_beam_sum_is_reciprocal_in_a_heterogeneous_medium():
    dx = L / N
    g = W.Grid(nx=N, nz=N, nth=N, dx=dx, dz=dx)
    X, Z = np.meshgrid(g.xc(), g.zc(), indexing="ij")
    v = np.full((N, N), 3000.0)
    for cx, cz, a, s in INCLUSIONS:
        v += a * np.exp(-((X - cx) ** 2 + (Z - cz) ** 2) / (2 * s * s))
    zero = np.zeros_like(v)
    med = W.Medium(vp0=v, eps=zero, delta=zero, tilt=zero, vs_ratio=0.5)
    ia, ka, ib, kb = int(700 / dx), int(700 / dx), int(1700 / dx), int(1600 / dx)
    pa, pb = (g.xc()[ia], g.zc()[ka]), (g.xc()[ib], g.zc()[kb])
    assert abs(v[ia, ka] - 3000.0) < 5.0 and abs(v[ib, kb] - 3000.0) < 5.0  # the inclusions are far
    om = W.hz([10.0, 20.0, 25.0, 30.0])
    G = {}
    for name, (xs, zs) in (("a", pa), ("b", pb)):
        src = W.Source(xs=xs, zs=zs, r0=4 * dx, beta=1.0 / (2 * L))
        o = oracle.solve(W.Problem("recip", g, med, src, 0, om), nsteps=0)
        U = oracle.march(g, o["vel"], src, o["U0"], o["dt"], int(np.ceil(0.8 / o["dt"])), Ub=o["U0"])
        G[name] = oracle.beam_sum(g, o["vel"], o["vaux"], src, U, om)
    gab, gba = G["b"][:, ia, ka], G["a"][:, ib, kb]
    mis = np.abs(gab - gba) / np.abs(gab)
    for w in range(len(om)):
        print(f"{om[w] / 2 / np.pi:4.0f} Hz  G(a;b) {gab[w]:.4e}  G(b;a) {gba[w]:.4e}  mismatch {mis[w]:.3e}")
    assert np.all(np.abs(gab) > 0.01)
    assert mis[1:].max() <= 0.08
    assert mis[1:].max() < mis[0]
