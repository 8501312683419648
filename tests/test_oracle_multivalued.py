"""Multivalued arrivals (the method's later arrivals, Gamma = {phi1 = 0} of
eq. 35): behind a low-velocity lens the rays from a point source form a
caustic and a triplication zone.  At receivers on a line below the lens,
the roots in theta of the oracle's marched phi1 with psi > 0 (bilinear in x
and z per theta plane, linear in theta, as in the first-arrival pick) must
be exactly as many as the rays from the source through the receiver
(ray-traced with classical Runge-Kutta steps in the analytic medium), and
each arrival's direction and traveltime must match its ray: directions
within a third of the theta spacing, 1.25 degrees (linear root in theta;
measured <= 0.9 degrees), traveltimes
within 1 % (the frozen-medium point-source data is O(h^2); measured <= 0.63 %
at 25 m cells).  Receivers are at least 40 m from the two caustic edges
(measured at x = 456 and 706 m), where two arrivals merge.

The same arrivals pin the KMAH phase (the continuous phase Phi of C carried
by the march): the branch index k = round((Phi - arg C) / 2 pi) that turns
the principal root of 1/C into the ray's branch equals the ray's own, from
the continuous phase of C integrated along the ray (DOP853 through the
oracle's Hamiltonian, (C, B) = (s, i beta s) at the source); the middle
arrival of the triplication has turned past pi (k = 1, the sign of its
amplitude flips), and away from the caustic (|C| at least 25, about half
its value on the single arrivals) Phi is within 0.4 rad of the ray's phase
(measured <= 0.26).  Near
the caustic, where |C| is small and the march resolves C poorly, Phi only
has to keep the branch (measured within 1.1 rad of 2 pi k)."""
import numpy as np

import oracle
import workloads as W
from oracle.raytrace import GaussianLensMedium, continuous_phase_of_c, fan_crossings

XS, ZS, ZR = 610.0, 100.0, 1000.0
RECEIVERS = (300.0, 350.0, 400.0, 520.0, 560.0, 600.0, 640.0, 680.0, 780.0, 850.0, 900.0)


def lens():
    return GaussianLensMedium(2000.0, -700.0, 600.0, 420.0, 110.0)


def ray_arrivals(xr, cross, take_off):
    """Rays crossing the receiver line at xr: sign changes of x(take-off) -
    xr; direction at the receiver, traveltime and take-off angle."""
    d = cross[0] - xr
    idx = np.flatnonzero(np.sign(d[1:]) != np.sign(d[:-1]))
    f = d[idx] / (d[idx] - d[idx + 1])
    th = cross[1, idx] + f * (cross[1, idx + 1] - cross[1, idx])
    t = cross[2, idx] + f * (cross[2, idx + 1] - cross[2, idx])
    t0 = take_off[idx] + f * (take_off[idx + 1] - take_off[idx])
    o = np.argsort(th)
    return th[o], t[o], t0[o]


def eulerian_arrivals(g, U, xr, zr):
    """Roots in theta of phi1 at (xr, zr) with psi > 0: direction,
    traveltime, C and the phase plane at each (linear in theta)."""
    fx, fz = (xr - g.x0) / g.dx - 0.5, (zr - g.z0) / g.dz - 0.5
    i, k = int(np.floor(fx)), int(np.floor(fz))
    a, b = fx - i, fz - k
    bil = lambda P: ((1 - a) * (1 - b) * P[:, i, k] + a * (1 - b) * P[:, i + 1, k] + (1 - a) * b * P[:, i, k + 1]
                     + a * b * P[:, i + 1, k + 1])
    ph, ps, C, PH = bil(U[0]), bil(U[1]), bil(U[2]) + 1j * bil(U[3]), bil(U[6])
    ph1, ps1, C1, PH1 = np.roll(ph, -1), np.roll(ps, -1), np.roll(C, -1), np.roll(PH, -1)
    root = (ph == 0) | (ph * ph1 < 0)
    w = np.where(root, ph / np.where(ph != ph1, ph - ph1, 1.0), 0.0)
    psr = ps + w * (ps1 - ps)
    sel = root & (psr > 0)
    th = np.angle(np.exp(1j * (g.th()[sel] + w[sel] * g.dth)))
    o = np.argsort(th)
    return th[o], psr[sel][o], (C + w * (C1 - C))[sel][o], (PH + w * (PH1 - PH))[sel][o]


def test_later_arrivals_and_their_branches_behind_a_lens_match_the_rays():
    med = lens()
    dx = 25.0
    g = W.Grid(nx=32, nz=44, nth=96, dx=dx, dz=dx, x0=210.0, z0=-50.0)
    X, Z = np.meshgrid(g.xc(), g.zc(), indexing="ij")
    v = med.vgrad(X, Z)[0]
    zero = np.zeros_like(v)
    m = W.Medium(vp0=v, eps=zero, delta=zero, tilt=zero, vs_ratio=0.5)
    src = W.Source(xs=XS, zs=ZS, r0=4 * dx, beta=1.0 / 2200.0)
    o = oracle.solve(W.Problem("lens", g, m, src, 0, W.hz([10.0])), nsteps=0)
    U = oracle.march(g, o["vel"], src, o["U0"], o["dt"], int(np.ceil(0.7 / o["dt"])), Ub=o["U0"])
    take_off = np.linspace(-1.0, 1.0, 4001)
    cross = fan_crossings(med, XS, ZS, take_off, ZR)
    counts, flipped = [], 0
    for xr in RECEIVERS:
        th_r, t_r, t0_r = ray_arrivals(xr, cross, take_off)
        th_e, t_e, C_e, ph_e = eulerian_arrivals(g, U, xr, ZR)
        counts.append((len(th_r), len(th_e)))
        print(f"x {xr:5.0f}: rays {np.degrees(th_r).round(1)} {t_r.round(4)}; march {np.degrees(th_e).round(1)} "
              f"{t_e.round(4)}")
        assert len(th_e) == len(th_r), xr
        assert np.abs(np.degrees(th_e - th_r)).max() < 1.25, xr
        assert (np.abs(t_e - t_r) / t_r).max() < 1e-2, xr
        # the KMAH branch of every arrival against its ray
        ph_r = np.array([continuous_phase_of_c(med, (XS, ZS, a), t, src.beta) for a, t in zip(t0_r, t_r)])
        k_r = np.rint((ph_r - np.angle(np.exp(1j * ph_r))) / (2 * np.pi))
        k_e = np.rint((ph_e - np.angle(C_e)) / (2 * np.pi))
        print(f"         ray phase of C {ph_r.round(3)}, march phase {ph_e.round(3)}, |C| {np.abs(C_e).round(1)}, "
              f"k rays {k_r} march {k_e}")
        assert np.array_equal(k_r, k_e), xr
        assert np.all(np.abs(ph_e - np.angle(C_e) - 2 * np.pi * k_e) < 0.5 * np.pi)
        far = np.abs(C_e) >= 25.0
        assert np.all(np.abs(ph_e - ph_r)[far] < 0.4), xr
        flipped += int(np.sum(k_r % 2 == 1))
    assert sorted(set(c for c, _ in counts)) == [1, 3]  # both zones are sampled
    assert flipped >= 5  # the middle arrival of the triplication at every receiver in the zone
