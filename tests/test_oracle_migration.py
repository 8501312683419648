"""Pins of the oracle's Green's-function migration (Born data of a
reflectivity and the image, its adjoint; section 6's application of the
depth march's Green's functions, eqs. 34-35)."""
import numpy as np

import oracle
import workloads as W
from oracle import closed_forms as CF
from oracle import migration as MG

TMAX = np.pi / 3


def test_image_is_the_adjoint_of_the_born_data():
    """Re <B m, d> = <m, I(d)> for random complex Green's functions, a random
    real reflectivity and random complex data (the dot-product test)."""
    rng = np.random.default_rng(20061194)
    ns, nw, nx, nz = 5, 3, 7, 6
    G = rng.standard_normal((ns, nw, nx, nz)) + 1j * rng.standard_normal((ns, nw, nx, nz))
    m = rng.standard_normal((nx, nz))
    d = rng.standard_normal((nw, ns, ns)) + 1j * rng.standard_normal((nw, ns, ns))
    om, dA = np.array([10.0, 20.0, 35.0]), 2.5
    lhs = np.real(np.vdot(MG.born_data(G, m, om, dA), d))
    rhs = np.sum(m * MG.migrate(G, d, om, dA))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the Born data are reciprocal: d[w][s][r] = d[w][r][s]
    b = MG.born_data(G, m, om, dA)
    assert np.allclose(b, np.transpose(b, (0, 2, 1)), rtol=1e-13, atol=0)


def _surface_image(Gfun, g, xs_list, om, x0, z0):
    """Image of a point scatterer at cell (x0, z0) from sources and receivers
    at the surface points xs_list, Green's functions from Gfun(xs, omega)."""
    G = np.stack([np.stack([Gfun(xs, o) for o in om]) for xs in xs_list])
    m = np.zeros((g.nx, g.nz))
    m[x0, z0] = 1.0
    dA = g.dx * g.dz
    return MG.migrate(G, MG.born_data(G, m, om, dA), om, dA)


def _assert_focused(img, x0, z0, tol_cells):
    i, k = np.unravel_index(np.argmax(img), img.shape)
    assert abs(i - x0) <= tol_cells and abs(k - z0) <= tol_cells, ((i, k), (x0, z0))
    far = np.ones_like(img, dtype=bool)
    far[max(x0 - 6, 0):x0 + 7, max(z0 - 6, 0):z0 + 7] = False
    assert img.max() > 3.0 * np.abs(img[far]).max()


def test_point_scatterer_is_imaged_with_closed_form_green_functions():
    """(i/4) H0 of a homogeneous isotropic medium as the Green's functions
    (no beams): the image of a point scatterer peaks at the scatterer (a
    conjugation or sign slip in either operator defocuses it)."""
    n, L, v = 64, 1000.0, 2000.0
    g = W.Grid(nx=n, nz=n, nth=n, dx=L / n, dz=L / n)
    X, Z = np.meshgrid(g.xc(), g.zc(), indexing="ij")
    om = W.hz(np.linspace(10.0, 60.0, 12))
    xs_list = np.linspace(0.1 * L, 0.9 * L, 24)
    img = _surface_image(lambda xs, o: CF.green_elliptic(X, Z, xs, 0.0, v, 0.0, o), g, xs_list, om, 30, 38)
    _assert_focused(img, 30, 38, 1)


def test_point_scatterer_is_imaged_with_depth_march_green_functions():
    """The same with the Green's functions of the depth march (one march, the
    beam sum of eq. 34 for every surface point): the scatterer is imaged
    within two cells."""
    n, L, v = 64, 1000.0, 2000.0
    g = W.Grid(nx=2 * n, nz=n, nth=n, dx=L / n, dz=L / n)
    r = oracle.psolve(g, W.homogeneous(g, v), TMAX, 1 / (2 * L))
    om = W.hz(np.linspace(10.0, 60.0, 8))
    xs_list = np.linspace(0.6 * L, 1.4 * L, 16)
    G = np.stack([oracle.pbeam_sum(g, r["tab"], r["U"], TMAX, xs, om) for xs in xs_list])
    m = np.zeros((g.nx, g.nz))
    x0, z0 = n, 38
    m[x0, z0] = 1.0
    dA = g.dx * g.dz
    img = MG.migrate(G, MG.born_data(G, m, om, dA), om, dA)
    _assert_focused(img, x0, z0, 2)
