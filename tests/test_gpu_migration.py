"""GPU parity of the Green's-function migration (Born data and image, the
application of section 6) against the oracle, through the C ABI.

Tolerances: both sides accumulate in float64 from the same stored Green's
functions (FP32 fields are rounded once on the host before the oracle sees
them), so only the summation order differs: 1e-11 relative.  The pipeline
test (march, beam sums, Born data, image) is FP64 end to end: 1e-9.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import migration as MG
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TMAX = np.pi / 3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def egb():
    import paper_2006_11945_amd as m
    return m


@pytest.mark.parametrize("dtype,ns,nw,nx,nz", [("f64", 5, 3, 23, 19), ("f32", 37, 35, 40, 33),
                                             ("f32", 64, 4, 64, 64), ("f64", 1, 1, 9, 8), ("f32", 32, 33, 48, 40)])
def test_born_data_and_image_parity(dtype, ns, nw, nx, nz):
    """Seeded random Green's functions: ragged source tiles (37 points: two
    32-wide tiles, the image on its general path), more frequencies than one
    launch takes (35 > 32), the maximum of 64 surface points, a single point
    and frequency, exactly one full 32 x 32 tile (both contractions on the
    matrix cores with every lane's tile entries in use).  A second call gives
    the same bits."""
    e = egb()
    rng = np.random.default_rng(1000 * ns + nw)
    g = W.Grid(nx=nx, nz=nz, nth=8, dx=12.5, dz=10.0)
    eg = e.make_grid(g, dtype)
    rd = np.float64 if dtype == "f64" else np.float32
    Gh = rng.standard_normal((ns, nw, nx, nz, 2)).astype(rd)
    m = rng.standard_normal((nx, nz))
    om = np.linspace(20.0, 300.0, nw)
    G = torch.as_tensor(Gh, device=DEV)
    d = e.egb_born_data(eg, G, om, torch.as_tensor(m, device=DEV))
    Gc = Gh[..., 0].astype(np.float64) + 1j * Gh[..., 1].astype(np.float64)
    do = MG.born_data(Gc, m, om, g.dx * g.dz)
    dg = d[..., 0].cpu().numpy() + 1j * d[..., 1].cpu().numpy()
    err = np.abs(dg - do).max() / np.abs(do).max()
    log(f"born {dtype} ns={ns} nw={nw} {nx}x{nz}: {err:.2e}")
    assert err < 1e-11
    # the split over image points adds its partial sums in a fixed order
    assert torch.equal(d, e.egb_born_data(eg, G, om, torch.as_tensor(m, device=DEV)))
    # the image of arbitrary data (not only Born data)
    dr = rng.standard_normal((nw, ns, ns, 2))
    img_t = e.egb_migrate(eg, G, om, torch.as_tensor(dr, device=DEV))
    assert torch.equal(img_t, e.egb_migrate(eg, G, om, torch.as_tensor(dr, device=DEV)))
    img = img_t.cpu().numpy()
    io = MG.migrate(Gc, dr[..., 0] + 1j * dr[..., 1], om, g.dx * g.dz)
    err = np.abs(img - io).max() / np.abs(io).max()
    log(f"image {dtype}: {err:.2e}")
    assert err < 1e-11


def test_migration_pipeline_fp64_matches_oracle_and_focuses():
    """One depth march, the Green's functions of 12 surface points, the Born
    data of a point scatterer and its image, on the GPU in FP64 against the
    oracle's pipeline; the image peaks at the scatterer."""
    e = egb()
    n, L = 48, 750.0
    g = W.Grid(nx=2 * n, nz=n, nth=n, dx=L / n, dz=L / n)
    med = W.homogeneous(g, 2000.0, 0.1, 0.05)
    beta = 1.0 / (2 * L)
    om = W.hz(np.linspace(15.0, 60.0, 6))
    xs_list = np.linspace(0.6 * L, 1.4 * L, 12)
    m = np.zeros((g.nx, g.nz))
    x0, z0 = n, 30
    m[x0, z0] = 1.0
    o = oracle.psolve(g, med, TMAX, beta)
    Go = np.stack([oracle.pbeam_sum(g, o["tab"], o["U"], TMAX, xs, om) for xs in xs_list])
    io = MG.migrate(Go, MG.born_data(Go, m, om, g.dx * g.dz), om, g.dx * g.dz)
    P = e.Paraxial(g, med, TMAX, DEV, "f64")
    P.velocity()
    assert P.substeps() == o["nsub"]
    P.init(beta)
    P.march(o["nsub"])
    G = P.greens(xs_list, om)
    d = e.egb_born_data(P.eg, G, om, torch.as_tensor(m, device=DEV))
    img = e.egb_migrate(P.eg, G, om, d).cpu().numpy()
    err = np.abs(img - io).max() / np.abs(io).max()
    log(f"pipeline image vs oracle: {err:.2e}")
    assert err < 1e-9
    i, k = np.unravel_index(np.argmax(img), img.shape)
    assert abs(i - x0) <= 2 and abs(k - z0) <= 2, (i, k)


def test_full_size_migration_images_point_scatterers():
    """The benchmark's medium (heterogeneous VTI, 256 x 256 slice, 256 theta
    nodes, all levels): one depth march, the Green's functions of 16 surface
    points at 8 frequencies, the Born data of three point scatterers and the
    image.  Each scatterer is the image's peak within ten cells of it, at its
    own cell, well above the image's median."""
    from dataclasses import replace

    e = egb()
    p = W.vti_256(n=256, nsteps=1)
    g = replace(p.grid, nth=256)
    L = g.nx * g.dx
    P = e.Paraxial(g, p.medium, TMAX, DEV, "f32")
    P.velocity()
    P.init(1.0 / (2 * L))
    P.march(P.substeps())
    om = W.hz(np.linspace(10.0, 60.0, 8))
    G = P.greens(np.linspace(0.1 * L, 0.9 * L, 16), om)
    m = np.zeros((g.nx, g.nz))
    pts = [(128, 128), (85, 170), (170, 85)]
    for i, k in pts:
        m[i, k] = 1.0
    d = e.egb_born_data(P.eg, G, om, torch.as_tensor(m, device=DEV))
    img = np.abs(e.egb_migrate(P.eg, G, om, d).cpu().numpy())
    assert np.isfinite(img).all()
    med = np.median(img)
    for i, k in pts:
        win = img[i - 10:i + 11, k - 10:k + 11]
        a, b = np.unravel_index(np.argmax(win), win.shape)
        log(f"  scatterer ({i}, {k}): peak offset ({a - 10}, {b - 10}), contrast {win.max() / med:.1f}")
        assert abs(a - 10) <= 1 and abs(b - 10) <= 1
        assert win.max() > 10 * med
