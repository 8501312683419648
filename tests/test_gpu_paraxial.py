"""GPU parity of the paraxial depth march (the paper's own formulation,
section 3 eqs. 13-15 and section 4 eqs. 16-24, picks by eq. 35) against the
FP64 oracle, through the C ABI.

Tolerances (fixed from the arithmetic before measuring):
  * FP64: 1e-10 of the plane maximum for the coefficients (as for the
    phase-space velocity: A21 cancels terms of its own size), 1e-12 for the
    surface data, 1e-10 for the marched levels (summation / FMA order only);
  * FP32 (tau kept in double): coefficients and surface data 2e-6 of the
    plane maximum (computed in double, rounded once); marched levels: tau
    1e-5 of the level's maximum, the other planes 1e-4 of the plane maximum
    (the oracle marched with one FP32 ulp of noise per stage stays below
    3e-5; test_oracle_paraxial pins that sensitivity);
  * picks on identical (oracle) levels: 1e-12 relative, the same NaN cells.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_helpers import log, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TMAX = np.pi / 3
# oracle plane index of each GPU level plane
OR = {"X": 0, "vartheta": 1, "tau": 2, "ReC": 3, "ImC": 4, "ReB": 5, "ImB": 6, "phase": 7}
PV = ("u", "w", "Stau", "A11", "A12", "A21", "A22")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def egb():
    import paper_2006_11945_amd as m
    return m


def par_problem(tilt=False, nx=42, nz=30, nth=36):
    """Heterogeneous VTI / TTI on a ragged slice (x: one 64-wide tile, partly
    filled; theta: 9 tiles of 4)."""
    dx = 15.625
    g = W.Grid(nx=nx, nz=nz, nth=nth, dx=dx, dz=dx)
    L = nx * dx
    med = W.vti_medium(W.rng_for(5 if tilt else 6, 11), g, L, tilt=tilt)
    return g, med, 1.0 / (2 * L)


def gpu_levels(P, n):
    return {k: v.double().cpu().numpy() for k, v in P.level(n).items()}


def write_levels(P, U):
    """Oracle levels [nz][7][nth][nx] (rounded to the storage) into the GPU buffer."""
    for n in range(U.shape[0]):
        v = P.level(n)
        for name, q in OR.items():
            v[name].copy_(torch.as_tensor(U[n, q]).to(v[name].dtype))


@pytest.mark.parametrize("dtype,tilt,drt", [("f64", False, 0), ("f32", False, 0), ("f64", True, 0), ("f32", True, 0),
                                            ("f64", True, 1), ("f32", True, 1)])
def test_paraxial_coefficients_and_surface_data(dtype, tilt, drt):
    # drt = 1: the lateral-frame DRT coefficients of eqs. 21-23 and their surface data
    g, med, beta = par_problem(tilt)
    tab = oracle.medium_table(g, med)
    pv, rate = oracle.pvelocity(g, tab, TMAX, drt)
    U0 = oracle.pinit(g, pv, TMAX, beta, drt)
    P = egb().Paraxial(g, med, TMAX, DEV, dtype, drt=drt)
    r = P.velocity()
    P.init(beta)
    torch.cuda.synchronize()
    assert r == pytest.approx(rate, rel=1e-12)
    tol = 1e-10 if dtype == "f64" else 2e-6
    for n in range(g.nz):
        G = {k: v.double().cpu().numpy() for k, v in P.pvel_level(n).items()}
        for q, name in enumerate(PV):
            assert rel_err(G[name], pv[n, q]) < tol, (n, name)
    tol = 1e-12 if dtype == "f64" else 2e-6
    L0 = gpu_levels(P, 0)
    for name, q in OR.items():
        sc = max(np.abs(U0[q]).max(), 1e-30)
        assert rel_err(L0[name], U0[q], sc) < tol, name


@pytest.mark.parametrize("dtype,tilt,nx,nth,drt", [("f64", False, 42, 36, 0), ("f64", True, 42, 36, 0),
                                                  ("f32", False, 42, 36, 0), ("f32", True, 42, 36, 0),
                                                  ("f64", True, 200, 37, 0), ("f32", True, 200, 37, 0),
                                                  ("f64", True, 42, 36, 1), ("f32", True, 42, 36, 1)])
def test_paraxial_march_parity(dtype, tilt, nx, nth, drt):
    # 42 x 36: one partly filled x tile (every tile touches an end); 200 x 37:
    # x tiles at 0, 64, 128, 192 (the middle two touch no end and take the
    # plain fill) and a last theta tile of one row; drt = 1: the DRT of eqs. 21-23
    g, med, beta = par_problem(tilt, nx=nx, nth=nth)
    o = oracle.psolve(g, med, TMAX, beta, drt=drt)
    log(f"paraxial march {dtype} tilt={tilt} drt={drt} {g.nx}x{g.nz}x{g.nth} nsub={o['nsub']}")
    P = egb().Paraxial(g, med, TMAX, DEV, dtype, drt=drt)
    P.velocity()
    assert P.substeps() == o["nsub"]
    P.init(beta)
    P.march(o["nsub"])
    torch.cuda.synchronize()
    U = o["U"]
    worst = {}
    for n in range(g.nz):
        G = gpu_levels(P, n)
        for name, q in OR.items():
            sc = max(np.abs(U[:, q]).max(), 1e-30)
            if name == "tau":
                sc = max(np.abs(U[n, q]).max(), 1e-30)
            worst[name] = max(worst.get(name, 0.0), rel_err(G[name], U[n, q], sc))
    log("  " + " ".join(f"{k}: {v:.2e}" for k, v in worst.items()))
    for name in worst:
        if dtype == "f64":
            assert worst[name] < 1e-10, name
        elif name == "tau":
            assert worst[name] < 1e-5, name
        else:
            assert worst[name] < 1e-4, name


def test_paraxial_pick_parity_and_edge_cases():
    g, med, beta = par_problem(tilt=True)
    o = oracle.psolve(g, med, TMAX, beta)
    L = g.nx * g.dx
    xs = np.array([0.31 * L, 0.5 * L + 3.0, 0.77 * L, g.xc()[5], -10.0 * L])  # the last: outside, no arrivals
    P = egb().Paraxial(g, med, TMAX, DEV, "f32")
    U = o["U"].copy()
    for q in (0, 1, 3, 4, 5, 6, 7):  # the storage of an FP32 march (tau stays double)
        U[:, q] = U[:, q].astype(np.float32).astype(np.float64)
    write_levels(P, U)
    T = P.pick(xs).cpu().numpy()
    To = oracle.ppick(g, U, xs, TMAX)
    assert np.array_equal(np.isnan(T), np.isnan(To))
    assert np.isnan(T[-1]).all()
    ok = ~np.isnan(To)
    assert ok[:-1].mean() > 0.5
    assert np.abs(T[ok] - To[ok]).max() <= 1e-12 * np.abs(To[ok]).max()
    # no sources: a no-op
    P.pick(np.zeros(0))


def test_paraxial_invalid_arguments():
    import ctypes
    e = egb()
    g, med, beta = par_problem()
    P = e.Paraxial(g, med, TMAX, DEV, "f32")
    L = e.lib()
    nul = ctypes.c_void_p(None)
    for t in (0.0, -0.1, 1.6, float("nan")):
        assert L.egb_paraxial_init(ctypes.byref(P.eg), e._ptr(P.pvel), t, beta, 0, e._ptr(P.levels),
                                   nul) == e.EGB_EINVAL
    assert L.egb_paraxial_init(ctypes.byref(P.eg), e._ptr(P.pvel), TMAX, beta, 2, e._ptr(P.levels),
                               nul) == e.EGB_EINVAL  # no such DRT frame
    assert L.egb_paraxial_march(ctypes.byref(P.eg), e._ptr(P.pvel), TMAX, 0, e._ptr(P.levels), e._ptr(P.work),
                                P.work.numel(), nul) == e.EGB_EINVAL
    assert L.egb_paraxial_march(ctypes.byref(P.eg), e._ptr(P.pvel), TMAX, 2, e._ptr(P.levels), e._ptr(P.work),
                                16, nul) == e.EGB_EWORKSPACE
    # a full horizontal aperture in a tilted anisotropic medium: near theta = 90
    # degrees the group direction points up (V_z < 0), which the oracle refuses too
    tm = W.homogeneous(g, 2000.0, eps=0.3, delta=-0.1, tilt=np.pi / 4)
    with pytest.raises(ValueError):
        oracle.pvelocity(g, oracle.medium_table(g, tm), np.pi / 2)
    Q = e.Paraxial(g, tm, np.pi / 2, DEV, "f32")
    with pytest.raises(e.EgbError) as ex:
        Q.velocity()
    assert ex.value.status == e.EGB_EINVAL


def test_paraxial_full_size_paper23_stays_bounded():
    """The DRT of eqs. 21-23 marched through all 256 levels of the 256 x 256
    heterogeneous VTI slice: every level finite, and the Green's function of
    the central surface source finite."""
    from dataclasses import replace

    p = W.vti_256(n=256, nsteps=1)
    g = replace(p.grid, nth=256)
    L = g.nx * g.dx
    P = egb().Paraxial(g, p.medium, TMAX, DEV, "f32", drt=1)
    P.velocity()
    P.init(1.0 / (2 * L))
    P.march(P.substeps())
    torch.cuda.synchronize()
    for n in range(0, g.nz, 15):
        G = gpu_levels(P, n)
        assert all(np.isfinite(v).all() for v in G.values()), n
    out = P.beam(0.5 * L, W.hz([5.0, 60.0]))
    assert torch.isfinite(out).all()


def test_paraxial_full_size_first_levels():
    """The 256 x 256 VTI medium with 256 theta nodes, marched through all 256
    levels in the benchmark's configuration; the first six levels are
    compared with the oracle on the top eight depth rows of the same medium
    (its coefficients there are identical), the rest must stay finite."""
    p = W.vti_256(n=256, nsteps=1)
    g = replace(p.grid, nth=256)
    m = p.medium
    L = g.nx * g.dx
    beta = 1.0 / (2 * L)
    P = egb().Paraxial(g, m, TMAX, DEV, "f32")
    P.velocity()
    nsub = P.substeps()
    log(f"paraxial full size 256x256x256, nsub={nsub}")
    P.init(beta)
    P.march(nsub)
    torch.cuda.synchronize()
    gc = replace(g, nz=8)
    cut = lambda a: None if a is None else np.ascontiguousarray(a[:, :8])
    mc = replace(m, vp0=cut(m.vp0), eps=cut(m.eps), delta=cut(m.delta), tilt=cut(m.tilt))
    tab = oracle.medium_table(gc, mc)
    pv, _ = oracle.pvelocity(gc, tab, TMAX)
    U = oracle.pmarch(gc, pv, TMAX, oracle.pinit(gc, pv, TMAX, beta), nsub)
    for n in range(6):
        G = gpu_levels(P, n)
        for name, q in OR.items():
            if name == "tau":
                assert rel_err(G[name], U[n, q], max(np.abs(U[n, q]).max(), 1e-30)) < 1e-5, n
                continue
            sc = max(np.abs(U[:6, q]).max(), 1e-30)
            assert rel_err(G[name], U[n, q], sc) < 1e-4, (n, name)
    # every level stays in its physical range (bounded march)
    dth = 2 * TMAX / g.nth
    for n in range(0, g.nz, 15):
        G = gpu_levels(P, n)
        assert all(np.isfinite(v).all() for v in G.values()), n
        assert G["X"].min() > -0.05 * L and G["X"].max() < 1.05 * L, n
        assert np.abs(G["vartheta"]).max() < TMAX + 4 * dth, n
        assert G["tau"].min() >= 0.0 and G["tau"].max() < 2 * L / 1000.0, n
    # the Green's function of the central source is finite at every depth
    out = P.beam(0.5 * L, W.hz([5.0, 60.0]))
    assert torch.isfinite(out).all()


@pytest.mark.parametrize("dtype,lin,comp,drt", [("f64", 0, -1, 0), ("f32", 0, -1, 0), ("f32", 1, -1, 0),
                                                ("f64", 0, 1, 0), ("f32", 0, 0, 0), ("f32", 0, 2, 0), ("f32", 0, 3, 0),
                                                ("f64", 0, -1, 1), ("f32", 0, -1, 1)])
def test_paraxial_beam_sum_parity(dtype, lin, comp, drt):
    """Green's function from the depth march (eq. 34 over Gamma = {X = x_s}),
    scalar (comp = -1) or a component of the qP Green's tensor, on identical
    input: the oracle's levels, rounded to the storage, written into the GPU
    buffer; relative L2 per frequency 1e-10 (FP64) and 1e-4 (FP32 planes:
    single-precision phase factors)."""
    g, med, beta = par_problem(tilt=True)
    o = oracle.psolve(g, med, TMAX, beta, drt=drt)
    U = o["U"].copy()
    if dtype == "f32":
        for q in (0, 1, 3, 4, 5, 6, 7):
            U[:, q] = U[:, q].astype(np.float32).astype(np.float64)
    P = egb().Paraxial(g, med, TMAX, DEV, dtype, drt=drt)
    P.velocity()
    write_levels(P, U)
    xs = 0.45 * g.nx * g.dx + 2.0
    om = W.hz([15.0, 40.0])
    out = P.beam(xs, om, lin=lin, comp=comp).cpu().numpy()
    G = out[..., 0] + 1j * out[..., 1]
    Go = oracle.pbeam_sum(g, o["tab"], U, TMAX, xs, om, lin=lin, comp=comp, drt=drt)
    for w in range(len(om)):
        e = np.linalg.norm(G[w] - Go[w]) / np.linalg.norm(Go[w])
        log(f"  paraxial beam {dtype} lin={lin} comp={comp} drt={drt} omega {om[w]:.1f}: rel L2 {e:.2e}")
        assert e < (1e-10 if dtype == "f64" else 1e-4)
    assert np.linalg.norm(Go[0]) > 0
