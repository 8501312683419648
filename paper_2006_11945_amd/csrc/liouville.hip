// SSP-RK3 stage of the stationary phase-space Liouville march.
//
// For every phase cell (x, z, theta) and state plane f:
//   L_f = -(V_x D_x + V_z D_z + V_theta D_theta) U_f + S_f,
//   S_phi1 = 0, S_psi = 1, S_(C,B) = A (C, B)          (eqs. 16, 19, 21 x dz/dtau)
//   S_phase = A12 Im(B / C)                  (arg C continued along the ray)
// with D the WENO5 Hamilton-Jacobi derivative on the upwind side (D- for a
// velocity component >= 0, D+ otherwise; for the phase plane the linear
// fifth-order upwind derivative), then
//   Uout = ca U0 + cb (Uin + dt L(Uin)),  (ca, cb) = (0,1), (3/4,1/4), (1/3,2/3),
// and cells inside the source ball copy U0.  Ghosts: x, z from the boundary
// data (fixed values: the point-source data extended linearly beyond each
// end), theta periodic.
//
// Precision: planes phi1, C, B, phase in R (float or double); psi is stored and
// combined in double, its WENO differences are formed in double and the
// derivative is evaluated in R.
//
// Work decomposition.  A block owns a (z, theta) tile of 64 x TK cells and
// walks a chunk of x.  Each thread keeps the seven x-neighbours of its own
// (theta, z) column in registers (a ring that takes one new entry per x
// step), so the x-stencil costs no extra memory traffic.  The current x
// slice of the tile, with a 3-cell halo in z (ghosts from the boundary data)
// and in theta (periodic), sits in LDS (double buffered, one barrier per x
// step); the z- and theta-stencils read it at immediate offsets.  Blocks are
// numbered so that consecutive tiles land on the same XCD (shared L2 for the
// theta halo).
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "egb_device.h"
#include "egb_internal.h"
#include "stage_common.h"

namespace egb {
namespace {

constexpr int PZ = TZ + 6;   // padded LDS row

// Tiles of one problem: ntz x ntk (z, theta) tiles; the batched queue also
// splits x into nxc chunks of kx; nblocks is the launch's block count.
// Buffer extents for the raw buffer descriptors: the grid-dtype planes of the
// state and of the boundary data, and their psi planes, each under its own
// descriptor (base + psi_off / bpsi_off), so that each extent stays below
// 4 GiB where the whole state would not (512^3 FP32: 3 GiB + 1 GiB).
struct TileArgs {
    int ntz, ntk, nxc, kx, nblocks;
    unsigned state_bytes, psi_bytes, vel_bytes, bd_bytes, bpsi_bytes;
    unsigned long long psi_off, bpsi_off;
};

template <typename R, int TK, int NP>
struct StageSmem {
    using W = typename LdsWord<R>::T;
    // words per plane, padded to a multiple of 64 so that two planes at one
    // address pair up in a single ds_read2st64
    static constexpr int PLANE = ((TK + 6) * PZ + 63) / 64 * 64;
    static constexpr int NW = NP + LdsWord<R>::PSI_WORDS;    // planes per slice
    static constexpr int BUF = NW * PLANE;                   // words per slice
    static constexpr int PB = PLANE * (int)sizeof(W);        // bytes per plane
    W w[2 * BUF];
};

// Upwind derivative of plane f from its six upwind-ordered values: WENO5,
// or the linear fifth-order scheme for the phase plane (f is a constant
// after unrolling).
template <typename R, typename T>
__device__ __forceinline__ R deriv(int f, T u0, T u1, T u2, T u3, T u4, T u5) {
    return f == EGB_PHASE ? upwind5_up<R>(u0, u1, u2, u3, u4, u5) : weno_up<R>(u0, u1, u2, u3, u4, u5);
}

// Store the NP plane values and psi of one cell at word index i.
template <typename R, int TK, int NP>
__device__ __forceinline__ void lds_put(StageSmem<R, TK, NP>& sm, int i, const R (&v)[NP], double p) {
    using S = StageSmem<R, TK, NP>;
    using W = typename S::W;
#pragma unroll
    for (int f = 0; f < NP; ++f) sm.w[i + f * S::PLANE] = __builtin_bit_cast(W, v[f]);
    const unsigned long long b = __builtin_bit_cast(unsigned long long, p);
    if constexpr (sizeof(R) == 4) {
        sm.w[i + NP * S::PLANE] = (unsigned)b;
        sm.w[i + (NP + 1) * S::PLANE] = (unsigned)(b >> 32);
    } else {
        sm.w[i + NP * S::PLANE] = b;
    }
}

// One (z, theta) tile (number `tile`, z fastest) over the x range [x0, x1)
// of an RK stage.
// KIN: only phi1 and psi (the planes a traveltime depends on).
//
// Per plane f the cell's new value is
//   ca U0 + cb Uin + cb dt S_f - sum_a (cb dt |V_a| / h_a) weno_up(stencil_a),
// the three stencils read in upwind order: x from the register queue (a
// wave whose lanes all upwind from the same side takes a select-free
// path), z and theta from LDS at per-lane mirrored addresses.  Cells in the
// source ball take U0 instead (stage 0 is called with Uin == U0).
//
// Memory traffic inside the x loop is straight-line per lane, so that the
// waits the compiler places before a use cover only the load that use
// needs: in tiles that touch a z end every halo lane loads both its state
// cell (clamped) and a boundary-data value and keeps one of them; the next
// x queue entry comes from the state or, past nx, from the boundary data
// (the buffer is chosen per block, the load is the same); lanes past nz
// load an in-domain column and write nothing.
template <typename R, int STAGE, int TK, bool KIN>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const TileArgs& t, int tile, int x0, int x1,
                                           StageSmem<R, TK, KIN ? 1 : EGB_PSI>& sm) {
    constexpr int NP = KIN ? 1 : EGB_PSI;  // R planes marched
    using S = StageSmem<R, TK, NP>;
    constexpr int WS = (int)sizeof(typename S::W);
    constexpr int NHALO = 6 * TZ + 6 * TK;
    static_assert(NHALO <= 64 * TK, "one halo slot per thread");
    static_assert(S::PB * (S::NW - 1) < 65536, "plane offsets fit the LDS immediate");
    constexpr unsigned ES = sizeof(R);

    const GridArgs& g = a.g;
    const int tzi = tile % t.ntz;
    const int tki = tile / t.ntz;

    const int tz = threadIdx.x, tk = threadIdx.y, tid = tk * TZ + tz;
    const int iz = tzi * TZ + tz;
    const int nv = min(TZ, g.nz - tzi * TZ);  // z columns of this tile inside the grid
    const int kraw = tki * TK + tk;
    const int k = kraw < g.nth ? kraw : kraw - g.nth;  // ragged theta tiles wrap (periodic rows, never written)
    const bool zin = tz < nv;
    const bool valid = zin && kraw < g.nth;
    const int izc = min(iz, g.nz - 1);  // in-domain column for the loads of lanes past nz
    const unsigned nxz = (unsigned)g.nxz, SS = (unsigned)g.stride;
    const unsigned kb = (unsigned)k * nxz;
    const auto rUi = make_rsrc(a.Uin, t.state_bytes);
    const auto rU0 = make_rsrc(a.U0, t.state_bytes);
    const auto rUo = make_rsrc(a.Uout, t.state_bytes);
    const auto rV = make_rsrc(a.vel, t.vel_bytes);
    const auto rB = make_rsrc(a.bd, t.bd_bytes);
    // the psi planes
    const auto pUi = make_rsrc(static_cast<const char*>(a.Uin) + t.psi_off, t.psi_bytes);
    const auto pU0 = make_rsrc(static_cast<const char*>(a.U0) + t.psi_off, t.psi_bytes);
    const auto pUo = make_rsrc(static_cast<char*>(a.Uout) + t.psi_off, t.psi_bytes);
    const auto pB = make_rsrc(static_cast<const char*>(a.bd) + t.bpsi_off, t.bpsi_bytes);
    const unsigned SP = SS * ES;         // bytes per R plane
    const unsigned BSP = (unsigned)g.bstride * ES;  // boundary data: bytes per R plane
    const unsigned XG = (unsigned)k * 6u * (unsigned)g.nz + (unsigned)izc;  // x ghost slot 0 of the column
    const unsigned ZG = (unsigned)g.nth * 6u * (unsigned)g.nz;            // first z ghost

    // Halo slot of this thread (if any): theta rows first (whole waves; z
    // clamped into the grid, columns past nz are never read), then z
    // columns: three on each side of the tile's nv inside columns, so that
    // in the last tile the right ones are the ghosts nz, nz + 1, nz + 2.
    const bool has_halo = tid < NHALO;
    int hk = 0, hz = 0;    // LDS coordinates (0-based, padded)
    unsigned hkb = kb;     // threads without a slot load their own column (unused)
    int hz0 = izc;         // global z of the halo cell (clamped)
    bool hgh = false;      // the halo cell is a z ghost
    unsigned hbo = ZG;     // its boundary-data index at x = 0 (step 6 per x)
    if (tid < 6 * TZ) {
        const int r = tid / TZ;
        hz = tid % TZ + 3;
        hk = r < 3 ? r : TK + r;
        int kk = tki * TK + hk - 3;
        kk = ((kk % g.nth) + g.nth) % g.nth;
        hkb = (unsigned)kk * nxz;
        hz0 = min(tzi * TZ + hz - 3, g.nz - 1);
    } else if (has_halo) {
        const int h = tid - 6 * TZ, r = h / TK;
        hk = h % TK + 3;
        hz = r < 3 ? r : nv + r;
        int kk = tki * TK + hk - 3;
        kk = kk < g.nth ? kk : kk - g.nth;
        hkb = (unsigned)kk * nxz;
        const int hzg = tzi * TZ + hz - 3;  // a ghost outside [0, nz)
        hz0 = min(max(hzg, 0), g.nz - 1);
        hgh = hzg < 0 || hzg >= g.nz;
        if (hgh) hbo = ZG + (unsigned)kk * 6u * (unsigned)g.nx + (unsigned)(hzg < 0 ? hzg + 3 : hzg - g.nz + 3);
    }
    const bool z_end = tzi == 0 || tzi == t.ntz - 1 || (tzi + 1) * TZ + 3 > g.nz;  // block-uniform

    // queue of the column's x-neighbours (at x = x0: q[f][j] at x0 - 3 + j;
    // a ring afterwards, see the x loop), entries from the state inside the
    // grid and from the boundary data beyond either end (position p: slot
    // p + 3 before x = 0, p - nx + 3 past nx - 1; a slot past nx + 2 is
    // never used and clamped)
    auto x_entry = [&](int p, R (&v)[NP], double& vp) {
        const bool gh = p < 0 || p >= g.nx;  // block-uniform
        const auto r = gh ? rB : rUi;
        const auto rp = gh ? pB : pUi;
        const unsigned sp = gh ? BSP : SP;
        const unsigned o = gh ? XG + (unsigned)(min(p < 0 ? p + 3 : p - g.nx + 3, 5) * g.nz)
                              : kb + (unsigned)(p * g.nz + izc);
#pragma unroll
        for (int f = 0; f < NP; ++f) v[f] = bload<R>(r, o * ES, f * sp);
        vp = bload<double>(rp, o * 8u, 0);
    };
    R q[NP][7];
    double qp[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        R v[NP];
        x_entry(x0 - 3 + j, v, qp[j]);
#pragma unroll
        for (int f = 0; f < NP; ++f) q[f][j] = v[f];
    }
    // halo loads of slice xs: the state cell of every thread and, where the
    // tile touches a z end, the boundary-data value (kept by ghost lanes)
    R hr0[NP], hr1[NP];
    double hq0, hq1 = 0.0;
    auto halo_load = [&](int xs) {
        const unsigned o0 = hkb + (unsigned)(xs * g.nz) + (unsigned)hz0;
#pragma unroll
        for (int f = 0; f < NP; ++f) hr0[f] = bload<R>(rUi, o0 * ES, f * SP);
        hq0 = bload<double>(pUi, o0 * 8u, 0);
        if (z_end) {
            const unsigned o1 = hbo + (unsigned)(xs * 6);
#pragma unroll
            for (int f = 0; f < NP; ++f) hr1[f] = bload<R>(rB, o1 * ES, f * BSP);
            hq1 = bload<double>(pB, o1 * 8u, 0);
        }
    };
    halo_load(x0);

    // RK-weighted coefficients: cb dt / h per axis (R planes and psi)
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    const double cdt = cb * a.dt;
    const R kxr = (R)(cdt / g.dx), kzr = (R)(cdt / g.dz), ktr = (R)(cdt / g.dth), cdtr = (R)cdt;
    const double zc = g.z0 + (iz + 0.5) * g.dz - a.zs;
    const int me = (tk + 3) * PZ + tz + 3;
    const int hi = hk * PZ + hz;

    // velocity components of the cell, fetched one x step ahead
    R cvx = (R)0, cvz = (R)0, cvt = (R)0;
    if (x0 < x1) {
        const unsigned cR = (kb + (unsigned)(x0 * g.nz + izc)) * ES;
        cvx = bload<R>(rV, cR, EGB_VX * SP);
        cvz = bload<R>(rV, cR, EGB_VZ * SP);
        cvt = bload<R>(rV, cR, EGB_VT * SP);
    }

    // The queue is a ring over each round of seven x steps: in step RT of a
    // round, entry j (position x - 3 + j) sits in q[.][(j + RT) % 7], so
    // advancing the queue writes only the new entry x + 4 (into the slot of
    // x - 3) instead of moving six entries per plane.
    int buf = 0;
    auto step = [&](const int x, auto rot) {
        constexpr int RT = decltype(rot)::value;
        R qx[NP][7];
        double qpx[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
#pragma unroll
            for (int f = 0; f < NP; ++f) qx[f][j] = q[f][(j + RT) % 7];
            qpx[j] = qp[(j + RT) % 7];
        }
        const int wb = buf * S::BUF;
        // slice x into LDS: own column from the queue, halo from its loads
        if (zin) {
            R own[NP];
#pragma unroll
            for (int f = 0; f < NP; ++f) own[f] = qx[f][3];
            lds_put(sm, wb + me, own, qpx[3]);
        }
        if (has_halo) {
            R hv[NP];
            double hp;
            if (z_end) {
#pragma unroll
                for (int f = 0; f < NP; ++f) hv[f] = hgh ? hr1[f] : hr0[f];
                hp = hgh ? hq1 : hq0;
            } else {
#pragma unroll
                for (int f = 0; f < NP; ++f) hv[f] = hr0[f];
                hp = hq0;
            }
            lds_put(sm, wb + hi, hv, hp);
        }
        // next queue entry (x + 4)
        R qn[NP];
        double qpn;
        x_entry(x + 4, qn, qpn);
        // next halo slice and the next cell's velocity (clamped at the chunk end)
        const int xn = min(x + 1, x1 - 1);
        halo_load(xn);
        R nvx, nvz, nvt;
        {
            const unsigned cR = (kb + (unsigned)(xn * g.nz + izc)) * ES;
            nvx = bload<R>(rV, cR, EGB_VX * SP);
            nvz = bload<R>(rV, cR, EGB_VZ * SP);
            nvt = bload<R>(rV, cR, EGB_VT * SP);
        }
        __syncthreads();

        {
            const unsigned cR = (kb + (unsigned)(x * g.nz + izc)) * ES;
            const unsigned c8 = cR / ES * 8u;
            const double xr = g.x0 + (x + 0.5) * g.dx - a.xs;
            const bool ball = xr * xr + zc * zc <= a.r02;  // source ball: Dirichlet data
            const R vx = cvx, vz = cvz, vt = cvt;
            const bool mx = vx >= (R)0, mz = vz >= (R)0, mt = vt >= (R)0;
            const R gx = fabs(vx) * kxr, gz = fabs(vz) * kzr, gt = fabs(vt) * ktr;
            // loads consumed after the stencils (their latency hides behind them)
            R u0[NP], Am[4];
            double p0;
            if constexpr (STAGE != 0) {
#pragma unroll
                for (int f = 0; f < NP; ++f) u0[f] = bload<R>(rU0, cR, f * SP);
                p0 = bload<double>(pU0, c8, 0);
            } else {
#pragma unroll
                for (int f = 0; f < NP; ++f) u0[f] = qx[f][3];
                p0 = qpx[3];
            }
            if constexpr (!KIN) {
#pragma unroll
                for (int j = 0; j < 4; ++j) Am[j] = bload<R>(rV, cR, (EGB_A11 + j) * SP);
            }
            // cb (Uin + dt S) - sum_a g_a W_a, then + ca U0; the psi stencil
            // terms (each already rounded to R) are summed in R and added to
            // the double psi once
            R acc[NP], convp;
#pragma unroll
            for (int f = 0; f < NP; ++f) acc[f] = (R)cb * qx[f][3];
            double accp = cb * qpx[3] + cdt;
            // x: upwind stencil from the register queue
            auto xpart = [&](auto dir) {
                constexpr int D = decltype(dir)::value;
#pragma unroll
                for (int f = 0; f < NP; ++f)
                    acc[f] -= gx * deriv<R>(f, upw<D>(qx[f], 0, mx), upw<D>(qx[f], 1, mx), upw<D>(qx[f], 2, mx),
                                            qx[f][3], upw<D>(qx[f], 4, mx), upw<D>(qx[f], 5, mx));
                convp = gx * weno_up<R>(upw<D>(qpx, 0, mx), upw<D>(qpx, 1, mx), upw<D>(qpx, 2, mx), qpx[3],
                                        upw<D>(qpx, 4, mx), upw<D>(qpx, 5, mx));
            };
            if (__all(mx)) xpart(std::integral_constant<int, 0>{});
            else if (!__any(mx)) xpart(std::integral_constant<int, 1>{});
            else xpart(std::integral_constant<int, 2>{});
            // z and theta: upwind stencils from LDS at mirrored addresses
            const int meB = (wb + me) * WS;
            auto lpart = [&](int step, R gR) {
                const int a0 = meB - 3 * step, a1 = meB - 2 * step, a2 = meB - step;
                const int a4 = meB + step, a5 = meB + 2 * step;
#pragma unroll
                for (int f = 0; f < NP; ++f)
                    acc[f] -= gR * deriv<R>(f, lds_r<R>(sm, a0, f), lds_r<R>(sm, a1, f), lds_r<R>(sm, a2, f), qx[f][3],
                                            lds_r<R>(sm, a4, f), lds_r<R>(sm, a5, f));
                convp += gR * weno_up<R>(lds_psi<NP>(sm, a0), lds_psi<NP>(sm, a1), lds_psi<NP>(sm, a2), qpx[3],
                                         lds_psi<NP>(sm, a4), lds_psi<NP>(sm, a5));
            };
            lpart(mz ? WS : -WS, gz);
            lpart(mt ? PZ * WS : -PZ * WS, gt);
            accp -= (double)convp;
            if constexpr (!KIN) {
                const R A11 = cdtr * Am[0], A12 = cdtr * Am[1], A21 = cdtr * Am[2], A22 = cdtr * Am[3];
                // the products are fused explicitly, so that the rounding
                // does not depend on how the compiler contracts them
                const R rc = qx[EGB_RE_C][3], ic = qx[EGB_IM_C][3], rb = qx[EGB_RE_B][3], ib = qx[EGB_IM_B][3];
                acc[EGB_RE_C] += fma(A11, rc, A12 * rb);
                acc[EGB_RE_B] += fma(A21, rc, A22 * rb);
                acc[EGB_IM_C] += fma(A11, ic, A12 * ib);
                acc[EGB_IM_B] += fma(A21, ic, A22 * ib);
                acc[EGB_PHASE] += A12 * (fma(rc, ib, -(rb * ic)) / fma(ic, ic, rc * rc));
            }
            if constexpr (STAGE != 0) {
#pragma unroll
                for (int f = 0; f < NP; ++f) acc[f] += (R)ca * u0[f];
                accp += ca * p0;
            }
            if (valid) {
#pragma unroll
                for (int f = 0; f < NP; ++f) bstore(ball ? u0[f] : acc[f], rUo, cR, f * SP);
                bstore(ball ? p0 : accp, pUo, c8, 0);
            }
        }
        // advance the queue: entry x + 4 takes the slot of x - 3
#pragma unroll
        for (int f = 0; f < NP; ++f) q[f][RT] = qn[f];
        qp[RT] = qpn;
        cvx = nvx;
        cvz = nvz;
        cvt = nvt;
        buf ^= 1;
        // keep each step's schedule to itself (as in a rolled loop), so that
        // the register use stays that of one step
        __builtin_amdgcn_sched_barrier(0);
    };
    for (int x = x0; x < x1; x += 7) {
        step(x, std::integral_constant<int, 0>{});
        if (x + 1 >= x1) break;
        step(x + 1, std::integral_constant<int, 1>{});
        if (x + 2 >= x1) break;
        step(x + 2, std::integral_constant<int, 2>{});
        if (x + 3 >= x1) break;
        step(x + 3, std::integral_constant<int, 3>{});
        if (x + 4 >= x1) break;
        step(x + 4, std::integral_constant<int, 4>{});
        if (x + 5 >= x1) break;
        step(x + 5, std::integral_constant<int, 5>{});
        if (x + 6 >= x1) break;
        step(x + 6, std::integral_constant<int, 6>{});
    }
}

// TK theta rows per tile (one wave each), WPE waves per SIMD the register
// allocation is sized for (the launch shapes of the autotuner)
template <typename R, int STAGE, int TK, bool KIN, int WPE>
__global__ __launch_bounds__(64 * TK) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_stage(StageArgs a, TileArgs t) {
    __shared__ StageSmem<R, TK, KIN ? 1 : EGB_PSI> sm;
    // The (tile, x) steps, x fastest, split into gridDim.x equal contiguous
    // ranges (the grid is what the chip holds at once, so every block runs in
    // one round); a range crossing a tile boundary is two segments.
    const long long W = (long long)t.ntz * t.ntk * a.g.nx;
    const long long b = xcd_remap(blockIdx.x, gridDim.x);
    long long w = W * b / gridDim.x;
    const long long w1 = W * (b + 1) / gridDim.x;
    while (w < w1) {
        const int tile = (int)(w / a.g.nx), xa = (int)(w % a.g.nx);
        const int xb = (int)min((long long)a.g.nx, xa + (w1 - w));
        stage_tile<R, STAGE, TK, KIN>(a, t, tile, xa, xb, sm);
        w += xb - xa;
        if (w < w1) __syncthreads();  // the segment's last LDS reads are done
    }
}

// Batched march: the (problem, tile, x) steps of every problem (uneven
// grids, own buffers and dt), x fastest, split into gridDim.x equal
// contiguous ranges like k_stage, so that many small problems fill the chip
// together; a range crossing a tile or problem boundary is several segments.
// wfirst[p] is the first step of problem p (wfirst[nprob] = total).
struct BatchItem {
    StageArgs a[3];  // stage 0, 1, 2 buffers of this problem
    TileArgs t;
};

constexpr long long MIN_STEPS = 16;  // fewest x steps worth a block's prologue

template <typename R, int STAGE, int TK, int WPE>
__global__ __launch_bounds__(64 * TK) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_stage_batched(const BatchItem* __restrict__ items, const long long* __restrict__ wfirst, int nprob) {
    __shared__ StageSmem<R, TK, EGB_PSI> sm;
    const long long W = wfirst[nprob];
    const long long b = xcd_remap(blockIdx.x, gridDim.x);
    long long w = W * b / gridDim.x;
    const long long w1 = W * (b + 1) / gridDim.x;
    bool first_seg = true;
    while (w < w1) {
        int lo = 0, hi = nprob;  // wfirst[lo] <= w < wfirst[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (wfirst[mid] <= w) lo = mid; else hi = mid;
        }
        // private copies: the stage's stores cannot alias them, so they stay in scalar registers
        const StageArgs a = items[lo].a[STAGE];
        const TileArgs ta = items[lo].t;
        const long long l = w - wfirst[lo];
        const int tile = (int)(l / a.g.nx), xa = (int)(l % a.g.nx);
        const int xb = (int)min((long long)a.g.nx, xa + (w1 - w));
        if (!first_seg) __syncthreads();  // the previous segment's last LDS reads are done
        first_seg = false;
        stage_tile<R, STAGE, TK, false>(a, ta, tile, xa, xb, sm);
        w += xb - xa;
    }
}

// Descriptor extents of one grid (see TileArgs).
void set_extents(TileArgs& t, const GridArgs& g, size_t es) {
    t.state_bytes = (unsigned)((unsigned long long)EGB_PSI * g.stride * es);
    t.psi_off = (unsigned long long)EGB_PSI * g.stride * es;
    t.psi_bytes = (unsigned)(g.stride * 8ull);
    t.vel_bytes = (unsigned)(7ull * (unsigned long long)g.stride * es);
    t.bd_bytes = (unsigned)((unsigned long long)EGB_PSI * g.bstride * es);
    t.bpsi_off = (unsigned long long)EGB_PSI * g.bstride * es;
    t.bpsi_bytes = (unsigned)(g.bstride * 8ull);
}

template <typename R, int TK, bool KIN, int WPE>
hipError_t launch_stage_t(const StageArgs& a, int stage, hipStream_t s, int blocks) {
    TileArgs t;
    t.ntz = (a.g.nz + TZ - 1) / TZ;
    t.ntk = (a.g.nth + TK - 1) / TK;
    t.kx = a.g.nx;
    t.nxc = 1;
    set_extents(t, a.g, sizeof(R));
    const void* k = stage == 0 ? (const void*)k_stage<R, 0, TK, KIN, WPE>
                  : stage == 1 ? (const void*)k_stage<R, 1, TK, KIN, WPE> : (const void*)k_stage<R, 2, TK, KIN, WPE>;
    // by default one round of resident blocks, each with at least MIN_STEPS
    // x steps; `blocks` > 0 (a tuned or fixed count) splits the steps over
    // that many blocks instead (the results do not depend on the split)
    const long long W = (long long)t.ntz * t.ntk * a.g.nx;
    long long G = blocks > 0 ? blocks : resident_blocks(k, 64 * TK);
    if (G <= 0) return hipErrorInvalidDeviceFunction;
    if (blocks <= 0) G = std::min(G, std::max(1LL, W / MIN_STEPS));
    G = std::min(G, W);
    t.nblocks = (int)G;
    const dim3 grid((unsigned)G), block(TZ, TK);
    switch (stage) {
        case 0: k_stage<R, 0, TK, KIN, WPE><<<grid, block, 0, s>>>(a, t); break;
        case 1: k_stage<R, 1, TK, KIN, WPE><<<grid, block, 0, s>>>(a, t); break;
        default: k_stage<R, 2, TK, KIN, WPE><<<grid, block, 0, s>>>(a, t); break;
    }
    return hipGetLastError();
}

template <typename R, int TK, int WPE>
hipError_t launch_batched_t(const void* items, const long long* wfirst, int nprob, long long total, int stage,
                            int grid, hipStream_t s) {
    const void* k = stage == 0 ? (const void*)k_stage_batched<R, 0, TK, WPE>
                  : stage == 1 ? (const void*)k_stage_batched<R, 1, TK, WPE> : (const void*)k_stage_batched<R, 2, TK, WPE>;
    // one round of resident blocks, each with at least MIN_STEPS x steps
    long long G = grid > 0 ? grid : resident_blocks(k, 64 * TK);
    if (G <= 0) return hipErrorInvalidDeviceFunction;
    if (grid <= 0) G = std::min(G, std::max(1LL, total / MIN_STEPS));
    G = std::max(1LL, std::min(G, total));
    const dim3 block(TZ, TK);
    const BatchItem* it = static_cast<const BatchItem*>(items);
    switch (stage) {
        case 0: k_stage_batched<R, 0, TK, WPE><<<(unsigned)G, block, 0, s>>>(it, wfirst, nprob); break;
        case 1: k_stage_batched<R, 1, TK, WPE><<<(unsigned)G, block, 0, s>>>(it, wfirst, nprob); break;
        default: k_stage_batched<R, 2, TK, WPE><<<(unsigned)G, block, 0, s>>>(it, wfirst, nprob); break;
    }
    return hipGetLastError();
}

}  // namespace

// Blocks of a kernel that the device holds at once (cached per kernel and device).
int resident_blocks(const void* kernel, int threads) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(kernel, dev);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int n = std::max(1, per_cu) * std::max(1, ncu);
    cache[key] = n;
    return n;
}

size_t batch_item_bytes() { return sizeof(BatchItem); }

// Launch shapes: theta rows per tile and the waves per SIMD the kernel's
// registers are sized for.  Shape 0 is the default.  A shape changes only how
// the (tile, x) steps are laid out over the chip: every shape gives
// bit-identical results.
namespace {
struct ShapeDef {
    int tk, wpe;
};
// FP32 full-plane march and batched march: 12 rows at 3 waves per SIMD (one
// 12-wave block per CU, <= 168 VGPRs), 8 rows at 2 (one 8-wave block, no
// register limit below 256), 16 rows at 4 (one 16-wave block, <= 128 VGPRs)
constexpr ShapeDef SHAPES_F32[] = {{12, 3}, {8, 2}, {16, 4}};
// FP32 kinematic march (two planes, about 100 VGPRs)
constexpr ShapeDef SHAPES_KIN[] = {{16, 4}, {8, 4}, {12, 3}};
// FP64 grids: 8 rows (the full-plane kernel needs about 250 VGPRs)
constexpr ShapeDef SHAPES_F64[] = {{8, 2}};
constexpr ShapeDef SHAPES_F64_KIN[] = {{8, 3}};

template <size_t N>
int shape_count(const ShapeDef (&)[N]) { return (int)N; }

const ShapeDef* shapes_of(int dtype, bool kin, int& n) {
    if (dtype == EGB_F64) {
        n = kin ? shape_count(SHAPES_F64_KIN) : shape_count(SHAPES_F64);
        return kin ? SHAPES_F64_KIN : SHAPES_F64;
    }
    n = kin ? shape_count(SHAPES_KIN) : shape_count(SHAPES_F32);
    return kin ? SHAPES_KIN : SHAPES_F32;
}
}  // namespace

int stage_shapes(int dtype, bool kinematic, int* tile_rows) {
    int n = 0;
    const ShapeDef* sh = shapes_of(dtype, kinematic, n);
    if (tile_rows)
        for (int i = 0; i < n; ++i) tile_rows[i] = sh[i].tk;
    return n;
}

int batched_shapes(int dtype, int* tile_rows) { return stage_shapes(dtype, false, tile_rows); }

// Fill the host-side item for one problem; returns its (tile, x) step count.
long long batch_item_fill(void* item, const GridArgs& g, int dtype, const void* vel, const void* bd, void* state,
                          void* U1, void* U2, double dt, double xs, double zs, double r02, bool last_to_work,
                          int shape) {
    BatchItem& it = *static_cast<BatchItem*>(item);
    int n = 0;
    const ShapeDef* sh = shapes_of(dtype, false, n);
    const int tk = sh[shape >= 0 && shape < n ? shape : 0].tk;
    const size_t es = dtype == EGB_F64 ? 8 : 4;
    TileArgs t;
    t.ntz = (g.nz + TZ - 1) / TZ;
    t.ntk = (g.nth + tk - 1) / tk;
    t.kx = g.nx;
    t.nxc = 1;
    t.nblocks = 0;
    set_extents(t, g, es);
    it.t = t;
    void* in[3] = {state, U1, U2};
    void* out[3] = {U1, U2, last_to_work ? U1 : state};  // U1 is free again in the last stage
    for (int s = 0; s < 3; ++s) {
        it.a[s].g = g;
        it.a[s].vel = vel;
        it.a[s].bd = bd;
        it.a[s].U0 = state;
        it.a[s].Uin = in[s];
        it.a[s].Uout = out[s];
        it.a[s].dt = dt;
        it.a[s].xs = xs;
        it.a[s].zs = zs;
        it.a[s].r02 = r02;
    }
    return (long long)t.ntz * t.ntk * g.nx;
}

hipError_t launch_stage_batched(const void* items, const long long* wfirst, int nprob, long long total, int dtype,
                                int stage, int grid, hipStream_t s, int shape) {
    if (dtype == EGB_F64) return launch_batched_t<double, 8, 2>(items, wfirst, nprob, total, stage, grid, s);
    switch (shape) {
        case 1: return launch_batched_t<float, 8, 2>(items, wfirst, nprob, total, stage, grid, s);
        case 2: return launch_batched_t<float, 16, 4>(items, wfirst, nprob, total, stage, grid, s);
        default: return launch_batched_t<float, 12, 3>(items, wfirst, nprob, total, stage, grid, s);
    }
}

// Every descriptor extent (and so every byte offset inside it) below 4 GiB:
// the velocity planes (7 per cell) are the largest.
bool stage_fits_32bit(const GridArgs& g, int dtype) {
    const unsigned long long es = dtype == EGB_F64 ? 8 : 4, lim = 1ull << 32;
    const unsigned long long S = (unsigned long long)g.stride, B = (unsigned long long)g.bstride;
    return 7ull * S * es < lim && EGB_PSI * S * es < lim && S * 8ull < lim && EGB_PSI * B * es < lim && B * 8ull < lim;
}

hipError_t launch_stage(const StageArgs& a, int dtype, int stage, hipStream_t s, bool kinematic, int blocks,
                        int shape) {
    if (dtype == EGB_F64)
        return kinematic ? launch_stage_t<double, 8, true, 3>(a, stage, s, blocks)
                         : launch_stage_t<double, 8, false, 2>(a, stage, s, blocks);
    if (kinematic) {
        switch (shape) {
            case 1: return launch_stage_t<float, 8, true, 4>(a, stage, s, blocks);
            case 2: return launch_stage_t<float, 12, true, 3>(a, stage, s, blocks);
            default: return launch_stage_t<float, 16, true, 4>(a, stage, s, blocks);
        }
    }
    switch (shape) {
        case 1: return launch_stage_t<float, 8, false, 2>(a, stage, s, blocks);
        case 2: return launch_stage_t<float, 16, false, 4>(a, stage, s, blocks);
        default: return launch_stage_t<float, 12, false, 3>(a, stage, s, blocks);
    }
}

namespace {
template <typename R, int TK, bool KIN, int WPE>
void stage_limits_t(const GridArgs& g, long long& resident, long long& work) {
    resident = resident_blocks((const void*)k_stage<R, 0, TK, KIN, WPE>, 64 * TK);
    work = (long long)((g.nz + TZ - 1) / TZ) * ((g.nth + TK - 1) / TK) * g.nx;
}
}  // namespace

void stage_limits(const GridArgs& g, int dtype, bool kinematic, long long& resident, long long& work, int shape) {
    if (dtype == EGB_F64) {
        if (kinematic) stage_limits_t<double, 8, true, 3>(g, resident, work);
        else stage_limits_t<double, 8, false, 2>(g, resident, work);
    } else if (kinematic) {
        switch (shape) {
            case 1: stage_limits_t<float, 8, true, 4>(g, resident, work); break;
            case 2: stage_limits_t<float, 12, true, 3>(g, resident, work); break;
            default: stage_limits_t<float, 16, true, 4>(g, resident, work); break;
        }
    } else {
        switch (shape) {
            case 1: stage_limits_t<float, 8, false, 2>(g, resident, work); break;
            case 2: stage_limits_t<float, 16, false, 4>(g, resident, work); break;
            default: stage_limits_t<float, 12, false, 3>(g, resident, work); break;
        }
    }
}

long long batched_resident(int dtype, int shape) {
    if (dtype == EGB_F64) return resident_blocks((const void*)k_stage_batched<double, 0, 8, 2>, 64 * 8);
    switch (shape) {
        case 1: return resident_blocks((const void*)k_stage_batched<float, 0, 8, 2>, 64 * 8);
        case 2: return resident_blocks((const void*)k_stage_batched<float, 0, 16, 4>, 64 * 16);
        default: return resident_blocks((const void*)k_stage_batched<float, 0, 12, 3>, 64 * 12);
    }
}

}  // namespace egb
