// Discrete adjoint of the march for traveltime misfits.
//
// A traveltime depends on phi1 and psi only, and their transport does not
// involve the dynamic-ray-tracing pair (C, B) or the matrix A (eqs. 16, 19),
// so the adjoint carries phi1 and psi and differentiates with respect to the
// Liouville velocity V only.  For one SSP-RK3 stage
//   Uout = ca U0 + cb (Uin + dt L(Uin; V)),  ball cells copy U0,
// with mu = lambda_out outside the ball (0 inside):
//   lambda_U0  += ca mu + [ball] lambda_out
//   lambda_Uin  = cb mu + cb dt (dL/dUin)^T mu
//   g_V        += cb dt (dL/dV)^T mu,  dL/dV_d = -W_d / Delta_d,
// where W_d is the upwind WENO5 derivative (upwind side frozen).  The
// transposed stencil (dL/dUin)^T is applied by the fused stage kernel below:
// every source cell forms its Jacobian rows and the rows are summed per
// target, x through a register queue and z, theta through LDS; theta wraps.
// The x and z ghosts hold boundary data, fixed extensions of the point-source
// data: slots aimed at them are sensitivities to that data.  Folded onto the
// two end cells the ghost extends (weights m + 1 and -m), they accumulate per
// source cell in a boundary buffer that the source gradient contracts like
// lambda of the initial state.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "egb_device.h"
#include "egb_internal.h"
#include "stage_common.h"

namespace egb {
namespace {

constexpr int NSLOT = 7;  // stencil positions -3..3

// ------------------------------------------------------------ fused stage
// One adjoint stage in one pass.  A block owns a (z, theta) tile of
// TZ x TK cells and an x range [x0, x1) of targets; it walks the source
// slices x0 - 3 .. x1 + 2 (the three extra on each side contribute through
// their x rows only).  Per source slice:
//  * x rows of the tile's own cells go into a register queue of seven
//    accumulators per plane (targets xs - 3 .. xs + 3); target xs - 3 is
//    complete afterwards and is written out;
//  * z and theta rows of the own cells, plus the theta rows of the three
//    theta rows on either side of the tile and the z rows of the three z
//    columns on either side (the only halo rows that reach into the tile),
//    are written to LDS as seven slots per source ("slot j" = coefficient of
//    the target at offset j - 3), then every own cell sums the seven slots
//    aimed at it per axis;
//  * rows are formed in upwind order (mirrored reads for a negative
//    velocity component); a slot aimed at a ghost is never summed into a
//    target: the block that owns the source adds its fold (weight m + 1 on
//    the end cell, -m on its neighbour, for the ghost m cells outside) to
//    the boundary buffer, one (source, weight) entry per thread.
// The stencil values of the slice sit in LDS with a 6-cell halo (the halo
// sources' own stencils); the own column's x stencil is a register queue.
template <typename R, int TK>
struct AdjSmem {
    using W = typename LdsWord<R>::T;
    static constexpr int VZ = TZ + 12;                             // z positions -6 .. TZ + 5
    static constexpr int PLANE = ((TK + 12) * VZ + 63) / 64 * 64;  // words per value plane
    static constexpr int NW = 1 + LdsWord<R>::PSI_WORDS;           // phi1, psi
    static constexpr int PB = PLANE * (int)sizeof(W);              // bytes per value plane
    static constexpr int CZW = TZ + 6;                             // z sources -3 .. TZ + 2
    static constexpr int ZPL = TK * CZW;                           // z slots per (plane, slot)
    static constexpr int TPL = (TK + 6) * TZ;                      // theta sources -3 .. TK + 2
    W w[NW * PLANE];
    R cz[2 * NSLOT * ZPL];
    R ct[2 * NSLOT * TPL];
};

struct AdjStageArgs {
    GridArgs g;
    const void* vel;     // vel3d
    const void* bd;      // boundary data (ghost values)
    double* bfold;       // boundary sensitivity, accumulated
    const void* Uin;     // stage input state (phi1 and psi are read)
    const void* lam;     // lambda of the stage output
    const void* acc_in;  // stages 0, 1: accumulated lambda of U0 so far (may alias acc_out)
    void* acc_out;
    void* lam_in;        // stages 1, 2: lambda of the stage input
    void* gvel;          // [3][stride] of R, accumulated
    double dt, xs, zs, r02;
    // descriptor extents: plane phi1 of the state-layout buffers and of the
    // boundary data, and their psi planes under descriptors of their own
    // (base + psi_off / bpsi_off), each below 4 GiB
    unsigned state_bytes, psi_bytes, vel_bytes, gvel_bytes, bd_bytes, bpsi_bytes;
    unsigned long long psi_off, bpsi_off;
    int ntz, ntk;
};

// Gradient of the upwind WENO5 value with respect to the six upwind-ordered
// values u0..u5 (differences formed in T); returns the value.
template <typename R, typename T>
__device__ __forceinline__ R wgrad_up(T u0, T u1, T u2, T u3, T u4, T u5, R (&du)[6]) {
    R gr[5];
    const R W = weno5_grad<R>((R)(u1 - u0), (R)(u2 - u1), (R)(u3 - u2), (R)(u4 - u3), (R)(u5 - u4), gr);
    du[0] = -gr[0];
    du[1] = gr[0] - gr[1];
    du[2] = gr[1] - gr[2];
    du[3] = gr[2] - gr[3];
    du[4] = gr[3] - gr[4];
    du[5] = gr[4];
    return W;
}

// Slots (target offset j - 3) from an upwind-ordered row scaled by c: value m
// sits at offset (m - 3) for a non-negative velocity component, 3 - m else.
template <typename R, typename C>
__device__ __forceinline__ void to_slots(const R (&du)[6], bool plus, C c, C (&d)[NSLOT]) {
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const R v = plus ? (j < 6 ? du[j] : (R)0) : (j > 0 ? du[6 - j] : (R)0);
        d[j] = c * (C)v;
    }
}

// Fold of the slots of a source at index s of a line of n cells that aim
// beyond an end: the ghost m cells outside extends the end cell (weight
// m + 1) and its neighbour (weight -m).
template <typename C>
__device__ __forceinline__ void fold_weights(const C (&d)[NSLOT], int s, int n, double& f0, double& f1) {
    f0 = 0.0;
    f1 = 0.0;
#pragma unroll
    for (int j = 0; j < NSLOT; ++j) {
        const int t = s + j - 3;
        const int m = t < 0 ? -t : (t > n - 1 ? t - (n - 1) : 0);
        if (m > 0) {
            f0 += (double)(m + 1) * (double)d[j];
            f1 -= (double)m * (double)d[j];
        }
    }
}

// *p += v as one atomic add whose old value is not returned: the kernels add
// to an entry of g_V or of the boundary buffer from one thread per launch
// (so the sums are deterministic), and an add in memory needs no wait for a
// load, which in a loop with loads in flight would wait for all of them.
template <typename T>
__device__ __forceinline__ void add_to(T* p, T v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index of a boundary-sensitivity entry: plane p (0 phi1, 1 psi), theta k,
// line end e (0 near, 1 far), source s (0..2 counted from that end, inward),
// weight w (0 end cell, 1 its neighbour); x lines by z, z lines by x.
__device__ __forceinline__ long long bfold_x(const GridArgs& g, int p, int k, int e, int s, int w, int z) {
    return (long long)p * g.nth * 12 * (g.nx + g.nz) + ((((long long)k * 2 + e) * 3 + s) * 2 + w) * g.nz + z;
}
__device__ __forceinline__ long long bfold_z(const GridArgs& g, int p, int k, int x, int e, int s, int w) {
    return (long long)p * g.nth * 12 * (g.nx + g.nz) + (long long)g.nth * 12 * g.nz +
           (((long long)k * g.nx + x) * 2 + e) * 6 + s * 2 + w;
}

template <typename R, int STAGE, int TK>
__device__ __forceinline__ void adj_tile(const AdjStageArgs& a, int tile, int x0, int x1, AdjSmem<R, TK>& sm) {
    using S = AdjSmem<R, TK>;
    using Wd = typename S::W;
    constexpr int WS = (int)sizeof(Wd);
    constexpr int NT = TZ * TK;
    constexpr int NV = (TK + 12) * S::VZ;       // value cells per slice
    constexpr int NVI = (NV + NT - 1) / NT;     // value cells per thread
    constexpr int NH = 6 * TZ + 6 * TK;         // halo sources per slice
    constexpr int NHI = (NH + NT - 1) / NT;     // halo sources per thread
    constexpr unsigned ES = sizeof(R);
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    static_assert(S::PB * (S::NW - 1) < 65536, "plane offsets fit the LDS immediate");

    const GridArgs& g = a.g;
    const int tzi = tile % a.ntz, tki = tile / a.ntz;
    const int tz = threadIdx.x, tk = threadIdx.y, tid = tk * TZ + tz;
    const int iz = tzi * TZ + tz;
    const int kraw = tki * TK + tk;
    const int k = kraw < g.nth ? kraw : kraw - g.nth;  // ragged theta tiles wrap
    const bool zin = iz < g.nz;
    const bool valid = zin && kraw < g.nth;  // own cell written by this tile
    const int izc = min(iz, g.nz - 1);
    const unsigned nxz = (unsigned)g.nxz, SP = (unsigned)g.stride * ES;
    const unsigned kb = (unsigned)k * nxz;
    const auto rUi = make_rsrc(a.Uin, a.state_bytes);
    const auto rL = make_rsrc(a.lam, a.state_bytes);
    const auto rV = make_rsrc(a.vel, a.vel_bytes);
    const auto rB = make_rsrc(a.bd, a.bd_bytes);
    const auto pUi = make_rsrc(static_cast<const char*>(a.Uin) + a.psi_off, a.psi_bytes);
    const auto pL = make_rsrc(static_cast<const char*>(a.lam) + a.psi_off, a.psi_bytes);
    const auto pB = make_rsrc(static_cast<const char*>(a.bd) + a.bpsi_off, a.bpsi_bytes);
    const unsigned XG = (unsigned)k * 6u * (unsigned)g.nz + (unsigned)izc;  // x ghost slot 0 of the column
    const unsigned ZG = (unsigned)g.nth * 6u * (unsigned)g.nz;            // first z ghost
    const double cbdt = cb * a.dt;
    const double kx = cbdt / g.dx, kz = cbdt / g.dz, kt = cbdt / g.dth;
    auto wrapk = [&](int kk) { return ((kk % g.nth) + g.nth) % g.nth; };
    auto in_ball = [&](int ix, int izz) {
        const double xr = g.x0 + (ix + 0.5) * g.dx - a.xs, zr = g.z0 + (izz + 0.5) * g.dz - a.zs;
        return xr * xr + zr * zr <= a.r02;
    };

    // value cell i of the LDS slice: base (theta row, clamped z), the ghost
    // distance (0 inside, +-m within 3 of an end, 100 beyond: never read by
    // a source inside the grid) and the boundary-data index at x = 0 of a
    // ghost (step 6 per x; a valid index for the other cells)
    auto vcell = [&](int i, unsigned& vb, int& vm, unsigned& vbd) {
        const int tl = i / S::VZ - 6, zl = i % S::VZ - 6;
        const int z = tzi * TZ + zl;
        const int kk = wrapk(tki * TK + tl);
        vb = (unsigned)kk * nxz + (unsigned)min(max(z, 0), g.nz - 1);
        vm = z < 0 ? (z >= -3 ? z : 100) : (z >= g.nz ? (z <= g.nz + 2 ? z - (g.nz - 1) : 100) : 0);
        const int gi = (vm < 0 ? vm + 3 : (vm < 100 ? vm + 2 : 0));
        vbd = ZG + (unsigned)kk * 6u * (unsigned)g.nx + (unsigned)gi;
    };
    const bool z_end = tzi == 0 || (tzi + 1) * TZ + 6 > g.nz;  // block-uniform: some value cell is a ghost
    // halo source h: theta rows (h < 6 TZ) then z columns; LDS row, z position,
    // whether it is a cell of the grid, and its (clamped) cell index
    auto hcell = [&](int h, int& tl, int& zl, bool& real, unsigned& c) {
        tl = 0;
        zl = 0;
        if (h < 6 * TZ) {
            const int rr = h / TZ;
            zl = h % TZ;
            tl = rr < 3 ? rr - 3 : TK + rr - 3;
        } else if (h < NH) {
            const int cc = (h - 6 * TZ) / TK;
            tl = (h - 6 * TZ) % TK;
            zl = cc < 3 ? cc - 3 : TZ + cc - 3;
        }
        const int z = tzi * TZ + zl;
        real = h < NH && z >= 0 && z < g.nz;
        c = (unsigned)wrapk(tki * TK + tl) * nxz + (unsigned)min(max(z, 0), g.nz - 1);
    };

    // own column's x stencil: values at xs - 3 .. xs + 3, from the state
    // inside the grid and from the boundary data beyond either end (the
    // buffer is chosen per block; slots beyond the three ghosts on either
    // side are only in stencils of sources outside the grid and clamped)
    auto x_value = [&](int p, R& v, double& vp) {
        const bool gh = p < 0 || p >= g.nx;  // block-uniform
        const auto r = gh ? rB : rUi;
        const auto rp = gh ? pB : pUi;
        const unsigned o = gh ? XG + (unsigned)(min(max(p < 0 ? p + 3 : p - g.nx + 3, 0), 5) * g.nz)
                              : kb + (unsigned)(p * g.nz + izc);
        v = bload<R>(r, o * ES, 0);
        vp = bload<double>(rp, o * 8u, 0);
    };
    R qv[7];
    double qp[7];
    const int xa = x0 - 3, xb = x1 + 3;  // source slices
#pragma unroll
    for (int j = 0; j < 7; ++j) x_value(xa - 3 + j, qv[j], qp[j]);
    // accumulators of targets xs - 3 .. xs + 3 (phi1, psi)
    R a0[7], a1[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        a0[j] = (R)0;
        a1[j] = (R)0;
    }
    // mu (lambda of the output, 0 in the source ball and outside the grid)
    // and V of the own cell, fetched one slice ahead: the raw lambda and the
    // live flag (the select waits for the load, so it is made at the shift)
    auto own_mu_v = [&](int x, R& l0, double& l1, bool& live, R& vx, R& vz, R& vt) {
        const int xc = min(max(x, 0), g.nx - 1);
        const unsigned c = kb + (unsigned)(xc * g.nz + izc);
        l0 = bload<R>(rL, c * ES, 0);
        l1 = bload<double>(pL, c * 8u, 0);
        vx = bload<R>(rV, c * ES, EGB_VX * SP);
        vz = bload<R>(rV, c * ES, EGB_VZ * SP);
        vt = bload<R>(rV, c * ES, EGB_VT * SP);
        live = zin && !in_ball(xc, izc);
    };
    R cm0, cvx, cvz, cvt;
    double cm1;
    {
        bool live;
        own_mu_v(xa, cm0, cm1, live, cvx, cvz, cvt);
        cm0 = live ? cm0 : (R)0;
        cm1 = live ? cm1 : 0.0;
    }

    // value cells of the next core slice, loaded at the end of the step before
    R vv[NVI], vv1[NVI];
    double vp[NVI], vp1[NVI];
    auto load_values = [&](int x) {
        const unsigned xo = (unsigned)(x * g.nz);
#pragma unroll
        for (int r = 0; r < NVI; ++r) {
            unsigned vb, vbd;
            int vm;
            vcell(tid + r * NT, vb, vm, vbd);
            const unsigned o = vb + xo;
            vv[r] = bload<R>(rUi, o * ES, 0);
            vp[r] = bload<double>(pUi, o * 8u, 0);
            if (z_end) {  // the boundary-data value, kept by ghost cells
                const unsigned o1 = vbd + (unsigned)(x * 6);
                vv1[r] = bload<R>(rB, o1 * ES, 0);
                vp1[r] = bload<double>(pB, o1 * 8u, 0);
            }
        }
    };

    // halo sources' mu and V of this core slice (h) and of the next (nh: raw
    // lambda and the live flag, selected at the shift), loaded with the
    // values one step ahead; the V plane goes into the per-lane offset (a
    // per-lane scalar offset would make the load a loop over its values)
    R hm0[NHI], hvel[NHI], nhm0[NHI], nhvel[NHI];
    double hm1[NHI], nhm1[NHI];
    bool nhlive[NHI];
    auto load_halo = [&](int x) {
        const unsigned xo = (unsigned)(x * g.nz);
#pragma unroll
        for (int r = 0; r < NHI; ++r) {
            int tl, zl;
            bool real;
            unsigned hc;
            hcell(tid + r * NT, tl, zl, real, hc);
            const unsigned c = (hc + xo) * ES, c8 = (hc + xo) * 8u;
            nhm0[r] = bload<R>(rL, c, 0);
            nhm1[r] = bload<double>(pL, c8, 0);
            nhvel[r] = bload<R>(rV, c + (unsigned)(tid + r * NT < 6 * TZ ? EGB_VT : EGB_VZ) * SP, 0);
            nhlive[r] = real && !in_ball(x, tzi * TZ + zl);
        }
    };

    for (int xs = xa; xs < xb; ++xs) {
        const bool src = xs >= 0 && xs < g.nx;  // block-uniform
        const bool core = xs >= x0 && xs < x1;
        if (core) {
            // value slice into LDS (every read of the previous slice ended
            // before the previous step's second barrier)
#pragma unroll
            for (int r = 0; r < NVI; ++r) {
                const int i = tid + r * NT;
                if (i < NV) {
                    R v0 = vv[r];
                    double v1 = vp[r];
                    unsigned vb, vbd;
                    int vm;
                    vcell(i, vb, vm, vbd);
                    if (z_end && vm != 0) {
                        v0 = vm != 100 ? vv1[r] : (R)0;
                        v1 = vm != 100 ? vp1[r] : 0.0;
                    }
                    sm.w[i] = __builtin_bit_cast(Wd, v0);
                    const unsigned long long b = __builtin_bit_cast(unsigned long long, v1);
                    if constexpr (sizeof(R) == 4) {
                        sm.w[i + S::PLANE] = (unsigned)b;
                        sm.w[i + 2 * S::PLANE] = (unsigned)(b >> 32);
                    } else {
                        sm.w[i + S::PLANE] = b;
                    }
                }
            }
        }
        // prefetch: queue entry xs + 4, own mu and V of slice xs + 1
        R qn;
        double qpn;
        x_value(xs + 4, qn, qpn);
        R nm0, nvx, nvz, nvt;
        double nm1;
        bool nlive;
        own_mu_v(xs + 1, nm0, nm1, nlive, nvx, nvz, nvt);
        const unsigned xo = (unsigned)(min(max(xs, 0), g.nx - 1) * g.nz);
        const unsigned cR = (kb + xo + (unsigned)izc) * ES;
        // loads consumed later in the step: the output target's lambda and
        // accumulated lambda (clamped, used only when written), own gvel
        const int xt = xs - 3;
        const bool out = valid && xt >= x0 && xt < x1;
        const unsigned co = kb + (unsigned)(min(max(xt, 0), g.nx - 1) * g.nz + izc);
        const R ol0 = bload<R>(rL, co * ES, 0);
        const double ol1 = bload<double>(pL, co * 8u, 0);
        R oa0 = (R)0;
        double oa1 = 0.0;
        if constexpr (STAGE != 2) {
            const auto rAi = make_rsrc(a.acc_in, a.state_bytes);
            const auto pAi = make_rsrc(static_cast<const char*>(a.acc_in) + a.psi_off, a.psi_bytes);
            oa0 = bload<R>(rAi, co * ES, 0);
            oa1 = bload<double>(pAi, co * 8u, 0);
        }
        const bool wlive = __any(cm0 != (R)0 || cm1 != 0.0);  // wave-uniform
        // the next core slice's values and halo, one step ahead: their latency
        // hides behind this step's rows (the registers of this slice's values
        // are free once it is in LDS)
        if (xs + 1 >= x0 && xs + 1 < x1) {  // block-uniform
            load_values(xs + 1);
            load_halo(xs + 1);
        }
        R gsx = (R)0;  // this step's x term of gvel
        // x rows of the own column
        if (src && wlive) {
            const bool plus = cvx >= (R)0;
            R du[6], d[NSLOT];
            auto u = [&](const auto& q, int m) { return plus ? q[m] : q[6 - m]; };
            // the block owning a source within 3 of an x end folds its ghost slots
            const bool xfold = (xs < 3 || xs > g.nx - 4) && core;  // block-uniform
            double f[4];
            const R W0 = wgrad_up<R>(u(qv, 0), u(qv, 1), u(qv, 2), qv[3], u(qv, 4), u(qv, 5), du);
            to_slots(du, plus, (R)(-kx) * fabs(cvx) * cm0, d);
            if (xfold) fold_weights(d, xs, g.nx, f[0], f[1]);
#pragma unroll
            for (int j = 0; j < NSLOT; ++j) a0[j] += d[j];
            const R W1 = wgrad_up<R>(u(qp, 0), u(qp, 1), u(qp, 2), qp[3], u(qp, 4), u(qp, 5), du);
            to_slots(du, plus, (R)(-kx * (double)fabs(cvx) * cm1), d);
            if (xfold) fold_weights(d, xs, g.nx, f[2], f[3]);
#pragma unroll
            for (int j = 0; j < NSLOT; ++j) a1[j] += d[j];
            if (xfold && valid) {
                const int e = xs < 3 ? 0 : 1, sidx = e == 0 ? xs : g.nx - 1 - xs;
#pragma unroll
                for (int q = 0; q < 4; ++q) add_to(&a.bfold[bfold_x(g, q >> 1, k, e, sidx, q & 1, iz)], f[q]);
            }
            // d(-cb dt V_x D_x U / dx)/dV_x with D_x U = sign * W_up / dx
            gsx = (R)(plus ? -kx : kx) * (cm0 * W0 + (R)cm1 * W1);
        }
        if (core) {
            __syncthreads();
            // z and theta rows of a source at LDS (tl, zl): slots scaled by
            // -cb dt |V| mu / h, stored at the source position; the own cell
            // of a valid lane within 3 of a z end folds its ghost slots
            auto row = [&](int tl, int zl, bool zaxis, R vel, R m0, double m1, int zg, R& Wsum, bool own) {
                const int base = ((tl + 6) * S::VZ + zl + 6) * WS;
                const bool plus = vel >= (R)0;
                const int step = (zaxis ? WS : S::VZ * WS) * (plus ? 1 : -1);
                const int b0 = base - 3 * step, b1 = base - 2 * step, b2 = base - step;
                const int b4 = base + step, b5 = base + 2 * step;
                R du[6], d[NSLOT];
                const double kk = zaxis ? kz : kt;
                const int stride = zaxis ? S::ZPL : S::TPL;
                R* dst = zaxis ? sm.cz + tl * S::CZW + zl + 3 : sm.ct + (tl + 3) * TZ + zl;
                const bool fold = own && zaxis && (zg < 3 || zg > g.nz - 4);
                double f[4];
                const R W0 = wgrad_up<R>(lds_r<R>(sm, b0, 0), lds_r<R>(sm, b1, 0), lds_r<R>(sm, b2, 0),
                                         lds_r<R>(sm, base, 0), lds_r<R>(sm, b4, 0), lds_r<R>(sm, b5, 0), du);
                to_slots(du, plus, (R)(-kk) * fabs(vel) * m0, d);
                if (fold) fold_weights(d, zg, g.nz, f[0], f[1]);
#pragma unroll
                for (int j = 0; j < NSLOT; ++j) dst[j * stride] = d[j];
                const R W1 = wgrad_up<R>(lds_psi<1>(sm, b0), lds_psi<1>(sm, b1), lds_psi<1>(sm, b2),
                                         lds_psi<1>(sm, base), lds_psi<1>(sm, b4), lds_psi<1>(sm, b5), du);
                to_slots(du, plus, (R)(-kk * (double)fabs(vel) * m1), d);
                if (fold) {
                    fold_weights(d, zg, g.nz, f[2], f[3]);
                    const int e = zg < 3 ? 0 : 1, sidx = e == 0 ? zg : g.nz - 1 - zg;
#pragma unroll
                    for (int q = 0; q < 4; ++q) add_to(&a.bfold[bfold_z(g, q >> 1, k, xs, e, sidx, q & 1)], f[q]);
                }
#pragma unroll
                for (int j = 0; j < NSLOT; ++j) dst[(NSLOT + j) * stride] = d[j];
                Wsum = (plus ? (R)1 : (R)-1) * (m0 * W0 + (R)m1 * W1);
            };
            auto zero_row = [&](int tl, int zl, bool zaxis) {
                R* dst0 = zaxis ? sm.cz + tl * S::CZW + zl + 3 : sm.ct + (tl + 3) * TZ + zl;
                const int stride = zaxis ? S::ZPL : S::TPL;
#pragma unroll
                for (int j = 0; j < 2 * NSLOT; ++j) dst0[j * stride] = (R)0;
            };
            R Wz = (R)0, Wt = (R)0;
            if (wlive) {
                row(tk, tz, true, cvz, cm0, cm1, izc, Wz, valid);
                row(tk, tz, false, cvt, cm0, cm1, izc, Wt, false);
            } else {
                zero_row(tk, tz, true);
                zero_row(tk, tz, false);
            }
#pragma unroll
            for (int r = 0; r < NHI; ++r) {
                const int h = tid + r * NT;
                if (h < NH) {
                    int tl, zl;
                    bool real;
                    unsigned hc;
                    hcell(h, tl, zl, real, hc);
                    const bool zaxis = h >= 6 * TZ;
                    R wh;  // a halo source's V term belongs to another tile
                    if (__any(hm0[r] != (R)0 || hm1[r] != 0.0))
                        row(tl, zl, zaxis, hvel[r], hm0[r], hm1[r], tzi * TZ + zl, wh, false);
                    else zero_row(tl, zl, zaxis);
                }
            }
            if (valid && wlive) {
                R* gv = reinterpret_cast<R*>(static_cast<char*>(a.gvel) + cR);
                add_to(gv, gsx);
                add_to(gv + g.stride, (R)(-kz) * Wz);
                add_to(gv + 2 * g.stride, (R)(-kt) * Wt);
            }
            __syncthreads();
            // sum the slots aimed at the own cell (all 28 reads issued
            // before the sums, which keep their order)
            R sz0[NSLOT], st0[NSLOT], sz1[NSLOT], st1[NSLOT];
#pragma unroll
            for (int j = 0; j < NSLOT; ++j) {
                const int zsrc = tz - (j - 3), tsrc = tk - (j - 3);
                sz0[j] = sm.cz[j * S::ZPL + tk * S::CZW + zsrc + 3];
                st0[j] = sm.ct[j * S::TPL + (tsrc + 3) * TZ + tz];
                sz1[j] = sm.cz[(NSLOT + j) * S::ZPL + tk * S::CZW + zsrc + 3];
                st1[j] = sm.ct[(NSLOT + j) * S::TPL + (tsrc + 3) * TZ + tz];
            }
            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int j = 0; j < NSLOT; ++j) {
                t0 += (double)sz0[j] + (double)st0[j];
                t1 += (double)sz1[j] + (double)st1[j];
            }
            a0[3] += (R)(t0 + cb * (double)cm0);
            a1[3] += (R)(t1 + cb * cm1);
        }
        // target xs - 3 is complete
        if (out) {
            const unsigned c = co;
            const R l0 = ol0;
            const double l1 = ol1;
            const bool ball = in_ball(xt, iz);
            const R add0 = ball ? l0 : (R)ca * l0;
            const double add1 = ball ? l1 : ca * l1;
            const auto rAo = make_rsrc(a.acc_out, a.state_bytes);
            const auto pAo = make_rsrc(static_cast<char*>(a.acc_out) + a.psi_off, a.psi_bytes);
            if constexpr (STAGE == 2) {
                bstore(add0, rAo, c * ES, 0);
                bstore(add1, pAo, c * 8u, 0);
            } else {
                R o0 = oa0 + add0;
                double o1 = oa1 + add1;
                if constexpr (STAGE == 0) {
                    o0 += a0[0];
                    o1 += (double)a1[0];
                }
                bstore(o0, rAo, c * ES, 0);
                bstore(o1, pAo, c * 8u, 0);
            }
            if constexpr (STAGE != 0) {
                const auto rLi = make_rsrc(a.lam_in, a.state_bytes);
                const auto pLi = make_rsrc(static_cast<char*>(a.lam_in) + a.psi_off, a.psi_bytes);
                bstore(a0[0], rLi, c * ES, 0);
                bstore((double)a1[0], pLi, c * 8u, 0);
            }
        }
        // shift
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            qv[j] = qv[j + 1];
            qp[j] = qp[j + 1];
            a0[j] = a0[j + 1];
            a1[j] = a1[j + 1];
        }
        qv[6] = qn;
        qp[6] = qpn;
        a0[6] = (R)0;
        a1[6] = (R)0;
        cm0 = nlive ? nm0 : (R)0;
        cm1 = nlive ? nm1 : 0.0;
        cvx = nvx;
        cvz = nvz;
        cvt = nvt;
#pragma unroll
        for (int r = 0; r < NHI; ++r) {
            hm0[r] = nhlive[r] ? nhm0[r] : (R)0;
            hm1[r] = nhlive[r] ? nhm1[r] : 0.0;
            hvel[r] = nhvel[r];
        }
    }
}

template <typename R, int STAGE, int TK>
__global__ __launch_bounds__(64 * TK) void k_adj_stage(AdjStageArgs a) {
    __shared__ AdjSmem<R, TK> sm;
    // the (tile, x) targets, x fastest, split into gridDim.x equal contiguous
    // ranges (one round of resident blocks), as in the forward stage
    const long long W = (long long)a.ntz * a.ntk * a.g.nx;
    const long long b = xcd_remap(blockIdx.x, gridDim.x);
    long long w = W * b / gridDim.x;
    const long long w1 = W * (b + 1) / gridDim.x;
    while (w < w1) {
        const int tile = (int)(w / a.g.nx), xa = (int)(w % a.g.nx);
        const int xb = (int)min((long long)a.g.nx, xa + (w1 - w));
        adj_tile<R, STAGE, TK>(a, tile, xa, xb, sm);
        w += xb - xa;
        if (w < w1) __syncthreads();  // the segment's last LDS reads are done
    }
}

// Adjoint of the first-arrival pick: lambda += tbar dt/d(phi1, psi).  One
// block: receivers are differentiated in parallel (256 at a time) and their
// 16 contributions applied by one thread in receiver order, so the sum is
// deterministic when receivers share cells.
template <typename R>
__global__ __launch_bounds__(256) void k_pick_adjoint(GridArgs a, const char* state, const double* rx, int nr,
                                                      const double* tbar, char* lam) {
    __shared__ long long cell[256][8];
    __shared__ double val[256][16];
    __shared__ int has[256];
    const R* phi = reinterpret_cast<const R*>(state);
    const double* psi = reinterpret_cast<const double*>(phi + EGB_PSI * a.stride);
    R* lphi = reinterpret_cast<R*>(lam);
    double* lpsi = reinterpret_cast<double*>(lphi + EGB_PSI * a.stride);
    for (int base = 0; base < nr; base += 256) {
        const int r = base + (int)threadIdx.x;
        has[threadIdx.x] = 0;
        if (r < nr) {
            const double fx = (rx[2 * r] - a.x0) / a.dx - 0.5, fz = (rx[2 * r + 1] - a.z0) / a.dz - 0.5;
            int ix = (int)floor(fx), iz = (int)floor(fz);
            ix = min(max(ix, 0), a.nx - 2);
            iz = min(max(iz, 0), a.nz - 2);
            const double tx = fmin(fmax(fx - ix, 0.0), 1.0), tz = fmin(fmax(fz - iz, 0.0), 1.0);
            const double w[4] = {(1 - tx) * (1 - tz), tx * (1 - tz), (1 - tx) * tz, tx * tz};
            const long long o = (long long)ix * a.nz + iz;
            const long long off[4] = {0, a.nz, 1, a.nz + 1};
            auto ip = [&](int k) {
                const R* p = phi + (long long)k * a.nxz + o;
                double s = 0.0;
                for (int q = 0; q < 4; ++q) s += w[q] * (double)p[off[q]];
                return s;
            };
            auto is = [&](int k) {
                const double* p = psi + (long long)k * a.nxz + o;
                double s = 0.0;
                for (int q = 0; q < 4; ++q) s += w[q] * p[off[q]];
                return s;
            };
            double best = 0.0, bf0 = 0, bf1 = 0, bs0 = 0, bs1 = 0;
            int kb = -1;
            double f0 = ip(0), s0 = is(0);
            const double fstart = f0, sstart = s0;
            for (int k = 0; k < a.nth; ++k) {
                const bool last = (k == a.nth - 1);
                const double f1 = last ? fstart : ip(k + 1);
                const double s1 = last ? sstart : is(k + 1);
                if (f0 == 0.0 || f0 * f1 < 0.0) {
                    const double t = f0 / (f0 - f1);
                    const double v = s0 + t * (s1 - s0);
                    if (v > 0.0 && (kb < 0 || v < best)) {
                        best = v;
                        kb = k;
                        bf0 = f0; bf1 = f1; bs0 = s0; bs1 = s1;
                    }
                }
                f0 = f1;
                s0 = s1;
            }
            if (kb >= 0) {
                const double tb = tbar[r];
                const double den = bf0 - bf1, t = bf0 / den;
                const double d_s0 = (1.0 - t) * tb, d_s1 = t * tb;
                const double d_f0 = (bs1 - bs0) * (-bf1) / (den * den) * tb;
                const double d_f1 = (bs1 - bs0) * bf0 / (den * den) * tb;
                const int k1 = kb == a.nth - 1 ? 0 : kb + 1;
                for (int q = 0; q < 4; ++q) {
                    cell[threadIdx.x][q] = (long long)kb * a.nxz + o + off[q];
                    cell[threadIdx.x][4 + q] = (long long)k1 * a.nxz + o + off[q];
                    val[threadIdx.x][q] = w[q] * d_f0;
                    val[threadIdx.x][4 + q] = w[q] * d_f1;
                    val[threadIdx.x][8 + q] = w[q] * d_s0;
                    val[threadIdx.x][12 + q] = w[q] * d_s1;
                }
                has[threadIdx.x] = 1;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int n = min(256, nr - base);
            for (int i = 0; i < n; ++i) {
                if (!has[i]) continue;
                for (int q = 0; q < 8; ++q) {
                    lphi[cell[i][q]] = (R)((double)lphi[cell[i][q]] + val[i][q]);
                    lpsi[cell[i][q]] += val[i][8 + q];
                }
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ long long cidx3(const GridArgs& a, int f, int t, int ix, int iz) {
    return ((long long)(f * NT + t)) * a.nxz + (long long)ix * a.nz + iz;
}

// dJ/d(table entry j) at (x, z) = sum over theta of g_V . dV/d(entry), for the
// 15 entries (field value, d/dx, d/dz) that V depends on (forward-mode dual).
template <typename R>
__global__ void k_adj_vtable(GridArgs a, const double* C, const R* gvel, double* gtab) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 15 * a.nxz) return;
    const int j = (int)(id / a.nxz);
    const long long cz = id % a.nxz;
    const int ix = (int)(cz / a.nz), iz = (int)(cz % a.nz);
    const int jf = j / 3, js = j % 3;
    Dual m[NF][3];
    for (int f = 0; f < NF; ++f)
        for (int s = 0; s < 3; ++s) m[f][s] = dual(C[cidx3(a, f, s, ix, iz)], (f == jf && s == js) ? 1.0 : 0.0);
    double acc = 0.0;
    for (int k = 0; k < a.nth; ++k) {
        Dual V[3];
        liouville_velocity_dual(m, k * a.dth, V);
        const long long c = (long long)k * a.nxz + cz;
        acc += (double)gvel[c] * V[0].d + (double)gvel[a.stride + c] * V[1].d + (double)gvel[2 * a.stride + c] * V[2].d;
    }
    gtab[id] = acc;
}

// Bilinear source weights of node (ix, iz) (medium frozen at the source).
__device__ double source_weight(const GridArgs& a, double xs, double zs, int ix, int iz) {
    const double fx = (xs - a.x0) / a.dx - 0.5, fz = (zs - a.z0) / a.dz - 0.5;
    int sx = (int)floor(fx), sz = (int)floor(fz);
    sx = min(max(sx, 0), a.nx - 2);
    sz = min(max(sz, 0), a.nz - 2);
    const double tx = fmin(fmax(fx - sx, 0.0), 1.0), tz = fmin(fmax(fz - sz, 0.0), 1.0);
    const double wx = ix == sx ? 1 - tx : (ix == sx + 1 ? tx : 0.0);
    const double wz = iz == sz ? 1 - tz : (iz == sz + 1 ? tz : 0.0);
    return wx * wz;
}

// Point-source data phi1 = (x - xs).g_perp(theta; m_s), psi = p(theta; m_s).(x - xs):
// per theta slice, contract lambda0 and the boundary sensitivity (its
// entries sit on the end cells of the lines) with (x - xs, z - zs), then
// differentiate g_perp and p with respect to the five source values (dual
// numbers); the slice's five partial derivatives go to gms[k][5] (summed in
// order later).
template <typename R>
__global__ __launch_bounds__(256) void k_adj_source(GridArgs a, const double* C, egb_source src, const char* lam0,
                                                    const double* bfold, double* gms) {
    const int k = blockIdx.x;
    const R* lphi = reinterpret_cast<const R*>(lam0);
    const double* lpsi = reinterpret_cast<const double*>(lphi + EGB_PSI * a.stride);
    double s[4] = {0, 0, 0, 0};
    for (long long cz = threadIdx.x; cz < a.nxz; cz += blockDim.x) {
        const int ix = (int)(cz / a.nz), iz = (int)(cz % a.nz);
        const double X = a.x0 + (ix + 0.5) * a.dx - src.xs, Z = a.z0 + (iz + 0.5) * a.dz - src.zs;
        const long long c = (long long)k * a.nxz + cz;
        const double lf = (double)lphi[c], lp = lpsi[c];
        s[0] += lf * X;
        s[1] += lf * Z;
        s[2] += lp * X;
        s[3] += lp * Z;
    }
    // x lines: entry (end e, source, weight w, z) sits at x = 0, 1 / nx-1, nx-2
    for (int i = threadIdx.x; i < 12 * a.nz; i += blockDim.x) {
        const int z = i % a.nz, w = (i / a.nz) & 1, e = i / (6 * a.nz), sidx = (i / (2 * a.nz)) % 3;
        const int ix = e == 0 ? w : a.nx - 1 - w;
        const double X = a.x0 + (ix + 0.5) * a.dx - src.xs, Z = a.z0 + (z + 0.5) * a.dz - src.zs;
        for (int p = 0; p < 2; ++p) {
            const double v = bfold[bfold_x(a, p, k, e, sidx, w, z)];
            s[2 * p] += v * X;
            s[2 * p + 1] += v * Z;
        }
    }
    // z lines: entry (x, end e, source, weight w) sits at z = 0, 1 / nz-1, nz-2
    for (int i = threadIdx.x; i < 12 * a.nx; i += blockDim.x) {
        const int x = i / 12, e = (i / 6) & 1, sidx = (i / 2) % 3, w = i & 1;
        const int iz = e == 0 ? w : a.nz - 1 - w;
        const double X = a.x0 + (x + 0.5) * a.dx - src.xs, Z = a.z0 + (iz + 0.5) * a.dz - src.zs;
        for (int p = 0; p < 2; ++p) {
            const double v = bfold[bfold_z(a, p, k, x, e, sidx, w)];
            s[2 * p] += v * X;
            s[2 * p + 1] += v * Z;
        }
    }
    __shared__ double red[4][256];
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x >= NF) return;
    // thread j differentiates with respect to source value j
    double ms[NF];
    {
        const double fx = (src.xs - a.x0) / a.dx - 0.5, fz = (src.zs - a.z0) / a.dz - 0.5;
        int sx = (int)floor(fx), sz = (int)floor(fz);
        sx = min(max(sx, 0), a.nx - 2);
        sz = min(max(sz, 0), a.nz - 2);
        const double tx = fmin(fmax(fx - sx, 0.0), 1.0), tz = fmin(fmax(fz - sz, 0.0), 1.0);
        for (int f = 0; f < NF; ++f)
            ms[f] = (1 - tx) * (1 - tz) * C[cidx3(a, f, 0, sx, sz)] + tx * (1 - tz) * C[cidx3(a, f, 0, sx + 1, sz)] +
                    (1 - tx) * tz * C[cidx3(a, f, 0, sx, sz + 1)] + tx * tz * C[cidx3(a, f, 0, sx + 1, sz + 1)];
    }
    const int j = threadIdx.x;
    Dual m[NF][3];
    for (int f = 0; f < NF; ++f) {
        m[f][0] = dual(ms[f], f == j ? 1.0 : 0.0);
        m[f][1] = dual(0.0);
        m[f][2] = dual(0.0);
    }
    const double th = k * a.dth;
    Dual V[3], v;
    liouville_velocity_dual(m, th, V, &v);
    const Dual nv = dsqrt(V[0] * V[0] + V[1] * V[1]);
    const Dual gpx = V[1] / nv, gpz = -(V[0] / nv);
    double sn, cs;
    sincos(th, &sn, &cs);
    const Dual px = dual(sn) / v, pz = dual(cs) / v;
    gms[k * NF + j] = red[0][0] * gpx.d + red[1][0] * gpz.d + red[2][0] * px.d + red[3][0] * pz.d;
}

__device__ const double AW1C[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
__device__ const double AW1E0[5] = {-25.0, 48.0, -36.0, 16.0, -3.0};
__device__ const double AW1E1[5] = {-3.0, -10.0, 18.0, -6.0, 1.0};

// weight of f[j] in the 4th-order first difference at i (line of length n)
__device__ double fd1_weight(int n, int i, int j, double h) {
    if (i >= 2 && i <= n - 3) {
        const int off = j - i;
        return (off >= -2 && off <= 2) ? AW1C[off + 2] / (12.0 * h) : 0.0;
    }
    const bool lo = i < 2;
    const int e = lo ? i : n - 1 - i;
    const double* w = e == 0 ? AW1E0 : AW1E1;
    for (int m = 0; m < 5; ++m) {
        const int off = -e + m;
        const int jj = lo ? i + off : i - off;
        if (jj == j) return (lo ? 1.0 : -1.0) * w[m] / (12.0 * h);
    }
    return 0.0;
}

// Table gradients -> field gradients (transposed differences + the source
// weights) -> Thomsen parameters.  grad = [vp0, eps, delta, tilt][x][z].
__global__ void k_adj_fields(GridArgs a, egb_medium med, const double* gtab, const double* gms, egb_source src,
                             double* grad) {
    const long long cz = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cz >= a.nxz) return;
    const int ix = (int)(cz / a.nz), iz = (int)(cz % a.nz);
    const double ws = source_weight(a, src.xs, src.zs, ix, iz);
    double gsrc[NF] = {0, 0, 0, 0, 0};
    if (ws != 0.0)
        for (int k = 0; k < a.nth; ++k)
            for (int f = 0; f < NF; ++f) gsrc[f] += gms[k * NF + f];
    double gF[NF];
    for (int f = 0; f < NF; ++f) {
        double s = gtab[(long long)(f * 3 + 0) * a.nxz + cz] + ws * gsrc[f];
        const double* gx = gtab + (long long)(f * 3 + 1) * a.nxz;
        const double* gz = gtab + (long long)(f * 3 + 2) * a.nxz;
        for (int i = max(ix - 4, 0); i <= min(ix + 4, a.nx - 1); ++i)
            s += fd1_weight(a.nx, i, ix, a.dx) * gx[(long long)i * a.nz + iz];
        for (int j = max(iz - 4, 0); j <= min(iz + 4, a.nz - 1); ++j)
            s += fd1_weight(a.nz, j, iz, a.dz) * gz[(long long)ix * a.nz + j];
        gF[f] = s;
    }
    const double vp = med.vp0[cz], ep = med.eps[cz], de = med.delta[cz], fs = med.vs_ratio;
    const double a33 = vp * vp, a55 = fs * fs * a33;
    const double b = sqrt((a33 - a55) * (a33 * (1.0 + 2.0 * de) - a55));
    grad[0 * a.nxz + cz] = gF[0] * 2.0 * vp * (1.0 + 2.0 * ep) + gF[1] * 2.0 * vp + gF[2] * 2.0 * b / vp +
                           gF[3] * 2.0 * fs * fs * vp;
    grad[1 * a.nxz + cz] = gF[0] * 2.0 * a33;
    grad[2 * a.nxz + cz] = gF[2] * (a33 - a55) * a33 / b;
    grad[3 * a.nxz + cz] = gF[4];
}

template <typename R, int TK>
hipError_t adj_stage_t(AdjStageArgs a, int stage, hipStream_t s, int blocks) {
    a.ntz = (a.g.nz + TZ - 1) / TZ;
    a.ntk = (a.g.nth + TK - 1) / TK;
    const void* k = stage == 0 ? (const void*)k_adj_stage<R, 0, TK>
                  : stage == 1 ? (const void*)k_adj_stage<R, 1, TK> : (const void*)k_adj_stage<R, 2, TK>;
    const long long W = (long long)a.ntz * a.ntk * a.g.nx;
    // by default one round of resident blocks, each with at least 16 target
    // steps; `blocks` > 0 splits the steps over that many blocks instead
    long long G = blocks > 0 ? blocks : resident_blocks(k, 64 * TK);
    if (G <= 0) return hipErrorInvalidDeviceFunction;
    if (blocks <= 0) G = std::min(G, W / 16);
    G = std::max(1LL, std::min(G, W));
    const dim3 grid((unsigned)G), block(TZ, TK);
    switch (stage) {
        case 0: k_adj_stage<R, 0, TK><<<grid, block, 0, s>>>(a); break;
        case 1: k_adj_stage<R, 1, TK><<<grid, block, 0, s>>>(a); break;
        default: k_adj_stage<R, 2, TK><<<grid, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_stage(const GridArgs& g, int dtype, int stage, const void* vel, const void* bd,
                                const void* Uin, const void* lam_out, void* lam_in, const void* acc_in, void* acc_out,
                                void* gvel, void* bfold, double dt, double xs, double zs, double r02, hipStream_t s,
                                int blocks) {
    const unsigned long long es = dtype == EGB_F64 ? 8 : 4, S = (unsigned long long)g.stride;
    AdjStageArgs a;
    a.g = g;
    a.vel = vel;
    a.bd = bd;
    a.bfold = static_cast<double*>(bfold);
    a.Uin = Uin;
    a.lam = lam_out;
    a.acc_in = acc_in;
    a.acc_out = acc_out;
    a.lam_in = lam_in;
    a.gvel = gvel;
    a.dt = dt;
    a.xs = xs;
    a.zs = zs;
    a.r02 = r02;
    a.state_bytes = (unsigned)(S * es);  // plane phi1
    a.psi_off = (unsigned long long)EGB_PSI * S * es;
    a.psi_bytes = (unsigned)(S * 8);
    a.vel_bytes = (unsigned)(7 * S * es);
    a.gvel_bytes = (unsigned)(3 * S * es);
    a.bd_bytes = (unsigned)((unsigned long long)g.bstride * es);
    a.bpsi_off = (unsigned long long)EGB_PSI * g.bstride * es;
    a.bpsi_bytes = (unsigned)((unsigned long long)g.bstride * 8);
    a.ntz = a.ntk = 0;
    return dtype == EGB_F64 ? adj_stage_t<double, 4>(a, stage, s, blocks) : adj_stage_t<float, 8>(a, stage, s, blocks);
}

hipError_t launch_pick_adjoint(const GridArgs& a, int dtype, const void* state, const double* rx, int nr,
                               const double* tbar, void* lam, hipStream_t s) {
    if (nr <= 0) return hipSuccess;
    if (dtype == EGB_F64)
        k_pick_adjoint<double><<<1, 256, 0, s>>>(a, (const char*)state, rx, nr, tbar, (char*)lam);
    else
        k_pick_adjoint<float><<<1, 256, 0, s>>>(a, (const char*)state, rx, nr, tbar, (char*)lam);
    return hipGetLastError();
}

hipError_t launch_adjoint_medium(const GridArgs& a, int dtype, const egb_medium& m, const double* coeff2d,
                                 const egb_source& src, const void* gvel, const void* lam0, const double* bfold,
                                 double* grad, double* gtab, double* gms, hipStream_t s) {
    const long long nt = 15 * a.nxz;
    if (dtype == EGB_F64) {
        k_adj_vtable<double><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(a, coeff2d, (const double*)gvel, gtab);
        k_adj_source<double><<<a.nth, 256, 0, s>>>(a, coeff2d, src, (const char*)lam0, bfold, gms);
    } else {
        k_adj_vtable<float><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(a, coeff2d, (const float*)gvel, gtab);
        k_adj_source<float><<<a.nth, 256, 0, s>>>(a, coeff2d, src, (const char*)lam0, bfold, gms);
    }
    k_adj_fields<<<(unsigned)((a.nxz + 255) / 256), 256, 0, s>>>(a, m, gtab, gms, src, grad);
    return hipGetLastError();
}

}  // namespace egb
