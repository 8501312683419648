// Paraxial depth march (eqs. 13-15 with the Liouville transport of eqs.
// 16-24 divided by dz/dtau): on (x, theta) slices with theta in
// (-theta_max, theta_max) the state
//   X (the surface position of the ray), vartheta (its take-off angle),
//   tau (traveltime), C, B (complex dynamic ray tracing pair)
// obeys U_z + u U_x + w U_theta = S,  u = V_x / V_z, w = V_theta / V_z,
// S_tau = 1 / V_z, S_(C,B) = (A / V_z)(C, B), the other sources zero.  Each
// depth interval dz is nsub SSP-RK3 steps of dz / nsub in z, the
// coefficients linear in z between the two levels (stage depths s, s + h,
// s + h / 2 of the interval, h = 1 / nsub); x and theta ghosts hold the
// surface data extended linearly, fixed in depth (a ray entering through a
// side or an aperture edge carries it).  Every level is kept; first arrivals
// for a surface source at x_s follow from the level set X = x_s (eq. 35),
// over the nodes whose take-off angle lies inside the aperture.
//
// Level layout: planes X, vartheta, Re C, Im C, Re B, Im B, Phi in R, then
// tau in double, each [theta][x] (x fastest) padded to a multiple of 64
// elements.  Phi is the continuous phase of C along the ray (the KMAH phase):
// Phi_z + u Phi_x + w Phi_theta = (A12 / V_z) Im(B / C), 0 on the surface.
//
// Work decomposition: a block owns a tile of 64 x by 2 theta cells of one
// slice and has one wave per (plane, theta row), so that a slice of nx nth
// cells still gives every SIMD several waves; the tile with a 3-cell halo
// (ghosts filled while loading) goes to LDS once, then every thread reads its
// plane's x and theta stencils there at per-lane mirrored addresses
// (V D(U) = |V| W(values in upwind order), as in the phase-space stage
// kernel).  The march is a long chain of short launches queued in order on
// one stream.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "egb_device.h"
#include "egb_internal.h"
#include "stage_common.h"

namespace egb {
namespace {

constexpr int PTX = 64, PTT = 2;         // tile: x cells, theta rows
constexpr int NPL = 8;                   // planes, one wave each per theta row
constexpr int PRX = PTX + 6;             // LDS row (3-cell halo each side)
constexpr int PROWS = PTT + 6;
constexpr int PCELLS = PROWS * PRX;      // LDS cells per plane
constexpr int NT = PTX * PTT * NPL;      // threads per block
constexpr int NPR = 7;                   // R planes: X, vartheta, ReC, ImC, ReB, ImB, Phi (then tau)
enum { Q_X = 0, Q_VT = 1, Q_RC = 2, Q_IC = 3, Q_RB = 4, Q_IB = 5, Q_PH = 6, Q_TAU = 7 };
// velocity planes: u, w, S_tau, A11/Vz, A12/Vz, A21/Vz, A22/Vz

template <typename R>
struct PSmem {
    using W = typename LdsWord<R>::T;
    static constexpr int PLANE = (PCELLS + 63) / 64 * 64;
    static constexpr int PB = PLANE * (int)sizeof(W);
    W w[(NPR + LdsWord<R>::PSI_WORDS) * PLANE];
};

// Source of the LDS cell at slice position (x, k) in a tile that touches an
// end: inside the slice the marched value u[i0] (no ghost); beyond an x end
// or a theta end the surface data b extended linearly from the two cells
// next to that end, w0 b[i0] + w1 b[i1] with (w0, w1) = (m + 1, -m) for the
// ghost m cells outside; cells beyond both ends are never read (weights 0).
// Branch-free: every lane of a wave takes the same instructions.
__device__ __forceinline__ void pghost_src(int nx, int nth, int x, int k, int& i0, int& i1, int& w0, int& w1,
                                           bool& ghost) {
    const int mx = x < 0 ? -x : max(x - (nx - 1), 0);
    const int mk = k < 0 ? -k : max(k - (nth - 1), 0);
    const int xa = mx ? (x < 0 ? 0 : nx - 1) : x, xb = mx ? (x < 0 ? 1 : nx - 2) : x;
    const int ka = mk ? (k < 0 ? 0 : nth - 1) : k, kb = mk ? (k < 0 ? 1 : nth - 2) : k;
    const int m = mx + mk;
    const bool both = mx != 0 && mk != 0;
    i0 = ka * nx + xa;
    i1 = kb * nx + xb;
    ghost = m != 0;
    w0 = both ? 0 : m + 1;
    w1 = both ? 0 : -m;
}

// One RK stage on a 64 x 2 (x, theta) tile: thread (x, row, plane), so
// every wave holds one plane of one theta row and all branches on the plane
// are wave-uniform.  The tile of every plane with its halo is loaded to LDS
// by the waves of that plane: each thread takes the rows y, y + 2, y + 4,
// y + 6 at its own column and the first 48 threads one of the six halo
// columns of a row (all loads of a thread issued together; the ghost logic
// only in tiles that touch an end).  The x and theta stencils are then read
// at per-lane mirrored addresses.  The cell's coefficients and stage-start
// value are fetched before the barrier.  Offsets are 32-bit (one level
// stays below 2 GiB).
template <typename R, int STAGE>
__global__ __launch_bounds__(NT) void k_pstage(PStageArgs a) {
    using S = PSmem<R>;
    using Wd = typename S::W;
    constexpr int WS = (int)sizeof(Wd);
    constexpr int NMAIN = PROWS / PTT;  // tile rows per thread
    static_assert(PROWS % PTT == 0 && 6 * PROWS <= PTX * PTT, "fill mapping");
    __shared__ S sm;
    const int nx = a.nx, nth = a.nth, P = (int)a.P;
    const int ntx = (nx + PTX - 1) / PTX;
    const int tx0 = (blockIdx.x % ntx) * PTX, tk0 = (blockIdx.x / ntx) * PTT;
    const int p = threadIdx.z;  // plane (wave-uniform)
    const int ty = threadIdx.y, tx = threadIdx.x;
    const int pt = ty * PTX + tx;
    const bool edge = tx0 < 3 || tx0 + PTX + 3 > nx || tk0 < 3 || tk0 + PTT + 3 > nth;  // block-uniform

    // own cell (clamped for threads past the slice) and its prefetched inputs
    const int x = tx0 + tx, k = tk0 + ty;
    const bool valid = x < nx && k < nth;
    const int c = min(k, nth - 1) * nx + min(x, nx - 1);
    const R* p0 = static_cast<const R*>(a.pv0);
    const R* p1 = static_cast<const R*>(a.pv1);
    const bool isC = p == Q_RC || p == Q_IC;
    const int qa = p == Q_TAU ? 2 : (p == Q_PH ? 4 : (isC ? 3 : 5));  // this plane's source coefficients
    const R u0 = p0[c], u1 = p1[c], w0 = p0[P + c], w1 = p1[P + c];
    const R a0 = p0[qa * P + c], a1 = p1[qa * P + c];
    const R b0 = p0[(qa + 1) * P + c], b1 = p1[(qa + 1) * P + c];
    const R* Ui = static_cast<const R*>(a.Uin);
    const R* Ub = static_cast<const R*>(a.Ub);  // surface data (level 0): the ghosts
    R r0 = (R)0;
    double t0 = 0.0;
    if constexpr (STAGE != 0) {
        const R* U0 = static_cast<const R*>(a.U0);
        if (p == Q_TAU) t0 = reinterpret_cast<const double*>(U0 + NPR * P)[c];
        else r0 = U0[p * P + c];
    }

    // this plane's tile + halo into LDS
    const bool hal = pt < 6 * PROWS;  // a halo-column cell: row pt / 6, column 0..2 or 67..69
    const int er = pt / 6, ej = pt - 6 * er;
    const int ec = ej < 3 ? ej : ej + PTX;
    auto fill = [&](auto tag) {
        using T = decltype(tag);
        const int po = p == Q_TAU ? NPR * P : p * P;
        const T* u = reinterpret_cast<const T*>(Ui + po);
        const T* ub = reinterpret_cast<const T*>(Ub + po);
        T v[NMAIN + 1];
        if (!edge) {
            const int base = (tk0 - 3 + ty) * nx + x;
#pragma unroll
            for (int j = 0; j < NMAIN; ++j) v[j] = u[base + j * PTT * nx];
            if (hal) v[NMAIN] = u[(tk0 - 3 + er) * nx + tx0 - 3 + ec];
        } else {
            T f[NMAIN + 1], g[NMAIN + 1];
            int wa[NMAIN + 1], wb[NMAIN + 1];
            bool gh[NMAIN + 1];
#pragma unroll
            for (int j = 0; j <= NMAIN; ++j) {
                if (j == NMAIN && !hal) break;
                const int gx = j < NMAIN ? x : tx0 - 3 + ec;
                const int gk = tk0 - 3 + (j < NMAIN ? ty + j * PTT : er);
                int i0, i1;
                pghost_src(nx, nth, gx, gk, i0, i1, wa[j], wb[j], gh[j]);
                f[j] = (gh[j] ? ub : u)[i0];
                g[j] = ub[i1];
            }
#pragma unroll
            for (int j = 0; j <= NMAIN; ++j) {
                if (j == NMAIN && !hal) break;
                v[j] = gh[j] ? (T)wa[j] * f[j] + (T)wb[j] * g[j] : f[j];
            }
        }
#pragma unroll
        for (int j = 0; j <= NMAIN; ++j) {
            if (j == NMAIN && !hal) break;
            const int i = j < NMAIN ? (ty + j * PTT) * PRX + tx + 3 : er * PRX + ec;
            if constexpr (sizeof(T) == sizeof(Wd)) {
                sm.w[(p == Q_TAU ? NPR : p) * S::PLANE + i] = __builtin_bit_cast(Wd, v[j]);
            } else {  // tau of an FP32 slice: two 32-bit planes
                const unsigned long long bits = __builtin_bit_cast(unsigned long long, v[j]);
                sm.w[NPR * S::PLANE + i] = (Wd)(unsigned)bits;
                sm.w[(NPR + 1) * S::PLANE + i] = (Wd)(unsigned)(bits >> 32);
            }
        }
    };
    if (p == Q_TAU) fill(0.0);
    else fill((R)0);
    __syncthreads();

    if (!valid) return;
    // coefficients at this stage's depth: u and w, then this plane's source
    const R s1 = (R)a.s, s0 = (R)(1.0 - a.s);
    const R cu = s0 * u0 + s1 * u1, cw = s0 * w0 + s1 * w1;
    const R ca_ = s0 * a0 + s1 * a1, cb_ = s0 * b0 + s1 * b1;
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    const double cdl = cb * a.dl;
    const R gx = fabs(cu) * (R)(cdl / a.dx), gt = fabs(cw) * (R)(cdl / a.dth), cdr = (R)cdl;
    const int meB = ((ty + 3) * PRX + tx + 3) * WS;
    const int sx = cu >= (R)0 ? WS : -WS, st = cw >= (R)0 ? PRX * WS : -PRX * WS;
    R* Uo = static_cast<R*>(a.Uout);
    if (p == Q_TAU) {
        const double own = lds_psi<NPR>(sm, meB);
        auto wup = [&](int step) {
            return weno_up<R>(lds_psi<NPR>(sm, meB - 3 * step), lds_psi<NPR>(sm, meB - 2 * step),
                              lds_psi<NPR>(sm, meB - step), own, lds_psi<NPR>(sm, meB + step),
                              lds_psi<NPR>(sm, meB + 2 * step));
        };
        const R conv = gx * wup(sx) + gt * wup(st);
        double acc = cb * own + cdl * (double)ca_ - (double)conv;
        if constexpr (STAGE != 0) acc += ca * t0;
        reinterpret_cast<double*>(Uo + NPR * P)[c] = acc;
        return;
    }
    const R own = lds_r<R>(sm, meB, p);
    auto wup = [&](int step) {
        return weno_up<R>(lds_r<R>(sm, meB - 3 * step, p), lds_r<R>(sm, meB - 2 * step, p),
                          lds_r<R>(sm, meB - step, p), own, lds_r<R>(sm, meB + step, p),
                          lds_r<R>(sm, meB + 2 * step, p));
    };
    R acc = (R)cb * own - gx * wup(sx) - gt * wup(st);
    if (p == Q_PH) {
        // continuous phase of C: (A12 / V_z) Im(B / C)
        const R rc = lds_r<R>(sm, meB, Q_RC), ic = lds_r<R>(sm, meB, Q_IC);
        const R rb = lds_r<R>(sm, meB, Q_RB), ib = lds_r<R>(sm, meB, Q_IB);
        acc += cdr * ca_ * ((ib * rc - rb * ic) / (rc * rc + ic * ic));
    } else if (p >= Q_RC) {
        // (C, B) pairs (Re C, Re B) and (Im C, Im B): C' = A11 C + A12 B, B' = A21 C + A22 B
        const R cC = lds_r<R>(sm, meB, isC ? p : p - 2), cB = lds_r<R>(sm, meB, isC ? p + 2 : p);
        acc += cdr * (ca_ * cC + cb_ * cB);
    }
    if constexpr (STAGE != 0) acc += (R)ca * r0;
    Uo[p * P + c] = acc;
}

// Surface data on level 0: X = x, vartheta = theta, tau = 0,
// C = cos(theta) + sin(theta) u, Phi = 0, B = i eps C with eps = beta for
// the ray-normal pair (B an angle) or beta / v for the lateral-frame pair of
// eqs. 21-23 (B / C a traveltime Hessian; v = u1 / S_tau, so B = i beta S_tau).
template <typename R>
__global__ __launch_bounds__(256) void k_pinit(int nx, int nth, long long P, double x0, double dx, double theta_max,
                                               double beta, int drt, const R* pv, R* U) {
    const int x = blockIdx.x * 64 + threadIdx.x, k = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || k >= nth) return;
    const double dth = 2.0 * theta_max / nth;
    const double th = -theta_max + (k + 0.5) * dth;
    const long long c = (long long)k * nx + x;
    double sn, cs;
    sincos(th, &sn, &cs);
    const double c0 = cs + sn * (double)pv[c];
    U[Q_X * P + c] = (R)(x0 + (x + 0.5) * dx);
    U[Q_VT * P + c] = (R)th;
    U[Q_RC * P + c] = (R)c0;
    U[Q_IC * P + c] = (R)0;
    U[Q_RB * P + c] = (R)0;
    U[Q_IB * P + c] = (R)(drt == EGB_DRT_PAPER23 ? beta * (double)pv[2 * P + c] : beta * c0);
    U[Q_PH * P + c] = (R)0;
    reinterpret_cast<double*>(U + NPR * P)[c] = 0.0;
}

// First arrival at (x_i, level n) for surface source s: roots in theta of
// X - x_s between adjacent nodes whose take-off angles lie inside the
// aperture, tau interpolated linearly, the smallest tau > 0 (NaN when there
// is none).  T[s][n][i].
template <typename R>
__global__ __launch_bounds__(256) void k_ppick(int nx, int nz, int nth, double theta_max, long long P,
                                               const char* levels, size_t level_bytes, const double* xs, int nsrc,
                                               double* T) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)nsrc * nz * nx;
    if (id >= total) return;
    const int i = (int)(id % nx), n = (int)((id / nx) % nz), s = (int)(id / ((long long)nx * nz));
    const R* X = reinterpret_cast<const R*>(levels + (size_t)n * level_bytes) + i;
    const double* tau = reinterpret_cast<const double*>(reinterpret_cast<const R*>(levels + (size_t)n * level_bytes) +
                                                        NPR * P) + i;
    const R* VT = X + P;  // take-off angle
    const double x_s = xs[s];
    double best = __longlong_as_double(0x7ff8000000000000LL);
    double f0 = (double)X[0] - x_s, t0 = tau[0];
    bool in0 = fabs((double)VT[0]) < theta_max;
    for (int k = 0; k + 1 < nth; ++k) {
        const double f1 = (double)X[(long long)(k + 1) * nx] - x_s, t1 = tau[(long long)(k + 1) * nx];
        const bool in1 = fabs((double)VT[(long long)(k + 1) * nx]) < theta_max;
        if ((f0 == 0.0 || f0 * f1 < 0.0) && in0 && in1) {
            const double t = f0 / (f0 - f1);
            const double v = t0 + t * (t1 - t0);
            if (v > 0.0 && (isnan(best) || v < best)) best = v;
        }
        f0 = f1;
        t0 = t1;
        in0 = in1;
    }
    T[id] = best;
}

template <typename R>
hipError_t pstage_t(const PStageArgs& a, int stage, hipStream_t s) {
    const int blocks = ((a.nx + PTX - 1) / PTX) * ((a.nth + PTT - 1) / PTT);
    const dim3 block(PTX, PTT, NPL);
    switch (stage) {
        case 0: k_pstage<R, 0><<<blocks, block, 0, s>>>(a); break;
        case 1: k_pstage<R, 1><<<blocks, block, 0, s>>>(a); break;
        default: k_pstage<R, 2><<<blocks, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pstage(const PStageArgs& a, int dtype, int stage, hipStream_t s) {
    return dtype == EGB_F64 ? pstage_t<double>(a, stage, s) : pstage_t<float>(a, stage, s);
}

hipError_t launch_pinit(int nx, int nth, long long P, double x0, double dx, double theta_max, double beta, int drt,
                        int dtype, const void* pvel, void* level0, hipStream_t s) {
    const dim3 grid((nx + 63) / 64, (nth + 3) / 4), block(64, 4);
    if (dtype == EGB_F64)
        k_pinit<double><<<grid, block, 0, s>>>(nx, nth, P, x0, dx, theta_max, beta, drt, (const double*)pvel,
                                               (double*)level0);
    else
        k_pinit<float><<<grid, block, 0, s>>>(nx, nth, P, x0, dx, theta_max, beta, drt, (const float*)pvel,
                                              (float*)level0);
    return hipGetLastError();
}

hipError_t launch_ppick(int nx, int nz, int nth, double theta_max, long long P, int dtype, const void* levels,
                        size_t level_bytes, const double* xs, int nsrc, double* T, hipStream_t s) {
    const long long total = (long long)nsrc * nz * nx;
    if (total == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (dtype == EGB_F64)
        k_ppick<double><<<blocks, 256, 0, s>>>(nx, nz, nth, theta_max, P, (const char*)levels, level_bytes, xs, nsrc, T);
    else
        k_ppick<float><<<blocks, 256, 0, s>>>(nx, nz, nth, theta_max, P, (const char*)levels, level_bytes, xs, nsrc, T);
    return hipGetLastError();
}

}  // namespace egb
