// Paraxial depth march (eqs. 13-15 with the Liouville transport of eqs.
// 16-24 divided by dz/dtau): on (x, theta) slices with theta in
// (-theta_max, theta_max) the state
//   X (the surface position of the ray), vartheta (its take-off angle),
//   tau (traveltime), C, B (complex dynamic ray tracing pair)
// obeys U_z + u U_x + w U_theta = S,  u = V_x / V_z, w = V_theta / V_z,
// S_tau = 1 / V_z, S_(C,B) = (A / V_z)(C, B), the other sources zero.  Each
// depth interval dz is nsub SSP-RK3 steps of dz / nsub in z, the
// coefficients linear in z between the two levels (stage depths s, s + h,
// s + h / 2 of the interval, h = 1 / nsub); x and theta ghosts continue the
// line of the two cells next to them.  Every level is kept; first arrivals
// for a surface source at x_s follow from the level set X = x_s (eq. 35).
//
// Level layout: planes X, vartheta, Re C, Im C, Re B, Im B in R, then tau in
// double, each [theta][x] (x fastest) padded to a multiple of 64 elements.
//
// Work decomposition: a block owns a tile of 64 x by 4 theta cells of one
// slice; the slice with a 3-cell halo (ghosts filled while loading) goes to
// LDS once, then every cell reads its x and theta stencils there at per-lane
// mirrored addresses (V D(U) = |V| W(values in upwind order), as in the
// phase-space stage kernel).  A slice is small (nx nth cells), so the march
// is a long chain of short launches, captured once into a hipGraph.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "egb_device.h"
#include "egb_internal.h"
#include "stage_common.h"

namespace egb {
namespace {

constexpr int PTX = 64, PTT = 4;         // tile: x cells, theta rows
constexpr int PRX = PTX + 6;             // LDS row (3-cell halo each side)
constexpr int PROWS = PTT + 6;
constexpr int PCELLS = PROWS * PRX;      // LDS cells per plane
constexpr int NPR = 6;                   // R planes: X, vartheta, ReC, ImC, ReB, ImB
enum { Q_X = 0, Q_VT = 1, Q_RC = 2, Q_IC = 3, Q_RB = 4, Q_IB = 5 };
// velocity planes: u, w, S_tau, A11/Vz, A12/Vz, A21/Vz, A22/Vz

template <typename R>
struct PSmem {
    using W = typename LdsWord<R>::T;
    static constexpr int PLANE = (PCELLS + 63) / 64 * 64;
    static constexpr int PB = PLANE * (int)sizeof(W);
    W w[(NPR + LdsWord<R>::PSI_WORDS) * PLANE];
};

// Value of a line through (x, k): inside the slice the stored value, beyond
// an x end or a theta end the line of the two cells next to it
// (u_{-m} = (m+1) u_0 - m u_1); cells beyond both are never read.
template <typename T>
__device__ __forceinline__ T pline_val(const T* u, int nx, int nth, int x, int k) {
    if (x >= 0 && x < nx && k >= 0 && k < nth) return u[(long long)k * nx + x];
    if (k >= 0 && k < nth) {
        const T* r = u + (long long)k * nx;
        if (x < 0) return (T)(1 - x) * r[0] + (T)x * r[1];
        const int e = x - (nx - 1);
        return (T)(e + 1) * r[nx - 1] - (T)e * r[nx - 2];
    }
    if (x >= 0 && x < nx) {
        if (k < 0) return (T)(1 - k) * u[x] + (T)k * u[nx + x];
        const int e = k - (nth - 1);
        return (T)(e + 1) * u[(long long)(nth - 1) * nx + x] - (T)e * u[(long long)(nth - 2) * nx + x];
    }
    return (T)0;
}

template <typename R, int STAGE>
__global__ __launch_bounds__(PTX * PTT) void k_pstage(PStageArgs a) {
    using S = PSmem<R>;
    using Wd = typename S::W;
    constexpr int WS = (int)sizeof(Wd);
    __shared__ S sm;
    const int ntx = (a.nx + PTX - 1) / PTX;
    const int tx0 = (blockIdx.x % ntx) * PTX, tk0 = (blockIdx.x / ntx) * PTT;
    const int tid = threadIdx.y * PTX + threadIdx.x;
    const R* Ui = static_cast<const R*>(a.Uin);
    const double* Tin = reinterpret_cast<const double*>(Ui + NPR * a.P);

    // slice tile + halo into LDS (ghosts by extrapolation)
    for (int i = tid; i < PCELLS; i += PTX * PTT) {
        const int x = tx0 + i % PRX - 3, k = tk0 + i / PRX - 3;
#pragma unroll
        for (int f = 0; f < NPR; ++f)
            sm.w[f * S::PLANE + i] = __builtin_bit_cast(Wd, pline_val<R>(Ui + f * a.P, a.nx, a.nth, x, k));
        const unsigned long long b = __builtin_bit_cast(unsigned long long, pline_val<double>(Tin, a.nx, a.nth, x, k));
        if constexpr (sizeof(R) == 4) {
            sm.w[NPR * S::PLANE + i] = (unsigned)b;
            sm.w[(NPR + 1) * S::PLANE + i] = (unsigned)(b >> 32);
        } else {
            sm.w[NPR * S::PLANE + i] = b;
        }
    }
    __syncthreads();

    const int x = tx0 + (int)threadIdx.x, k = tk0 + (int)threadIdx.y;
    if (x >= a.nx || k >= a.nth) return;
    const long long c = (long long)k * a.nx + x;
    // coefficients at this stage's depth
    const R* p0 = static_cast<const R*>(a.pv0);
    const R* p1 = static_cast<const R*>(a.pv1);
    const R s1 = (R)a.s, s0 = (R)(1.0 - a.s);
    R cv[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) cv[q] = s0 * p0[q * a.P + c] + s1 * p1[q * a.P + c];
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    const double cdl = cb * a.dl;
    const R gx = fabs(cv[0]) * (R)(cdl / a.dx), gt = fabs(cv[1]) * (R)(cdl / a.dth), cdr = (R)cdl;
    const bool mx = cv[0] >= (R)0, mt = cv[1] >= (R)0;

    const int me = ((int)threadIdx.y + 3) * PRX + (int)threadIdx.x + 3;
    const int meB = me * WS;
    R own[NPR];
#pragma unroll
    for (int f = 0; f < NPR; ++f) own[f] = lds_r<R>(sm, meB, f);
    const double ownp = lds_psi<NPR>(sm, meB);
    R acc[NPR];
#pragma unroll
    for (int f = 0; f < NPR; ++f) acc[f] = (R)cb * own[f];
    double accp = cb * ownp + cdl * (double)cv[2];
    R convp = (R)0;
    auto axis = [&](int step, R g) {
        const int a0 = meB - 3 * step, a1 = meB - 2 * step, a2 = meB - step, a4 = meB + step, a5 = meB + 2 * step;
#pragma unroll
        for (int f = 0; f < NPR; ++f)
            acc[f] -= g * weno_up<R>(lds_r<R>(sm, a0, f), lds_r<R>(sm, a1, f), lds_r<R>(sm, a2, f), own[f],
                                     lds_r<R>(sm, a4, f), lds_r<R>(sm, a5, f));
        convp += g * weno_up<R>(lds_psi<NPR>(sm, a0), lds_psi<NPR>(sm, a1), lds_psi<NPR>(sm, a2), ownp,
                                lds_psi<NPR>(sm, a4), lds_psi<NPR>(sm, a5));
    };
    axis(mx ? WS : -WS, gx);
    axis(mt ? PRX * WS : -PRX * WS, gt);
    accp -= (double)convp;
    const R A11 = cdr * cv[3], A12 = cdr * cv[4], A21 = cdr * cv[5], A22 = cdr * cv[6];
    acc[Q_RC] += A11 * own[Q_RC] + A12 * own[Q_RB];
    acc[Q_RB] += A21 * own[Q_RC] + A22 * own[Q_RB];
    acc[Q_IC] += A11 * own[Q_IC] + A12 * own[Q_IB];
    acc[Q_IB] += A21 * own[Q_IC] + A22 * own[Q_IB];
    R* Uo = static_cast<R*>(a.Uout);
    double* To = reinterpret_cast<double*>(Uo + NPR * a.P);
    if constexpr (STAGE != 0) {
        const R* U0 = static_cast<const R*>(a.U0);
        const double* T0 = reinterpret_cast<const double*>(U0 + NPR * a.P);
#pragma unroll
        for (int f = 0; f < NPR; ++f) acc[f] += (R)ca * U0[f * a.P + c];
        accp += ca * T0[c];
    }
#pragma unroll
    for (int f = 0; f < NPR; ++f) Uo[f * a.P + c] = acc[f];
    To[c] = accp;
}

// Surface data on level 0: X = x, vartheta = theta, tau = 0,
// C = cos(theta) + sin(theta) u, B = i beta C.
template <typename R>
__global__ __launch_bounds__(256) void k_pinit(int nx, int nth, long long P, double x0, double dx, double theta_max,
                                               double beta, const R* pv, R* U) {
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
    U[Q_IB * P + c] = (R)(beta * c0);
    reinterpret_cast<double*>(U + NPR * P)[c] = 0.0;
}

// First arrival at (x_i, level n) for surface source s: roots in theta of
// X - x_s between adjacent nodes, tau interpolated linearly, the smallest
// tau > 0 (NaN when there is none).  T[s][n][i].
template <typename R>
__global__ __launch_bounds__(256) void k_ppick(int nx, int nz, int nth, long long P, const char* levels,
                                               size_t level_bytes, const double* xs, int nsrc, double* T) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)nsrc * nz * nx;
    if (id >= total) return;
    const int i = (int)(id % nx), n = (int)((id / nx) % nz), s = (int)(id / ((long long)nx * nz));
    const R* X = reinterpret_cast<const R*>(levels + (size_t)n * level_bytes) + i;
    const double* tau = reinterpret_cast<const double*>(reinterpret_cast<const R*>(levels + (size_t)n * level_bytes) +
                                                        NPR * P) + i;
    const double x_s = xs[s];
    double best = __longlong_as_double(0x7ff8000000000000LL);
    double f0 = (double)X[0] - x_s, t0 = tau[0];
    for (int k = 0; k + 1 < nth; ++k) {
        const double f1 = (double)X[(long long)(k + 1) * nx] - x_s, t1 = tau[(long long)(k + 1) * nx];
        if (f0 == 0.0 || f0 * f1 < 0.0) {
            const double t = f0 / (f0 - f1);
            const double v = t0 + t * (t1 - t0);
            if (v > 0.0 && (isnan(best) || v < best)) best = v;
        }
        f0 = f1;
        t0 = t1;
    }
    T[id] = best;
}

template <typename R>
hipError_t pstage_t(const PStageArgs& a, int stage, hipStream_t s) {
    const int blocks = ((a.nx + PTX - 1) / PTX) * ((a.nth + PTT - 1) / PTT);
    const dim3 block(PTX, PTT);
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

hipError_t launch_pinit(int nx, int nth, long long P, double x0, double dx, double theta_max, double beta, int dtype,
                        const void* pvel, void* level0, hipStream_t s) {
    const dim3 grid((nx + 63) / 64, (nth + 3) / 4), block(64, 4);
    if (dtype == EGB_F64)
        k_pinit<double><<<grid, block, 0, s>>>(nx, nth, P, x0, dx, theta_max, beta, (const double*)pvel,
                                               (double*)level0);
    else
        k_pinit<float><<<grid, block, 0, s>>>(nx, nth, P, x0, dx, theta_max, beta, (const float*)pvel, (float*)level0);
    return hipGetLastError();
}

hipError_t launch_ppick(int nx, int nz, int nth, long long P, int dtype, const void* levels, size_t level_bytes,
                        const double* xs, int nsrc, double* T, hipStream_t s) {
    const long long total = (long long)nsrc * nz * nx;
    if (total == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (dtype == EGB_F64)
        k_ppick<double><<<blocks, 256, 0, s>>>(nx, nz, nth, P, (const char*)levels, level_bytes, xs, nsrc, T);
    else
        k_ppick<float><<<blocks, 256, 0, s>>>(nx, nz, nth, P, (const char*)levels, level_bytes, xs, nsrc, T);
    return hipGetLastError();
}

}  // namespace egb
