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
// kernel).  The march is a long chain of short launches, captured once into
// a hipGraph.
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

// LDS cell i of a tile (x0, k0): inside the slice the marched value u[i0]
// ((w0, w1) = (1, 0)); beyond an x end or a theta end (a ghost) the surface
// data b extended linearly from the two cells next to that end,
// w0 b[i0] + w1 b[i1] with (w0, w1) = (m + 1, -m); cells beyond both are
// never read (weights 0).
__device__ __forceinline__ void pline_src(int nx, int nth, int x, int k, int& i0, int& i1, int& w0, int& w1) {
    const bool xin = x >= 0 && x < nx, kin = k >= 0 && k < nth;
    if (xin && kin) {
        i0 = i1 = k * nx + x;
        w0 = 1;
        w1 = 0;
    } else if (kin) {
        const bool lo = x < 0;
        const int m = lo ? -x : x - (nx - 1);
        i0 = k * nx + (lo ? 0 : nx - 1);
        i1 = k * nx + (lo ? 1 : nx - 2);
        w0 = m + 1;
        w1 = -m;
    } else if (xin) {
        const bool lo = k < 0;
        const int m = lo ? -k : k - (nth - 1);
        i0 = (lo ? 0 : nth - 1) * nx + x;
        i1 = (lo ? 1 : nth - 2) * nx + x;
        w0 = m + 1;
        w1 = -m;
    } else {
        i0 = i1 = 0;
        w0 = w1 = 0;
    }
}

// One RK stage on a 64 x 2 (x, theta) tile: thread (x, row, plane), so
// every wave holds one plane of one theta row and all branches on the plane
// are wave-uniform.  The tile of every plane with its halo is loaded to LDS
// by the waves of that plane (all loads of a thread issued together; the
// second point of a ghost only in tiles that touch an edge); the x and theta
// stencils are then read at per-lane mirrored addresses.  The cell's
// coefficients and stage-start value are fetched before the barrier.
template <typename R, int STAGE>
__global__ __launch_bounds__(NT) void k_pstage(PStageArgs a) {
    using S = PSmem<R>;
    using Wd = typename S::W;
    constexpr int WS = (int)sizeof(Wd);
    constexpr int NLD = (PCELLS + PTX * PTT - 1) / (PTX * PTT);  // LDS cells per thread
    __shared__ S sm;
    const int ntx = (a.nx + PTX - 1) / PTX;
    const int tx0 = (blockIdx.x % ntx) * PTX, tk0 = (blockIdx.x / ntx) * PTT;
    const int p = threadIdx.z;  // plane (wave-uniform)
    const int pt = threadIdx.y * PTX + threadIdx.x;
    const bool edge = tx0 < 3 || tx0 + PTX + 3 > a.nx || tk0 < 3 || tk0 + PTT + 3 > a.nth;  // block-uniform

    // own cell (clamped for threads past the slice) and its prefetched inputs
    const int x = tx0 + (int)threadIdx.x, k = tk0 + (int)threadIdx.y;
    const bool valid = x < a.nx && k < a.nth;
    const long long c = (long long)min(k, a.nth - 1) * a.nx + min(x, a.nx - 1);
    const R* p0 = static_cast<const R*>(a.pv0);
    const R* p1 = static_cast<const R*>(a.pv1);
    const bool isC = p == Q_RC || p == Q_IC;
    const int qa = p == Q_TAU ? 2 : (p == Q_PH ? 4 : (isC ? 3 : 5));  // this plane's source coefficients
    const R u0 = p0[c], u1 = p1[c], w0 = p0[a.P + c], w1 = p1[a.P + c];
    const R a0 = p0[qa * a.P + c], a1 = p1[qa * a.P + c];
    const R b0 = p0[(qa + 1) * a.P + c], b1 = p1[(qa + 1) * a.P + c];
    const R* Ui = static_cast<const R*>(a.Uin);
    const R* Ub = static_cast<const R*>(a.Ub);  // surface data (level 0): the ghosts
    R r0 = (R)0;
    double t0 = 0.0;
    if constexpr (STAGE != 0) {
        const R* U0 = static_cast<const R*>(a.U0);
        if (p == Q_TAU) t0 = reinterpret_cast<const double*>(U0 + NPR * a.P)[c];
        else r0 = U0[p * a.P + c];
    }

    // this plane's tile + halo into LDS
    auto fill = [&](auto tag) {
        using T = decltype(tag);
        const T* u = p == Q_TAU ? reinterpret_cast<const T*>(Ui + NPR * a.P) : reinterpret_cast<const T*>(Ui + p * a.P);
        const T* ub = p == Q_TAU ? reinterpret_cast<const T*>(Ub + NPR * a.P) : reinterpret_cast<const T*>(Ub + p * a.P);
        T v0[NLD], b0[NLD], b1[NLD];
        int wa[NLD], wb[NLD];
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int i = min(pt + r * PTX * PTT, PCELLS - 1);
            int i0, i1;
            pline_src(a.nx, a.nth, tx0 + i % PRX - 3, tk0 + i / PRX - 3, i0, i1, wa[r], wb[r]);
            v0[r] = u[i0];
            b0[r] = edge ? ub[i0] : (T)0;
            b1[r] = edge ? ub[i1] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < NLD; ++r) {
            const int i = pt + r * PTX * PTT;
            if (i < PCELLS) {
                const bool ghost = wa[r] != 1 || wb[r] != 0;
                const T v = edge && ghost ? (T)wa[r] * b0[r] + (T)wb[r] * b1[r] : v0[r];
                if constexpr (sizeof(T) == sizeof(Wd)) {
                    sm.w[(p == Q_TAU ? NPR : p) * S::PLANE + i] = __builtin_bit_cast(Wd, v);
                } else {  // tau of an FP32 slice: two 32-bit planes
                    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
                    sm.w[NPR * S::PLANE + i] = (Wd)(unsigned)b;
                    sm.w[(NPR + 1) * S::PLANE + i] = (Wd)(unsigned)(b >> 32);
                }
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
    const int meB = (((int)threadIdx.y + 3) * PRX + (int)threadIdx.x + 3) * WS;
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
        reinterpret_cast<double*>(Uo + NPR * a.P)[c] = acc;
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
    Uo[p * a.P + c] = acc;
}

// Surface data on level 0: X = x, vartheta = theta, tau = 0,
// C = cos(theta) + sin(theta) u, B = i beta C, Phi = 0.
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
