// SSP-RK3 stage of the stationary phase-space Liouville march.
//
// For every phase cell (x, z, theta) and state plane f:
//   L_f = -(V_x D_x + V_z D_z + V_theta D_theta) U_f + S_f,
//   S_phi1 = 0, S_psi = 1, S_(C,B) = A (C, B)          (eqs. 16, 19, 21 x dz/dtau)
// with D the WENO5 Hamilton-Jacobi derivative on the upwind side (D- for a
// velocity component >= 0, D+ otherwise), then
//   Uout = ca U0 + cb (Uin + dt L(Uin)),  (ca, cb) = (0,1), (3/4,1/4), (1/3,2/3),
// and cells inside the source ball copy U0.  Ghosts: x, z by linear
// extrapolation u_{-m} = (m+1) u_0 - m u_1, theta periodic.
//
// Precision: planes phi1, C, B in R (float or double); psi is stored and
// combined in double, its WENO differences are formed in double and the
// derivative is evaluated in R.
#include <hip/hip_runtime.h>

#include "egb_device.h"
#include "egb_internal.h"

namespace egb {
namespace {

template <int STAGE>
struct RK;
template <>
struct RK<0> {
    static constexpr double ca = 0.0, cb = 1.0;
};
template <>
struct RK<1> {
    static constexpr double ca = 0.75, cb = 0.25;
};
template <>
struct RK<2> {
    static constexpr double ca = 1.0 / 3.0, cb = 2.0 / 3.0;
};

// value of a line at index i + m with linear-extrapolation ghosts; base points
// at index 0 of the line, st its stride, n its length
template <typename T>
__device__ __forceinline__ T ghost_at(const T* base, long long st, int n, int idx) {
    if (idx < 0) return (T)(1 - idx) * base[0] + (T)idx * base[st];
    if (idx > n - 1) {
        const int e = idx - (n - 1);
        return (T)(e + 1) * base[(long long)(n - 1) * st] - (T)e * base[(long long)(n - 2) * st];
    }
    return base[(long long)idx * st];
}

// Six stencil values u[s..s+5] around the cell along one axis (s = -3 for
// D-, -2 for D+), returned as the five upwind-ordered differences.
template <typename T, typename R>
__device__ __forceinline__ void diffs_from(const T (&u)[6], bool minus, R (&v)[5]) {
    T d[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) d[m] = u[m + 1] - u[m];
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] = (R)(minus ? d[m] : d[4 - m]);
}

template <typename T, typename R>
__device__ __forceinline__ R weno_axis_interior(const T* p, long long st, bool minus) {
    const int s = minus ? -3 : -2;
    T u[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) u[m] = p[(long long)(s + m) * st];
    R v[5];
    diffs_from<T, R>(u, minus, v);
    return weno5<R>(v[0], v[1], v[2], v[3], v[4]);
}

template <typename T, typename R>
__device__ __forceinline__ R weno_axis_ghost(const T* line, long long st, int n, int i, bool minus) {
    const int s = minus ? -3 : -2;
    T u[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) u[m] = ghost_at<T>(line, st, n, i + s + m);
    R v[5];
    diffs_from<T, R>(u, minus, v);
    return weno5<R>(v[0], v[1], v[2], v[3], v[4]);
}

template <typename T, typename R>
__device__ __forceinline__ R weno_theta(const T* plane_cell, long long nxz, int nth, int k, bool minus) {
    // plane_cell points at (theta = 0, x, z) of the cell's column
    const int s = minus ? -3 : -2;
    T u[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        int kk = k + s + m;
        kk += (kk < 0) ? nth : 0;
        kk -= (kk >= nth) ? nth : 0;
        u[m] = plane_cell[(long long)kk * nxz];
    }
    R v[5];
    diffs_from<T, R>(u, minus, v);
    return weno5<R>(v[0], v[1], v[2], v[3], v[4]);
}

// Convective term V.grad of one plane at the cell: c_d = V_d / Delta_d.
template <typename T, typename R>
__device__ __forceinline__ R convect(const T* P, const GridArgs& g, int k, int ix, int iz, R cx, R cz, R ct,
                                     bool xin, bool zin) {
    const long long kb = (long long)k * g.nxz;
    const long long c = kb + (long long)ix * g.nz + iz;
    const R Dx = xin ? weno_axis_interior<T, R>(P + c, g.nz, cx >= (R)0)
                     : weno_axis_ghost<T, R>(P + kb + iz, g.nz, g.nx, ix, cx >= (R)0);
    const R Dz = zin ? weno_axis_interior<T, R>(P + c, 1, cz >= (R)0)
                     : weno_axis_ghost<T, R>(P + kb + (long long)ix * g.nz, 1, g.nz, iz, cz >= (R)0);
    const R Dt = weno_theta<T, R>(P + (long long)ix * g.nz + iz, g.nxz, g.nth, k, ct >= (R)0);
    return cx * Dx + cz * Dz + ct * Dt;
}

template <typename R, int STAGE>
__global__ __launch_bounds__(256) void k_stage(StageArgs a) {
    const GridArgs& g = a.g;
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (iz >= g.nz || ix >= g.nx) return;
    const long long c = (long long)k * g.nxz + (long long)ix * g.nz + iz;
    const long long S = g.stride;
    const R* U0 = reinterpret_cast<const R*>(a.U0);
    const R* Ui = reinterpret_cast<const R*>(a.Uin);
    R* Uo = reinterpret_cast<R*>(a.Uout);
    const double* psi0 = reinterpret_cast<const double*>(U0 + 5 * S);
    const double* psii = reinterpret_cast<const double*>(Ui + 5 * S);
    double* psio = reinterpret_cast<double*>(Uo + 5 * S);

    const double ddx = g.x0 + (ix + 0.5) * g.dx - a.xs, ddz = g.z0 + (iz + 0.5) * g.dz - a.zs;
    if (ddx * ddx + ddz * ddz <= a.r02) {  // source ball: Dirichlet data
#pragma unroll
        for (int f = 0; f < 5; ++f) Uo[f * S + c] = U0[f * S + c];
        psio[c] = psi0[c];
        return;
    }
    const R* V = reinterpret_cast<const R*>(a.vel);
    const R cx = V[EGB_VX * S + c] * (R)(1.0 / g.dx);
    const R cz = V[EGB_VZ * S + c] * (R)(1.0 / g.dz);
    const R ct = V[EGB_VT * S + c] * (R)(1.0 / g.dth);
    const R A11 = V[EGB_A11 * S + c], A12 = V[EGB_A12 * S + c];
    const R A21 = V[EGB_A21 * S + c], A22 = V[EGB_A22 * S + c];
    const bool xin = ix >= 3 && ix <= g.nx - 4;
    const bool zin = iz >= 3 && iz <= g.nz - 4;

    R L[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) L[f] = -convect<R, R>(Ui + f * S, g, k, ix, iz, cx, cz, ct, xin, zin);
    const R uc[4] = {Ui[EGB_RE_C * S + c], Ui[EGB_IM_C * S + c], Ui[EGB_RE_B * S + c], Ui[EGB_IM_B * S + c]};
    L[EGB_RE_C] += A11 * uc[0] + A12 * uc[2];
    L[EGB_RE_B] += A21 * uc[0] + A22 * uc[2];
    L[EGB_IM_C] += A11 * uc[1] + A12 * uc[3];
    L[EGB_IM_B] += A21 * uc[1] + A22 * uc[3];

    // psi: differences in double, derivative in R, accumulation in double
    const R conv_psi = convect<double, R>(psii, g, k, ix, iz, cx, cz, ct, xin, zin);
    const double Lpsi = 1.0 - (double)conv_psi;

    const R dt = (R)a.dt;
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    const R uf[5] = {Ui[c], uc[0], uc[1], uc[2], uc[3]};
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const R y = uf[f] + dt * L[f];
        Uo[f * S + c] = (STAGE == 0) ? y : (R)ca * U0[f * S + c] + (R)cb * y;
    }
    const double yp = psii[c] + a.dt * Lpsi;
    psio[c] = (STAGE == 0) ? yp : ca * psi0[c] + cb * yp;
}

inline dim3 cell_grid(const GridArgs& a) { return dim3((a.nz + 63) / 64, (a.nx + 3) / 4, a.nth); }

template <typename R>
hipError_t launch_stage_t(const StageArgs& a, int stage, hipStream_t s) {
    const dim3 grid = cell_grid(a.g), block(64, 4);
    switch (stage) {
        case 0: k_stage<R, 0><<<grid, block, 0, s>>>(a); break;
        case 1: k_stage<R, 1><<<grid, block, 0, s>>>(a); break;
        default: k_stage<R, 2><<<grid, block, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, int dtype, int stage, hipStream_t s) {
    return dtype == EGB_F64 ? launch_stage_t<double>(a, stage, s) : launch_stage_t<float>(a, stage, s);
}

}  // namespace egb
