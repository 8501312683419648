// Medium table, Liouville velocity + DRT matrix, point-source data and the
// receiver pick.  These run once per medium / source / solve; the march and
// the beam sum are in liouville.hip and beam.hip.
#include <hip/hip_runtime.h>
#include <math.h>

#include "egb_device.h"
#include "egb_internal.h"

namespace egb {
namespace {

// coeff2d[(field * NT + taylor) * nxz + ix * nz + iz]
__device__ __forceinline__ long long cidx(const GridArgs& a, int f, int t, int ix, int iz) {
    return ((long long)(f * NT + t)) * a.nxz + (long long)ix * a.nz + iz;
}

// Thomsen (vp0, eps, delta) + tilt -> (a11, a33, b = a13 + a55, a55, nu):
// a33 = vp0^2, a55 = (fs vp0)^2, a11 = a33 (1 + 2 eps),
// (a13 + a55)^2 = (a33 - a55)(a33 (1 + 2 delta) - a55)  (eq. 5, rho cancels).
__global__ void k_fields(GridArgs a, const double* vp0, const double* eps, const double* dlt, const double* tilt,
                         double fs, double* C) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nxz) return;
    const int ix = (int)(c / a.nz), iz = (int)(c % a.nz);
    const double v = vp0[c];
    const double a33 = v * v, a55 = fs * fs * a33;
    C[cidx(a, 0, 0, ix, iz)] = a33 * (1.0 + 2.0 * eps[c]);
    C[cidx(a, 1, 0, ix, iz)] = a33;
    C[cidx(a, 2, 0, ix, iz)] = sqrt((a33 - a55) * (a33 * (1.0 + 2.0 * dlt[c]) - a55));
    C[cidx(a, 3, 0, ix, iz)] = a55;
    C[cidx(a, 4, 0, ix, iz)] = tilt ? tilt[c] : 0.0;
}

// 4th-order difference weights.  first: central (-2..2), one-sided at the
// first two points (offsets 0..4 and -1..3); second: central, one-sided at
// the first two points (offsets 0..5 and -1..4).  The far end mirrors them
// (first derivative changes sign).
__device__ const double W1C[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
__device__ const double W1E0[5] = {-25.0, 48.0, -36.0, 16.0, -3.0};
__device__ const double W1E1[5] = {-3.0, -10.0, 18.0, -6.0, 1.0};
__device__ const double W2C[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
__device__ const double W2E0[6] = {45.0, -154.0, 214.0, -156.0, 61.0, -10.0};
__device__ const double W2E1[6] = {10.0, -15.0, -4.0, 14.0, -6.0, 1.0};

// derivative (order 1 or 2) of the line f[i * st], i in [0, n)
__device__ double fd_line(const double* f, long long st, int n, int i, double h, int order) {
    double s = 0.0;
    if (i >= 2 && i <= n - 3) {
        const double* w = order == 1 ? W1C : W2C;
        for (int m = 0; m < 5; ++m) s += w[m] * f[(long long)(i - 2 + m) * st];
    } else {
        const bool lo = i < 2;
        const int e = lo ? i : n - 1 - i;  // 0 or 1: distance from the end
        const int len = order == 1 ? 5 : 6;
        const double* w = order == 1 ? (e == 0 ? W1E0 : W1E1) : (e == 0 ? W2E0 : W2E1);
        const int first = -e;  // stencil starts at offset -e from the point, toward the interior
        for (int m = 0; m < len; ++m) {
            const int off = first + m;
            const int j = lo ? i + off : i - off;
            s += w[m] * f[(long long)j * st];
        }
        if (!lo && order == 1) s = -s;
    }
    return order == 1 ? s / (12.0 * h) : s / (12.0 * h * h);
}

// slots f_x, f_z, f_xx, f_zz from the values
__global__ void k_derivs(GridArgs a, double* C) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nxz * NF) return;
    const int f = (int)(c / a.nxz);
    const long long r = c % a.nxz;
    const int ix = (int)(r / a.nz), iz = (int)(r % a.nz);
    const double* v = C + cidx(a, f, 0, 0, 0);
    C[cidx(a, f, 1, ix, iz)] = fd_line(v + iz, a.nz, a.nx, ix, a.dx, 1);
    C[cidx(a, f, 2, ix, iz)] = fd_line(v + (long long)ix * a.nz, 1, a.nz, iz, a.dz, 1);
    C[cidx(a, f, 3, ix, iz)] = fd_line(v + iz, a.nz, a.nx, ix, a.dx, 2);
    C[cidx(a, f, 5, ix, iz)] = fd_line(v + (long long)ix * a.nz, 1, a.nz, iz, a.dz, 2);
}

// f_xz = d/dx of the f_z slot
__global__ void k_mixed(GridArgs a, double* C) {
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nxz * NF) return;
    const int f = (int)(c / a.nxz);
    const long long r = c % a.nxz;
    const int ix = (int)(r / a.nz), iz = (int)(r % a.nz);
    const double* fz = C + cidx(a, f, 2, 0, 0);
    C[cidx(a, f, 4, ix, iz)] = fd_line(fz + iz, a.nz, a.nx, ix, a.dx, 1);
}

__device__ __forceinline__ void load_point(const GridArgs& a, const double* C, int ix, int iz, MediumPoint& M) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t) M.m[f][t] = C[cidx(a, f, t, ix, iz)];
}

// positive doubles order like their bit patterns
__device__ __forceinline__ void atomic_max_pos(unsigned long long* p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

template <typename R>
__global__ __launch_bounds__(256) void k_velocity(GridArgs a, const double* C, R* vel, unsigned long long* rate_bits) {
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    double rate = 0.0;
    if (iz < a.nz && ix < a.nx) {
        MediumPoint M;
        load_point(a, C, ix, iz, M);
        const double th = k * a.dth;
        const VJet J = qp_velocity(M, th);
        const VelA r = velocity_and_drt(J, th);
        const long long c = (long long)k * a.nxz + (long long)ix * a.nz + iz;
        for (int q = 0; q < 3; ++q) vel[q * a.stride + c] = (R)r.V[q];
        for (int q = 0; q < 4; ++q) vel[(3 + q) * a.stride + c] = (R)r.A[q];
        rate = fabs(r.V[0]) / a.dx + fabs(r.V[1]) / a.dz + fabs(r.V[2]) / a.dth;
        if (!isfinite(rate)) rate = __longlong_as_double(0x7ff0000000000000LL);  // +inf flags a bad medium
    }
    // wave-level max, one atomic per wave
    for (int o = 32; o > 0; o >>= 1) rate = fmax(rate, __shfl_xor(rate, o, 64));
    if ((threadIdx.x & 63) == 0) atomic_max_pos(rate_bits, rate);
}

// Coefficients of the paraxial depth march at theta_k = -theta_max +
// (k + 1/2) dtheta, dtheta = 2 theta_max / nth: the Liouville velocity and
// DRT matrix divided by V_z (eqs. 13-15), planes u, w, S_tau, A11..A22 / V_z,
// layout [nz][7][P] with index k nx + x.  rate: max |u|/dx + |w|/dtheta, +inf
// where V_z <= 0 (beyond the paraxial range) or not finite.
template <typename R>
__global__ __launch_bounds__(256) void k_pvelocity(GridArgs a, double theta_max, int drt, const double* C, R* pvel,
                                                   long long P, unsigned long long* rate_bits) {
    const int ix = blockIdx.x * 64 + threadIdx.x, k = blockIdx.y * 4 + threadIdx.y, n = blockIdx.z;
    double rate = 0.0;
    if (ix < a.nx && k < a.nth) {
        MediumPoint M;
        load_point(a, C, ix, n, M);
        const double dth = 2.0 * theta_max / a.nth;
        const double th = -theta_max + (k + 0.5) * dth;
        const VJet J = qp_velocity(M, th);
        const VelA r = velocity_and_drt(J, th);
        const long long c = (long long)n * 7 * P + (long long)k * a.nx + ix;
        const double vz = r.V[1];
        const double u = r.V[0] / vz, w = r.V[2] / vz;
        pvel[c] = (R)u;
        pvel[P + c] = (R)w;
        pvel[2 * P + c] = (R)(1.0 / vz);
        if (drt == EGB_DRT_PAPER23) {
            // eqs. 21-23 in the lateral frame, per unit depth: u1 = cos + sin u,
            // H_pp = v u1^3, H_xp = u1^2 (v_x / v) u,
            // H_xx = (u1 (v v_xx - 3 v_x^2) + u1^3 v_x^2) / v^3 (v_x, v_xx at fixed theta);
            // C' = H_xp C + H_pp B, B' = -H_xx C - H_xp B
            double sn, cs;
            sincos_d(th, &sn, &cs);
            const double v = J.v, vx = J.g[0], vxx = J.h[0][0];
            const double u1 = cs + sn * u, u13 = u1 * u1 * u1;
            const double hxp = u1 * u1 * (vx / v) * u;
            const double hxx = (u1 * (v * vxx - 3.0 * vx * vx) + u13 * vx * vx) / (v * v * v);
            pvel[3 * P + c] = (R)hxp;
            pvel[4 * P + c] = (R)(v * u13);
            pvel[5 * P + c] = (R)(-hxx);
            pvel[6 * P + c] = (R)(-hxp);
        } else {  // the ray-normal pair of the phase-space system divided by dz/dtau
            for (int q = 0; q < 4; ++q) pvel[(3 + q) * P + c] = (R)(r.A[q] / vz);
        }
        rate = fabs(u) / a.dx + fabs(w) / dth;
        if (!(vz > 0.0) || !isfinite(rate)) rate = __longlong_as_double(0x7ff0000000000000LL);
    }
    for (int o = 32; o > 0; o >>= 1) rate = fmax(rate, __shfl_xor(rate, o, 64));
    if ((threadIdx.x & 63) == 0) atomic_max_pos(rate_bits, rate);
}

// Bilinear interpolation of the table values at (xs, zs) (medium frozen at the source).
__device__ void source_medium(const GridArgs& a, const double* C, double xs, double zs, MediumPoint& M) {
    double fx = (xs - a.x0) / a.dx - 0.5, fz = (zs - a.z0) / a.dz - 0.5;
    int ix = (int)floor(fx), iz = (int)floor(fz);
    ix = min(max(ix, 0), a.nx - 2);
    iz = min(max(iz, 0), a.nz - 2);
    const double tx = fmin(fmax(fx - ix, 0.0), 1.0), tz = fmin(fmax(fz - iz, 0.0), 1.0);
    for (int f = 0; f < NF; ++f) {
        M.m[f][0] = (1 - tx) * (1 - tz) * C[cidx(a, f, 0, ix, iz)] + tx * (1 - tz) * C[cidx(a, f, 0, ix + 1, iz)] +
                    (1 - tx) * tz * C[cidx(a, f, 0, ix, iz + 1)] + tx * tz * C[cidx(a, f, 0, ix + 1, iz + 1)];
        for (int t = 1; t < NT; ++t) M.m[f][t] = 0.0;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_init_state(GridArgs a, const double* C, egb_source src, char* state) {
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (iz >= a.nz || ix >= a.nx) return;
    MediumPoint M;
    source_medium(a, C, src.xs, src.zs, M);
    const double th = k * a.dth;
    const VJet J = qp_velocity(M, th);
    const VelA r = velocity_and_drt(J, th);
    const double v = J.v;
    const double sp = sqrt(r.V[0] * r.V[0] + r.V[1] * r.V[1]);
    const double ex = r.V[1] / sp, ez = -r.V[0] / sp;  // unit normal to the ray
    double sn, cs;
    sincos_d(th, &sn, &cs);
    const double W = M.m[1][0] / (v * v);  // a33 / v^2
    const double s = cbrt((sqrt(v) / W) * (sqrt(v) / W));
    const double ddx = a.x0 + (ix + 0.5) * a.dx - src.xs, ddz = a.z0 + (iz + 0.5) * a.dz - src.zs;
    const double psi = (sn * ddx + cs * ddz) / v;
    const long long c = (long long)k * a.nxz + (long long)ix * a.nz + iz;
    R* P = reinterpret_cast<R*>(state);
    double* Ps = reinterpret_cast<double*>(P + EGB_PSI * a.stride);
    P[EGB_PHI1 * a.stride + c] = (R)(ddx * ex + ddz * ez);
    P[EGB_RE_C * a.stride + c] = (R)s;
    P[EGB_IM_C * a.stride + c] = (R)(s * src.beta * r.A[1] * psi);
    P[EGB_RE_B * a.stride + c] = (R)0;
    P[EGB_IM_B * a.stride + c] = (R)(src.beta * s);
    P[EGB_PHASE * a.stride + c] = (R)atan(src.beta * r.A[1] * psi);  // arg C, s > 0
    Ps[c] = psi;
}

// Boundary data: thread i < nth*6*nz is x ghost (theta, slot, z), the rest z
// ghosts (theta, x, slot); slot 0..2 = position -3..-1, 3..5 = n..n+2 of the
// line; the value continues the line through the two end cells.
template <typename R>
__global__ __launch_bounds__(256) void k_boundary_data(GridArgs a, const char* state, char* bd) {
    const long long nxg = (long long)a.nth * 6 * a.nz, n = (long long)a.nth * 6 * (a.nx + a.nz);
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int gi, len;
    long long c0, step;  // cell at line position 0 and the stride along the line
    if (i < nxg) {
        const int k = (int)(i / (6 * a.nz)), z = (int)(i % a.nz);
        gi = (int)((i / a.nz) % 6);
        c0 = (long long)k * a.nxz + z;
        step = a.nz;
        len = a.nx;
    } else {
        const long long j = i - nxg;
        const int k = (int)(j / (6 * a.nx)), x = (int)((j / 6) % a.nx);
        gi = (int)(j % 6);
        c0 = (long long)k * a.nxz + (long long)x * a.nz;
        step = 1;
        len = a.nz;
    }
    // ghost at distance m beyond the end cell e, e1 the cell next to e
    const int m = gi < 3 ? 3 - gi : gi - 2;
    const long long e = gi < 3 ? c0 : c0 + (long long)(len - 1) * step;
    const long long e1 = gi < 3 ? c0 + step : c0 + (long long)(len - 2) * step;
    const R* P = reinterpret_cast<const R*>(state);
    const double* Ps = reinterpret_cast<const double*>(P + EGB_PSI * a.stride);
    R* B = reinterpret_cast<R*>(bd);
    double* Bs = reinterpret_cast<double*>(B + EGB_PSI * a.bstride);
    for (int f = 0; f < EGB_PSI; ++f)
        B[f * a.bstride + i] = (R)((m + 1) * (double)P[f * a.stride + e] - m * (double)P[f * a.stride + e1]);
    Bs[i] = (m + 1) * Ps[e] - m * Ps[e1];
}

// One thread per receiver; see egb_pick_receivers.
template <typename R>
__global__ void k_pick(GridArgs a, const char* state, const double* rx, int nr, double* t_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const double fx = (rx[2 * r] - a.x0) / a.dx - 0.5, fz = (rx[2 * r + 1] - a.z0) / a.dz - 0.5;
    int ix = (int)floor(fx), iz = (int)floor(fz);
    ix = min(max(ix, 0), a.nx - 2);
    iz = min(max(iz, 0), a.nz - 2);
    const double tx = fmin(fmax(fx - ix, 0.0), 1.0), tz = fmin(fmax(fz - iz, 0.0), 1.0);
    const double w00 = (1 - tx) * (1 - tz), w10 = tx * (1 - tz), w01 = (1 - tx) * tz, w11 = tx * tz;
    const R* phi = reinterpret_cast<const R*>(state);
    const double* psi = reinterpret_cast<const double*>(phi + EGB_PSI * a.stride);
    const long long o = (long long)ix * a.nz + iz;
    auto interp_phi = [&](int k) {
        const R* p = phi + (long long)k * a.nxz + o;
        return w00 * (double)p[0] + w10 * (double)p[a.nz] + w01 * (double)p[1] + w11 * (double)p[a.nz + 1];
    };
    auto interp_psi = [&](int k) {
        const double* p = psi + (long long)k * a.nxz + o;
        return w00 * p[0] + w10 * p[a.nz] + w01 * p[1] + w11 * p[a.nz + 1];
    };
    double best = __longlong_as_double(0x7ff8000000000000LL);  // NaN: no arrival
    double f0 = interp_phi(0), s0 = interp_psi(0);
    const double fstart = f0, sstart = s0;
    for (int k = 0; k < a.nth; ++k) {
        const bool last = (k == a.nth - 1);
        const double f1 = last ? fstart : interp_phi(k + 1);
        const double s1 = last ? sstart : interp_psi(k + 1);
        if (f0 == 0.0 || f0 * f1 < 0.0) {
            const double t = f0 / (f0 - f1);
            const double val = s0 + t * (s1 - s0);
            if (val > 0.0 && (isnan(best) || val < best)) best = val;
        }
        f0 = f1;
        s0 = s1;
    }
    t_out[r] = best;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline dim3 cell_grid(const GridArgs& a) { return dim3((a.nz + 63) / 64, (a.nx + 3) / 4, a.nth); }

}  // namespace

hipError_t launch_medium_table(const GridArgs& a, const egb_medium& m, double* C, hipStream_t s) {
    const int bs = 256;
    k_fields<<<(unsigned)((a.nxz + bs - 1) / bs), bs, 0, s>>>(a, m.vp0, m.eps, m.delta, m.tilt, m.vs_ratio, C);
    k_derivs<<<(unsigned)((a.nxz * NF + bs - 1) / bs), bs, 0, s>>>(a, C);
    k_mixed<<<(unsigned)((a.nxz * NF + bs - 1) / bs), bs, 0, s>>>(a, C);
    return hipGetLastError();
}

hipError_t launch_velocity(const GridArgs& a, int dtype, const double* C, void* vel, unsigned long long* rate_bits,
                           hipStream_t s) {
    if (dtype == EGB_F64)
        k_velocity<double><<<cell_grid(a), dim3(64, 4), 0, s>>>(a, C, (double*)vel, rate_bits);
    else
        k_velocity<float><<<cell_grid(a), dim3(64, 4), 0, s>>>(a, C, (float*)vel, rate_bits);
    return hipGetLastError();
}

hipError_t launch_pvelocity(const GridArgs& a, int dtype, double theta_max, int drt, const double* C, void* pvel,
                            long long P, unsigned long long* rate_bits, hipStream_t s) {
    const dim3 grid((a.nx + 63) / 64, (a.nth + 3) / 4, a.nz), block(64, 4);
    if (dtype == EGB_F64)
        k_pvelocity<double><<<grid, block, 0, s>>>(a, theta_max, drt, C, (double*)pvel, P, rate_bits);
    else
        k_pvelocity<float><<<grid, block, 0, s>>>(a, theta_max, drt, C, (float*)pvel, P, rate_bits);
    return hipGetLastError();
}

hipError_t launch_init_state(const GridArgs& a, int dtype, const double* C, const egb_source& src, void* state,
                             hipStream_t s) {
    if (dtype == EGB_F64)
        k_init_state<double><<<cell_grid(a), dim3(64, 4), 0, s>>>(a, C, src, (char*)state);
    else
        k_init_state<float><<<cell_grid(a), dim3(64, 4), 0, s>>>(a, C, src, (char*)state);
    return hipGetLastError();
}

hipError_t launch_boundary_data(const GridArgs& a, int dtype, const void* state, void* bdata, hipStream_t s) {
    const long long n = (long long)a.nth * 6 * (a.nx + a.nz);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (dtype == EGB_F64)
        k_boundary_data<double><<<blocks, 256, 0, s>>>(a, (const char*)state, (char*)bdata);
    else
        k_boundary_data<float><<<blocks, 256, 0, s>>>(a, (const char*)state, (char*)bdata);
    return hipGetLastError();
}

hipError_t launch_pick(const GridArgs& a, int dtype, const void* state, const double* rx, int nr, double* t_out,
                       hipStream_t s) {
    if (nr <= 0) return hipSuccess;
    const int bs = 64;
    if (dtype == EGB_F64)
        k_pick<double><<<(nr + bs - 1) / bs, bs, 0, s>>>(a, (const char*)state, rx, nr, t_out);
    else
        k_pick<float><<<(nr + bs - 1) / bs, bs, 0, s>>>(a, (const char*)state, rx, nr, t_out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace egb
