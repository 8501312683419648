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
// transposed stencil is applied in two passes: every cell writes its seven
// Jacobian coefficients per plane and axis scaled by -cb dt c_d mu ("packets",
// slot j for the target at offset j), then every cell gathers the packets aimed
// at it; packets aimed at extrapolated ghosts go to the two cells the ghost is
// extrapolated from (weights m + 1 and -m), theta wraps.
#include <hip/hip_runtime.h>
#include <math.h>

#include "egb_device.h"
#include "egb_internal.h"

namespace egb {
namespace {

constexpr int NSLOT = 7;
constexpr int NQ = 2 * 3 * NSLOT;  // packets per cell: plane x axis x slot

// Packet layout: per (theta, x, 64-cell z strip) the NQ packets of the strip
// are contiguous (NQ rows of 64), so a wave reads or writes whole 256-byte
// rows that sit next to each other.
__device__ __forceinline__ long long pk_idx(const GridArgs& g, int q, int k, int x, int z) {
    const int ntz = (g.nz + 63) >> 6;
    return ((((long long)k * g.nx + x) * ntz + (z >> 6)) * NQ + q) * 64 + (z & 63);
}

// value of a line at index idx with linear-extrapolation ghosts
template <typename T>
__device__ __forceinline__ T line_at(const T* base, long long st, int n, int idx) {
    if (idx < 0) return (T)(1 - idx) * base[0] + (T)idx * base[st];
    if (idx > n - 1) {
        const int e = idx - (n - 1);
        return (T)(e + 1) * base[(long long)(n - 1) * st] - (T)e * base[(long long)(n - 2) * st];
    }
    return base[(long long)idx * st];
}

// the seven stencil values along axis (0 x, 1 z, 2 theta) at offsets -3..3
template <typename T>
__device__ __forceinline__ void stencil7(const T* P, const GridArgs& g, int k, int ix, int iz, int axis, T (&u)[7]) {
    const long long kb = (long long)k * g.nxz;
    if (axis == 0) {
        for (int m = 0; m < 7; ++m) u[m] = line_at(P + kb + iz, g.nz, g.nx, ix + m - 3);
    } else if (axis == 1) {
        for (int m = 0; m < 7; ++m) u[m] = line_at(P + kb + (long long)ix * g.nz, 1, g.nz, iz + m - 3);
    } else {
        for (int m = 0; m < 7; ++m) {
            int kk = k + m - 3;
            kk += kk < 0 ? g.nth : 0;
            kk -= kk >= g.nth ? g.nth : 0;
            u[m] = P[(long long)kk * g.nxz + (long long)ix * g.nz + iz];
        }
    }
}

// Upwind WENO5 derivative W and its Jacobian row dW/du[m] (m = 0..6 at
// offsets -3..3); differences formed in T, the derivative in R.
template <typename T, typename R>
__device__ __forceinline__ R weno_row(const T (&u)[7], bool minus, R (&row)[7]) {
    R d[6];
    for (int m = 0; m < 6; ++m) d[m] = (R)(u[m + 1] - u[m]);
    R gr[5];
    if (minus) {
        const R W = weno5_grad<R>(d[0], d[1], d[2], d[3], d[4], gr);
        row[0] = -gr[0];
        row[1] = gr[0] - gr[1];
        row[2] = gr[1] - gr[2];
        row[3] = gr[2] - gr[3];
        row[4] = gr[3] - gr[4];
        row[5] = gr[4];
        row[6] = (R)0;
        return W;
    }
    const R W = weno5_grad<R>(d[5], d[4], d[3], d[2], d[1], gr);
    row[6] = gr[0];
    row[5] = gr[1] - gr[0];
    row[4] = gr[2] - gr[1];
    row[3] = gr[3] - gr[2];
    row[2] = gr[4] - gr[3];
    row[1] = -gr[4];
    row[0] = (R)0;
    return W;
}

struct AdjArgs {
    GridArgs g;
    const void* vel;    // vel3d
    const void* Uin;    // stage input state
    const void* lam;    // lambda of the stage output (state layout)
    void* pk;           // packets [2][3][7][stride] in R
    void* gvel;         // [3][stride] in R, accumulated
    double cbdt;        // cb * dt
    double xs, zs, r02;
};

__device__ __forceinline__ bool in_ball(const GridArgs& g, int ix, int iz, double xs, double zs, double r02) {
    const double ddx = g.x0 + (ix + 0.5) * g.dx - xs, ddz = g.z0 + (iz + 0.5) * g.dz - zs;
    return ddx * ddx + ddz * ddz <= r02;
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_packets(AdjArgs a) {
    const GridArgs& g = a.g;
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (iz >= g.nz || ix >= g.nx) return;
    const long long S = g.stride, c = (long long)k * g.nxz + (long long)ix * g.nz + iz;
    R* pk = static_cast<R*>(a.pk);
    const R* lamR = static_cast<const R*>(a.lam);
    const double* lamP = reinterpret_cast<const double*>(lamR + 5 * S);
    const bool ball = in_ball(g, ix, iz, a.xs, a.zs, a.r02);
    const R mu[2] = {ball ? (R)0 : lamR[c], ball ? (R)0 : (R)lamP[c]};
    if (mu[0] == (R)0 && mu[1] == (R)0) {
        for (int q = 0; q < NQ; ++q) pk[pk_idx(g, q, k, ix, iz)] = (R)0;
        return;
    }
    const R* V = static_cast<const R*>(a.vel);
    const double inv[3] = {1.0 / g.dx, 1.0 / g.dz, 1.0 / g.dth};
    const R cvel[3] = {V[EGB_VX * S + c] * (R)inv[0], V[EGB_VZ * S + c] * (R)inv[1], V[EGB_VT * S + c] * (R)inv[2]};
    const R* phi = static_cast<const R*>(a.Uin);
    const double* psi = reinterpret_cast<const double*>(phi + 5 * S);
    R* gv = static_cast<R*>(a.gvel);
    for (int axis = 0; axis < 3; ++axis) {
        const bool minus = cvel[axis] >= (R)0;
        R row[7], Wsum = (R)0;
        {
            R u[7];
            stencil7<R>(phi, g, k, ix, iz, axis, u);
            const R W = weno_row<R, R>(u, minus, row);
            const R coef = (R)(-a.cbdt) * cvel[axis] * mu[0];
            for (int j = 0; j < NSLOT; ++j) pk[pk_idx(g, (0 * 3 + axis) * NSLOT + j, k, ix, iz)] = coef * row[j];
            Wsum += mu[0] * W;
        }
        {
            double u[7];
            stencil7<double>(psi, g, k, ix, iz, axis, u);
            const R W = weno_row<double, R>(u, minus, row);
            const R coef = (R)(-a.cbdt) * cvel[axis] * mu[1];
            for (int j = 0; j < NSLOT; ++j) pk[pk_idx(g, (1 * 3 + axis) * NSLOT + j, k, ix, iz)] = coef * row[j];
            Wsum += mu[1] * W;
        }
        gv[axis * S + c] += (R)(-a.cbdt * inv[axis]) * Wsum;
    }
}

// Sum of the packets of plane f aimed at cell (k, ix, iz).
template <typename R>
__device__ __forceinline__ double gather_plane(const R* pk, const GridArgs& g, int f, int k, int ix, int iz) {
    double acc = 0.0;
    // x: source ix - j, slot j
    {
        const int q0 = (f * 3 + 0) * NSLOT + 3;
        R v[7];
#pragma unroll
        for (int j = -3; j <= 3; ++j) {  // branch-free: clamped source, weight 0 outside
            const int xs = ix - j;
            const R r = pk[pk_idx(g, q0 + j, k, min(max(xs, 0), g.nx - 1), iz)];
            v[j + 3] = (xs >= 0 && xs < g.nx) ? r : (R)0;
        }
#pragma unroll
        for (int j = 0; j < 7; ++j) acc += (double)v[j];
        if (ix <= 1 || ix >= g.nx - 2) {
            for (int m = 1; m <= 3; ++m) {
                const bool lo = ix <= 1;
                const double w = (ix == 0 || ix == g.nx - 1) ? (double)(m + 1) : (double)(-m);
                const int gpos = lo ? -m : g.nx - 1 + m;
                for (int j = -3; j <= 3; ++j) {
                    const int xs = gpos - j;
                    if (xs >= 0 && xs < g.nx) acc += w * (double)pk[pk_idx(g, q0 + j, k, xs, iz)];
                }
            }
        }
    }
    // z
    {
        const int q0 = (f * 3 + 1) * NSLOT + 3;
        R v[7];
#pragma unroll
        for (int j = -3; j <= 3; ++j) {
            const int zs = iz - j;
            const R r = pk[pk_idx(g, q0 + j, k, ix, min(max(zs, 0), g.nz - 1))];
            v[j + 3] = (zs >= 0 && zs < g.nz) ? r : (R)0;
        }
#pragma unroll
        for (int j = 0; j < 7; ++j) acc += (double)v[j];
        if (iz <= 1 || iz >= g.nz - 2) {
            for (int m = 1; m <= 3; ++m) {
                const bool lo = iz <= 1;
                const double w = (iz == 0 || iz == g.nz - 1) ? (double)(m + 1) : (double)(-m);
                const int gpos = lo ? -m : g.nz - 1 + m;
                for (int j = -3; j <= 3; ++j) {
                    const int zs = gpos - j;
                    if (zs >= 0 && zs < g.nz) acc += w * (double)pk[pk_idx(g, q0 + j, k, ix, zs)];
                }
            }
        }
    }
    // theta (periodic)
    {
        const int q0 = (f * 3 + 2) * NSLOT + 3;
        R v[7];
#pragma unroll
        for (int j = -3; j <= 3; ++j) {
            int ks = k - j;
            ks += ks < 0 ? g.nth : 0;
            ks -= ks >= g.nth ? g.nth : 0;
            v[j + 3] = pk[pk_idx(g, q0 + j, ks, ix, iz)];
        }
#pragma unroll
        for (int j = 0; j < 7; ++j) acc += (double)v[j];
    }
    return acc;
}

// STAGE 2: lam_acc = ca mu + [ball] lam (may alias lam), lam_in = cb mu + T^T mu
// STAGE 1: lam_acc += ca mu + [ball] lam,               lam_in = cb mu + T^T mu
// STAGE 0: lam_acc += [ball] lam + cb mu + T^T mu       (Uin is U0)
template <typename R, int STAGE>
__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs a, void* lam_in, void* lam_acc, double ca, double cb) {
    const GridArgs& g = a.g;
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (iz >= g.nz || ix >= g.nx) return;
    const long long S = g.stride, c = (long long)k * g.nxz + (long long)ix * g.nz + iz;
    const R* lamR = static_cast<const R*>(a.lam);
    const double* lamP = reinterpret_cast<const double*>(lamR + 5 * S);
    const bool ball = in_ball(g, ix, iz, a.xs, a.zs, a.r02);
    const double lo[2] = {(double)lamR[c], lamP[c]};
    const double mu[2] = {ball ? 0.0 : lo[0], ball ? 0.0 : lo[1]};
    const R* pk = static_cast<const R*>(a.pk);
    double lin[2];
    for (int f = 0; f < 2; ++f) lin[f] = cb * mu[f] + gather_plane<R>(pk, g, f, k, ix, iz);
    R* accR = static_cast<R*>(lam_acc);
    double* accP = reinterpret_cast<double*>(accR + 5 * S);
    double add[2];
    for (int f = 0; f < 2; ++f) add[f] = ball ? lo[f] : ca * mu[f];
    if (STAGE == 2) {
        accR[c] = (R)add[0];
        accP[c] = add[1];
    } else if (STAGE == 1) {
        accR[c] = (R)((double)accR[c] + add[0]);
        accP[c] += add[1];
    } else {
        accR[c] = (R)((double)accR[c] + add[0] + lin[0]);
        accP[c] += add[1] + lin[1];
    }
    if (STAGE != 0) {
        R* inR = static_cast<R*>(lam_in);
        double* inP = reinterpret_cast<double*>(inR + 5 * S);
        inR[c] = (R)lin[0];
        inP[c] = lin[1];
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
    const double* psi = reinterpret_cast<const double*>(phi + 5 * a.stride);
    R* lphi = reinterpret_cast<R*>(lam);
    double* lpsi = reinterpret_cast<double*>(lphi + 5 * a.stride);
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
// per theta slice, contract lambda0 with (x - xs, z - zs), then differentiate
// g_perp and p with respect to the five source values (dual numbers); the
// slice's five partial derivatives go to gms[k][5] (summed in order later).
template <typename R>
__global__ __launch_bounds__(256) void k_adj_source(GridArgs a, const double* C, egb_source src, const char* lam0,
                                                    double* gms) {
    const int k = blockIdx.x;
    const R* lphi = reinterpret_cast<const R*>(lam0);
    const double* lpsi = reinterpret_cast<const double*>(lphi + 5 * a.stride);
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

inline dim3 cells(const GridArgs& a) { return dim3((a.nz + 63) / 64, (a.nx + 3) / 4, a.nth); }

template <typename R>
hipError_t adj_stage_t(const AdjArgs& a, int stage, void* lam_in, void* lam_acc, hipStream_t s) {
    static const double CA[3] = {0.0, 0.75, 1.0 / 3.0}, CB[3] = {1.0, 0.25, 2.0 / 3.0};
    k_adj_packets<R><<<cells(a.g), dim3(64, 4), 0, s>>>(a);
    switch (stage) {
        case 2: k_adj_gather<R, 2><<<cells(a.g), dim3(64, 4), 0, s>>>(a, lam_in, lam_acc, CA[2], CB[2]); break;
        case 1: k_adj_gather<R, 1><<<cells(a.g), dim3(64, 4), 0, s>>>(a, lam_in, lam_acc, CA[1], CB[1]); break;
        default: k_adj_gather<R, 0><<<cells(a.g), dim3(64, 4), 0, s>>>(a, lam_in, lam_acc, CA[0], CB[0]); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t adjoint_packet_bytes(const egb_grid& g) {
    return (size_t)NQ * 64 * (size_t)((g.nz + 63) / 64) * (size_t)g.nx * (size_t)g.nth * real_size(g);
}

hipError_t launch_adjoint_stage(const GridArgs& g, int dtype, int stage, const void* vel, const void* Uin,
                                const void* lam_out, void* lam_in, void* lam_acc, void* packets, void* gvel,
                                double dt, double xs, double zs, double r02, hipStream_t s) {
    static const double CB[3] = {1.0, 0.25, 2.0 / 3.0};
    AdjArgs a;
    a.g = g;
    a.vel = vel;
    a.Uin = Uin;
    a.lam = lam_out;
    a.pk = packets;
    a.gvel = gvel;
    a.cbdt = CB[stage] * dt;
    a.xs = xs;
    a.zs = zs;
    a.r02 = r02;
    return dtype == EGB_F64 ? adj_stage_t<double>(a, stage, lam_in, lam_acc, s)
                            : adj_stage_t<float>(a, stage, lam_in, lam_acc, s);
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
                                 const egb_source& src, const void* gvel, const void* lam0, double* grad, double* gtab,
                                 double* gms, hipStream_t s) {
    const long long nt = 15 * a.nxz;
    if (dtype == EGB_F64) {
        k_adj_vtable<double><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(a, coeff2d, (const double*)gvel, gtab);
        k_adj_source<double><<<a.nth, 256, 0, s>>>(a, coeff2d, src, (const char*)lam0, gms);
    } else {
        k_adj_vtable<float><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(a, coeff2d, (const float*)gvel, gtab);
        k_adj_source<float><<<a.nth, 256, 0, s>>>(a, coeff2d, src, (const char*)lam0, gms);
    }
    k_adj_fields<<<(unsigned)((a.nxz + 255) / 256), 256, 0, s>>>(a, m, gtab, gms, src, grad);
    return hipGetLastError();
}

}  // namespace egb
