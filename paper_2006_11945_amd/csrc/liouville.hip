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
//
// Work decomposition.  A block owns a (z, theta) tile of 64 x TK cells and
// walks a chunk of x.  Each thread keeps the seven x-neighbours of its own
// (theta, z) column in registers (a queue shifted once per x step), so the
// x-stencil and the x-ghosts cost no memory traffic.  The current x slice of
// the tile, with a 3-cell halo in z (ghosts by extrapolation) and in theta
// (periodic), sits in LDS (double buffered, one barrier per x step); the z-
// and theta-stencils read it at immediate offsets.  Blocks are numbered so
// that consecutive tiles land on the same XCD (shared L2 for the theta halo).
#include <hip/hip_runtime.h>
#include <stdlib.h>

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

#ifndef WAVES_PER_EU
#define WAVES_PER_EU 3
#endif
constexpr int TZ = 64;       // z cells per tile (one wavefront row)
constexpr int PZ = TZ + 6;   // padded LDS row

// WENO5 on seven values u[0..6] at offsets -3..3 (upwind side chosen by
// `minus`); differences are formed in T and the derivative in R.
template <typename T, typename R>
__device__ __forceinline__ R weno7(const T (&u)[7], bool minus) {
    // written with scalars: an indexed select would become a computed index
    const T d0 = u[1] - u[0], d1 = u[2] - u[1], d2 = u[3] - u[2];
    const T d3 = u[4] - u[3], d4 = u[5] - u[4], d5 = u[6] - u[5];
    const R v1 = (R)(minus ? d0 : d5), v2 = (R)(minus ? d1 : d4), v3 = (R)(minus ? d2 : d3);
    const R v4 = (R)(minus ? d3 : d2), v5 = (R)(minus ? d4 : d1);
    return weno5<R>(v1, v2, v3, v4, v5);
}

// Raw buffer access: one descriptor per array (base, size < 4 GiB), a 32-bit
// per-lane byte offset and the plane offset in the scalar offset register.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          (int)voff, (int)soff, 0);
}

// Value of one plane at (slice kb, x, z) with the ghost rules: x or z outside
// the domain -> linear extrapolation from the two nearest cells along that
// axis; both outside (a corner, never read) -> 0.  `soff` is the plane's
// byte offset in the array.
template <typename T>
__device__ __forceinline__ T fetch(__amdgpu_buffer_rsrc_t r, unsigned soff, const GridArgs& g, unsigned kb, int x,
                                   int z) {
    const bool xo = x < 0 || x >= g.nx, zo = z >= g.nz || z < 0;
    if (!xo && !zo) return bload<T>(r, (kb + (unsigned)(x * g.nz + z)) * (unsigned)sizeof(T), soff);
    if (xo && zo) return (T)0;
    if (xo) {
        const int b0 = x < 0 ? 0 : g.nx - 1, b1 = x < 0 ? 1 : g.nx - 2, e = x < 0 ? -x : x - (g.nx - 1);
        return (T)(e + 1) * bload<T>(r, (kb + (unsigned)(b0 * g.nz + z)) * (unsigned)sizeof(T), soff) -
               (T)e * bload<T>(r, (kb + (unsigned)(b1 * g.nz + z)) * (unsigned)sizeof(T), soff);
    }
    const int b0 = z < 0 ? 0 : g.nz - 1, b1 = z < 0 ? 1 : g.nz - 2, e = z < 0 ? -z : z - (g.nz - 1);
    const unsigned xb = kb + (unsigned)(x * g.nz);
    return (T)(e + 1) * bload<T>(r, (xb + b0) * (unsigned)sizeof(T), soff) -
           (T)e * bload<T>(r, (xb + b1) * (unsigned)sizeof(T), soff);
}

struct TileArgs {
    int ntz, ntk, nxc, kx, nblocks;
    unsigned state_bytes, vel_bytes;
};

// XCD-aware numbering: hardware block b runs on XCD b % 8; give each XCD a
// contiguous range of logical tiles (a bijection of [0, n)).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q8 = n >> 3, r8 = n & 7, xcd = b & 7;
    return xcd * q8 + min(xcd, r8) + (b >> 3);
}

template <typename R, int TK>
struct StageSmem {
    static constexpr int PLANE = (TK + 6) * PZ;
    R r[2][5 * PLANE];
    double p[2][PLANE];
};

// One (z, theta) tile x one x chunk of an RK stage; `logical` numbers the
// tile within its problem.
// KIN: only phi1 and psi (the planes a traveltime depends on).
template <typename R, int STAGE, int TK, bool KIN>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const TileArgs& t, int logical,
                                           StageSmem<R, TK>& sm) {
    constexpr int PLANE = StageSmem<R, TK>::PLANE;
    constexpr int NHALO = 6 * TZ + 6 * TK;
    static_assert(NHALO <= 64 * TK, "one halo slot per thread");
    constexpr unsigned ES = sizeof(R);
    constexpr int NP = KIN ? 1 : 5;  // R planes marched
    auto& sR = sm.r;
    auto& sP = sm.p;

    const GridArgs& g = a.g;
    const int tzi = logical % t.ntz;
    const int rest = logical / t.ntz;
    const int tki = rest % t.ntk;
    const int xc = rest / t.ntk;

    const int tz = threadIdx.x, tk = threadIdx.y, tid = tk * TZ + tz;
    const int iz = tzi * TZ + tz;
    const int kraw = tki * TK + tk;
    const int k = kraw < g.nth ? kraw : kraw - g.nth;  // ragged theta tiles wrap (never written)
    const bool valid = iz < g.nz && kraw < g.nth;
    const unsigned nxz = (unsigned)g.nxz, S = (unsigned)g.stride;
    const unsigned kb = (unsigned)k * nxz;
    const auto rUi = make_rsrc(a.Uin, t.state_bytes);
    const auto rU0 = make_rsrc(a.U0, t.state_bytes);
    const auto rUo = make_rsrc(a.Uout, t.state_bytes);
    const auto rV = make_rsrc(a.vel, t.vel_bytes);
    const unsigned SP = S * ES;          // bytes per R plane
    const unsigned PSI = 5u * SP;        // byte offset of the psi plane

    // halo slot of this thread (if any): theta rows first, then z columns
    bool has_halo = tid < NHALO;
    int hk = 0, hz = 0;  // LDS coordinates (0-based, padded)
    unsigned hkb = 0;
    int hzg = 0;         // global z of the halo cell
    if (has_halo) {
        if (tid < 6 * TZ) {
            const int r = tid / TZ;
            hz = tid % TZ + 3;
            hk = r < 3 ? r : TK + r;
            int kk = tki * TK + hk - 3;
            kk = ((kk % g.nth) + g.nth) % g.nth;
            hkb = (unsigned)kk * nxz;
            hzg = min(tzi * TZ + hz - 3, g.nz - 1);  // columns beyond nz are never read
        } else {
            const int h = tid - 6 * TZ, r = h / TK;
            hk = h % TK + 3;
            hz = r < 3 ? r : TZ + r;
            int kk = tki * TK + hk - 3;
            kk = kk < g.nth ? kk : kk - g.nth;
            hkb = (unsigned)kk * nxz;
            hzg = tzi * TZ + hz - 3;
            if (hzg > g.nz + 2) has_halo = false;  // beyond the last ghost: never read
        }
    }

    const int x0 = xc * t.kx;
    const int x1 = min(x0 + t.kx, g.nx);
    // queue of the column's x-neighbours: q[f][j] at x - 3 + j
    R q[NP][7];
    double qp[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int x = x0 - 3 + j;
#pragma unroll
        for (int f = 0; f < NP; ++f) q[f][j] = fetch<R>(rUi, f * SP, g, kb, x, iz);
        qp[j] = fetch<double>(rUi, PSI, g, kb, x, iz);
    }
    // halo values of the first slice
    R hv[NP];
    double hp = 0.0;
#pragma unroll
    for (int f = 0; f < NP; ++f) hv[f] = has_halo ? fetch<R>(rUi, f * SP, g, hkb, x0, hzg) : (R)0;
    if (has_halo) hp = fetch<double>(rUi, PSI, g, hkb, x0, hzg);

    const R inv_dx = (R)(1.0 / g.dx), inv_dz = (R)(1.0 / g.dz), inv_dt = (R)(1.0 / g.dth);
    const R dtR = (R)a.dt;
    constexpr double ca = RK<STAGE>::ca, cb = RK<STAGE>::cb;
    const double zc = g.z0 + (iz + 0.5) * g.dz - a.zs;
    const int me = (tk + 3) * PZ + tz + 3;
    const int hi = hk * PZ + hz;

    int buf = 0;
    for (int x = x0; x < x1; ++x, buf ^= 1) {
        // slice x into LDS: own column from the queue, halo from registers
        R* L = sR[buf];
        double* LP = sP[buf];
#pragma unroll
        for (int f = 0; f < NP; ++f) L[f * PLANE + me] = q[f][3];
        LP[me] = qp[3];
        if (has_halo) {
#pragma unroll
            for (int f = 0; f < NP; ++f) L[f * PLANE + hi] = hv[f];
            LP[hi] = hp;
        }
        // next queue entry (x + 4) and next halo slice (x + 1)
        R qn[NP];
        double qpn;
        if (x + 4 < g.nx && iz < g.nz) {
            const unsigned o = kb + (unsigned)((x + 4) * g.nz + iz);
#pragma unroll
            for (int f = 0; f < NP; ++f) qn[f] = bload<R>(rUi, o * ES, f * SP);
            qpn = bload<double>(rUi, o * 8u, PSI);
        } else {
#pragma unroll
            for (int f = 0; f < NP; ++f) qn[f] = fetch<R>(rUi, f * SP, g, kb, x + 4, iz);
            qpn = fetch<double>(rUi, PSI, g, kb, x + 4, iz);
        }
        if (has_halo && x + 1 < x1) {
            if (hzg >= 0 && hzg < g.nz) {
                const unsigned o = hkb + (unsigned)((x + 1) * g.nz + hzg);
#pragma unroll
                for (int f = 0; f < NP; ++f) hv[f] = bload<R>(rUi, o * ES, f * SP);
                hp = bload<double>(rUi, o * 8u, PSI);
            } else {
#pragma unroll
                for (int f = 0; f < NP; ++f) hv[f] = fetch<R>(rUi, f * SP, g, hkb, x + 1, hzg);
                hp = fetch<double>(rUi, PSI, g, hkb, x + 1, hzg);
            }
        }
        __syncthreads();

        if (valid) {
            const unsigned c = kb + (unsigned)(x * g.nz + iz);
            const unsigned cR = c * ES, c8 = c * 8u;
            const double xr = g.x0 + (x + 0.5) * g.dx - a.xs;
            if (xr * xr + zc * zc <= a.r02) {  // source ball: Dirichlet data
#pragma unroll
                for (int f = 0; f < NP; ++f) bstore(bload<R>(rU0, cR, f * SP), rUo, cR, f * SP);
                bstore(bload<double>(rU0, c8, PSI), rUo, c8, PSI);
            } else {
                const R cx = bload<R>(rV, cR, EGB_VX * SP) * inv_dx;
                const R cz = bload<R>(rV, cR, EGB_VZ * SP) * inv_dz;
                const R ct = bload<R>(rV, cR, EGB_VT * SP) * inv_dt;
                R A11 = 0, A12 = 0, A21 = 0, A22 = 0;
                if constexpr (!KIN) {
                    A11 = bload<R>(rV, cR, EGB_A11 * SP);
                    A12 = bload<R>(rV, cR, EGB_A12 * SP);
                    A21 = bload<R>(rV, cR, EGB_A21 * SP);
                    A22 = bload<R>(rV, cR, EGB_A22 * SP);
                }
                R u0[NP];
                double p0 = 0.0;
                if (STAGE != 0) {
#pragma unroll
                    for (int f = 0; f < NP; ++f) u0[f] = bload<R>(rU0, cR, f * SP);
                    p0 = bload<double>(rU0, c8, PSI);
                }
                const bool mx = cx >= (R)0, mz = cz >= (R)0, mt = ct >= (R)0;
                R Lf[NP];
#pragma unroll
                for (int f = 0; f < NP; ++f) {
                    const R* Lp = L + f * PLANE + me;
                    R uz[7], ut[7];
#pragma unroll
                    for (int m = 0; m < 7; ++m) {
                        uz[m] = Lp[m - 3];
                        ut[m] = Lp[(m - 3) * PZ];
                    }
                    Lf[f] = -(cx * weno7<R, R>(q[f], mx) + cz * weno7<R, R>(uz, mz) + ct * weno7<R, R>(ut, mt));
                }
                if constexpr (!KIN) {
                    Lf[EGB_RE_C] += A11 * q[EGB_RE_C][3] + A12 * q[EGB_RE_B][3];
                    Lf[EGB_RE_B] += A21 * q[EGB_RE_C][3] + A22 * q[EGB_RE_B][3];
                    Lf[EGB_IM_C] += A11 * q[EGB_IM_C][3] + A12 * q[EGB_IM_B][3];
                    Lf[EGB_IM_B] += A21 * q[EGB_IM_C][3] + A22 * q[EGB_IM_B][3];
                }
                double pz[7], pt[7];
                const double* LPp = LP + me;
#pragma unroll
                for (int m = 0; m < 7; ++m) {
                    pz[m] = LPp[m - 3];
                    pt[m] = LPp[(m - 3) * PZ];
                }
                const double conv = (double)cx * (double)weno7<double, R>(qp, mx) +
                                    (double)cz * (double)weno7<double, R>(pz, mz) +
                                    (double)ct * (double)weno7<double, R>(pt, mt);
                const double Lpsi = 1.0 - conv;
#pragma unroll
                for (int f = 0; f < NP; ++f) {
                    const R y = q[f][3] + dtR * Lf[f];
                    bstore((STAGE == 0) ? y : (R)ca * u0[f] + (R)cb * y, rUo, cR, f * SP);
                }
                const double yp = qp[3] + a.dt * Lpsi;
                bstore((STAGE == 0) ? yp : ca * p0 + cb * yp, rUo, c8, PSI);
            }
        }
        // shift the queue
#pragma unroll
        for (int j = 0; j < 6; ++j) {
#pragma unroll
            for (int f = 0; f < NP; ++f) q[f][j] = q[f][j + 1];
            qp[j] = qp[j + 1];
        }
#pragma unroll
        for (int f = 0; f < NP; ++f) q[f][6] = qn[f];
        qp[6] = qpn;
    }
}

template <typename R, int STAGE, int TK, bool KIN>
__global__ __launch_bounds__(64 * TK) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU)))
void k_stage(StageArgs a, TileArgs t) {
    __shared__ StageSmem<R, TK> sm;
    stage_tile<R, STAGE, TK, KIN>(a, t, xcd_remap(blockIdx.x, t.nblocks), sm);
}

// Batched march: a persistent grid walks one queue of tiles spanning every
// problem (uneven grids, own buffers and dt).  first[p] is the first queue
// index of problem p (first[nprob] = total).
struct BatchItem {
    StageArgs a[3];  // stage 0, 1, 2 buffers of this problem
    TileArgs t;
};

template <typename R, int STAGE, int TK>
__global__ __launch_bounds__(64 * TK) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU)))
void k_stage_batched(const BatchItem* __restrict__ items, const int* __restrict__ first, int nprob, int total) {
    __shared__ StageSmem<R, TK> sm;
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        const int t = xcd_remap(q, total);
        int lo = 0, hi = nprob;  // first[lo] <= t < first[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (first[mid] <= t) lo = mid; else hi = mid;
        }
        // private copies: the stage's stores cannot alias them, so they stay in scalar registers
        const StageArgs a = items[lo].a[STAGE];
        const TileArgs ta = items[lo].t;
        __syncthreads();  // the previous tile's last LDS reads are done
        stage_tile<R, STAGE, TK, false>(a, ta, t - first[lo], sm);
    }
}

unsigned long long state_bytes_of(const GridArgs& g, size_t es) {
    return (unsigned long long)g.stride * (5ull * es + 8ull);
}

template <typename R, int TK, bool KIN>
hipError_t launch_stage_t(const StageArgs& a, int stage, int kx, hipStream_t s) {
    TileArgs t;
    t.ntz = (a.g.nz + TZ - 1) / TZ;
    t.ntk = (a.g.nth + TK - 1) / TK;
    t.kx = kx;
    t.nxc = (a.g.nx + kx - 1) / kx;
    t.nblocks = t.ntz * t.ntk * t.nxc;
    t.state_bytes = (unsigned)state_bytes_of(a.g, sizeof(R));
    t.vel_bytes = (unsigned)(7ull * (unsigned long long)a.g.stride * sizeof(R));
    const dim3 grid(t.nblocks), block(TZ, TK);
    switch (stage) {
        case 0: k_stage<R, 0, TK, KIN><<<grid, block, 0, s>>>(a, t); break;
        case 1: k_stage<R, 1, TK, KIN><<<grid, block, 0, s>>>(a, t); break;
        default: k_stage<R, 2, TK, KIN><<<grid, block, 0, s>>>(a, t); break;
    }
    return hipGetLastError();
}

// x-chunk length: enough blocks to fill the chip several times over
// (EGB_STAGE_KX overrides, for tuning sweeps).
int choose_kx(const GridArgs& g, int tk) {
    static const int forced = [] {
        const char* e = getenv("EGB_STAGE_KX");
        return e ? atoi(e) : 0;
    }();
    if (forced > 0) return forced < g.nx ? forced : g.nx;
    const long long tiles = (long long)((g.nz + TZ - 1) / TZ) * ((g.nth + tk - 1) / tk);
    int kx = g.nx;
    while (kx > 8 && tiles * ((g.nx + kx - 1) / kx) < 512) kx = (kx + 1) / 2;
    return kx;
}

template <typename R, int TK>
hipError_t launch_batched_t(const void* items, const int* first, int nprob, int total, int stage, int grid,
                            hipStream_t s) {
    const dim3 block(TZ, TK);
    const BatchItem* it = static_cast<const BatchItem*>(items);
    switch (stage) {
        case 0: k_stage_batched<R, 0, TK><<<grid, block, 0, s>>>(it, first, nprob, total); break;
        case 1: k_stage_batched<R, 1, TK><<<grid, block, 0, s>>>(it, first, nprob, total); break;
        default: k_stage_batched<R, 2, TK><<<grid, block, 0, s>>>(it, first, nprob, total); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t batch_item_bytes() { return sizeof(BatchItem); }

// Fill the host-side item for one problem; returns its tile count.
int batch_item_fill(void* item, const GridArgs& g, int dtype, const void* vel, void* state, void* U1, void* U2,
                    double dt, double xs, double zs, double r02) {
    BatchItem& it = *static_cast<BatchItem*>(item);
    const int tk = dtype == EGB_F64 ? 8 : 12;
    const size_t es = dtype == EGB_F64 ? 8 : 4;
    TileArgs t;
    t.ntz = (g.nz + TZ - 1) / TZ;
    t.ntk = (g.nth + tk - 1) / tk;
    t.kx = choose_kx(g, tk);
    t.nxc = (g.nx + t.kx - 1) / t.kx;
    t.nblocks = t.ntz * t.ntk * t.nxc;
    t.state_bytes = (unsigned)state_bytes_of(g, es);
    t.vel_bytes = (unsigned)(7ull * (unsigned long long)g.stride * es);
    it.t = t;
    void* in[3] = {state, U1, U2};
    void* out[3] = {U1, U2, state};
    for (int s = 0; s < 3; ++s) {
        it.a[s].g = g;
        it.a[s].vel = vel;
        it.a[s].U0 = state;
        it.a[s].Uin = in[s];
        it.a[s].Uout = out[s];
        it.a[s].dt = dt;
        it.a[s].xs = xs;
        it.a[s].zs = zs;
        it.a[s].r02 = r02;
    }
    return t.nblocks;
}

hipError_t launch_stage_batched(const void* items, const int* first, int nprob, int total, int dtype, int stage,
                                int grid, hipStream_t s) {
    if (dtype == EGB_F64) return launch_batched_t<double, 8>(items, first, nprob, total, stage, grid, s);
    return launch_batched_t<float, 12>(items, first, nprob, total, stage, grid, s);
}

int stage_block_threads(int dtype) { return dtype == EGB_F64 ? 64 * 8 : 64 * 12; }

const void* stage_batched_kernel(int dtype, int stage) {
    if (dtype == EGB_F64)
        return stage == 0 ? (const void*)k_stage_batched<double, 0, 8>
                          : stage == 1 ? (const void*)k_stage_batched<double, 1, 8> : (const void*)k_stage_batched<double, 2, 8>;
    return stage == 0 ? (const void*)k_stage_batched<float, 0, 12>
                      : stage == 1 ? (const void*)k_stage_batched<float, 1, 12> : (const void*)k_stage_batched<float, 2, 12>;
}

bool stage_fits_32bit(const GridArgs& g, int dtype) {
    const size_t es = dtype == EGB_F64 ? 8 : 4;
    return state_bytes_of(g, es) < (1ull << 32) && 7ull * (unsigned long long)g.stride * es < (1ull << 32);
}

hipError_t launch_stage(const StageArgs& a, int dtype, int stage, hipStream_t s, bool kinematic) {
    if (dtype == EGB_F64)
        return kinematic ? launch_stage_t<double, 8, true>(a, stage, choose_kx(a.g, 8), s)
                         : launch_stage_t<double, 8, false>(a, stage, choose_kx(a.g, 8), s);
    return kinematic ? launch_stage_t<float, 12, true>(a, stage, choose_kx(a.g, 12), s)
                     : launch_stage_t<float, 12, false>(a, stage, choose_kx(a.g, 12), s);
}

}  // namespace egb
