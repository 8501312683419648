// Green's-function migration on the depth march's wavefields (section 6's
// application of eqs. 34-35).  With G[s][w][x] the Green's function of
// surface point s at frequency w (egb_paraxial_beam_sum's output of ns
// points one after another, x = ix nz + iz):
//   Born data  d[w][s][r] = omega_w^2 dA sum_x G[s][w][x] m[x] G[r][w][x]
//   image      I[x] = Re sum_w omega_w^2 dA sum_{s,r} conj(G[s][w][x])
//                     conj(G[r][w][x]) d[w][s][r],
// the adjoint of the data for a real reflectivity m (dA = dx dz).  Both are
// complex contractions over ns x ns x (nx nz) per frequency, small next to
// the beam sums that produce G; they run on the vector units with FP64
// accumulation and stage their operands in LDS.
#include <hip/hip_runtime.h>

#include "egb_internal.h"

namespace egb {
namespace {

constexpr int MG_MAXS = 64;   // surface points
constexpr int MG_WCH = 32;    // frequencies per launch
constexpr int BT = 16;        // Born tile: 16 sources x 16 receivers per block
constexpr int BK = 64;        // Born: image points per LDS chunk

struct MigW {
    double w2[MG_WCH];  // omega^2 dA of this chunk's frequencies
    int n, first;
};

template <typename R>
__device__ __forceinline__ double2 gval(const R* G, long long off) {
    return make_double2((double)G[2 * off], (double)G[2 * off + 1]);
}

// d[w][s][r]: block (r tile, s tile, frequency of the chunk), thread (r, s)
// of the tile; the image points run in chunks of BK through LDS.
template <typename R>
__global__ __launch_bounds__(BT* BT) void k_born(const R* G, const double* m, int ns, int nw, long long npt, MigW wc,
                                                 double* d) {
    __shared__ double2 As[BT][BK + 1];  // G[s] m over the chunk
    __shared__ double2 Bs[BT][BK + 1];  // G[r] over the chunk
    const int tr = threadIdx.x, ts = threadIdx.y, t = ts * BT + tr;
    const int r0 = blockIdx.x * BT, s0 = blockIdx.y * BT, wl = blockIdx.z;
    const int w = wc.first + wl;
    double re = 0.0, im = 0.0;
    for (long long x0 = 0; x0 < npt; x0 += BK) {
#pragma unroll
        for (int q = 0; q < (BT * BK) / (BT * BT); ++q) {
            const int idx = t + q * BT * BT, row = idx / BK, col = idx % BK;
            const long long x = x0 + col;
            const bool xin = x < npt;
            const int s = s0 + row, r = r0 + row;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            if (xin && s < ns) {
                a = gval(G, ((long long)s * nw + w) * npt + x);
                const double mx = m[x];
                a.x *= mx;
                a.y *= mx;
            }
            if (xin && r < ns) b = gval(G, ((long long)r * nw + w) * npt + x);
            As[row][col] = a;
            Bs[row][col] = b;
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < BK; ++k) {
            const double2 a = As[ts][k], b = Bs[tr][k];
            re = fma(a.x, b.x, fma(-a.y, b.y, re));
            im = fma(a.x, b.y, fma(a.y, b.x, im));
        }
        __syncthreads();
    }
    const int s = s0 + ts, r = r0 + tr;
    if (s < ns && r < ns) {
        const long long o = (((long long)w * ns + s) * ns + r) * 2;
        d[o] = wc.w2[wl] * re;
        d[o + 1] = wc.w2[wl] * im;
    }
}

// I[x] for a chunk of XC image points: per frequency the data matrix and the
// chunk's G of every surface point go to LDS; thread (x, s-group) forms
// y_s = sum_r d[s][r] conj(g_r) for its sources and adds Re(conj(g_s) y_s);
// the s-groups of one x are summed in LDS.  accumulate: add to the image
// (later frequency chunks), else overwrite it.
template <typename R, int XC>
__global__ __launch_bounds__(256) void k_migrate(const R* G, const double* d, int ns, int nw, long long npt, MigW wc,
                                                 int accumulate, double* img) {
    constexpr int NG = 256 / XC;  // source groups per image point
    __shared__ double2 Ds[MG_MAXS * MG_MAXS];
    __shared__ double2 Gs[MG_MAXS][XC];
    __shared__ double part[NG][XC];
    const int t = threadIdx.x, xl = t % XC, sg = t / XC;
    const long long x0 = (long long)blockIdx.x * XC, x = x0 + xl;
    double acc = 0.0;
    for (int wl = 0; wl < wc.n; ++wl) {
        const int w = wc.first + wl;
        for (int i = t; i < ns * ns; i += 256) {
            const long long o = ((long long)w * ns * ns + i) * 2;
            Ds[i] = make_double2(d[o], d[o + 1]);
        }
        for (int i = t; i < ns * XC; i += 256) {
            const int s = i / XC, c = i % XC;
            const long long xx = x0 + c;
            Gs[s][c] = xx < npt ? gval(G, ((long long)s * nw + w) * npt + xx) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        double aw = 0.0;
        for (int s = sg; s < ns; s += NG) {
            double yre = 0.0, yim = 0.0;  // y_s = sum_r d[s][r] conj(g_r)
            for (int r = 0; r < ns; ++r) {
                const double2 dv = Ds[s * ns + r], g = Gs[r][xl];
                yre = fma(dv.x, g.x, fma(dv.y, g.y, yre));
                yim = fma(dv.y, g.x, fma(-dv.x, g.y, yim));
            }
            const double2 gs = Gs[s][xl];
            aw = fma(gs.x, yre, fma(gs.y, yim, aw));  // Re(conj(g_s) y_s)
        }
        acc = fma(wc.w2[wl], aw, acc);
        __syncthreads();
    }
    part[sg][xl] = acc;
    __syncthreads();
    if (sg == 0 && x < npt) {
        double sum = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) sum += part[g][xl];
        img[x] = accumulate ? img[x] + sum : sum;
    }
}

MigW chunk_of(const double* omegas, int first, int nw, double dA) {
    MigW wc;
    wc.first = first;
    wc.n = nw - first < MG_WCH ? nw - first : MG_WCH;
    for (int i = 0; i < MG_WCH; ++i) wc.w2[i] = i < wc.n ? omegas[first + i] * omegas[first + i] * dA : 0.0;
    return wc;
}

}  // namespace

int migration_max_points() { return MG_MAXS; }

hipError_t launch_born_data(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                            const double* m, double* d, hipStream_t s) {
    const long long npt = (long long)g.nx * g.nz;
    const double dA = g.dx * g.dz;
    const dim3 block(BT, BT);
    for (int first = 0; first < nw; first += MG_WCH) {
        const MigW wc = chunk_of(omegas, first, nw, dA);
        const dim3 grid((ns + BT - 1) / BT, (ns + BT - 1) / BT, wc.n);
        if (dtype == EGB_F64)
            k_born<double><<<grid, block, 0, s>>>(static_cast<const double*>(G), m, ns, nw, npt, wc, d);
        else
            k_born<float><<<grid, block, 0, s>>>(static_cast<const float*>(G), m, ns, nw, npt, wc, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_migrate(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                          const double* d, double* image, hipStream_t s) {
    const long long npt = (long long)g.nx * g.nz;
    const double dA = g.dx * g.dz;
    for (int first = 0; first < nw; first += MG_WCH) {
        const MigW wc = chunk_of(omegas, first, nw, dA);
        const int acc = first > 0;
        if (dtype == EGB_F64) {
            const unsigned blocks = (unsigned)((npt + 31) / 32);
            k_migrate<double, 32><<<blocks, 256, 0, s>>>(static_cast<const double*>(G), d, ns, nw, npt, wc, acc, image);
        } else {
            const unsigned blocks = (unsigned)((npt + 31) / 32);
            k_migrate<float, 32><<<blocks, 256, 0, s>>>(static_cast<const float*>(G), d, ns, nw, npt, wc, acc, image);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace egb
