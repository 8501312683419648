// Green's-function migration on the depth march's wavefields (section 6's
// application of eqs. 34-35).  With G[s][w][x] the Green's function of
// surface point s at frequency w (egb_paraxial_beam_sum's output of ns
// points one after another, x = ix nz + iz):
//   Born data  d[w][s][r] = omega_w^2 dA sum_x G[s][w][x] m[x] G[r][w][x]
//   image      I[x] = Re sum_w omega_w^2 dA sum_{s,r} conj(G[s][w][x])
//                     conj(G[r][w][x]) d[w][s][r],
// the adjoint of the data for a real reflectivity m (dA = dx dz).  Both are
// complex contractions over ns x ns x (nx nz) per frequency, computed in FP64
// on the matrix cores (v_mfma_f64_16x16x4f64; the Green's functions are
// converted from the grid dtype as they are staged).  The Born data is a
// long reduction over image points with a small output (ns x ns per
// frequency): the points are split over blocks, each block stages chunks of
// the Green's functions in LDS (the next chunk loaded into registers while
// the current one is multiplied), and the partial sums (caller's workspace)
// are added in a fixed order, so the result does not depend on timing.  The
// image forms Y = d conj(g) for 64 image points per wavefront, then
// Re conj(g)^T Y per point.
#include <hip/hip_runtime.h>

#include "egb_internal.h"

namespace egb {
namespace {

constexpr int MG_MAXS = 64;   // surface points
constexpr int MG_WCH = 32;    // frequencies per launch
constexpr int BO = 32;        // Born: output tile of 32 sources x 32 receivers per block
constexpr int BKC = 64;       // Born: image points per LDS chunk (16 per wavefront)
constexpr int BORN_BLOCKS = 2048;  // Born: blocks aimed at per launch (points split to reach it)
constexpr int MS = 32;        // image kernel on the matrix cores: up to 32 surface points

struct MigW {
    double w2[MG_WCH];  // omega^2 dA of this chunk's frequencies
    int n, first;
};

template <typename R>
__device__ __forceinline__ double2 gval(const R* G, long long off) {
    return make_double2((double)G[2 * off], (double)G[2 * off + 1]);
}

// Partial Born sums on the matrix cores: block (split p, frequency w,
// output tile), 4 wavefronts.  The block's image points [p kc, (p + 1) kc)
// run through LDS in chunks of BKC (the tile's 32 source rows times m, and
// its 32 receiver rows); wavefront q takes points 16 q .. 16 q + 15 of each
// chunk, 4 at a time, as the K = 4 of v_mfma_f64_16x16x4f64 (A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, C[i][j] in lane j + 16 (i % 4), item
// i / 4).  The complex tile is 2 x 2 blocks of 16 x 16, real and imaginary
// parts apart: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br (four products per
// block).  The four wavefronts' sums are added in order through LDS and the
// tile is written to part[p][w][s][r] (complex).
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename R>
__global__ __launch_bounds__(256, 2) void k_born_part(const R* G, const double* m, int ns, int nw, long long npt,
                                                   long long kc, double* part) {
    constexpr int ROW = BKC + 1;  // padded LDS row (double2)
    __shared__ double2 sm[2 * BO * ROW];
    double2* As = sm;
    double2* Bs = sm + BO * ROW;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    const int p = blockIdx.x, w = blockIdx.y;
    const int nt = (ns + BO - 1) / BO;
    const int s0 = (int)(blockIdx.z / nt) * BO, r0 = (int)(blockIdx.z % nt) * BO;
    const long long xa = (long long)p * kc, xb = xa + kc < npt ? xa + kc : npt;
    v4d cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
            cim[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
        }
    // thread t stages point c = t % 64 of the rows t / 64 + 4 q; the values of
    // the next chunk are loaded into registers while this one is multiplied.
    // A diagonal tile (the same source and receiver rows) loads each row once.
    const int c = t & 63;
    const bool diag = s0 == r0;  // block-uniform
    R ga[BO / 4][2], gb[BO / 4][2];
    double mx = 0.0;
    auto fetch = [&](long long x0) {
        const long long x = x0 + c;
        const bool xin = x < xb;
        mx = xin ? m[x] : 0.0;
#pragma unroll
        for (int q = 0; q < BO / 4; ++q) {
            const int row = (t >> 6) + 4 * q;
            const int sr = s0 + row, rr = r0 + row;
            ga[q][0] = ga[q][1] = gb[q][0] = gb[q][1] = (R)0;
            if (xin && sr < ns) {
                const long long o = ((long long)sr * nw + w) * npt + x;
                ga[q][0] = G[2 * o];
                ga[q][1] = G[2 * o + 1];
            }
            if (!diag && xin && rr < ns) {
                const long long o = ((long long)rr * nw + w) * npt + x;
                gb[q][0] = G[2 * o];
                gb[q][1] = G[2 * o + 1];
            }
        }
    };
    if (xa < xb) fetch(xa);
    for (long long x0 = xa; x0 < xb; x0 += BKC) {
#pragma unroll
        for (int q = 0; q < BO / 4; ++q) {
            const int row = (t >> 6) + 4 * q;
            const double2 g = make_double2((double)ga[q][0], (double)ga[q][1]);
            As[row * ROW + c] = make_double2(g.x * mx, g.y * mx);
            Bs[row * ROW + c] = diag ? g : make_double2((double)gb[q][0], (double)gb[q][1]);
        }
        __syncthreads();
        if (x0 + BKC < xb) fetch(x0 + BKC);
#pragma unroll
        for (int q = 0; q < BKC / 16; ++q) {
            const int k = wave * (BKC / 4) + 4 * q + lk;
            const double2 a[2] = {As[li * ROW + k], As[(16 + li) * ROW + k]};
            const double2 b[2] = {Bs[li * ROW + k], Bs[(16 + li) * ROW + k]};
#pragma unroll
            for (int ts = 0; ts < 2; ++ts)
#pragma unroll
                for (int tr = 0; tr < 2; ++tr) {
                    cre[ts][tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].x, b[tr].x, cre[ts][tr], 0, 0, 0);
                    cre[ts][tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ts].y, b[tr].y, cre[ts][tr], 0, 0, 0);
                    cim[ts][tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].x, b[tr].y, cim[ts][tr], 0, 0, 0);
                    cim[ts][tr] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].y, b[tr].x, cim[ts][tr], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // the wavefronts' sums through LDS (the staging buffer, free after the
    // loop's last barrier), added in wavefront order; entry e = ((ts 2 + tr)
    // 2 + part) 4 + item
    double* red = reinterpret_cast<double*>(sm);  // [wave][e][lane], 4 x 32 x 64
#pragma unroll
    for (int ts = 0; ts < 2; ++ts)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = ((ts * 2 + tr) * 2) * 4 + v;
                red[(wave * 32 + e) * 64 + lane] = cre[ts][tr][v];
                red[(wave * 32 + e + 4) * 64 + lane] = cim[ts][tr][v];
            }
    __syncthreads();
#pragma unroll
    for (int e2 = 0; e2 < 8; ++e2) {
        const int idx = t + 256 * e2, e = idx >> 6, ln = idx & 63;
        const int v = e & 3, part_im = (e >> 2) & 1, tr = (e >> 3) & 1, ts = e >> 4;
        const int s = s0 + ts * 16 + (ln >> 4) + 4 * v, r = r0 + tr * 16 + (ln & 15);
        double sum = red[e * 64 + ln];
#pragma unroll
        for (int q = 1; q < 4; ++q) sum += red[(q * 32 + e) * 64 + ln];
        if (s < ns && r < ns) part[((((long long)p * nw + w) * ns + s) * ns + r) * 2 + part_im] = sum;
    }
}

// d[w][s][r] = omega_w^2 dA sum_p part[p][w][s][r], p in order: one thread
// per (frequency of the chunk, s, r).
__global__ __launch_bounds__(256) void k_born_reduce(const double* part, long long nsplit, int nw, int ns, MigW wc,
                                                     double* d) {
    const long long n = (long long)wc.n * ns * ns;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int wl = (int)(i / ((long long)ns * ns));
    const long long sr = i - (long long)wl * ns * ns;
    const long long e = (long long)(wc.first + wl) * ns * ns + sr;  // (w, s, r) entry
    const long long step = (long long)nw * ns * ns;
    double re = 0.0, im = 0.0;
    for (long long p = 0; p < nsplit; ++p) {
        re += part[2 * (p * step + e)];
        im += part[2 * (p * step + e) + 1];
    }
    d[2 * e] = wc.w2[wl] * re;
    d[2 * e + 1] = wc.w2[wl] * im;
}

// I[x] for more than MS surface points, XC image points per block: per
// frequency the data matrix and the chunk's G of every surface point go to LDS; thread (x, s-group) forms
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

// I[x] for 64 image points per block and ns <= MS surface points, on the
// matrix cores: wavefront q takes the chunk's frequencies q, q + 4, ...; per
// frequency it stages the data matrix (zero-padded to MS x MS) in its own LDS
// region and forms Y = d conj(g) over its 64 points (s x x, K = r) with
// v_mfma_f64_16x16x4f64: A = d[s][r] (2 tiles of 16 s), B = conj(g_r(x))
// read from the Green's functions (4 tiles of 16 x), Re Y += dr gr + di gi,
// Im Y += di gr - dr gi.  Lane (j, i) then holds Y for x = 16 tx + j and
// s = 16 ts + i + 4 v and adds Re conj(g_s) Y; the four lanes of one x are
// added by cross-lane exchange and the four wavefronts through LDS, both in
// a fixed order.  accumulate: add to the image (later frequency chunks),
// else overwrite it.
template <typename R>
__global__ __launch_bounds__(256, 2) void k_migrate_mfma(const R* G, const double* d, int ns, int nw, long long npt,
                                                         MigW wc, int accumulate, double* img) {
    constexpr int DR = MS + 1;  // padded LDS row (double2) of the data matrix
    __shared__ double2 Ds[4][MS * DR];
    __shared__ double part[4][64];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, lj = lane & 15, lq = lane >> 4;
    const long long xb0 = (long long)blockIdx.x * 64;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // per x tile: x = xb0 + 16 tx + lj
    const int nit = (wc.n + 3) / 4;
    const int nks = (ns + 3) / 4;  // K steps of 4 receivers
    for (int it = 0; it < nit; ++it) {
        const int wl = wave + 4 * it;
        const bool has = wl < wc.n;  // wavefront-uniform
        const int w = wc.first + (has ? wl : 0);
        if (has) {
            for (int i = lane; i < MS * MS; i += 64) {
                const int sr = i / MS, rr = i % MS;
                double2 v = make_double2(0.0, 0.0);
                if (sr < ns && rr < ns) {
                    const long long o = (((long long)w * ns + sr) * ns + rr) * 2;
                    v = make_double2(d[o], d[o + 1]);
                }
                Ds[wave][sr * DR + rr] = v;
            }
        }
        __syncthreads();
        if (has) {
            v4d yre[2][4], yim[2][4];
#pragma unroll
            for (int ts = 0; ts < 2; ++ts)
#pragma unroll
                for (int tx = 0; tx < 4; ++tx) {
                    yre[ts][tx] = (v4d){0.0, 0.0, 0.0, 0.0};
                    yim[ts][tx] = (v4d){0.0, 0.0, 0.0, 0.0};
                }
            // B operands one K step ahead (raw values, converted at use)
            R bn[4][2];
            auto fetch_b = [&](int ks) {
                const int rr = 4 * ks + lq;
#pragma unroll
                for (int tx = 0; tx < 4; ++tx) {
                    const long long x = xb0 + 16 * tx + lj;
                    bn[tx][0] = bn[tx][1] = (R)0;
                    if (rr < ns && x < npt) {
                        const long long o = ((long long)rr * nw + w) * npt + x;
                        bn[tx][0] = G[2 * o];
                        bn[tx][1] = G[2 * o + 1];
                    }
                }
            };
            fetch_b(0);
            for (int ks = 0; ks < nks; ++ks) {
                const int rr = 4 * ks + lq;
                const double2 a[2] = {Ds[wave][lj * DR + rr], Ds[wave][(16 + lj) * DR + rr]};
                double2 b[4];
#pragma unroll
                for (int tx = 0; tx < 4; ++tx) b[tx] = make_double2((double)bn[tx][0], (double)bn[tx][1]);
                if (ks + 1 < nks) fetch_b(ks + 1);
#pragma unroll
                for (int ts = 0; ts < 2; ++ts)
#pragma unroll
                    for (int tx = 0; tx < 4; ++tx) {
                        yre[ts][tx] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].x, b[tx].x, yre[ts][tx], 0, 0, 0);
                        yre[ts][tx] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].y, b[tx].y, yre[ts][tx], 0, 0, 0);
                        yim[ts][tx] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ts].y, b[tx].x, yim[ts][tx], 0, 0, 0);
                        yim[ts][tx] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ts].x, b[tx].y, yim[ts][tx], 0, 0, 0);
                    }
            }
            // Re sum_s conj(g_s) Y_s over this lane's sources, per x tile
#pragma unroll
            for (int tx = 0; tx < 4; ++tx) {
                const long long x = xb0 + 16 * tx + lj;
                double aw = 0.0;
#pragma unroll
                for (int ts = 0; ts < 2; ++ts)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int sr = 16 * ts + lq + 4 * v;
                        if (sr < ns && x < npt) {
                            const double2 g = gval(G, ((long long)sr * nw + w) * npt + x);
                            aw = fma(g.x, yre[ts][tx][v], fma(g.y, yim[ts][tx][v], aw));
                        }
                    }
                acc[tx] = fma(wc.w2[wl], aw, acc[tx]);
            }
        }
        __syncthreads();
    }
    // the four lanes of each x (lq = 0..3), then the four wavefronts
#pragma unroll
    for (int tx = 0; tx < 4; ++tx) {
        const double a1 = __shfl_xor(acc[tx], 16);
        const double s01 = lq & 1 ? a1 + acc[tx] : acc[tx] + a1;  // (lane lq even) + (lq odd)
        const double s23 = __shfl_xor(s01, 32);
        acc[tx] = lq & 2 ? s23 + s01 : s01 + s23;
    }
    if (lq == 0) {
#pragma unroll
        for (int tx = 0; tx < 4; ++tx) part[wave][16 * tx + lj] = acc[tx];
    }
    __syncthreads();
    const long long x = xb0 + lane;
    if (wave == 0 && x < npt) {
        const double sum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
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

// Split of the Born reduction: about BORN_BLOCKS blocks, at least one chunk
// of points per split; kc points per split, a multiple of the chunk.
static void born_split(long long npt, int ns, int nw, long long& nsplit, long long& kc) {
    const long long nt = (ns + BO - 1) / BO;
    const long long tiles = (long long)nw * nt * nt;
    const long long want = (BORN_BLOCKS + tiles - 1) / tiles;
    const long long most = (npt + BKC - 1) / BKC;
    nsplit = want < most ? want : most;
    if (nsplit < 1) nsplit = 1;
    kc = ((npt + nsplit - 1) / nsplit + BKC - 1) / BKC * BKC;
}

size_t born_workspace_bytes(long long npt, int ns, int nw) {
    long long nsplit, kc;
    born_split(npt, ns, nw, nsplit, kc);
    return (size_t)nsplit * (size_t)nw * (size_t)ns * (size_t)ns * 2 * sizeof(double);
}

hipError_t launch_born_data(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                            const double* m, double* d, void* work, hipStream_t s) {
    const long long npt = (long long)g.nx * g.nz;
    const double dA = g.dx * g.dz;
    long long nsplit, kc;
    born_split(npt, ns, nw, nsplit, kc);
    const int nt = (ns + BO - 1) / BO;
    double* part = static_cast<double*>(work);
    const dim3 grid((unsigned)nsplit, (unsigned)nw, (unsigned)(nt * nt));
    if (dtype == EGB_F64)
        k_born_part<double><<<grid, 256, 0, s>>>(static_cast<const double*>(G), m, ns, nw, npt, kc, part);
    else
        k_born_part<float><<<grid, 256, 0, s>>>(static_cast<const float*>(G), m, ns, nw, npt, kc, part);
    hipError_t e = hipGetLastError();
    for (int first = 0; first < nw && e == hipSuccess; first += MG_WCH) {
        const MigW wc = chunk_of(omegas, first, nw, dA);
        const long long n = (long long)wc.n * ns * ns;
        k_born_reduce<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(part, nsplit, nw, ns, wc, d);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_migrate(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                          const double* d, double* image, hipStream_t s) {
    const long long npt = (long long)g.nx * g.nz;
    const double dA = g.dx * g.dz;
    for (int first = 0; first < nw; first += MG_WCH) {
        const MigW wc = chunk_of(omegas, first, nw, dA);
        const int acc = first > 0;
        if (ns <= MS) {  // on the matrix cores
            const unsigned blocks = (unsigned)((npt + 63) / 64);
            if (dtype == EGB_F64)
                k_migrate_mfma<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(G), d, ns, nw, npt, wc, acc,
                                                             image);
            else
                k_migrate_mfma<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(G), d, ns, nw, npt, wc, acc,
                                                            image);
        } else if (dtype == EGB_F64) {
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
