// Green's-function migration on the depth march's wavefields (section 6's
// application of eqs. 34-35).  With G[s][w][x] the Green's function of
// surface point s at frequency w (egb_paraxial_beam_sum's output of ns
// points one after another, x = ix nz + iz):
//   Born data  d[w][s][r] = omega_w^2 dA sum_x G[s][w][x] m[x] G[r][w][x]
//   image      I[x] = Re sum_w omega_w^2 dA sum_{s,r} conj(G[s][w][x])
//                     conj(G[r][w][x]) d[w][s][r],
// the adjoint of the data for a real reflectivity m (dA = dx dz).  Both are
// complex contractions over ns x ns x (nx nz) per frequency with FP64
// accumulation on the vector units (FP64 matrix cores run no faster than the
// vector units on this chip, and the operands arrive as the grid dtype).
// The Born data is a long reduction over image points with a small output
// (ns x ns per frequency): the points are split over blocks, each block
// stages a chunk of the Green's functions in LDS and every lane keeps a 4 x 4
// register tile of the output, and the partial sums (caller's workspace) are
// added in a fixed order, so the result does not depend on timing.  The
// image keeps, per image point, the ns sums over receivers in registers
// while the data matrix is read from LDS by the whole wavefront at once.
#include <hip/hip_runtime.h>

#include "egb_internal.h"

namespace egb {
namespace {

constexpr int MG_MAXS = 64;   // surface points
constexpr int MG_WCH = 32;    // frequencies per launch
constexpr int BO = 32;        // Born: output tile of 32 sources x 32 receivers per block
constexpr int BKC = 64;       // Born: image points per LDS chunk (16 per wavefront)
constexpr int BORN_BLOCKS = 2048;  // Born: blocks aimed at per launch (points split to reach it)
constexpr int MS = 32;        // image kernel: surface points held per image point

struct MigW {
    double w2[MG_WCH];  // omega^2 dA of this chunk's frequencies
    int n, first;
};

template <typename R>
__device__ __forceinline__ double2 gval(const R* G, long long off) {
    return make_double2((double)G[2 * off], (double)G[2 * off + 1]);
}

// Partial Born sums: block (split p, frequency w, output tile), 4
// wavefronts.  The block's image points [p kc, (p + 1) kc) run through LDS in
// chunks of BKC (the tile's source rows times m, and its receiver rows);
// wavefront q takes points 16 q .. 16 q + 15 of each chunk and lane (ls, lr)
// the outputs s = s0 + ls + 8 i, r = r0 + lr + 8 j (i, j < 4).  The four
// wavefronts' sums are added in order through LDS and the tile is written
// to part[p][w][s][r] (complex).
template <typename R>
__global__ __launch_bounds__(256) void k_born_part(const R* G, const double* m, int ns, int nw, long long npt,
                                                   long long kc, double* part) {
    constexpr int ROW = BKC + 1;  // padded LDS row (double2): the 8 rows a read touches hit distinct banks
    __shared__ double2 sm[2 * BO * ROW];
    double2* As = sm;
    double2* Bs = sm + BO * ROW;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, ls = lane >> 3, lr = lane & 7;
    const int p = blockIdx.x, w = blockIdx.y;
    const int nt = (ns + BO - 1) / BO;
    const int s0 = (int)(blockIdx.z / nt) * BO, r0 = (int)(blockIdx.z % nt) * BO;
    const long long xa = (long long)p * kc, xb = xa + kc < npt ? xa + kc : npt;
    double are[4][4], aim[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) are[i][j] = aim[i][j] = 0.0;
    for (long long x0 = xa; x0 < xb; x0 += BKC) {
        // thread t stages point c = t % 64 of the rows t / 64 + 4 q
        const int c = t & 63;
        const long long x = x0 + c;
        const bool xin = x < xb;
        const double mx = xin ? m[x] : 0.0;
#pragma unroll
        for (int q = 0; q < BO / 4; ++q) {
            const int row = (t >> 6) + 4 * q;
            const int sr = s0 + row, rr = r0 + row;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            if (xin && sr < ns) {
                a = gval(G, ((long long)sr * nw + w) * npt + x);
                a.x *= mx;
                a.y *= mx;
            }
            if (xin && rr < ns) b = gval(G, ((long long)rr * nw + w) * npt + x);
            As[row * ROW + c] = a;
            Bs[row * ROW + c] = b;
        }
        __syncthreads();
        const int k0 = wave * (BKC / 4);
#pragma unroll 2
        for (int k = k0; k < k0 + BKC / 4; ++k) {
            double2 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[(ls + 8 * i) * ROW + k];
                b[i] = Bs[(lr + 8 * i) * ROW + k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    are[i][j] = fma(a[i].x, b[j].x, fma(-a[i].y, b[j].y, are[i][j]));
                    aim[i][j] = fma(a[i].x, b[j].y, fma(a[i].y, b[j].x, aim[i][j]));
                }
        }
        __syncthreads();
    }
    // the wavefronts' sums through LDS (the staging buffer, free after the
    // loop's last barrier), added in wavefront order
    double2* red = sm;  // [wave][entry i * 4 + j][lane]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[(wave * 16 + i * 4 + j) * 64 + lane] = make_double2(are[i][j], aim[i][j]);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = t + 256 * e, entry = idx >> 6, ln = idx & 63;
        const int s = s0 + (ln >> 3) + 8 * (entry >> 2), r = r0 + (ln & 7) + 8 * (entry & 3);
        double2 v = red[entry * 64 + ln];
#pragma unroll
        for (int q = 1; q < 4; ++q) {
            const double2 u = red[(q * 16 + entry) * 64 + ln];
            v.x += u.x;
            v.y += u.y;
        }
        if (s < ns && r < ns) {
            const long long o = ((((long long)p * nw + w) * ns + s) * ns + r) * 2;
            part[o] = v.x;
            part[o + 1] = v.y;
        }
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

// I[x] for 64 image points per block and ns <= MS surface points: wavefront
// q takes the chunk's frequencies q, q + 4, ...; per frequency it stages the
// data matrix (zero-padded to MS x MS) in its own LDS region, lane x forms
// y_s = sum_r d[s][r] conj(g_r) for all s at once (r outer, the MS sums in
// registers, d[s][r] read by the whole wavefront from one address) and adds
// Re sum_s conj(g_s) y_s; the four wavefronts' sums are added in order.
// accumulate: add to the image (later frequency chunks), else overwrite it.
template <typename R>
__global__ __launch_bounds__(256) void k_migrate_regs(const R* G, const double* d, int ns, int nw, long long npt,
                                                      MigW wc, int accumulate, double* img) {
    __shared__ double2 Ds[4][MS * MS];
    __shared__ double part[4][64];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const long long x = (long long)blockIdx.x * 64 + lane;
    const bool xin = x < npt;
    const long long xc = xin ? x : npt - 1;  // lanes past the end read a valid point and write nothing
    double acc = 0.0;
    const int nit = (wc.n + 3) / 4;
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
                Ds[wave][i] = v;
            }
        }
        __syncthreads();
        if (has) {
            double yre[MS], yim[MS];
#pragma unroll
            for (int sr = 0; sr < MS; ++sr) yre[sr] = yim[sr] = 0.0;
            // g_r two receivers ahead of its use (raw values, converted at use)
            const long long gofs = (long long)w * npt + xc, gstep = (long long)nw * npt;
            R p0x = G[2 * gofs], p0y = G[2 * gofs + 1];
            R p1x = (R)0, p1y = (R)0;
            if (ns > 1) {
                p1x = G[2 * (gofs + gstep)];
                p1y = G[2 * (gofs + gstep) + 1];
            }
            for (int rr = 0; rr < ns; ++rr) {
                const double2 g = make_double2((double)p0x, (double)p0y);  // conj(g_r) = (g.x, -g.y)
                p0x = p1x;
                p0y = p1y;
                if (rr + 2 < ns) {
                    const long long o = gofs + (long long)(rr + 2) * gstep;
                    p1x = G[2 * o];
                    p1y = G[2 * o + 1];
                }
#pragma unroll
                for (int sr = 0; sr < MS; ++sr) {
                    const double2 dv = Ds[wave][sr * MS + rr];
                    yre[sr] = fma(dv.x, g.x, fma(dv.y, g.y, yre[sr]));
                    yim[sr] = fma(dv.y, g.x, fma(-dv.x, g.y, yim[sr]));
                }
            }
            double aw = 0.0;  // Re sum_s conj(g_s) y_s
#pragma unroll
            for (int sr = 0; sr < MS; ++sr) {
                if (sr < ns) {
                    const double2 g = gval(G, ((long long)sr * nw + w) * npt + xc);
                    aw = fma(g.x, yre[sr], fma(g.y, yim[sr], aw));
                }
            }
            acc = fma(wc.w2[wl], aw, acc);
        }
        __syncthreads();
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && xin) {
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
        if (ns <= MS) {  // the sums over receivers in registers
            const unsigned blocks = (unsigned)((npt + 63) / 64);
            if (dtype == EGB_F64)
                k_migrate_regs<double><<<blocks, 256, 0, s>>>(static_cast<const double*>(G), d, ns, nw, npt, wc, acc,
                                                             image);
            else
                k_migrate_regs<float><<<blocks, 256, 0, s>>>(static_cast<const float*>(G), d, ns, nw, npt, wc, acc,
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
