// Eulerian Gaussian beam superposition (eqs. 25-27, 33-35).
//
// Pass 1 (k_beam_compact): every phase cell on (near) Gamma = {phi1 = 0,
// psi > 0} becomes one beam record in the list of its row (z = const) and of
// its column (x = const).  The take-off-angle measure comes from a smoothed
// delta of the signed distance d = phi1 / |grad phi1| (theta scaled by
// lambda = dx / dtheta, width h = 2 dx) and from the imaginary DRT part
// Im(C, B) = beta s (dn, dth_perp) per unit take-off angle.  Each record holds
//   pos (x or z of the cell), psi, p (p1 or p3 of eq. 7, or eq. 28's
//   coefficient for the lin=paper28 variant), M (traveltime Hessian along
//   the line, complex) and amp = w sqrt(v / C) dtheta (complex),
// w = cos^4 / (cos^4 + sin^4) of the ray angle for rows and 1 - w for columns,
// and sqrt(v / C) on the branch the ray carries: the principal root times
// (-1)^k, k the nearest whole number of turns between the phase plane (arg C
// continued along the ray) and the principal arg C.
// Cells whose line Hessian has Im(M) <= 0 give no record: a Gaussian beam
// decays away from its centre (the exact transport keeps Im(B conj(C)) > 0,
// a discrete field can lose it).  The gate psi > 0 is taken as psi above
// 1e-6 min(dx, dz) / v: the point-source data leave psi = 0 in exact
// arithmetic (+-1e-17 after rounding) on cells at the closest point of their
// ray to the source, and such a cell's wide beam must not hang on rounding.
// Pass 2 (k_beam_line): for every output cell and frequency,
//   G += amp exp(i omega T),  T = psi + p d + M d^2 / 2,
// skipping beams with omega Im(M) d^2 / 2 > 16, and G is scaled by i/(4 pi).
// A wavefront owns 64 output cells of one row (or column) and walks the
// line's records in key order, gathered 64 at a time into LDS and read by
// all lanes from one address; equally spaced frequencies rotate the term by
// exp(i step T) from one frequency to the next (chunks of 32 in FP32, else
// 16 per launch).  The depth march's beams (rows only) go through the
// same line sums after k_pbeam_compact.
#include <hip/hip_runtime.h>
#include <math.h>

#include "egb_device.h"
#include "egb_internal.h"

namespace egb {

// key: the record's source cell along its line (theta row times the line
// length plus the position), unique within a line; it fixes the order of
// the sum (see k_beam_order)
struct BeamRec {
    double psi, pos, p, Mre, Mim, are, aim, key;
};

size_t beam_record_bytes() { return sizeof(BeamRec); }

namespace {

__device__ __forceinline__ long long cidx2(const GridArgs& a, int f, int t, int ix, int iz) {
    return ((long long)(f * NT + t)) * a.nxz + (long long)ix * a.nz + iz;
}

template <typename T>
__device__ __forceinline__ double line_at(const T* base, long long st, int n, int idx) {
    if (idx < 0) return (1.0 - idx) * (double)base[0] + (double)idx * (double)base[st];
    if (idx > n - 1) {
        const int e = idx - (n - 1);
        return (e + 1.0) * (double)base[(long long)(n - 1) * st] - (double)e * (double)base[(long long)(n - 2) * st];
    }
    return (double)base[(long long)idx * st];
}

// 4th-order central difference of a line (ghosts as in the march)
template <typename T>
__device__ __forceinline__ double cd4(const T* base, long long st, int n, int i, double h) {
    return (line_at(base, st, n, i - 2) - 8.0 * line_at(base, st, n, i - 1) + 8.0 * line_at(base, st, n, i + 1) -
            line_at(base, st, n, i + 2)) /
           (12.0 * h);
}

// Eq. 28's linear phase coefficient for phase angle (s, c) = (sin, cos) and
// ray direction u = dx/dz: sqrt(s (s u^2 + 2 c u - s)) / (v (c + s u)), with
// the sign of p1 (that of s) restored and a negative radicand taken as 0;
// sin / v in isotropic media.  Columns use the mirror image.
__device__ __forceinline__ double lin28(double s, double c, double u, double v) {
    const double rad = s * (s * u * u + 2.0 * c * u - s);
    const double L = sqrt(fmax(rad, 0.0)) / (v * (c + s * u));
    return copysign(fabs(L), s);
}

__device__ __forceinline__ double delta_h(double d, double h) {
    return fabs(d) < h ? (1.0 + cos(M_PI * d / h)) / (2.0 * h) : 0.0;
}

template <typename R>
__global__ __launch_bounds__(256) void k_beam_compact(BeamArgs a) {
    const GridArgs& g = a.g;
    const int iz = blockIdx.x * 64 + threadIdx.x, ix = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (iz >= g.nz || ix >= g.nx) return;
    const long long S = g.stride, kb = (long long)k * g.nxz, c = kb + (long long)ix * g.nz + iz;
    const R* U = reinterpret_cast<const R*>(a.U);
    const double psi = reinterpret_cast<const double*>(U + EGB_PSI * S)[c];
    if (!(psi > 0.0)) return;
    const R* phi = U + EGB_PHI1 * S;
    const double fx = cd4(phi + kb + iz, g.nz, g.nx, ix, g.dx);
    const double fz = cd4(phi + kb + (long long)ix * g.nz, 1, g.nz, iz, g.dz);
    double ft;
    {
        const R* col = phi + (long long)ix * g.nz + iz;
        auto at = [&](int m) {
            int kk = k + m;
            kk += kk < 0 ? g.nth : 0;
            kk -= kk >= g.nth ? g.nth : 0;
            return (double)col[(long long)kk * g.nxz];
        };
        ft = (at(-2) - 8.0 * at(-1) + 8.0 * at(1) - at(2)) / (12.0 * g.dth);
    }
    const double f0 = (double)phi[c];
    const double lx = g.dx / g.dth, lz = g.dz / g.dth, hx = 2.0 * g.dx, hz = 2.0 * g.dz;
    const double drow = f0 / sqrt(fx * fx + (ft / lx) * (ft / lx));
    const double dcol = f0 / sqrt(fz * fz + (ft / lz) * (ft / lz));
    const bool arow = fabs(drow) < hx, acol = fabs(dcol) < hz;
    if (!arow && !acol) return;

    // local Hamiltonian (first derivatives of v are all that is needed)
    MediumPoint M;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t) M.m[f][t] = a.coeff2d[cidx2(g, f, t, ix, iz)];
    const double th = k * g.dth;
    const VJet J = qp_velocity(M, th);
    const VelA va = velocity_and_drt(J, th);
    double sn, cs;
    sincos_d(th, &sn, &cs);
    const double v = J.v, vx = J.g[0], vz = J.g[1], vt = J.g[2];
    // the gate psi > 0 taken as psi above a millionth of a cell's traveltime:
    // cells at the closest point of their ray to the source hold psi = 0 in
    // exact arithmetic and +-1e-17 after rounding
    if (!(psi > 1e-6 * fmin(g.dx, g.dz) / v)) return;
    const double Vt = va.V[2];
    const double sp = sqrt(va.V[0] * va.V[0] + va.V[1] * va.V[1]);
    const double hxr = va.V[0] / sp, hzr = va.V[1] / sp;  // ray direction (sin, cos of its angle)
    const double ex = hzr, ez = -hxr;                     // ray normal
    const double reC = (double)U[EGB_RE_C * S + c], imC = (double)U[EGB_IM_C * S + c];
    const double reB = (double)U[EGB_RE_B * S + c], imB = (double)U[EGB_IM_B * S + c];
    // Hessian of the beam traveltime in the ray frame:
    //   across the ray  Mn = [(e.p_theta) B + (e^T d_x p e) C] / C,
    //   mixed / along    from q = (dp/dtau)/|V| = -grad v / (v |V|).
    const double e_pth = ex * (cs / v - sn * vt / (v * v)) + ez * (-sn / v - cs * vt / (v * v));
    const double e_dxp_e = -(ex * sn + ez * cs) * (vx * ex + vz * ez) / (v * v);
    const double qx = -vx / (v * sp), qz = -vz / (v * sp);
    const double gq = hxr * qx + hzr * qz, eq = ex * qx + ez * qz;
    // Mn = (e_pth * B) / C + e_dxp_e
    const double den = reC * reC + imC * imC;
    const double BCre = (reB * reC + imB * imC) / den, BCim = (imB * reC - reB * imC) / den;
    const double Mnre = e_pth * BCre + e_dxp_e, Mnim = e_pth * BCim;
    // sqrt(v / C): the principal root, times (-1)^k on the ray's branch, k the
    // whole turns between the continued phase of C and its principal arg
    const double vCre = v * reC / den, vCim = -v * imC / den;
    const double mod = sqrt(vCre * vCre + vCim * vCim);
    double sqre = sqrt(0.5 * (mod + vCre));
    double sqim = sqrt(0.5 * fmax(mod - vCre, 0.0));
    sqim = vCim < 0.0 ? -sqim : sqim;
    {
        const double turns = rint(((double)U[EGB_PHASE * S + c] - atan2(imC, reC)) / 6.283185307179586476925286766559);
        if (fmod(fabs(turns), 2.0) == 1.0) {
            sqre = -sqre;
            sqim = -sqim;
        }
    }
    const double c4 = hzr * hzr * hzr * hzr, s4 = hxr * hxr * hxr * hxr, wrow = c4 / (c4 + s4);
    const double dn = imC, dtp = imB;
    BeamRec* rows = reinterpret_cast<BeamRec*>(a.rows);
    BeamRec* cols = reinterpret_cast<BeamRec*>(a.cols);
    if (arow && fabs(hzr) > 1e-4) {
        const double ds = dn * hxr / hzr, px = dn / hzr, pt = dtp + ds * Vt / sp;
        const double dthc = a.beta * delta_h(drow, hx) * lx * g.dx * g.dth / sqrt(px * px + lx * lx * pt * pt);
        const double w = wrow * dthc;
        BeamRec r;
        r.psi = psi;
        r.pos = g.x0 + (ix + 0.5) * g.dx;
        r.p = a.lin == EGB_LIN_PAPER28 ? lin28(sn, cs, va.V[0] / va.V[1], v) : sn / v;
        r.Mre = Mnre * hzr * hzr + 2.0 * eq * hxr * hzr + gq * hxr * hxr;
        r.Mim = Mnim * hzr * hzr;
        r.are = w * sqre;
        r.aim = w * sqim;
        r.key = (double)((long long)k * g.nx + ix);
        if (r.Mim > 0.0) {  // a Gaussian beam decays away from its centre
            const int slot = atomicAdd(&a.counts[iz], 1);
            if (slot < a.cap) rows[(long long)iz * a.cap + slot] = r;
        }
    }
    if (acol && fabs(hxr) > 1e-4) {
        const double ds = -dn * hzr / hxr, pz = -dn / hxr, pt = dtp + ds * Vt / sp;
        const double dthc = a.beta * delta_h(dcol, hz) * lz * g.dz * g.dth / sqrt(pz * pz + lz * lz * pt * pt);
        const double w = (1.0 - wrow) * dthc;
        BeamRec r;
        r.psi = psi;
        r.pos = g.z0 + (iz + 0.5) * g.dz;
        r.p = a.lin == EGB_LIN_PAPER28 ? lin28(cs, sn, va.V[1] / va.V[0], v) : cs / v;
        r.Mre = Mnre * hxr * hxr - 2.0 * eq * hxr * hzr + gq * hzr * hzr;
        r.Mim = Mnim * hxr * hxr;
        r.are = w * sqre;
        r.aim = w * sqim;
        r.key = (double)((long long)k * g.nz + iz);
        if (r.Mim > 0.0) {
            const int slot = atomicAdd(&a.counts[g.nz + ix], 1);
            if (slot < a.cap) cols[(long long)ix * a.cap + slot] = r;
        }
    }
}

constexpr int WCHUNK = 32;  // frequencies per launch of the FP32 recurrence (equally spaced, full chunk)
constexpr int WGEN = 16;    // frequencies per launch otherwise
struct Omegas {
    double w[WCHUNK];
    float tcut[WCHUNK];  // 16 / w[k] rounded to float: the window test of the FP32 recurrence
    double step;  // w[k] = w[0] + k step for every k < n when uniform
    int n, first, uniform;
};

// Sum over one row (ROW) or column list for a chunk of NCH frequencies.
// block: 64 lanes = 64 consecutive output cells along the line; grid.x: chunks
// along the line, grid.y: the line index.  FAST: FP32, NCH equally spaced
// frequencies (the recurrence of the weighted term); otherwise up to NCH
// frequencies, equally spaced or not.
template <typename R, bool ROW, int NCH, bool FAST>
__global__ __launch_bounds__(64) void k_beam_line(BeamArgs a, Omegas om, R* out) {
    static_assert(!FAST || sizeof(R) == 4, "the fast recurrence is the FP32 one");
    const GridArgs& g = a.g;
    const int line = blockIdx.y;
    const int j = blockIdx.x * 64 + threadIdx.x;  // position along the line
    const int nalong = ROW ? g.nx : g.nz;
    const bool valid = j < nalong;
    const double pos = ROW ? g.x0 + (j + 0.5) * g.dx : g.z0 + (j + 0.5) * g.dz;
    const int cnt = min(a.counts[ROW ? line : g.nz + line], a.cap);
    const BeamRec* recs = reinterpret_cast<const BeamRec*>(ROW ? a.rows : a.cols) + (long long)line * a.cap;
    const int* ord = a.order + ((ROW ? 0LL : (long long)g.nz) + line) * a.cap;
    R gre[NCH], gim[NCH];
#pragma unroll
    for (int w = 0; w < NCH; ++w) gre[w] = gim[w] = (R)0;
    const double two_pi = 6.283185307179586476925286766559, inv_two_pi = 1.0 / two_pi;
    // exp(i o T) = exp(-o Im T) (cos + i sin)(o Re T), the phase reduced mod 2 pi in double
    auto expi = [&](double o, double Tre, double Tim, R& er, R& ei) {
        const double ph = o * Tre;
        const double red = ph - two_pi * rint(ph * inv_two_pi);
        R sph, cph, mag;
        if constexpr (sizeof(R) == 4) {
            sincosf((float)red, &sph, &cph);
            mag = __expf(-(float)(o * Tim));
        } else {
            sincos(red, &sph, &cph);
            mag = exp(-o * Tim);
        }
        er = mag * cph;
        ei = mag * sph;
    };
    // the line's records in key order (the sum does not depend on the append
    // order), 64 at a time through LDS: lane l gathers record r0 + l, then
    // every lane reads each record from one LDS address
    __shared__ BeamRec srec[64];
    for (int r = 0; r < cnt; ++r) {
        if (r % 64 == 0) {
            __syncthreads();  // the previous chunk's reads are done
            if (r + (int)threadIdx.x < cnt) srec[threadIdx.x] = recs[ord[r + threadIdx.x]];
            __syncthreads();
        }
        const BeamRec b = srec[r % 64];
        const double d = pos - b.pos;
        const double Tre = b.psi + b.p * d + 0.5 * b.Mre * d * d;
        const double Tim = 0.5 * b.Mim * d * d;
        if constexpr (FAST) {
            // FP32, equally spaced frequencies: z_k = A exp(i w_k T) =
            // z_0 exp(i step T)^k, one complex rotation and one add per
            // frequency; a term enters while Im T <= 16 / w_k (float test:
            // a term at the edge of the window is e^-16 of its beam)
            R er, ei, dr, di;
            expi(om.w[0], Tre, Tim, er, ei);
            expi(om.step, Tre, Tim, dr, di);
            R zr = (R)b.are * er - (R)b.aim * ei, zi = (R)b.are * ei + (R)b.aim * er;
            const float tf = (float)Tim;
#pragma unroll
            for (int w = 0; w < NCH; ++w) {
                if (tf <= om.tcut[w]) {
                    gre[w] += zr;
                    gim[w] += zi;
                }
                const R nr = zr * dr - zi * di, ni = zr * di + zi * dr;
                zr = nr;
                zi = ni;
            }
            continue;
        } else if (om.uniform) {
            // equally spaced frequencies: exp(i w_k T) = exp(i w_0 T) exp(i step T)^k,
            // two exponentials per beam and output instead of one per frequency
            R er, ei, dr, di;
            expi(om.w[0], Tre, Tim, er, ei);
            expi(om.step, Tre, Tim, dr, di);
#pragma unroll
            for (int w = 0; w < NCH; ++w) {
                if (w < om.n) {
                    if (om.w[w] * Tim <= 16.0) {
                        gre[w] += (R)b.are * er - (R)b.aim * ei;
                        gim[w] += (R)b.are * ei + (R)b.aim * er;
                    }
                    const R nr = er * dr - ei * di;
                    ei = er * di + ei * dr;
                    er = nr;
                }
            }
            continue;
        }
#pragma unroll
        for (int w = 0; w < NCH; ++w) {
            if (w < om.n) {
                const double o = om.w[w];
                const double decay = o * Tim;
                if (decay <= 16.0) {
                    // exp(i o T) = exp(-o Im T) (cos + i sin)(o Re T); phase reduced mod 2 pi in double
                    const double ph = o * Tre;
                    const double red = ph - two_pi * rint(ph * inv_two_pi);
                    R sph, cph;
                    if constexpr (sizeof(R) == 4) {
                        sincosf((float)red, &sph, &cph);
                        const R mag = __expf(-(float)decay);
                        const R er = mag * cph, ei = mag * sph;
                        gre[w] += (R)b.are * er - (R)b.aim * ei;
                        gim[w] += (R)b.are * ei + (R)b.aim * er;
                    } else {
                        sincos(red, &sph, &cph);
                        const R mag = exp(-decay);
                        const R er = mag * cph, ei = mag * sph;
                        gre[w] += b.are * er - b.aim * ei;
                        gim[w] += b.are * ei + b.aim * er;
                    }
                }
            }
        }
    }
    if (!valid) return;
    const int ix = ROW ? j : line, iz = ROW ? line : j;
    // W = i / (4 pi): (gre + i gim) * i / (4 pi) = (-gim + i gre) / (4 pi)
    const R s = (R)(1.0 / (4.0 * M_PI));
#pragma unroll
    for (int w = 0; w < NCH; ++w) {
        if (w < om.n) {
            const long long o = (((long long)(om.first + w) * g.nx + ix) * g.nz + iz) * 2;
            if (ROW) {
                out[o] = -gim[w] * s;
                out[o + 1] = gre[w] * s;
            } else {
                out[o] += -gim[w] * s;
                out[o + 1] += gre[w] * s;
            }
        }
    }
}

// The order of one line's records by key: record r goes to position
// #{s : key_s < key_r} (keys are unique within a line), so every run sums a
// line in the same order whatever order the compaction's atomic appends took.
// grid: (ORDER_BLOCKS, lines), 256 threads; the keys of the line pass through
// LDS 256 at a time.
constexpr int ORDER_BLOCKS = 16;
template <bool ROW>
__global__ __launch_bounds__(256) void k_beam_order(BeamArgs a) {
    __shared__ double ks[256];
    const int line = blockIdx.y;
    const int cnt = min(a.counts[ROW ? line : a.g.nz + line], a.cap);
    const BeamRec* recs = reinterpret_cast<const BeamRec*>(ROW ? a.rows : a.cols) + (long long)line * a.cap;
    int* ord = a.order + ((ROW ? 0LL : (long long)a.g.nz) + line) * a.cap;
    for (int r0 = blockIdx.x * 256; r0 < cnt; r0 += gridDim.x * 256) {  // block-uniform
        const int r = r0 + (int)threadIdx.x;
        const double kr = r < cnt ? recs[r].key : 0.0;
        int rank = 0;
        for (int s0 = 0; s0 < cnt; s0 += 256) {
            __syncthreads();
            ks[threadIdx.x] = s0 + (int)threadIdx.x < cnt ? recs[s0 + threadIdx.x].key : INFINITY;
            __syncthreads();
            for (int j = 0; j < 256; ++j) rank += ks[j] < kr;
        }
        if (r < cnt) ord[rank] = r;
    }
}

__global__ void k_fill_i32(int* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// *out = max(p[0 .. n)), one block of 256 threads
__global__ __launch_bounds__(256) void k_max_i32(const int* p, int n, int* out) {
    __shared__ int part[4];
    int m = 0;
    for (int i = threadIdx.x; i < n; i += 256) m = max(m, p[i]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = max(max(part[0], part[1]), max(part[2], part[3]));
}

// qP polarisation (eqs. 4, 31-32) for table values m = (a11, a33, a13 + a55,
// a55, nu) and phase angle theta: the unit eigenvector of the 2x2
// Christoffel matrix for the larger eigenvalue, found in the symmetry frame
// (phase angle theta - nu) from the longer of its two null-space forms,
// turned back by nu and signed along the phase direction.
__device__ __forceinline__ void qp_polarization(const double (&m)[NF], double theta, double& gx, double& gz) {
    double n1, n3;
    sincos_d(theta - m[4], &n1, &n3);
    const double g11 = m[0] * n1 * n1 + m[3] * n3 * n3, g33 = m[3] * n1 * n1 + m[1] * n3 * n3;
    const double g13 = m[2] * n1 * n3;
    const double G = 0.5 * (g11 + g33 + sqrt((g11 - g33) * (g11 - g33) + 4.0 * g13 * g13));
    const double a1 = G - g33, a3 = g13, b1 = g13, b3 = G - g11;
    const bool first = a1 * a1 + a3 * a3 >= b1 * b1 + b3 * b3;
    double vx = first ? a1 : b1, vz = first ? a3 : b3;
    double nv = sqrt(vx * vx + vz * vz);
    if (nv == 0.0) {
        vx = n1;
        vz = n3;
        nv = 1.0;
    }
    vx /= nv;
    vz /= nv;
    if (vx * n1 + vz * n3 < 0.0) {
        vx = -vx;
        vz = -vz;
    }
    double sn, cn;
    sincos_d(m[4], &sn, &cn);
    gx = vx * cn + vz * sn;
    gz = -vx * sn + vz * cn;
}

// Beam records of the depth march for a surface source at xs: thread
// (x, theta, level n >= 1).  A cell whose transported take-off angle lies
// inside the aperture and that is near Gamma = {X = xs} (signed distance d
// = (X - xs) / |grad X|, theta scaled by lambda = dx / dtheta, |d| < 2 dx)
// becomes a row-n record with the take-off-angle measure
// delta_h(d) |det d(X, vartheta)/d(x, theta)| / |grad X| dx dtheta, the row
// Hessian of the phase-space beam sum, traveltime tau + p_s (X - xs) (the ray
// through the cell starts at X) and amplitude sqrt(v / C) sqrt(u1 / s) / s:
// the depth march starts a beam with C(0) = u1 = cos + sin u, the point-source
// data with C(0) = s, both for the medium frozen at the source.
template <typename R>
__device__ __forceinline__ void pbeam_cell(const PBeamArgs& a, int ix, int k, int n, bool record) {
    const long long P = a.P, c = (long long)k * a.nx + ix;
    const R* L = reinterpret_cast<const R*>(static_cast<const char*>(a.levels) + (size_t)n * a.level_bytes);
    const double tau = reinterpret_cast<const double*>(L + 7 * P)[c];
    if (!(tau > 0.0)) return;
    const R* X = L;           // plane 0
    const R* T = L + P;       // plane 1: vartheta
    const double Xx = cd4(X + (long long)k * a.nx, 1, a.nx, ix, a.dx);
    const double Xt = cd4(X + ix, a.nx, a.nth, k, a.dth);
    const double Tx = cd4(T + (long long)k * a.nx, 1, a.nx, ix, a.dx);
    const double Tt = cd4(T + ix, a.nx, a.nth, k, a.dth);
    const double lam = a.dx / a.dth, h = 2.0 * a.dx;
    const double gX = sqrt(Xx * Xx + (Xt / lam) * (Xt / lam));
    const double Xc = (double)X[c];
    const double d = (Xc - a.xs) / gX;
    if (!(fabs(d) < h)) return;
    const double vt0 = (double)T[c];  // take-off angle; outside the aperture: edge data, not a ray
    if (!(fabs(vt0) < a.theta_max)) return;
    if (!record) {  // the gate only: the cell is a beam candidate of the block
        a.cand[atomicAdd(a.ncand, 1)] = k * a.nx + ix;
        return;
    }
    const double meas = delta_h(d, h) * fabs(Xx * Tt - Xt * Tx) / gX * a.dx * a.dth;
    // local phase-velocity jet and ray direction at (x, z_n, theta)
    MediumPoint M;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t) M.m[f][t] = a.coeff2d[cidx2(a.g, f, t, ix, n)];
    const double th = -a.theta_max + (k + 0.5) * a.dth;
    const VJet J = qp_velocity(M, th);
    const VelA va = velocity_and_drt(J, th);
    double sn, cs;
    sincos_d(th, &sn, &cs);
    const double v = J.v, vx = J.g[0], vz = J.g[1], vt = J.g[2];
    const double sp = sqrt(va.V[0] * va.V[0] + va.V[1] * va.V[1]);
    const double hxr = va.V[0] / sp, hzr = va.V[1] / sp;
    const double ex = hzr, ez = -hxr;
    const double reC = (double)L[2 * P + c], imC = (double)L[3 * P + c];
    const double reB = (double)L[4 * P + c], imB = (double)L[5 * P + c];
    const double e_pth = ex * (cs / v - sn * vt / (v * v)) + ez * (-sn / v - cs * vt / (v * v));
    const double e_dxp_e = -(ex * sn + ez * cs) * (vx * ex + vz * ez) / (v * v);
    const double qx = -vx / (v * sp), qz = -vz / (v * sp);
    const double gq = hxr * qx + hzr * qz, eq = ex * qx + ez * qz;
    const double den = reC * reC + imC * imC;
    const double BCre = (reB * reC + imB * imC) / den, BCim = (imB * reC - reB * imC) / den;
    const double Mnre = e_pth * BCre + e_dxp_e, Mnim = e_pth * BCim;
    const double vCre = v * reC / den, vCim = -v * imC / den;
    const double mod = sqrt(vCre * vCre + vCim * vCim);
    double sqre = sqrt(0.5 * (mod + vCre));
    double sqim = sqrt(0.5 * fmax(mod - vCre, 0.0));
    sqim = vCim < 0.0 ? -sqim : sqim;
    {
        // the branch the ray carries: (-1)^k, k full turns between the continuous
        // phase Phi of C and arg C (the KMAH phase)
        const double turns = rint(((double)L[6 * P + c] - atan2(imC, reC)) / 6.283185307179586476925286766559);
        if (fmod(fabs(turns), 2.0) == 1.0) {
            sqre = -sqre;
            sqim = -sqim;
        }
    }
    // source normalisation at the take-off angle (medium frozen at the source)
    MediumPoint Ms;
    {
        // bilinear in the table at (xs, depth of level 0)
        const double fx = (a.xs - a.g.x0) / a.dx - 0.5;
        const int sx = min(max((int)floor(fx), 0), a.nx - 2);
        const double tx = fmin(fmax(fx - sx, 0.0), 1.0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int t = 0; t < NT; ++t) Ms.m[f][t] = 0.0;
            Ms.m[f][0] = (1.0 - tx) * a.coeff2d[cidx2(a.g, f, 0, sx, 0)] + tx * a.coeff2d[cidx2(a.g, f, 0, sx + 1, 0)];
        }
    }
    const VJet Js = qp_velocity(Ms, vt0);
    const VelA vs = velocity_and_drt(Js, vt0);
    double s0, c0;
    sincos_d(vt0, &s0, &c0);
    const double u1 = c0 + s0 * vs.V[0] / vs.V[1];
    const double Wt = Ms.m[1][0] / (Js.v * Js.v);
    const double ssrc = cbrt((sqrt(Js.v) / Wt) * (sqrt(Js.v) / Wt));
    double w = sqrt(u1 / ssrc) / ssrc * meas;
    if (a.comp >= 0) {  // Green's tensor component (i, k): g_i at the cell, g_k at the source
        double mr[NF], ms[NF], grx, grz, gsx, gsz;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            mr[f] = M.m[f][0];
            ms[f] = Ms.m[f][0];
        }
        qp_polarization(mr, th, grx, grz);
        qp_polarization(ms, vt0, gsx, gsz);
        w *= ((a.comp >> 1) ? grz : grx) * ((a.comp & 1) ? gsz : gsx);
    }
    BeamRec r;
    r.psi = tau + s0 / Js.v * (Xc - a.xs);
    r.pos = a.g.x0 + (ix + 0.5) * a.dx;
    r.p = a.lin == EGB_LIN_PAPER28 ? lin28(sn, cs, va.V[0] / va.V[1], v) : sn / v;
    r.Mre = Mnre * hzr * hzr + 2.0 * eq * hxr * hzr + gq * hxr * hxr;
    r.Mim = Mnim * hzr * hzr;
    if (a.drt == EGB_DRT_PAPER23) {
        // lateral frame: the row Hessian is B / C itself, and the lateral
        // displacement is the normal one over g_z (both started at u1), so
        // sqrt(v / C_normal) = sqrt(v / C) sqrt(g_z0 / g_z)
        r.Mre = BCre;
        r.Mim = BCim;
        w *= sqrt((vs.V[1] / sqrt(vs.V[0] * vs.V[0] + vs.V[1] * vs.V[1])) / hzr);
    }
    r.are = w * sqre;
    r.aim = w * sqim;
    r.key = (double)c;
    if (!(r.Mim > 0.0)) return;  // not a Gaussian beam (grows away from its centre)
    const int slot = atomicAdd(&a.counts[n], 1);
    if (slot < a.cap) reinterpret_cast<BeamRec*>(a.rows)[(long long)n * a.cap + slot] = r;
}

// Block: 64 x 8 cells (x, theta) of level n.  Every thread evaluates the gate
// of its cell and the block's candidates are gathered in LDS; then one thread
// per candidate forms the record, so the long FP64 path runs on full
// wavefronts instead of once in every wavefront that holds a candidate (a
// few cells per theta row lie near Gamma).  The append order does not
// matter: the line sums take the records in key order.
template <typename R>
__global__ __launch_bounds__(512) void k_pbeam_compact(PBeamArgs a) {
    __shared__ int cand[512];
    __shared__ int ncand;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const int ix = blockIdx.x * 64 + threadIdx.x, k = blockIdx.y * 8 + threadIdx.y, n = blockIdx.z + 1;
    if (tid == 0) ncand = 0;
    __syncthreads();
    PBeamArgs g = a;
    g.cand = cand;
    g.ncand = &ncand;
    if (ix < a.nx && k < a.nth && n < a.nz) pbeam_cell<R>(g, ix, k, n, false);
    __syncthreads();
    if (tid < ncand) {
        const int c = cand[tid];
        pbeam_cell<R>(a, c % a.nx, c / a.nx, n, true);
    }
}

}  // namespace

hipError_t launch_pbeam_compact(const PBeamArgs& a, int dtype, hipStream_t s) {
    const int nl = a.g.nz + a.g.nx;
    k_fill_i32<<<(nl + 255) / 256, 256, 0, s>>>(a.counts, nl);
    if (a.nz < 2) return hipGetLastError();
    const dim3 grid((a.nx + 63) / 64, (a.nth + 7) / 8, a.nz - 1), block(64, 8);
    if (dtype == EGB_F64)
        k_pbeam_compact<double><<<grid, block, 0, s>>>(a);
    else
        k_pbeam_compact<float><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_beam_compact(const BeamArgs& a, int dtype, hipStream_t s) {
    const int nl = a.g.nz + a.g.nx;
    k_fill_i32<<<(nl + 255) / 256, 256, 0, s>>>(a.counts, nl);
    const dim3 grid((a.g.nz + 63) / 64, (a.g.nx + 3) / 4, a.g.nth), block(64, 4);
    if (dtype == EGB_F64)
        k_beam_compact<double><<<grid, block, 0, s>>>(a);
    else
        k_beam_compact<float><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_max_i32(const int* p, int n, int* out, hipStream_t s) {
    k_max_i32<<<1, 256, 0, s>>>(p, n, out);
    return hipGetLastError();
}

hipError_t launch_beam_sum(const BeamArgs& a, int dtype, const double* omegas, int nw, void* out, hipStream_t s) {
    k_beam_order<true><<<dim3(ORDER_BLOCKS, a.g.nz), 256, 0, s>>>(a);
    if (!a.rows_only) k_beam_order<false><<<dim3(ORDER_BLOCKS, a.g.nx), 256, 0, s>>>(a);
    // a chunk of equally spaced frequencies (to 1e-12 of the largest)
    auto chunk = [&](int w0, int n) {
        Omegas om;
        om.n = n;
        om.first = w0;
        for (int w = 0; w < WCHUNK; ++w) om.w[w] = w < om.n ? omegas[w0 + w] : 0.0;
        for (int w = 0; w < WCHUNK; ++w) om.tcut[w] = w < om.n ? (float)(16.0 / om.w[w]) : 0.0f;
        om.step = om.n > 1 ? (om.w[om.n - 1] - om.w[0]) / (om.n - 1) : 0.0;
        om.uniform = om.n > 1 && om.step > 0.0;
        for (int w = 0; w < om.n && om.uniform; ++w)
            if (fabs(om.w[w] - (om.w[0] + w * om.step)) > 1e-12 * fabs(om.w[om.n - 1])) om.uniform = 0;
        return om;
    };
    const dim3 grow((a.g.nx + 63) / 64, a.g.nz), gcol((a.g.nz + 63) / 64, a.g.nx);
    for (int w0 = 0; w0 < nw;) {
        if (dtype == EGB_F32 && nw - w0 >= WCHUNK) {
            const Omegas om = chunk(w0, WCHUNK);
            if (om.uniform) {  // FP32 recurrence over a full chunk
                k_beam_line<float, true, WCHUNK, true><<<grow, 64, 0, s>>>(a, om, (float*)out);
                if (!a.rows_only) k_beam_line<float, false, WCHUNK, true><<<gcol, 64, 0, s>>>(a, om, (float*)out);
                w0 += WCHUNK;
                continue;
            }
        }
        const Omegas om = chunk(w0, nw - w0 < WGEN ? nw - w0 : WGEN);
        if (dtype == EGB_F64) {
            k_beam_line<double, true, WGEN, false><<<grow, 64, 0, s>>>(a, om, (double*)out);
            if (!a.rows_only) k_beam_line<double, false, WGEN, false><<<gcol, 64, 0, s>>>(a, om, (double*)out);
        } else {
            k_beam_line<float, true, WGEN, false><<<grow, 64, 0, s>>>(a, om, (float*)out);
            if (!a.rows_only) k_beam_line<float, false, WGEN, false><<<gcol, 64, 0, s>>>(a, om, (float*)out);
        }
        w0 += om.n;
    }
    return hipGetLastError();
}

}  // namespace egb
