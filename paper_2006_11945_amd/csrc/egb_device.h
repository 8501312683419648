// Device-side building blocks shared by the libegb kernels (gfx950).
//
//  * qP phase velocity of a 2D TTI medium and its derivatives up to second
//    order in (x, z, theta), by an explicit chain rule through the
//    Christoffel eigenvalue (eqs. 3-5, 7);
//  * the Liouville velocity (eqs. 8-9, 12) and the ray-normal dynamic ray
//    tracing matrix (eq. 21 read in the ray-normal frame);
//  * the WENO5 Hamilton-Jacobi one-sided derivative used by the march.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace egb {

constexpr int NF = 5;  // a11, a33, b = a13 + a55, a55, nu
constexpr int NT = 6;  // f, f_x, f_z, f_xx, f_xz, f_zz

// Medium values at one (x, z) point: m[field][taylor].
struct MediumPoint {
    double m[NF][NT];
};

// Phase velocity and derivatives: gradient index 0 = x, 1 = z, 2 = theta;
// Hessian stored symmetric as h[a][b].
struct VJet {
    double v;
    double g[3];
    double h[3][3];
};

__device__ inline void sincos_d(double a, double* s, double* c) { sincos(a, s, c); }

// Second-order derivatives of F(m(x), phi(x, theta)) = sum_m m * kappa_m(phi),
// phi = theta - nu(x), given F's phi-derivatives Fp, Fpp and the medium sums
//   Fm[i]   = sum_m m_i kappa_m,  Fmm[i][j] = sum_m m_ij kappa_m,
//   Fmp[i]  = sum_m m_i kappa_m'.
struct Lin2 {
    double f, g[3], h[3][3];
};

__device__ inline Lin2 chain_linear(double F, double Fp, double Fpp, const double Fm[2], const double Fmm[2][2],
                                    const double Fmp[2], const double nu[2], const double nuh[2][2]) {
    Lin2 r;
    r.f = F;
    for (int i = 0; i < 2; ++i) r.g[i] = Fm[i] - Fp * nu[i];
    r.g[2] = Fp;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            r.h[i][j] = Fmm[i][j] - Fmp[i] * nu[j] - Fmp[j] * nu[i] + Fpp * nu[i] * nu[j] - Fp * nuh[i][j];
    for (int i = 0; i < 2; ++i) {
        r.h[i][2] = Fmp[i] - Fpp * nu[i];
        r.h[2][i] = r.h[i][2];
    }
    r.h[2][2] = Fpp;
    return r;
}

// sqrt of a positive quantity carried with gradient and Hessian.
__device__ inline Lin2 sqrt2(const Lin2& E) {
    Lin2 r;
    r.f = sqrt(E.f);
    double i2 = 0.5 / r.f;
    for (int a = 0; a < 3; ++a) r.g[a] = E.g[a] * i2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) r.h[a][b] = (E.h[a][b] - 2.0 * r.g[a] * r.g[b]) * i2;
    return r;
}

// qP phase velocity v(x, z, theta) = sqrt(G), G the larger eigenvalue of the
// 2x2 Christoffel matrix for the unit phase direction at angle phi = theta - nu
// from the symmetry axis:
//   G = (P + sqrt(Q^2 + R^2)) / 2,
//   P = (a11 + a55) sin^2 + (a33 + a55) cos^2,  Q = (a11 - a55) sin^2 - (a33 - a55) cos^2,
//   R = 2 b sin cos.
__device__ inline VJet qp_velocity(const MediumPoint& M, double theta) {
    const double* a11 = M.m[0];
    const double* a33 = M.m[1];
    const double* b = M.m[2];
    const double* a55 = M.m[3];
    const double* nuT = M.m[4];
    double sp, cp;
    sincos_d(theta - nuT[0], &sp, &cp);
    double S2 = sp * sp, C2 = cp * cp, s2 = 2.0 * sp * cp, c2 = C2 - S2;
    double nu[2] = {nuT[1], nuT[2]};
    double nuh[2][2] = {{nuT[3], nuT[4]}, {nuT[4], nuT[5]}};
    // first / second spatial derivative slots of field f: d[f][i], dd[f][i][j]
    auto d1 = [&](const double* f, int i) { return f[1 + i]; };
    auto d2 = [&](const double* f, int i, int j) { return (i == j) ? f[3 + 2 * i] : f[4]; };

    double Pm[2], Pmm[2][2], Pmp[2], Qm[2], Qmm[2][2], Qmp[2], Rm[2], Rmm[2][2], Rmp[2];
    for (int i = 0; i < 2; ++i) {
        Pm[i] = d1(a11, i) * S2 + d1(a33, i) * C2 + d1(a55, i);
        Qm[i] = d1(a11, i) * S2 - d1(a33, i) * C2 + d1(a55, i) * c2;
        Rm[i] = d1(b, i) * s2;
        Pmp[i] = (d1(a11, i) - d1(a33, i)) * s2;
        Qmp[i] = (d1(a11, i) + d1(a33, i) - 2.0 * d1(a55, i)) * s2;
        Rmp[i] = 2.0 * d1(b, i) * c2;
        for (int j = 0; j < 2; ++j) {
            Pmm[i][j] = d2(a11, i, j) * S2 + d2(a33, i, j) * C2 + d2(a55, i, j);
            Qmm[i][j] = d2(a11, i, j) * S2 - d2(a33, i, j) * C2 + d2(a55, i, j) * c2;
            Rmm[i][j] = d2(b, i, j) * s2;
        }
    }
    double P = (a11[0] + a55[0]) * S2 + (a33[0] + a55[0]) * C2;
    double Q = (a11[0] - a55[0]) * S2 - (a33[0] - a55[0]) * C2;
    double R = b[0] * s2;
    double Pp = (a11[0] - a33[0]) * s2, Ppp = 2.0 * (a11[0] - a33[0]) * c2;
    double Qp = (a11[0] + a33[0] - 2.0 * a55[0]) * s2, Qpp = 2.0 * (a11[0] + a33[0] - 2.0 * a55[0]) * c2;
    double Rp = 2.0 * b[0] * c2, Rpp = -4.0 * b[0] * s2;

    Lin2 LP = chain_linear(P, Pp, Ppp, Pm, Pmm, Pmp, nu, nuh);
    Lin2 LQ = chain_linear(Q, Qp, Qpp, Qm, Qmm, Qmp, nu, nuh);
    Lin2 LR = chain_linear(R, Rp, Rpp, Rm, Rmm, Rmp, nu, nuh);

    Lin2 E;  // Q^2 + R^2
    E.f = LQ.f * LQ.f + LR.f * LR.f;
    for (int a = 0; a < 3; ++a) E.g[a] = 2.0 * (LQ.f * LQ.g[a] + LR.f * LR.g[a]);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            E.h[a][c] = 2.0 * (LQ.g[a] * LQ.g[c] + LQ.f * LQ.h[a][c] + LR.g[a] * LR.g[c] + LR.f * LR.h[a][c]);
    Lin2 D = sqrt2(E);
    Lin2 G;
    G.f = 0.5 * (LP.f + D.f);
    for (int a = 0; a < 3; ++a) G.g[a] = 0.5 * (LP.g[a] + D.g[a]);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G.h[a][c] = 0.5 * (LP.h[a][c] + D.h[a][c]);
    Lin2 v = sqrt2(G);
    VJet out;
    out.v = v.f;
    for (int a = 0; a < 3; ++a) out.g[a] = v.g[a];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) out.h[a][c] = v.h[a][c];
    return out;
}

// Liouville velocity and ray-normal DRT matrix at phase angle theta.
//   group velocity  Vg = v n + v_theta m,   n = (sin, cos), m = dn/dtheta = (cos, -sin);
//   angle rate      V_t = -(grad v . m)      (dp/dtau = -grad_x v / v at fixed theta);
// Perturbation (dn, dt) normal to the ray: position offset dn along
// e = (gz, -gx) (unit, perpendicular to Vg) and angle offset dt with the
// along-ray drift removed.  Writing dV/dy for the phase-space Jacobian,
//   A11 = e.(Jx e), A12 = e.dVg/dtheta,
//   A21 = e.grad V_t - (gh.(Jx e) + phidot) V_t/|Vg|,
//   A22 = dV_t/dtheta - (gh.dVg/dtheta) V_t/|Vg|,
// gh = Vg/|Vg|, Jx = d Vg / d(x, z), phidot the turning rate of gh.
struct VelA {
    double V[3];
    double A[4];
};

__device__ inline VelA velocity_and_drt(const VJet& J, double theta) {
    double sn, cs;
    sincos_d(theta, &sn, &cs);
    const double v = J.v, vx = J.g[0], vz = J.g[1], vt = J.g[2];
    const double vxx = J.h[0][0], vxz = J.h[0][1], vzz = J.h[1][1];
    const double vxt = J.h[0][2], vzt = J.h[1][2], vtt = J.h[2][2];
    VelA r;
    const double gx_ = v * sn + vt * cs, gz_ = v * cs - vt * sn;
    const double Vt = -(vx * cs - vz * sn);
    r.V[0] = gx_;
    r.V[1] = gz_;
    r.V[2] = Vt;
    const double speed = sqrt(gx_ * gx_ + gz_ * gz_), inv = 1.0 / speed;
    const double hx = gx_ * inv, hz = gz_ * inv;  // unit ray direction
    const double ex = hz, ez = -hx;               // unit normal
    // d Vg / dx and d Vg / dz at fixed theta
    const double dVx_dx = vx * sn + vxt * cs, dVx_dz = vz * sn + vzt * cs;
    const double dVz_dx = vx * cs - vxt * sn, dVz_dz = vz * cs - vzt * sn;
    // d Vg / dtheta = (v + v_tt) m
    const double w = v + vtt;
    const double dVx_dt = w * cs, dVz_dt = -w * sn;
    // Jx applied to e
    const double Je_x = dVx_dx * ex + dVx_dz * ez, Je_z = dVz_dx * ex + dVz_dz * ez;
    // dVg/dtau along the ray = Jx Vg + dVg/dtheta V_t
    const double dgx = dVx_dx * gx_ + dVx_dz * gz_ + dVx_dt * Vt;
    const double dgz = dVz_dx * gx_ + dVz_dz * gz_ + dVz_dt * Vt;
    const double phidot = (ex * dgx + ez * dgz) * inv;
    // grad of V_t and its theta derivative
    const double dVt_dx = -(vxx * cs - vxz * sn), dVt_dz = -(vxz * cs - vzz * sn);
    const double dVt_dt = vx * sn + vz * cs - (vxt * cs - vzt * sn);
    r.A[0] = ex * Je_x + ez * Je_z;
    r.A[1] = ex * dVx_dt + ez * dVz_dt;
    r.A[2] = ex * dVt_dx + ez * dVt_dz - (hx * Je_x + hz * Je_z + phidot) * Vt * inv;
    r.A[3] = dVt_dt - (hx * dVx_dt + hz * dVz_dt) * Vt * inv;
    return r;
}

// ---------------------------------------------------------------- WENO5
// One-sided WENO5 Hamilton-Jacobi derivative, undivided (derivative times
// the spacing), from the five differences v1..v5 ordered away from the
// upwind side, eps = 1e-6 max v^2.  Rewritten with the second differences
// s_j = v_{j+1} - v_j (j = 1..4):
//   W = v3 + (1/6) sum_k omega_k r_k,  r = (5 s2 - 2 s1, s2 + 2 s3, 4 s3 - s4),
//   beta_k = 13/12 t_k^2 + 1/4 u_k^2,  t = (s2 - s1, s3 - s2, s4 - s3),
//                                      u = (3 s2 - s1, s2 + s3, s4 - 3 s3),
//   omega_k proportional to d_k / (eps + beta_k)^2,  d = (0.1, 0.6, 0.3),
// which is the textbook form (q_k - v3 = r_k / 6) with fewer operations.
// With b_k = 4 (eps + beta_k) the weights relative to omega_0 are
// (1, 6 (b0/b1)^2, 3 (b0/b2)^2): every b_k lies between 4 eps and a few tens
// of max v^2, so each ratio lies within about 1e-7 .. 1e7 whatever the scale
// of v (no rescaling), at the cost of three reciprocals.  eps is kept at
// least the smallest normal number, so that all differences zero give W = 0.
template <typename R>
__device__ __forceinline__ R weno5(R v1, R v2, R v3, R v4, R v5) {
    constexpr bool F = sizeof(R) == 4;
    const R m = fmax(fmax(fmax(fmax(fabs(v1), fabs(v2)), fabs(v3)), fabs(v4)), fabs(v5));
    auto rcp = [](R x) {
        if constexpr (F) return __builtin_amdgcn_rcpf(x);
        else return (R)1 / x;
    };
    const R eps4 = fmax(((R)4e-6 * m) * m, F ? (R)1.17549435e-38 : (R)2.2250738585072014e-308);
    const R s1 = v2 - v1, s2 = v3 - v2, s3 = v4 - v3, s4 = v5 - v4;
    const R t0 = s2 - s1, u0 = (R)3 * s2 - s1;
    const R t1 = s3 - s2, u1 = s2 + s3;
    const R t2 = s4 - s3, u2 = s4 - (R)3 * s3;
    constexpr R c13 = (R)(13.0 / 3.0);
    const R b0 = (c13 * t0) * t0 + (u0 * u0 + eps4);
    const R b1 = (c13 * t1) * t1 + (u1 * u1 + eps4);
    const R b2 = (c13 * t2) * t2 + (u2 * u2 + eps4);
    const R q1 = b0 * rcp(b1), q2 = b0 * rcp(b2);
    const R w1 = ((R)6 * q1) * q1, w2 = ((R)3 * q2) * q2;
    const R r0 = (R)5 * s2 - (R)2 * s1, r1 = s2 + (R)2 * s3, r2 = (R)4 * s3 - s4;
    const R num = r0 + w1 * r1 + w2 * r2;
    const R den = ((R)1 + w1) + w2;
    return v3 + (num * rcp(den)) * (R)(1.0 / 6.0);
}

// WENO5 value (undivided) and its gradient g[k] = dW/dv_{k+1}, by reverse-mode
// differentiation of the formula above (the same weights relative to
// omega_0, no rescaling): with omega_k = w_k / D, Rb = sum omega_k r_k and
// W = v3 + Rb / 6,
//   dW/db_k = -omega_k (r_k - Rb) / (3 b_k)   (b_k enters squared in w),
//   dW/dr_k = omega_k / 6,  dW/deps4 = sum_k dW/db_k,
// then back through t, u, r, s to v; eps4 = 4e-6 v_J^2 for the first entry J
// of largest magnitude (its floor, the smallest normal number, has no
// derivative).  When all differences vanish W and the gradient are 0.
template <typename R>
__device__ __forceinline__ R weno5_grad(R v1, R v2, R v3, R v4, R v5, R (&g)[5]) {
    constexpr bool F = sizeof(R) == 4;
    const R m = fmax(fmax(fmax(fmax(fabs(v1), fabs(v2)), fabs(v3)), fabs(v4)), fabs(v5));
    // first entry of largest magnitude (its index and value)
    const int J = fabs(v1) == m ? 0 : fabs(v2) == m ? 1 : fabs(v3) == m ? 2 : fabs(v4) == m ? 3 : 4;
    const R vJ = J == 0 ? v1 : J == 1 ? v2 : J == 2 ? v3 : J == 3 ? v4 : v5;
    auto rcp = [](R x) {
        if constexpr (F) return __builtin_amdgcn_rcpf(x);
        else return (R)1 / x;
    };
    constexpr R tiny = F ? (R)1.17549435e-38 : (R)2.2250738585072014e-308;
    const R e4 = ((R)4e-6 * m) * m;
    const R eps4 = fmax(e4, tiny);
    const R s1 = v2 - v1, s2 = v3 - v2, s3 = v4 - v3, s4 = v5 - v4;
    const R t0 = s2 - s1, u0 = (R)3 * s2 - s1;
    const R t1 = s3 - s2, u1 = s2 + s3;
    const R t2 = s4 - s3, u2 = s4 - (R)3 * s3;
    constexpr R c13 = (R)(13.0 / 3.0);
    const R b0 = (c13 * t0) * t0 + (u0 * u0 + eps4);
    const R b1 = (c13 * t1) * t1 + (u1 * u1 + eps4);
    const R b2 = (c13 * t2) * t2 + (u2 * u2 + eps4);
    const R rb0 = rcp(b0), rb1 = rcp(b1), rb2 = rcp(b2);
    const R q1 = b0 * rb1, q2 = b0 * rb2;
    const R w1 = ((R)6 * q1) * q1, w2 = ((R)3 * q2) * q2;
    const R rD = rcp(((R)1 + w1) + w2);
    const R o0 = rD, o1 = w1 * rD, o2 = w2 * rD;
    const R r0 = (R)5 * s2 - (R)2 * s1, r1 = s2 + (R)2 * s3, r2 = (R)4 * s3 - s4;
    const R Rb = o0 * r0 + o1 * r1 + o2 * r2;
    const R W = v3 + Rb * (R)(1.0 / 6.0);
    // backward: beta_k = omega_k (r_k - Rb) / b_k, dW/db_k = -beta_k / 3
    const R be0 = o0 * (r0 - Rb) * rb0, be1 = o1 * (r1 - Rb) * rb1, be2 = o2 * (r2 - Rb) * rb2;
    constexpr R kt = (R)(-2.0 * 13.0 / 9.0), ku = (R)(-2.0 / 3.0);  // d b / d t = 2 c t, d b / d u = 2 u
    const R tb0 = kt * t0 * be0, tb1 = kt * t1 * be1, tb2 = kt * t2 * be2;
    const R ub0 = ku * u0 * be0, ub1 = ku * u1 * be1, ub2 = ku * u2 * be2;
    const R epsb = (be0 + be1 + be2) * (R)(-1.0 / 3.0);
    const R s1b = -tb0 - ub0 - o0 * (R)(1.0 / 3.0);
    const R s2b = tb0 + (R)3 * ub0 - tb1 + ub1 + (o0 * (R)5 + o1) * (R)(1.0 / 6.0);
    const R s3b = tb1 + ub1 - tb2 - (R)3 * ub2 + (o1 + o2 * (R)2) * (R)(1.0 / 3.0);
    const R s4b = tb2 + ub2 - o2 * (R)(1.0 / 6.0);
    const R ej = e4 >= tiny ? epsb * (R)8e-6 * vJ : (R)0;
    const bool ok = m > (R)0;
    g[0] = ok ? -s1b + (J == 0 ? ej : (R)0) : (R)0;
    g[1] = ok ? s1b - s2b + (J == 1 ? ej : (R)0) : (R)0;
    g[2] = ok ? (R)1 + s2b - s3b + (J == 2 ? ej : (R)0) : (R)0;
    g[3] = ok ? s3b - s4b + (J == 3 ? ej : (R)0) : (R)0;
    g[4] = ok ? s4b + (J == 4 ? ej : (R)0) : (R)0;
    return ok ? W : (R)0;
}

// ------------------------------------------------------------ dual numbers
// Forward-mode derivative carrier: value and one directional derivative.
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual dual(double v, double d = 0.0) { return Dual{v, d}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double r = a.v / b.v;
    return {r, (a.d - r * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
    const double r = sqrt(a.v);
    return {r, 0.5 * a.d / r};
}
__device__ __forceinline__ void dsincos(Dual a, Dual* s, Dual* c) {
    double sv, cv;
    sincos(a.v, &sv, &cv);
    *s = {sv, cv * a.d};
    *c = {cv, -sv * a.d};
}

// First-order velocity jet for the medium adjoint: from the five fields'
// values and first derivatives m[f][0..2] = (f, f_x, f_z) (as duals), the qP
// phase velocity v and v_x, v_z, v_theta, then the Liouville velocity
// V = (v sin + v_t cos, v cos - v_t sin, -(v_x cos - v_z sin)).
__device__ inline void liouville_velocity_dual(const Dual (&m)[NF][3], double theta, Dual (&V)[3],
                                               Dual* vout = nullptr) {
    Dual sp, cp;
    dsincos(dual(theta) - m[4][0], &sp, &cp);
    const Dual S2 = sp * sp, C2 = cp * cp, s2 = 2.0 * (sp * cp), c2 = C2 - S2;
    const Dual a11 = m[0][0], a33 = m[1][0], b = m[2][0], a55 = m[3][0];
    const Dual P = (a11 + a55) * S2 + (a33 + a55) * C2;
    const Dual Q = (a11 - a55) * S2 - (a33 - a55) * C2;
    const Dual R = b * s2;
    // phi-derivatives
    const Dual Pp = (a11 - a33) * s2;
    const Dual Qp = (a11 + a33 - 2.0 * a55) * s2;
    const Dual Rp = 2.0 * (b * c2);
    Dual Fx[3], Fz[3];  // spatial derivatives of P, Q, R at fixed theta
    for (int i = 0; i < 2; ++i) {
        const int sl = 1 + i;
        const Dual nui = m[4][sl];
        const Dual Pm = m[0][sl] * S2 + m[1][sl] * C2 + m[3][sl];
        const Dual Qm = m[0][sl] * S2 - m[1][sl] * C2 + m[3][sl] * c2;
        const Dual Rm = m[2][sl] * s2;
        Dual* out = i == 0 ? Fx : Fz;
        out[0] = Pm - Pp * nui;
        out[1] = Qm - Qp * nui;
        out[2] = Rm - Rp * nui;
    }
    const Dual D = dsqrt(Q * Q + R * R);
    const Dual v = dsqrt(0.5 * (P + D));
    // dv = (dP + (Q dQ + R dR)/D) / (4 v)
    auto dv = [&](Dual dP, Dual dQ, Dual dR) { return (dP + (Q * dQ + R * dR) / D) / (4.0 * v); };
    const Dual vt = dv(Pp, Qp, Rp);
    const Dual vx = dv(Fx[0], Fx[1], Fx[2]);
    const Dual vz = dv(Fz[0], Fz[1], Fz[2]);
    double sn, cs;
    sincos(theta, &sn, &cs);
    V[0] = sn * v + cs * vt;
    V[1] = cs * v - sn * vt;
    V[2] = -(cs * vx - sn * vz);
    if (vout) *vout = v;
}

}  // namespace egb
