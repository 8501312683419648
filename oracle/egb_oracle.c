/*
 * FP64 CPU oracle for the anisotropic Eulerian Gaussian beam hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP library.
 *
 * Plain, slow, obviously-correct loops in double precision, written from the
 * paper (Huang, "Eulerian Gaussian beams ... arbitrary anisotropy"):
 *   - density-normalised moduli and the 2D Christoffel matrix (Sec. 2, eqs. 4-5)
 *   - qP eigenvalue G(x,p) = 1 as the Hamiltonian F = G - 1 (eqs. 3, 6)
 *   - ray velocity dx/dtau, dz/dtau (eqs. 8-9) and angle rate dtheta/dtau
 *     (eq. 12, with the Hamiltonian minus sign of dp/dtau restored)
 *   - level-set / traveltime / dynamic-ray-tracing transport (eqs. 16, 19, 21)
 *     solved as the stationary phase-space Liouville system V.grad U = S(U)
 *     by explicit pseudo-time marching (WENO5 Hamilton-Jacobi upwinding,
 *     SSP-RK3), with the point source imposed as local homogeneous data
 *   - Gaussian-beam superposition on the Cartesian grid (eqs. 25-27, 34-35)
 *   - first-arrival pick on the level set {phi1 = 0} (eq. 35)
 * Where the paper is silent or garbled the reading used is stated next to the
 * code.  No blocking, fusion or reordering beyond the definitions.
 *
 * Layouts: phase-space planes are [theta][x][z] (z fastest).  Oracle state
 * planes, in this order: phi1, psi, Re C, Im C, Re B, Im B.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NFLD 5 /* medium fields: a11, a33, b = a13 + a55, a55, tilt nu */
#define NTAY 6 /* per field: f, f_x, f_z, f_xx, f_xz, f_zz             */
#define NSTATE 7
/* S_PH: the continuous phase of C along the ray (the KMAH phase); it only
 * decides the branch of sqrt(1/C) in the beam sum */
enum { S_PHI = 0, S_PSI = 1, S_RC = 2, S_IC = 3, S_RB = 4, S_IB = 5, S_PH = 6 };

/* ------------------------------------------------------------------------ */
/* 4th-order finite differences on a uniform line (central inside, one-sided
 * 4th order within two points of either end).  Reading: the paper gives no
 * discretisation; these fix the spatial derivatives of the medium.          */

static double fd1_line(const double *f, long st, int n, int i, double h)
{
#define F(k) f[(long)(k) * st]
    if (i >= 2 && i <= n - 3)
        return (F(i - 2) - 8.0 * F(i - 1) + 8.0 * F(i + 1) - F(i + 2)) / (12.0 * h);
    if (i == 0)
        return (-25.0 * F(0) + 48.0 * F(1) - 36.0 * F(2) + 16.0 * F(3) - 3.0 * F(4)) / (12.0 * h);
    if (i == 1)
        return (-3.0 * F(0) - 10.0 * F(1) + 18.0 * F(2) - 6.0 * F(3) + F(4)) / (12.0 * h);
    if (i == n - 2)
        return -(-3.0 * F(n - 1) - 10.0 * F(n - 2) + 18.0 * F(n - 3) - 6.0 * F(n - 4) + F(n - 5)) / (12.0 * h);
    return -(-25.0 * F(n - 1) + 48.0 * F(n - 2) - 36.0 * F(n - 3) + 16.0 * F(n - 4) - 3.0 * F(n - 5)) / (12.0 * h);
#undef F
}

static double fd2_line(const double *f, long st, int n, int i, double h)
{
#define F(k) f[(long)(k) * st]
    double h2 = 12.0 * h * h;
    if (i >= 2 && i <= n - 3)
        return (-F(i - 2) + 16.0 * F(i - 1) - 30.0 * F(i) + 16.0 * F(i + 1) - F(i + 2)) / h2;
    if (i == 0)
        return (45.0 * F(0) - 154.0 * F(1) + 214.0 * F(2) - 156.0 * F(3) + 61.0 * F(4) - 10.0 * F(5)) / h2;
    if (i == 1)
        return (10.0 * F(0) - 15.0 * F(1) - 4.0 * F(2) + 14.0 * F(3) - 6.0 * F(4) + F(5)) / h2;
    if (i == n - 2)
        return (10.0 * F(n - 1) - 15.0 * F(n - 2) - 4.0 * F(n - 3) + 14.0 * F(n - 4) - 6.0 * F(n - 5) + F(n - 6)) / h2;
    return (45.0 * F(n - 1) - 154.0 * F(n - 2) + 214.0 * F(n - 3) - 156.0 * F(n - 4) + 61.0 * F(n - 5) - 10.0 * F(n - 6)) / h2;
#undef F
}

/* Exposed for the finite-difference pins. */
double oc_fd1(const double *f, int n, int i, double h) { return fd1_line(f, 1, n, i, h); }
double oc_fd2(const double *f, int n, int i, double h) { return fd2_line(f, 1, n, i, h); }

/* ------------------------------------------------------------------------ */
/* Medium table (eqs. 4-5).  Thomsen parameters -> density-normalised moduli
 * in the symmetry frame (rho cancels, eq. 5):
 *   a33 = vp0^2, a55 = (fs vp0)^2, a11 = vp0^2 (1 + 2 eps),
 *   (a13 + a55)^2 = (a33 - a55) (a33 (1 + 2 delta) - a55)   (Thomsen's delta)
 * Reading: the configs give vp0, eps, delta and tilt only; the shear ratio fs
 * is a parameter (0.5 by default).  Output per (x,z) cell: for each field
 * (a11, a33, b = a13 + a55, a55, nu) its value and 4th-order first and second
 * spatial derivatives.  tab index: ((ix*nz + iz)*NFLD + field)*NTAY + t.   */
int oc_medium_table(int nx, int nz, double dx, double dz, const double *vp0, const double *eps,
                    const double *dlt, const double *tilt, double fs, double *tab)
{
    if (nx < 6 || nz < 6) return -1;
    long n2 = (long)nx * nz;
    double *fld = (double *)malloc(sizeof(double) * n2 * NFLD);
    double *tmp = (double *)malloc(sizeof(double) * n2);
    if (!fld || !tmp) { free(fld); free(tmp); return -2; }
    for (long c = 0; c < n2; ++c) {
        double a33 = vp0[c] * vp0[c];
        double a55 = fs * fs * a33;
        double a11 = a33 * (1.0 + 2.0 * eps[c]);
        double b = sqrt((a33 - a55) * (a33 * (1.0 + 2.0 * dlt[c]) - a55));
        fld[0 * n2 + c] = a11;
        fld[1 * n2 + c] = a33;
        fld[2 * n2 + c] = b;
        fld[3 * n2 + c] = a55;
        fld[4 * n2 + c] = tilt ? tilt[c] : 0.0;
    }
    for (int m = 0; m < NFLD; ++m) {
        const double *f = fld + (long)m * n2;
        /* f_z on the whole grid, then f_xz = d/dx of it */
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz)
                tmp[(long)ix * nz + iz] = fd1_line(f + (long)ix * nz, 1, nz, iz, dz);
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                long c = (long)ix * nz + iz;
                double *t = tab + (c * NFLD + m) * NTAY;
                t[0] = f[c];
                t[1] = fd1_line(f + iz, nz, nx, ix, dx);
                t[2] = tmp[c];
                t[3] = fd2_line(f + iz, nz, nx, ix, dx);
                t[4] = fd1_line(tmp + iz, nz, nx, ix, dx);
                t[5] = fd2_line(f + (long)ix * nz, 1, nz, iz, dz);
            }
    }
    free(fld);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Second-order jets in the three phase-space variables (x, z, theta):
 * value, gradient and Hessian, propagated by the chain rule.               */
typedef struct { double f, g[3], h[3][3]; } jet;

static jet jconst(double c) { jet r; memset(&r, 0, sizeof r); r.f = c; return r; }
static jet jadd(jet a, jet b)
{
    jet r;
    r.f = a.f + b.f;
    for (int i = 0; i < 3; ++i) {
        r.g[i] = a.g[i] + b.g[i];
        for (int j = 0; j < 3; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
    }
    return r;
}
static jet jscale(jet a, double s)
{
    jet r;
    r.f = a.f * s;
    for (int i = 0; i < 3; ++i) {
        r.g[i] = a.g[i] * s;
        for (int j = 0; j < 3; ++j) r.h[i][j] = a.h[i][j] * s;
    }
    return r;
}
static jet jsub(jet a, jet b) { return jadd(a, jscale(b, -1.0)); }
static jet jmul(jet a, jet b)
{
    jet r;
    r.f = a.f * b.f;
    for (int i = 0; i < 3; ++i) {
        r.g[i] = a.f * b.g[i] + b.f * a.g[i];
        for (int j = 0; j < 3; ++j)
            r.h[i][j] = a.f * b.h[i][j] + b.f * a.h[i][j] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
    }
    return r;
}
/* r = phi(a) given phi, phi', phi'' at a.f */
static jet jchain(jet a, double f0, double f1, double f2)
{
    jet r;
    r.f = f0;
    for (int i = 0; i < 3; ++i) {
        r.g[i] = f1 * a.g[i];
        for (int j = 0; j < 3; ++j) r.h[i][j] = f1 * a.h[i][j] + f2 * a.g[i] * a.g[j];
    }
    return r;
}
static jet jsqrt(jet a)
{
    double s = sqrt(a.f);
    return jchain(a, s, 0.5 / s, -0.25 / (s * a.f));
}
static jet jsin(jet a) { return jchain(a, sin(a.f), cos(a.f), -sin(a.f)); }
static jet jcos(jet a) { return jchain(a, cos(a.f), -sin(a.f), -cos(a.f)); }

/* Jet of one medium field (a function of x and z only). */
static jet field_jet(const double *t)
{
    jet r = jconst(t[0]);
    r.g[0] = t[1];
    r.g[1] = t[2];
    r.h[0][0] = t[3];
    r.h[0][1] = r.h[1][0] = t[4];
    r.h[1][1] = t[5];
    return r;
}

/* Phase velocity v(x,z,theta) as a jet.  v^2 is the qP eigenvalue of the
 * 2x2 Christoffel matrix Gamma_ik = a_ijkl n_j n_l (eqs. 3-4) for the unit
 * phase direction n = (sin phi, cos phi), phi = theta - nu measured in the
 * symmetry frame; with p = n / v (eq. 7) this is G(x, p) = 1.              */
static jet phase_velocity_jet(const double *t /* NFLD*NTAY */, double theta)
{
    jet a11 = field_jet(t + 0 * NTAY), a33 = field_jet(t + 1 * NTAY);
    jet b = field_jet(t + 2 * NTAY), a55 = field_jet(t + 3 * NTAY);
    jet phi = jsub(jconst(theta), field_jet(t + 4 * NTAY));
    phi.g[2] = 1.0; /* d phi / d theta */
    jet n1 = jsin(phi), n3 = jcos(phi);
    jet g11 = jadd(jmul(a11, jmul(n1, n1)), jmul(a55, jmul(n3, n3)));
    jet g33 = jadd(jmul(a55, jmul(n1, n1)), jmul(a33, jmul(n3, n3)));
    jet g13 = jmul(b, jmul(n1, n3));
    jet dif = jsub(g11, g33);
    jet disc = jadd(jmul(dif, dif), jscale(jmul(g13, g13), 4.0));
    jet G = jscale(jadd(jadd(g11, g33), jsqrt(disc)), 0.5);
    return jsqrt(G);
}

/* v-jet flattened: v, v_x, v_z, v_t, v_xx, v_xz, v_zz, v_xt, v_zt, v_tt */
static void vjet_flat(jet v, double o[10])
{
    o[0] = v.f;       o[1] = v.g[0];    o[2] = v.g[1];    o[3] = v.g[2];
    o[4] = v.h[0][0]; o[5] = v.h[0][1]; o[6] = v.h[1][1];
    o[7] = v.h[0][2]; o[8] = v.h[1][2]; o[9] = v.h[2][2];
}

void oc_vjet(const double *t, double theta, double *o) { vjet_flat(phase_velocity_jet(t, theta), o); }

/* Liouville velocity and ray-normal dynamic ray tracing matrix from the
 * v-jet at phase angle theta.
 *   V_x = dx/dtau, V_z = dz/dtau: the group velocity v n + v_theta n_perp
 *     (eqs. 8-9 with F = G - 1, p.grad_p F = 2, so tau is traveltime);
 *   V_t = dtheta/dtau = -(v_x cos theta - v_z sin theta)  (eq. 12; reading:
 *     dp/dtau = -grad_x F / (p.grad_p F), the sign eq. 10 drops).
 * A: the linearised flow d(dy)/dtau = grad V . dy written for the
 * perturbation components (dn, dth_perp) normal to the ray, dn = g_perp.dx,
 * dth_perp = dtheta - (g.dx) V_t/|V|, the along-ray drift projected out.
 * Reading: replaces the row-based B, C of eqs. 21-23 (singular for
 * horizontal rays); in isotropic media it reduces to A = [[0, v],
 * [-v_nn, v_s]], i.e. eqs. 21-22 with H_pp = v u1^3.                       */
void oc_va(const double *vj, double theta, double *V, double *A)
{
    double v = vj[0], vx = vj[1], vz = vj[2], vt = vj[3];
    double vxx = vj[4], vxz = vj[5], vzz = vj[6], vxt = vj[7], vzt = vj[8], vtt = vj[9];
    double s = sin(theta), c = cos(theta);
    double Vx = v * s + vt * c, Vz = v * c - vt * s, Vt = -(vx * c - vz * s);
    double J[2][2] = {{vx * s + vxt * c, vz * s + vzt * c}, {vx * c - vxt * s, vz * c - vzt * s}};
    double Vth[2] = {(v + vtt) * c, -(v + vtt) * s};
    double gVt[2] = {-(vxx * c - vxz * s), -(vxz * c - vzz * s)};
    double dVt = -(vxt * c - vx * s - vzt * s - vz * c);
    double nv = sqrt(Vx * Vx + Vz * Vz);
    double g[2] = {Vx / nv, Vz / nv};
    double gp[2] = {g[1], -g[0]};
    double Jgp[2] = {J[0][0] * gp[0] + J[0][1] * gp[1], J[1][0] * gp[0] + J[1][1] * gp[1]};
    double dV[2] = {J[0][0] * Vx + J[0][1] * Vz + Vth[0] * Vt, J[1][0] * Vx + J[1][1] * Vz + Vth[1] * Vt};
    double phidot = (gp[0] * dV[0] + gp[1] * dV[1]) / nv;
    double sig_n = g[0] * Jgp[0] + g[1] * Jgp[1] + phidot;
    double sig_t = g[0] * Vth[0] + g[1] * Vth[1];
    V[0] = Vx; V[1] = Vz; V[2] = Vt;
    A[0] = gp[0] * Jgp[0] + gp[1] * Jgp[1];
    A[1] = gp[0] * Vth[0] + gp[1] * Vth[1];
    A[2] = gp[0] * gVt[0] + gp[1] * gVt[1] - sig_n * Vt / nv;
    A[3] = dVt - sig_t * Vt / nv;
}

/* ------------------------------------------------------------------------ */
/* Per-cell velocity field (7 planes V_x, V_z, V_t, A11, A12, A21, A22) and
 * the phase-velocity aux planes (v, v_x, v_z, v_t) used by the beam sum.
 * Returns the CFL step dt = 0.5 / max(|V_x|/dx + |V_z|/dz + |V_t|/dth).   */
int oc_velocity(int nx, int nz, int nth, double dx, double dz, const double *tab, double *vel,
                double *vaux, double *dt_out)
{
    long n = (long)nth * nx * nz;
    double dth = 2.0 * M_PI / nth;
    double rate = 0.0;
#pragma omp parallel for reduction(max : rate) schedule(static)
    for (int k = 0; k < nth; ++k) {
        double th = k * dth;
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                long c2 = (long)ix * nz + iz, c = (long)k * nx * nz + c2;
                double vj[10], V[3], A[4];
                vjet_flat(phase_velocity_jet(tab + c2 * NFLD * NTAY, th), vj);
                oc_va(vj, th, V, A);
                for (int q = 0; q < 3; ++q) vel[q * n + c] = V[q];
                for (int q = 0; q < 4; ++q) vel[(3 + q) * n + c] = A[q];
                for (int q = 0; q < 4; ++q) vaux[q * n + c] = vj[q];
                double r = fabs(V[0]) / dx + fabs(V[1]) / dz + fabs(V[2]) / dth;
                if (r > rate) rate = r;
            }
    }
    *dt_out = 0.5 / rate;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* qP polarisation (eqs. 4, 31-32): the unit eigenvector of the 2x2
 * Christoffel matrix for its larger eigenvalue, phase angle theta, medium
 * values ms = (a11, a33, b = a13 + a55, a55, nu).  Built in the symmetry
 * frame (phase angle theta - nu), turned back by nu, and signed so that it
 * points along the phase direction (g . n > 0).                            */
void oc_qp_polarization(const double *ms, double theta, double g[2])
{
    double ph = theta - ms[4], n1 = sin(ph), n3 = cos(ph);
    double g11 = ms[0] * n1 * n1 + ms[3] * n3 * n3, g33 = ms[3] * n1 * n1 + ms[1] * n3 * n3, g13 = ms[2] * n1 * n3;
    double G = 0.5 * (g11 + g33 + sqrt((g11 - g33) * (g11 - g33) + 4.0 * g13 * g13));
    /* (G - g33, g13) and (g13, G - g11) both solve the system; take the longer */
    double a1 = G - g33, a3 = g13, b1 = g13, b3 = G - g11;
    double vx, vz;
    if (a1 * a1 + a3 * a3 >= b1 * b1 + b3 * b3) { vx = a1; vz = a3; } else { vx = b1; vz = b3; }
    double nv = sqrt(vx * vx + vz * vz);
    if (nv == 0.0) { vx = n1; vz = n3; nv = 1.0; } /* isotropic: any vector; the phase direction */
    vx /= nv;
    vz /= nv;
    if (vx * n1 + vz * n3 < 0.0) { vx = -vx; vz = -vz; }
    double cn = cos(ms[4]), sn = sin(ms[4]);
    g[0] = vx * cn + vz * sn;
    g[1] = -vx * sn + vz * cn;
}

/* Point-source data (reading of eqs. 20 and 24 for a point source).  The
 * medium is frozen at the source: the table fields are bilinearly
 * interpolated there.  For each theta the homogeneous solution is
 *   phi1 = (x - xs) . g_perp(theta)       (ray-family level set; Gamma: phi1 = 0)
 *   psi  = p(theta) . (x - xs)            (traveltime, p = n / v, eq. 7)
 *   C    = s (1 + i beta A12 psi),  B = i beta s   (C(0) real, B(0) = i beta C(0))
 * with s = (sqrt(v_s) / W)^(2/3) and W = a33 / v_s^2: the take-off-angle
 * weight of the beam superposition (eqs. 31-33 redone in 2D) folded into the
 * data so that the beam sum needs no take-off angle.                       */
static double bilin(const double *tab, int nx, int nz, double dx, double dz, double x0, double z0,
                    double xs, double zs, int fld)
{
    double fx = (xs - x0) / dx - 0.5, fz = (zs - z0) / dz - 0.5;
    int ix = (int)floor(fx), iz = (int)floor(fz);
    if (ix < 0) ix = 0;
    if (ix > nx - 2) ix = nx - 2;
    if (iz < 0) iz = 0;
    if (iz > nz - 2) iz = nz - 2;
    double tx = fx - ix, tz = fz - iz;
    if (tx < 0.0) tx = 0.0;
    if (tx > 1.0) tx = 1.0;
    if (tz < 0.0) tz = 0.0;
    if (tz > 1.0) tz = 1.0;
#define T(i, j) tab[(((long)(i) * nz + (j)) * NFLD + fld) * NTAY]
    return (1 - tx) * (1 - tz) * T(ix, iz) + tx * (1 - tz) * T(ix + 1, iz) + (1 - tx) * tz * T(ix, iz + 1) +
           tx * tz * T(ix + 1, iz + 1);
#undef T
}

/* Source-frozen homogeneous quantities at phase angle theta. */
static void source_data(const double *ms /* a11,a33,b,a55,nu */, double theta, double *v_out,
                        double g_perp[2], double p[2], double *A12, double *s_out)
{
    double t[NFLD * NTAY];
    memset(t, 0, sizeof t);
    for (int m = 0; m < NFLD; ++m) t[m * NTAY] = ms[m];
    double vj[10], V[3], A[4];
    vjet_flat(phase_velocity_jet(t, theta), vj);
    oc_va(vj, theta, V, A);
    double v = vj[0], nv = sqrt(V[0] * V[0] + V[1] * V[1]);
    g_perp[0] = V[1] / nv;
    g_perp[1] = -V[0] / nv;
    p[0] = sin(theta) / v;
    p[1] = cos(theta) / v;
    *A12 = A[1];
    double W = ms[1] / (v * v);
    *s_out = pow(sqrt(v) / W, 2.0 / 3.0);
    *v_out = v;
}

int oc_init_state(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *tab,
                  double xs, double zs, double beta, double *U)
{
    long n = (long)nth * nx * nz;
    double dth = 2.0 * M_PI / nth;
    double ms[NFLD];
    for (int m = 0; m < NFLD; ++m) ms[m] = bilin(tab, nx, nz, dx, dz, x0, z0, xs, zs, m);
    for (int k = 0; k < nth; ++k) {
        double v, gp[2], p[2], A12, s;
        source_data(ms, k * dth, &v, gp, p, &A12, &s);
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                long c = ((long)k * nx + ix) * nz + iz;
                double ddx = x0 + (ix + 0.5) * dx - xs, ddz = z0 + (iz + 0.5) * dz - zs;
                double psi = p[0] * ddx + p[1] * ddz;
                U[S_PHI * n + c] = ddx * gp[0] + ddz * gp[1];
                U[S_PSI * n + c] = psi;
                U[S_RC * n + c] = s;
                U[S_IC * n + c] = s * beta * A12 * psi;
                U[S_RB * n + c] = 0.0;
                U[S_IB * n + c] = beta * s;
                /* arg C of the data: C = s (1 + i beta A12 psi), s > 0 */
                U[S_PH * n + c] = atan(beta * A12 * psi);
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* WENO5 Hamilton-Jacobi derivative (Jiang-Peng / Osher-Shu form), undivided:
 * returns the one-sided derivative times the spacing.  u[0..6] holds the
 * values at offsets -3..+3; minus != 0 selects the backward-biased D-.
 * Smoothness tolerance eps_W = 1e-6 max_k v_k^2 (scale invariant); when all
 * five differences vanish the derivative is 0.                             */
double oc_weno(const double *u, int minus)
{
    double v[5];
    for (int m = 0; m < 5; ++m)
        v[m] = minus ? u[m + 1] - u[m] : u[6 - m] - u[5 - m];
    /* W is positively 1-homogeneous in v (eps scales with max v^2), so it is
     * evaluated on v / max|v| and scaled back: the textbook formula as
     * written, without overflow of 1 / (eps + beta)^2 for tiny differences */
    double am = 0.0;
    for (int m = 0; m < 5; ++m)
        if (fabs(v[m]) > am) am = fabs(v[m]);
    if (am == 0.0) return 0.0;
    for (int m = 0; m < 5; ++m) v[m] /= am;
    double mx = 0.0;
    for (int m = 0; m < 5; ++m)
        if (v[m] * v[m] > mx) mx = v[m] * v[m];
    double q0 = v[0] / 3.0 - 7.0 * v[1] / 6.0 + 11.0 * v[2] / 6.0;
    double q1 = -v[1] / 6.0 + 5.0 * v[2] / 6.0 + v[3] / 3.0;
    double q2 = v[2] / 3.0 + 5.0 * v[3] / 6.0 - v[4] / 6.0;
    double s0 = 13.0 / 12.0 * pow(v[0] - 2.0 * v[1] + v[2], 2) + 0.25 * pow(v[0] - 4.0 * v[1] + 3.0 * v[2], 2);
    double s1 = 13.0 / 12.0 * pow(v[1] - 2.0 * v[2] + v[3], 2) + 0.25 * pow(v[1] - v[3], 2);
    double s2 = 13.0 / 12.0 * pow(v[2] - 2.0 * v[3] + v[4], 2) + 0.25 * pow(3.0 * v[2] - 4.0 * v[3] + v[4], 2);
    double e = 1e-6 * mx;
    double a0 = 0.1 / pow(e + s0, 2), a1 = 0.6 / pow(e + s1, 2), a2 = 0.3 / pow(e + s2, 2);
    return am * ((a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2));
}

/* The upwind derivative of the WENO5 stencils with their linear weights
 * d = (0.1, 0.6, 0.3) (the fifth-order linear upwind scheme), undivided:
 * q0 = v1/3 - 7v2/6 + 11v3/6, q1 = -v2/6 + 5v3/6 + v4/3,
 * q2 = v3/3 + 5v4/6 - v5/6, D = 0.1 q0 + 0.6 q1 + 0.3 q2, with v the
 * one-sided differences as in oc_weno.  Used for the phase plane, which is
 * smooth in phase space (it has no fronts for nonlinear weights to guard)
 * and only has to stay well within pi of the ray's phase.                 */
double oc_upwind5(const double *u, int minus)
{
    double v[5];
    for (int m = 0; m < 5; ++m)
        v[m] = minus ? u[m + 1] - u[m] : u[6 - m] - u[5 - m];
    double q0 = v[0] / 3.0 - 7.0 * v[1] / 6.0 + 11.0 * v[2] / 6.0;
    double q1 = -v[1] / 6.0 + 5.0 * v[2] / 6.0 + v[3] / 3.0;
    double q2 = v[2] / 3.0 + 5.0 * v[3] / 6.0 - v[4] / 6.0;
    return 0.1 * q0 + 0.6 * q1 + 0.3 * q2;
}

/* Value of plane u at (k, ix + m, iz) / (k, ix, iz + m) with ghosts: outside
 * the grid in x or z the point-source data b of the same plane, extended by
 * linear extrapolation b_{-m} = (m+1) b_0 - m b_1 (exact for that data, which
 * is affine in position per theta): a Dirichlet condition fixed in time, like
 * the source ball.  theta is periodic.                                      */
static double at_x(const double *u, const double *b, int nx, int nz, long base_k, int ix, int iz, int m)
{
    int i = ix + m;
    if (i < 0) return (1 - i) * b[base_k + (long)0 * nz + iz] + i * b[base_k + (long)1 * nz + iz];
    if (i > nx - 1) {
        int e = i - (nx - 1);
        return (e + 1) * b[base_k + (long)(nx - 1) * nz + iz] - e * b[base_k + (long)(nx - 2) * nz + iz];
    }
    return u[base_k + (long)i * nz + iz];
}
static double at_z(const double *u, const double *b, int nz, long base_kx, int iz, int m)
{
    int j = iz + m;
    if (j < 0) return (1 - j) * b[base_kx] + j * b[base_kx + 1];
    if (j > nz - 1) {
        int e = j - (nz - 1);
        return (e + 1) * b[base_kx + nz - 1] - e * b[base_kx + nz - 2];
    }
    return u[base_kx + j];
}

/* Right-hand side of the stationary Liouville system (eqs. 16, 19, 21 times
 * dz/dtau):  L_f = -(V_x D_x + V_z D_z + V_t D_t) U_f + S_f with
 * S_phi1 = 0, S_psi = 1 (dT/dtau = p.dx/dtau = 1), S_(C,B) = A (C, B).
 * Upwinding: D- where the velocity component is >= 0... precisely D- when
 * V_d > 0 or V_d == 0, D+ when V_d < 0.                                    */
static void rhs(int nx, int nz, int nth, double dx, double dz, const double *vel, const double *U,
                const double *Ub, double *L)
{
    long n = (long)nth * nx * nz, nxz = (long)nx * nz;
    double dth = 2.0 * M_PI / nth;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nth; ++k)
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                long c = (long)k * nxz + (long)ix * nz + iz;
                double cx = vel[0 * n + c] / dx, cz = vel[1 * n + c] / dz, ct = vel[2 * n + c] / dth;
                double Lf[NSTATE];
                for (int f = 0; f < NSTATE; ++f) {
                    const double *u = U + f * n, *ub = Ub + f * n;
                    double (*D)(const double *, int) = f == S_PH ? oc_upwind5 : oc_weno;
                    double w[7];
                    for (int m = -3; m <= 3; ++m) w[m + 3] = at_x(u, ub, nx, nz, (long)k * nxz, ix, iz, m);
                    double Dx = D(w, cx >= 0.0);
                    for (int m = -3; m <= 3; ++m) w[m + 3] = at_z(u, ub, nz, (long)k * nxz + (long)ix * nz, iz, m);
                    double Dz = D(w, cz >= 0.0);
                    for (int m = -3; m <= 3; ++m) {
                        int kk = ((k + m) % nth + nth) % nth;
                        w[m + 3] = u[(long)kk * nxz + (long)ix * nz + iz];
                    }
                    double Dt = D(w, ct >= 0.0);
                    Lf[f] = -(cx * Dx + cz * Dz + ct * Dt);
                }
                double A11 = vel[3 * n + c], A12 = vel[4 * n + c], A21 = vel[5 * n + c], A22 = vel[6 * n + c];
                Lf[S_PSI] += 1.0;
                Lf[S_RC] += A11 * U[S_RC * n + c] + A12 * U[S_RB * n + c];
                Lf[S_RB] += A21 * U[S_RC * n + c] + A22 * U[S_RB * n + c];
                Lf[S_IC] += A11 * U[S_IC * n + c] + A12 * U[S_IB * n + c];
                Lf[S_IB] += A21 * U[S_IC * n + c] + A22 * U[S_IB * n + c];
                /* continuous phase of C: d(log C)/dtau = A11 + A12 B / C with A
                 * real, so dPhi/dtau = A12 Im(B / C)                          */
                {
                    double rc = U[S_RC * n + c], ic = U[S_IC * n + c], rb = U[S_RB * n + c], ib = U[S_IB * n + c];
                    Lf[S_PH] += A12 * (ib * rc - rb * ic) / (rc * rc + ic * ic);
                }
                for (int f = 0; f < NSTATE; ++f) L[f * n + c] = Lf[f];
            }
}

/* Source ball: cells with |x - xs| <= r0 keep the point-source data. */
static int in_ball(double x0, double z0, double dx, double dz, int ix, int iz, double xs, double zs, double r0)
{
    double ddx = x0 + (ix + 0.5) * dx - xs, ddz = z0 + (iz + 0.5) * dz - zs;
    return ddx * ddx + ddz * ddz <= r0 * r0;
}

/* nsteps SSP-RK3 steps (Shu-Osher form) of U_t = L(U), in place:
 *   U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U  = 1/3 U + 2/3 (U2 + dt L(U2)),
 * ball cells copying U after every stage (Dirichlet point-source data).   */
int oc_march(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *vel,
             double xs, double zs, double r0, const double *Ub, double *U, double dt, int nsteps)
{
    long n = (long)nth * nx * nz, nxz = (long)nx * nz;
    double *U1 = (double *)malloc(sizeof(double) * n * NSTATE);
    double *U2 = (double *)malloc(sizeof(double) * n * NSTATE);
    double *L = (double *)malloc(sizeof(double) * n * NSTATE);
    char *ball = (char *)malloc(nxz);
    if (!U1 || !U2 || !L || !ball) { free(U1); free(U2); free(L); free(ball); return -2; }
    for (int ix = 0; ix < nx; ++ix)
        for (int iz = 0; iz < nz; ++iz) ball[(long)ix * nz + iz] = (char)in_ball(x0, z0, dx, dz, ix, iz, xs, zs, r0);
    static const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int step = 0; step < nsteps; ++step) {
        const double *in[3] = {U, U1, U2};
        double *out[3] = {U1, U2, U};
        for (int st = 0; st < 3; ++st) {
            rhs(nx, nz, nth, dx, dz, vel, in[st], Ub, L);
#pragma omp parallel for schedule(static)
            for (long c = 0; c < n; ++c) {
                int b = ball[c % nxz];
                for (int f = 0; f < NSTATE; ++f) {
                    long q = f * n + c;
                    out[st][q] = b ? U[q] : ca[st] * U[q] + cb[st] * (in[st][q] + dt * L[q]);
                }
            }
        }
    }
    free(U1); free(U2); free(L); free(ball);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gaussian-beam superposition (eqs. 25-27, 33-35), 2D reading.
 *
 * Each phase cell c on (near) Gamma = {phi1 = 0, psi > 0} is one beam of the
 * family.  Row quadrature (output row z0 = z_c): the integral over take-off
 * angle becomes a sum over the (x, theta) cells of that row with a smoothed
 * delta of the signed distance d = phi1 / |grad phi1| (theta scaled by
 * lambda = dx/dth), and the Jacobian from the imaginary DRT part,
 * Im(C, B) = beta s (dn, dth_perp) per unit take-off angle.  Column quadrature
 * is the mirror image along x = x0.  Each beam contributes
 *   w * sqrt(v / C) * dtheta_c * exp(i omega T),
 *   T = psi + p1 (x0 - x_c) + 1/2 M_row (x0 - x_c)^2          (row; eqs. 25, 27)
 * with M the complex traveltime Hessian restricted to the line (M = B C^-1 in
 * the ray-normal frame, eq. 25), w = cos^4/(cos^4 + sin^4) of the ray angle
 * for rows and 1 - w for columns, and the total scaled by W = i / (4 pi).
 * Beams with 1/2 omega Im(M) dist^2 > 16 are skipped, and cells whose line
 * Hessian has Im(M) <= 0 are no beams: a Gaussian beam decays away from its
 * centre (the exact transport keeps Im(B conj(C)) > 0; a discrete field can
 * lose it, and such a cell would grow without bound).  lin != 0 takes the
 * linear coefficient p1 (p3) from eq. 28 (oc_lin28) instead of eq. 7.
 * Output layout out[w][ix][iz][re/im].                                     */
typedef struct { double pos, psi, p; double complex M, amp; } beamrec;

/* Linear phase coefficient of eq. 28 (the lin=paper28 variant): for a ray
 * with phase angle th (sin s, cos c) and direction u = dx/dz, phase velocity
 * v, sqrt(s (s u^2 + 2 c u - s)) / (v (c + s u)).  Reading: the square root
 * drops the sign of p1, which is restored from sin th, and a negative
 * radicand (no real value) counts as 0.  In isotropic media (u = tan th) it
 * is sin th / v, eq. 7's p1.  Column quadrature: the mirror image (s <-> c,
 * u -> dz/dx).                                                             */
double oc_lin28(double s, double c, double u, double v)
{
    double rad = s * (s * u * u + 2.0 * c * u - s);
    double L = sqrt(rad > 0.0 ? rad : 0.0) / (v * (c + s * u));
    return copysign(fabs(L), s);
}

static double delta_h(double d, double h) { return fabs(d) < h ? (1.0 + cos(M_PI * d / h)) / (2.0 * h) : 0.0; }

/* The beams of the state, as per-row and per-column lists of records. */
typedef struct { beamrec *rows, *cols; int *nrow, *ncol; int cap; } beamlists;

static void free_beams(beamlists *bl) { free(bl->rows); free(bl->cols); free(bl->nrow); free(bl->ncol); }

/* 0, -2 (no memory) or -3 (a line holds more beams than the list's room) */
static int beam_lists(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *vel,
                      const double *vaux, double beta, int lin, const double *U, beamlists *bl)
{
    long n = (long)nth * nx * nz, nxz = (long)nx * nz;
    double dth = 2.0 * M_PI / nth, lx = dx / dth, lz = dz / dth, hx = 2.0 * dx, hz = 2.0 * dz;
    const double *phi = U + S_PHI * n;
    int cap = 8 * (nx + nz + nth) + 64;
    beamrec *rows = (beamrec *)malloc(sizeof(beamrec) * (long)nz * cap);
    beamrec *cols = (beamrec *)malloc(sizeof(beamrec) * (long)nx * cap);
    int *nrow = (int *)calloc(nz, sizeof(int)), *ncol = (int *)calloc(nx, sizeof(int));
    int overflow = 0;
    bl->rows = rows; bl->cols = cols; bl->nrow = nrow; bl->ncol = ncol; bl->cap = cap;
    if (!rows || !cols || !nrow || !ncol) { free_beams(bl); return -2; }
    for (int k = 0; k < nth; ++k) {
        double th = k * dth, sn = sin(th), cs = cos(th);
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                long kb = (long)k * nxz, c = kb + (long)ix * nz + iz;
                double psi = U[S_PSI * n + c];
                /* eq. 35's gate psi > 0, taken as psi above a millionth of a
                 * cell's traveltime: the point-source data put psi = 0 in
                 * exact arithmetic on cells at the closest point of their ray
                 * to the source (a source on a cell corner, diagonal phase
                 * angles), which rounding leaves at +-1e-17 either way     */
                if (!(psi > 1e-6 * fmin(dx, dz) / vaux[0 * n + c])) continue;
                /* 4th-order central differences of phi1 (ghost rules as in the march) */
                double fx = (at_x(phi, phi, nx, nz, kb, ix, iz, -2) - 8.0 * at_x(phi, phi, nx, nz, kb, ix, iz, -1) +
                             8.0 * at_x(phi, phi, nx, nz, kb, ix, iz, 1) - at_x(phi, phi, nx, nz, kb, ix, iz, 2)) / (12.0 * dx);
                long kx = kb + (long)ix * nz;
                double fz = (at_z(phi, phi, nz, kx, iz, -2) - 8.0 * at_z(phi, phi, nz, kx, iz, -1) + 8.0 * at_z(phi, phi, nz, kx, iz, 1) -
                             at_z(phi, phi, nz, kx, iz, 2)) / (12.0 * dz);
                int km2 = (k + nth - 2) % nth, km1 = (k + nth - 1) % nth, kp1 = (k + 1) % nth, kp2 = (k + 2) % nth;
                long o = (long)ix * nz + iz;
                double ft = (phi[km2 * nxz + o] - 8.0 * phi[km1 * nxz + o] + 8.0 * phi[kp1 * nxz + o] - phi[kp2 * nxz + o]) /
                            (12.0 * dth);
                double f0 = phi[c];
                double drow = f0 / sqrt(fx * fx + (ft / lx) * (ft / lx));
                double dcol = f0 / sqrt(fz * fz + (ft / lz) * (ft / lz));
                int arow = fabs(drow) < hx, acol = fabs(dcol) < hz;
                if (!arow && !acol) continue;
                double Vx = vel[0 * n + c], Vz = vel[1 * n + c], Vt = vel[2 * n + c];
                double nv = sqrt(Vx * Vx + Vz * Vz), gx = Vx / nv, gz = Vz / nv;
                double gp[2] = {gz, -gx};
                double v = vaux[0 * n + c], vx = vaux[1 * n + c], vz = vaux[2 * n + c], vt = vaux[3 * n + c];
                double complex C = U[S_RC * n + c] + I * U[S_IC * n + c];
                double complex B = U[S_RB * n + c] + I * U[S_IB * n + c];
                double dn = U[S_IC * n + c], dtp = U[S_IB * n + c];
                /* traveltime Hessian pieces: p = n/v, p_theta, d_x p, q = (dp/dtau)/|V| */
                double pth[2] = {cs / v - sn * vt / (v * v), -sn / v - cs * vt / (v * v)};
                double gp_pth = gp[0] * pth[0] + gp[1] * pth[1];
                double gp_dxp_gp = -(gp[0] * sn + gp[1] * cs) * (vx * gp[0] + vz * gp[1]) / (v * v);
                double q[2] = {-vx / (v * nv), -vz / (v * nv)};
                double gq = gx * q[0] + gz * q[1], gpq = gp[0] * q[0] + gp[1] * q[1];
                double complex Mn = (gp_pth * B + gp_dxp_gp * C) / C;
                /* sqrt(v / C) on the ray's branch: the principal root times
                 * (-1)^k, k the full turns between the continuous phase Phi
                 * and arg C (Phi = arg C + 2 pi k)                           */
                int kmah = (int)lround((U[S_PH * n + c] - carg(C)) / (2.0 * M_PI));
                double complex amp0 = csqrt(v / C) * ((kmah & 1) ? -1.0 : 1.0);
                double c4 = pow(gz, 4), s4 = pow(gx, 4), wrow = c4 / (c4 + s4);
                if (arow && fabs(gz) > 1e-4) {
                    double ds = dn * gx / gz, px = dn / gz, pt = dtp + ds * Vt / nv;
                    double dth_c = beta * delta_h(drow, hx) * lx * dx * dth / sqrt(px * px + lx * lx * pt * pt);
                    beamrec r;
                    r.pos = x0 + (ix + 0.5) * dx;
                    r.psi = psi;
                    r.p = lin ? oc_lin28(sn, cs, Vx / Vz, v) : sn / v;
                    r.M = Mn * gz * gz + 2.0 * gpq * gx * gz + gq * gx * gx;
                    r.amp = wrow * amp0 * dth_c;
                    if (cimag(r.M) > 0.0) {
                        if (nrow[iz] < cap) rows[(long)iz * cap + nrow[iz]++] = r; else overflow = 1;
                    }
                }
                if (acol && fabs(gx) > 1e-4) {
                    double ds = -dn * gz / gx, pz = -dn / gx, pt = dtp + ds * Vt / nv;
                    double dth_c = beta * delta_h(dcol, hz) * lz * dz * dth / sqrt(pz * pz + lz * lz * pt * pt);
                    beamrec r;
                    r.pos = z0 + (iz + 0.5) * dz;
                    r.psi = psi;
                    r.p = lin ? oc_lin28(cs, sn, Vz / Vx, v) : cs / v;
                    r.M = Mn * gx * gx - 2.0 * gpq * gx * gz + gq * gz * gz;
                    r.amp = (1.0 - wrow) * amp0 * dth_c;
                    if (cimag(r.M) > 0.0) {
                        if (ncol[ix] < cap) cols[(long)ix * cap + ncol[ix]++] = r; else overflow = 1;
                    }
                }
            }
    }
    return overflow ? -3 : 0;
}

/* G at the output cell (ix, iz) and frequency om: the beams of row iz, then
 * those of column ix, times W = i / (4 pi).                               */
static double complex beam_point(const beamlists *bl, int ix, int iz, double x0, double z0, double dx, double dz,
                                 double om)
{
    double xo = x0 + (ix + 0.5) * dx, zo = z0 + (iz + 0.5) * dz;
    double complex G = 0.0;
    for (int r = 0; r < bl->nrow[iz]; ++r) {
        const beamrec *b = &bl->rows[(long)iz * bl->cap + r];
        double d = xo - b->pos;
        double complex T = b->psi + b->p * d + 0.5 * b->M * d * d;
        if (0.5 * om * cimag(b->M) * d * d > 16.0) continue;
        G += b->amp * cexp(I * om * T);
    }
    for (int r = 0; r < bl->ncol[ix]; ++r) {
        const beamrec *b = &bl->cols[(long)ix * bl->cap + r];
        double d = zo - b->pos;
        double complex T = b->psi + b->p * d + 0.5 * b->M * d * d;
        if (0.5 * om * cimag(b->M) * d * d > 16.0) continue;
        G += b->amp * cexp(I * om * T);
    }
    return G * (I / (4.0 * M_PI));
}

int oc_beam_sum(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *vel,
                const double *vaux, double beta, int lin, const double *U, const double *omegas, int nw, double *out)
{
    beamlists bl;
    int rc = beam_lists(nx, nz, nth, x0, z0, dx, dz, vel, vaux, beta, lin, U, &bl);
    if (rc == -2) return rc;
#pragma omp parallel for collapse(2) schedule(static)
    for (int w = 0; w < nw; ++w)
        for (int ix = 0; ix < nx; ++ix)
            for (int iz = 0; iz < nz; ++iz) {
                double complex G = beam_point(&bl, ix, iz, x0, z0, dx, dz, omegas[w]);
                long o = (((long)w * nx + ix) * nz + iz) * 2;
                out[o] = creal(G);
                out[o + 1] = cimag(G);
            }
    free_beams(&bl);
    return rc;
}

/* The same sum at npts output cells pts[j] = (ix, iz) only; out[w][j][re/im]. */
int oc_beam_sum_at(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *vel,
                   const double *vaux, double beta, int lin, const double *U, const double *omegas, int nw,
                   const int *pts, int npts, double *out)
{
    for (int j = 0; j < npts; ++j)
        if (pts[2 * j] < 0 || pts[2 * j] >= nx || pts[2 * j + 1] < 0 || pts[2 * j + 1] >= nz) return -1;
    beamlists bl;
    int rc = beam_lists(nx, nz, nth, x0, z0, dx, dz, vel, vaux, beta, lin, U, &bl);
    if (rc == -2) return rc;
#pragma omp parallel for collapse(2) schedule(static)
    for (int w = 0; w < nw; ++w)
        for (int j = 0; j < npts; ++j) {
            double complex G = beam_point(&bl, pts[2 * j], pts[2 * j + 1], x0, z0, dx, dz, omegas[w]);
            long o = ((long)w * npts + j) * 2;
            out[o] = creal(G);
            out[o + 1] = cimag(G);
        }
    free_beams(&bl);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* First-arrival pick at receivers (eq. 35's gate).  phi1 and psi are
 * bilinearly interpolated in (x, z) on every theta plane; a root of phi1 lies
 * in [theta_k, theta_k+1) (periodic) when phi1_k == 0 or phi1_k phi1_k+1 < 0;
 * t = phi1_k / (phi1_k - phi1_k+1), psi* = psi_k + t (psi_k+1 - psi_k).  The
 * pick is the smallest psi* > 0 (first such k on ties); NaN if none.       */
int oc_pick(int nx, int nz, int nth, double x0, double z0, double dx, double dz, const double *U,
            const double *rx, int nr, double *tout)
{
    long n = (long)nth * nx * nz, nxz = (long)nx * nz;
    for (int r = 0; r < nr; ++r) {
        double fx = (rx[2 * r] - x0) / dx - 0.5, fz = (rx[2 * r + 1] - z0) / dz - 0.5;
        int ix = (int)floor(fx), iz = (int)floor(fz);
        if (ix < 0) ix = 0;
        if (ix > nx - 2) ix = nx - 2;
        if (iz < 0) iz = 0;
        if (iz > nz - 2) iz = nz - 2;
        double tx = fx - ix, tz = fz - iz;
        if (tx < 0.0) tx = 0.0;
        if (tx > 1.0) tx = 1.0;
        if (tz < 0.0) tz = 0.0;
        if (tz > 1.0) tz = 1.0;
        double w00 = (1 - tx) * (1 - tz), w10 = tx * (1 - tz), w01 = (1 - tx) * tz, w11 = tx * tz;
        double best = NAN;
        for (int k = 0; k < nth; ++k) {
            int k1 = (k + 1) % nth;
            double ph[2], ps[2];
            for (int e = 0; e < 2; ++e) {
                long b = (long)(e ? k1 : k) * nxz + (long)ix * nz + iz;
                const double *P = U + S_PHI * n + b, *S = U + S_PSI * n + b;
                ph[e] = w00 * P[0] + w10 * P[nz] + w01 * P[1] + w11 * P[nz + 1];
                ps[e] = w00 * S[0] + w10 * S[nz] + w01 * S[1] + w11 * S[nz + 1];
            }
            if (!(ph[0] == 0.0 || ph[0] * ph[1] < 0.0)) continue;
            double t = ph[0] / (ph[0] - ph[1]);
            double v = ps[0] + t * (ps[1] - ps[0]);
            if (v > 0.0 && (isnan(best) || v < best)) best = v;
        }
        tout[r] = best;
    }
    return 0;
}

/* ======================================================================== */
/* Paraxial depth march (section 3 eqs. 13-15, section 4 eqs. 16-24, the
 * level set of eq. 35).
 *
 * Depth z is the evolution variable and the phase space is (x, theta), with
 * theta restricted to (-theta_max, theta_max) where rays go down (eq. 13).
 * With the stationary Liouville velocity V = d(x, z, theta)/dtau (eqs. 7-12):
 *   u = dx/dz = V_x / V_z,   w = dtheta/dz = V_theta / V_z   (eqs. 14, 15, 17, 18)
 * and every field U of (X, vartheta, tau, C, B) obeys
 *   U_z + u U_x + w U_theta = S                                (eqs. 16, 19, 21)
 *   S_X = S_vartheta = 0,  S_tau = 1 / V_z  (= p . dx/dz of eq. 19, since p . V = 1),
 *   S_(C,B) = (A / V_z) (C, B)  (the ray-normal dynamic ray tracing of the
 *                                 stationary system, per unit depth)
 * with data on the first depth row (eqs. 20, 24):
 *   X = x, vartheta = theta, tau = 0, C = cos(theta) + sin(theta) u = v / V_z,
 *   B = i beta C.
 * Grid: x_i = x0 + (i + 1/2) dx, z_n = z0 + (n + 1/2) dz,
 *       theta_k = -theta_max + (k + 1/2) dtheta, dtheta = 2 theta_max / nth.
 * Plane order of the oracle state: X, vartheta, tau, Re C, Im C, Re B, Im B,
 * Phi.  Phi is the continuous phase of C along the ray (the KMAH phase):
 * with C' = (A11 C + A12 B) / V_z and A real, d(log C)/dz has the imaginary
 * part (A12 / V_z) Im(B / C), so Phi_z + u Phi_x + w Phi_theta =
 * (A12 / V_z) Im(B / C), Phi = 0 on the surface (C(0) > 0); exp(i Phi) =
 * C / |C| while Phi keeps counting past +-pi where the ray crosses caustics.
 * Velocity table pvel[n][7][k][i]: u, w, 1/V_z, A11/V_z, A12/V_z, A21/V_z, A22/V_z.
 */
#define P_X 0
#define P_VT 1
#define P_TAU 2
#define P_RC 3
#define P_IC 4
#define P_RB 5
#define P_IB 6
#define P_PH 7
#define NPAR 8

/* DRT coefficients of the depth march per unit depth, written in the
 * lateral frame of eqs. 21-23: C = dx/dgamma at fixed z, B = dp1/dgamma,
 *   C_z + u C_x + w C_th =  H_xp C + H_pp B,
 *   B_z + u B_x + w B_th = -H_xx C - H_xp B,
 * with eq. 23's substitution u1 = cos th + sin th dx/dz for anisotropic
 * media, N = dx/dz, v the phase velocity at th and v_x, v_xx its lateral
 * derivatives at fixed th:
 *   H_pp = v u1^3,  H_xp = u1^2 (v_x / v) N,
 *   H_xx = (u1 (v v_xx - 3 v_x^2) + u1^3 v_x^2) / v^3.
 * Two corrections of the printed eqs. 22-23 make this the exact linearised
 * depth march of an isotropic medium (h = sqrt(1/v^2 - p1^2), C' = -h_px C -
 * h_pp B, B' = h_xx C + h_xp B): H_pp carries u1^3 (printed u1^2) and the B
 * term of the C equation is +H_pp B (printed -H_pp B).  a[] = (a11, a12,
 * a21, a22) in C' = a11 C + a12 B, B' = a21 C + a22 B. */
static void paper23_drt(const double vj[10], double th, double u, double a[4])
{
    double v = vj[0], vx = vj[1], vxx = vj[4];
    double u1 = cos(th) + sin(th) * u;
    double hpp = v * u1 * u1 * u1;
    double hxp = u1 * u1 * (vx / v) * u;
    double hxx = (u1 * (v * vxx - 3.0 * vx * vx) + u1 * u1 * u1 * vx * vx) / (v * v * v);
    a[0] = hxp;
    a[1] = hpp;
    a[2] = -hxx;
    a[3] = -hxp;
}

int oc_paper23_drt(const double *vj, double th, double u, double *a)
{
    paper23_drt(vj, th, u, a);
    return 0;
}

int oc_pvelocity(int nx, int nz, int nth, double dx, double dz, double theta_max, int drt, const double *tab,
                 double *pvel, double *rate_out)
{
    (void)dz;
    double dth = 2.0 * theta_max / nth;
    long plane = (long)nth * nx;
    double rate = 0.0;
    int bad = 0;
#pragma omp parallel for reduction(max : rate) reduction(| : bad) schedule(static)
    for (int n = 0; n < nz; ++n)
        for (int k = 0; k < nth; ++k) {
            double th = -theta_max + (k + 0.5) * dth;
            for (int i = 0; i < nx; ++i) {
                long c2 = (long)i * nz + n;
                double vj[10], V[3], A[4];
                vjet_flat(phase_velocity_jet(tab + c2 * NFLD * NTAY, th), vj);
                oc_va(vj, th, V, A);
                if (!(V[1] > 0.0)) {
                    bad = 1;
                    continue;
                }
                double *o = pvel + (long)n * 7 * plane + (long)k * nx + i;
                o[0] = V[0] / V[1];
                o[plane] = V[2] / V[1];
                o[2 * plane] = 1.0 / V[1];
                if (drt) { /* eqs. 21-23 in the lateral frame, already per unit depth */
                    double a[4];
                    paper23_drt(vj, th, o[0], a);
                    for (int q = 0; q < 4; ++q) o[(3 + q) * plane] = a[q];
                } else {   /* the ray-normal pair of the phase-space system divided by dz/dtau */
                    for (int q = 0; q < 4; ++q) o[(3 + q) * plane] = A[q] / V[1];
                }
                double r = fabs(o[0]) / dx + fabs(o[plane]) / dth;
                if (r > rate) rate = r;
            }
        }
    *rate_out = rate; /* max (|u| / dx + |w| / dtheta) over the table */
    return bad ? -1 : 0;
}

/* Surface data of level 0 (eqs. 20, 24): X = x, vartheta = theta, tau = 0,
 * C = u1 = cos theta + sin theta u and B = i eps C with the beam parameter
 * eps = beta (the ray-normal pair: B an angle, B / C in 1/m) or, for the
 * lateral-frame DRT of eqs. 21-23 (drt = 1, B / C a traveltime Hessian in
 * s/m^2), eps = beta / v with v = u1 / S_tau the phase velocity (p . V = 1),
 * i.e. B = i beta S_tau.  pvel0: the coefficient planes of level 0. */
int oc_pinit(int nx, int nth, double x0, double dx, double theta_max, const double *pvel0, double beta, int drt,
             double *U)
{
    double dth = 2.0 * theta_max / nth;
    long plane = (long)nth * nx;
    for (int k = 0; k < nth; ++k) {
        double th = -theta_max + (k + 0.5) * dth;
        for (int i = 0; i < nx; ++i) {
            long c = (long)k * nx + i;
            double c0 = cos(th) + sin(th) * pvel0[c];
            U[P_X * plane + c] = x0 + (i + 0.5) * dx;
            U[P_VT * plane + c] = th;
            U[P_TAU * plane + c] = 0.0;
            U[P_RC * plane + c] = c0;
            U[P_IC * plane + c] = 0.0;
            U[P_RB * plane + c] = 0.0;
            U[P_IB * plane + c] = drt ? beta * pvel0[2 * plane + c] : beta * c0;
            U[P_PH * plane + c] = 0.0;
        }
    }
    return 0;
}

/* value of a line of n values (stride st) at index idx, ghosts by linear
 * extrapolation u_{-m} = (m+1) u_0 - m u_1 at either end */
static double pline(const double *u, long st, int n, int idx)
{
    if (idx < 0) return (1 - idx) * u[0] + idx * u[st];
    if (idx > n - 1) {
        int e = idx - (n - 1);
        return (e + 1) * u[(long)(n - 1) * st] - e * u[(long)(n - 2) * st];
    }
    return u[(long)idx * st];
}

/* value at index idx of a line whose in-range values are u and whose ghosts
 * extend the line of the fixed data b (linear, from the two end values) */
static double pline_b(const double *u, const double *b, long st, int n, int idx)
{
    if (idx < 0) return (1 - idx) * b[0] + idx * b[st];
    if (idx > n - 1) {
        int e = idx - (n - 1);
        return (e + 1) * b[(long)(n - 1) * st] - e * b[(long)(n - 2) * st];
    }
    return u[(long)idx * st];
}

/* L = -(u D_x U + w D_theta U) + S at fractional depth s of the level
 * interval (velocity table (1 - s) pv0 + s pv1); WENO5 upwind on both axes,
 * D- where the coefficient is >= 0.  Ghosts beyond the x ends and the
 * aperture ends hold the surface data Ub extended linearly, fixed in depth:
 * a ray entering through a side or an aperture edge carries that data (its
 * take-off angle lies outside the aperture at the aperture edges), the
 * reading that keeps the march bounded at inflow edges where extending the
 * marched state grows without bound. */
static void prhs(int nx, int nth, double dx, double dth, const double *pv0, const double *pv1, double s,
                 const double *U, const double *Ub, double *L)
{
    long plane = (long)nth * nx;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nth; ++k)
        for (int i = 0; i < nx; ++i) {
            long c = (long)k * nx + i;
            double cv[7];
            for (int q = 0; q < 7; ++q) cv[q] = (1.0 - s) * pv0[q * plane + c] + s * pv1[q * plane + c];
            double cx = cv[0] / dx, ct = cv[1] / dth;
            double Lf[NPAR];
            for (int f = 0; f < NPAR; ++f) {
                const double *u = U + f * plane;
                double w7[7];
                for (int m = -3; m <= 3; ++m)
                    w7[m + 3] = pline_b(u + (long)k * nx, Ub + f * plane + (long)k * nx, 1, nx, i + m);
                double Dx = oc_weno(w7, cx >= 0.0);
                for (int m = -3; m <= 3; ++m) w7[m + 3] = pline_b(u + i, Ub + f * plane + i, nx, nth, k + m);
                double Dt = oc_weno(w7, ct >= 0.0);
                Lf[f] = -(cx * Dx + ct * Dt);
            }
            Lf[P_TAU] += cv[2];
            Lf[P_RC] += cv[3] * U[P_RC * plane + c] + cv[4] * U[P_RB * plane + c];
            Lf[P_RB] += cv[5] * U[P_RC * plane + c] + cv[6] * U[P_RB * plane + c];
            Lf[P_IC] += cv[3] * U[P_IC * plane + c] + cv[4] * U[P_IB * plane + c];
            Lf[P_IB] += cv[5] * U[P_IC * plane + c] + cv[6] * U[P_IB * plane + c];
            {
                double rc = U[P_RC * plane + c], ic = U[P_IC * plane + c];
                double rb = U[P_RB * plane + c], ib = U[P_IB * plane + c];
                Lf[P_PH] += cv[4] * (ib * rc - rb * ic) / (rc * rc + ic * ic);
            }
            for (int f = 0; f < NPAR; ++f) L[f * plane + c] = Lf[f];
        }
}

/* March from level 0 (Uall[0] holds the start) to level nz - 1: each level
 * interval dz is nsub SSP-RK3 steps of dz / nsub, stage depths s, s + h,
 * s + h / 2 (h = 1 / nsub); Ub: the surface data the ghosts extend.  Every
 * level is kept: Uall[n][7][k][i]. */
int oc_pmarch(int nx, int nz, int nth, double dx, double dz, double theta_max, const double *pvel, int nsub,
              const double *Ub, double *Uall)
{
    double dth = 2.0 * theta_max / nth, h = 1.0 / nsub, dl = dz * h;
    long plane = (long)nth * nx, lev = NPAR * plane;
    double *U = (double *)malloc(sizeof(double) * lev), *U1 = (double *)malloc(sizeof(double) * lev);
    double *U2 = (double *)malloc(sizeof(double) * lev), *L = (double *)malloc(sizeof(double) * lev);
    if (!U || !U1 || !U2 || !L) { free(U); free(U1); free(U2); free(L); return -2; }
    memcpy(U, Uall, sizeof(double) * lev);
    for (int n = 0; n + 1 < nz; ++n) {
        const double *pv0 = pvel + (long)n * 7 * plane, *pv1 = pv0 + 7 * plane;
        for (int j = 0; j < nsub; ++j) {
            double s = j * h;
            prhs(nx, nth, dx, dth, pv0, pv1, s, U, Ub, L);
            for (long q = 0; q < lev; ++q) U1[q] = U[q] + dl * L[q];
            prhs(nx, nth, dx, dth, pv0, pv1, s + h, U1, Ub, L);
            for (long q = 0; q < lev; ++q) U2[q] = 0.75 * U[q] + 0.25 * (U1[q] + dl * L[q]);
            prhs(nx, nth, dx, dth, pv0, pv1, s + 0.5 * h, U2, Ub, L);
            for (long q = 0; q < lev; ++q) U[q] = U[q] / 3.0 + 2.0 / 3.0 * (U2[q] + dl * L[q]);
        }
        memcpy(Uall + (long)(n + 1) * lev, U, sizeof(double) * lev);
    }
    free(U); free(U1); free(U2); free(L);
    return 0;
}

/* Gaussian-beam superposition from the depth march (eqs. 25-27, 33-35 in
 * the paper's own setting): for a surface source at x_s on level 0, the
 * Green's function on depth row n is the integral over take-off angle of the
 * beams on Gamma(z_n) = {X = x_s} (eq. 35).  On the (x, theta) slice the
 * take-off-angle measure of a cell is
 *   d vartheta = delta_h(d) |det d(X, vartheta)/d(x, theta)| / |grad X| dx dtheta,
 * d = (X - x_s) / |grad X| the signed distance to Gamma with theta scaled by
 * lambda = dx / dtheta (width h = 2 dx), derivatives by 4th-order central
 * differences (ghosts as in the march).  Each beam contributes, as a row of
 * the phase-space superposition,
 *   sqrt(v / C) sqrt(u1 / s) s^-1 d vartheta exp(i omega T),
 * sqrt(v / C) on the branch the ray carries: the principal root times
 * (-1)^k, k = round((Phi - arg C) / 2 pi) full turns of the continuous phase
 * Phi (the KMAH phase: the principal root alone is wrong past a second
 * caustic; arg C keeps the phase consistent with M = B / C),
 *   T = tau + p_s (X - x_s) + p1 (x0 - x) + 1/2 M_row (x0 - x)^2,
 * with the traveltime Hessian of the phase-space beam sum (M = B C^-1 in the
 * ray-normal frame), and the whole scaled by i / (4 pi).  Reading: the depth
 * march starts the beam of take-off angle vartheta with C(0) = u1 =
 * cos + sin u (eq. 24), the point-source data with C(0) = s (the 2D beam
 * weight); both solve the same linear transport, so sqrt(u1 / s) (medium
 * frozen at the source, level 0) turns one normalisation into the other,
 * and s^-1 is the weight the phase-space sum's take-off-angle measure
 * carries (its Im(C, B) = beta s (dn, dtheta_perp) per unit angle).
 * Only cells whose transported take-off angle lies inside the aperture are
 * beams (the others hold data that entered at an aperture edge, not a ray
 * from the source), and, as in the phase-space sum, only those with
 * Im(M_row) > 0.  A cell within the smoothed delta but off Gamma carries the
 * ray from X, not from x_s: its traveltime is moved to the source to first
 * order by the
 * take-off slowness p_s = sin(vartheta) / v_s (the point-source data of the
 * phase-space march carries this term in psi itself).  lin != 0: eq. 28's
 * linear coefficient.  comp >= 0: component (i, k) = (comp / 2, comp % 2)
 * (0 = x, 1 = z) of the Green's tensor, each beam weighted by the qP
 * polarisations g_i at the cell and g_k at the source for the take-off angle
 * (eqs. 31-32); comp < 0: the scalar sum.  Row 0 (the source row) is 0.
 * Output out[w][ix][n][re/im].                                             */
int oc_pbeam_sum(int nx, int nz, int nth, double x0, double z0, double dx, double dz, double theta_max,
                 const double *tab, const double *Uall, double xs, int lin, int drt, int comp, const double *omegas,
                 int nw, double *out)
{
    double dth = 2.0 * theta_max / nth, lam = dx / dth, h = 2.0 * dx;
    long plane = (long)nth * nx, lev = NPAR * plane;
    double ms[NFLD];
    for (int m = 0; m < NFLD; ++m) ms[m] = bilin(tab, nx, nz, dx, dz, x0, z0, xs, z0 + 0.5 * dz, m);
    int cap = 8 * (nx + nth) + 64, overflow = 0;
    beamrec *rows = (beamrec *)malloc(sizeof(beamrec) * (long)nz * cap);
    int *nrow = (int *)calloc(nz, sizeof(int));
    if (!rows || !nrow) { free(rows); free(nrow); return -2; }
#pragma omp parallel for schedule(dynamic) reduction(| : overflow)
    for (int n = 1; n < nz; ++n) {
        const double *U = Uall + (long)n * lev;
        const double *X = U + P_X * plane, *T = U + P_VT * plane;
        for (int k = 0; k < nth; ++k)
            for (int i = 0; i < nx; ++i) {
                long c = (long)k * nx + i;
                double tau = U[P_TAU * plane + c];
                if (!(tau > 0.0)) continue;
#define DX(f) ((pline((f) + (long)k * nx, 1, nx, i - 2) - 8.0 * pline((f) + (long)k * nx, 1, nx, i - 1) + \
                8.0 * pline((f) + (long)k * nx, 1, nx, i + 1) - pline((f) + (long)k * nx, 1, nx, i + 2)) / (12.0 * dx))
#define DT(f) ((pline((f) + i, nx, nth, k - 2) - 8.0 * pline((f) + i, nx, nth, k - 1) + \
                8.0 * pline((f) + i, nx, nth, k + 1) - pline((f) + i, nx, nth, k + 2)) / (12.0 * dth))
                double Xx = DX(X), Xt = DT(X), Tx = DX(T), Tt = DT(T);
#undef DX
#undef DT
                double gX = sqrt(Xx * Xx + (Xt / lam) * (Xt / lam));
                double d = (X[c] - xs) / gX;
                if (!(fabs(d) < h)) continue;
                double vt0 = T[c];
                if (!(fabs(vt0) < theta_max)) continue; /* not a ray that left the source inside the aperture */
                double meas = delta_h(d, h) * fabs(Xx * Tt - Xt * Tx) / gX * dx * dth;
                double th = -theta_max + (k + 0.5) * dth, sn = sin(th), cs = cos(th);
                double vj[10], V[3], A[4];
                vjet_flat(phase_velocity_jet(tab + ((long)i * nz + n) * NFLD * NTAY, th), vj);
                oc_va(vj, th, V, A);
                double v = vj[0], vx = vj[1], vz = vj[2], vt = vj[3];
                double nv = sqrt(V[0] * V[0] + V[1] * V[1]), gx = V[0] / nv, gz = V[1] / nv;
                double gp[2] = {gz, -gx};
                double complex C = U[P_RC * plane + c] + I * U[P_IC * plane + c];
                double complex B = U[P_RB * plane + c] + I * U[P_IB * plane + c];
                double pth[2] = {cs / v - sn * vt / (v * v), -sn / v - cs * vt / (v * v)};
                double gp_pth = gp[0] * pth[0] + gp[1] * pth[1];
                double gp_dxp_gp = -(gp[0] * sn + gp[1] * cs) * (vx * gp[0] + vz * gp[1]) / (v * v);
                double q[2] = {-vx / (v * nv), -vz / (v * nv)};
                double gq = gx * q[0] + gz * q[1], gpq = gp[0] * q[0] + gp[1] * q[1];
                double complex Mn = (gp_pth * B + gp_dxp_gp * C) / C;
                /* source normalisation at the take-off angle */
                double vs, gps[2], ps[2], A12s, ss;
                source_data(ms, vt0, &vs, gps, ps, &A12s, &ss);
                double u1 = cos(vt0) - sin(vt0) * gps[1] / gps[0];
                beamrec r;
                r.pos = x0 + (i + 0.5) * dx;
                r.psi = tau + ps[0] * (X[c] - xs);
                r.p = lin ? oc_lin28(sn, cs, gx / gz, v) : sn / v;
                r.M = Mn * gz * gz + 2.0 * gpq * gx * gz + gq * gx * gx;
                /* sqrt(v / C) on the branch the ray carries: the principal root turned by
                 * the number of full turns between the continuous phase Phi and arg C */
                double turns = nearbyint((U[P_PH * plane + c] - carg(C)) / (2.0 * M_PI));
                double sgn = fmod(fabs(turns), 2.0) == 1.0 ? -1.0 : 1.0;
                r.amp = sgn * csqrt(v / C) * sqrt(u1 / ss) / ss * meas;
                if (drt) {
                    /* lateral frame: the row Hessian is B / C itself; the lateral
                     * displacement of a ray is its normal one over g_z, both started
                     * at u1, so sqrt(v / C_normal) = sqrt(v / C) sqrt(g_z0 / g_z) */
                    r.M = B / C;
                    r.amp *= sqrt(gps[0] / gz);
                }
                if (comp >= 0) { /* g_i at the cell (phase angle theta) times g_k at the source (vartheta) */
                    double mr[NFLD], gr[2], gs[2];
                    for (int m = 0; m < NFLD; ++m) mr[m] = tab[(((long)i * nz + n) * NFLD + m) * NTAY];
                    oc_qp_polarization(mr, th, gr);
                    oc_qp_polarization(ms, vt0, gs);
                    r.amp *= gr[comp / 2] * gs[comp % 2];
                }
                if (!(cimag(r.M) > 0.0)) continue;
                if (nrow[n] < cap) rows[(long)n * cap + nrow[n]++] = r; else overflow = 1;
            }
    }
    const double complex W = I / (4.0 * M_PI);
    memset(out, 0, sizeof(double) * 2 * (long)nw * nx * nz);
#pragma omp parallel for collapse(2) schedule(static)
    for (int w = 0; w < nw; ++w)
        for (int n = 1; n < nz; ++n) {
            double om = omegas[w];
            for (int ix = 0; ix < nx; ++ix) {
                double xo = x0 + (ix + 0.5) * dx;
                double complex G = 0.0;
                for (int r = 0; r < nrow[n]; ++r) {
                    const beamrec *b = &rows[(long)n * cap + r];
                    double dd = xo - b->pos;
                    double complex Tc = b->psi + b->p * dd + 0.5 * b->M * dd * dd;
                    if (0.5 * om * cimag(b->M) * dd * dd > 16.0) continue;
                    G += b->amp * cexp(I * om * Tc);
                }
                G *= W;
                long o = (((long)w * nx + ix) * nz + n) * 2;
                out[o] = creal(G);
                out[o + 1] = cimag(G);
            }
        }
    free(rows); free(nrow);
    return overflow ? -3 : 0;
}

/* First arrival at every (x_i, z_n) from a source at x = xs on the first
 * depth row: roots in theta of X(z_n, x_i, .) - xs between adjacent theta
 * nodes (eq. 35's Gamma = {X = x_s}; linear interpolation of X and tau)
 * whose two nodes carry take-off angles inside the aperture (rays from the
 * source, not data entering at an aperture edge), the smallest tau > 0
 * among them; NaN where there is none.  T[s][n][i]. */
int oc_ppick(int nx, int nz, int nth, double theta_max, const double *Uall, const double *xs, int nsrc, double *T)
{
    long plane = (long)nth * nx, lev = NPAR * plane;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < nz; ++n)
        for (int s = 0; s < nsrc; ++s)
            for (int i = 0; i < nx; ++i) {
                const double *X = Uall + (long)n * lev + P_X * plane + i;
                const double *tau = Uall + (long)n * lev + P_TAU * plane + i;
                const double *vt = Uall + (long)n * lev + P_VT * plane + i;
                double best = NAN;
                for (int k = 0; k + 1 < nth; ++k) {
                    double f0 = X[(long)k * nx] - xs[s], f1 = X[(long)(k + 1) * nx] - xs[s];
                    if (!(f0 == 0.0 || f0 * f1 < 0.0)) continue;
                    if (!(fabs(vt[(long)k * nx]) < theta_max && fabs(vt[(long)(k + 1) * nx]) < theta_max)) continue;
                    double t = f0 / (f0 - f1);
                    double v = tau[(long)k * nx] + t * (tau[(long)(k + 1) * nx] - tau[(long)k * nx]);
                    if (v > 0.0 && (isnan(best) || v < best)) best = v;
                }
                T[((long)s * nz + n) * nx + i] = best;
            }
    return 0;
}
