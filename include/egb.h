/*
 * egb.h - C ABI of the MI355X Eulerian Gaussian beam library (libegb.so).
 *
 * The library marches the stationary phase-space Liouville system of the
 * anisotropic Eulerian Gaussian beam method (Huang, arXiv 2006.11945) on a
 * regular (x, z, theta) grid and superposes the beams on the Cartesian grid.
 *
 * Conventions for every call:
 *  - Buffers are caller-owned DEVICE pointers unless marked "host".  The
 *    library never allocates device memory: scratch space comes from the
 *    caller, sized by egb_workspace_size().
 *  - Calls are asynchronous and ordered on `stream` (NULL = default stream)
 *    unless stated otherwise.
 *  - Arguments are validated on the host before anything is launched; on an
 *    error nothing is launched and an egb_status < 0 is returned.  No C++
 *    exception crosses this interface.
 *  - Device pointers must be 16-byte aligned.
 *  - x is horizontal, z is depth (positive down); theta is the phase angle
 *    measured from +z toward +x, so the slowness is p = (sin, cos)(theta)/v
 *    (eq. 7).  Cell (i, j, k) sits at x = x0 + (i+1/2) dx, z = z0 + (j+1/2) dz,
 *    theta = k * 2 pi / nth.  Phase-space planes are stored [theta][x][z],
 *    z fastest, each plane padded to egb_plane_stride() elements.
 */
#ifndef EGB_H
#define EGB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EGB_OK = 0,
    EGB_EINVAL = -1,        /* bad argument: null, size, alignment, dtype, range */
    EGB_ECFL = -2,          /* dt not positive and finite, or dt > dt_cfl (1 + 1e-12) of the velocity */
    EGB_EWORKSPACE = -3,    /* workspace too small, or a beam list overflowed it */
    EGB_EHIP = -4,          /* a HIP launch or runtime call failed */
    EGB_ENONFINITE = -5,    /* a non-finite value was produced */
    EGB_EUNSUPPORTED = -6   /* valid request the library does not implement */
} egb_status;

/* Arithmetic type of the phase-space planes.  EGB_F32: six planes in float,
 * traveltime psi in double (FP64 traveltime accumulation); EGB_F64: all
 * planes in double. */
typedef enum { EGB_F32 = 0, EGB_F64 = 1 } egb_dtype;

/* State planes (order in memory).  phi1: ray-family level set, the signed
 * miss distance of the ray from the source (X - x_s of eqs. 19-20, 35);
 * (C, B): complex dynamic ray tracing pair of eq. 21 in the ray-normal frame;
 * phase: arg C continued along the ray (its Liouville equation follows from
 * eq. 21: d(arg C)/dtau = A12 Im(B / C)), which picks the branch of
 * sqrt(1 / C) in the beam amplitude past caustics (the KMAH index: the
 * number of full turns between it and the principal arg C);
 * psi: traveltime (tau of eq. 19).  The planes before EGB_PSI are in the grid
 * dtype, psi is double. */
enum { EGB_PHI1 = 0, EGB_RE_C = 1, EGB_IM_C = 2, EGB_RE_B = 3, EGB_IM_B = 4, EGB_PHASE = 5, EGB_PSI = 6,
       EGB_NSTATE = 7 };

/* Velocity planes (order in memory): the Liouville velocity V = (dx/dtau,
 * dz/dtau, dtheta/dtau) of eqs. 8, 9, 12 and the 2x2 ray-normal dynamic ray
 * tracing matrix A (row major), all in the grid dtype. */
enum { EGB_VX = 0, EGB_VZ = 1, EGB_VT = 2, EGB_A11 = 3, EGB_A12 = 4, EGB_A21 = 5, EGB_A22 = 6, EGB_NVEL = 7 };

/* Medium table (coeff2d): float64 [EGB_NFIELD][EGB_NTAYLOR][nx][nz]; fields
 * a11, a33, b = a13 + a55, a55 (density-normalised moduli, eq. 5) and tilt nu;
 * Taylor slots f, f_x, f_z, f_xx, f_xz, f_zz (4th-order differences). */
enum { EGB_NFIELD = 5, EGB_NTAYLOR = 6 };

/* Workspace queries (egb_workspace_size op argument). */
enum { EGB_OP_VELOCITY = 0, EGB_OP_STEP = 1, EGB_OP_BEAM = 2, EGB_OP_ADJOINT = 3, EGB_OP_PARAXIAL = 4,
       EGB_OP_PBEAM = 5 };

typedef struct {
    int32_t nx, nz, nth; /* cells in x, z (>= 8) and theta (>= 8) */
    int32_t dtype;       /* egb_dtype */
    double x0, z0;       /* domain origin (m) */
    double dx, dz;       /* cell size (m), > 0 */
} egb_grid;

/* Thomsen-parameter medium, device float64 arrays [nx][nz]; tilt may be NULL
 * (VTI).  vs_ratio = vs0/vp0 fixes a55 (0 <= vs_ratio < 1). */
typedef struct {
    const double *vp0, *eps, *delta, *tilt;
    double vs_ratio;
} egb_medium;

/* Point source at (xs, zs); r0 is the radius of the source ball whose cells
 * hold the point-source data; beta > 0 the initial beam parameter
 * (B(0) = i beta C(0), eq. 24).  lin_variant selects the linear phase
 * coefficient of the beam sum (read by egb_beam_sum only):
 * EGB_LIN_EXACT, p1 = sin(theta)/v of eq. 7, or EGB_LIN_PAPER28, eq. 28's
 * coefficient sqrt(s (s u^2 + 2 c u - s)) / (v (c + s u)), u = V_x/V_z
 * (s, c = sin, cos theta; the sign of p1 restored, a negative radicand
 * counted as 0; columns mirrored), an approximation away from isotropy. */
enum { EGB_LIN_EXACT = 0, EGB_LIN_PAPER28 = 1 };
typedef struct {
    double xs, zs, r0, beta;
    int32_t lin_variant;
} egb_source;

/* ------------------------------------------------------------------ sizes */
size_t egb_plane_stride(const egb_grid *g);         /* elements per plane */
size_t egb_coeff2d_bytes(const egb_grid *g);
size_t egb_vel3d_bytes(const egb_grid *g);
size_t egb_state_bytes(const egb_grid *g);
size_t egb_state_plane_offset(const egb_grid *g, int32_t plane); /* bytes */
size_t egb_workspace_size(const egb_grid *g, int32_t op);        /* bytes; 0 on bad args */
size_t egb_bdata_bytes(const egb_grid *g);          /* boundary data of the march */

/* ------------------------------------------------------------------ calls */

/* Medium -> Christoffel table -> Liouville velocity and DRT matrix.
 * Paper: eqs. 3-5 (qP eigenvalue of Gamma_ik = a_ijkl p_j p_l with
 * a = c/rho), eqs. 8-9 (dx/dtau, dz/dtau = grad_p G / 2, the group
 * velocity), eq. 12 (dtheta/dtau, Hamiltonian sign), eq. 21 (the linearised
 * flow, in the ray-normal frame).
 * In:  g, m (device float64 [nx][nz] each).
 * Out: coeff2d (egb_coeff2d_bytes), vel3d (egb_vel3d_bytes, grid dtype),
 *      *dt_cfl (host) = 0.5 / max(|V_x|/dx + |V_z|/dz + |V_theta|/dtheta).
 * work: egb_workspace_size(g, EGB_OP_VELOCITY) bytes.
 * Synchronises `stream` once (to return dt_cfl).  EGB_ENONFINITE if the
 * medium yields a non-finite velocity.  The library records dt_cfl for the
 * buffer vel3d and this grid (host memory, process-wide, mutex-guarded, at
 * most 4096 buffers: the least recently written record makes room): every
 * call that marches with vel3d refuses dt > dt_cfl (1 + 1e-12) with
 * EGB_ECFL before launching anything, and returns EGB_EINVAL for a buffer
 * without a record for its grid. */
egb_status egb_hamiltonian_velocity(const egb_grid *g, const egb_medium *m, void *coeff2d, void *vel3d,
                                    double *dt_cfl, void *work, size_t work_bytes, hipStream_t stream);

/* The CFL limit recorded for vel3d on grid g (host out); EGB_EINVAL if there
 * is none.  Host only: touches no device. */
egb_status egb_velocity_dt_cfl(const egb_grid *g, const void *vel3d, double *dt_cfl);

/* Record the CFL limit of a velocity buffer filled by other means (for
 * example a copy of another buffer of the same medium): dt_cfl > 0 and
 * finite, 0.5 / max(|V_x|/dx + |V_z|/dz + |V_theta|/dtheta) over the buffer's
 * cells.  Host only. */
egb_status egb_declare_velocity(const egb_grid *g, const void *vel3d, double dt_cfl);

/* Point-source data (eqs. 20 and 24 read for a point source): with the medium
 * frozen at the source (bilinear in coeff2d), every cell gets
 * phi1 = (x - xs).g_perp(theta), psi = p(theta).(x - xs),
 * C = s (1 + i beta A12 psi), B = i beta s, s = (sqrt(v)/W)^(2/3),
 * W = a33/v^2 (the beam weight of eqs. 31-33 redone in 2D),
 * phase = arg C = atan(beta A12 psi) (s > 0).
 * Out: state (egb_state_bytes). */
egb_status egb_init_state(const egb_grid *g, const void *coeff2d, const egb_source *src, void *state,
                          hipStream_t stream);

/* Boundary data of the march: the values of the six ghost cells beyond each
 * end of every x line and z line, per state plane, taken from the point-source
 * data and extended linearly, u(-m) = (m+1) u(0) - m u(1) for m = 1, 2, 3 (and
 * the mirror image at the far end).  The march holds these values fixed, a
 * Dirichlet condition like the source ball (the reading of the boundary that
 * eqs. 16-21 leave open: the point-source data is the solution of the
 * homogeneous problem, so it is what enters through the edges).
 * In: state holding the point-source data (egb_init_state).
 * Out: bdata, egb_bdata_bytes(g) bytes.  Layout per plane (the six planes
 * before EGB_PSI in the grid dtype, then psi in double, each padded to egb_bdata_plane_stride()
 * elements): x ghosts [theta][6][nz], then z ghosts [theta][nx][6], ghost
 * slots 0..2 at positions -3..-1 and 3..5 at n, n+1, n+2 of the line. */
size_t egb_bdata_plane_stride(const egb_grid *g);
egb_status egb_boundary_data(const egb_grid *g, const void *state, void *bdata, hipStream_t stream);

/* nsteps SSP-RK3 pseudo-time steps of U_t + V.grad U = S(U) (eqs. 16, 19, 21
 * multiplied by dz/dtau): WENO5 Hamilton-Jacobi upwind derivatives (for the
 * phase plane the fifth-order linear upwind derivative, the WENO5 stencils
 * at their linear weights), sources S_psi = 1, S_(C,B) = A (C, B),
 * S_phase = A12 Im(B / C); ghosts: x, z from bdata (egb_boundary_data),
 * theta periodic; cells within r0 of the source keep their values (Dirichlet
 * data).  In/out: state.  vel3d from egb_hamiltonian_velocity.
 * work: egb_workspace_size(g, EGB_OP_STEP) bytes (two RK stage buffers).
 * dt must be positive, finite and at most the CFL limit recorded for vel3d
 * (egb_hamiltonian_velocity) times 1 + 1e-12: EGB_ECFL otherwise, and
 * EGB_EINVAL if vel3d has no record for this grid; nothing is launched
 * then.  EGB_EUNSUPPORTED (nothing launched) for grids beyond the kernels'
 * 32-bit buffer offsets: the velocity planes, the grid-dtype state planes
 * and the psi plane must each stay below 4 GiB (FP32: up to about 153 M
 * cells, 512^3 included; FP64: about 76 M); the same limit holds for every
 * march below. */
egb_status egb_liouville_step(const egb_grid *g, const void *vel3d, const egb_source *src, const void *bdata,
                              void *state, void *work, size_t work_bytes, double dt, int32_t nsteps,
                              hipStream_t stream);

/* Eulerian Gaussian beam superposition (eqs. 25-27, 33-35).  For every
 * output cell (x0, z0) and frequency omega:
 *   G = (i/4pi) [ sum_row w A dtheta exp(i omega T) + sum_col (1-w) A dtheta exp(i omega T) ]
 * over the phase cells of the same row / column on Gamma = {phi1 = 0, psi > 0}
 * (smoothed delta of width 2 dx), T = psi + p1 (x0 - x) + M (x0 - x)^2 / 2,
 * A = sqrt(v / C) on the ray's branch: the principal root times (-1)^k, k
 * the nearest whole number of turns in (phase - arg C) / 2 pi.
 * In: omegas (HOST float64 [nw], rad/s).  Out: out, complex [nw][nx][nz]
 * interleaved (re, im) in the grid dtype (complex64 / complex128).
 * Each row and column sums its beams in the order of their phase cells
 * (theta, then the position along the line), so the result is the same bit
 * for bit on every call, whatever order the beams were collected in.
 * work: egb_workspace_size(g, EGB_OP_BEAM).  Synchronises `stream` once;
 * EGB_EWORKSPACE if a per-row/column beam list overflowed. */
egb_status egb_beam_sum(const egb_grid *g, const void *coeff2d, const void *vel3d, const egb_source *src,
                        const void *state, const double *omegas, int32_t nw, void *out, void *work,
                        size_t work_bytes, hipStream_t stream);

/* egb_beam_sum for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the scratch (line counts, beam record lists
 * and their order) in a fixed array of egb_beam_scratch_bytes() = 128 MiB that the
 * library holds on every device it runs on until the process ends.  The
 * caller passes inputs and outputs as for egb_beam_sum; nothing is
 * allocated on the device or the host.  Each line list holds as many
 * records as fit in the array: EGB_EUNSUPPORTED (nothing launched) when
 * fewer than 256 records per line would fit (nx + nz above about 8000),
 * EGB_EWORKSPACE after the call when a line held more records than fit
 * (egb_beam_sum with a larger workspace then serves the grid).  All calls on
 * one device share its array: calls that overlap on one device (other host
 * threads, other streams) race and must not be made; the counts are cleared
 * by a kernel at the start of every call.  Synchronises `stream` once. */
size_t egb_beam_scratch_bytes(void);
egb_status egb_beam_sum_noalloc(const egb_grid *g, const void *coeff2d, const void *vel3d, const egb_source *src,
                                const void *state, const double *omegas, int32_t nw, void *out, hipStream_t stream);

/* One problem of a batched march (independent source, own grid and dt). */
typedef struct {
    egb_grid grid;
    const void *vel3d; /* from egb_hamiltonian_velocity for this grid */
    egb_source src;
    const void *bdata; /* egb_boundary_data of this problem */
    void *state;       /* in/out */
    double dt;         /* this problem's pseudo-time step */
} egb_problem;

/* Workspace for egb_liouville_step_batched: the device problem table plus two
 * RK stage buffers per problem.  0 on bad arguments. */
size_t egb_workspace_size_batched(const egb_problem *probs, int32_t nprob);

/* nsteps SSP-RK3 steps of every problem in `probs` (HOST array, nprob >= 1;
 * same dtype for all), the same scheme as egb_liouville_step.  All problems
 * advance together: each stage is ONE launch over the (tile, x) steps of all
 * grids, split into one contiguous range per block (by default one round of
 * resident blocks; see launch tuning), and the 3 * nsteps
 * launches are captured in one hipGraph replayed on `stream`.  Synchronises `stream` before returning
 * (the graph is destroyed).  Errors as egb_liouville_step; EGB_EINVAL if the
 * dtypes differ. */
egb_status egb_liouville_step_batched(const egb_problem *probs, int32_t nprob, int32_t nsteps, void *work,
                                      size_t work_bytes, hipStream_t stream);

/* First-arrival traveltime at receivers on the level set phi1 = 0 (eq. 35):
 * bilinear in (x, z) per theta plane, linear root of phi1 in theta, the
 * smallest interpolated psi > 0 (lowest theta on ties); NaN if no arrival.
 * In: rx (device float64 [nr][2] = x, z).  Out: t_out (device float64 [nr]). */
egb_status egb_pick_receivers(const egb_grid *g, const void *state, const double *rx, int32_t nr, double *t_out,
                              hipStream_t stream);

/* ----------------------------------------------- traveltime adjoint
 * The adjoint covers objectives that depend on the traveltime field, such as
 * the misfit J = sum_r (t_r - t_obs_r)^2 of egb_pick_receivers.  phi1 and psi
 * are transported without coupling to (C, B) (eqs. 16, 19), so only those two
 * planes carry adjoint values and only the Liouville velocity V (eqs. 8-9, 12)
 * is differentiated.  `lambda` buffers use the state layout
 * (egb_state_bytes; planes EGB_PHI1 and EGB_PSI are read and written, the
 * others are left untouched); `gvel` is [3][egb_plane_stride] in the grid
 * dtype (dJ/dV_x, dJ/dV_z, dJ/dV_theta), egb_gvel_bytes() bytes.  `bfold`
 * accumulates the sensitivity to the boundary data (the ghosts are fixed
 * extensions of the point-source data, so it reaches the medium through the
 * source): float64, egb_bfold_bytes() bytes, per line end and per source
 * cell within three cells of it, the weights of the two cells the ghosts are
 * extrapolated from.  The caller zero-initialises lambda, gvel and bfold
 * before the reverse sweep. */
size_t egb_gvel_bytes(const egb_grid *g);
size_t egb_bfold_bytes(const egb_grid *g);

/* egb_liouville_step restricted to the planes phi1 and psi (identical
 * values for them; the DRT planes are left untouched). */
egb_status egb_liouville_step_kinematic(const egb_grid *g, const void *vel3d, const egb_source *src,
                                        const void *bdata, void *state, void *work, size_t work_bytes, double dt,
                                        int32_t nsteps, hipStream_t stream);

/* Adjoint of egb_pick_receivers: lambda += sum_r tbar[r] d t_r / d(phi1, psi)
 * evaluated on `state` (the final state of the march).  rx, tbar: device
 * float64 [nr][2] and [nr]; receivers without an arrival contribute nothing. */
egb_status egb_pick_adjoint(const egb_grid *g, const void *state, const double *rx, int32_t nr,
                            const double *tbar, void *lambda, hipStream_t stream);

/* Exact discrete adjoint of one SSP-RK3 step of the march (WENO5 weights
 * differentiated, upwind sides frozen, ball cells pass their adjoint to the
 * step's start).  In: state_n = U^n (the step's start), lambda = dJ/dU^{n+1},
 * bdata as given to the forward march.  Out: lambda = dJ/dU^n; gvel += dJ/dV
 * and bfold += dJ/d(boundary data) through this step.  The step's inner
 * stages are recomputed from state_n.
 * work: egb_workspace_size(g, EGB_OP_ADJOINT). */
egb_status egb_adjoint_step(const egb_grid *g, const void *vel3d, const egb_source *src, const void *bdata,
                            const void *state_n, void *lambda, void *gvel, void *bfold, void *work,
                            size_t work_bytes, double dt, hipStream_t stream);

/* Medium gradient from the reverse sweep: dJ/dV (gvel, accumulated over all
 * steps) through the velocity (eqs. 3-5, 7-12) and the medium table, plus
 * dJ/dU^0 (lambda0) and the boundary-data sensitivity (bfold) through the
 * point-source data (medium frozen at the source), then the Thomsen map.
 * Out: grad, device float64 [4][nx][nz] = dJ/d(vp0, eps, delta, tilt).  The
 * time step is held fixed.  work: egb_workspace_size(g, EGB_OP_ADJOINT). */
egb_status egb_adjoint_medium(const egb_grid *g, const egb_medium *m, const void *coeff2d, const egb_source *src,
                              const void *gvel, const void *lambda0, const void *bfold, double *grad, void *work,
                              size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------ paraxial depth march
 * The paper's own formulation (eqs. 13-15, 16-24): the Liouville equations
 * divided by dz/dtau, marched in depth on (x, theta) slices with theta in
 * (-theta_max, theta_max), dtheta = 2 theta_max / nth, theta_k = -theta_max +
 * (k + 1/2) dtheta.  Level state (one per depth z_n, n = 0 .. nz-1): X (the
 * surface position of the ray, eqs. 17, 19), vartheta (its take-off angle),
 * C, B (eqs. 21-24), Phi (the continuous phase of C along the ray, the KMAH
 * phase: Phi_z + u Phi_x + w Phi_theta = (A12/V_z) Im(B/C), 0 on the
 * surface) and tau (traveltime, eq. 19).  One march serves every surface
 * source: the first arrival from a source at x_s is read on the level set
 * X = x_s (eq. 35).  Layout of one level: planes X, vartheta, Re C, Im C,
 * Re B, Im B, Phi in the grid dtype, then tau in float64, each [theta][x] (x
 * fastest) padded to egb_paraxial_plane_stride() elements; `levels` holds nz
 * levels of egb_paraxial_level_bytes() each.  The grid's nth counts the
 * theta nodes of the aperture; z0 is the depth of level 0 (the surface).
 * Coefficients `pvel`: [nz][7][stride] in the grid dtype, planes
 * u = V_x/V_z, w = V_theta/V_z, S_tau = 1/V_z, then the four DRT
 * coefficients per unit depth (C' = a11 C + a12 B, B' = a21 C + a22 B).
 *
 * DRT frame (drt_variant): EGB_DRT_EXACT transports the ray-normal pair of
 * the phase-space system (A11..A22 / V_z; B an angle).  EGB_DRT_PAPER23
 * transports the lateral-frame pair of eqs. 21-23 (C = dx, B = dp1 at fixed
 * depth; B / C is the row traveltime Hessian), with eq. 23's substitution
 * u1 = cos(theta) + sin(theta) u for anisotropic media: a11 = H_xp,
 * a12 = H_pp, a21 = -H_xx, a22 = -H_xp, H_pp = v u1^3, H_xp = u1^2 (v_x/v) u,
 * H_xx = (u1 (v v_xx - 3 v_x^2) + u1^3 v_x^2) / v^3 (v the phase velocity,
 * v_x, v_xx at fixed theta).  The printed eqs. 21-22 carry u1^2 in H_pp and
 * -H_pp B in the C equation; u1^3 and +H_pp B make the variant the exact
 * linearised depth march of an isotropic medium.  It exists to measure eq.
 * 23's approximation against EGB_DRT_EXACT; the same drt_variant must be
 * given to egb_paraxial_velocity, egb_paraxial_init and
 * egb_paraxial_beam_sum. */
enum { EGB_DRT_EXACT = 0, EGB_DRT_PAPER23 = 1 };
size_t egb_paraxial_plane_stride(const egb_grid *g);
size_t egb_paraxial_level_bytes(const egb_grid *g);
size_t egb_paraxial_vel_bytes(const egb_grid *g);

/* Medium table alone (the first part of egb_hamiltonian_velocity, eqs. 4-5).
 * Out: coeff2d (egb_coeff2d_bytes). */
egb_status egb_medium_table(const egb_grid *g, const egb_medium *m, void *coeff2d, hipStream_t stream);

/* Depth-march coefficients (eqs. 8-9, 12 and 21 divided by dz/dtau, eq. 13)
 * at every level and theta node from the medium table.  Out: pvel
 * (egb_paraxial_vel_bytes); *rate (host) = max(|u|/dx + |w|/dtheta), so that
 * nsub >= dz rate / 0.5 substeps per level keep the march stable.
 * 0 < theta_max <= pi/2; EGB_EINVAL if V_z <= 0 at some node (rays that do
 * not go down: beyond the paraxial range of this medium).  work:
 * egb_workspace_size(g, EGB_OP_VELOCITY).  Synchronises `stream` once. */
egb_status egb_paraxial_velocity(const egb_grid *g, const void *coeff2d, double theta_max, int32_t drt_variant,
                                 void *pvel, double *rate, void *work, size_t work_bytes, hipStream_t stream);

/* Surface data on level 0 (eqs. 20, 24 on the surface line): X = x,
 * vartheta = theta, tau = 0, C = cos(theta) + sin(theta) u, Phi = 0, and
 * B = i eps C with eq. 24's beam parameter read as eps = beta (1/m) for
 * EGB_DRT_EXACT and eps = beta / v (s/m^2, B / C a traveltime Hessian) for
 * EGB_DRT_PAPER23, i.e. B = i beta S_tau there. */
egb_status egb_paraxial_init(const egb_grid *g, const void *pvel, double theta_max, double beta, int32_t drt_variant,
                             void *levels, hipStream_t stream);

/* March levels 0 -> nz-1: each depth interval is nsub SSP-RK3 steps of
 * dz/nsub of U_z + u U_x + w U_theta = S (S_tau = 1/V_z, S_(C,B) = A/V_z (C,
 * B), the rest zero) with WENO5 upwind x and theta derivatives, the
 * coefficients linear in z between the two levels; x and theta ghosts hold
 * the surface data of level 0 extended linearly, fixed in depth (rays
 * entering through a side or an aperture edge carry it: their take-off
 * angle lies outside the aperture at the aperture edges).  In: level 0 of
 * levels (kept).  Out: levels 1 .. nz-1.  work: egb_workspace_size(g, EGB_OP_PARAXIAL).  The
 * 3 nsub (nz - 1) stage launches are queued in order on `stream` (the call
 * returns without waiting for them).
 * EGB_EUNSUPPORTED if one level (egb_paraxial_level_bytes) reaches 2 GiB. */
egb_status egb_paraxial_march(const egb_grid *g, const void *pvel, double theta_max, int32_t nsub, void *levels,
                              void *work, size_t work_bytes, hipStream_t stream);

/* Green's function of a surface source at xs (on level 0) from the depth
 * march: eq. 34 summed over Gamma(z_n) = {X = xs} (eq. 35) on every level.
 * Per cell of the (x, theta) slice, the take-off-angle measure is the smoothed
 * delta (width 2 dx) of the signed distance d = (X - xs)/|grad X| (theta
 * scaled by dx/dtheta) times |det d(X, vartheta)/d(x, theta)| / |grad X|; the
 * beam is sqrt(v/C) sqrt(u1/s)/s exp(i omega T) (sqrt(v/C) on the branch
 * of the ray: the principal root times (-1)^k, k the full turns between Phi
 * and arg C), T = tau + p_s (X - xs) +
 * p1 (x0 - x) + M (x0 - x)^2 / 2, with M the traveltime Hessian along the
 * row (M = B C^-1 across the ray), u1 = cos + sin u and s the 2D beam weight
 * at the take-off angle for the medium frozen at the source, p_s the
 * take-off slowness (the ray through a cell off Gamma starts at X), p1 as
 * chosen by lin_variant (see egb_source); the sum is scaled by i/(4 pi).
 * component = -1 gives this scalar sum; component = 2 i + k (0 = x, 1 = z)
 * gives G_ik of the qP Green's tensor (eqs. 31-32): every beam weighted by
 * g_i, the qP polarisation (unit eigenvector of the Christoffel matrix, eq. 4,
 * along the phase direction) at the cell, times g_k at the source for the
 * take-off angle.  drt_variant names the frame the levels were marched in:
 * for EGB_DRT_PAPER23 the row Hessian is M = B/C itself and the beam carries
 * sqrt(g_z0/g_z) (g_z, g_z0: the vertical component of the unit ray
 * direction at the cell and at the source), which turns the lateral C into
 * the normal one.
 * In: coeff2d (egb_medium_table), levels (egb_paraxial_march), omegas (HOST
 * float64 [nw], rad/s).  Out: out, complex [nw][nx][nz] (re, im) in the grid
 * dtype, row n = level n (row 0 is 0).  work: egb_workspace_size(g,
 * EGB_OP_PBEAM).  Synchronises `stream` once; EGB_EWORKSPACE if a level's
 * beam list overflowed. */
egb_status egb_paraxial_beam_sum(const egb_grid *g, const void *coeff2d, const void *levels, double theta_max,
                                 double xs, int32_t lin_variant, int32_t drt_variant, int32_t component,
                                 const double *omegas, int32_t nw, void *out, void *work, size_t work_bytes,
                                 hipStream_t stream);

/* First arrivals of nsrc surface sources at every (x_i, z_n): roots in theta
 * of X - x_s between adjacent nodes whose take-off angles vartheta lie inside
 * (-theta_max, theta_max) (linear interpolation of X and tau), the smallest
 * tau > 0; NaN where there is none.  In: xs (device float64 [nsrc]).
 * Out: T (device float64 [nsrc][nz][nx]). */
egb_status egb_paraxial_pick(const egb_grid *g, const void *levels, double theta_max, const double *xs, int32_t nsrc,
                             double *T, hipStream_t stream);

/* ---------------------------------------- Green's-function migration
 * The application the paper ends with (section 6): imaging with the Green's
 * functions of the depth march (eq. 34 over Gamma = {X = x_s}, eq. 35; one
 * march serves every surface point).  The paper gives no imaging condition;
 * these two calls are single-scattering (Born) data of a reflectivity and
 * its exact adjoint for a real reflectivity, the image:
 *   d[w][s][r] = omega_w^2 dx dz sum_x G[s][w][x] m[x] G[r][w][x],
 *   I[x] = Re sum_w omega_w^2 dx dz sum_{s,r} conj(G[s][w][x])
 *          conj(G[r][w][x]) d[w][s][r]
 * (sources and receivers at the same ns surface points, x = ix nz + iz).
 * G: device, complex [ns][nw][nx][nz] (re, im) in the grid dtype, i.e. the
 * outputs of egb_paraxial_beam_sum for the ns points one after another;
 * omegas: HOST float64 [nw] (the frequencies G was summed at, rad/s).
 * Accumulation is float64.  1 <= ns <= 64 and nw <= 65535
 * (EGB_EUNSUPPORTED above).  Stream-ordered; nothing is allocated. */

/* Bytes of the workspace egb_born_data needs for this grid, ns points and nw
 * frequencies (the partial sums of its split over image points); 0 on bad
 * arguments. */
size_t egb_born_workspace_size(const egb_grid *g, int32_t ns, int32_t nw);

/* In: m (device float64 [nx][nz]).  Out: d (device complex128 [nw][ns][ns],
 * (re, im)).  work: device, 16-byte aligned, at least
 * egb_born_workspace_size(g, ns, nw) bytes (EGB_EWORKSPACE otherwise),
 * overwritten.  The partial sums are added in a fixed order: the same
 * inputs give the same bits on every call. */
egb_status egb_born_data(const egb_grid *g, const void *G, int32_t ns, const double *omegas, int32_t nw,
                         const double *m, double *d, void *work, size_t work_bytes, hipStream_t stream);

/* In: d (device complex128 [nw][ns][ns]).  Out: image (device float64
 * [nx][nz]). */
egb_status egb_migrate(const egb_grid *g, const void *G, int32_t ns, const double *omegas, int32_t nw,
                       const double *d, double *image, hipStream_t stream);

/* ------------------------------------------------------ launch tuning
 * Not a step of the method: the stage kernels of egb_liouville_step, its
 * kinematic variant, the reverse stages of egb_adjoint_step and
 * egb_liouville_step_batched split the (tile, x) steps of their grids into
 * one contiguous range per block.  A launch is a tile shape (the theta rows
 * of a (z, theta) tile of 64 z cells, with its LDS slice and halo, and the
 * waves per SIMD its registers are sized for) and a block count; both
 * decide only how the work is laid out over the chip, and every launch
 * gives bit-identical results.  By default a launch uses the first tile
 * shape and one round of resident blocks.  The library keeps a launch per
 * (operation, grid shape(s), dtype, current device), process-wide behind a
 * mutex; these calls read it, fix it or measure it.  They allocate nothing
 * on the device. */
#define EGB_TUNE_STEP 0      /* egb_liouville_step */
#define EGB_TUNE_KINEMATIC 1 /* egb_liouville_step_kinematic, and the stages egb_adjoint_step recomputes */
#define EGB_TUNE_ADJOINT 2   /* the reverse stages of egb_adjoint_step */

typedef struct {
    int32_t tile_rows; /* theta rows per tile (one of egb_tile_rows); 0 = the default shape */
    int32_t blocks;    /* blocks per launch; 0 = one round of resident blocks */
} egb_launch;

/* The tile heights `op` supports on grids of g's dtype, the default first,
 * into rows[] (if not NULL; at most 8); returns their number (0 for bad
 * arguments).  FP32: 12, 8, 16 rows for EGB_TUNE_STEP (at 3, 2, 4 waves per
 * SIMD), 16, 8, 12 for EGB_TUNE_KINEMATIC; FP64 and EGB_TUNE_ADJOINT: 8. */
int32_t egb_tile_rows(const egb_grid *g, int32_t op, int32_t *rows);

/* The block count in use for `op` on grids of g's shape and dtype (0 = the
 * default); 0 also for bad arguments. */
int32_t egb_get_blocks(const egb_grid *g, int32_t op);

/* Fix the count (blocks >= 1) or restore the default (blocks = 0), keeping
 * the tile shape.  EGB_EINVAL for a bad grid, op or count; EGB_EHIP without
 * a device. */
egb_status egb_set_blocks(const egb_grid *g, int32_t op, int32_t blocks);

/* The launch in use (tile_rows of the shape, blocks as egb_get_blocks). */
egb_status egb_get_launch(const egb_grid *g, int32_t op, egb_launch *out);

/* Fix a launch; tile_rows must be one of egb_tile_rows (0: the default
 * shape), blocks >= 0 (0: one round of resident blocks).  EGB_EINVAL
 * otherwise. */
egb_status egb_set_launch(const egb_grid *g, int32_t op, const egb_launch *l);

/* The autotuner for op = EGB_TUNE_STEP or EGB_TUNE_KINEMATIC: times `reps`
 * (>= 1) RK3 steps with HIP events on `stream`, first of every tile shape
 * at its default block count, then of the fastest shape at the default and
 * 1/2 to 3 rounds of resident blocks, and keeps the fastest launch for this
 * grid shape (a candidate replaces the default only when faster by more
 * than 1 %); *blocks receives the count (egb_get_launch the shape).
 * Arguments as egb_liouville_step; the timed steps read `state` and write
 * only `work` (the last stage too), so no buffer of the caller changes.
 * Synchronises `stream`. */
egb_status egb_tune_step(const egb_grid *g, const void *vel3d, const egb_source *src, const void *bdata,
                         const void *state, void *work, size_t work_bytes, double dt, int32_t op, int32_t reps,
                         hipStream_t stream, int32_t *blocks);

/* The same for a batch (egb_liouville_step_batched's arguments), keyed by
 * the shapes of all its grids in order; the timed steps write only `work`.
 * Synchronises `stream`. */
egb_status egb_tune_batched(const egb_problem *probs, int32_t nprob, void *work, size_t work_bytes, int32_t reps,
                            hipStream_t stream, int32_t *blocks);

/* Fix (blocks >= 1) or restore (0) the count of a batch of this shape. */
egb_status egb_set_blocks_batched(const egb_problem *probs, int32_t nprob, int32_t blocks);

/* The launch of a batch of this shape (tile heights as EGB_TUNE_STEP's). */
egb_status egb_get_launch_batched(const egb_problem *probs, int32_t nprob, egb_launch *out);
egb_status egb_set_launch_batched(const egb_problem *probs, int32_t nprob, const egb_launch *l);

/* Human-readable text for a status code (static storage). */
const char *egb_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* EGB_H */
