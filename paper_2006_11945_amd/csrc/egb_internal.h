// Internal host/device interface of libegb: layouts and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/egb.h"

namespace egb {

// Elements per phase-space plane: nth * nx * nz rounded up to 64.
inline size_t plane_stride(const egb_grid& g) {
    size_t n = (size_t)g.nth * (size_t)g.nx * (size_t)g.nz;
    return (n + 63) / 64 * 64;
}
inline size_t real_size(const egb_grid& g) { return g.dtype == EGB_F64 ? 8 : 4; }

// Byte offset of state plane p: planes before EGB_PSI in the grid dtype, psi
// in double.
inline size_t state_plane_offset(const egb_grid& g, int p) {
    return (size_t)p * plane_stride(g) * real_size(g);
}
inline size_t state_bytes(const egb_grid& g) { return state_plane_offset(g, EGB_PSI) + plane_stride(g) * 8; }

// Boundary data: per plane, x ghosts [theta][6][nz] then z ghosts
// [theta][nx][6], padded to 64 elements; the state's planes before EGB_PSI in
// the grid dtype, psi in double.
inline size_t bdata_stride(const egb_grid& g) {
    size_t n = (size_t)g.nth * 6 * ((size_t)g.nx + (size_t)g.nz);
    return (n + 63) / 64 * 64;
}
inline size_t bdata_bytes(const egb_grid& g) { return bdata_stride(g) * (EGB_PSI * real_size(g) + 8); }
// Adjoint boundary accumulator (float64): [2 planes: phi1, psi][theta] x
// ([2 ends][3 sources][2 weights][nz] then [nx][2 ends][3 sources][2 weights]).
inline size_t bfold_bytes(const egb_grid& g) { return (size_t)2 * g.nth * 12 * ((size_t)g.nx + g.nz) * 8; }

// Geometry passed to kernels by value.
struct GridArgs {
    int nx, nz, nth;
    long long nxz, stride, bstride;  // cells per theta slice; plane strides of state and boundary data
    double x0, z0, dx, dz, dth;
};

inline GridArgs grid_args(const egb_grid& g) {
    GridArgs a;
    a.nx = g.nx;
    a.nz = g.nz;
    a.nth = g.nth;
    a.nxz = (long long)g.nx * g.nz;
    a.stride = (long long)plane_stride(g);
    a.bstride = (long long)bdata_stride(g);
    a.x0 = g.x0;
    a.z0 = g.z0;
    a.dx = g.dx;
    a.dz = g.dz;
    a.dth = 6.283185307179586476925286766559 / g.nth;
    return a;
}

// Launchers (return hipSuccess or the launch error).
hipError_t launch_medium_table(const GridArgs& a, const egb_medium& m, double* coeff2d, hipStream_t s);
hipError_t launch_velocity(const GridArgs& a, int dtype, const double* coeff2d, void* vel3d, unsigned long long* rate_bits,
                           hipStream_t s);
hipError_t launch_init_state(const GridArgs& a, int dtype, const double* coeff2d, const egb_source& src, void* state,
                             hipStream_t s);
hipError_t launch_boundary_data(const GridArgs& a, int dtype, const void* state, void* bdata, hipStream_t s);
hipError_t launch_pick(const GridArgs& a, int dtype, const void* state, const double* rx, int nr, double* t_out,
                       hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t s);

// One SSP-RK3 stage: Uout = ca U0 + cb (Uin + dt L(Uin)), ball cells copy U0.
struct StageArgs {
    GridArgs g;
    const void* vel;
    const void* bd;  // boundary data (ghost values)
    const void* U0;
    const void* Uin;
    void* Uout;
    double dt;
    double xs, zs, r02;
};
// Blocks of `kernel` (launched with `threads` threads) that the current device
// holds at once; 0 on a HIP error.
int resident_blocks(const void* kernel, int threads);
// Launch shapes of the stage kernels: theta rows per tile (and the waves per
// SIMD their registers are sized for); shape 0 is the default.  The number
// of shapes for (dtype, kinematic); their tile heights in tile_rows (if not
// NULL, at least 4 entries).
int stage_shapes(int dtype, bool kinematic, int* tile_rows);
int batched_shapes(int dtype, int* tile_rows);
// kinematic: march phi1 and psi only (the planes a traveltime depends on)
// blocks <= 0: one round of resident blocks; > 0: the steps split over that many
hipError_t launch_stage(const StageArgs& a, int dtype, int stage, hipStream_t s, bool kinematic = false,
                        int blocks = 0, int shape = 0);
// resident blocks of the stage kernel (one round) and its (tile, x) steps on grid g
void stage_limits(const GridArgs& g, int dtype, bool kinematic, long long& resident, long long& work, int shape = 0);
long long batched_resident(int dtype, int shape = 0);

// Launch-shape cache and autotuner (tune.hip).  Operation ids: the public
// EGB_TUNE_* values, and TUNE_BATCHED for a batch keyed by all its grids.
constexpr int TUNE_BATCHED = 3;
struct Launch {
    int blocks;  // 0: one round of resident blocks
    int shape;   // index into the shapes of the operation (0: default)
};
unsigned long long grid_shape_key(const egb_grid& g);
unsigned long long batch_shape_key(const egb_problem* p, int n);
Launch tuned_launch(int op, unsigned long long shape, int dtype);  // {0, 0}: none (the default)
hipError_t set_tuned_launch(int op, unsigned long long shape, int dtype, Launch l);  // {<= 0, 0}: forget
// the fastest launch for the three stages a[0..2] of one RK3 step (each
// writes only its Uout): every shape at its default count, then block
// counts for the fastest shape
hipError_t tune_stage(const StageArgs (&a)[3], int dtype, bool kinematic, int reps, hipStream_t s, Launch& best);
// `fill(shape)` rewrites the batch items for a shape (tile counts change)
hipError_t tune_batched(const void* items, const long long* wfirst, int nprob, int dtype, int reps, hipStream_t s,
                        hipError_t (*fill)(void* ctx, int shape, long long& total), void* ctx, Launch& best);
// The stage kernel addresses each array with 32-bit byte offsets.
bool stage_fits_32bit(const GridArgs& g, int dtype);

// Batched march (see liouville.hip).
size_t batch_item_bytes();
// last_to_work: the last stage writes U1 instead of the state (timing runs)
long long batch_item_fill(void* item, const GridArgs& g, int dtype, const void* vel, const void* bd, void* state,
                          void* U1, void* U2, double dt, double xs, double zs, double r02, bool last_to_work = false,
                          int shape = 0);
// grid <= 0: one round of resident blocks
hipError_t launch_stage_batched(const void* items, const long long* wfirst, int nprob, long long total, int dtype,
                                int stage, int grid, hipStream_t s, int shape = 0);

// Adjoint of the kinematic march (see adjoint.hip).
// One reverse stage: lam_in (stages 1, 2) and acc_out = acc_in + ... (see
// adjoint.hip); lam_out must not alias any output.
hipError_t launch_adjoint_stage(const GridArgs& g, int dtype, int stage, const void* vel, const void* bd,
                                const void* Uin, const void* lam_out, void* lam_in, const void* acc_in, void* acc_out,
                                void* gvel, void* bfold, double dt, double xs, double zs, double r02, hipStream_t s,
                                int blocks = 0);
hipError_t launch_pick_adjoint(const GridArgs& a, int dtype, const void* state, const double* rx, int nr,
                               const double* tbar, void* lam, hipStream_t s);
hipError_t launch_adjoint_medium(const GridArgs& a, int dtype, const egb_medium& m, const double* coeff2d,
                                 const egb_source& src, const void* gvel, const void* lam0, const double* bfold,
                                 double* grad, double* gtab, double* gms, hipStream_t s);

// Paraxial depth march (see paraxial.hip).  Level planes: seven in the grid
// dtype, then tau in double, each of paraxial_stride() elements.
inline size_t paraxial_stride(const egb_grid& g) {
    size_t n = (size_t)g.nth * (size_t)g.nx;
    return (n + 63) / 64 * 64;
}
inline size_t paraxial_level_bytes(const egb_grid& g) { return paraxial_stride(g) * (7 * real_size(g) + 8); }
inline size_t paraxial_vel_bytes(const egb_grid& g) { return (size_t)g.nz * 7 * paraxial_stride(g) * real_size(g); }
struct PStageArgs {
    int nx, nth;
    long long P;               // plane stride (elements)
    double dx, dth, dl, s;     // dl: the substep in z; s: stage depth as a fraction of the level interval
    const void* pv0;           // coefficients at the interval's two levels
    const void* pv1;
    const void* Ub;            // surface data (level 0): the ghost values
    const void* U0;            // the substep's starting state
    const void* Uin;
    void* Uout;
};
hipError_t launch_pvelocity(const GridArgs& a, int dtype, double theta_max, int drt, const double* coeff2d,
                            void* pvel, long long P, unsigned long long* rate_bits, hipStream_t s);
hipError_t launch_pinit(int nx, int nth, long long P, double x0, double dx, double theta_max, double beta, int drt,
                        int dtype, const void* pvel, void* level0, hipStream_t s);
hipError_t launch_pstage(const PStageArgs& a, int dtype, int stage, hipStream_t s);
hipError_t launch_ppick(int nx, int nz, int nth, double theta_max, long long P, int dtype, const void* levels,
                        size_t level_bytes, const double* xs, int nsrc, double* T, hipStream_t s);

// Beam superposition.
struct BeamArgs {
    GridArgs g;
    const double* coeff2d;
    const void* vel;
    const void* U;
    double beta;
    int lin;          // EGB_LIN_EXACT or EGB_LIN_PAPER28
    int cap;          // records per row / column list
    int* counts;      // [nz rows][nx cols]
    void* rows;       // row records
    void* cols;       // column records
    int* order;       // per line, cap entries: the record indices in the order of their keys
    int rows_only = 0;  // the column lists are empty (the depth march's sums): no column pass
};
hipError_t launch_beam_compact(const BeamArgs& a, int dtype, hipStream_t s);
// Beam records of the depth march (rows = levels; see beam.hip).
struct PBeamArgs {
    GridArgs g;               // output geometry (rows: levels, columns: x)
    const double* coeff2d;
    const void* levels;
    size_t level_bytes;
    long long P;              // level plane stride (elements)
    int nx, nz, nth, lin, comp, cap;  // comp: -1 scalar, else 2 i + k of the Green's tensor
    int drt;                  // the DRT frame the levels were marched in (EGB_DRT_*)
    double dx, dth, theta_max, xs;
    int* counts;              // [nz rows][nx columns] (columns stay 0)
    void* rows;
    int* cand;                // inside the compaction kernel: its block's candidates (LDS)
    int* ncand;
};
hipError_t launch_pbeam_compact(const PBeamArgs& a, int dtype, hipStream_t s);

// Green's-function migration (migration.hip)
int migration_max_points();
size_t born_workspace_bytes(long long npt, int ns, int nw);
hipError_t launch_born_data(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                            const double* m, double* d, void* work, hipStream_t s);
hipError_t launch_migrate(const GridArgs& g, int dtype, const void* G, int ns, const double* omegas, int nw,
                          const double* d, double* image, hipStream_t s);
hipError_t launch_beam_sum(const BeamArgs& a, int dtype, const double* omegas, int nw, void* out, hipStream_t s);
// *out = max(p[0 .. n)) (one block)
hipError_t launch_max_i32(const int* p, int n, int* out, hipStream_t s);
size_t beam_record_bytes();
// bytes per record slot of a line list: the record and its entry in the line's order
inline size_t beam_slot_bytes() { return beam_record_bytes() + sizeof(int); }

}  // namespace egb
