// C ABI of libegb: argument validation, workspace carving, launch order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "egb_internal.h"

using namespace egb;

namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

bool grid_ok(const egb_grid* g) {
    if (!g) return false;
    if (g->nx < 8 || g->nz < 8 || g->nth < 8) return false;
    if (g->dtype != EGB_F32 && g->dtype != EGB_F64) return false;
    if (!(g->dx > 0.0) || !(g->dz > 0.0) || !isfinite(g->dx) || !isfinite(g->dz)) return false;
    if (!isfinite(g->x0) || !isfinite(g->z0)) return false;
    // keep every plane index below 2^62 bytes and per-axis products in range
    const double n = (double)g->nx * (double)g->nz * (double)g->nth;
    return n < 4.0e12;
}

bool source_ok(const egb_source* s) {
    return s && isfinite(s->xs) && isfinite(s->zs) && isfinite(s->r0) && s->r0 >= 0.0 && isfinite(s->beta) &&
           s->beta > 0.0 && (s->lin_variant == EGB_LIN_EXACT || s->lin_variant == EGB_LIN_PAPER28);
}

egb_status hip_status(hipError_t e) { return e == hipSuccess ? EGB_OK : EGB_EHIP; }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Default beam-list capacity per row / column.
int beam_cap_default(const egb_grid& g) { return 16 * ((g.nx > g.nz ? g.nx : g.nz) + g.nth) + 64; }
// ... per depth level of the paraxial beam sum.
int pbeam_cap_default(const egb_grid& g) { return 16 * (g.nx + g.nth) + 64; }

// Line counts of the beam lists, then one int for their maximum.
size_t beam_counts_bytes(const egb_grid& g) { return align256((size_t)(g.nx + g.nz + 1) * sizeof(int)); }

// CFL limits of velocity buffers.  egb_hamiltonian_velocity records the
// limit of every buffer it fills (keyed by its address, with the grid it was
// computed for); the marching calls look the buffer up and refuse a time
// step above the limit.  A buffer filled by other means is declared with
// egb_declare_velocity.  At most VEL_CAP records are kept; the least
// recently written one makes room.
struct VelRecord {
    int nx, nz, nth, dtype;
    double dx, dz, dt_cfl;
    unsigned long long seq;
};
constexpr size_t VEL_CAP = 4096;
std::mutex vel_mu;
std::map<const void*, VelRecord>& vel_table() {
    static std::map<const void*, VelRecord> t;
    return t;
}

void vel_record(const egb_grid& g, const void* vel3d, double dt_cfl) {
    static unsigned long long seq = 0;
    std::lock_guard<std::mutex> lock(vel_mu);
    auto& t = vel_table();
    if (t.size() >= VEL_CAP && t.find(vel3d) == t.end()) {
        auto old = t.begin();
        for (auto it = t.begin(); it != t.end(); ++it)
            if (it->second.seq < old->second.seq) old = it;
        t.erase(old);
    }
    t[vel3d] = VelRecord{g.nx, g.nz, g.nth, g.dtype, g.dx, g.dz, dt_cfl, ++seq};
}

// The recorded CFL limit of vel3d for grid g; false if the buffer is unknown
// or was recorded for another grid.
bool vel_lookup(const egb_grid& g, const void* vel3d, double& dt_cfl) {
    std::lock_guard<std::mutex> lock(vel_mu);
    const auto& t = vel_table();
    const auto it = t.find(vel3d);
    if (it == t.end()) return false;
    const VelRecord& r = it->second;
    if (r.nx != g.nx || r.nz != g.nz || r.nth != g.nth || r.dtype != g.dtype || r.dx != g.dx || r.dz != g.dz)
        return false;
    dt_cfl = r.dt_cfl;
    return true;
}

// dt against the limit of vel3d: EGB_ECFL for a step that is not positive
// and finite or exceeds dt_cfl (1 + 1e-12), EGB_EINVAL for an unknown buffer.
egb_status dt_check(const egb_grid& g, const void* vel3d, double dt) {
    if (!(dt > 0.0) || !isfinite(dt)) return EGB_ECFL;
    double lim = 0.0;
    if (!vel_lookup(g, vel3d, lim)) return EGB_EINVAL;
    return dt <= lim * (1.0 + 1e-12) ? EGB_OK : EGB_ECFL;
}

// Fixed scratch of egb_beam_sum_noalloc (the line counts and the beam
// record lists), one copy per device, held until the process ends.  Host
// code never uses the array's name as an address: the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t BEAM_SCRATCH_BYTES = (size_t)128 << 20;
constexpr size_t BEAM_SCRATCH_MIN_CAP = 256;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[BEAM_SCRATCH_BYTES];
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES] = {};

hipError_t beam_scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t egb_plane_stride(const egb_grid* g) { return grid_ok(g) ? plane_stride(*g) : 0; }

size_t egb_coeff2d_bytes(const egb_grid* g) {
    return grid_ok(g) ? (size_t)EGB_NFIELD * EGB_NTAYLOR * (size_t)g->nx * (size_t)g->nz * sizeof(double) : 0;
}

size_t egb_vel3d_bytes(const egb_grid* g) { return grid_ok(g) ? (size_t)EGB_NVEL * plane_stride(*g) * real_size(*g) : 0; }

size_t egb_state_bytes(const egb_grid* g) { return grid_ok(g) ? state_bytes(*g) : 0; }

size_t egb_state_plane_offset(const egb_grid* g, int32_t plane) {
    if (!grid_ok(g) || plane < 0 || plane >= EGB_NSTATE) return 0;
    return state_plane_offset(*g, plane);
}

size_t egb_bdata_bytes(const egb_grid* g) { return grid_ok(g) ? bdata_bytes(*g) : 0; }
size_t egb_bdata_plane_stride(const egb_grid* g) { return grid_ok(g) ? bdata_stride(*g) : 0; }
size_t egb_bfold_bytes(const egb_grid* g) { return grid_ok(g) ? bfold_bytes(*g) : 0; }

size_t egb_workspace_size(const egb_grid* g, int32_t op) {
    if (!grid_ok(g)) return 0;
    switch (op) {
        case EGB_OP_VELOCITY: return 256;
        case EGB_OP_STEP: return 2 * align256(state_bytes(*g));
        case EGB_OP_BEAM:
            return beam_counts_bytes(*g) + (size_t)(g->nx + g->nz) * beam_cap_default(*g) * beam_slot_bytes();
        case EGB_OP_PARAXIAL: return 2 * align256(paraxial_level_bytes(*g));
        case EGB_OP_PBEAM: return beam_counts_bytes(*g) + (size_t)g->nz * pbeam_cap_default(*g) * beam_slot_bytes();
        case EGB_OP_ADJOINT: {
            const size_t step = 5 * align256(state_bytes(*g));
            const size_t med = align256((size_t)15 * g->nx * g->nz * sizeof(double)) +
                               align256((size_t)g->nth * EGB_NFIELD * sizeof(double));
            return step > med ? step : med;
        }
        default: return 0;
    }
}

egb_status egb_hamiltonian_velocity(const egb_grid* g, const egb_medium* m, void* coeff2d, void* vel3d,
                                    double* dt_cfl, void* work, size_t work_bytes, hipStream_t stream) {
    if (!grid_ok(g) || !m || !m->vp0 || !m->eps || !m->delta || !coeff2d || !vel3d || !dt_cfl || !work)
        return EGB_EINVAL;
    if (!(m->vs_ratio >= 0.0) || !(m->vs_ratio < 1.0)) return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(vel3d) || !aligned16(work) || !aligned16(m->vp0) || !aligned16(m->eps) ||
        !aligned16(m->delta) || (m->tilt && !aligned16(m->tilt)))
        return EGB_EINVAL;
    if (work_bytes < egb_workspace_size(g, EGB_OP_VELOCITY)) return EGB_EWORKSPACE;
    const GridArgs a = grid_args(*g);
    unsigned long long* rate = static_cast<unsigned long long*>(work);
    hipError_t e = launch_fill_u64(rate, 1, 0ull, stream);
    if (e == hipSuccess) e = launch_medium_table(a, *m, static_cast<double*>(coeff2d), stream);
    if (e == hipSuccess) e = launch_velocity(a, g->dtype, static_cast<const double*>(coeff2d), vel3d, rate, stream);
    unsigned long long bits = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bits, rate, sizeof(bits), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return EGB_EHIP;
    double r;
    memcpy(&r, &bits, sizeof(r));
    if (!(r > 0.0) || !isfinite(r)) return EGB_ENONFINITE;
    *dt_cfl = 0.5 / r;
    vel_record(*g, vel3d, *dt_cfl);
    return EGB_OK;
}

egb_status egb_declare_velocity(const egb_grid* g, const void* vel3d, double dt_cfl) {
    if (!grid_ok(g) || !vel3d || !aligned16(vel3d) || !(dt_cfl > 0.0) || !isfinite(dt_cfl)) return EGB_EINVAL;
    vel_record(*g, vel3d, dt_cfl);
    return EGB_OK;
}

egb_status egb_velocity_dt_cfl(const egb_grid* g, const void* vel3d, double* dt_cfl) {
    if (!grid_ok(g) || !vel3d || !dt_cfl) return EGB_EINVAL;
    double lim = 0.0;
    if (!vel_lookup(*g, vel3d, lim)) return EGB_EINVAL;
    *dt_cfl = lim;
    return EGB_OK;
}

egb_status egb_medium_table(const egb_grid* g, const egb_medium* m, void* coeff2d, hipStream_t stream) {
    if (!grid_ok(g) || !m || !m->vp0 || !m->eps || !m->delta || !coeff2d) return EGB_EINVAL;
    if (!(m->vs_ratio >= 0.0) || !(m->vs_ratio < 1.0)) return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(m->vp0) || !aligned16(m->eps) || !aligned16(m->delta) ||
        (m->tilt && !aligned16(m->tilt)))
        return EGB_EINVAL;
    return hip_status(launch_medium_table(grid_args(*g), *m, static_cast<double*>(coeff2d), stream));
}

egb_status egb_init_state(const egb_grid* g, const void* coeff2d, const egb_source* src, void* state,
                          hipStream_t stream) {
    if (!grid_ok(g) || !coeff2d || !state || !source_ok(src)) return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(state)) return EGB_EINVAL;
    return hip_status(launch_init_state(grid_args(*g), g->dtype, static_cast<const double*>(coeff2d), *src, state, stream));
}

egb_status egb_boundary_data(const egb_grid* g, const void* state, void* bdata, hipStream_t stream) {
    if (!grid_ok(g) || !state || !bdata) return EGB_EINVAL;
    if (!aligned16(state) || !aligned16(bdata)) return EGB_EINVAL;
    return hip_status(launch_boundary_data(grid_args(*g), g->dtype, state, bdata, stream));
}

static egb_status liouville_steps(const egb_grid* g, const void* vel3d, const egb_source* src, const void* bdata,
                                  void* state, void* work, size_t work_bytes, double dt, int32_t nsteps,
                                  hipStream_t stream, bool kin) {
    if (!grid_ok(g) || !vel3d || !bdata || !state || !source_ok(src) || nsteps < 0) return EGB_EINVAL;
    if (nsteps > 0 && !work) return EGB_EINVAL;
    if (!aligned16(vel3d) || !aligned16(bdata) || !aligned16(state) || (work && !aligned16(work))) return EGB_EINVAL;
    const egb_status ds = dt_check(*g, vel3d, dt);
    if (ds != EGB_OK) return ds;
    if (nsteps == 0) return EGB_OK;
    if (work_bytes < egb_workspace_size(g, EGB_OP_STEP)) return EGB_EWORKSPACE;
    if (!stage_fits_32bit(grid_args(*g), g->dtype)) return EGB_EUNSUPPORTED;
    char* w = static_cast<char*>(work);
    void* U1 = w;
    void* U2 = w + align256(state_bytes(*g));
    StageArgs sa;
    sa.g = grid_args(*g);
    sa.vel = vel3d;
    sa.bd = bdata;
    sa.dt = dt;
    sa.xs = src->xs;
    sa.zs = src->zs;
    sa.r02 = src->r0 * src->r0;
    const Launch L = tuned_launch(kin ? EGB_TUNE_KINEMATIC : EGB_TUNE_STEP, grid_shape_key(*g), g->dtype);
    for (int n = 0; n < nsteps; ++n) {
        sa.U0 = state;
        sa.Uin = state;
        sa.Uout = U1;
        hipError_t e = launch_stage(sa, g->dtype, 0, stream, kin, L.blocks, L.shape);
        if (e != hipSuccess) return EGB_EHIP;
        sa.Uin = U1;
        sa.Uout = U2;
        e = launch_stage(sa, g->dtype, 1, stream, kin, L.blocks, L.shape);
        if (e != hipSuccess) return EGB_EHIP;
        sa.Uin = U2;
        sa.Uout = state;
        e = launch_stage(sa, g->dtype, 2, stream, kin, L.blocks, L.shape);
        if (e != hipSuccess) return EGB_EHIP;
    }
    return EGB_OK;
}

egb_status egb_liouville_step(const egb_grid* g, const void* vel3d, const egb_source* src, const void* bdata,
                              void* state, void* work, size_t work_bytes, double dt, int32_t nsteps,
                              hipStream_t stream) {
    return liouville_steps(g, vel3d, src, bdata, state, work, work_bytes, dt, nsteps, stream, false);
}

egb_status egb_liouville_step_kinematic(const egb_grid* g, const void* vel3d, const egb_source* src,
                                        const void* bdata, void* state, void* work, size_t work_bytes, double dt,
                                        int32_t nsteps, hipStream_t stream) {
    return liouville_steps(g, vel3d, src, bdata, state, work, work_bytes, dt, nsteps, stream, true);
}

size_t egb_gvel_bytes(const egb_grid* g) { return grid_ok(g) ? (size_t)3 * plane_stride(*g) * real_size(*g) : 0; }

egb_status egb_pick_adjoint(const egb_grid* g, const void* state, const double* rx, int32_t nr, const double* tbar,
                            void* lambda, hipStream_t stream) {
    if (!grid_ok(g) || !state || !lambda || nr < 0 || (nr > 0 && (!rx || !tbar))) return EGB_EINVAL;
    if (!aligned16(state) || !aligned16(lambda) || (rx && !aligned16(rx)) || (tbar && ((uintptr_t)tbar & 7u)))
        return EGB_EINVAL;
    return hip_status(launch_pick_adjoint(grid_args(*g), g->dtype, state, rx, nr, tbar, lambda, stream));
}

egb_status egb_adjoint_step(const egb_grid* g, const void* vel3d, const egb_source* src, const void* bdata,
                            const void* state_n, void* lambda, void* gvel, void* bfold, void* work, size_t work_bytes,
                            double dt, hipStream_t stream) {
    if (!grid_ok(g) || !vel3d || !bdata || !state_n || !lambda || !gvel || !bfold || !work || !source_ok(src))
        return EGB_EINVAL;
    if (!aligned16(vel3d) || !aligned16(bdata) || !aligned16(state_n) || !aligned16(lambda) || !aligned16(gvel) ||
        !aligned16(bfold) || !aligned16(work))
        return EGB_EINVAL;
    if (state_n == lambda) return EGB_EINVAL;
    const egb_status ds = dt_check(*g, vel3d, dt);
    if (ds != EGB_OK) return ds;
    if (work_bytes < egb_workspace_size(g, EGB_OP_ADJOINT)) return EGB_EWORKSPACE;
    if (!stage_fits_32bit(grid_args(*g), g->dtype)) return EGB_EUNSUPPORTED;
    const size_t sb = align256(state_bytes(*g));
    char* w = static_cast<char*>(work);
    void* U1 = w;
    void* U2 = w + sb;
    void* L2 = w + 2 * sb;
    void* L1 = w + 3 * sb;
    void* L3 = w + 4 * sb;
    const GridArgs a = grid_args(*g);
    // recompute the inner stages of this step (phi1 and psi only)
    StageArgs sa;
    sa.g = a;
    sa.vel = vel3d;
    sa.bd = bdata;
    sa.dt = dt;
    sa.xs = src->xs;
    sa.zs = src->zs;
    sa.r02 = src->r0 * src->r0;
    sa.U0 = state_n;
    sa.Uin = state_n;
    sa.Uout = U1;
    const unsigned long long key = grid_shape_key(*g);
    const Launch kl = tuned_launch(EGB_TUNE_KINEMATIC, key, g->dtype);
    const int ab = tuned_launch(EGB_TUNE_ADJOINT, key, g->dtype).blocks;
    hipError_t e = launch_stage(sa, g->dtype, 0, stream, true, kl.blocks, kl.shape);
    if (e == hipSuccess) {
        sa.Uin = U1;
        sa.Uout = U2;
        e = launch_stage(sa, g->dtype, 1, stream, true, kl.blocks, kl.shape);
    }
    const double r02 = src->r0 * src->r0;
    // Reverse: stage 2 (input U2), stage 1 (input U1), stage 0 (input U^n).
    // A stage reads the lambda of its output around every cell, so no output
    // may overwrite it: the accumulated lambda of U^n lives in L1 until stage
    // 0 writes the result back into `lambda`.
    if (e == hipSuccess)  // lambda -> L2 (of U2), acc L1 = (ca mu + ball) part
        e = launch_adjoint_stage(a, g->dtype, 2, vel3d, bdata, U2, lambda, L2, nullptr, L1, gvel, bfold, dt, src->xs,
                                 src->zs, r02, stream, ab);
    if (e == hipSuccess)  // L2 -> L3 (of U1), acc L1 +=
        e = launch_adjoint_stage(a, g->dtype, 1, vel3d, bdata, U1, L2, L3, L1, L1, gvel, bfold, dt, src->xs, src->zs,
                                 r02, stream, ab);
    if (e == hipSuccess)  // L3 -> lambda = L1 + stage 0 terms
        e = launch_adjoint_stage(a, g->dtype, 0, vel3d, bdata, state_n, L3, nullptr, L1, lambda, gvel, bfold, dt,
                                 src->xs, src->zs, r02, stream, ab);
    return hip_status(e);
}

egb_status egb_adjoint_medium(const egb_grid* g, const egb_medium* m, const void* coeff2d, const egb_source* src,
                              const void* gvel, const void* lambda0, const void* bfold, double* grad, void* work,
                              size_t work_bytes, hipStream_t stream) {
    if (!grid_ok(g) || !m || !m->vp0 || !m->eps || !m->delta || !coeff2d || !gvel || !lambda0 || !bfold || !grad ||
        !work || !source_ok(src))
        return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(gvel) || !aligned16(lambda0) || !aligned16(bfold) || !aligned16(grad) ||
        !aligned16(work))
        return EGB_EINVAL;
    if (work_bytes < egb_workspace_size(g, EGB_OP_ADJOINT)) return EGB_EWORKSPACE;
    char* w = static_cast<char*>(work);
    double* gtab = reinterpret_cast<double*>(w);
    double* gms = reinterpret_cast<double*>(w + align256((size_t)15 * g->nx * g->nz * sizeof(double)));
    return hip_status(launch_adjoint_medium(grid_args(*g), g->dtype, *m, static_cast<const double*>(coeff2d), *src,
                                            gvel, lambda0, static_cast<const double*>(bfold), grad, gtab, gms,
                                            stream));
}

size_t egb_paraxial_plane_stride(const egb_grid* g) { return grid_ok(g) ? paraxial_stride(*g) : 0; }
size_t egb_paraxial_level_bytes(const egb_grid* g) { return grid_ok(g) ? paraxial_level_bytes(*g) : 0; }
size_t egb_paraxial_vel_bytes(const egb_grid* g) { return grid_ok(g) ? paraxial_vel_bytes(*g) : 0; }

static bool theta_max_ok(double t) { return isfinite(t) && t > 0.0 && t <= 1.5707963267948966; }

static bool drt_ok(int32_t drt) { return drt == EGB_DRT_EXACT || drt == EGB_DRT_PAPER23; }

egb_status egb_paraxial_velocity(const egb_grid* g, const void* coeff2d, double theta_max, int32_t drt_variant,
                                 void* pvel, double* rate_out, void* work, size_t work_bytes, hipStream_t stream) {
    if (!grid_ok(g) || !coeff2d || !pvel || !rate_out || !work || !theta_max_ok(theta_max) || !drt_ok(drt_variant))
        return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(pvel) || !aligned16(work)) return EGB_EINVAL;
    if (work_bytes < egb_workspace_size(g, EGB_OP_VELOCITY)) return EGB_EWORKSPACE;
    unsigned long long* rate = static_cast<unsigned long long*>(work);
    hipError_t e = launch_fill_u64(rate, 1, 0ull, stream);
    if (e == hipSuccess)
        e = launch_pvelocity(grid_args(*g), g->dtype, theta_max, drt_variant, static_cast<const double*>(coeff2d),
                             pvel, (long long)paraxial_stride(*g), rate, stream);
    unsigned long long bits = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bits, rate, sizeof(bits), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return EGB_EHIP;
    double r;
    memcpy(&r, &bits, sizeof(r));
    if (!isfinite(r)) return EGB_EINVAL;  // V_z <= 0 inside (-theta_max, theta_max): beyond the paraxial range
    *rate_out = r;
    return EGB_OK;
}

egb_status egb_paraxial_init(const egb_grid* g, const void* pvel, double theta_max, double beta, int32_t drt_variant,
                             void* levels, hipStream_t stream) {
    if (!grid_ok(g) || !pvel || !levels || !theta_max_ok(theta_max) || !isfinite(beta) || !(beta > 0.0) ||
        !drt_ok(drt_variant))
        return EGB_EINVAL;
    if (!aligned16(pvel) || !aligned16(levels)) return EGB_EINVAL;
    return hip_status(launch_pinit(g->nx, g->nth, (long long)paraxial_stride(*g), g->x0, g->dx, theta_max, beta,
                                   drt_variant, g->dtype, pvel, levels, stream));
}

egb_status egb_paraxial_march(const egb_grid* g, const void* pvel, double theta_max, int32_t nsub, void* levels,
                              void* work, size_t work_bytes, hipStream_t stream) {
    if (!grid_ok(g) || !pvel || !levels || !work || !theta_max_ok(theta_max) || nsub < 1) return EGB_EINVAL;
    if (!aligned16(pvel) || !aligned16(levels) || !aligned16(work)) return EGB_EINVAL;
    if (work_bytes < egb_workspace_size(g, EGB_OP_PARAXIAL)) return EGB_EWORKSPACE;
    const size_t lb = paraxial_level_bytes(*g);
    if (lb >= ((size_t)1 << 31)) return EGB_EUNSUPPORTED;  // the stage kernel's 32-bit offsets
    const long long P = (long long)paraxial_stride(*g);
    const size_t vb = (size_t)7 * P * real_size(*g);  // coefficient bytes per level
    char* lev = static_cast<char*>(levels);
    const char* pv = static_cast<const char*>(pvel);
    void* U1 = work;
    void* U2 = static_cast<char*>(work) + align256(lb);
    PStageArgs a;
    a.nx = g->nx;
    a.nth = g->nth;
    a.P = P;
    a.dx = g->dx;
    a.dth = 2.0 * theta_max / g->nth;
    a.Ub = levels;  // level 0 keeps the surface data
    const double h = 1.0 / nsub;
    a.dl = g->dz * h;
    // 3 nsub (nz - 1) stage launches in order on `stream`: the host enqueues
    // a stage faster than the GPU runs one, so the queue never drains
    for (int n = 0; n + 1 < g->nz; ++n) {
        a.pv0 = pv + (size_t)n * vb;
        a.pv1 = pv + (size_t)(n + 1) * vb;
        void* next = lev + (size_t)(n + 1) * lb;
        for (int j = 0; j < nsub; ++j) {
            const double s0 = j * h;
            a.U0 = j == 0 ? lev + (size_t)n * lb : next;  // the substep's start
            a.Uin = a.U0;
            a.Uout = U1;
            a.s = s0;
            hipError_t e = launch_pstage(a, g->dtype, 0, stream);
            a.Uin = U1;
            a.Uout = U2;
            a.s = s0 + h;
            if (e == hipSuccess) e = launch_pstage(a, g->dtype, 1, stream);
            a.Uin = U2;
            a.Uout = next;  // in place for j > 0: each cell reads the start only at itself
            a.s = s0 + 0.5 * h;
            if (e == hipSuccess) e = launch_pstage(a, g->dtype, 2, stream);
            if (e != hipSuccess) return hip_status(e);
        }
    }
    return EGB_OK;
}

egb_status egb_paraxial_beam_sum(const egb_grid* g, const void* coeff2d, const void* levels, double theta_max,
                                 double xs, int32_t lin_variant, int32_t drt_variant, int32_t component,
                                 const double* omegas, int32_t nw, void* out, void* work, size_t work_bytes,
                                 hipStream_t stream) {
    if (!grid_ok(g) || !coeff2d || !levels || !theta_max_ok(theta_max) || !isfinite(xs) || !omegas || nw < 1 ||
        !out || !work || (lin_variant != EGB_LIN_EXACT && lin_variant != EGB_LIN_PAPER28) || !drt_ok(drt_variant) ||
        component < -1 || component > 3)
        return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(levels) || !aligned16(out) || !aligned16(work)) return EGB_EINVAL;
    for (int w = 0; w < nw; ++w)
        if (!isfinite(omegas[w]) || !(omegas[w] > 0.0)) return EGB_EINVAL;
    const size_t cb = beam_counts_bytes(*g);
    const size_t per = (size_t)g->nz * beam_slot_bytes();
    if (work_bytes < cb + per) return EGB_EWORKSPACE;
    const size_t capz = (work_bytes - cb) / per;
    const int cap = capz > (size_t)(1 << 30) ? (1 << 30) : (int)capz;
    char* w = static_cast<char*>(work);
    PBeamArgs pa;
    pa.g = grid_args(*g);
    pa.coeff2d = static_cast<const double*>(coeff2d);
    pa.levels = levels;
    pa.level_bytes = paraxial_level_bytes(*g);
    pa.P = (long long)paraxial_stride(*g);
    pa.nx = g->nx;
    pa.nz = g->nz;
    pa.nth = g->nth;
    pa.lin = lin_variant;
    pa.drt = drt_variant;
    pa.comp = component;
    pa.cap = cap;
    pa.dx = g->dx;
    pa.dth = 2.0 * theta_max / g->nth;
    pa.theta_max = theta_max;
    pa.xs = xs;
    pa.counts = reinterpret_cast<int*>(w);
    pa.rows = w + cb;
    // the line sums of the phase-space beam sum, rows only (column lists empty)
    BeamArgs ba;
    ba.g = pa.g;
    ba.coeff2d = pa.coeff2d;
    ba.vel = nullptr;
    ba.U = levels;
    ba.beta = 0.0;
    ba.lin = lin_variant;
    ba.cap = cap;
    ba.counts = pa.counts;
    ba.rows = pa.rows;
    ba.cols = pa.rows;
    ba.rows_only = 1;
    ba.order = reinterpret_cast<int*>(w + cb + (size_t)g->nz * cap * beam_record_bytes());
    hipError_t e = launch_pbeam_compact(pa, g->dtype, stream);
    if (e == hipSuccess) e = launch_beam_sum(ba, g->dtype, omegas, nw, out, stream);
    std::vector<int> counts(g->nz);
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts.data(), pa.counts, counts.size() * sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return EGB_EHIP;
    for (int c : counts)
        if (c > cap) return EGB_EWORKSPACE;
    return EGB_OK;
}

egb_status egb_paraxial_pick(const egb_grid* g, const void* levels, double theta_max, const double* xs, int32_t nsrc,
                             double* T, hipStream_t stream) {
    if (!grid_ok(g) || !levels || !theta_max_ok(theta_max) || nsrc < 0 || (nsrc > 0 && (!xs || !T)))
        return EGB_EINVAL;
    if (!aligned16(levels) || (xs && ((uintptr_t)xs & 7u)) || (T && ((uintptr_t)T & 7u))) return EGB_EINVAL;
    return hip_status(launch_ppick(g->nx, g->nz, g->nth, theta_max, (long long)paraxial_stride(*g), g->dtype, levels,
                                   paraxial_level_bytes(*g), xs, nsrc, T, stream));
}

size_t egb_workspace_size_batched(const egb_problem* probs, int32_t nprob) {
    if (!probs || nprob < 1) return 0;
    size_t b = align256((size_t)nprob * batch_item_bytes()) + align256((size_t)(nprob + 1) * sizeof(long long));
    for (int p = 0; p < nprob; ++p) {
        if (!grid_ok(&probs[p].grid)) return 0;
        b += 2 * align256(state_bytes(probs[p].grid));
    }
    return b;
}

// Validate a batch and write its item table and step offsets into the
// workspace (item table | wfirst[] | per-problem U1, U2).
static egb_status prepare_batch(const egb_problem* probs, int32_t nprob, void* work, size_t work_bytes,
                                char*& d_items, long long*& d_first, long long& total, bool last_to_work = false,
                                int shape = 0) {
    const int dtype = probs[0].grid.dtype;
    if (!work || !aligned16(work)) return EGB_EINVAL;
    if (work_bytes < egb_workspace_size_batched(probs, nprob)) return EGB_EWORKSPACE;
    char* w = static_cast<char*>(work);
    d_items = w;
    d_first = reinterpret_cast<long long*>(w + align256((size_t)nprob * batch_item_bytes()));
    char* bufs = reinterpret_cast<char*>(d_first) + align256((size_t)(nprob + 1) * sizeof(long long));
    std::vector<char> items((size_t)nprob * batch_item_bytes());
    std::vector<long long> first(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        const egb_problem& q = probs[p];
        const size_t sb = align256(state_bytes(q.grid));
        void* U1 = bufs;
        void* U2 = bufs + sb;
        bufs += 2 * sb;
        const long long n = batch_item_fill(items.data() + (size_t)p * batch_item_bytes(), grid_args(q.grid), dtype,
                                            q.vel3d, q.bdata, q.state, U1, U2, q.dt, q.src.xs, q.src.zs,
                                            q.src.r0 * q.src.r0, last_to_work, shape);
        first[p + 1] = first[p] + n;
    }
    total = first[nprob];
    hipError_t e = hipMemcpy(d_items, items.data(), items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_first, first.data(), first.size() * sizeof(long long), hipMemcpyHostToDevice);
    return e == hipSuccess ? EGB_OK : EGB_EHIP;
}

static egb_status batch_ok(const egb_problem* probs, int32_t nprob) {
    if (!probs || nprob < 1) return EGB_EINVAL;
    const int dtype = probs[0].grid.dtype;
    for (int p = 0; p < nprob; ++p) {
        const egb_problem& q = probs[p];
        if (!grid_ok(&q.grid) || q.grid.dtype != dtype || !q.vel3d || !q.bdata || !q.state || !source_ok(&q.src))
            return EGB_EINVAL;
        if (!aligned16(q.vel3d) || !aligned16(q.bdata) || !aligned16(q.state)) return EGB_EINVAL;
        const egb_status ds = dt_check(q.grid, q.vel3d, q.dt);
        if (ds != EGB_OK) return ds;
        if (!stage_fits_32bit(grid_args(q.grid), dtype)) return EGB_EUNSUPPORTED;
    }
    return EGB_OK;
}

egb_status egb_liouville_step_batched(const egb_problem* probs, int32_t nprob, int32_t nsteps, void* work,
                                      size_t work_bytes, hipStream_t stream) {
    egb_status st = batch_ok(probs, nprob);
    if (st != EGB_OK) return st;
    if (nsteps < 0) return EGB_EINVAL;
    if (nsteps == 0) return EGB_OK;
    const int dtype = probs[0].grid.dtype;
    char* d_items = nullptr;
    long long* d_first = nullptr;
    long long total = 0;
    // one round of resident blocks of the default tile over all problems'
    // steps unless a launch is tuned or fixed for this batch
    const Launch L = tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), dtype);
    st = prepare_batch(probs, nprob, work, work_bytes, d_items, d_first, total, false, L.shape);
    if (st != EGB_OK) return st;
    const int grid = L.blocks;
    // capture the whole march in one graph on a private stream, replay on `stream`
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        for (int n = 0; n < nsteps && le == hipSuccess; ++n)
            for (int s = 0; s < 3 && le == hipSuccess; ++s)
                le = launch_stage_batched(d_items, d_first, nprob, total, dtype, s, grid, cs, L.shape);
        e = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cs) hipStreamDestroy(cs);
    return hip_status(e);
}

// ------------------------------------------------------ Green's-function migration
static egb_status migration_args(const egb_grid* g, const void* G, int32_t ns, const double* omegas, int32_t nw) {
    if (!grid_ok(g) || !G || !aligned16(G) || ns < 1 || !omegas || nw < 1) return EGB_EINVAL;
    if (ns > migration_max_points() || nw > 65535) return EGB_EUNSUPPORTED;
    for (int w = 0; w < nw; ++w)
        if (!isfinite(omegas[w]) || !(omegas[w] > 0.0)) return EGB_EINVAL;
    return EGB_OK;
}

size_t egb_born_workspace_size(const egb_grid* g, int32_t ns, int32_t nw) {
    if (!grid_ok(g) || ns < 1 || ns > migration_max_points() || nw < 1 || nw > 65535) return 0;
    return born_workspace_bytes((long long)g->nx * g->nz, ns, nw);
}

egb_status egb_born_data(const egb_grid* g, const void* G, int32_t ns, const double* omegas, int32_t nw,
                         const double* m, double* d, void* work, size_t work_bytes, hipStream_t stream) {
    const egb_status st = migration_args(g, G, ns, omegas, nw);
    if (st != EGB_OK) return st;
    if (!m || !d || !aligned16(m) || !aligned16(d) || !work || !aligned16(work)) return EGB_EINVAL;
    if (work_bytes < egb_born_workspace_size(g, ns, nw)) return EGB_EWORKSPACE;
    return hip_status(launch_born_data(grid_args(*g), g->dtype, G, ns, omegas, nw, m, d, work, stream));
}

egb_status egb_migrate(const egb_grid* g, const void* G, int32_t ns, const double* omegas, int32_t nw,
                       const double* d, double* image, hipStream_t stream) {
    const egb_status st = migration_args(g, G, ns, omegas, nw);
    if (st != EGB_OK) return st;
    if (!d || !image || !aligned16(d) || !aligned16(image)) return EGB_EINVAL;
    return hip_status(launch_migrate(grid_args(*g), g->dtype, G, ns, omegas, nw, d, image, stream));
}

// ------------------------------------------------------------ launch tuning
static bool tune_op_ok(int32_t op) { return op == EGB_TUNE_STEP || op == EGB_TUNE_KINEMATIC || op == EGB_TUNE_ADJOINT; }

// Tile heights of an operation's shapes (the reverse stages have one).
static int op_shapes(const egb_grid* g, int32_t op, int* rows) {
    if (op == EGB_TUNE_ADJOINT) {
        if (rows) rows[0] = 8;
        return 1;
    }
    return stage_shapes(g->dtype, op == EGB_TUNE_KINEMATIC, rows);
}

int32_t egb_get_blocks(const egb_grid* g, int32_t op) {
    if (!grid_ok(g) || !tune_op_ok(op)) return 0;
    return tuned_launch(op, grid_shape_key(*g), g->dtype).blocks;
}

egb_status egb_set_blocks(const egb_grid* g, int32_t op, int32_t blocks) {
    if (!grid_ok(g) || !tune_op_ok(op) || blocks < 0) return EGB_EINVAL;
    Launch l = tuned_launch(op, grid_shape_key(*g), g->dtype);
    l.blocks = blocks;
    return set_tuned_launch(op, grid_shape_key(*g), g->dtype, l) == hipSuccess ? EGB_OK : EGB_EHIP;
}

int32_t egb_tile_rows(const egb_grid* g, int32_t op, int32_t* rows) {
    if (!grid_ok(g) || !tune_op_ok(op)) return 0;
    int r[8] = {0};
    const int n = op_shapes(g, op, r);
    if (rows)
        for (int i = 0; i < n; ++i) rows[i] = r[i];
    return n;
}

static int shape_of_rows(const int* r, int n, int32_t tile_rows) {
    if (tile_rows == 0) return 0;
    for (int i = 0; i < n; ++i)
        if (r[i] == tile_rows) return i;
    return -1;
}

egb_status egb_get_launch(const egb_grid* g, int32_t op, egb_launch* out) {
    if (!grid_ok(g) || !tune_op_ok(op) || !out) return EGB_EINVAL;
    int r[8] = {0};
    op_shapes(g, op, r);
    const Launch l = tuned_launch(op, grid_shape_key(*g), g->dtype);
    out->tile_rows = r[l.shape];
    out->blocks = l.blocks;
    return EGB_OK;
}

egb_status egb_set_launch(const egb_grid* g, int32_t op, const egb_launch* l) {
    if (!grid_ok(g) || !tune_op_ok(op) || !l || l->blocks < 0) return EGB_EINVAL;
    int r[8] = {0};
    const int n = op_shapes(g, op, r);
    const int sh = shape_of_rows(r, n, l->tile_rows);
    if (sh < 0) return EGB_EINVAL;
    return set_tuned_launch(op, grid_shape_key(*g), g->dtype, Launch{l->blocks, sh}) == hipSuccess ? EGB_OK
                                                                                                   : EGB_EHIP;
}

egb_status egb_tune_step(const egb_grid* g, const void* vel3d, const egb_source* src, const void* bdata,
                         const void* state, void* work, size_t work_bytes, double dt, int32_t op, int32_t reps,
                         hipStream_t stream, int32_t* blocks) {
    if (!grid_ok(g) || !vel3d || !bdata || !state || !work || !source_ok(src) || !blocks || reps < 1) return EGB_EINVAL;
    if (op != EGB_TUNE_STEP && op != EGB_TUNE_KINEMATIC) return EGB_EINVAL;
    if (!aligned16(vel3d) || !aligned16(bdata) || !aligned16(state) || !aligned16(work)) return EGB_EINVAL;
    const egb_status ds = dt_check(*g, vel3d, dt);
    if (ds != EGB_OK) return ds;
    if (work_bytes < egb_workspace_size(g, EGB_OP_STEP)) return EGB_EWORKSPACE;
    if (!stage_fits_32bit(grid_args(*g), g->dtype)) return EGB_EUNSUPPORTED;
    StageArgs sa;
    sa.g = grid_args(*g);
    sa.vel = vel3d;
    sa.bd = bdata;
    sa.dt = dt;
    sa.xs = src->xs;
    sa.zs = src->zs;
    sa.r02 = src->r0 * src->r0;
    sa.U0 = state;
    // one step whose stages write only the workspace: state -> U1 -> U2, and
    // the last stage (from U2 and the state) into U1 instead of the state
    void* U1 = work;
    void* U2 = static_cast<char*>(work) + align256(state_bytes(*g));
    StageArgs st[3] = {sa, sa, sa};
    st[0].Uin = state;
    st[0].Uout = U1;
    st[1].Uin = U1;
    st[1].Uout = U2;
    st[2].Uin = U2;
    st[2].Uout = U1;
    Launch best{0, 0};
    hipError_t e = tune_stage(st, g->dtype, op == EGB_TUNE_KINEMATIC, reps, stream, best);
    if (e == hipSuccess) e = set_tuned_launch(op, grid_shape_key(*g), g->dtype, best);
    if (e != hipSuccess) return hip_status(e);
    *blocks = best.blocks;
    return EGB_OK;
}

namespace {
// Re-fill the device item table of a batch for a launch shape (tuning).
struct BatchFill {
    const egb_problem* probs;
    int32_t nprob;
    void* work;
    size_t work_bytes;
};
hipError_t refill_batch(void* ctx, int shape, long long& total) {
    BatchFill& f = *static_cast<BatchFill*>(ctx);
    char* d_items = nullptr;
    long long* d_first = nullptr;
    const egb_status st = prepare_batch(f.probs, f.nprob, f.work, f.work_bytes, d_items, d_first, total, true, shape);
    return st == EGB_OK ? hipSuccess : hipErrorInvalidValue;
}
}  // namespace

egb_status egb_tune_batched(const egb_problem* probs, int32_t nprob, void* work, size_t work_bytes, int32_t reps,
                            hipStream_t stream, int32_t* blocks) {
    egb_status st = batch_ok(probs, nprob);
    if (st != EGB_OK) return st;
    if (!blocks || reps < 1) return EGB_EINVAL;
    const int dtype = probs[0].grid.dtype;
    char* d_items = nullptr;
    long long* d_first = nullptr;
    long long total = 0;
    st = prepare_batch(probs, nprob, work, work_bytes, d_items, d_first, total, true);
    if (st != EGB_OK) return st;
    BatchFill f{probs, nprob, work, work_bytes};
    Launch best{0, 0};
    hipError_t e = tune_batched(d_items, d_first, nprob, dtype, reps, stream, refill_batch, &f, best);
    if (e == hipSuccess) e = set_tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), dtype, best);
    if (e != hipSuccess) return hip_status(e);
    *blocks = best.blocks;
    return EGB_OK;
}

egb_status egb_set_blocks_batched(const egb_problem* probs, int32_t nprob, int32_t blocks) {
    egb_status st = batch_ok(probs, nprob);
    if (st != EGB_OK) return st;
    if (blocks < 0) return EGB_EINVAL;
    const int dtype = probs[0].grid.dtype;
    Launch l = tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), dtype);
    l.blocks = blocks;
    return set_tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), dtype, l) == hipSuccess ? EGB_OK : EGB_EHIP;
}

egb_status egb_get_launch_batched(const egb_problem* probs, int32_t nprob, egb_launch* out) {
    egb_status st = batch_ok(probs, nprob);
    if (st != EGB_OK) return st;
    if (!out) return EGB_EINVAL;
    int r[8] = {0};
    batched_shapes(probs[0].grid.dtype, r);
    const Launch l = tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), probs[0].grid.dtype);
    out->tile_rows = r[l.shape];
    out->blocks = l.blocks;
    return EGB_OK;
}

egb_status egb_set_launch_batched(const egb_problem* probs, int32_t nprob, const egb_launch* l) {
    egb_status st = batch_ok(probs, nprob);
    if (st != EGB_OK) return st;
    if (!l || l->blocks < 0) return EGB_EINVAL;
    int r[8] = {0};
    const int n = batched_shapes(probs[0].grid.dtype, r);
    const int sh = shape_of_rows(r, n, l->tile_rows);
    if (sh < 0) return EGB_EINVAL;
    return set_tuned_launch(TUNE_BATCHED, batch_shape_key(probs, nprob), probs[0].grid.dtype, Launch{l->blocks, sh}) ==
                   hipSuccess
               ? EGB_OK
               : EGB_EHIP;
}

static egb_status beam_sum_checks(const egb_grid* g, const void* coeff2d, const void* vel3d, const egb_source* src,
                                  const void* state, const double* omegas, int32_t nw, const void* out) {
    if (!grid_ok(g) || !coeff2d || !vel3d || !state || !omegas || nw < 1 || !out || !source_ok(src))
        return EGB_EINVAL;
    if (!aligned16(coeff2d) || !aligned16(vel3d) || !aligned16(state) || !aligned16(out)) return EGB_EINVAL;
    for (int w = 0; w < nw; ++w)
        if (!isfinite(omegas[w]) || !(omegas[w] > 0.0)) return EGB_EINVAL;
    return EGB_OK;
}

// The beam sum on a checked request with `work_bytes` of scratch at `work`:
// record lists of as many records per line as fit.
static egb_status beam_sum_run(const egb_grid* g, const void* coeff2d, const void* vel3d, const egb_source* src,
                               const void* state, const double* omegas, int32_t nw, void* out, void* work,
                               size_t work_bytes, hipStream_t stream) {
    const size_t cb = beam_counts_bytes(*g);
    const size_t per = (size_t)(g->nx + g->nz) * beam_slot_bytes();
    if (work_bytes < cb + per) return EGB_EWORKSPACE;
    const size_t capz = (work_bytes - cb) / per;
    const int cap = capz > (size_t)(1 << 30) ? (1 << 30) : (int)capz;
    char* w = static_cast<char*>(work);
    BeamArgs ba;
    ba.g = grid_args(*g);
    ba.coeff2d = static_cast<const double*>(coeff2d);
    ba.vel = vel3d;
    ba.U = state;
    ba.beta = src->beta;
    ba.lin = src->lin_variant;
    ba.cap = cap;
    ba.counts = reinterpret_cast<int*>(w);
    ba.rows = w + cb;
    ba.cols = w + cb + (size_t)g->nz * cap * beam_record_bytes();
    ba.order = reinterpret_cast<int*>(w + cb + (size_t)(g->nx + g->nz) * cap * beam_record_bytes());
    hipError_t e = launch_beam_compact(ba, g->dtype, stream);
    if (e == hipSuccess) e = launch_beam_sum(ba, g->dtype, omegas, nw, out, stream);
    // the longest list (a device reduction into the slot after the counts)
    const int nl = g->nx + g->nz;
    int longest = 0;
    if (e == hipSuccess) e = launch_max_i32(ba.counts, nl, ba.counts + nl, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&longest, ba.counts + nl, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return EGB_EHIP;
    return longest > cap ? EGB_EWORKSPACE : EGB_OK;
}

egb_status egb_beam_sum(const egb_grid* g, const void* coeff2d, const void* vel3d, const egb_source* src,
                        const void* state, const double* omegas, int32_t nw, void* out, void* work,
                        size_t work_bytes, hipStream_t stream) {
    const egb_status st = beam_sum_checks(g, coeff2d, vel3d, src, state, omegas, nw, out);
    if (st != EGB_OK) return st;
    if (!work || !aligned16(work)) return EGB_EINVAL;
    return beam_sum_run(g, coeff2d, vel3d, src, state, omegas, nw, out, work, work_bytes, stream);
}

size_t egb_beam_scratch_bytes(void) { return BEAM_SCRATCH_BYTES; }

egb_status egb_beam_sum_noalloc(const egb_grid* g, const void* coeff2d, const void* vel3d, const egb_source* src,
                                const void* state, const double* omegas, int32_t nw, void* out, hipStream_t stream) {
    const egb_status st = beam_sum_checks(g, coeff2d, vel3d, src, state, omegas, nw, out);
    if (st != EGB_OK) return st;
    // the fixed scratch must hold the line counts and at least BEAM_SCRATCH_MIN_CAP records per line
    const size_t need = beam_counts_bytes(*g) + (size_t)(g->nx + g->nz) * BEAM_SCRATCH_MIN_CAP * beam_slot_bytes();
    if (need > BEAM_SCRATCH_BYTES) return EGB_EUNSUPPORTED;
    void* ptr = nullptr;
    if (beam_scratch_address(&ptr) != hipSuccess) return EGB_EHIP;
    return beam_sum_run(g, coeff2d, vel3d, src, state, omegas, nw, out, ptr, BEAM_SCRATCH_BYTES, stream);
}

egb_status egb_pick_receivers(const egb_grid* g, const void* state, const double* rx, int32_t nr, double* t_out,
                              hipStream_t stream) {
    if (!grid_ok(g) || !state || nr < 0 || (nr > 0 && (!rx || !t_out))) return EGB_EINVAL;
    if (!aligned16(state) || (rx && !aligned16(rx)) || (t_out && !aligned16(t_out))) return EGB_EINVAL;
    return hip_status(launch_pick(grid_args(*g), g->dtype, state, rx, nr, t_out, stream));
}

const char* egb_status_string(int32_t s) {
    switch (s) {
        case EGB_OK: return "ok";
        case EGB_EINVAL: return "invalid argument";
        case EGB_ECFL: return "time step not positive and finite, or above the CFL limit of the velocity";
        case EGB_EWORKSPACE: return "workspace too small";
        case EGB_EHIP: return "HIP runtime or launch error";
        case EGB_ENONFINITE: return "non-finite value";
        case EGB_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

}  // extern "C"
