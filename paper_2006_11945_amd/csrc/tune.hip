// Launch-shape tuning.  The stage kernels (forward, kinematic, reverse and
// batched) split the (tile, x) steps of their grids into one contiguous
// range per block, so the number of blocks decides only how the work is
// spread over the chip: every count gives bit-identical results.  The
// default is one round of resident blocks; a process-wide cache keyed by
// (operation, grid shape(s), dtype, device) holds a count fixed by the
// caller or found by the autotuner, which times RK steps whose stages write
// only the workspace at a few counts around one round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "egb_internal.h"

namespace egb {
namespace {

struct TuneKey {
    int op, dtype, dev;
    unsigned long long shape;
    bool operator<(const TuneKey& o) const {
        return std::tie(op, dtype, dev, shape) < std::tie(o.op, o.dtype, o.dev, o.shape);
    }
};

std::mutex tune_mu;
std::map<TuneKey, Launch>& tune_table() {
    static std::map<TuneKey, Launch> t;
    return t;
}

// FNV-1a over the 8 bytes of v
unsigned long long fnv_mix(unsigned long long h, unsigned long long v) {
    for (int i = 0; i < 8; ++i) {
        h ^= (v >> (8 * i)) & 0xffull;
        h *= 0x100000001b3ull;
    }
    return h;
}
constexpr unsigned long long FNV0 = 0xcbf29ce484222325ull;

// The default count and 1/2, 3/4, 5/4, 3/2, 2 and 3 rounds of resident
// blocks, within [1, work], each once.
std::vector<int> block_candidates(long long resident, long long work, long long dflt) {
    std::vector<int> c;
    auto add = [&](long long b) {
        b = std::max(1LL, std::min(b, work));
        if (std::find(c.begin(), c.end(), (int)b) == c.end()) c.push_back((int)b);
    };
    add(dflt);
    for (int q : {2, 3, 4, 5, 6, 8, 12}) add(resident * q / 4);
    return c;
}

// Time of `reps` launches of `launch(candidate)` on `s` for every candidate:
// after 4 reps of the first candidate (clocks and caches settle), two passes
// over the candidates, in order and then in reverse, each timing summed over
// both so that a drift during the search favours none.  The first
// candidate (the default) is kept unless another is faster by more than
// 1 %, so that timing noise does not move the choice.  Returns the index of
// the choice in `best`.
template <typename F>
hipError_t pick_fastest(int nc, int reps, hipStream_t s, F launch, int& best) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    std::vector<float> total(nc, 0.0f);
    for (int r = 0; r < 4 * reps && e == hipSuccess; ++r) e = launch(0);
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass)
        for (int j = 0; j < nc && e == hipSuccess; ++j) {
            const int i = pass == 0 ? j : nc - 1 - j;
            e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(i);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            total[i] += ms;
        }
    best = 0;
    if (e == hipSuccess) {
        const int k = (int)(std::min_element(total.begin(), total.end()) - total.begin());
        if (total[k] < 0.99f * total[0]) best = k;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    return e;
}

}  // namespace

unsigned long long grid_shape_key(const egb_grid& g) {
    return fnv_mix(fnv_mix(fnv_mix(FNV0, (unsigned)g.nx), (unsigned)g.nz), (unsigned)g.nth);
}

unsigned long long batch_shape_key(const egb_problem* p, int n) {
    unsigned long long h = fnv_mix(FNV0, (unsigned)n);
    for (int i = 0; i < n; ++i) h = fnv_mix(h, grid_shape_key(p[i].grid));
    return h;
}

Launch tuned_launch(int op, unsigned long long shape, int dtype) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return Launch{0, 0};
    std::lock_guard<std::mutex> lock(tune_mu);
    const auto it = tune_table().find(TuneKey{op, dtype, dev, shape});
    return it == tune_table().end() ? Launch{0, 0} : it->second;
}

hipError_t set_tuned_launch(int op, unsigned long long shape, int dtype, Launch l) {
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(tune_mu);
    const TuneKey k{op, dtype, dev, shape};
    if (l.blocks <= 0 && l.shape == 0) tune_table().erase(k);
    else tune_table()[k] = Launch{l.blocks > 0 ? l.blocks : 0, l.shape};
    return hipSuccess;
}

hipError_t tune_stage(const StageArgs (&a)[3], int dtype, bool kinematic, int reps, hipStream_t s, Launch& best) {
    // one RK3 step: the three stages differ in their inputs and all count
    auto step = [&](int shape, int blocks) {
        hipError_t e = hipSuccess;
        for (int st = 0; st < 3 && e == hipSuccess; ++st) e = launch_stage(a[st], dtype, st, s, kinematic, blocks, shape);
        return e;
    };
    // every shape at its default count (one round of resident blocks)
    const int ns = stage_shapes(dtype, kinematic, nullptr);
    int sh = 0;
    hipError_t e = ns > 1 ? pick_fastest(ns, reps, s, [&](int i) { return step(i, 0); }, sh) : hipSuccess;
    if (e != hipSuccess) return e;
    // then block counts for that shape
    long long resident = 0, work = 0;
    stage_limits(a[0].g, dtype, kinematic, resident, work, sh);
    if (resident <= 0) return hipErrorInvalidDeviceFunction;
    const long long dflt = std::min(resident, std::max(1LL, work / 16));
    const auto cand = block_candidates(resident, work, dflt);
    int bi = 0;
    e = pick_fastest((int)cand.size(), reps, s, [&](int i) { return step(sh, cand[i]); }, bi);
    if (e != hipSuccess) return e;
    best = Launch{cand[bi], sh};
    return hipSuccess;
}

// `items` must send the last stage into the workspace (batch_item_fill's
// last_to_work); `fill` rewrites them (and the step offsets) for a shape
hipError_t tune_batched(const void* items, const long long* wfirst, int nprob, int dtype, int reps, hipStream_t s,
                        hipError_t (*fill)(void* ctx, int shape, long long& total), void* ctx, Launch& best) {
    auto step = [&](int shape, long long total, int blocks) {
        hipError_t e = hipSuccess;
        for (int st = 0; st < 3 && e == hipSuccess; ++st)
            e = launch_stage_batched(items, wfirst, nprob, total, dtype, st, blocks, s, shape);
        return e;
    };
    // shapes at the default count; the items are rewritten per shape, so
    // each shape is timed in a pass of its own (after a warm-up launch)
    const int ns = batched_shapes(dtype, nullptr);
    std::vector<float> ms(ns, 0.0f);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int pass = 0; pass < 2 && e == hipSuccess && ns > 1; ++pass)
        for (int j = 0; j < ns && e == hipSuccess; ++j) {
            const int i = pass == 0 ? j : ns - 1 - j;
            long long total = 0;
            e = fill(ctx, i, total);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = step(i, total, 0);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = step(i, total, 0);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            ms[i] += t;
        }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    int sh = 0;
    if (ns > 1) {
        const int k = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
        if (ms[k] < 0.99f * ms[0]) sh = k;
    }
    long long total = 0;
    e = fill(ctx, sh, total);
    if (e != hipSuccess) return e;
    const long long resident = batched_resident(dtype, sh);
    if (resident <= 0) return hipErrorInvalidDeviceFunction;
    const long long dflt = std::min(resident, std::max(1LL, total / 16));
    const auto cand = block_candidates(resident, total, dflt);
    int bi = 0;
    e = pick_fastest((int)cand.size(), reps, s, [&](int i) { return step(sh, total, cand[i]); }, bi);
    if (e != hipSuccess) return e;
    best = Launch{cand[bi], sh};
    return hipSuccess;
}

}  // namespace egb
