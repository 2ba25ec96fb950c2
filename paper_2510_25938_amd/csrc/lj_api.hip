// C ABI of liblj_bh.so: argument validation, workspace layout, launch
// scheduling and the HIP-graph cache of the basin-hopping step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lj_kernels.hpp"

namespace {

thread_local std::string g_err;

lj_status fail(lj_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define LJ_HIP_TRY(expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LJ_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

struct DeviceInfo {
    bool valid = false;
    bool gfx950 = false;
    int cus = 0;
};

std::mutex g_dev_mu;
std::vector<DeviceInfo> g_dev;

lj_status device_info(DeviceInfo& out) {
    int dev = 0;
    LJ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    if (!g_dev[dev].valid) {
        hipDeviceProp_t prop;
        LJ_HIP_TRY(hipGetDeviceProperties(&prop, dev));
        g_dev[dev].cus = prop.multiProcessorCount;
        g_dev[dev].gfx950 = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        g_dev[dev].valid = true;
    }
    out = g_dev[dev];
    if (!out.gfx950) return fail(LJ_E_UNSUPPORTED, "device %d is not gfx950", dev);
    return LJ_OK;
}

lj_status check_batch(const lj_batch* b, int limit, const char* what) {
    if (!b) return fail(LJ_E_ARG, "%s: batch is NULL", what);
    if (b->num < 0) return fail(LJ_E_ARG, "%s: num = %d < 0", what, b->num);
    if (b->num > 0 && !b->offset) return fail(LJ_E_ARG, "%s: offset is NULL", what);
    if (b->max_n < 0) return fail(LJ_E_ARG, "%s: max_n = %d < 0", what, b->max_n);
    if (b->max_n > limit)
        return fail(LJ_E_UNSUPPORTED, "%s: max_n = %d exceeds the limit %d", what, b->max_n, limit);
    if (b->total_atoms < 0 || b->total_atoms > INT32_MAX)
        return fail(LJ_E_ARG, "%s: total_atoms = %lld out of range", what,
                    (long long)b->total_atoms);
    if ((int64_t)b->num * b->max_n < b->total_atoms)
        return fail(LJ_E_ARG, "%s: total_atoms exceeds num * max_n", what);
    if (b->pair != LJ_PAIR_LJ && b->pair != LJ_PAIR_MORSE)
        return fail(LJ_E_ARG, "%s: pair = %d is neither LJ_PAIR_LJ nor LJ_PAIR_MORSE", what,
                    b->pair);
    if (b->pair == LJ_PAIR_MORSE && !(b->pair_rho > 0.0 && b->pair_rho <= 1.0e6))
        return fail(LJ_E_ARG, "%s: Morse pair_rho = %g is not in (0, 1e6]", what, b->pair_rho);
    if (!(b->sigma == 0.0 || (b->sigma > 0.0 && std::isfinite(b->sigma))) ||
        !(b->epsilon == 0.0 || (b->epsilon > 0.0 && std::isfinite(b->epsilon))))
        return fail(LJ_E_ARG, "%s: sigma = %g and epsilon = %g must be finite and > 0 (or 0 for 1)",
                    what, b->sigma, b->epsilon);
    return LJ_OK;
}

// The batch's units; a zero sigma or epsilon means 1.
lj::Units units_of(const lj_batch* b) {
    const double sg = b->sigma == 0.0 ? 1.0 : b->sigma;
    const double ep = b->epsilon == 0.0 ? 1.0 : b->epsilon;
    return lj::Units{sg, ep, ep / sg, sg != 1.0};
}

bool reduced_units(const lj_batch* b) {
    const lj::Units u = units_of(b);
    return u.sigma == 1.0 && u.escale == 1.0;
}

lj_status check_params(const lj_lbfgs_params* p) {
    if (!p) return fail(LJ_E_ARG, "params is NULL");
    if (p->m < 0 || p->m > LJ_MAX_M) return fail(LJ_E_ARG, "m = %d outside [0, %d]", p->m, LJ_MAX_M);
    if (!(p->gtol > 0.0)) return fail(LJ_E_ARG, "gtol must be > 0");
    if (p->max_iter < 0) return fail(LJ_E_ARG, "max_iter < 0");
    if (!(p->max_step > 0.0)) return fail(LJ_E_ARG, "max_step must be > 0");
    if (!(p->c1 > 0.0 && p->c1 < 1.0)) return fail(LJ_E_ARG, "c1 must be in (0, 1)");
    if (p->max_ls < 1) return fail(LJ_E_ARG, "max_ls must be >= 1");
    if (!(p->curv_eps >= 0.0)) return fail(LJ_E_ARG, "curv_eps must be >= 0");
    if (!(p->gtol_mixed_per_atom >= 0.0)) return fail(LJ_E_ARG, "gtol_mixed_per_atom < 0");
    if (!(p->ls_noise >= 0.0)) return fail(LJ_E_ARG, "ls_noise < 0");
    return LJ_OK;
}

lj::LbfgsDev to_dev(const lj_lbfgs_params* p) {
    lj::LbfgsDev d;
    d.m = p->m;
    d.gtol = p->gtol;
    d.max_iter = p->max_iter;
    d.max_step = p->max_step;
    d.c1 = p->c1;
    d.max_ls = p->max_ls;
    d.curv_eps = p->curv_eps;
    d.gtol_mixed_per_atom = p->gtol_mixed_per_atom;
    d.polish = p->polish;
    d.ls_noise = p->ls_noise;
    return d;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Launch-schedule table, filled by lj_autotune / lj_set_schedule.  Keys:
// eval: (precision, next_pow2(max_n)); large minimiser: (precision).
std::mutex g_sched_mu;
std::map<std::pair<int, int>, lj::EvalShape> g_eval_sched;
int g_large_sched[2] = {1, 0};  // FP64: 8 x 2 (no spills); mixed: 16 x 1 (tiled FP32 loop)

int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p *= 2;
    return p;
}

lj::EvalShape eval_schedule(int precision, int max_n) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    auto it = g_eval_sched.find({precision, pow2_at_least(max_n < 1 ? 1 : max_n)});
    if (it != g_eval_sched.end() && it->second.W * 64 * it->second.A >= max_n) return it->second;
    return lj::eval_shape(max_n);
}

int large_schedule(int precision) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    return g_large_sched[precision == LJ_MIXED ? 1 : 0];
}

// Minimiser shapes of classes 0-2, filled by lj_autotune / lj_set_schedule:
// (precision, class, largest class of the batch, power of two >= the class's
// largest N) -> shape.
std::map<std::array<int, 4>, int> g_class_sched;

// The largest N that class c can hold in a batch whose largest N is max_n.
int class_cap(int c, int max_n) {
    const int cap = lj::kClassMaxN[c];
    return max_n < cap ? (max_n < 0 ? 0 : max_n) : cap;
}

std::array<int, 4> class_key(int precision, int c, int max_n) {
    return {precision == LJ_MIXED ? 1 : 0, c, lj::class_of(max_n < 0 ? 0 : max_n),
            pow2_at_least(class_cap(c, max_n) < 1 ? 1 : class_cap(c, max_n))};
}

// Built-in rule for the shape of class c (0-2).
int default_class_shape(int c, int max_n, int top_class, int mixed, int num, int cus) {
    const int cmax = class_cap(c, max_n);
    if (c == 0) {
        // Several clusters per wavefront once the batch has more than two
        // clusters per SIMD: each wavefront then does the work of two or four
        // (16384 x LJ13: 1.75 instead of 4.2 ms, FP64); below that the batch
        // waits for its slowest cluster, and a packed wavefront waits for the
        // slowest of its clusters, so one cluster per wavefront is as fast.
        const bool many = num > 2 * 4 * cus;
        int shape = 0;
        if (cmax <= 16)
            shape = many ? 3 : 1;
        else if (cmax <= 32 && many)
            shape = 2;
        // Two wavefronts per SIMD (registers capped, some spilled) once the
        // call holds only this class and has more wavefronts than SIMDs: the
        // second wavefront fills the first one's issue gaps (2048 x LJ38
        // mixed: 3.85 instead of 4.39 ms; 16384 x LJ13: 1.82 instead of 2.27
        // ms FP64), while with one wavefront per SIMD the spills only cost.
        const long waves = ((long)num + lj::shape_clusters_per_wg(0, shape) - 1) /
                           lj::shape_clusters_per_wg(0, shape);
        if (top_class == 0 && waves > 4L * cus) shape += 4;
        return shape;
    }
    if (c == 2) return cmax <= 192 ? 1 : 0; // three wavefronts
    // Class 1 as one wavefront with two atoms per lane: about 1.5 times the
    // time per iteration of two wavefronts, but one SIMD per team instead of
    // two, so twice the teams drain the class.  That wins when the class
    // shares the call with larger clusters, and on the FP64 path when the
    // batch has at least one cluster per SIMD; otherwise the slowest cluster
    // decides and two wavefronts are faster (mixed-path registers spill more
    // in the one-wavefront form).
    return (top_class >= 2 || (!mixed && num >= 4 * cus)) ? 1 : 0;
}

int class_schedule(int precision, int c, int max_n, int num, int cus) {
    const int top = lj::class_of(max_n < 0 ? 0 : max_n);
    if (c == 3) return large_schedule(precision);
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        auto it = g_class_sched.find(class_key(precision, c, max_n));
        if (it != g_class_sched.end() && lj::shape_max_n(c, it->second) >= class_cap(c, max_n))
            return it->second;
    }
    return default_class_shape(c, max_n, top, precision == LJ_MIXED, num, cus);
}

// Workspace carve-up of one minimisation call, and the shape of each class.
struct MinLayout {
    size_t list = 0, cls = 0, queue = 0, hist = 0, total = 0;
    int top_class = -1;
    int shape[lj::kNumClasses] = {0, 0, 0, 0};
    int grid[lj::kNumClasses] = {0, 0, 0, 0};
};

// force (nullable): a shape per class, -1 for the schedule table's choice.
lj_status min_layout(int num, int max_n, int mixed, int pot, MinLayout& L,
                     const int* force = nullptr) {
    DeviceInfo di;
    lj_status s = device_info(di);
    if (s != LJ_OK) return s;
    const int prec = mixed ? LJ_MIXED : LJ_FP64;
    size_t off = 0;
    L.list = off;
    off = align_up(off + sizeof(int32_t) * (size_t)(num > 0 ? num : 1));
    L.cls = off;
    off = align_up(off + sizeof(int32_t) * 2 * lj::kNumClasses);
    L.queue = off;
    off = align_up(off + sizeof(int32_t) * lj::kNumClasses);
    // the plan rejects clusters above max_n, so max_n bounds every class
    L.top_class = lj::class_of(max_n < 0 ? 0 : max_n);
    for (int c = 0; c <= L.top_class; ++c) {
        L.shape[c] = (force && force[c] >= 0) ? force[c] : class_schedule(prec, c, max_n, num, di.cus);
        if (L.shape[c] < 0 || L.shape[c] >= lj::class_shapes(c) ||
            lj::shape_max_n(c, L.shape[c]) < class_cap(c, max_n))
            return fail(LJ_E_ARG, "minimiser shape %d of class %d does not hold %d atoms",
                        L.shape[c], c, class_cap(c, max_n));
    }
    auto grid_for = [&](int c, int shape, int& g_out) -> lj_status {
        int per_cu = 0;
        LJ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, lj::minimize_kernel_for(mixed, pot, c, shape), lj::class_block(c, shape),
            lj::class_dyn_lds(c, shape, max_n, pot)));
        if (per_cu < 1) per_cu = 1;
        const int per_wg = lj::shape_clusters_per_wg(c, shape);
        long g = (long)per_cu * di.cus;
        const long need = ((long)num + per_wg - 1) / per_wg;
        if (g > need) g = need;
        if (g < 1) g = 1;
        g_out = (int)g;
        return LJ_OK;
    };
    for (int c = 0; c <= L.top_class; ++c)
        if ((s = grid_for(c, L.shape[c], L.grid[c])) != LJ_OK) return s;
    L.hist = off;
    if (L.top_class >= 3) {
        // sized for the largest grid of any large-cluster shape, so a workspace
        // stays valid whichever shape the schedule table selects
        size_t hist = 0;
        for (int k = 0; k < lj::class_shapes(3); ++k) {
            int g = 0;
            if ((s = grid_for(3, k, g)) != LJ_OK) return s;
            const size_t b = lj::class_hist_bytes_per_wg(3, k) * (size_t)g;
            if (b > hist) hist = b;
        }
        off = align_up(off + hist);
    }
    L.total = off;
    return LJ_OK;
}

// Side streams (default priority) and events used to run the minimiser's size
// classes concurrently: fork from the caller's stream after the plan kernel,
// the largest class on the caller's stream and each other class on a side
// stream, join back before returning.  The pattern is also
// valid under stream capture (parallel graph branches).  Each (device, caller
// stream) pair has its own set: a side stream pulled into a capture stays in
// capture mode until the capture ends, so a set shared with callers on other
// streams would let their eager launches land in that graph.
struct SideStreams {
    bool ready = false;
    hipStream_t s[lj::kNumClasses];
    hipEvent_t fork;
    hipEvent_t join[lj::kNumClasses];
    std::mutex mu;
};
std::mutex g_side_mu;
std::map<std::pair<int, hipStream_t>, SideStreams*> g_side;
constexpr size_t kMaxSideSets = 16;  // beyond this, classes run in turn on the caller's stream

// out = nullptr (and LJ_OK) once kMaxSideSets caller streams have a set.
lj_status side_streams(hipStream_t caller, SideStreams*& out) {
    out = nullptr;
    int dev = 0;
    LJ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto it = g_side.find({dev, caller});
    if (it == g_side.end()) {
        if (g_side.size() >= kMaxSideSets) return LJ_OK;
        it = g_side.emplace(std::make_pair(dev, caller), new SideStreams()).first;  // kept until exit
    }
    SideStreams* ss = it->second;
    if (!ss->ready) {
        for (int c = 0; c < lj::kNumClasses; ++c) {
            LJ_HIP_TRY(hipStreamCreateWithFlags(&ss->s[c], hipStreamNonBlocking));
            LJ_HIP_TRY(hipEventCreateWithFlags(&ss->join[c], hipEventDisableTiming));
        }
        LJ_HIP_TRY(hipEventCreateWithFlags(&ss->fork, hipEventDisableTiming));
        ss->ready = true;
    }
    out = ss;
    return LJ_OK;
}

lj_status enqueue_minimize(const lj_batch* b, const int32_t* active, double* xyz, double* energy,
                           double* gnorm, int32_t* iters, int32_t* evals, int32_t* status,
                           double* xyz_switch, const lj::LbfgsDev& p, int mixed,
                           const MinLayout& L, char* ws, hipStream_t st,
                           bool concurrent = true) {
    if (b->num == 0) return LJ_OK;
    lj::Plan plan;
    plan.list = reinterpret_cast<int32_t*>(ws + L.list);
    plan.cls = reinterpret_cast<int32_t*>(ws + L.cls);
    plan.queue = reinterpret_cast<int32_t*>(ws + L.queue);
    LJ_HIP_TRY(lj::launch_plan(b->offset, b->num, b->max_n, active, plan, status, st));
    lj::MinArgs a;
    a.offset = b->offset;
    a.total = b->total_atoms;
    a.xyz = xyz;
    a.energy = energy;
    a.gnorm = gnorm;
    a.iters = iters;
    a.evals = evals;
    a.status = status;
    a.xyz_switch = mixed ? xyz_switch : nullptr;
    a.plan = plan;
    a.p = p;
    a.pot = b->pair;
    a.rho = b->pair_rho;
    a.u = units_of(b);
    a.max_n = b->max_n;
    a.up_n = 0;
    if (L.top_class == 0) {
        a.cls = 0;
        a.hist = nullptr;
        LJ_HIP_TRY(lj::launch_minimize_class(mixed, 0, L.shape[0], L.grid[0], a, st));
        return LJ_OK;
    }
    // several size classes: run them concurrently on side streams
    SideStreams* ss = nullptr;
    if (concurrent) {
        lj_status r = side_streams(st, ss);
        if (r != LJ_OK) return r;
    }
    if (!ss) {  // no side streams (for this caller stream): the classes run in turn
        for (int c = L.top_class; c >= 0; --c) {
            a.cls = c;
            a.hist = (c == 3) ? reinterpret_cast<double*>(ws + L.hist) : nullptr;
            LJ_HIP_TRY(lj::launch_minimize_class(mixed, c, L.shape[c], L.grid[c], a, st));
        }
        return LJ_OK;
    }
    std::lock_guard<std::mutex> lk(ss->mu);
    LJ_HIP_TRY(hipEventRecord(ss->fork, st));
    // The largest class goes first, on the caller's stream, and the others on
    // the first side streams.  Streams share the device's few hardware queues,
    // which run in order: with a side stream per class, two classes could land
    // on one queue and run one after the other (the uneven 4096-cluster batch
    // took 60 instead of 47 ms that way).
    a.cls = L.top_class;
    a.hist = (L.top_class == 3) ? reinterpret_cast<double*>(ws + L.hist) : nullptr;
    LJ_HIP_TRY(lj::launch_minimize_class(mixed, L.top_class, L.shape[L.top_class],
                                         L.grid[L.top_class], a, st));
    a.hist = nullptr;
    for (int c = L.top_class - 1; c >= 0; --c) {
        const int k = L.top_class - 1 - c;
        a.cls = c;
        LJ_HIP_TRY(hipStreamWaitEvent(ss->s[k], ss->fork, 0));
        LJ_HIP_TRY(lj::launch_minimize_class(mixed, c, L.shape[c], L.grid[c], a, ss->s[k]));
        LJ_HIP_TRY(hipEventRecord(ss->join[k], ss->s[k]));
    }
    for (int k = 0; k < L.top_class; ++k) LJ_HIP_TRY(hipStreamWaitEvent(st, ss->join[k], 0));
    return LJ_OK;
}

// Basin-hopping workspace carve-up.
struct BhLayout {
    size_t xc = 0, cand_off = 0, ce = 0, cg = 0, ci = 0, cv = 0, cs = 0, dec = 0, pe = 0, pg = 0,
           pi = 0, pv = 0, ps = 0, min = 0, total = 0;
    MinLayout cand_min, polish_min;
    int64_t cand_total = 0;
    int cand_num = 0;
};

lj_status bh_layout(const lj_batch* ch, const lj_bh_params* bh, int mixed, BhLayout& L) {
    const int n = bh->cands;
    L.cand_num = ch->num * n;
    L.cand_total = ch->total_atoms * n;
    if (L.cand_total > INT32_MAX) return fail(LJ_E_ARG, "candidate atom count exceeds int32");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes > 0 ? bytes : 1));
        return at;
    };
    L.xc = take(sizeof(double) * 3 * (size_t)L.cand_total);
    L.cand_off = take(sizeof(int32_t) * ((size_t)L.cand_num + 1));
    L.ce = take(sizeof(double) * (size_t)L.cand_num);
    L.cg = take(sizeof(double) * (size_t)L.cand_num);
    L.ci = take(sizeof(int32_t) * (size_t)L.cand_num);
    L.cv = take(sizeof(int32_t) * (size_t)L.cand_num);
    L.cs = take(sizeof(int32_t) * (size_t)L.cand_num);
    L.dec = take(sizeof(int32_t) * 2 * (size_t)ch->num);
    L.pe = take(sizeof(double) * (size_t)ch->num);
    L.pg = take(sizeof(double) * (size_t)ch->num);
    L.pi = take(sizeof(int32_t) * (size_t)ch->num);
    L.pv = take(sizeof(int32_t) * (size_t)ch->num);
    L.ps = take(sizeof(int32_t) * (size_t)ch->num);
    lj_status s = min_layout(L.cand_num, ch->max_n, mixed, ch->pair, L.cand_min);
    if (s != LJ_OK) return s;
    s = min_layout(ch->num, ch->max_n, 0, ch->pair, L.polish_min);
    if (s != LJ_OK) return s;
    L.min = off;
    const size_t m = L.cand_min.total > L.polish_min.total ? L.cand_min.total : L.polish_min.total;
    off = align_up(off + m);
    L.total = off;
    return LJ_OK;
}

lj_status check_bh(const lj_batch* ch, const lj_bh_params* bh) {
    if (!bh) return fail(LJ_E_ARG, "bh params is NULL");
    if (!reduced_units(ch))
        return fail(LJ_E_UNSUPPORTED, "basin hopping runs in reduced units: sigma and epsilon "
                    "of the chains' batch must be 1 (or 0)");
    if (bh->cands < 1 || bh->cands > LJ_MAX_CANDS)
        return fail(LJ_E_ARG, "cands = %d outside [1, %d]", bh->cands, LJ_MAX_CANDS);
    if (!(bh->kT > 0.0)) return fail(LJ_E_ARG, "kT must be > 0");
    if (bh->adapt_interval < 1) return fail(LJ_E_ARG, "adapt_interval must be >= 1");
    if (!(bh->factor > 0.0)) return fail(LJ_E_ARG, "factor must be > 0");
    if (!std::isfinite(bh->target_rate)) return fail(LJ_E_ARG, "target_rate not finite");
    if ((int64_t)ch->num * bh->cands > INT32_MAX) return fail(LJ_E_ARG, "too many candidates");
    return LJ_OK;
}

// One basin-hopping step enqueued on st.
lj_status enqueue_bh_step(const lj_batch* ch, const lj::BhStateDev& s, const lj::BhDev& p,
                          const lj_lbfgs_params* lp, int mixed, const lj::BhTraceDev& tr,
                          const BhLayout& L, char* ws, hipStream_t st) {
    double* xc = reinterpret_cast<double*>(ws + L.xc);
    int32_t* cand_off = reinterpret_cast<int32_t*>(ws + L.cand_off);
    double* ce = reinterpret_cast<double*>(ws + L.ce);
    int32_t* dec = reinterpret_cast<int32_t*>(ws + L.dec);
    LJ_HIP_TRY(lj::launch_perturb(ch->offset, ch->num, ch->max_n, ch->total_atoms, s, p, xc,
                                  cand_off, st));
    lj_batch cb;
    cb.num = L.cand_num;
    cb.offset = cand_off;
    cb.max_n = ch->max_n;
    cb.total_atoms = L.cand_total;
    cb.pair = ch->pair;
    cb.pair_rho = ch->pair_rho;
    cb.sigma = 1.0;
    cb.epsilon = 1.0;
    lj::LbfgsDev d = to_dev(lp);
    if (mixed) d.polish = 0;  // only the accepted candidate is polished
    lj_status r = enqueue_minimize(&cb, nullptr, xc, ce, reinterpret_cast<double*>(ws + L.cg),
                                   reinterpret_cast<int32_t*>(ws + L.ci),
                                   reinterpret_cast<int32_t*>(ws + L.cv),
                                   reinterpret_cast<int32_t*>(ws + L.cs), nullptr, d, mixed,
                                   L.cand_min, ws + L.min, st);
    if (r != LJ_OK) return r;
    // without a polish, decide also finalizes the step (one launch fewer)
    LJ_HIP_TRY(lj::launch_decide(ch->offset, ch->num, ch->max_n, ch->total_atoms, s, p, xc, ce, dec,
                                 mixed ? nullptr : &tr, st));
    if (!mixed) return LJ_OK;
    // FP64 polish of the accepted candidates (the active mask is the accepted flags)
    double* pe = reinterpret_cast<double*>(ws + L.pe);
    r = enqueue_minimize(ch, dec + ch->num, s.xyz_cur, pe, reinterpret_cast<double*>(ws + L.pg),
                         reinterpret_cast<int32_t*>(ws + L.pi),
                         reinterpret_cast<int32_t*>(ws + L.pv),
                         reinterpret_cast<int32_t*>(ws + L.ps), nullptr, to_dev(lp), 0,
                         L.polish_min, ws + L.min, st);
    if (r != LJ_OK) return r;
    LJ_HIP_TRY(lj::launch_finalize(ch->offset, ch->num, ch->max_n, ch->total_atoms, s, p, ce, dec, pe,
                                   reinterpret_cast<const int32_t*>(ws + L.ps), tr, st));
    return LJ_OK;
}

// HIP-graph cache of one basin-hopping step, keyed by every argument byte.
// `done` is recorded after each launch, so an evicted graph is destroyed only
// once its last launch has finished.
struct GraphEntry {
    std::vector<unsigned char> key;
    int device;
    hipGraphExec_t exec;
    hipEvent_t done;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
constexpr size_t kMaxGraphs = 16;

std::atomic<int64_t> g_graph_captures{0};

// Appends the bytes of one scalar or pointer.  Structs are keyed field by
// field: their padding bytes are indeterminate and would make equal
// arguments compare unequal.
template <typename T>
void key_add(std::vector<unsigned char>& k, const T& v) {
    static_assert(std::is_arithmetic<T>::value || std::is_pointer<T>::value,
                  "key structs field by field");
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
    k.insert(k.end(), p, p + sizeof(T));
}

std::vector<unsigned char> step_key(const lj_batch* ch, const lj::BhStateDev& sd,
                                    const lj::BhDev& pd, const lj_lbfgs_params* lp,
                                    int32_t precision, const lj::BhTraceDev& td, const void* ws,
                                    size_t ws_bytes, hipStream_t st, const BhLayout& L) {
    std::vector<unsigned char> k;
    k.reserve(320);
    key_add(k, ch->num);
    key_add(k, ch->offset);
    key_add(k, ch->max_n);
    key_add(k, ch->total_atoms);
    key_add(k, ch->pair);
    key_add(k, ch->pair_rho);
    key_add(k, ch->sigma);
    key_add(k, ch->epsilon);
    for (const void* ptr : {(const void*)sd.xyz_cur, (const void*)sd.e_cur, (const void*)sd.step,
                            (const void*)sd.win_accepts, (const void*)sd.step_index,
                            (const void*)sd.e_best_seen, (const void*)sd.e_best_acc,
                            (const void*)sd.xyz_best})
        key_add(k, ptr);
    key_add(k, pd.cands);
    key_add(k, pd.kT);
    key_add(k, pd.adapt_interval);
    key_add(k, pd.target_rate);
    key_add(k, pd.factor);
    key_add(k, pd.seed);
    key_add(k, lp->m);
    key_add(k, lp->gtol);
    key_add(k, lp->max_iter);
    key_add(k, lp->max_step);
    key_add(k, lp->c1);
    key_add(k, lp->max_ls);
    key_add(k, lp->curv_eps);
    key_add(k, lp->gtol_mixed_per_atom);
    key_add(k, lp->polish);
    key_add(k, lp->ls_noise);
    key_add(k, precision);
    for (const void* ptr : {(const void*)td.e_trial, (const void*)td.accepted,
                            (const void*)td.e_best, (const void*)td.e_best_acc,
                            (const void*)td.e_cur, (const void*)td.step, (const void*)td.e_cand,
                            (const void*)td.polish_status})
        key_add(k, ptr);
    key_add(k, td.cap);
    key_add(k, ws);
    key_add(k, ws_bytes);
    key_add(k, st);
    // a graph keeps the launch shapes it captured: the candidates' minimiser
    // shapes and, on the mixed path, those of the accepted candidates' polish
    for (int c = 0; c < lj::kNumClasses; ++c) {
        key_add(k, L.cand_min.shape[c]);
        key_add(k, L.polish_min.shape[c]);
    }
    return k;
}


}  // namespace

// Scratch of lj_bh_minimize_batch_noalloc: the work list, size-class table and
// claim counters of one call, in a fixed array that every device holding the
// library keeps until the process ends.  Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[LJ_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_ptr;  // per device

lj_status noalloc_scratch(char*& out) {
    int dev = 0;
    LJ_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        LJ_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LJ_E_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    out = g_scratch_ptr[dev];
    return LJ_OK;
}

}  // namespace

extern "C" {

const char* lj_status_string(lj_status s) {
    switch (s) {
        case LJ_OK: return "LJ_OK";
        case LJ_E_ARG: return "LJ_E_ARG: invalid argument";
        case LJ_E_HIP: return "LJ_E_HIP: HIP runtime error";
        case LJ_E_WORKSPACE: return "LJ_E_WORKSPACE: workspace missing or too small";
        case LJ_E_UNSUPPORTED: return "LJ_E_UNSUPPORTED: size above the compiled limit or not gfx950";
    }
    return "unknown lj_status";
}

const char* lj_last_error(void) { return g_err.c_str(); }

int32_t lj_abi_version(void) { return LJ_ABI_VERSION; }

int64_t lj_bh_graph_captures(void) { return g_graph_captures.load(); }

void lj_lbfgs_defaults(lj_lbfgs_params* p) {
    if (!p) return;
    p->m = 10;
    p->gtol = 1e-6;
    p->max_iter = 10000;
    p->max_step = 0.2;
    p->c1 = 1e-4;
    p->max_ls = 30;
    p->curv_eps = 1e-10;
    p->gtol_mixed_per_atom = 1e-5;
    p->polish = 1;
    p->ls_noise = 5e-7;
}

lj_status lj_energy_grad_batch(const lj_batch* batch, const double* xyz, double* energy,
                               double* grad, int32_t precision, void* stream) {
    g_err.clear();
    lj_status s = check_batch(batch, LJ_MAX_ATOMS_EVAL, "lj_energy_grad_batch");
    if (s != LJ_OK) return s;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return fail(LJ_E_ARG, "precision = %d is neither LJ_FP64 nor LJ_MIXED", precision);
    if (batch->num == 0) return LJ_OK;
    if (!energy) return fail(LJ_E_ARG, "energy is NULL");
    if (batch->total_atoms > 0 && !xyz) return fail(LJ_E_ARG, "xyz is NULL");
    DeviceInfo di;
    s = device_info(di);
    if (s != LJ_OK) return s;
    LJ_HIP_TRY(lj::launch_energy_grad(precision == LJ_MIXED, batch->pair,
                                      eval_schedule(precision, batch->max_n), batch->num,
                                      batch->offset, batch->total_atoms, xyz, energy, grad,
                                      batch->pair_rho, units_of(batch),
                                      static_cast<hipStream_t>(stream)));
    return LJ_OK;
}

size_t lj_minimize_workspace_bytes(const lj_batch* batch, const lj_lbfgs_params* params,
                                   int32_t precision) {
    (void)params;
    if (check_batch(batch, LJ_MAX_ATOMS_MIN, "lj_minimize_workspace_bytes") != LJ_OK) return 0;
    MinLayout L;
    if (min_layout(batch->num, batch->max_n, precision == LJ_MIXED, batch->pair, L) != LJ_OK)
        return 0;
    return L.total;
}

lj_status lj_bh_minimize_batch(const lj_batch* batch, double* xyz, double* energy, double* gnorm,
                               int32_t* iters, int32_t* evals, int32_t* status,
                               double* xyz_switch, const lj_lbfgs_params* params,
                               int32_t precision, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    lj_status s = check_batch(batch, LJ_MAX_ATOMS_MIN, "lj_bh_minimize_batch");
    if (s != LJ_OK) return s;
    if ((s = check_params(params)) != LJ_OK) return s;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return fail(LJ_E_ARG, "precision = %d is neither LJ_FP64 nor LJ_MIXED", precision);
    if (batch->num == 0) return LJ_OK;
    if (!energy || !gnorm || !iters || !evals || !status)
        return fail(LJ_E_ARG, "an output array is NULL");
    if (batch->total_atoms > 0 && !xyz) return fail(LJ_E_ARG, "xyz is NULL");
    MinLayout L;
    if ((s = min_layout(batch->num, batch->max_n, precision == LJ_MIXED, batch->pair, L)) != LJ_OK) return s;
    if (!ws || ws_bytes < L.total)
        return fail(LJ_E_WORKSPACE, "workspace of %zu bytes given, %zu needed", ws_bytes, L.total);
    return enqueue_minimize(batch, nullptr, xyz, energy, gnorm, iters, evals, status, xyz_switch,
                            to_dev(params), precision == LJ_MIXED, L, static_cast<char*>(ws),
                            static_cast<hipStream_t>(stream));
}

lj_status lj_bh_minimize_batch_noalloc(const lj_batch* batch, double* xyz, double* energy,
                                       double* gnorm, int32_t* iters, int32_t* evals,
                                       int32_t* status, double* xyz_switch,
                                       const lj_lbfgs_params* params, int32_t precision,
                                       void* stream) {
    g_err.clear();
    lj_status s = check_batch(batch, LJ_MAX_ATOMS_MIN, "lj_bh_minimize_batch_noalloc");
    if (s != LJ_OK) return s;
    if ((s = check_params(params)) != LJ_OK) return s;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return fail(LJ_E_ARG, "precision = %d is neither LJ_FP64 nor LJ_MIXED", precision);
    if (batch->num == 0) return LJ_OK;
    if (!energy || !gnorm || !iters || !evals || !status)
        return fail(LJ_E_ARG, "an output array is NULL");
    if (batch->total_atoms > 0 && !xyz) return fail(LJ_E_ARG, "xyz is NULL");
    if (batch->max_n > LJ_NOALLOC_MAX_ATOMS)
        return fail(LJ_E_UNSUPPORTED,
                    "lj_bh_minimize_batch_noalloc: max_n = %d exceeds %d (larger clusters keep "
                    "their L-BFGS history in a workspace; use lj_bh_minimize_batch)",
                    batch->max_n, LJ_NOALLOC_MAX_ATOMS);
    if (batch->num > LJ_NOALLOC_MAX_CLUSTERS)
        return fail(LJ_E_WORKSPACE,
                    "lj_bh_minimize_batch_noalloc: %d clusters exceed the %d that its %d-byte "
                    "static scratch holds; use lj_bh_minimize_batch",
                    batch->num, LJ_NOALLOC_MAX_CLUSTERS, LJ_NOALLOC_SCRATCH_BYTES);
    MinLayout L;
    if ((s = min_layout(batch->num, batch->max_n, precision == LJ_MIXED, batch->pair, L)) != LJ_OK)
        return s;
    if (L.total > (size_t)LJ_NOALLOC_SCRATCH_BYTES)
        return fail(LJ_E_WORKSPACE, "lj_bh_minimize_batch_noalloc: %zu bytes of scratch needed, "
                    "%d available", L.total, LJ_NOALLOC_SCRATCH_BYTES);
    char* ws = nullptr;
    if ((s = noalloc_scratch(ws)) != LJ_OK) return s;
    // the size classes run in turn on the caller's stream (no side streams are
    // created); the plan kernel rewrites the whole scratch it uses, counters
    // included, before the minimiser reads it
    return enqueue_minimize(batch, nullptr, xyz, energy, gnorm, iters, evals, status, xyz_switch,
                            to_dev(params), precision == LJ_MIXED, L, ws,
                            static_cast<hipStream_t>(stream), false);
}

size_t lj_bh_workspace_bytes(const lj_batch* chains, const lj_bh_params* bh,
                             const lj_lbfgs_params* params, int32_t precision) {
    (void)params;
    if (check_batch(chains, LJ_MAX_ATOMS_MIN, "lj_bh_workspace_bytes") != LJ_OK) return 0;
    if (check_bh(chains, bh) != LJ_OK) return 0;
    BhLayout L;
    if (bh_layout(chains, bh, precision == LJ_MIXED, L) != LJ_OK) return 0;
    return L.total;
}

lj_status lj_bh_step(const lj_batch* chains, const lj_bh_state* state, const lj_bh_params* bh,
                     const lj_lbfgs_params* params, int32_t precision, int32_t num_steps,
                     const lj_bh_trace* trace, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    lj_status s = check_batch(chains, LJ_MAX_ATOMS_MIN, "lj_bh_step");
    if (s != LJ_OK) return s;
    if ((s = check_params(params)) != LJ_OK) return s;
    if ((s = check_bh(chains, bh)) != LJ_OK) return s;
    if (precision != LJ_FP64 && precision != LJ_MIXED)
        return fail(LJ_E_ARG, "precision = %d is neither LJ_FP64 nor LJ_MIXED", precision);
    if (num_steps < 0) return fail(LJ_E_ARG, "num_steps < 0");
    if (!state) return fail(LJ_E_ARG, "state is NULL");
    if (chains->num == 0 || num_steps == 0) return LJ_OK;
    if (!state->xyz_cur || !state->e_cur || !state->step || !state->win_accepts ||
        !state->step_index || !state->e_best_seen || !state->e_best_acc || !state->xyz_best)
        return fail(LJ_E_ARG, "a state array is NULL");
    if (trace && trace->capacity_steps < 0) return fail(LJ_E_ARG, "trace capacity < 0");
    const int mixed = precision == LJ_MIXED;
    BhLayout L;
    if ((s = bh_layout(chains, bh, mixed, L)) != LJ_OK) return s;
    if (!ws || ws_bytes < L.total)
        return fail(LJ_E_WORKSPACE, "workspace of %zu bytes given, %zu needed", ws_bytes, L.total);

    lj::BhStateDev sd{state->xyz_cur, state->e_cur,       state->step,       state->win_accepts,
                      state->step_index, state->e_best_seen, state->e_best_acc, state->xyz_best};
    lj::BhDev pd{bh->cands, bh->kT, bh->adapt_interval, bh->target_rate, bh->factor, bh->seed};
    lj::BhTraceDev td{};
    if (trace)
        td = lj::BhTraceDev{trace->e_trial, trace->accepted, trace->e_best, trace->e_best_acc,
                            trace->e_cur,   trace->step,     trace->e_cand, trace->polish_status,
                            trace->capacity_steps};
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);

    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st) LJ_HIP_TRY(hipStreamIsCapturing(st, &cap));
    if (!st || cap != hipStreamCaptureStatusNone) {
        for (int k = 0; k < num_steps; ++k)
            if ((s = enqueue_bh_step(chains, sd, pd, params, mixed, td, L, w, st)) != LJ_OK) return s;
        return LJ_OK;
    }

    int dev = 0;
    LJ_HIP_TRY(hipGetDevice(&dev));
    const std::vector<unsigned char> key =
        step_key(chains, sd, pd, params, precision, td, ws, ws_bytes, st, L);
    // Graphs are launched with the cache locked, so another thread's insertion
    // cannot evict and destroy a graph between its lookup and its launch.
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto& e : g_graphs)
            if (e.device == dev && e.key == key) {
                for (int k = 0; k < num_steps; ++k) LJ_HIP_TRY(hipGraphLaunch(e.exec, st));
                LJ_HIP_TRY(hipEventRecord(e.done, st));
                return LJ_OK;
            }
    }
    LJ_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    s = enqueue_bh_step(chains, sd, pd, params, mixed, td, L, w, st);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(st, &graph);
    if (s != LJ_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (ec != hipSuccess) return fail(LJ_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess) return fail(LJ_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ec));
    hipEvent_t done = nullptr;
    ec = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (ec != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return fail(LJ_E_HIP, "hipEventCreateWithFlags: %s", hipGetErrorString(ec));
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graphs.size() >= kMaxGraphs) {
        GraphEntry& old = g_graphs.front();
        (void)hipEventSynchronize(old.done);  // its last launch has finished
        (void)hipGraphExecDestroy(old.exec);
        (void)hipEventDestroy(old.done);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back(GraphEntry{key, dev, exec, done});
    g_graph_captures.fetch_add(1);
    for (int k = 0; k < num_steps; ++k) LJ_HIP_TRY(hipGraphLaunch(exec, st));
    LJ_HIP_TRY(hipEventRecord(done, st));
    return LJ_OK;
}

lj_status lj_set_schedule(int32_t kind, int32_t precision, int32_t max_n, int32_t w, int32_t a) {
    g_err.clear();
    if (precision != LJ_FP64 && precision != LJ_MIXED) return fail(LJ_E_ARG, "bad precision");
    if (kind == LJ_SCHED_EVAL) {
        lj::EvalShape sh{w, a};
        if (!lj::eval_shape_supported(sh)) return fail(LJ_E_ARG, "unsupported shape %dx%d", w, a);
        if (max_n < 0 || max_n > LJ_MAX_ATOMS_EVAL) return fail(LJ_E_ARG, "max_n out of range");
        if (64 * w * a < max_n) return fail(LJ_E_ARG, "shape %dx%d holds fewer than %d atoms", w, a, max_n);
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_eval_sched[{precision, pow2_at_least(max_n < 1 ? 1 : max_n)}] = sh;
        return LJ_OK;
    }
    if (kind == LJ_SCHED_MIN_LARGE) {
        if (w < 0 || w >= lj::kNumLargeShapes) return fail(LJ_E_ARG, "large-cluster shape %d", w);
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_large_sched[precision == LJ_MIXED ? 1 : 0] = w;
        return LJ_OK;
    }
    if (kind >= LJ_SCHED_MIN_CLASS0 && kind <= LJ_SCHED_MIN_CLASS2) {
        const int c = kind - LJ_SCHED_MIN_CLASS0;
        if (max_n < 0 || max_n > LJ_MAX_ATOMS_MIN) return fail(LJ_E_ARG, "max_n out of range");
        if (lj::class_of(max_n) < c)
            return fail(LJ_E_ARG, "a batch of at most %d atoms has no class-%d clusters", max_n, c);
        if (w == -1) {  // back to the built-in rule
            std::lock_guard<std::mutex> lk(g_sched_mu);
            g_class_sched.erase(class_key(precision, c, max_n));
            return LJ_OK;
        }
        if (w < 0 || w >= lj::class_shapes(c)) return fail(LJ_E_ARG, "class-%d shape %d", c, w);
        if (lj::shape_max_n(c, w) < class_cap(c, max_n))
            return fail(LJ_E_ARG, "class-%d shape %d holds at most %d atoms, not %d", c, w,
                        lj::shape_max_n(c, w), class_cap(c, max_n));
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_class_sched[class_key(precision, c, max_n)] = w;
        return LJ_OK;
    }
    return fail(LJ_E_ARG, "unknown schedule kind %d", kind);
}

lj_status lj_get_schedule(int32_t kind, int32_t precision, int32_t max_n, int32_t* w, int32_t* a) {
    g_err.clear();
    if (!w || !a) return fail(LJ_E_ARG, "NULL output");
    if (precision != LJ_FP64 && precision != LJ_MIXED) return fail(LJ_E_ARG, "bad precision");
    if (kind == LJ_SCHED_EVAL) {
        const lj::EvalShape sh = eval_schedule(precision, max_n);
        *w = sh.W;
        *a = sh.A;
        return LJ_OK;
    }
    if (kind == LJ_SCHED_MIN_LARGE) {
        *w = large_schedule(precision);
        *a = 0;
        return LJ_OK;
    }
    if (kind >= LJ_SCHED_MIN_CLASS0 && kind <= LJ_SCHED_MIN_CLASS2) {
        const int c = kind - LJ_SCHED_MIN_CLASS0;
        if (max_n < 0 || max_n > LJ_MAX_ATOMS_MIN) return fail(LJ_E_ARG, "max_n out of range");
        std::lock_guard<std::mutex> lk(g_sched_mu);
        auto it = g_class_sched.find(class_key(precision, c, max_n));
        *w = it == g_class_sched.end() ? -1 : it->second;
        *a = *w < 0 ? 0 : lj::shape_clusters_per_wg(c, *w);
        return LJ_OK;
    }
    return fail(LJ_E_ARG, "unknown schedule kind %d", kind);
}

size_t lj_autotune_workspace_bytes(const lj_batch* batch, int32_t precision) {
    if (check_batch(batch, LJ_MAX_ATOMS_EVAL, "lj_autotune_workspace_bytes") != LJ_OK) return 0;
    size_t off = align_up(sizeof(double) * (size_t)(batch->num > 0 ? batch->num : 1));  // energy
    off = align_up(off + sizeof(double) * 3 * (size_t)batch->total_atoms);              // grad
    if (batch->max_n <= LJ_MAX_ATOMS_MIN) {
        off = align_up(off + sizeof(double) * 3 * (size_t)batch->total_atoms);  // xyz copy
        off = align_up(off + 5 * sizeof(double) * (size_t)batch->num);          // outputs
        MinLayout L;
        if (min_layout(batch->num, batch->max_n, precision == LJ_MIXED, batch->pair, L) != LJ_OK)
        return 0;
        off = align_up(off + L.total);
    }
    return off;
}

lj_status lj_autotune(const lj_batch* batch, const double* xyz, int32_t precision, void* ws,
                      size_t ws_bytes, void* stream, float* best_eval_ms, float* best_min_ms) {
    g_err.clear();
    lj_status s = check_batch(batch, LJ_MAX_ATOMS_EVAL, "lj_autotune");
    if (s != LJ_OK) return s;
    if (precision != LJ_FP64 && precision != LJ_MIXED) return fail(LJ_E_ARG, "bad precision");
    if (batch->num == 0) return LJ_OK;
    if (batch->total_atoms > 0 && !xyz) return fail(LJ_E_ARG, "xyz is NULL");
    DeviceInfo di;
    if ((s = device_info(di)) != LJ_OK) return s;
    const size_t need = lj_autotune_workspace_bytes(batch, precision);
    if (!ws || ws_bytes < need)
        return fail(LJ_E_WORKSPACE, "workspace of %zu bytes given, %zu needed", ws_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    double* e = reinterpret_cast<double*>(w);
    size_t off = align_up(sizeof(double) * (size_t)batch->num);
    double* g = reinterpret_cast<double*>(w + off);
    off = align_up(off + sizeof(double) * 3 * (size_t)batch->total_atoms);
    const int mixed = precision == LJ_MIXED;
    struct Events {  // destroyed on every return path
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    LJ_HIP_TRY(hipEventCreate(&evs.e[0]));
    LJ_HIP_TRY(hipEventCreate(&evs.e[1]));
    hipEvent_t e0 = evs.e[0], e1 = evs.e[1];
    // median of five timed launches after a warm-up (a minimum would follow
    // the luckiest launch of a shape whose launches vary)
    auto time_it = [&](auto&& launch, float& ms) -> lj_status {
        lj_status r = launch();  // warm-up
        if (r != LJ_OK) return r;
        constexpr int kReps = 5;
        float t[kReps];
        for (int rep = 0; rep < kReps; ++rep) {
            LJ_HIP_TRY(hipEventRecord(e0, st));
            if ((r = launch()) != LJ_OK) return r;
            LJ_HIP_TRY(hipEventRecord(e1, st));
            LJ_HIP_TRY(hipEventSynchronize(e1));
            LJ_HIP_TRY(hipEventElapsedTime(&t[rep], e0, e1));
        }
        std::sort(t, t + kReps);
        ms = t[kReps / 2];
        return LJ_OK;
    };
    // pair kernel: every shape holding max_n atoms without more than doubling the padding
    const int need_slots = batch->max_n < 1 ? 1 : batch->max_n;
    const int cap = 2 * (pow2_at_least(need_slots) < 64 ? 64 : pow2_at_least(need_slots));
    lj::EvalShape best_shape = lj::eval_shape(batch->max_n);
    float best_ms = 1e30f;
    const int Ws[] = {1, 2, 4, 8, 16}, As[] = {1, 2, 4};
    for (int wi : Ws)
        for (int ai : As) {
            const int slots = 64 * wi * ai;
            if (slots < need_slots || slots > cap) continue;
            lj::EvalShape sh{wi, ai};
            float ms = 0.f;
            s = time_it([&]() -> lj_status {
                LJ_HIP_TRY(lj::launch_energy_grad(mixed, batch->pair, sh, batch->num,
                                                  batch->offset, batch->total_atoms, xyz, e, g,
                                                  batch->pair_rho, units_of(batch), st));
                return LJ_OK;
            }, ms);
            if (s != LJ_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_shape = sh;
            }
        }
    if (s == LJ_OK) {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        g_eval_sched[{precision, pow2_at_least(need_slots)}] = best_shape;
    }
    if (best_eval_ms) *best_eval_ms = best_ms;
    // Minimiser shapes (batches of at most LJ_MAX_ATOMS_MIN atoms): the
    // large-cluster class on a 3-iteration minimisation of a copy per shape;
    // then classes 2, 1, 0 in turn, each shape on a whole minimisation of a
    // copy (at most 1000 iterations per phase) with the other classes at their
    // current choice.  A shape replaces the current one when it is at least
    // 2 % faster; the choices go into the schedule table.
    float best_min = -1.f;
    if (s == LJ_OK && batch->max_n <= LJ_MAX_ATOMS_MIN) {
        double* xc = reinterpret_cast<double*>(w + off);
        off = align_up(off + sizeof(double) * 3 * (size_t)batch->total_atoms);
        double* outs = reinterpret_cast<double*>(w + off);
        off = align_up(off + 5 * sizeof(double) * (size_t)batch->num);
        int32_t* it = reinterpret_cast<int32_t*>(outs + 2 * (size_t)batch->num);
        int32_t* ev = it + batch->num;
        int32_t* stt = ev + batch->num;
        MinLayout base;
        if ((s = min_layout(batch->num, batch->max_n, mixed, batch->pair, base)) != LJ_OK)
            return s;
        int chosen[lj::kNumClasses] = {-1, -1, -1, -1};
        for (int c = 0; c <= base.top_class; ++c) chosen[c] = base.shape[c];
        lj_lbfgs_params lp;
        lj_lbfgs_defaults(&lp);
        auto time_shapes = [&](const int* force, const lj_lbfgs_params& prm, float& ms) -> lj_status {
            MinLayout L;
            lj_status r = min_layout(batch->num, batch->max_n, mixed, batch->pair, L, force);
            if (r != LJ_OK) return r;
            return time_it([&]() -> lj_status {
                LJ_HIP_TRY(hipMemcpyAsync(xc, xyz, sizeof(double) * 3 * (size_t)batch->total_atoms,
                                          hipMemcpyDeviceToDevice, st));
                return enqueue_minimize(batch, nullptr, xc, outs, outs + batch->num, it, ev, stt,
                                        nullptr, to_dev(&prm), mixed, L, w + off, st);
            }, ms);
        };
        if (base.top_class >= 3) {
            lj_lbfgs_params lp3 = lp;
            lp3.max_iter = 3;
            lp3.polish = 0;
            float best3 = 1e30f;
            for (int k = 0; k < lj::class_shapes(3) && s == LJ_OK; ++k) {
                int force[lj::kNumClasses];
                for (int c = 0; c < lj::kNumClasses; ++c) force[c] = chosen[c];
                force[3] = k;
                float ms = 0.f;
                s = time_shapes(force, lp3, ms);
                if (s == LJ_OK && ms < best3) {
                    best3 = ms;
                    chosen[3] = k;
                }
            }
            if (s == LJ_OK) {
                std::lock_guard<std::mutex> lk(g_sched_mu);
                g_large_sched[mixed] = chosen[3];
            }
        }
        lp.max_iter = 1000;
        float cur = 0.f;
        if (s == LJ_OK) s = time_shapes(chosen, lp, cur);
        // the class sizes of this batch, from the plan of the last timed call
        int32_t counts[2 * lj::kNumClasses] = {0};
        if (s == LJ_OK) {
            MinLayout L;
            if ((s = min_layout(batch->num, batch->max_n, mixed, batch->pair, L, chosen)) != LJ_OK)
                return s;
            LJ_HIP_TRY(hipMemcpyAsync(counts, w + off + L.cls, sizeof(counts),
                                      hipMemcpyDeviceToHost, st));
            LJ_HIP_TRY(hipStreamSynchronize(st));
        }
        for (int c = base.top_class < 2 ? base.top_class : 2; c >= 0 && s == LJ_OK; --c) {
            if (counts[lj::kNumClasses + c] == 0) continue;  // no cluster of this class
            const int cap = class_cap(c, batch->max_n);
            for (int k = 0; k < lj::class_shapes(c) && s == LJ_OK; ++k) {
                if (k == chosen[c] || lj::shape_max_n(c, k) < cap) continue;
                int force[lj::kNumClasses];
                for (int q = 0; q < lj::kNumClasses; ++q) force[q] = chosen[q];
                force[c] = k;
                float ms = 0.f;
                s = time_shapes(force, lp, ms);
                if (s == LJ_OK && ms < 0.98f * cur) {
                    cur = ms;
                    chosen[c] = k;
                }
            }
            if (s == LJ_OK) {
                std::lock_guard<std::mutex> lk(g_sched_mu);
                g_class_sched[class_key(precision, c, batch->max_n)] = chosen[c];
            }
        }
        if (s == LJ_OK) best_min = cur;
    }
    if (best_min_ms) *best_min_ms = best_min;
    return s;
}

}  // extern "C"
