// api.hip -- host side of the C ABI (include/mcpr.h): context, argument
// validation, work tables, the launch sequence of each call, and the
// MC-moments Parareal driver.
//
// Every sum over particles is formed on the device in the canonical order of
// common.hpp; the host only combines per-slice macro quantities (the coarse
// propagator and the Parareal iterator work on a few doubles per slice).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "mcpr.h"

static_assert(sizeof(mcpr_region_stats) == sizeof(mcpr::RegionStats), "record layout");
static_assert(sizeof(mcpr_region_map) == sizeof(mcpr::RegionMap), "map layout");
static_assert(sizeof(mcpr_region_stats) == 48, "record size");

using mcpr::RegionMap;
using mcpr::RegionPartial;
using mcpr::RegionStats;
using mcpr::WorkItem;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
};

} // namespace

// Launches in the step-variant autotuner's trial (at most 4 candidates x 4).
constexpr int kTuneSteps = 16;
// Instantiated fine sweeps kept per context.
constexpr size_t kGraphCache = 8;
// The adjoint's backward steps use one-quad superchunks below this many particles.
constexpr int64_t kAdjointSmall = 262144;

struct mcpr_ctx {
    int device = 0;
    std::string err;
    // the work table, block table and region maps of the last upload, one
    // allocation (tables) so that an upload is one copy; items, blocks and
    // maps point into it
    DevBuf tables;
    WorkItem *items = nullptr;
    int2 *blocks = nullptr;
    RegionMap *maps = nullptr;
    DevBuf part[2], shift[2], rpart, rshift[2], recs;
    DevBuf adj_ckpt, adj_traj, adj_lam[2], adj_part[2], adj_acc, adj_trace, adj_grad, adj_sums; // adjoint scratch
    DevBuf adj_tables; // the adjoint's work tables (every slice's), block tables and upstream derivatives
    // empirical-CDF drift: states and labels in sorted order, the library
    // sort's item pass and scratch, the bucket engine's tables and staging
    DevBuf cdf_keys[2], cdf_lab[2], cdf_seg[2], cdf_kl[2], cdf_beg, cdf_tmp;
    DevBuf cdf_bcount, cdf_bmeta, cdf_stage, cdf_flag, cdf_defer;
    mcpr::CdfBuffers cdfb{};
    uint32_t *cdf_flag_host = nullptr; // pinned copy of the overflow flag
    int cdf_engine = 1;                // 1: bucket engine after a sweep's first steps; 0: library sort every step
    int64_t cdf_sweeps[3] = {0, 0, 0}; // sweeps by the bucket engine, by the library sort, redone
    HostBuf staging;
    hipEvent_t staged = nullptr; // the last upload from staging has completed
    DevBuf trace; // trace of the last fine sweep (copied to the caller's array)
    // profiling of the Euler-Maruyama step launches (off unless enabled): one
    // event pair around each call's run of step launches, read lazily
    bool profile = false;
    std::vector<hipEvent_t> prof0, prof1;
    std::vector<int64_t> prof_ps;
    size_t prof_used = 0;
    int64_t prof_launches = 0;
    // the same for the adjoint's backward step launches (one pair per slice)
    std::vector<hipEvent_t> aprof0, aprof1;
    size_t aprof_used = 0;
    int64_t aprof_launches = 0, aprof_ps = 0;
    // hipGraph of the fine sweep (sum init, m steps, finish, records), replayed
    // on a library stream ordered against the caller's stream by events
    bool graphs = true;
    hipStream_t gstream = nullptr;
    hipEvent_t gin = nullptr, gout = nullptr;
    // instantiated sweeps by launch shape, least recently used evicted first
    // (a Parareal step alternates lifting and sweep shapes, the adjoint its
    // traced forward sweeps and the recomputations)
    struct GraphEntry {
        std::vector<char> key;
        hipGraphExec_t exec = nullptr;
        int64_t used = 0;
    };
    std::vector<GraphEntry> graphs_cached;
    int64_t graph_builds = 0, graph_launches = 0;
    // the adjoint's second stream (recomputation of slice n-1 while the
    // backward steps of slice n run) and its events
    hipStream_t astream = nullptr;
    hipEvent_t a_fwd = nullptr, a_rec[2] = {}, a_bwd[2] = {};
    // step-kernel variant per launch shape: -1 autotune, 0..3 forced
    int tuning = -1;
    std::map<std::vector<char>, int> tuned;
    hipEvent_t tune_ev[2][kTuneSteps] = {};
    int tune_steps = 0;
    int tune_cand[4] = {0, 1, 2, 3}; // variants of the trial, the first is the reference
    int tune_nc = 4;
    DevBuf mv; // per-item (mean, variance) of the separate-combine variant
    DevBuf znorm;                 // resident sweeps: the normals of every step of the sweep
    int resident = 1;             // 1: resident sweeps where every ensemble fits one block
    int64_t resident_sweeps = 0;  // fine sweeps run resident so far
    // scratch sizing: buffers grow only inside mcpr_reserve (and the Parareal
    // driver's create); a hot-path call that needs more fails with
    // MCPR_E_NOT_RESERVED before launching anything
    bool growing = false;
    int64_t allocs = 0, alloc_bytes = 0; // device and pinned allocations made so far
};

namespace {

// Error text of the calls that take no context (mcpr_fine_propagate_static),
// per host thread.
thread_local char g_static_err[512] = "no error";

mcpr_status fail(mcpr_ctx *ctx, mcpr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        std::memcpy(g_static_err, buf, sizeof buf);
    return st;
}

#define HIP_TRY(expr)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) return fail(ctx, MCPR_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

// Scratch buffer b of at least `bytes`: grown (with a device synchronisation)
// only while the context is sizing, else MCPR_E_NOT_RESERVED.
mcpr_status ensure(mcpr_ctx *ctx, DevBuf &b, size_t bytes) {
    if (bytes <= b.cap) return MCPR_OK;
    if (!ctx->growing)
        return fail(ctx, MCPR_E_NOT_RESERVED,
                    "%zu bytes of scratch needed where %zu are reserved: call mcpr_reserve with this call's "
                    "ensembles first",
                    bytes, b.cap);
    size_t want = std::max(bytes, b.cap * 3 / 2);
    want = (want + 255) & ~(size_t)255;
    if (b.p) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        return fail(ctx, MCPR_E_OOM, "device allocation of %zu bytes failed", want);
    }
    b.cap = want;
    ctx->allocs++;
    ctx->alloc_bytes += (int64_t)want;
    return MCPR_OK;
}

// Pinned host buffer of at least `bytes`, under the same rule as ensure().
mcpr_status ensure_host(mcpr_ctx *ctx, HostBuf &b, size_t bytes) {
    if (bytes <= b.cap) return MCPR_OK;
    if (!ctx->growing)
        return fail(ctx, MCPR_E_NOT_RESERVED,
                    "%zu bytes of pinned staging needed where %zu are reserved: call mcpr_reserve first", bytes,
                    b.cap);
    if (b.p) HIP_TRY(hipHostFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    const size_t want = std::max(bytes, (size_t)1 << 16);
    if (hipHostMalloc(&b.p, want, hipHostMallocDefault) != hipSuccess) {
        b.p = nullptr;
        return fail(ctx, MCPR_E_OOM, "pinned allocation of %zu bytes failed", want);
    }
    b.cap = want;
    ctx->allocs++;
    ctx->alloc_bytes += (int64_t)want;
    return MCPR_OK;
}

// Sizing mode for the duration of a scope (mcpr_reserve, the driver's create).
struct Growing {
    mcpr_ctx *ctx;
    explicit Growing(mcpr_ctx *c) : ctx(c) { ctx->growing = true; }
    ~Growing() { ctx->growing = false; }
};

// Host staging of the per-call tables (pinned, reused once its last upload is done).
mcpr_status stage(mcpr_ctx *ctx, size_t bytes, char **out) {
    mcpr_status st = ensure_host(ctx, ctx->staging, bytes);
    if (st != MCPR_OK) return st;
    HIP_TRY(hipEventSynchronize(ctx->staged));
    *out = (char *)ctx->staging.p;
    return MCPR_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ----------------------------------------------------------------------------
// validation
// ----------------------------------------------------------------------------
bool is_trig(const mcpr_problem &p) { return p.coef.ksin != 0.0 || p.coef.kc != 0.0; }
bool is_cdf(const mcpr_problem &p) { return p.coef.acdf != 0.0; }

mcpr_status check_problem(mcpr_ctx *ctx, const mcpr_problem &p, int idx) {
    if (p.precision != MCPR_FP64 && p.precision != MCPR_FP32)
        return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: precision %d", idx, p.precision);
    if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: dt must be > 0", idx);
    if (p.steps_per_slice < 1) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: steps_per_slice < 1", idx);
    if (p.n_slices < 1) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: n_slices < 1", idx);
    if ((int64_t)p.n_slices * p.steps_per_slice > 0x7fffffffLL)
        return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: too many steps", idx);
    if (p.n_regions < 1 || p.n_regions > MCPR_MAX_REGIONS)
        return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: n_regions must be in 1..%d", idx, MCPR_MAX_REGIONS);
    for (int i = 0; i + 1 < p.n_regions; ++i) {
        if (!std::isfinite(p.split[i])) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: split %d", idx, i);
        if (i > 0 && !(p.split[i] > p.split[i - 1]))
            return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: splits must increase", idx);
    }
    if (p.coarse_substeps < 1) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: coarse_substeps < 1", idx);
    if (p.coarse_model < MCPR_COARSE_TAYLOR || p.coarse_model > MCPR_COARSE_GAUSS3)
        return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: coarse_model %d", idx, p.coarse_model);
    if (p.p0_kind < 0 || p.p0_kind > 2) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: p0_kind", idx);
    const double *c = &p.coef.a0;
    for (int i = 0; i < 14; ++i)
        if (!std::isfinite(c[i])) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: coefficient %d not finite", idx, i);
    // invalid values first, then combinations the kernels do not support
    if (p.wrap != 0 && p.wrap != 1) return fail(ctx, MCPR_E_INVALID_ARG, "problem %d: wrap must be 0 or 1", idx);
    if (is_cdf(p) && (p.coef.am != 0.0 || p.coef.av != 0.0 || p.coef.axs != 0.0 || p.coef.bm != 0.0 ||
                      p.coef.bv != 0.0 || is_trig(p) || p.wrap != 0 || p.n_regions != 1 ||
                      p.coarse_model != MCPR_COARSE_TAYLOR))
        return fail(ctx, MCPR_E_UNSUPPORTED,
                    "problem %d: the empirical-CDF drift needs one region, the Taylor model and no other "
                    "mean-field coefficient",
                    idx);
    if (is_trig(p) && (p.coef.am != 0.0 || p.coef.av != 0.0 || p.coef.axs != 0.0 || p.coef.bm != 0.0 ||
                       p.coef.bv != 0.0))
        return fail(ctx, MCPR_E_UNSUPPORTED,
                    "problem %d: trigonometric drift terms exclude the (m, v) mean-field coefficients", idx);
    return MCPR_OK;
}

bool same_layout(const mcpr_problem &a, const mcpr_problem &b) {
    if (a.precision != b.precision || a.steps_per_slice != b.steps_per_slice || a.n_regions != b.n_regions ||
        is_trig(a) != is_trig(b) || is_cdf(a) != is_cdf(b))
        return false;
    for (int i = 0; i + 1 < a.n_regions; ++i)
        if (a.split[i] != b.split[i]) return false;
    return true;
}

// Arguments of a call on ensembles (ctx may be NULL: errors then go to the
// calling thread's context-free error text).
mcpr_status check_args(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                       int32_t n_ens) {
    if (!problems || n_problems < 1) return fail(ctx, MCPR_E_INVALID_ARG, "no problems");
    if (!ens || n_ens < 1) return fail(ctx, MCPR_E_INVALID_ARG, "no ensembles");
    for (int i = 0; i < n_problems; ++i) {
        mcpr_status st = check_problem(ctx, problems[i], i);
        if (st != MCPR_OK) return st;
    }
    const mcpr_problem *first = &problems[ens[0].problem >= 0 && ens[0].problem < n_problems ? ens[0].problem : 0];
    int64_t total_sc = 0;
    for (int e = 0; e < n_ens; ++e) {
        const mcpr_ensemble &E = ens[e];
        if (E.problem < 0 || E.problem >= n_problems)
            return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: problem index %d", e, E.problem);
        if (!same_layout(problems[E.problem], *first))
            return fail(ctx, MCPR_E_INVALID_ARG,
                        "ensemble %d: precision, steps_per_slice, regions and the kind of mean field must agree "
                        "within a call",
                        e);
        if (!E.x) return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: null particle pointer", e);
        if (((uintptr_t)E.x & 15) != 0) return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: pointer not 16-byte aligned", e);
        if (E.n_particles < 1 || E.n_particles > ((int64_t)1 << 34))
            return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: n_particles %lld", e, (long long)E.n_particles);
        if (E.instance < 0) return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: instance < 0", e);
        if (E.slice < 0 || (int64_t)(E.slice + 1) * problems[E.problem].steps_per_slice > 0x7fffffffLL)
            return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: slice %d", e, E.slice);
        total_sc += mcpr::superchunks(E.n_particles, mcpr::canonical_quads_per_thread(E.n_particles));
    }
    if (total_sc > 0x7fffffffLL) return fail(ctx, MCPR_E_INVALID_ARG, "too many particles in one call");
    return MCPR_OK;
}

mcpr_status check_call(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                       int32_t n_ens) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    return check_args(ctx, problems, n_problems, ens, n_ens);
}

// ----------------------------------------------------------------------------
// work tables
// ----------------------------------------------------------------------------
struct Tables {
    std::vector<WorkItem> items;
    std::vector<int2> blocks; // one entry per superchunk: (item, superchunk)
    int total_sc = 0;
    int64_t total_dense = 0;  // dense sort positions, the sum of P (empirical-CDF drift)
    int nbuckets = 0;         // bucket engine: buckets of the launch
    int64_t total_z = 0;      // resident sweep: normals of all steps (items' zoff)
    int zm = 0;               // the steps per slice they are laid out for (-1: the items differ)
};

void build_tables(const mcpr_problem *problems, const mcpr_ensemble *ens, int32_t n_ens, Tables &t) {
    t.items.resize(n_ens);
    t.blocks.clear();
    t.total_dense = 0;
    t.nbuckets = 0;
    t.total_z = 0;
    t.zm = n_ens > 0 ? problems[ens[0].problem].steps_per_slice : 0;
    int off = 0;
    for (int e = 0; e < n_ens; ++e) {
        const mcpr_ensemble &E = ens[e];
        const mcpr_problem &p = problems[E.problem];
        WorkItem &w = t.items[e];
        std::memset(&w, 0, sizeof w);
        w.x = E.x;
        w.P = E.n_particles;
        w.inst = E.instance;
        w.step0 = E.slice * p.steps_per_slice;
        // (the empirical-CDF step gathers its states in sorted order and
        // reserves bucket slots per round of 1024 states: two rounds per
        // block amortise a block's start, more would leave fewer blocks in
        // flight; still a function of the ensemble alone)
        w.R = is_cdf(p) ? 2 : mcpr::canonical_quads_per_thread(E.n_particles);
        w.nsc = (int32_t)mcpr::superchunks(E.n_particles, w.R);
        w.part_off = off;
        w.p0_kind = p.p0_kind;
        w.key0 = (uint32_t)(p.seed & 0xffffffffu);
        w.key1 = (uint32_t)(p.seed >> 32);
        const double *c = &p.coef.a0;
        for (int i = 0; i < 14; ++i) w.c[i] = c[i];
        w.wrap = p.wrap;
        w.trig = is_trig(p) ? 1 : 0;
        w.cdf = is_cdf(p) ? 1 : 0;
        w.doff = t.total_dense;
        t.total_dense += E.n_particles;
        if (w.cdf) {
            w.nbk = (int32_t)std::max<int64_t>(1, (E.n_particles + mcpr::kCdfBucket - 1) / mcpr::kCdfBucket);
            w.bbase = t.nbuckets;
            t.nbuckets += w.nbk;
        }
        if (p.steps_per_slice != t.zm) t.zm = -1;
        w.zoff = t.total_z;
        t.total_z += (int64_t)p.steps_per_slice * 4 * mcpr::kThreads * w.R * w.nsc; // every quad of its superchunks
        w.dt = p.dt;
        w.sdt = std::sqrt(p.dt);
        w.p0[0] = p.p0_w;
        w.p0[1] = p.p0_mu1;
        w.p0[2] = p.p0_sd1;
        w.p0[3] = p.p0_mu2;
        w.p0[4] = p.p0_sd2;
        for (int s = 0; s < w.nsc; ++s) t.blocks.push_back(make_int2(e, s));
        off += w.nsc;
    }
    t.total_sc = off;
}

// Upload the work and block tables (and optionally maps) through the pinned
// staging buffer, in one copy into the tables buffer.
// Bytes of an upload of the tables t and map_bytes of maps.
size_t tables_bytes(const Tables &t, size_t map_bytes) {
    return align256(t.items.size() * sizeof(WorkItem)) + align256(t.blocks.size() * sizeof(int2)) +
           align256(map_bytes);
}
mcpr_status size_upload(mcpr_ctx *ctx, const Tables &t, size_t map_bytes) {
    mcpr_status st;
    if ((st = ensure(ctx, ctx->tables, tables_bytes(t, map_bytes))) != MCPR_OK) return st;
    return ensure_host(ctx, ctx->staging, tables_bytes(t, map_bytes));
}

mcpr_status upload(mcpr_ctx *ctx, const Tables &t, const void *maps, size_t map_bytes, hipStream_t s) {
    const size_t ib = t.items.size() * sizeof(WorkItem), bb = t.blocks.size() * sizeof(int2);
    const size_t total = tables_bytes(t, map_bytes);
    mcpr_status st;
    if ((st = size_upload(ctx, t, map_bytes)) != MCPR_OK) return st;
    char *h;
    if ((st = stage(ctx, total, &h)) != MCPR_OK) return st;
    std::memcpy(h, t.items.data(), ib);
    std::memcpy(h + align256(ib), t.blocks.data(), bb);
    if (map_bytes) std::memcpy(h + align256(ib) + align256(bb), maps, map_bytes);
    HIP_TRY(hipMemcpyAsync(ctx->tables.p, h, total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->staged, s));
    char *d = (char *)ctx->tables.p;
    ctx->items = (WorkItem *)d;
    ctx->blocks = (int2 *)(d + align256(ib));
    ctx->maps = map_bytes ? (RegionMap *)(d + align256(ib) + align256(bb)) : nullptr;
    return MCPR_OK;
}

mcpr::Splits splits_of(const mcpr_problem &p) {
    mcpr::Splits sp;
    for (int i = 0; i < mcpr::kMaxRegions - 1; ++i) sp.s[i] = (i + 1 < p.n_regions) ? p.split[i] : 0.0;
    return sp;
}

// Restriction records of the ensembles in the tables.  shift: per-item shift of
// the first pass (NULL: x[0]).  Two passes when the ensemble is split into
// regions, so that each region's sums are taken about that region's mean.
mcpr_status ensure_records(mcpr_ctx *ctx, const Tables &t, int nreg) {
    const int nr = nreg + 1, n = (int)t.items.size();
    mcpr_status st;
    if ((st = ensure(ctx, ctx->rpart, (size_t)t.total_sc * nr * sizeof(RegionPartial))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->rshift[0], (size_t)n * nr * sizeof(double))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->rshift[1], (size_t)n * nr * sizeof(double))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->recs, (size_t)n * nr * sizeof(RegionStats))) != MCPR_OK) return st;
    return MCPR_OK;
}

// Device scratch of one fine sweep or restriction: the work and block
// tables, the step partials and shifts (ping-pong), the per-item mean field,
// the region partials and shifts, and where the records and the trace go.
struct Bufs {
    const WorkItem *items;
    const int2 *blocks;
    double2 *part[2];
    double *shift[2];
    double2 *mv;
    RegionPartial *rpart;
    double *rshift[2];
    RegionStats *recs;
    double2 *trace;
};

Bufs ctx_bufs(mcpr_ctx *ctx) {
    Bufs b;
    b.items = ctx->items;
    b.blocks = ctx->blocks;
    for (int k = 0; k < 2; ++k) {
        b.part[k] = (double2 *)ctx->part[k].p;
        b.shift[k] = (double *)ctx->shift[k].p;
        b.rshift[k] = (double *)ctx->rshift[k].p;
    }
    b.mv = (double2 *)ctx->mv.p;
    b.rpart = (RegionPartial *)ctx->rpart.p;
    b.recs = (RegionStats *)ctx->recs.p;
    b.trace = (double2 *)ctx->trace.p;
    return b;
}

mcpr_status enqueue_records(mcpr_ctx *ctx, const Bufs &bf, const Tables &t, int prec, int nreg,
                            const mcpr::Splits &sp, const double *shift, bool two_pass, int mode,
                            const RegionMap *maps, RegionStats *out, hipStream_t s) {
    const int nr = nreg + 1, n = (int)t.items.size();
    const WorkItem *items = bf.items;
    const int2 *blocks = bf.blocks;
    const int nb = (int)t.blocks.size();
    double *rs0 = bf.rshift[0], *rs1 = bf.rshift[1];
    RegionPartial *rp = bf.rpart;
    HIP_TRY(mcpr::launch_fill_shift(prec, nr, items, n, shift, rs0, s));
    if (two_pass) {
        // first pass: region means only; second pass about each region's mean
        HIP_TRY(mcpr::launch_region_partials(prec, nr, mode, false, items, blocks, nb, rs0, sp, maps, rp, s));
        HIP_TRY(mcpr::launch_region_combine(nr, false, items, n, rp, rs0, nullptr, rs1, s));
        HIP_TRY(mcpr::launch_region_partials(prec, nr, mode, true, items, blocks, nb, rs1, sp, maps, rp, s));
        HIP_TRY(mcpr::launch_region_combine(nr, true, items, n, rp, rs1, out, nullptr, s));
    } else {
        HIP_TRY(mcpr::launch_region_partials(prec, nr, mode, true, items, blocks, nb, rs0, sp, maps, rp, s));
        HIP_TRY(mcpr::launch_region_combine(nr, true, items, n, rp, rs0, out, nullptr, s));
    }
    return MCPR_OK;
}

mcpr_status records(mcpr_ctx *ctx, const Tables &t, int prec, int nreg, const mcpr::Splits &sp, const double *shift,
                    bool two_pass, int mode, const RegionMap *maps, RegionStats *out, hipStream_t s) {
    mcpr_status st = ensure_records(ctx, t, nreg);
    if (st != MCPR_OK) return st;
    return enqueue_records(ctx, ctx_bufs(ctx), t, prec, nreg, sp, shift, two_pass, mode, maps, out, s);
}

// Resident sweeps: the normals' scratch limit, and the step "variant" that
// marks a resident sweep (in graph keys).
constexpr size_t kResidentZBytes = (size_t)256 << 20;
constexpr int kResidentVariant = 16;

// The step sequence of the fine propagator on already uploaded tables:
// step-0 sums, m Euler-Maruyama launches, the final moments (if traced) and
// the restriction records (if wanted), into ctx-owned buffers.
// variant == kResidentVariant: the resident sweep instead of the step-0 sums
// and the m launches.
// variant < 0: the first tune_steps steps run the candidate variants in turn,
// each launch bracketed by events (the autotuner's trial; every variant gives
// the same bits).
// j0, j1: only steps [j0, j1) (the empirical-CDF sweep is enqueued in parts);
// the sums of step 0 come with the first part, the moments and records with
// the last.
mcpr_status enqueue_fine(mcpr_ctx *ctx, const Bufs &bf, const Tables &t, int prec, int deg, int variant, int m,
                         int nreg, const mcpr::Splits &sp, bool want_stats, bool want_trace, hipStream_t s,
                         bool profile, int cdf_lib_steps = 0, int j0 = 0, int j1 = -1) {
    if (j1 < 0) j1 = m;
    const int n = (int)t.items.size();
    const WorkItem *items = bf.items;
    const int2 *blocks = bf.blocks;
    const int nb = (int)t.blocks.size();
    double2 *const *part = bf.part;
    double *const *shift = bf.shift;
    double2 *trace = want_trace ? bf.trace : nullptr;
    const bool trig = t.items[0].trig != 0; // the same for every item of a call
    const bool cdf = t.items[0].cdf != 0;
    const uint32_t ndense = (uint32_t)t.total_dense;
    if (variant == kResidentVariant) {
        // the whole sweep in two launches (normals, then one block per ensemble)
        if (profile) HIP_TRY(hipEventRecord(ctx->prof0[ctx->prof_used], s));
        HIP_TRY(mcpr::launch_em_sweep_resident(prec, deg, items, n, blocks, nb, m, ctx->znorm.p, part[m & 1],
                                               shift[m & 1], trace, s));
        if (profile) HIP_TRY(hipEventRecord(ctx->prof1[ctx->prof_used], s));
        if (trace) HIP_TRY(mcpr::launch_finish(items, n, part[m & 1], shift[m & 1], trace, m, s));
        if (want_stats)
            return enqueue_records(ctx, bf, t, prec, nreg, sp, shift[m & 1], nreg > 1, 0, nullptr, bf.recs, s);
        return MCPR_OK;
    }
    if (j0 == 0) {
        if (cdf) HIP_TRY(mcpr::launch_cdf_start(prec, items, n, blocks, nb, ctx->cdfb, s));
        if (trig)
            HIP_TRY(mcpr::launch_sum_init_trig(prec, items, blocks, nb, part[0], shift[0], s));
        else
            HIP_TRY(mcpr::launch_sum_init(prec, items, blocks, nb, part[0], shift[0], s));
        if (profile) HIP_TRY(hipEventRecord(ctx->prof0[ctx->prof_used], s));
    }
    double2 *mv = bf.mv;
    for (int j = j0; j < j1; ++j) {
        const int a = j & 1, b = a ^ 1;
        const bool trial = variant < 0 && j < ctx->tune_steps;
        const int v = trial ? ctx->tune_cand[j / (ctx->tune_steps / ctx->tune_nc)]
                            : (variant < 0 ? ctx->tune_cand[0] : variant);
        if (trial) HIP_TRY(hipEventRecord(ctx->tune_ev[0][j], s));
        if (cdf) {
            // the library sort on the first cdf_lib_steps steps, else the
            // buckets the previous step filled (step j's sorted input is the
            // splitter set of its output)
            const bool from_buckets = j >= cdf_lib_steps;
            if (from_buckets)
                HIP_TRY(mcpr::launch_cdf_buckets(prec, items, n, ctx->cdfb, s));
            else
                HIP_TRY(mcpr::launch_cdf_sort(prec, n, ndense, ctx->cdfb, s));
            const int mode = j == m - 1 ? 2 : (j + 1 >= cdf_lib_steps ? 1 : 0);
            HIP_TRY(mcpr::launch_em_step_sorted(prec, deg, items, n, blocks, nb, j, mode, !from_buckets && n > 1,
                                                part[a], shift[a], mv, ctx->cdfb, part[b], shift[b], trace, m, s));
        } else if (trig)
            HIP_TRY(mcpr::launch_em_step_trig(prec, deg, items, blocks, nb, j, part[a], part[b], shift[b], trace, m, s));
        else
            HIP_TRY(mcpr::launch_em_step(prec, deg, v, items, n, blocks, nb, j, part[a], shift[a], mv, part[b],
                                         shift[b], trace, m, s));
        if (trial) HIP_TRY(hipEventRecord(ctx->tune_ev[1][j], s));
    }
    if (j1 < m) return MCPR_OK;
    if (profile) HIP_TRY(hipEventRecord(ctx->prof1[ctx->prof_used], s));
    if (trace) {
        if (trig)
            HIP_TRY(mcpr::launch_finish_trig(items, n, part[m & 1], trace, m, s));
        else
            HIP_TRY(mcpr::launch_finish(items, n, part[m & 1], shift[m & 1], trace, m, s));
    }
    if (want_stats) {
        // shift of the record sums: the mean the last step used (with the
        // trigonometric mean field there is none: two passes then)
        return enqueue_records(ctx, bf, t, prec, nreg, sp, shift[m & 1], nreg > 1 || trig, 0, nullptr, bf.recs,
                               s);
    }
    return MCPR_OK;
}

// Everything a captured fine sweep depends on besides the device tables.
std::vector<char> graph_key(mcpr_ctx *ctx, const Tables &t, int prec, int deg, int variant, int m, int nreg,
                            const mcpr::Splits &sp, bool want_stats, bool want_trace) {
    const void *ptrs[] = {ctx->items, ctx->blocks, ctx->part[0].p, ctx->part[1].p, ctx->shift[0].p,
                          ctx->shift[1].p, ctx->rpart.p, ctx->rshift[0].p, ctx->rshift[1].p, ctx->recs.p,
                          ctx->trace.p,  ctx->mv.p,       ctx->znorm.p};
    const int64_t ints[] = {(int64_t)t.items.size(), (int64_t)t.blocks.size(), t.total_sc, prec, deg, m, nreg,
                            want_stats, want_trace, variant, t.items[0].trig};
    std::vector<char> k(sizeof ptrs + sizeof ints + sizeof sp);
    std::memcpy(k.data(), ptrs, sizeof ptrs);
    std::memcpy(k.data() + sizeof ptrs, ints, sizeof ints);
    std::memcpy(k.data() + sizeof ptrs + sizeof ints, &sp, sizeof sp);
    return k;
}

// Buffers of the empirical-CDF drift for the concatenated ensembles of t.
mcpr_status ensure_cdf(mcpr_ctx *ctx, const Tables &t, int prec) {
    const size_t n = (size_t)t.total_dense, es = prec == 0 ? sizeof(double) : sizeof(float);
    const int nseg = (int)t.items.size();
    if (t.total_dense >= ((int64_t)1 << 32) - 1)
        return fail(ctx, MCPR_E_UNSUPPORTED, "empirical-CDF drift: %lld particles in one launch exceed 2^32 - 1",
                    (long long)t.total_dense);
    const size_t kls = prec == 0 ? sizeof(mcpr::KeyLabel<double>) : sizeof(mcpr::KeyLabel<float>);
    mcpr_status st;
    for (int b = 0; b < 2; ++b) {
        if ((st = ensure(ctx, ctx->cdf_keys[b], n * es)) != MCPR_OK) return st;
        if ((st = ensure(ctx, ctx->cdf_lab[b], n * sizeof(uint32_t))) != MCPR_OK) return st;
        if (nseg > 1) {
            if ((st = ensure(ctx, ctx->cdf_seg[b], n * sizeof(uint32_t))) != MCPR_OK) return st;
            if ((st = ensure(ctx, ctx->cdf_kl[b], n * kls)) != MCPR_OK) return st;
        }
    }
    if ((st = ensure(ctx, ctx->cdf_beg, (size_t)nseg * sizeof(uint32_t))) != MCPR_OK) return st;
    const size_t nbk = (size_t)t.nbuckets;
    if ((st = ensure(ctx, ctx->cdf_bcount, nbk * sizeof(uint32_t))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->cdf_flag, sizeof(uint32_t))) != MCPR_OK) return st;
    if (ctx->cdf_engine) {
        if ((st = ensure(ctx, ctx->cdf_bmeta, nbk * sizeof(uint2))) != MCPR_OK) return st;
        if ((st = ensure(ctx, ctx->cdf_stage, mcpr::stage_bytes(prec, (int)nbk))) != MCPR_OK) return st;
        if ((st = ensure(ctx, ctx->cdf_defer, (nbk + 1) * sizeof(uint32_t))) != MCPR_OK) return st;
    }
    if (!ctx->cdf_flag_host) {
        if (!ctx->growing)
            return fail(ctx, MCPR_E_NOT_RESERVED, "empirical-CDF drift: call mcpr_reserve for this call first");
        void *h = nullptr;
        if (hipHostMalloc(&h, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
            return fail(ctx, MCPR_E_OOM, "pinned host allocation failed");
        ctx->cdf_flag_host = (uint32_t *)h;
        ctx->allocs++;
        ctx->alloc_bytes += (int64_t)sizeof(uint32_t);
    }
    size_t tb = 0;
    HIP_TRY(mcpr::cdf_scratch_bytes(prec, (uint32_t)n, (uint32_t)nseg, tb));
    if ((st = ensure(ctx, ctx->cdf_tmp, tb > 0 ? tb : 1)) != MCPR_OK) return st;
    mcpr::CdfBuffers &c = ctx->cdfb;
    for (int b = 0; b < 2; ++b) {
        c.keys[b] = ctx->cdf_keys[b].p;
        c.lab[b] = (uint32_t *)ctx->cdf_lab[b].p;
        c.seg[b] = (uint32_t *)ctx->cdf_seg[b].p;
        c.kl[b] = ctx->cdf_kl[b].p;
    }
    c.seg_begin = (uint32_t *)ctx->cdf_beg.p;
    c.tmp = ctx->cdf_tmp.p;
    c.tmp_bytes = ctx->cdf_tmp.cap;
    c.nbuckets = t.nbuckets;
    c.bcount = (uint32_t *)ctx->cdf_bcount.p;
    c.bmeta = (uint2 *)ctx->cdf_bmeta.p;
    c.stage = ctx->cdf_stage.p;
    c.defer = (uint32_t *)ctx->cdf_defer.p;
    c.flag = (uint32_t *)ctx->cdf_flag.p;
    return MCPR_OK;
}

// An event pair for the next profiled run of step launches (slot prof_used).
mcpr_status next_prof_slot(mcpr_ctx *ctx) {
    if (ctx->prof_used < ctx->prof0.size()) return MCPR_OK;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    ctx->prof0.push_back(e0);
    ctx->prof1.push_back(e1);
    ctx->prof_ps.push_back(0);
    return MCPR_OK;
}

// Whether the fine sweep of t runs resident: every ensemble in place, at most
// kResidentMaxP particles, no trigonometric or empirical-CDF term, and the
// sweep's normals within kResidentZBytes.
bool resident_ok(const mcpr_ctx *ctx, const Tables &t, int prec, int m) {
    if (!ctx->resident || t.items.empty() || t.zm != m || m < 1 || m > 65535) return false;
    if ((size_t)t.total_z * (prec == 0 ? sizeof(double) : sizeof(float)) > kResidentZBytes) return false;
    for (const WorkItem &w : t.items)
        if (w.trig || w.cdf || w.traj != 0 || w.src || w.R != 1 || w.P > mcpr::kResidentMaxP ||
            w.nsc > mcpr::kResidentMaxSc)
            return false;
    return true;
}

// Buffers of a fine sweep of the tables t (records and trace if wanted).
mcpr_status size_fine(mcpr_ctx *ctx, const Tables &t, int prec, int m, int nreg, bool stats, bool trace) {
    const int n = (int)t.items.size();
    mcpr_status st;
    for (int b = 0; b < 2; ++b) {
        if ((st = ensure(ctx, ctx->part[b], (size_t)t.total_sc * sizeof(double2))) != MCPR_OK) return st;
        if ((st = ensure(ctx, ctx->shift[b], (size_t)n * sizeof(double))) != MCPR_OK) return st;
    }
    if (stats && (st = ensure_records(ctx, t, nreg)) != MCPR_OK) return st;
    if (trace && (st = ensure(ctx, ctx->trace, (size_t)n * (m + 1) * sizeof(double2))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->mv, (size_t)n * sizeof(double2))) != MCPR_OK) return st;
    if (t.items[0].cdf && (st = ensure_cdf(ctx, t, prec)) != MCPR_OK) return st;
    // (the normals' scratch is sized only when reserving: a call it does not
    // fit runs the per-step launches, which give the same bits)
    if (ctx->growing && resident_ok(ctx, t, prec, m) &&
        (st = ensure(ctx, ctx->znorm, (size_t)t.total_z * (prec == 0 ? sizeof(double) : sizeof(float)))) != MCPR_OK)
        return st;
    return MCPR_OK;
}

// Replays the graph cached under key on the library's graph stream, ordered
// after the work on s and before s's later work; on a miss the sequence that
// enqueue puts on the stream it is given is captured and instantiated first
// (the least recently used graph is evicted when the cache is full).
template <typename Enqueue>
mcpr_status replay(mcpr_ctx *ctx, const std::vector<char> &key, hipStream_t s, Enqueue enqueue) {
    mcpr_ctx::GraphEntry *ge = nullptr;
    for (auto &e : ctx->graphs_cached)
        if (e.key == key) ge = &e;
    if (!ge) {
        if (ctx->graphs_cached.size() >= kGraphCache) {
            size_t lru = 0;
            for (size_t i = 1; i < ctx->graphs_cached.size(); ++i)
                if (ctx->graphs_cached[i].used < ctx->graphs_cached[lru].used) lru = i;
            HIP_TRY(hipStreamSynchronize(ctx->gstream)); // (the evicted graph may still run)
            HIP_TRY(hipGraphExecDestroy(ctx->graphs_cached[lru].exec));
            ctx->graphs_cached.erase(ctx->graphs_cached.begin() + lru);
        }
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
        mcpr_status st = enqueue(ctx->gstream);
        hipError_t ec = hipStreamEndCapture(ctx->gstream, &g);
        if (st != MCPR_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ec != hipSuccess) return fail(ctx, MCPR_E_DEVICE, "graph capture: %s", hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(ctx, MCPR_E_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
        ctx->graphs_cached.push_back(mcpr_ctx::GraphEntry{key, exec, 0});
        ge = &ctx->graphs_cached.back();
        ctx->graph_builds++;
    }
    ge->used = ++ctx->graph_launches;
    HIP_TRY(hipEventRecord(ctx->gin, s));
    HIP_TRY(hipStreamWaitEvent(ctx->gstream, ctx->gin, 0));
    HIP_TRY(hipGraphLaunch(ge->exec, ctx->gstream));
    HIP_TRY(hipEventRecord(ctx->gout, ctx->gstream));
    HIP_TRY(hipStreamWaitEvent(s, ctx->gout, 0));
    return MCPR_OK;
}

mcpr_status fine_sequence(mcpr_ctx *ctx, const Tables &t, int prec, int m, int nreg, const mcpr::Splits &sp,
                          bool want_stats, RegionStats *stats, double2 *trace, hipStream_t s) {
    const int n = (int)t.items.size();
    mcpr_status st;
    if ((st = size_fine(ctx, t, prec, m, nreg, want_stats, trace != nullptr)) != MCPR_OK) return st;
    const Bufs bf = ctx_bufs(ctx);
    int deg = 1, max_nsc = 0;
    int64_t ps = 0;
    for (const WorkItem &w : t.items) {
        if (w.c[2] != 0.0 || w.c[3] != 0.0) deg = 3;
        ps += w.P;
        max_nsc = std::max(max_nsc, w.nsc);
    }
    if (t.items[0].cdf) {
        // The empirical-CDF sweep: launched directly (no graph, no variants).
        // With the bucket engine the library sort takes the first two steps
        // (the input may be a point mass, which gives no splitters); the host
        // reads the overflow flag after the first bucket step and after the
        // sweep and, if a bucket overflowed (a law still spreading fast, as in
        // the first steps from a point mass), redoes the sweep with the library
        // sort on its first 8 steps, then 32, then all of them.  The particles
        // are untouched until the sweep's last step, and the steps of an
        // overflowed sweep that are already enqueued do nothing.
        size_t slot = 0;
        if (ctx->profile) {
            if ((st = next_prof_slot(ctx)) != MCPR_OK) return st;
            slot = ctx->prof_used;
        }
        const int tries[4] = {2, 8, 32, m};
        for (int a = ctx->cdf_engine ? 0 : 3; a < 4; ++a) {
            const int lib = std::min(tries[a], m);
            // (the profile events of a later attempt replace those of a failed one)
            if (lib >= m) {
                if ((st = enqueue_fine(ctx, bf, t, prec, deg, 0, m, nreg, sp, want_stats, trace != nullptr, s,
                                       ctx->profile, lib)) != MCPR_OK)
                    return st;
                ctx->cdf_sweeps[1]++;
                break;
            }
            const int mid = lib + 1; // through the first bucket step, then the rest
            bool over = false;
            for (int part = 0; part < 2 && !over; ++part) {
                const int j0 = part == 0 ? 0 : mid, j1 = part == 0 ? mid : m;
                if (j0 >= j1) continue;
                if ((st = enqueue_fine(ctx, bf, t, prec, deg, 0, m, nreg, sp, want_stats, trace != nullptr, s,
                                       ctx->profile, lib, j0, j1)) != MCPR_OK)
                    return st;
                HIP_TRY(hipMemcpyAsync(ctx->cdf_flag_host, ctx->cdfb.flag, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                       s));
                HIP_TRY(hipStreamSynchronize(s));
                over = *ctx->cdf_flag_host != 0;
            }
            if (!over) {
                ctx->cdf_sweeps[0]++;
                break;
            }
            ctx->cdf_sweeps[2]++;
        }
        if (ctx->profile) {
            ctx->prof_ps[slot] = ps * m;
            ctx->prof_launches += m;
            ctx->prof_used = slot + 1;
        }
        if (stats)
            HIP_TRY(hipMemcpyAsync(stats, ctx->recs.p, (size_t)n * (nreg + 1) * sizeof(RegionStats),
                                   hipMemcpyDeviceToDevice, s));
        if (trace)
            HIP_TRY(hipMemcpyAsync(trace, ctx->trace.p, (size_t)n * (m + 1) * sizeof(double2),
                                   hipMemcpyDeviceToDevice, s));
        return MCPR_OK;
    }
    // An ensemble of more than 256 superchunks makes every block of the
    // in-block-combine variants read more than one partial per thread: only
    // the separate-combine variants are candidates then, and the default is
    // the plain one of those.
    const bool many = max_nsc > mcpr::kThreads;
    const bool resident = resident_ok(ctx, t, prec, m) &&
                          ctx->znorm.cap >= (size_t)t.total_z * (prec == 0 ? sizeof(double) : sizeof(float));
    // step-kernel variant: forced, tuned for this launch shape, or tuned now
    std::vector<char> tkey(6 * sizeof(int64_t));
    {
        const int64_t tk[6] = {prec, deg, n, (int64_t)t.blocks.size(), t.total_sc, ps};
        std::memcpy(tkey.data(), tk, sizeof tk);
    }
    int variant = many ? 2 : 0;
    bool tune_now = false;
    if (resident) {
        variant = kResidentVariant;
        ctx->resident_sweeps++;
    } else if (ctx->tuning >= 0) {
        variant = ctx->tuning & 3;
    } else {
        auto it = ctx->tuned.find(tkey);
        if (it != ctx->tuned.end()) {
            variant = it->second;
        } else if (!ctx->profile && !t.items[0].trig && !t.items[0].cdf) {
            tune_now = true;
        }
    }
    if (tune_now) {
        int nc = 0;
        for (int v = many ? 2 : 0; v < 4; ++v) ctx->tune_cand[nc++] = v;
        // K/nc consecutive launches per candidate: four when the sweep is long
        // enough, else two, else no trial (the default is kept)
        const int per = m >= 4 * nc ? 4 : (m >= 2 * nc ? 2 : 0);
        ctx->tune_nc = nc;
        ctx->tune_steps = per * nc;
        if (per == 0) {
            ctx->tuned[tkey] = variant;
            tune_now = false;
        }
    }
    if (tune_now) {
        // trial: the first K steps run each candidate on K/nc consecutive
        // launches; a candidate's time is the mean of its launches after the
        // first (the first one inherits the cache state the previous candidate
        // left); a candidate other than the first must beat it by 1 %
        if (!ctx->tune_ev[0][0])
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < kTuneSteps; ++j) HIP_TRY(hipEventCreate(&ctx->tune_ev[k][j]));
        if ((st = enqueue_fine(ctx, bf, t, prec, deg, -1, m, nreg, sp, want_stats, trace != nullptr, s,
                               false)) != MCPR_OK)
            return st;
        HIP_TRY(hipEventSynchronize(ctx->tune_ev[1][ctx->tune_steps - 1]));
        float tv[4] = {0, 0, 0, 0};
        const int per = ctx->tune_steps / ctx->tune_nc;
        for (int j = 0; j < ctx->tune_steps; ++j) {
            if (j % per == 0) continue;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ctx->tune_ev[0][j], ctx->tune_ev[1][j]));
            tv[j / per] += ms / (float)(per - 1);
        }
        int pick = 0;
        for (int c = 1; c < ctx->tune_nc; ++c)
            if (tv[c] < 0.99f * tv[0] && tv[c] < tv[pick]) pick = c;
        ctx->tuned[tkey] = ctx->tune_cand[pick];
    } else if (ctx->profile) {
        if ((st = next_prof_slot(ctx)) != MCPR_OK) return st;
        ctx->prof_ps[ctx->prof_used] = ps * m;
        ctx->prof_launches += m;
        if ((st = enqueue_fine(ctx, bf, t, prec, deg, variant, m, nreg, sp, want_stats, trace != nullptr, s,
                               true)) != MCPR_OK)
            return st;
        ctx->prof_used++;
    } else if (ctx->graphs && !t.items[0].cdf) {
        // (the empirical-CDF sweep runs the library sort eagerly: never captured)
        std::vector<char> key = graph_key(ctx, t, prec, deg, variant, m, nreg, sp, want_stats, trace != nullptr);
        if ((st = replay(ctx, key, s,
                         [&](hipStream_t gs) {
                             return enqueue_fine(ctx, bf, t, prec, deg, variant, m, nreg, sp, want_stats,
                                                 trace != nullptr, gs, false);
                         })) != MCPR_OK)
            return st;
    } else {
        if ((st = enqueue_fine(ctx, bf, t, prec, deg, variant, m, nreg, sp, want_stats, trace != nullptr, s,
                               false)) != MCPR_OK)
            return st;
    }
    if (stats)
        HIP_TRY(hipMemcpyAsync(stats, ctx->recs.p, (size_t)n * (nreg + 1) * sizeof(RegionStats),
                               hipMemcpyDeviceToDevice, s));
    if (trace)
        HIP_TRY(hipMemcpyAsync(trace, ctx->trace.p, (size_t)n * (m + 1) * sizeof(double2), hipMemcpyDeviceToDevice, s));
    return MCPR_OK;
}

} // namespace

namespace {

// Tables of the adjoint's backward steps from those of the recomputed slice:
// the backward steps have sums of their own (the adjoint's ensemble sums and
// the gradient sums), so they need not share the forward superchunks; one quad
// per thread below 262144 particles, where a single ensemble's launch is
// latency bound and short blocks finish sooner.
Tables backward_tables(const Tables &tt, int64_t P) {
    Tables tb = tt;
    WorkItem &w = tb.items[0];
    w.R = P < kAdjointSmall ? 1 : mcpr::kMaxQuadsPerThread;
    w.nsc = (int32_t)mcpr::superchunks(P, w.R);
    tb.blocks.clear();
    for (int sc = 0; sc < w.nsc; ++sc) tb.blocks.push_back(make_int2(0, sc));
    tb.total_sc = w.nsc;
    return tb;
}

// ---- adjoint: one launch sequence over device tables, run directly or replayed from a graph ----
// Shape of an adjoint call and its host tables (counts and flags only: the
// kernels read every per-slice item from the device).
struct AdjPlan {
    int prec = 0, deg = 1, variant = 0, m = 0, NS = 0, n0 = 0, nreg = 1;
    int64_t P = 0, Ps = 0;
    size_t esz = 4;
    mcpr::Splits sp{};
    bool grad = false;
    Tables t1; // one forward or recomputed slice (one item)
    Tables tb; // the backward steps' item
};

AdjPlan adjoint_plan(mcpr_ctx *ctx, const mcpr_problem &p, const mcpr_ensemble &e, bool grad) {
    AdjPlan pl;
    pl.prec = p.precision;
    pl.m = p.steps_per_slice;
    pl.n0 = e.slice;
    pl.NS = p.n_slices - e.slice;
    pl.nreg = p.n_regions;
    pl.P = e.n_particles;
    pl.Ps = (pl.P + 3) / 4 * 4;
    pl.esz = p.precision == MCPR_FP64 ? 8 : 4;
    pl.sp = splits_of(p);
    pl.grad = grad;
    mcpr_ensemble one = e;
    one.problem = 0;
    build_tables(&p, &one, 1, pl.t1);
    pl.deg = (p.coef.a2 != 0.0 || p.coef.a3 != 0.0) ? 3 : 1;
    // the step variant this launch shape was tuned to, else the untuned default
    std::vector<char> tkey(6 * sizeof(int64_t));
    const int64_t tk[6] = {pl.prec, pl.deg, 1, (int64_t)pl.t1.blocks.size(), pl.t1.total_sc, pl.P};
    std::memcpy(tkey.data(), tk, sizeof tk);
    const bool many = pl.t1.items[0].nsc > mcpr::kThreads;
    pl.variant = many ? 2 : 0;
    if (ctx->tuning >= 0) {
        pl.variant = ctx->tuning & 3;
    } else {
        auto it = ctx->tuned.find(tkey);
        if (it != ctx->tuned.end()) pl.variant = it->second;
    }
    Tables tt = pl.t1;
    tt.items[0].traj = pl.Ps;
    pl.tb = backward_tables(tt, pl.P);
    return pl;
}

// Staging layout of the adjoint's tables: forward items [NS], recomputed
// items [NS], the slice block table, the backward item and block table, the
// upstream derivatives [NS][2].
struct AdjLayout {
    size_t fitems, ritems, fblocks, bitem, bblocks, dl, total;
};
AdjLayout adjoint_layout(const AdjPlan &pl) {
    AdjLayout L;
    size_t o = 0;
    auto take = [&o](size_t b) {
        const size_t r = o;
        o += align256(b);
        return r;
    };
    L.fitems = take((size_t)pl.NS * sizeof(WorkItem));
    L.ritems = take((size_t)pl.NS * sizeof(WorkItem));
    L.fblocks = take(pl.t1.blocks.size() * sizeof(int2));
    L.bitem = take(sizeof(WorkItem));
    L.bblocks = take(pl.tb.blocks.size() * sizeof(int2));
    L.dl = take((size_t)pl.NS * 2 * sizeof(double));
    L.total = o;
    return L;
}

mcpr_status upload_adjoint(mcpr_ctx *ctx, const AdjPlan &pl, const mcpr_problem &p, const mcpr_ensemble &e,
                           const double *dL, hipStream_t s) {
    const AdjLayout L = adjoint_layout(pl);
    char *h;
    mcpr_status st;
    if ((st = stage(ctx, L.total, &h)) != MCPR_OK) return st;
    std::memset(h, 0, L.total);
    char *ckpt = (char *)ctx->adj_ckpt.p;
    const size_t tstride = (size_t)(pl.m + 1) * pl.Ps * pl.esz;
    WorkItem *fi = (WorkItem *)(h + L.fitems), *ri = (WorkItem *)(h + L.ritems);
    for (int n = 0; n < pl.NS; ++n) {
        fi[n] = pl.t1.items[0];
        fi[n].x = ckpt + (size_t)(n + 1) * pl.Ps * pl.esz; // slice n runs in place on the copy of its start
        fi[n].step0 = (pl.n0 + n) * pl.m;
        ri[n] = pl.t1.items[0];
        ri[n].x = (char *)ctx->adj_traj.p + (size_t)(n & 1) * tstride; // recomputed out of place
        ri[n].traj = pl.Ps;
        ri[n].step0 = (pl.n0 + n) * pl.m;
    }
    std::memcpy(h + L.fblocks, pl.t1.blocks.data(), pl.t1.blocks.size() * sizeof(int2));
    std::memcpy(h + L.bitem, pl.tb.items.data(), sizeof(WorkItem));
    std::memcpy(h + L.bblocks, pl.tb.blocks.data(), pl.tb.blocks.size() * sizeof(int2));
    if (dL) std::memcpy(h + L.dl, dL, (size_t)pl.NS * 2 * sizeof(double));
    (void)p;
    (void)e;
    HIP_TRY(hipMemcpyAsync(ctx->adj_tables.p, h, L.total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->staged, s));
    return MCPR_OK;
}

// Everything a captured adjoint depends on besides the tables' contents.
std::vector<char> adjoint_key(mcpr_ctx *ctx, const AdjPlan &pl) {
    const void *ptrs[] = {ctx->adj_tables.p, ctx->adj_ckpt.p, ctx->adj_traj.p, ctx->adj_trace.p, ctx->adj_lam[0].p,
                          ctx->adj_lam[1].p, ctx->adj_part[0].p, ctx->adj_part[1].p, ctx->adj_acc.p, ctx->adj_grad.p,
                          ctx->adj_sums.p, ctx->part[0].p, ctx->part[1].p, ctx->shift[0].p, ctx->shift[1].p, ctx->mv.p};
    const int64_t ints[] = {-1 /* an adjoint, not a sweep */, pl.prec, pl.deg, pl.variant, pl.m, pl.NS, pl.n0,
                            pl.nreg, pl.P, pl.grad ? 1 : 0};
    std::vector<char> k(sizeof ptrs + sizeof ints + sizeof pl.sp);
    std::memcpy(k.data(), ptrs, sizeof ptrs);
    std::memcpy(k.data() + sizeof ptrs, ints, sizeof ints);
    std::memcpy(k.data() + sizeof ptrs + sizeof ints, &pl.sp, sizeof pl.sp);
    return k;
}

// The adjoint's launch sequence on stream s (forward, then the backward steps)
// and r (the recomputations, overlapped with the backward steps of the next
// slice).  Every scalar the kernels need comes from device memory (tables,
// trace, upstream derivatives), so the sequence can be captured once and
// replayed.  Forward: each slice copies its start to its checkpoint slot and
// runs in place there with its moments traced.  Backward: see mcpr_adjoint.
mcpr_status enqueue_adjoint(mcpr_ctx *ctx, const AdjPlan &pl, hipStream_t s, hipStream_t r, bool profile) {
    const AdjLayout L = adjoint_layout(pl);
    char *tab = (char *)ctx->adj_tables.p;
    const WorkItem *fitems = (const WorkItem *)(tab + L.fitems), *ritems = (const WorkItem *)(tab + L.ritems);
    const int2 *fblocks = (const int2 *)(tab + L.fblocks);
    const WorkItem *bitem = (const WorkItem *)(tab + L.bitem);
    const int2 *bblocks = (const int2 *)(tab + L.bblocks);
    const double *dl = (const double *)(tab + L.dl);
    const int m = pl.m, NS = pl.NS, n0 = pl.n0;
    const size_t esz = pl.esz, slot = (size_t)pl.Ps * esz, tstride = (size_t)(m + 1) * slot;
    char *ckpt = (char *)ctx->adj_ckpt.p;
    char *trajb[2] = {(char *)ctx->adj_traj.p, (char *)ctx->adj_traj.p + tstride};
    double2 *trace = (double2 *)ctx->adj_trace.p;
    Bufs bf = ctx_bufs(ctx);
    bf.blocks = fblocks;
    mcpr_status st;
    for (int n = 0; n < NS; ++n) {
        HIP_TRY(hipMemcpyAsync(ckpt + (size_t)(n + 1) * slot, ckpt + (size_t)n * slot, (size_t)pl.P * esz,
                               hipMemcpyDeviceToDevice, s));
        bf.items = fitems + n;
        bf.trace = trace + (size_t)n * (m + 1);
        if ((st = enqueue_fine(ctx, bf, pl.t1, pl.prec, pl.deg, pl.variant, m, pl.nreg, pl.sp, false, true, s,
                               false)) != MCPR_OK)
            return st;
    }
    if (!pl.grad) return MCPR_OK;

    const int nsc = pl.tb.total_sc, nb = (int)pl.tb.blocks.size();
    double2 *sums = nsc > mcpr::kThreads ? (double2 *)ctx->adj_sums.p : nullptr;
    double *lam[2] = {(double *)ctx->adj_lam[0].p, (double *)ctx->adj_lam[1].p};
    double2 *apart[2] = {(double2 *)ctx->adj_part[0].p, (double2 *)ctx->adj_part[1].p};
    double *acc = (double *)ctx->adj_acc.p;
    const bool zprev = pl.tb.items[0].c[8] != 0.0 || pl.tb.items[0].c[9] != 0.0;
    const double invP = 1.0 / (double)pl.P;
    HIP_TRY(mcpr::launch_zero(acc, (int64_t)nsc * 10, s));
    int cur = 0, pc = 0;
    {
        // lambda at the final state: the slice-end term of the last slice
        mcpr::AdjRef a{nullptr, dl + 2 * (NS - 1), trace + (size_t)(NS - 1) * (m + 1) + m, invP, (n0 + NS) * m,
                       0, 0, 0};
        HIP_TRY(mcpr::launch_adj_init(pl.prec, bitem, bblocks, nb, ckpt + (size_t)NS * slot, lam[cur], a, apart[pc],
                                      s));
    }
    // the forward sweeps (and their use of the slice scratch) are done
    HIP_TRY(hipEventRecord(ctx->a_fwd, s));
    HIP_TRY(hipStreamWaitEvent(r, ctx->a_fwd, 0));
    Bufs rb = ctx_bufs(ctx);
    rb.blocks = fblocks;
    rb.trace = nullptr;
    auto recompute = [&](int n) -> mcpr_status {
        HIP_TRY(hipMemcpyAsync(trajb[n & 1], ckpt + (size_t)n * slot, (size_t)pl.P * esz, hipMemcpyDeviceToDevice, r));
        rb.items = ritems + n;
        mcpr_status st2;
        if ((st2 = enqueue_fine(ctx, rb, pl.t1, pl.prec, pl.deg, pl.variant, m, pl.nreg, pl.sp, false, false, r,
                                false)) != MCPR_OK)
            return st2;
        HIP_TRY(hipEventRecord(ctx->a_rec[n & 1], r));
        return MCPR_OK;
    };
    if ((st = recompute(NS - 1)) != MCPR_OK) return st;
    for (int n = NS - 1; n >= 0; --n) {
        if (n >= 1) {
            // buffer (n - 1) & 1 was last read by the backward steps of slice n + 1
            if (n + 1 < NS) HIP_TRY(hipStreamWaitEvent(r, ctx->a_bwd[(n + 1) & 1], 0));
            if ((st = recompute(n - 1)) != MCPR_OK) return st;
        }
        HIP_TRY(hipStreamWaitEvent(s, ctx->a_rec[n & 1], 0));
        char *traj = trajb[n & 1];
        if (profile) {
            if (ctx->aprof_used == ctx->aprof0.size()) {
                hipEvent_t e0, e1;
                HIP_TRY(hipEventCreate(&e0));
                HIP_TRY(hipEventCreate(&e1));
                ctx->aprof0.push_back(e0);
                ctx->aprof1.push_back(e1);
            }
            HIP_TRY(hipEventRecord(ctx->aprof0[ctx->aprof_used], s));
        }
        for (int j = m - 1; j >= 0; --j) {
            mcpr::AdjRef a{trace + (size_t)n * (m + 1) + j, nullptr, nullptr, invP, (n0 + n) * m + j,
                           (zprev && (n > 0 || j > 0)) ? 1 : 0, 1, 0};
            if (j == 0 && n > 0) { // slice end n-1 (the state that starts slice n)
                a.dl = dl + 2 * (n - 1);
                a.end = trace + (size_t)(n - 1) * (m + 1) + m;
            }
            HIP_TRY(mcpr::launch_adj_step(pl.prec, bitem, 1, bblocks, nb, traj + (size_t)j * slot, lam[cur],
                                          lam[cur ^ 1], a, apart[pc], sums, apart[pc ^ 1], acc, s));
            cur ^= 1;
            pc ^= 1;
        }
        HIP_TRY(hipEventRecord(ctx->a_bwd[n & 1], s));
        if (profile) {
            HIP_TRY(hipEventRecord(ctx->aprof1[ctx->aprof_used], s));
            ctx->aprof_used++;
            ctx->aprof_launches += m;
            ctx->aprof_ps += pl.P * m;
        }
    }
    HIP_TRY(mcpr::launch_adj_reduce(bitem, 1, acc, (double *)ctx->adj_grad.p, s));
    return MCPR_OK;
}

// Buffers of mcpr_adjoint on ensemble e (problem p): the forward sweeps with
// their trace and checkpoints and, with the backward sweep, the recomputed
// trajectory, the adjoint state and the gradient sums.
mcpr_status size_adjoint(mcpr_ctx *ctx, const mcpr_problem &p, const mcpr_ensemble &e, bool backward) {
    const int m = p.steps_per_slice, NS = p.n_slices - e.slice;
    const int64_t P = e.n_particles, Ps = (P + 3) / 4 * 4;
    const size_t esz = p.precision == MCPR_FP64 ? 8 : 4;
    mcpr_ensemble one = e;
    one.problem = 0;
    Tables t;
    build_tables(&p, &one, 1, t);
    mcpr_status st;
    // the slice scratch of the forward sweeps and the recomputations
    if ((st = size_fine(ctx, t, p.precision, m, p.n_regions, false, true)) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->adj_ckpt, (size_t)(NS + 1) * Ps * esz)) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->adj_trace, (size_t)NS * (m + 1) * 2 * sizeof(double))) != MCPR_OK) return st;
    Tables tt = t;
    tt.items[0].traj = Ps;
    const Tables tb = backward_tables(tt, P);
    AdjPlan pl;
    pl.m = m;
    pl.NS = NS;
    pl.t1 = t;
    pl.tb = tb;
    const AdjLayout L = adjoint_layout(pl);
    if ((st = ensure(ctx, ctx->adj_tables, L.total)) != MCPR_OK) return st;
    if ((st = ensure_host(ctx, ctx->staging, L.total)) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->adj_traj, 2 * (size_t)(m + 1) * Ps * esz)) != MCPR_OK) return st;
    const int nsc = tb.total_sc;
    for (int b = 0; b < 2; ++b) {
        if ((st = ensure(ctx, ctx->adj_lam[b], (size_t)Ps * sizeof(double))) != MCPR_OK) return st;
        if ((st = ensure(ctx, ctx->adj_part[b], (size_t)nsc * sizeof(double2))) != MCPR_OK) return st;
    }
    if ((st = ensure(ctx, ctx->adj_acc, (size_t)nsc * 10 * sizeof(double))) != MCPR_OK) return st;
    if ((st = ensure(ctx, ctx->adj_grad, 10 * sizeof(double))) != MCPR_OK) return st;
    (void)backward; // the backward buffers are sized always: a context that has run the forward alone can differentiate
    return ensure(ctx, ctx->adj_sums, sizeof(double2));
}

// Buffers of the calls named in `calls` (MCPR_RESERVE_*) on the ensembles of
// t (problems: the call's problems, for the adjoint).
mcpr_status size_calls(mcpr_ctx *ctx, const Tables &t, const mcpr_problem *problems, const mcpr_ensemble *ens,
                       int32_t calls, size_t map_bytes) {
    const mcpr_problem &p = problems[ens[0].problem];
    mcpr_status st;
    if ((st = size_upload(ctx, t, map_bytes)) != MCPR_OK) return st;
    if ((calls & (MCPR_RESERVE_MOMENTS | MCPR_RESERVE_MATCH)) && (st = ensure_records(ctx, t, p.n_regions)) != MCPR_OK)
        return st;
    if ((calls & MCPR_RESERVE_QOI) &&
        (st = ensure(ctx, ctx->part[0], (size_t)t.total_sc * sizeof(double2))) != MCPR_OK)
        return st;
    if ((calls & MCPR_RESERVE_FINE) &&
        (st = size_fine(ctx, t, p.precision, p.steps_per_slice, p.n_regions, true, true)) != MCPR_OK)
        return st;
    if (calls & MCPR_RESERVE_ADJOINT) {
        for (size_t e = 0; e < t.items.size(); ++e)
            if ((st = size_adjoint(ctx, problems[ens[e].problem], ens[e], true)) != MCPR_OK) return st;
    }
    return MCPR_OK;
}

} // namespace

// ============================================================================
// Static scratch of mcpr_fine_propagate_static (no allocation on any call)
// ============================================================================
// Holds the work and block tables, the step partials and shifts, the mean
// field and the region partials of one call; each device has its own copy,
// which lives until the process ends.  Nothing in it needs clearing: every
// part is written before it is read within a call.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up
// once per device: the array's name in host code is not a device address.
mcpr_status static_scratch(int dev, char **out) {
    mcpr_ctx *ctx = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return fail(ctx, MCPR_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(ctx, MCPR_E_DEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return MCPR_OK;
}

// Work item e (by value) and its block-table entries (e, s), s < nsc, at its
// first superchunk.
__global__ __launch_bounds__(mcpr::kThreads) void k_put_item(WorkItem w, int32_t e, WorkItem *__restrict__ items,
                                                            int2 *__restrict__ blocks) {
    if (blockIdx.x == 0 && threadIdx.x == 0) items[e] = w;
    for (int sc = blockIdx.x * mcpr::kThreads + threadIdx.x; sc < w.nsc; sc += gridDim.x * mcpr::kThreads)
        blocks[w.part_off + sc] = make_int2(e, sc);
}

} // namespace

namespace {

// The fine propagator of mcpr_fine_propagate.  want_stats: the restriction
// records are formed; stats (may be NULL then) receives a copy of them, which
// otherwise stay in the context's records buffer (ctx->recs) for the caller
// inside the library to read.
mcpr_status fine_propagate(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                           const mcpr_ensemble *ens, int32_t n_ens, bool want_stats, RegionStats *stats,
                           double2 *trace, hipStream_t s) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    const mcpr_problem &p = problems[ens[0].problem];
    Tables t;
    build_tables(problems, ens, n_ens, t);
    if ((st = size_fine(ctx, t, p.precision, p.steps_per_slice, p.n_regions, want_stats, trace != nullptr)) !=
        MCPR_OK)
        return st;
    if ((st = upload(ctx, t, nullptr, 0, s)) != MCPR_OK) return st;
    return fine_sequence(ctx, t, p.precision, p.steps_per_slice, p.n_regions, splits_of(p), want_stats, stats,
                         trace, s);
}

} // namespace

// ============================================================================
// C ABI: context
// ============================================================================
extern "C" {

const char *mcpr_version(void) { return "mcpr 0.1 (gfx950)"; }

mcpr_status mcpr_create(mcpr_ctx **out, int32_t device) {
    if (!out) return MCPR_E_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return MCPR_E_DEVICE;
    if (device < 0 || device >= count) return MCPR_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return MCPR_E_DEVICE;
    mcpr_ctx *ctx = new mcpr_ctx();
    ctx->device = device;
    if (hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->gin, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->gout, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->astream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->a_fwd, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->a_rec[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->a_rec[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->a_bwd[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->a_bwd[1], hipEventDisableTiming) != hipSuccess) {
        mcpr_destroy(ctx);
        return MCPR_E_DEVICE;
    }
    *out = ctx;
    return MCPR_OK;
}

void mcpr_destroy(mcpr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    DevBuf *bufs[] = {&ctx->tables,      &ctx->part[0],     &ctx->part[1],     &ctx->shift[0],
                      &ctx->shift[1],      &ctx->rpart,       &ctx->rshift[0],   &ctx->rshift[1],
                      &ctx->recs,          &ctx->adj_ckpt,    &ctx->adj_traj,    &ctx->adj_lam[0],  &ctx->adj_lam[1],
                      &ctx->adj_part[0],   &ctx->adj_part[1], &ctx->adj_acc,     &ctx->adj_trace,   &ctx->adj_grad,
                      &ctx->adj_sums,      &ctx->adj_tables,  &ctx->trace,       &ctx->mv,
                      &ctx->cdf_keys[0],   &ctx->cdf_keys[1], &ctx->cdf_lab[0],  &ctx->cdf_lab[1],  &ctx->cdf_seg[0],
                      &ctx->cdf_seg[1],    &ctx->cdf_kl[0],   &ctx->cdf_kl[1],   &ctx->cdf_beg,     &ctx->cdf_tmp,
                      &ctx->cdf_bcount,    &ctx->cdf_bmeta,   &ctx->cdf_stage,   &ctx->cdf_flag,    &ctx->cdf_defer,
                      &ctx->znorm};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->staging.p) (void)hipHostFree(ctx->staging.p);
    if (ctx->cdf_flag_host) (void)hipHostFree(ctx->cdf_flag_host);
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    for (hipEvent_t e : ctx->prof0) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->prof1) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->aprof0) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->aprof1) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < kTuneSteps; ++j)
            if (ctx->tune_ev[k][j]) (void)hipEventDestroy(ctx->tune_ev[k][j]);
    for (auto &e : ctx->graphs_cached) (void)hipGraphExecDestroy(e.exec);
    if (ctx->astream) (void)hipStreamDestroy(ctx->astream);
    for (hipEvent_t e : {ctx->a_fwd, ctx->a_rec[0], ctx->a_rec[1], ctx->a_bwd[0], ctx->a_bwd[1]})
        if (e) (void)hipEventDestroy(e);
    if (ctx->gin) (void)hipEventDestroy(ctx->gin);
    if (ctx->gout) (void)hipEventDestroy(ctx->gout);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    delete ctx;
}

const char *mcpr_last_error(const mcpr_ctx *ctx) { return ctx ? ctx->err.c_str() : g_static_err; }

mcpr_status mcpr_profile_enable(mcpr_ctx *ctx, int32_t on) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->profile = on != 0;
    return MCPR_OK;
}

mcpr_status mcpr_profile_read(mcpr_ctx *ctx, double *em_ms, int64_t *em_launches, int64_t *particle_steps,
                              int32_t reset) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    double ms_total = 0.0;
    int64_t ps = 0;
    for (size_t i = 0; i < ctx->prof_used; ++i) {
        HIP_TRY(hipEventSynchronize(ctx->prof1[i]));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->prof0[i], ctx->prof1[i]));
        ms_total += ms;
        ps += ctx->prof_ps[i];
    }
    if (em_ms) *em_ms = ms_total;
    if (em_launches) *em_launches = ctx->prof_launches;
    if (particle_steps) *particle_steps = ps;
    if (reset) {
        ctx->prof_used = 0;
        ctx->prof_launches = 0;
    }
    return MCPR_OK;
}

mcpr_status mcpr_profile_read_adjoint(mcpr_ctx *ctx, double *ms, int64_t *launches, int64_t *particle_steps,
                                      int32_t reset) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    HIP_TRY(hipSetDevice(ctx->device));
    double ms_total = 0.0;
    for (size_t i = 0; i < ctx->aprof_used; ++i) {
        HIP_TRY(hipEventSynchronize(ctx->aprof1[i]));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, ctx->aprof0[i], ctx->aprof1[i]));
        ms_total += t;
    }
    if (ms) *ms = ms_total;
    if (launches) *launches = ctx->aprof_launches;
    if (particle_steps) *particle_steps = ctx->aprof_ps;
    if (reset) {
        ctx->aprof_used = 0;
        ctx->aprof_launches = 0;
        ctx->aprof_ps = 0;
    }
    return MCPR_OK;
}

mcpr_status mcpr_stream_probe(void *x, int64_t n, int32_t reps, mcpr_stream stream, double *ms_per_pass) {
    mcpr_ctx *ctx = nullptr;
    if (!x || ((uintptr_t)x & 15) || n < 4096 || n % 4096 || n / 4 > 0xffffffffLL || reps < 1 || !ms_per_pass)
        return fail(ctx, MCPR_E_INVALID_ARG, "stream probe: a 16-byte aligned array of a multiple of 4096 floats");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, MCPR_E_DEVICE, "event creation failed");
    }
    hipError_t e = mcpr::launch_stream_inplace((float *)x, n, s); // warm-up pass
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = mcpr::launch_stream_inplace((float *)x, n, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ctx, MCPR_E_DEVICE, "stream probe: %s", hipGetErrorString(e));
    *ms_per_pass = (double)ms / reps;
    return MCPR_OK;
}

mcpr_status mcpr_set_graphs(mcpr_ctx *ctx, int32_t on) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    ctx->graphs = on != 0;
    return MCPR_OK;
}

mcpr_status mcpr_set_tuning(mcpr_ctx *ctx, int32_t mode) {
    if (!ctx || mode < -1 || mode > 3) return MCPR_E_INVALID_ARG;
    ctx->tuning = mode;
    return MCPR_OK;
}

int32_t mcpr_tuned_variant(const mcpr_ctx *ctx, int32_t index) {
    if (!ctx || index < 0) return -1;
    for (const auto &kv : ctx->tuned)
        if (index-- == 0) return kv.second;
    return -1;
}

mcpr_status mcpr_graph_stats(const mcpr_ctx *ctx, int64_t *builds, int64_t *launches) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    if (builds) *builds = ctx->graph_builds;
    if (launches) *launches = ctx->graph_launches;
    return MCPR_OK;
}

mcpr_status mcpr_set_resident(mcpr_ctx *ctx, int32_t enable) {
    if (!ctx || enable < 0 || enable > 1) return MCPR_E_INVALID_ARG;
    ctx->resident = enable;
    return MCPR_OK;
}

mcpr_status mcpr_resident_sweeps(const mcpr_ctx *ctx, int64_t *sweeps) {
    if (!ctx || !sweeps) return MCPR_E_INVALID_ARG;
    *sweeps = ctx->resident_sweeps;
    return MCPR_OK;
}

mcpr_status mcpr_set_cdf_sort(mcpr_ctx *ctx, int32_t mode) {
    if (!ctx || mode < 0 || mode > 1) return MCPR_E_INVALID_ARG;
    ctx->cdf_engine = mode;
    return MCPR_OK;
}

mcpr_status mcpr_cdf_stats(const mcpr_ctx *ctx, int64_t *bucket_sweeps, int64_t *library_sweeps,
                           int64_t *redone_sweeps) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    if (bucket_sweeps) *bucket_sweeps = ctx->cdf_sweeps[0];
    if (library_sweeps) *library_sweeps = ctx->cdf_sweeps[1];
    if (redone_sweeps) *redone_sweeps = ctx->cdf_sweeps[2];
    return MCPR_OK;
}

mcpr_status mcpr_reserve(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                         int32_t n_ens, int32_t calls) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    if (calls <= 0 || (calls & ~MCPR_RESERVE_ALL))
        return fail(ctx, MCPR_E_INVALID_ARG, "calls %d: a nonempty mask of MCPR_RESERVE_*", calls);
    if (calls & MCPR_RESERVE_ADJOINT)
        for (int e = 0; e < n_ens; ++e) {
            const mcpr_problem &p = problems[ens[e].problem];
            if (ens[e].slice >= p.n_slices)
                return fail(ctx, MCPR_E_INVALID_ARG, "ensemble %d: first slice beyond n_slices", e);
            if (p.coef.axs != 0.0 || is_trig(p) || is_cdf(p) || p.wrap)
                return fail(ctx, MCPR_E_UNSUPPORTED, "the adjoint needs axs = ksin = kc = acdf = 0 and no wrap");
        }
    HIP_TRY(hipSetDevice(ctx->device));
    Tables t;
    build_tables(problems, ens, n_ens, t);
    Growing grow(ctx);
    return size_calls(ctx, t, problems, ens, calls, 0);
}

mcpr_status mcpr_alloc_stats(const mcpr_ctx *ctx, int64_t *allocations, int64_t *bytes) {
    if (!ctx) return MCPR_E_INVALID_ARG;
    if (allocations) *allocations = ctx->allocs;
    if (bytes) *bytes = ctx->alloc_bytes;
    return MCPR_OK;
}

// ============================================================================
// C ABI: hot-path calls
// ============================================================================
mcpr_status mcpr_init_particles(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                const mcpr_ensemble *ens, int32_t n_ens, mcpr_stream stream) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Tables t;
    build_tables(problems, ens, n_ens, t);
    if ((st = upload(ctx, t, nullptr, 0, s)) != MCPR_OK) return st;
    HIP_TRY(mcpr::launch_init(problems[ens[0].problem].precision, ctx->items,
                              ctx->blocks, (int)t.blocks.size(), s));
    return MCPR_OK;
}

mcpr_status mcpr_moments(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                         int32_t n_ens, mcpr_region_stats *stats, mcpr_stream stream) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    if (!stats) return fail(ctx, MCPR_E_INVALID_ARG, "stats is null");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const mcpr_problem &p = problems[ens[0].problem];
    Tables t;
    build_tables(problems, ens, n_ens, t);
    if ((st = ensure_records(ctx, t, p.n_regions)) != MCPR_OK) return st;
    if ((st = upload(ctx, t, nullptr, 0, s)) != MCPR_OK) return st;
    return records(ctx, t, p.precision, p.n_regions, splits_of(p), nullptr, true, 0, nullptr, (RegionStats *)stats, s);
}

mcpr_status mcpr_qoi(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                     int32_t n_ens, int32_t kind, double *out, mcpr_stream stream) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    if (!out) return fail(ctx, MCPR_E_INVALID_ARG, "out is null");
    if (kind < MCPR_QOI_X || kind > MCPR_QOI_SIN_X2) return fail(ctx, MCPR_E_INVALID_ARG, "QoI kind %d", kind);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Tables t;
    build_tables(problems, ens, n_ens, t);
    if ((st = ensure(ctx, ctx->part[0], (size_t)t.total_sc * sizeof(double2))) != MCPR_OK) return st;
    if ((st = upload(ctx, t, nullptr, 0, s)) != MCPR_OK) return st;
    HIP_TRY(mcpr::launch_qoi(problems[ens[0].problem].precision, kind, ctx->items, n_ens,
                             ctx->blocks, (int)t.blocks.size(), (double2 *)ctx->part[0].p, out, s));
    return MCPR_OK;
}

mcpr_status mcpr_fine_propagate(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                const mcpr_ensemble *ens, int32_t n_ens, mcpr_region_stats *stats, double *trace,
                                mcpr_stream stream) {
    return fine_propagate(ctx, problems, n_problems, ens, n_ens, stats != nullptr, (RegionStats *)stats,
                          (double2 *)trace, (hipStream_t)stream);
}

mcpr_status mcpr_fine_propagate_static(const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                                       int32_t n_ens, mcpr_region_stats *stats, double *trace, mcpr_stream stream) {
    mcpr_ctx *ctx = nullptr; // errors go to the calling thread's context-free error text
    mcpr_status st = check_args(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    const mcpr_problem &p = problems[ens[0].problem];
    if (is_cdf(p))
        return fail(ctx, MCPR_E_UNSUPPORTED, "the empirical-CDF drift sorts every step and needs a context's buffers");
    Tables t;
    build_tables(problems, ens, n_ens, t);
    const int n = n_ens, nr = p.n_regions + 1, m = p.steps_per_slice;
    // the scratch layout of this call, every part 256-byte aligned
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t o_items = take((size_t)n * sizeof(WorkItem)), o_blocks = take((size_t)t.total_sc * sizeof(int2));
    const size_t o_part0 = take((size_t)t.total_sc * sizeof(double2)), o_part1 = take((size_t)t.total_sc * sizeof(double2));
    const size_t o_shift0 = take((size_t)n * sizeof(double)), o_shift1 = take((size_t)n * sizeof(double));
    const size_t o_mv = take((size_t)n * sizeof(double2));
    size_t o_rpart = 0, o_rs0 = 0, o_rs1 = 0;
    if (stats) {
        o_rpart = take((size_t)t.total_sc * nr * sizeof(RegionPartial));
        o_rs0 = take((size_t)n * nr * sizeof(double));
        o_rs1 = take((size_t)n * nr * sizeof(double));
    }
    if (off > kStaticScratchBytes)
        return fail(ctx, MCPR_E_INVALID_ARG,
                    "the call needs %zu bytes of scratch (%d superchunks, %d ensembles, %d regions); the static "
                    "scratch holds %zu",
                    off, t.total_sc, n, nr - 1, kStaticScratchBytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    char *base = nullptr;
    if ((st = static_scratch(dev, &base)) != MCPR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Bufs bf;
    WorkItem *items = (WorkItem *)(base + o_items);
    int2 *blocks = (int2 *)(base + o_blocks);
    bf.items = items;
    bf.blocks = blocks;
    bf.part[0] = (double2 *)(base + o_part0);
    bf.part[1] = (double2 *)(base + o_part1);
    bf.shift[0] = (double *)(base + o_shift0);
    bf.shift[1] = (double *)(base + o_shift1);
    bf.mv = (double2 *)(base + o_mv);
    bf.rpart = stats ? (RegionPartial *)(base + o_rpart) : nullptr;
    bf.rshift[0] = stats ? (double *)(base + o_rs0) : nullptr;
    bf.rshift[1] = stats ? (double *)(base + o_rs1) : nullptr;
    bf.recs = (RegionStats *)stats;  // the records and the trace go straight to the caller's arrays
    bf.trace = (double2 *)trace;
    // the work and block tables are written by kernels from their arguments (nothing is copied from the host)
    for (int e = 0; e < n; ++e) {
        const int grid = std::max(1, std::min(1024, (t.items[e].nsc + mcpr::kThreads - 1) / mcpr::kThreads));
        hipLaunchKernelGGL(k_put_item, dim3(grid), dim3(mcpr::kThreads), 0, s, t.items[e], e, items, blocks);
        HIP_TRY(hipGetLastError());
    }
    int deg = 1, max_nsc = 0;
    for (const WorkItem &w : t.items) {
        if (w.c[2] != 0.0 || w.c[3] != 0.0) deg = 3;
        max_nsc = std::max(max_nsc, w.nsc);
    }
    // the untuned default launch variant (every variant gives the same bits)
    const int variant = max_nsc > mcpr::kThreads ? 2 : 0;
    return enqueue_fine(ctx, bf, t, p.precision, deg, variant, m, p.n_regions, splits_of(p), stats != nullptr,
                        trace != nullptr, s, false);
}

mcpr_status mcpr_match(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems, const mcpr_ensemble *ens,
                       int32_t n_ens, const mcpr_region_map *maps, int32_t dry_run, mcpr_region_stats *probe,
                       mcpr_stream stream) {
    mcpr_status st = check_call(ctx, problems, n_problems, ens, n_ens);
    if (st != MCPR_OK) return st;
    if (!maps) return fail(ctx, MCPR_E_INVALID_ARG, "maps is null");
    if (dry_run && !probe) return fail(ctx, MCPR_E_INVALID_ARG, "dry run needs a probe array");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const mcpr_problem &p = problems[ens[0].problem];
    Tables t;
    build_tables(problems, ens, n_ens, t);
    if (dry_run && (st = ensure_records(ctx, t, p.n_regions)) != MCPR_OK) return st;
    if ((st = upload(ctx, t, nullptr, 0, s)) != MCPR_OK) return st;
    if (dry_run)
        return records(ctx, t, p.precision, p.n_regions, splits_of(p), nullptr, true, 1, (const RegionMap *)maps,
                       (RegionStats *)probe, s);
    HIP_TRY(mcpr::launch_match_apply(p.precision, p.n_regions, ctx->items,
                                     ctx->blocks, (int)t.blocks.size(), splits_of(p),
                                     (const RegionMap *)maps, s));
    return MCPR_OK;
}

mcpr_status mcpr_adjoint(mcpr_ctx *ctx, const mcpr_problem *problem, const mcpr_ensemble *ens,
                         const double *dL_dmoments, double *moments_out, double *grad_out, mcpr_stream stream) {
    mcpr_status st = check_call(ctx, problem, 1, ens, 1);
    if (st != MCPR_OK) return st;
    if (ens->problem != 0) return fail(ctx, MCPR_E_INVALID_ARG, "ensemble must use problem 0");
    if (ens->slice >= problem->n_slices) return fail(ctx, MCPR_E_INVALID_ARG, "first slice beyond n_slices");
    if (problem->coef.axs != 0.0 || is_trig(*problem) || is_cdf(*problem) || problem->wrap)
        return fail(ctx, MCPR_E_UNSUPPORTED, "the adjoint needs axs = ksin = kc = acdf = 0 and no wrap");
    if (dL_dmoments && !grad_out) return fail(ctx, MCPR_E_INVALID_ARG, "grad_out is null");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if ((st = size_adjoint(ctx, *problem, *ens, dL_dmoments != nullptr)) != MCPR_OK) return st;
    AdjPlan pl = adjoint_plan(ctx, *problem, *ens, dL_dmoments != nullptr);
    const int m = pl.m, NS = pl.NS;
    // the work tables of every forward and recomputed slice, the backward
    // item and the upstream derivatives: one upload
    if ((st = upload_adjoint(ctx, pl, *problem, *ens, dL_dmoments, s)) != MCPR_OK) return st;
    HIP_TRY(hipMemcpyAsync(ctx->adj_ckpt.p, ens->x, (size_t)pl.P * pl.esz, hipMemcpyDeviceToDevice, s));
    if (ctx->graphs && !ctx->profile) {
        // the whole sequence from one graph, instantiated once per shape
        if ((st = replay(ctx, adjoint_key(ctx, pl), s,
                         [&](hipStream_t gs) { return enqueue_adjoint(ctx, pl, gs, ctx->astream, false); })) != MCPR_OK)
            return st;
    } else if ((st = enqueue_adjoint(ctx, pl, s, ctx->astream, ctx->profile)) != MCPR_OK) {
        return st;
    }
    std::vector<double> tr((size_t)NS * (m + 1) * 2);
    HIP_TRY(hipMemcpyAsync(tr.data(), ctx->adj_trace.p, tr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    if (dL_dmoments)
        HIP_TRY(hipMemcpyAsync(grad_out, ctx->adj_grad.p, 10 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (moments_out)
        for (int n = 0; n < NS; ++n) {
            moments_out[2 * n] = tr[((size_t)n * (m + 1) + m) * 2];
            moments_out[2 * n + 1] = tr[((size_t)n * (m + 1) + m) * 2 + 1];
        }
    return MCPR_OK;
}

} // extern "C"

// ============================================================================
// MC-moments Parareal driver
// ============================================================================
namespace {

// ---- coarse propagator: Taylor moment model per region, fractions frozen ----
// dM_i/dt = a(M_i, mbar, vbar) + a_xx(M_i) V_i / 2
// dV_i/dt = (2 a_x(M_i) + b_x(M_i)^2) V_i + b(M_i, mbar, vbar)^2
// (mbar, vbar) = mixture mean and variance of the regional moments.
struct Macro {
    double f[mcpr::kMaxRegions];
    double M[mcpr::kMaxRegions];
    double V[mcpr::kMaxRegions];
};

void mixture(int I, const Macro &r, double &mbar, double &vbar) {
    double m = 0.0;
    for (int i = 0; i < I; ++i)
        if (r.f[i] > 0.0) m += r.f[i] * r.M[i];
    double v = 0.0;
    for (int i = 0; i < I; ++i)
        if (r.f[i] > 0.0) {
            const double d = r.M[i] - m;
            v += r.f[i] * (r.V[i] + d * d);
        }
    mbar = m;
    vbar = v;
}

// Drift and diffusion at x with the mean field (mbar, vbar) and, for the
// trigonometric terms, (S, C) = the means of sin X and cos X.
double drift_at(const mcpr_coef &c, double x, double mbar, double vbar, double S, double C) {
    double a = c.a0 + x * (c.a1 + x * (c.a2 + x * c.a3)) + c.am * mbar + c.av * vbar + c.axs * x * (vbar + mbar * mbar);
    if (c.ksin != 0.0 || c.kc != 0.0) a += c.ksin * std::sin(x) + c.kc * (S * std::cos(x) - C * std::sin(x));
    return a;
}

double diffusion_at(const mcpr_coef &c, double x, double mbar, double vbar) {
    return c.b0 + c.b1 * x + c.bm * mbar + c.bv * vbar;
}

// Sigma points of N(M, V) (Gauss-Hermite): 2 points M +- sqrt V, weights 1/2;
// 3 points M, M +- sqrt(3V), weights 2/3, 1/6, 1/6; V < 0 as V = 0.
int sigma_points(int npts, double M, double V, double *xs, double *ws) {
    const double Vp = V > 0.0 ? V : 0.0;
    if (npts == 2) {
        xs[0] = M - std::sqrt(Vp);
        xs[1] = M + std::sqrt(Vp);
        ws[0] = ws[1] = 0.5;
        return 2;
    }
    const double h = std::sqrt(3.0 * Vp);
    xs[0] = M - h;
    xs[1] = M;
    xs[2] = M + h;
    ws[0] = 1.0 / 6.0;
    ws[1] = 2.0 / 3.0;
    ws[2] = 1.0 / 6.0;
    return 3;
}

// Gaussian assumed-density model: dM = E[a], dV = 2 E[(x - M) a] + E[b^2] over
// N(M, V) by the sigma points.
void gaussian_rhs(const mcpr_coef &c, int npts, double M, double V, double mbar, double vbar, double S, double C,
                  double &dM, double &dV) {
    double xs[3], ws[3];
    const int K = sigma_points(npts, M, V, xs, ws);
    double ea = 0.0, exa = 0.0, eb2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const double a = drift_at(c, xs[k], mbar, vbar, S, C), b = diffusion_at(c, xs[k], mbar, vbar);
        ea += ws[k] * a;
        exa += ws[k] * (xs[k] - M) * a;
        eb2 += ws[k] * b * b;
    }
    dM = ea;
    dV = 2.0 * exa + eb2;
}

// Trigonometric mean field of a macro state: S = sum_i f_i E_i[sin X], C
// likewise, E_i at the region mean (Taylor model) or by its sigma points.
void trig_field(const mcpr_coef &c, int model, int I, const Macro &r, double &S, double &C) {
    S = C = 0.0;
    if (c.ksin == 0.0 && c.kc == 0.0) return;
    for (int i = 0; i < I; ++i) {
        if (!(r.f[i] > 0.0)) continue;
        if (model == MCPR_COARSE_TAYLOR) {
            S += r.f[i] * std::sin(r.M[i]);
            C += r.f[i] * std::cos(r.M[i]);
        } else {
            double xs[3], ws[3];
            const int K = sigma_points(model == MCPR_COARSE_GAUSS2 ? 2 : 3, r.M[i], r.V[i], xs, ws);
            for (int k = 0; k < K; ++k) {
                S += r.f[i] * ws[k] * std::sin(xs[k]);
                C += r.f[i] * ws[k] * std::cos(xs[k]);
            }
        }
    }
}

void moment_rhs(const mcpr_coef &c, int model, int I, const Macro &r, Macro &d) {
    double mbar, vbar, S, C;
    mixture(I, r, mbar, vbar);
    trig_field(c, model, I, r, S, C);
    if (model != MCPR_COARSE_TAYLOR) {
        for (int i = 0; i < I; ++i) {
            gaussian_rhs(c, model == MCPR_COARSE_GAUSS2 ? 2 : 3, r.M[i], r.V[i], mbar, vbar, S, C, d.M[i], d.V[i]);
            d.f[i] = 0.0;
        }
        return;
    }
    for (int i = 0; i < I; ++i) {
        const double x = r.M[i];
        const double a = drift_at(c, x, mbar, vbar, S, C);
        double ax = c.a1 + x * (2.0 * c.a2 + 3.0 * c.a3 * x) + c.axs * (vbar + mbar * mbar);
        double axx = 2.0 * c.a2 + 6.0 * c.a3 * x;
        if (c.ksin != 0.0 || c.kc != 0.0) {
            const double sx = std::sin(x), cx = std::cos(x);
            ax += c.ksin * cx - c.kc * (S * sx + C * cx);
            axx += -c.ksin * sx - c.kc * (S * cx - C * sx);
        }
        const double b = c.b0 + c.b1 * x + c.bm * mbar + c.bv * vbar;
        const double bx = c.b1;
        d.M[i] = a + 0.5 * axx * r.V[i];
        d.V[i] = (2.0 * ax + bx * bx) * r.V[i] + b * b;
        if (c.acdf != 0.0) {
            // a N(M, V) density: 1 - F is 1/2 at the mean, its slope there
            // -1/sqrt(2 pi V) and its curvature zero
            const double vp = r.V[i] > 0.0 ? r.V[i] : 0.0;
            d.M[i] += 0.5 * c.acdf;
            d.V[i] += -2.0 * c.acdf * std::sqrt(vp) / std::sqrt(2.0 * 3.141592653589793);
        }
        d.f[i] = 0.0;
    }
}

Macro coarse_step(const mcpr_problem &p, const Macro &in) {
    const int I = p.n_regions;
    const double h = (p.dt * p.steps_per_slice) / p.coarse_substeps;
    Macro y = in, k1, k2, k3, k4, tmp;
    for (int s = 0; s < p.coarse_substeps; ++s) {
        moment_rhs(p.coef, p.coarse_model, I, y, k1);
        tmp = y;
        for (int i = 0; i < I; ++i) { tmp.M[i] = y.M[i] + 0.5 * h * k1.M[i]; tmp.V[i] = y.V[i] + 0.5 * h * k1.V[i]; }
        moment_rhs(p.coef, p.coarse_model, I, tmp, k2);
        for (int i = 0; i < I; ++i) { tmp.M[i] = y.M[i] + 0.5 * h * k2.M[i]; tmp.V[i] = y.V[i] + 0.5 * h * k2.V[i]; }
        moment_rhs(p.coef, p.coarse_model, I, tmp, k3);
        for (int i = 0; i < I; ++i) { tmp.M[i] = y.M[i] + h * k3.M[i]; tmp.V[i] = y.V[i] + h * k3.V[i]; }
        moment_rhs(p.coef, p.coarse_model, I, tmp, k4);
        for (int i = 0; i < I; ++i) {
            y.M[i] += (h / 6.0) * (k1.M[i] + 2.0 * k2.M[i] + 2.0 * k3.M[i] + k4.M[i]);
            y.V[i] += (h / 6.0) * (k1.V[i] + 2.0 * k2.V[i] + 2.0 * k3.V[i] + k4.V[i]);
        }
    }
    return y;
}

bool bit_equal(const Macro &a, const Macro &b, int I) {
    return std::memcmp(a.f, b.f, sizeof(double) * I) == 0 && std::memcmp(a.M, b.M, sizeof(double) * I) == 0 &&
           std::memcmp(a.V, b.V, sizeof(double) * I) == 0;
}

Macro macro_of(const RegionStats *st, int I, int64_t P) {
    Macro r;
    std::memset(&r, 0, sizeof r);
    for (int i = 0; i < I; ++i) {
        r.f[i] = (double)st[i].n / (double)P;
        r.M[i] = st[i].mean;
        r.V[i] = st[i].var;
    }
    return r;
}

int region_of(const mcpr_problem &p, double x) {
    int g = 0;
    for (int i = 0; i + 1 < p.n_regions; ++i) g += (x >= p.split[i]) ? 1 : 0;
    return g;
}

// The device's evaluation of an affine map, reproduced on the host.
double mapped(int prec, const RegionMap &mp, double x) {
    const double y = std::fma(mp.scale, x - mp.from, mp.to);
    return prec == MCPR_FP32 ? (double)(float)y : y;
}

// ---- particle-fraction model (two regions): P1(t) = P* + (P1(0) - P*) e^{-kappa t}
double frac_model(double y0, double kappa, double pstar, double t) { return pstar + (y0 - pstar) * std::exp(-kappa * t); }

void fit_fractions(const std::vector<double> &t, const std::vector<double> &y, double &kappa, double &pstar) {
    const int n = (int)t.size();
    auto sse_of = [&](double k, double p) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) {
            const double r = frac_model(y[0], k, p, t[j]) - y[j];
            s += r * r;
        }
        return s;
    };
    double lam = 1e-3, sse = sse_of(kappa, pstar);
    for (int it = 0; it < 200; ++it) {
        double g0 = 0, g1 = 0, h00 = 0, h01 = 0, h11 = 0;
        for (int j = 0; j < n; ++j) {
            const double e = std::exp(-kappa * t[j]);
            const double r = frac_model(y[0], kappa, pstar, t[j]) - y[j];
            const double dk = -(y[0] - pstar) * t[j] * e, dp = 1.0 - e;
            g0 += dk * r; g1 += dp * r; h00 += dk * dk; h01 += dk * dp; h11 += dp * dp;
        }
        bool improved = false, converged = false;
        for (int tries = 0; tries < 40 && !improved; ++tries) {
            const double a00 = h00 * (1.0 + lam), a11 = h11 * (1.0 + lam), det = a00 * a11 - h01 * h01;
            if (!(det > 0.0) || !std::isfinite(det)) { lam *= 10.0; continue; }
            double kn = kappa - (a11 * g0 - h01 * g1) / det, pn = pstar - (a00 * g1 - h01 * g0) / det;
            kn = std::max(kn, 0.0);
            pn = std::min(std::max(pn, 0.0), 1.0);
            const double sn = sse_of(kn, pn);
            if (sn < sse) {
                converged = std::fabs(kn - kappa) + std::fabs(pn - pstar) <= 1e-14 * (std::fabs(kappa) + std::fabs(pstar));
                kappa = kn; pstar = pn; sse = sn;
                lam = std::max(lam / 10.0, 1e-12);
                improved = true;
            } else {
                lam *= 10.0;
            }
        }
        if (!improved || converged) break;
    }
}

struct Instance {
    mcpr_problem pb;
    int32_t inst;
    int64_t P, stride;
    char *ring;
    std::vector<Macro> rho;          // rho^k_n, n = 0..N
    std::vector<Macro> cache;        // C_n(rho^k_n), n = 0..N-1
    std::vector<RegionStats> rec;    // R(F(u^k_{n-1})) at boundary n (n = 1..N), [(N+1)][I+1]
    std::vector<RegionStats> st0;    // R(u0)
    std::vector<int32_t> flags;      // [N][I] of the last iteration
    bool done = false;
    bool have_fit = false;
    double kappa = 0.0, pstar = 0.0;
    std::vector<double> fgiven;      // [(N+1)][I] given fractions (empty: the method's own)
    int k = 0;                       // this instance's iteration count (it stops early at tol)
    std::vector<double> qcache;      // [(N+1)][3] QoI of each slice when it became exact
};

// The given fractions replace those of macro state n (the exact-fraction
// reference variant); the cached coarse outputs keep the fractions they were
// computed with.
void apply_given(const Instance &in, int I, int n, Macro &o) {
    if (in.fgiven.empty()) return;
    for (int r = 0; r < I; ++r) o.f[r] = in.fgiven[(size_t)n * I + r];
}

} // namespace

struct mcpr_parareal {
    mcpr_ctx *ctx;
    int N, m, I, prec;
    int k = 0;
    bool learning;
    double tol;
    size_t esize;
    std::vector<Instance> inst;
    DevBuf dstats, dmaps;
    HostBuf hmaps;                 // pinned source of the matching maps
    hipEvent_t hmaps_done = nullptr; // the last copy out of hmaps has completed
    // QoI of the newest exact slice of each instance, queued at the end of
    // init and iterate when tracking is on, harvested at the next call
    bool track_qoi = false;
    DevBuf dq;
    HostBuf hq;
    hipEvent_t hq_done = nullptr;
    std::vector<std::pair<int, int>> hq_who; // (instance, slice) of each queued entry
};

namespace {

char *slot_ptr(const mcpr_parareal *pr, const Instance &in, int n, int k) {
    const int N = pr->N;
    const int idx = ((n - k) % (N + 1) + (N + 1)) % (N + 1);
    return in.ring + (size_t)idx * in.stride * pr->esize;
}


// Fetch device records [n][I+1] into host memory (synchronises the stream).
mcpr_status fetch(mcpr_parareal *pr, const void *src, size_t count, std::vector<RegionStats> &out, hipStream_t s) {
    mcpr_ctx *ctx = pr->ctx;
    out.resize(count);
    HIP_TRY(hipMemcpyAsync(out.data(), src, count * sizeof(RegionStats), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MCPR_OK;
}

// Move the QoI values queued by the previous call into the instances' caches.
mcpr_status harvest_qoi(mcpr_parareal *pr) {
    if (pr->hq_who.empty()) return MCPR_OK;
    mcpr_ctx *ctx = pr->ctx;
    HIP_TRY(hipEventSynchronize(pr->hq_done));
    const size_t cnt = pr->hq_who.size();
    const double *h = (const double *)pr->hq.p;
    for (size_t j = 0; j < cnt; ++j) {
        Instance &in = pr->inst[pr->hq_who[j].first];
        const int n = pr->hq_who[j].second;
        for (int kind = 0; kind < 3; ++kind) in.qcache[(size_t)n * 3 + kind] = h[kind * cnt + j];
    }
    pr->hq_who.clear();
    return MCPR_OK;
}

// Queue the QoI (every kind) of slot 0, the newest exact slice, of the given
// instances; the values arrive in host memory with the stream.
mcpr_status queue_exact_qoi(mcpr_parareal *pr, const std::vector<int> &insts, mcpr_stream stream) {
    if (!pr->track_qoi || insts.empty()) return MCPR_OK;
    mcpr_ctx *ctx = pr->ctx;
    hipStream_t s = (hipStream_t)stream;
    mcpr_status st;
    if ((st = harvest_qoi(pr)) != MCPR_OK) return st;
    const size_t cnt = insts.size(), bytes = 3 * cnt * sizeof(double);
    std::vector<mcpr_problem> probs(cnt);
    std::vector<mcpr_ensemble> ens(cnt);
    for (size_t j = 0; j < cnt; ++j) {
        Instance &in = pr->inst[insts[j]];
        probs[j] = in.pb;
        ens[j] = mcpr_ensemble{slot_ptr(pr, in, in.k, in.k), in.P, in.inst, in.k, (int)j, 0};
        pr->hq_who.emplace_back(insts[j], in.k);
    }
    if ((st = ensure(ctx, pr->dq, bytes)) != MCPR_OK) return st;
    if ((st = ensure_host(ctx, pr->hq, bytes)) != MCPR_OK) return st;
    for (int kind = 0; kind < 3; ++kind)
        if ((st = mcpr_qoi(ctx, probs.data(), (int)cnt, ens.data(), (int)cnt, kind, (double *)pr->dq.p + kind * cnt,
                           stream)) != MCPR_OK)
            return st;
    HIP_TRY(hipMemcpyAsync(pr->hq.p, pr->dq.p, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(pr->hq_done, s));
    return MCPR_OK;
}

} // namespace

extern "C" {

mcpr_status mcpr_parareal_create(mcpr_ctx *ctx, const mcpr_problem *problems, int32_t n_problems,
                                 const mcpr_instance *inst, int32_t n_inst, int32_t learning, double tol,
                                 mcpr_parareal **out) {
    if (!ctx || !out) return MCPR_E_INVALID_ARG;
    *out = nullptr;
    if (!problems || n_problems < 1 || !inst || n_inst < 1) return fail(ctx, MCPR_E_INVALID_ARG, "empty driver");
    for (int i = 0; i < n_problems; ++i) {
        mcpr_status st = check_problem(ctx, problems[i], i);
        if (st != MCPR_OK) return st;
    }
    const mcpr_problem &p0 = problems[inst[0].problem >= 0 && inst[0].problem < n_problems ? inst[0].problem : 0];
    for (int i = 0; i < n_inst; ++i) {
        const mcpr_instance &I = inst[i];
        if (I.problem < 0 || I.problem >= n_problems) return fail(ctx, MCPR_E_INVALID_ARG, "instance %d: problem", i);
        const mcpr_problem &p = problems[I.problem];
        if (!same_layout(p, p0) || p.n_slices != p0.n_slices)
            return fail(ctx, MCPR_E_INVALID_ARG, "instance %d: layout differs from instance 0", i);
        if (!I.ring || ((uintptr_t)I.ring & 15)) return fail(ctx, MCPR_E_INVALID_ARG, "instance %d: ring pointer", i);
        if (I.n_particles < 1 || I.slot_stride < I.n_particles || (I.slot_stride & 3))
            return fail(ctx, MCPR_E_INVALID_ARG, "instance %d: n_particles / slot_stride", i);
        if (I.instance < 0) return fail(ctx, MCPR_E_INVALID_ARG, "instance %d: RNG stream", i);
    }
    if (learning && p0.n_regions != 2) return fail(ctx, MCPR_E_UNSUPPORTED, "learning needs two regions");
    if (!(tol >= 0.0)) return fail(ctx, MCPR_E_INVALID_ARG, "tol must be >= 0");
    mcpr_parareal *pr = new mcpr_parareal();
    pr->ctx = ctx;
    pr->N = p0.n_slices;
    pr->m = p0.steps_per_slice;
    pr->I = p0.n_regions;
    pr->prec = p0.precision;
    pr->learning = learning != 0;
    pr->tol = tol;
    pr->esize = pr->prec == MCPR_FP64 ? 8 : 4;
    pr->inst.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        in.pb = problems[inst[i].problem];
        in.inst = inst[i].instance;
        in.P = inst[i].n_particles;
        in.stride = inst[i].slot_stride;
        in.ring = (char *)inst[i].ring;
        in.rho.resize(pr->N + 1);
        in.cache.resize(pr->N);
        in.rec.resize((size_t)(pr->N + 1) * (pr->I + 1));
        in.flags.assign((size_t)pr->N * pr->I, 0);
        in.qcache.assign((size_t)(pr->N + 1) * 3, 0.0);
    }
    // Every buffer of init, iterate and qoi is sized here, for the largest
    // batch they use (every slot of every instance: the lifting writes slices
    // 1..N, the first iteration propagates slices 0..N-1, the QoI of one
    // instance reads slices k..N), so those calls allocate nothing.
    mcpr_status st = MCPR_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) st = fail(ctx, MCPR_E_DEVICE, "hipSetDevice(%d) failed", ctx->device);
    if (st == MCPR_OK) {
        Growing grow(ctx);
        const int N = pr->N, I = pr->I;
        std::vector<mcpr_problem> probs(n_inst);
        std::vector<mcpr_ensemble> all;
        for (int i = 0; i < n_inst; ++i) {
            const Instance &in = pr->inst[i];
            probs[i] = in.pb;
            for (int n = 0; n <= N; ++n)
                all.push_back(mcpr_ensemble{in.ring + (size_t)n * in.stride * pr->esize, in.P, in.inst, n, i, 0});
        }
        Tables t;
        build_tables(probs.data(), all.data(), (int)all.size(), t);
        const size_t nmaps = all.size() * I * sizeof(RegionMap);
        const size_t nstats = std::max(all.size() * (I + 1) * sizeof(RegionStats), (size_t)(N + 1) * sizeof(double));
        const size_t nq = 3 * (size_t)n_inst * sizeof(double);
        const int32_t calls = MCPR_RESERVE_INIT | MCPR_RESERVE_MOMENTS | MCPR_RESERVE_QOI | MCPR_RESERVE_FINE |
                              MCPR_RESERVE_MATCH;
        if ((st = size_calls(ctx, t, probs.data(), all.data(), calls, nmaps)) == MCPR_OK &&
            (st = ensure(ctx, pr->dstats, nstats)) == MCPR_OK && (st = ensure(ctx, pr->dmaps, nmaps)) == MCPR_OK &&
            (st = ensure_host(ctx, pr->hmaps, nmaps)) == MCPR_OK && (st = ensure(ctx, pr->dq, nq)) == MCPR_OK &&
            (st = ensure_host(ctx, pr->hq, nq)) == MCPR_OK) {
            if (hipEventCreateWithFlags(&pr->hmaps_done, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&pr->hq_done, hipEventDisableTiming) != hipSuccess)
                st = fail(ctx, MCPR_E_DEVICE, "event creation failed");
        }
    }
    if (st != MCPR_OK) {
        mcpr_parareal_destroy(pr);
        return st;
    }
    *out = pr;
    return MCPR_OK;
}

void mcpr_parareal_destroy(mcpr_parareal *pr) {
    if (!pr) return;
    (void)hipDeviceSynchronize();
    if (pr->dstats.p) (void)hipFree(pr->dstats.p);
    if (pr->dmaps.p) (void)hipFree(pr->dmaps.p);
    if (pr->hmaps.p) (void)hipHostFree(pr->hmaps.p);
    if (pr->hmaps_done) (void)hipEventDestroy(pr->hmaps_done);
    if (pr->dq.p) (void)hipFree(pr->dq.p);
    if (pr->hq.p) (void)hipHostFree(pr->hq.p);
    if (pr->hq_done) (void)hipEventDestroy(pr->hq_done);
    delete pr;
}

int32_t mcpr_parareal_iteration(const mcpr_parareal *pr) { return pr ? pr->k : -1; }

mcpr_status mcpr_parareal_init(mcpr_parareal *pr, int32_t sample_u0, mcpr_stream stream) {
    if (!pr) return MCPR_E_INVALID_ARG;
    mcpr_ctx *ctx = pr->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int N = pr->N, I = pr->I, n_inst = (int)pr->inst.size();
    std::vector<mcpr_problem> probs(n_inst);
    std::vector<mcpr_ensemble> ens(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        probs[i] = in.pb;
        ens[i] = mcpr_ensemble{in.ring, in.P, in.inst, 0, i, 0};
    }
    mcpr_status st;
    if (sample_u0 && (st = mcpr_init_particles(ctx, probs.data(), n_inst, ens.data(), n_inst, stream)) != MCPR_OK)
        return st;
    if ((st = ensure(ctx, pr->dstats, (size_t)n_inst * N * (I + 1) * sizeof(RegionStats))) != MCPR_OK) return st;
    if ((st = mcpr_moments(ctx, probs.data(), n_inst, ens.data(), n_inst, (mcpr_region_stats *)pr->dstats.p, stream)) !=
        MCPR_OK)
        return st;
    std::vector<RegionStats> h;
    if ((st = fetch(pr, pr->dstats.p, (size_t)n_inst * (I + 1), h, s)) != MCPR_OK) return st;

    // coarse sweep and the lifting maps u^0_n = T(rho^0_n, u0), n = 1..N
    std::vector<mcpr_ensemble> lens;
    std::vector<mcpr_problem> lprobs;
    std::vector<RegionMap> maps;
    std::vector<const void *> lsrc;
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        in.done = false;
        in.k = 0;
        in.have_fit = false;
        in.st0.assign(h.begin() + (size_t)i * (I + 1), h.begin() + (size_t)(i + 1) * (I + 1));
        for (const RegionStats &r : in.st0)
            if (r.nonfinite) return fail(ctx, MCPR_E_NONFINITE, "instance %d: non-finite initial particles", i);
        in.rho[0] = macro_of(in.st0.data(), I, in.P);
        apply_given(in, I, 0, in.rho[0]);
        for (int n = 0; n < N; ++n) {
            in.rho[n + 1] = coarse_step(in.pb, in.rho[n]);
            in.cache[n] = in.rho[n + 1];
            apply_given(in, I, n + 1, in.rho[n + 1]);
        }
        std::fill(in.flags.begin(), in.flags.end(), 0);
        for (int n = 1; n <= N; ++n) {
            char *dst = in.ring + (size_t)n * in.stride * pr->esize;
            lsrc.push_back(in.ring);
            lprobs.push_back(in.pb);
            lens.push_back(mcpr_ensemble{dst, in.P, in.inst, n, (int)lprobs.size() - 1, 0});
            for (int r = 0; r < I; ++r) {
                RegionMap mp{0.0, 0.0, 0.0, MCPR_MAP_KEEP, n};
                const RegionStats &src = in.st0[r];
                const double mu = in.rho[n].M[r], sig = in.rho[n].V[r];
                if (src.n > 0 && sig >= 0.0 && std::isfinite(sig) && std::isfinite(mu)) {
                    if (src.min == src.max) {
                        mp.mode = MCPR_MAP_RESAMPLE;
                        mp.scale = std::sqrt(sig);
                        mp.to = mu;
                    } else {
                        mp.mode = MCPR_MAP_AFFINE;
                        mp.from = src.mean;
                        mp.scale = std::sqrt(sig / src.var);
                        mp.to = mu;
                    }
                }
                maps.push_back(mp);
            }
        }
    }
    if (!lens.empty()) {
        // one launch writes every lifted slot from u0 (slot 0 of its instance)
        Tables t;
        build_tables(lprobs.data(), lens.data(), (int)lens.size(), t);
        for (size_t e = 0; e < lens.size(); ++e) t.items[e].src = lsrc[e];
        if ((st = upload(ctx, t, maps.data(), maps.size() * sizeof(RegionMap), s)) != MCPR_OK) return st;
        HIP_TRY(mcpr::launch_match_apply(pr->prec, I, ctx->items, ctx->blocks,
                                         (int)t.blocks.size(), splits_of(pr->inst[0].pb),
                                         ctx->maps, s));
    }
    // no final synchronisation: the lifting is ordered on the stream, and the
    // host has already taken everything it needs
    pr->k = 0;
    pr->hq_who.clear();
    std::vector<int> all(n_inst);
    for (int i = 0; i < n_inst; ++i) all[i] = i;
    return queue_exact_qoi(pr, all, stream);
}

mcpr_status mcpr_parareal_iterate(mcpr_parareal *pr, double *delta_out, mcpr_stream stream) {
    if (!pr) return MCPR_E_INVALID_ARG;
    mcpr_ctx *ctx = pr->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int N = pr->N, I = pr->I, k = pr->k, n_inst = (int)pr->inst.size();

    // 1. fine propagator on every active slice of every running instance
    std::vector<mcpr_problem> probs;
    std::vector<mcpr_ensemble> ens;
    std::vector<std::pair<int, int>> who; // (instance, slice) of each ensemble
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        if (delta_out) delta_out[i] = 0.0;
        if (in.done || k >= N) continue;
        probs.push_back(in.pb);
        for (int n = k; n < N; ++n) {
            ens.push_back(mcpr_ensemble{slot_ptr(pr, in, n, in.k), in.P, in.inst, n, (int)probs.size() - 1, 0});
            who.emplace_back(i, n);
        }
    }
    if (ens.empty()) return MCPR_OK;
    mcpr_status st;
    if ((st = ensure(ctx, pr->dstats, ens.size() * (I + 1) * sizeof(RegionStats))) != MCPR_OK) return st;
    // (the records stay in the context's buffer and come to the host from there)
    if ((st = fine_propagate(ctx, probs.data(), (int)probs.size(), ens.data(), (int)ens.size(), true, nullptr,
                             nullptr, s)) != MCPR_OK)
        return st;
    std::vector<RegionStats> h;
    if ((st = fetch(pr, ctx->recs.p, ens.size() * (I + 1), h, s)) != MCPR_OK) return st;
    for (size_t e = 0; e < ens.size(); ++e) {
        Instance &in = pr->inst[who[e].first];
        const int n = who[e].second;
        std::memcpy(&in.rec[(size_t)(n + 1) * (I + 1)], &h[e * (I + 1)], sizeof(RegionStats) * (I + 1));
        for (int r = 0; r <= I; ++r)
            if (h[e * (I + 1) + r].nonfinite)
                return fail(ctx, MCPR_E_NONFINITE, "instance %d slice %d: non-finite particles", who[e].first, n);
    }

    // 2. per instance: learning fit, then the sequential coarse sweep with the iterator
    std::vector<RegionMap> maps(ens.size() * I);
    std::vector<char> touched(ens.size(), 0);
    size_t ebase = 0;
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        if (in.done || k >= N) continue;
        const mcpr_problem &p = in.pb;
        const double dT = p.dt * p.steps_per_slice;

        // particle-fraction model fitted to the exact slices 0..k+1 (Sec. 3.6)
        std::vector<double> phat(N + 1, -1.0);
        if (pr->learning) {
            std::vector<double> tt, yy;
            for (int n = 0; n <= k + 1 && n <= N; ++n) {
                tt.push_back(n * dT);
                yy.push_back(n == 0 ? (double)in.st0[0].n / (double)in.P
                                    : (double)in.rec[(size_t)n * (I + 1)].n / (double)in.P);
            }
            if (tt.size() >= 3) {
                double kap = in.have_fit ? in.kappa : 1.0 / (N * dT);
                double pst = in.have_fit ? in.pstar : yy.back();
                fit_fractions(tt, yy, kap, pst);
                in.kappa = kap;
                in.pstar = pst;
                in.have_fit = true;
            }
            if (in.have_fit) {
                const double tk = (k + 1) * dT, yk = yy.back();
                for (int n = k + 2; n <= N; ++n) phat[n] = frac_model(yk, in.kappa, in.pstar, n * dT - tk);
            }
        }

        std::vector<Macro> nrho(N + 1), ncache(N);
        nrho[0] = in.rho[0];
        for (int n = 0; n < N; ++n) {
            const Macro a = coarse_step(p, nrho[n]);
            const Macro &c = in.cache[n];
            ncache[n] = a;
            const RegionStats *b = &in.rec[(size_t)(n + 1) * (I + 1)];
            int32_t *fl = &in.flags[(size_t)n * I];
            Macro &o = nrho[n + 1];
            // I(a, b, a) = (R(b), b).  Slices below k and their successors are
            // exact, so their coarse inputs agree bit for bit; n < k can only
            // take this branch.
            if (bit_equal(a, c, I) || n < k) {
                o = macro_of(b, I, in.P);
                for (int r = 0; r < I; ++r) fl[r] = 0;
                apply_given(in, I, n + 1, o);
                continue;
            }
            const size_t e = ebase + (size_t)(n - k); // this slice's ensemble (n >= k here)
            std::memset(&o, 0, sizeof o);
            for (int r = 0; r < I; ++r) {
                RegionMap &mp = maps[e * I + r];
                mp = RegionMap{0.0, 0.0, 0.0, MCPR_MAP_KEEP, n + 1};
                const double fr = (double)b[r].n / (double)in.P;
                if (b[r].n == 0) {
                    o.f[r] = 0.0; o.M[r] = a.M[r]; o.V[r] = a.V[r];
                    fl[r] = 4;
                    continue;
                }
                const double alM = (a.M[r] - c.M[r]) + b[r].mean;
                const double alV = (a.V[r] - c.V[r]) + b[r].var;
                if (!(alV >= 0.0) || !std::isfinite(alV) || !std::isfinite(alM)) {
                    o.f[r] = fr; o.M[r] = b[r].mean; o.V[r] = b[r].var;
                    fl[r] = 2;
                    continue;
                }
                RegionMap cand{0.0, 0.0, alM, MCPR_MAP_AFFINE, n + 1};
                bool inside = true;
                if (b[r].min == b[r].max) {
                    cand.mode = MCPR_MAP_RESAMPLE;
                    cand.scale = std::sqrt(alV);
                    if (I > 1) {
                        // the resampled particles: check them on the device
                        std::vector<RegionMap> pm(I, RegionMap{0.0, 0.0, 0.0, MCPR_MAP_KEEP, n + 1});
                        pm[r] = cand;
                        if ((st = ensure(ctx, pr->dmaps, I * sizeof(RegionMap))) != MCPR_OK) return st;
                        HIP_TRY(hipMemcpyAsync(pr->dmaps.p, pm.data(), I * sizeof(RegionMap), hipMemcpyHostToDevice, s));
                        mcpr_problem one = p;
                        mcpr_ensemble oe = ens[e];
                        oe.problem = 0;
                        if ((st = mcpr_match(ctx, &one, 1, &oe, 1, (const mcpr_region_map *)pr->dmaps.p, 1,
                                             (mcpr_region_stats *)pr->dstats.p, stream)) != MCPR_OK)
                            return st;
                        std::vector<RegionStats> pr_h;
                        if ((st = fetch(pr, pr->dstats.p, (size_t)(I + 1), pr_h, s)) != MCPR_OK) return st;
                        inside = region_of(p, pr_h[r].min) == r && region_of(p, pr_h[r].max) == r;
                    }
                } else {
                    cand.from = b[r].mean;
                    cand.scale = std::sqrt(alV / b[r].var);
                    if (I > 1)
                        inside = region_of(p, mapped(pr->prec, cand, b[r].min)) == r &&
                                 region_of(p, mapped(pr->prec, cand, b[r].max)) == r;
                }
                if (!inside) {
                    o.f[r] = fr; o.M[r] = b[r].mean; o.V[r] = b[r].var;
                    fl[r] = 3;
                    continue;
                }
                mp = cand;
                touched[e] = 1;
                o.f[r] = fr; o.M[r] = alM; o.V[r] = alV;
                fl[r] = 1;
            }
            if (phat[n + 1] >= 0.0) {
                o.f[0] = phat[n + 1];
                o.f[1] = 1.0 - phat[n + 1];
            }
            apply_given(in, I, n + 1, o);
        }

        // successive-iterate difference of the global moments
        double d = 0.0;
        for (int n = 1; n <= N; ++n) {
            double M0, V0, M1, V1;
            mixture(I, in.rho[n], M0, V0);
            mixture(I, nrho[n], M1, V1);
            d = std::max(d, std::max(std::fabs(M1 - M0), std::fabs(V1 - V0)));
        }
        if (delta_out) delta_out[i] = d;
        in.rho = nrho;
        in.cache = ncache;
        if (d <= pr->tol || k + 1 >= N) in.done = true;
        ebase += (size_t)(N - k);
    }

    // 3. matching on the device, only ensembles with a moved region
    std::vector<mcpr_ensemble> mens;
    std::vector<RegionMap> mmaps;
    for (size_t e = 0; e < ens.size(); ++e)
        if (touched[e]) {
            mens.push_back(ens[e]);
            mmaps.insert(mmaps.end(), maps.begin() + e * I, maps.begin() + (e + 1) * I);
        }
    if (!mens.empty()) {
        const size_t mb = mmaps.size() * sizeof(RegionMap);
        if ((st = ensure(ctx, pr->dmaps, mb)) != MCPR_OK) return st;
        // through a pinned buffer, so that the call can return before the copy ends
        if ((st = ensure_host(ctx, pr->hmaps, mb)) != MCPR_OK) return st;
        HIP_TRY(hipEventSynchronize(pr->hmaps_done));
        std::memcpy(pr->hmaps.p, mmaps.data(), mb);
        HIP_TRY(hipMemcpyAsync(pr->dmaps.p, pr->hmaps.p, mb, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(pr->hmaps_done, s));
        if ((st = mcpr_match(ctx, probs.data(), (int)probs.size(), mens.data(), (int)mens.size(),
                             (const mcpr_region_map *)pr->dmaps.p, 0, nullptr, stream)) != MCPR_OK)
            return st;
    }
    // no final synchronisation: the matching is ordered on the stream
    pr->k = k + 1;
    std::vector<int> moved;
    for (int i = 0; i < n_inst; ++i) {
        Instance &in = pr->inst[i];
        if (in.k == k && k < N) { // propagated in this call
            in.k = k + 1;
            moved.push_back(i);
        }
    }
    return queue_exact_qoi(pr, moved, stream);
}

mcpr_status mcpr_parareal_qoi(mcpr_parareal *pr, int32_t inst, int32_t kind, double *out, mcpr_stream stream) {
    if (!pr) return MCPR_E_INVALID_ARG;
    mcpr_ctx *ctx = pr->ctx;
    if (inst < 0 || inst >= (int)pr->inst.size()) return fail(ctx, MCPR_E_INVALID_ARG, "instance %d", inst);
    if (!out) return fail(ctx, MCPR_E_INVALID_ARG, "out is null");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (kind < MCPR_QOI_X || kind > MCPR_QOI_SIN_X2) return fail(ctx, MCPR_E_INVALID_ARG, "QoI kind %d", kind);
    const Instance &in = pr->inst[inst];
    const int N = pr->N, k0 = in.k;
    if (k0 > 0 && !pr->track_qoi)
        return fail(ctx, MCPR_E_INVALID_ARG, "slices below k are no longer held: enable QoI tracking before init");
    mcpr_status st;
    if ((st = harvest_qoi(pr)) != MCPR_OK) return st;
    for (int n = 0; n < k0; ++n) out[n] = in.qcache[(size_t)n * 3 + kind];
    // slices k..N are in the ring
    std::vector<mcpr_ensemble> ens(N + 1 - k0);
    for (int n = k0; n <= N; ++n) ens[n - k0] = mcpr_ensemble{slot_ptr(pr, in, n, k0), in.P, in.inst, n, 0, 0};
    if ((st = ensure(ctx, pr->dstats, (size_t)(N + 1) * sizeof(double))) != MCPR_OK) return st;
    if ((st = mcpr_qoi(ctx, &in.pb, 1, ens.data(), N + 1 - k0, kind, (double *)pr->dstats.p, stream)) != MCPR_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(out + k0, pr->dstats.p, (size_t)(N + 1 - k0) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MCPR_OK;
}

mcpr_status mcpr_parareal_track_qoi(mcpr_parareal *pr, int32_t on) {
    if (!pr) return MCPR_E_INVALID_ARG;
    pr->track_qoi = on != 0;
    return MCPR_OK;
}

mcpr_status mcpr_parareal_set_fractions(mcpr_parareal *pr, int32_t inst, const double *fractions) {
    if (!pr) return MCPR_E_INVALID_ARG;
    if (inst < 0 || inst >= (int)pr->inst.size()) return fail(pr->ctx, MCPR_E_INVALID_ARG, "instance %d", inst);
    Instance &in = pr->inst[inst];
    if (!fractions) {
        in.fgiven.clear();
        return MCPR_OK;
    }
    const size_t n = (size_t)(pr->N + 1) * pr->I;
    for (size_t j = 0; j < n; ++j)
        if (!(fractions[j] >= 0.0) || !std::isfinite(fractions[j]))
            return fail(pr->ctx, MCPR_E_INVALID_ARG, "fraction %zu is negative or not finite", j);
    in.fgiven.assign(fractions, fractions + n);
    return MCPR_OK;
}

} // extern "C"

// ---- checkpoint and resume of the driver's host state ----------------------
namespace {

constexpr char kStateMagic[8] = {'M', 'C', 'P', 'R', 'S', 'T', '0', '1'};

// Appends (or, reading, takes) plain values and arrays in a fixed order.
struct Blob {
    char *out = nullptr;       // writing: destination (NULL: count only)
    const char *in = nullptr;  // reading: source
    size_t pos = 0, cap = 0;
    bool ok = true;
    void raw(void *p, size_t n) {
        if (in) {
            if (pos + n > cap) {
                ok = false;
                return;
            }
            std::memcpy(p, in + pos, n);
        } else if (out) {
            std::memcpy(out + pos, p, n);
        }
        pos += n;
    }
    template <typename T> void val(T &v) { raw(&v, sizeof v); }
    template <typename T> void vec(std::vector<T> &v) {
        uint64_t n = v.size();
        val(n);
        if (in) {
            if (!ok || n > (cap - pos) / std::max<size_t>(sizeof(T), 1)) {
                ok = false;
                return;
            }
            v.resize(n);
        }
        if (n) raw(v.data(), n * sizeof(T));
    }
};

// The driver's host state in a fixed order: a header that identifies the
// driver's shape, then per instance its iteration count, stop flag, fraction
// fit, macro states, cached coarse outputs, records, iterator flags, QoI of
// the exact slices and given fractions.
void state_fields(mcpr_parareal *pr, Blob &b) {
    char magic[8];
    std::memcpy(magic, kStateMagic, 8);
    b.raw(magic, 8);
    if (b.in && std::memcmp(magic, kStateMagic, 8) != 0) b.ok = false;
    int32_t shape[5] = {pr->N, pr->m, pr->I, pr->prec, (int32_t)pr->inst.size()};
    int32_t got[5];
    std::memcpy(got, shape, sizeof shape);
    b.raw(got, sizeof got);
    if (b.in && std::memcmp(got, shape, sizeof shape) != 0) b.ok = false;
    int32_t k = pr->k;
    b.val(k);
    for (Instance &in : pr->inst) {
        int64_t id[2] = {in.P, in.inst};
        int64_t gid[2] = {id[0], id[1]};
        b.raw(gid, sizeof gid);
        if (b.in && (gid[0] != id[0] || gid[1] != id[1])) b.ok = false;
        int32_t flags3[3] = {in.k, in.done ? 1 : 0, in.have_fit ? 1 : 0};
        b.raw(flags3, sizeof flags3);
        double fit[2] = {in.kappa, in.pstar};
        b.raw(fit, sizeof fit);
        b.vec(in.rho);
        b.vec(in.cache);
        b.vec(in.rec);
        b.vec(in.st0);
        b.vec(in.flags);
        b.vec(in.qcache);
        b.vec(in.fgiven);
        if (b.in && b.ok) {
            in.k = flags3[0];
            in.done = flags3[1] != 0;
            in.have_fit = flags3[2] != 0;
            in.kappa = fit[0];
            in.pstar = fit[1];
        }
    }
    if (b.in && b.ok) pr->k = k;
}

} // namespace

extern "C" {

mcpr_status mcpr_parareal_save(mcpr_parareal *pr, void *buf, size_t capacity, size_t *bytes) {
    if (!pr || !bytes) return MCPR_E_INVALID_ARG;
    mcpr_ctx *ctx = pr->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    mcpr_status st;
    if ((st = harvest_qoi(pr)) != MCPR_OK) return st; // the QoI still in flight belongs to the state
    Blob count;
    state_fields(pr, count);
    *bytes = count.pos;
    if (!buf) return MCPR_OK;
    if (capacity < count.pos) return fail(ctx, MCPR_E_INVALID_ARG, "state needs %zu bytes, %zu given", count.pos, capacity);
    Blob w;
    w.out = (char *)buf;
    state_fields(pr, w);
    return MCPR_OK;
}

mcpr_status mcpr_parareal_restore(mcpr_parareal *pr, const void *buf, size_t bytes) {
    if (!pr || !buf) return MCPR_E_INVALID_ARG;
    mcpr_ctx *ctx = pr->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    mcpr_status st;
    if ((st = harvest_qoi(pr)) != MCPR_OK) return st;
    // read into a copy first, so that a bad blob leaves the driver as it was
    std::vector<Instance> keep = pr->inst;
    const int k_keep = pr->k;
    Blob r;
    r.in = (const char *)buf;
    r.cap = bytes;
    state_fields(pr, r);
    const size_t N = pr->N, I = pr->I;
    for (const Instance &in : pr->inst)
        if (in.rho.size() != N + 1 || in.cache.size() != N || in.rec.size() != (N + 1) * (I + 1) ||
            in.st0.size() != (in.k > 0 || !in.st0.empty() ? I + 1 : 0) || in.flags.size() != N * I ||
            in.qcache.size() != (N + 1) * 3 || (!in.fgiven.empty() && in.fgiven.size() != (N + 1) * I) ||
            in.k < 0 || in.k > (int)N)
            r.ok = false;
    if (!r.ok || r.pos != bytes) {
        pr->inst = keep;
        pr->k = k_keep;
        return fail(ctx, MCPR_E_INVALID_ARG, "not a state of this driver (shape, particle counts or length differ)");
    }
    return MCPR_OK;
}

mcpr_status mcpr_parareal_macro(const mcpr_parareal *pr, int32_t inst, double *rho, double *glob) {
    if (!pr || inst < 0 || inst >= (int)pr->inst.size()) return MCPR_E_INVALID_ARG;
    const Instance &in = pr->inst[inst];
    for (int n = 0; n <= pr->N; ++n) {
        if (rho)
            for (int r = 0; r < pr->I; ++r) {
                rho[((size_t)n * pr->I + r) * 3 + 0] = in.rho[n].f[r];
                rho[((size_t)n * pr->I + r) * 3 + 1] = in.rho[n].M[r];
                rho[((size_t)n * pr->I + r) * 3 + 2] = in.rho[n].V[r];
            }
        if (glob) mixture(pr->I, in.rho[n], glob[2 * n], glob[2 * n + 1]);
    }
    return MCPR_OK;
}

mcpr_status mcpr_parareal_flags(const mcpr_parareal *pr, int32_t inst, int32_t *flags) {
    if (!pr || !flags || inst < 0 || inst >= (int)pr->inst.size()) return MCPR_E_INVALID_ARG;
    std::memcpy(flags, pr->inst[inst].flags.data(), pr->inst[inst].flags.size() * sizeof(int32_t));
    return MCPR_OK;
}

mcpr_status mcpr_parareal_slot(const mcpr_parareal *pr, int32_t inst, int32_t n, void **x) {
    if (!pr || !x || inst < 0 || inst >= (int)pr->inst.size() || n < 0 || n > pr->N) return MCPR_E_INVALID_ARG;
    const Instance &in = pr->inst[inst];
    if (n < in.k) return fail(pr->ctx, MCPR_E_INVALID_ARG, "slice %d is below the iteration count %d: not held", n, in.k);
    *x = slot_ptr(pr, in, n, in.k);
    return MCPR_OK;
}

} // extern "C"
