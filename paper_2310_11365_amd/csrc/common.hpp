// common.hpp -- internal types shared by the host library and its kernels.
//
// Canonical reduction order (every sum the library forms over particles):
//   quad      particles 4q..4q+3:  ((d0 + d1) + (d2 + d3)), absent particles add +0.0
//   thread    a superchunk is 256 threads x R quads; thread t owns quads
//             Q = sc*256*R + r*256 + t, r = 0..R-1, and adds them in r order
//   block     pairwise tree over the 256 thread sums (xor butterfly in each
//             64-lane wave, then (w0 + w1) + (w2 + w3))
//   ensemble  thread t adds the superchunk sums s = t, t+256, ... in order,
//             then the same 256-thread tree.
// R depends on the particle count only (canonical_quads_per_thread), so the
// result is a function of the ensemble alone: independent of batching, of the
// launch shape and of the other ensembles in the call.  This is what lets a
// Parareal iteration reproduce the serial run bit for bit.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace mcpr {

constexpr int kThreads = 256;        // threads per block; fixed by the canonical tree
constexpr int kQuadsPerChunk = kThreads; // quads per thread-row of a superchunk
constexpr int kMaxRegions = 8;

// Quads per thread R of a superchunk: 1 below 65536 particles (at most 64
// superchunks; short blocks suit small ensembles, whose launches are latency
// bound), else 4 (1024 quads, 16 KB of fp32 state per superchunk; every
// kernel issues a thread's four 16-byte loads before using them).  Measured
// on MI355X over ensembles of 1e4 to 1.6e7 particles, four quads per thread
// stream HBM better than shorter or longer superchunks; large ensembles simply
// have many superchunks, whose partials the step kernel's separate-combine
// variant reduces once per step.
constexpr int kMaxQuadsPerThread = 4;
// Resident fine sweep (an ensemble held in one block's registers through all
// the steps of a sweep): at most kResidentMaxSc superchunks of one quad per
// thread, i.e. 12288 particles (the fp64 sweep keeps a step's state and the
// next step's normals in registers without spilling).
constexpr int kResidentMaxSc = 12;
constexpr int64_t kResidentMaxP = (int64_t)kResidentMaxSc * kThreads * 4;
constexpr int64_t kSmallEnsemble = 65536;
inline int canonical_quads_per_thread(int64_t P) { return P < kSmallEnsemble ? 1 : kMaxQuadsPerThread; }

inline int64_t superchunks(int64_t P, int R) {
    int64_t quads = (P + 3) / 4;
    return (quads + (int64_t)kThreads * R - 1) / ((int64_t)kThreads * R);
}

// One ensemble of a launch.
struct WorkItem {
    void *x;
    int64_t P;
    int32_t inst;
    int32_t step0;     // global step index of step 0 of this call (slice * m)
    int32_t nsc;       // superchunks
    int32_t R;         // quads per thread per superchunk
    int32_t part_off;  // first superchunk partial of this item
    int32_t p0_kind;   // initial law (sampling only)
    uint32_t key0, key1; // Philox key: seed low and high words
    int32_t wrap;      // 1: shift modulo 2 pi into [0, 2 pi) after every step
    int32_t trig;      // 1: trigonometric drift terms; the step's mean field is (mean sin, mean cos)
    int32_t cdf;       // 1: empirical-CDF drift term (every step ranks the ensemble)
    int32_t nbk;       // empirical-CDF drift: buckets of this item (ceil(P / kCdfBucket))
    int32_t bbase;     // its first bucket in the launch's bucket tables
    int32_t pad;
    int64_t doff;      // first position of this item in the launch's dense sort arrays
    double c[14];      // a0 a1 a2 a3 am av b0 b1 bm bv axs ksin kc acdf
    double dt, sdt;    // step and its square root
    double p0[5];      // w, mu1, sd1, mu2, sd2
    int64_t traj;      // 0: steps work in place; else step j reads x + j*traj and writes x + (j+1)*traj
    const void *src;   // matching only: read from src instead of x (NULL: in place)
    int64_t zoff;      // resident sweep: first normal of this item in the sweep's normal buffer
};

// Per-superchunk region partial: count, sum d, sum d^2, min, max (d = x - shift).
struct RegionPartial {
    double cnt, s1, s2, mn, mx;
};

// Device-side record; layout identical to mcpr_region_stats.
struct RegionStats {
    int64_t n;
    double mean, var, min, max;
    int32_t nonfinite;
    int32_t reserved;
};

struct RegionMap {
    double from, scale, to;
    int32_t mode;
    int32_t boundary;
};

// Scalars of one backward (adjoint) step s.
struct AdjStep {
    double m, v;      // moments step s used
    double dm, dv;    // direct term at X_s: dm + dv (X_s - mdir)  (zero if none)
    double mdir;
    int32_t step;     // global step index s
    int32_t zprev;    // 1: form sum lambda_s z_{s-1} for the next launch
    int32_t grad;     // 1: accumulate the parameter gradient of step s
    int32_t pad;
};

// Where the scalars of a backward step live on the device, so that a whole
// adjoint can be replayed from a graph while they change from call to call:
// the step's traced moments (m_s, v_s) (NULL: none, the initial step), and
// for a step at a slice end the upstream derivatives dL/d(m, v) of that end
// (NULL: no direct term) and its traced (mean, variance).  The step's
// AdjStep follows as dm = dl[0] invP, dv = 2 dl[1] invP, mdir = end->x.
struct AdjRef {
    const double2 *mv;
    const double *dl;
    const double2 *end;
    double invP;
    int32_t step;
    int32_t zprev;
    int32_t grad;
    int32_t pad;
};

struct Splits {
    double s[kMaxRegions - 1];
};

} // namespace mcpr
