// launch.hpp -- host-side launchers of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace mcpr {

// prec: 0 = fp64 particles, 1 = fp32 particles (fp64 reductions either way)
hipError_t launch_sum_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, double2 *part_out,
                           double *shift_out, hipStream_t s);
// deg: 1 if every ensemble of the launch has a2 = a3 = 0 (drift affine in x), else 3.
// variant (bitwise-equivalent launch shapes): bit 0 non-temporal state access,
// bit 1 mean field combined by one block per item (into mv, n_items entries)
// instead of by every block.
hipError_t launch_em_step(int prec, int deg, int variant, const WorkItem *items, int n_items, const int2 *blocks,
                          int nblocks, int j, const double2 *part_in, const double *shift_in, double2 *mv,
                          double2 *part_out, double *shift_out, double2 *trace, int m, hipStream_t s);
// trace entry m of each item: moments of its final state from the last step's partials
// Resident fine sweep of every item (each at most kResidentMaxP particles, in
// place): the normals of all m steps into z (the items' zoff), then one
// block per item through all the steps; leaves the last step's partials and
// shift in part_out / shift_out and trace entries 0..m-1 as the per-step
// launches do.
hipError_t launch_em_sweep_resident(int prec, int deg, const WorkItem *items, int n_items, const int2 *blocks,
                                    int nblocks, int m, void *z, double2 *part_out, double *shift_out,
                                    double2 *trace, hipStream_t s);
hipError_t launch_finish(const WorkItem *items, int n_items, const double2 *part_in, const double *shift_in,
                         double2 *trace, int m, hipStream_t s);
hipError_t launch_adj_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, const void *xS,
                           double *lam, const AdjRef &a, double2 *part_out, hipStream_t s);
// sums: scratch of n_items entries; when given, the two ensemble sums of the
// adjoint are formed once per item by a separate launch (for ensembles of many
// superchunks) instead of by every block.
hipError_t launch_adj_step(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                           const void *xs, const double *lam_in, double *lam_out, const AdjRef &a,
                           const double2 *part_in, double2 *sums, double2 *part_out, double *acc, hipStream_t s);
hipError_t launch_adj_reduce(const WorkItem *items, int n_items, const double *acc, double *out, hipStream_t s);
// In-place streaming pass over n floats (n a multiple of 4096) with the step
// kernel's block shape (the measurement behind mcpr_stream_probe).
hipError_t launch_stream_inplace(float *x, int64_t n, hipStream_t s);
// x[0..n) = 0 (a kernel: safe to replay from a graph)
hipError_t launch_zero(double *x, int64_t n, hipStream_t s);
// Restriction: nr = regions + 1 (record stride).  full = false: region counts
// and means only (a first pass, whose combine writes the region means to
// rshift_next); full = true: complete records.
hipError_t launch_region_partials(int prec, int nr, int mode, bool full, const WorkItem *items, const int2 *blocks,
                                  int nblocks, const double *rshift, const Splits &sp, const RegionMap *maps,
                                  RegionPartial *rpart, hipStream_t s);
hipError_t launch_region_combine(int nr, bool full, const WorkItem *items, int n_items, const RegionPartial *rpart,
                                 const double *rshift, RegionStats *out, double *rshift_next, hipStream_t s);
hipError_t launch_fill_shift(int prec, int nr, const WorkItem *items, int n_items, const double *shift, double *rshift,
                             hipStream_t s);
hipError_t launch_match_apply(int prec, int nreg, const WorkItem *items, const int2 *blocks, int nblocks,
                              const Splits &sp, const RegionMap *maps, hipStream_t s);
hipError_t launch_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, hipStream_t s);
// Trigonometric mean field (every item of the launch has ksin or kc nonzero):
// step-0 sums, the step, and the final trace entry (mean sin, mean cos).
hipError_t launch_sum_init_trig(int prec, const WorkItem *items, const int2 *blocks, int nblocks,
                                double2 *part_out, double *shift_out, hipStream_t s);
hipError_t launch_em_step_trig(int prec, int deg, const WorkItem *items, const int2 *blocks, int nblocks, int j,
                               const double2 *part_in, double2 *part_out, double *shift_out, double2 *trace, int m,
                               hipStream_t s);
hipError_t launch_finish_trig(const WorkItem *items, int n_items, const double2 *part_in, double2 *trace, int m,
                              hipStream_t s);
// Empirical-CDF drift (in cdf.hip): the states of the items laid end to end
// (item i at dense offset doff, n positions in all) with their labels
// (doff + p), kept in sorted order through a fine sweep.
template <typename T>
struct KeyLabel {
    T k;
    uint32_t l;
};
// Bucket engine of the sort (steps after the first of a sweep): the bucket
// of a new state is found among the previous step's sorted states at stride
// kCdfBucket (kCdfBucket states per bucket on average); each bucket holds at
// most kCdfBucketCap states (else the sweep is marked and redone with the
// library sort).  The staging area holds, per bucket slot, the state, its
// label, and its position in the previous step's order (the tie-breaker that
// makes the order equal to the stable library sort's), as three arrays.
// The stride leaves room for the count of a bucket to drift by a few
// standard deviations while the law changes from step to step, so that
// nearly every bucket fits the bucket sort's smaller tile (kCdfTileSmall).
constexpr int kCdfBucket = 1792;
constexpr int kCdfBucketCap = 4096;
constexpr int kCdfTileSmall = 2048;
static_assert(kCdfBucketCap == 4096, "the step kernel indexes staging slots by shifts");
static_assert(kCdfBucket < kCdfTileSmall && kCdfTileSmall < kCdfBucketCap, "tile sizes");
template <typename T>
struct StageView {
    T *u;
    uint32_t *lab, *pos;
};
template <typename T>
inline StageView<T> stage_view(void *stage, int nbuckets) {
    const size_t slots = (size_t)nbuckets * kCdfBucketCap;
    StageView<T> v;
    v.u = (T *)stage;
    v.lab = (uint32_t *)((char *)stage + slots * sizeof(T));
    v.pos = v.lab + slots;
    return v;
}
inline size_t stage_bytes(int prec, int nbuckets) {
    return (size_t)nbuckets * kCdfBucketCap * ((prec == 0 ? sizeof(double) : sizeof(float)) + 2 * sizeof(uint32_t));
}
struct CdfBuffers {
    void *keys[2];       // state type, n each: [0] the step's output (sort input), [1] sorted by value
    uint32_t *lab[2];    // their labels
    uint32_t *seg[2];    // item of each value-sorted pair, before / after the item pass
    void *kl[2];         // KeyLabel<state type> pairs before / after the item pass
    uint32_t *seg_begin; // doff of every item
    void *tmp;
    size_t tmp_bytes;
    // bucket engine
    int nbuckets;        // buckets of the launch
    uint32_t *bcount;    // states per bucket (zero between steps)
    uint2 *bmeta;        // per bucket: first dense output position and states (k_cdf_bscan)
    void *stage;         // staging area (stage_view), kCdfBucketCap slots per bucket
    uint32_t *defer;     // [0] count, [1..] buckets left to the block sort (k_cdf_wsort appends, k_cdf_bscan clears)
    uint32_t *flag;      // nonzero once a bucket overflowed in this sweep
};
// Once per fine sweep: the dense first position of every item; the states and
// labels into keys[0], lab[0]; bucket counts and the overflow flag cleared.
hipError_t launch_cdf_start(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                            const CdfBuffers &b, hipStream_t s);
// Bytes of library scratch the sorts need for n positions of nseg items.
hipError_t cdf_scratch_bytes(int prec, uint32_t n, uint32_t nseg, size_t &bytes);
// Library engine: sorts (keys[0], lab[0]) so that each item's pairs are
// ascending at [doff, doff + P) in keys[1], lab[1] (one item) or kl[1]
// (several items).
hipError_t launch_cdf_sort(int prec, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s);
// Bucket engine: the staged states of every bucket sorted by (value,
// previous position) into keys[1], lab[1] at their item's positions.
hipError_t launch_cdf_buckets(int prec, const WorkItem *items, int n_items, const CdfBuffers &b, hipStream_t s);
// The Euler-Maruyama step with the empirical-CDF drift, in sorted order (the
// pairs in kl[1] if packed, else keys[1], lab[1]); the input's mean field is
// combined once per item first (into mv).  mode 0: the new states
// and labels go to keys[0], lab[0] at the sorted positions (the library
// sort's input); 1: into the buckets; 2 (the last step of the sweep): to the
// particles' slots, unless the overflow flag is set.
hipError_t launch_em_step_sorted(int prec, int deg, const WorkItem *items, int n_items, const int2 *blocks,
                                 int nblocks, int j, int mode, bool packed, const double2 *part_in,
                                 const double *shift_in, double2 *mv, const CdfBuffers &b, double2 *part_out,
                                 double *shift_out, double2 *trace, int m, hipStream_t s);
// out[i] = (1/P) sum Phi(x_p) of item i; part: scratch of one partial per superchunk.
hipError_t launch_qoi(int prec, int kind, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                      double2 *part, double *out, hipStream_t s);

} // namespace mcpr
