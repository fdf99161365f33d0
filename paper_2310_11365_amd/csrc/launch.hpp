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
hipError_t launch_finish(const WorkItem *items, int n_items, const double2 *part_in, const double *shift_in,
                         double2 *trace, int m, hipStream_t s);
hipError_t launch_adj_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, const void *xS,
                           double *lam, const AdjStep &a, double2 *part_out, hipStream_t s);
// sums: scratch of n_items entries; when given, the two ensemble sums of the
// adjoint are formed once per item by a separate launch (for ensembles of many
// superchunks) instead of by every block.
hipError_t launch_adj_step(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                           const void *xs, const double *lam_in, double *lam_out, const AdjStep &a,
                           const double2 *part_in, double2 *sums, double2 *part_out, double *acc, hipStream_t s);
hipError_t launch_adj_reduce(const WorkItem *items, int n_items, const double *acc, double *out, hipStream_t s);
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
struct CdfBuffers {
    void *keys[2];       // state type, n each: [0] the step's output (sort input), [1] sorted by value
    uint32_t *lab[2];    // their labels
    uint32_t *seg[2];    // item of each value-sorted pair, before / after the item pass
    void *kl[2];         // KeyLabel<state type> pairs before / after the item pass
    uint32_t *seg_begin; // doff of every item
    void *tmp;
    size_t tmp_bytes;
};
// Once per fine sweep: the dense first position of every item; the states and
// labels into keys[0], lab[0].
hipError_t launch_cdf_start(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                            const CdfBuffers &b, hipStream_t s);
// Bytes of library scratch the sorts need for n positions of nseg items.
hipError_t cdf_scratch_bytes(int prec, uint32_t n, uint32_t nseg, size_t &bytes);
// Sorts (keys[0], lab[0]): each item's pairs ascending at [doff, doff + P) in
// keys[1], lab[1] (one item) or kl[1] (several items).
hipError_t launch_cdf_sort(int prec, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s);
// The Euler-Maruyama step with the empirical-CDF drift, in sorted order: the
// new states go to keys[0], lab[0], or on the last step of the sweep to the
// particles' slots.
hipError_t launch_em_step_sorted(int prec, int deg, const WorkItem *items, int n_items, const int2 *blocks,
                                 int nblocks, int j, bool last, const double2 *part_in, const double *shift_in,
                                 const CdfBuffers &b, double2 *part_out, double *shift_out, double2 *trace, int m,
                                 hipStream_t s);
// out[i] = (1/P) sum Phi(x_p) of item i; part: scratch of one partial per superchunk.
hipError_t launch_qoi(int prec, int kind, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                      double2 *part, double *out, hipStream_t s);

} // namespace mcpr
