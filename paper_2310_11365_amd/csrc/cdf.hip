// cdf.hip -- the sorted order the empirical-CDF drift term needs (the
// particle system of the viscous Burgers equation, Sec. 5.2).
//
// The drift acdf (1 - F_P(x_p)) needs, at every step and for every particle,
// the count sum_q H(x_p - x_q) with H(0) = 1/2: the number of particles below
// x_p plus half the number equal to it (itself included).  Each item's states
// in ascending order give it: position r of a run [lo, hi] of equal keys has
// the count lo + (hi - lo + 1) / 2 (the step kernel, k_em_step_sorted, finds
// the run).  The items of a launch are laid end to end in a dense index space
// (item i at doff_i); a particle's label is its dense index doff + p.
//
// A fine sweep keeps its ensembles in sorted order from step to step: the
// first step gathers the states (with labels doff + p) into keys[0] and
// lab[0]; every step sorts (keys[0], lab[0]); the step kernel reads the
// sorted pairs, and writes the new states with their labels back into keys[0]
// and lab[0] at the sorted positions, except the last step of the sweep,
// which writes each new state to its particle's slot.  The sort per step:
//   1. one device-wide radix sort of (key, label) pairs over all items into
//      keys[1], lab[1];
//   2. with several items: each pair's item (from its label) and the pair
//      packed into one value, then a stable radix sort by item (a few bits)
//      into kl[1], which leaves each item's pairs in ascending key order at
//      [doff, doff + P).
// A device-wide sort rather than a segmented one: the segmented sort gives
// each segment to one workgroup, which leaves the chip idle for the few large
// ensembles a Parareal sweep batches.
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "common.hpp"
#include "launch.hpp"

namespace mcpr {
namespace {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_gather(const WorkItem *__restrict__ items,
                                                         const int2 *__restrict__ blocks, T *__restrict__ keys,
                                                         uint32_t *__restrict__ lab) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x);
    const int64_t P = W.P;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * W.R;
    for (int r = 0; r < W.R; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x) + e;
            if (p < P) {
                keys[W.doff + p] = x[p];
                lab[W.doff + p] = (uint32_t)(W.doff + p);
            }
        }
}

// Item of every value-sorted pair (the last item whose first dense position
// is at or below the label; beg holds n_items ascending starts) and the pair
// packed for the item pass.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_pack(const T *__restrict__ keys, const uint32_t *__restrict__ lab,
                                                       uint32_t n, const uint32_t *__restrict__ beg, int n_items,
                                                       uint32_t *__restrict__ seg, KeyLabel<T> *__restrict__ kl) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t g = lab[i];
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (beg[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    seg[i] = (uint32_t)lo;
    KeyLabel<T> v;
    v.k = keys[i];
    v.l = g;
    kl[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_cdf_setup(const WorkItem *__restrict__ items, int n_items,
                                                        uint32_t *__restrict__ beg) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n_items) beg[i] = (uint32_t)items[i].doff;
}

// Bits that hold every item number below n_items.
unsigned seg_bits(uint32_t n_items) {
    unsigned b = 1;
    while (b < 32 && ((uint64_t)1 << b) < n_items) ++b;
    return b;
}

template <typename T>
hipError_t sort_values(void *tmp, size_t &bytes, const T *kin, T *kout, const uint32_t *lin, uint32_t *lout,
                       uint32_t n, hipStream_t s) {
    return rocprim::radix_sort_pairs(tmp, bytes, kin, kout, lin, lout, (size_t)n, 0u, (unsigned)(8 * sizeof(T)), s);
}

template <typename T>
hipError_t sort_items(void *tmp, size_t &bytes, const uint32_t *sin, uint32_t *sout, const KeyLabel<T> *vin,
                      KeyLabel<T> *vout, uint32_t n, unsigned bits, hipStream_t s) {
    return rocprim::radix_sort_pairs(tmp, bytes, sin, sout, vin, vout, (size_t)n, 0u, bits, s);
}

template <typename T>
hipError_t scratch_bytes(uint32_t n, uint32_t nseg, size_t &bytes) {
    size_t a = 0, b = 0;
    hipError_t e = sort_values<T>(nullptr, a, nullptr, nullptr, nullptr, nullptr, n, 0);
    if (e != hipSuccess) return e;
    if (nseg > 1 &&
        (e = sort_items<T>(nullptr, b, nullptr, nullptr, nullptr, nullptr, n, seg_bits(nseg), 0)) != hipSuccess)
        return e;
    bytes = a > b ? a : b;
    return hipSuccess;
}

template <typename T>
hipError_t sorted(int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s) {
    size_t bytes = b.tmp_bytes;
    hipError_t e = sort_values<T>(b.tmp, bytes, (const T *)b.keys[0], (T *)b.keys[1], b.lab[0], b.lab[1], n, s);
    if (e != hipSuccess) return e;
    if (n_items > 1) {
        hipLaunchKernelGGL(k_cdf_pack<T>, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                           (const T *)b.keys[1], b.lab[1], n, b.seg_begin, n_items, b.seg[0], (KeyLabel<T> *)b.kl[0]);
        bytes = b.tmp_bytes;
        if ((e = sort_items<T>(b.tmp, bytes, b.seg[0], b.seg[1], (const KeyLabel<T> *)b.kl[0], (KeyLabel<T> *)b.kl[1],
                               n, seg_bits((uint32_t)n_items), s)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_cdf_start(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                            const CdfBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_cdf_setup, dim3((n_items + kThreads - 1) / kThreads), dim3(kThreads), 0, s, items, n_items,
                       b.seg_begin);
    if (prec == 0)
        hipLaunchKernelGGL(k_cdf_gather<double>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks,
                           (double *)b.keys[0], b.lab[0]);
    else
        hipLaunchKernelGGL(k_cdf_gather<float>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks,
                           (float *)b.keys[0], b.lab[0]);
    return hipGetLastError();
}

hipError_t cdf_scratch_bytes(int prec, uint32_t n, uint32_t nseg, size_t &bytes) {
    return prec == 0 ? scratch_bytes<double>(n, nseg, bytes) : scratch_bytes<float>(n, nseg, bytes);
}

hipError_t launch_cdf_sort(int prec, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s) {
    return prec == 0 ? sorted<double>(n_items, n, b, s) : sorted<float>(n_items, n, b, s);
}

} // namespace mcpr
