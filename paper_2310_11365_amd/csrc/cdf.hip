// cdf.hip -- the sorted order the empirical-CDF drift term needs (the
// particle system of the viscous Burgers equation, Sec. 5.2).
//
// The drift acdf (1 - F_P(x_p)) needs, at every step and for every particle,
// the count sum_q H(x_p - x_q) with H(0) = 1/2: the number of particles below
// x_p plus half the number equal to it (itself included).  Each item's states
// in ascending order give it: position r of a run [lo, hi] of equal keys has
// the count lo + (hi - lo + 1) / 2 (the step kernel, k_em_step_sorted, finds
// the run).  The items of a launch are laid end to end in a dense index space
// (item i at doff_i).  Per step:
//   1. gather: every item's state into keys[0] at doff + p;
//   2. one device-wide radix sort of (key, dense index) pairs over all items;
//   3. with several items: each sorted key's item, then a stable radix sort
//      by item (a few bits), which leaves each item's keys in ascending order
//      at [doff, doff + P); keys and indices are permuted into that order.
// A device-wide sort rather than a segmented one: the segmented sort gives
// each segment to one workgroup, which leaves the chip idle for the few large
// ensembles a Parareal sweep batches.
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "common.hpp"
#include "launch.hpp"

namespace mcpr {
namespace {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_gather(const WorkItem *__restrict__ items,
                                                         const int2 *__restrict__ blocks, int32_t j,
                                                         T *__restrict__ keys) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x) + (int64_t)j * W.traj;
    const int64_t P = W.P;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * W.R;
    for (int r = 0; r < W.R; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x) + e;
            if (p < P) keys[W.doff + p] = x[p];
        }
}

// Item of every value-sorted key: the last item whose first dense position is
// at or below the key's dense index (beg holds n_items ascending starts).
__global__ __launch_bounds__(kThreads) void k_cdf_segkey(const uint32_t *__restrict__ idx, uint32_t n,
                                                         const uint32_t *__restrict__ beg, int n_items,
                                                         uint32_t *__restrict__ seg) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t g = idx[i];
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (beg[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    seg[i] = (uint32_t)lo;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_permute(const uint32_t *__restrict__ pos, uint32_t n,
                                                          const T *__restrict__ kin, const uint32_t *__restrict__ iin,
                                                          T *__restrict__ kout, uint32_t *__restrict__ iout) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t q = pos[i];
    kout[i] = kin[q];
    iout[i] = iin[q];
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
hipError_t sort_values(void *tmp, size_t &bytes, const T *kin, T *kout, uint32_t *iout, uint32_t n, hipStream_t s) {
    return rocprim::radix_sort_pairs(tmp, bytes, kin, kout, rocprim::counting_iterator<uint32_t>(0u), iout, (size_t)n,
                                     0u, (unsigned)(8 * sizeof(T)), s);
}

hipError_t sort_items(void *tmp, size_t &bytes, const uint32_t *sin, uint32_t *sout, uint32_t *pos, uint32_t n,
                      unsigned bits, hipStream_t s) {
    return rocprim::radix_sort_pairs(tmp, bytes, sin, sout, rocprim::counting_iterator<uint32_t>(0u), pos, (size_t)n,
                                     0u, bits, s);
}

template <typename T>
hipError_t scratch_bytes(uint32_t n, uint32_t nseg, size_t &bytes) {
    size_t a = 0, b = 0;
    hipError_t e = sort_values<T>(nullptr, a, nullptr, nullptr, nullptr, n, 0);
    if (e != hipSuccess) return e;
    if (nseg > 1 && (e = sort_items(nullptr, b, nullptr, nullptr, nullptr, n, seg_bits(nseg), 0)) != hipSuccess)
        return e;
    bytes = a > b ? a : b;
    return hipSuccess;
}

template <typename T>
hipError_t sorted(const WorkItem *items, int n_items, const int2 *blocks, int nblocks, uint32_t n, int j,
                  const CdfBuffers &b, const void **ks, const uint32_t **ix, hipStream_t s) {
    T *k0 = (T *)b.keys[0], *k1 = (T *)b.keys[1], *k2 = (T *)b.keys[2];
    const dim3 flat((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_cdf_gather<T>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j, k0);
    size_t bytes = b.tmp_bytes;
    hipError_t e = sort_values<T>(b.tmp, bytes, k0, k1, b.idx[0], n, s);
    if (e != hipSuccess) return e;
    *ks = k1;
    *ix = b.idx[0];
    if (n_items > 1) {
        hipLaunchKernelGGL(k_cdf_segkey, flat, dim3(kThreads), 0, s, b.idx[0], n, b.seg_begin, n_items, b.seg[0]);
        bytes = b.tmp_bytes;
        if ((e = sort_items(b.tmp, bytes, b.seg[0], b.seg[1], b.pos, n, seg_bits((uint32_t)n_items), s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_cdf_permute<T>, flat, dim3(kThreads), 0, s, b.pos, n, k1, b.idx[0], k2, b.idx[1]);
        *ks = k2;
        *ix = b.idx[1];
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_cdf_setup(const WorkItem *items, int n_items, const CdfBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_cdf_setup, dim3((n_items + kThreads - 1) / kThreads), dim3(kThreads), 0, s, items, n_items,
                       b.seg_begin);
    return hipGetLastError();
}

hipError_t cdf_scratch_bytes(int prec, uint32_t n, uint32_t nseg, size_t &bytes) {
    return prec == 0 ? scratch_bytes<double>(n, nseg, bytes) : scratch_bytes<float>(n, nseg, bytes);
}

hipError_t launch_cdf_sort(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks, uint32_t n,
                           int j, const CdfBuffers &b, const void **ks, const uint32_t **ix, hipStream_t s) {
    return prec == 0 ? sorted<double>(items, n_items, blocks, nblocks, n, j, b, ks, ix, s)
                     : sorted<float>(items, n_items, blocks, nblocks, n, j, b, ks, ix, s);
}

} // namespace mcpr
