// cdf.hip -- ranks for the empirical-CDF drift term (the particle system of
// the viscous Burgers equation, Sec. 5.2).
//
// The drift acdf (1 - F_P(x_p)) needs, at every step and for every particle,
// the count sum_q H(x_p - x_q) with H(0) = 1/2: the number of particles below
// x_p plus half the number equal to it (itself included).  Per step:
//   1. gather: the state of every item of the launch into one key array (at
//      the item's offset koff) with the particle index as value;
//   2. a segmented radix sort of the pairs, one segment per item (rocPRIM);
//   3. run flags: fwd[i] = i at the first position of a run of equal keys
//      (a segment start is always one), bwd[n-1-i] = n-1-i at the last one;
//   4. two inclusive max-scans: fwd gives each position the start of its
//      run, bwd (indexed from the end) its last position;
//   5. rank: F[koff + index] = (start - koff) + (end - start + 1) / 2.
// Runs never cross a segment, so the whole launch is one pair of scans.
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "common.hpp"
#include "launch.hpp"

namespace mcpr {
namespace {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_gather(const WorkItem *__restrict__ items,
                                                         const int2 *__restrict__ blocks, int32_t j,
                                                         T *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x) + (int64_t)j * W.traj;
    const int64_t P = W.P;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * W.R;
    for (int r = 0; r < W.R; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x) + e;
            if (p < P) {
                keys[W.koff + p] = x[p];
                vals[W.koff + p] = (uint32_t)p;
            }
        }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_flags(const WorkItem *__restrict__ items,
                                                        const int2 *__restrict__ blocks,
                                                        const T *__restrict__ keys, uint32_t n,
                                                        uint32_t *__restrict__ fwd, uint32_t *__restrict__ bwd) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const int64_t P = W.P;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * W.R;
    for (int r = 0; r < W.R; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t rp = base + 4 * (int64_t)(r * kThreads + threadIdx.x) + e;
            if (rp < P) {
                const uint32_t i = (uint32_t)(W.koff + rp);
                const bool first = rp == 0 || keys[i] != keys[i - 1];
                const bool last = rp == P - 1 || keys[i] != keys[i + 1];
                fwd[i] = first ? i : 0u;
                bwd[n - 1u - i] = last ? n - 1u - i : 0u;
            }
        }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cdf_rank(const WorkItem *__restrict__ items,
                                                       const int2 *__restrict__ blocks,
                                                       const uint32_t *__restrict__ vals,
                                                       const uint32_t *__restrict__ start,
                                                       const uint32_t *__restrict__ bwd_scan, uint32_t n,
                                                       T *__restrict__ F) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const int64_t P = W.P;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * W.R;
    for (int r = 0; r < W.R; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t rp = base + 4 * (int64_t)(r * kThreads + threadIdx.x) + e;
            if (rp < P) {
                const uint32_t i = (uint32_t)(W.koff + rp);
                const uint32_t s = start[i];
                const uint32_t last = n - 1u - bwd_scan[n - 1u - i];
                const double cnt = (double)((int64_t)s - W.koff) + 0.5 * (double)(last - s + 1u);
                F[W.koff + vals[i]] = (T)cnt;
            }
        }
}

template <typename T>
hipError_t sort_pairs(void *tmp, size_t &bytes, const T *kin, T *kout, const uint32_t *vin, uint32_t *vout,
                      uint32_t n, uint32_t nseg, const uint32_t *beg, const uint32_t *end, hipStream_t s) {
    return rocprim::segmented_radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, n, nseg, beg, end, 0,
                                               (unsigned)(8 * sizeof(T)), s);
}

hipError_t scan_max(void *tmp, size_t &bytes, const uint32_t *in, uint32_t *out, uint32_t n, hipStream_t s) {
    return rocprim::inclusive_scan(tmp, bytes, in, out, (size_t)n, rocprim::maximum<uint32_t>(), s);
}

template <typename T>
hipError_t scratch_bytes(uint32_t n, uint32_t nseg, size_t &bytes) {
    size_t a = 0, b = 0;
    hipError_t e = sort_pairs<T>(nullptr, a, nullptr, nullptr, nullptr, nullptr, n, nseg, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    e = scan_max(nullptr, b, nullptr, nullptr, n, 0);
    if (e != hipSuccess) return e;
    bytes = a > b ? a : b;
    return hipSuccess;
}

template <typename T>
hipError_t counts(const WorkItem *items, int n_items, const int2 *blocks, int nblocks, uint32_t n, int j,
                  const CdfBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_cdf_gather<T>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j, (T *)b.keys[0],
                       b.vals[0]);
    size_t bytes = b.tmp_bytes;
    hipError_t e = sort_pairs<T>(b.tmp, bytes, (const T *)b.keys[0], (T *)b.keys[1], b.vals[0], b.vals[1], n,
                                 (uint32_t)n_items, b.seg_begin, b.seg_end, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_flags<T>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, (const T *)b.keys[1], n,
                       b.fwd[0], b.bwd[0]);
    bytes = b.tmp_bytes;
    if ((e = scan_max(b.tmp, bytes, b.fwd[0], b.fwd[1], n, s)) != hipSuccess) return e;
    bytes = b.tmp_bytes;
    if ((e = scan_max(b.tmp, bytes, b.bwd[0], b.bwd[1], n, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_rank<T>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, b.vals[1], b.fwd[1],
                       b.bwd[1], n, (T *)b.F);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_cdf_setup(const WorkItem *__restrict__ items, int n_items, uint32_t n,
                                                        uint32_t *__restrict__ beg, uint32_t *__restrict__ end,
                                                        uint32_t *__restrict__ fwd, uint32_t *__restrict__ bwd) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) {
        fwd[i] = 0u;
        bwd[i] = 0u;
    }
    if ((int)i < n_items) {
        beg[i] = (uint32_t)items[i].koff;
        end[i] = (uint32_t)(items[i].koff + items[i].P);
    }
}

} // namespace

hipError_t launch_cdf_setup(const WorkItem *items, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s) {
    const uint32_t cover = n > (uint32_t)n_items ? n : (uint32_t)n_items;
    hipLaunchKernelGGL(k_cdf_setup, dim3((cover + kThreads - 1) / kThreads), dim3(kThreads), 0, s, items, n_items, n,
                       b.seg_begin, b.seg_end, b.fwd[0], b.bwd[0]);
    return hipGetLastError();
}

hipError_t cdf_scratch_bytes(int prec, uint32_t n, uint32_t nseg, size_t &bytes) {
    return prec == 0 ? scratch_bytes<double>(n, nseg, bytes) : scratch_bytes<float>(n, nseg, bytes);
}

hipError_t launch_cdf_counts(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks, uint32_t n,
                             int j, const CdfBuffers &b, hipStream_t s) {
    return prec == 0 ? counts<double>(items, n_items, blocks, nblocks, n, j, b, s)
                     : counts<float>(items, n_items, blocks, nblocks, n, j, b, s);
}

} // namespace mcpr
