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
//
// From the second step of a sweep on, each step's sorted input also serves
// as the splitter set of its output (the bucket engine): the step kernel puts
// every new state into the bucket between two sorted inputs at stride
// kCdfBucket, k_cdf_bscan turns the bucket counts into positions, and
// k_cdf_bsort sorts each bucket in LDS by (state, previous position), which
// is the order the stable library sort gives; the library sort then runs only
// on the first two steps.  (The first step's input may be a point mass, which
// splits nothing.)  Buckets stay near kCdfBucket states while the law changes
// little per step; one above kCdfBucketCap marks the sweep, whose remaining
// steps then do nothing and leave the particles untouched, and the host
// redoes the sweep with the library sort on its first 8 steps, then 32, then
// all of them.  Each bucket is sorted in a tile of kCdfTileSmall states when
// it fits, else of kCdfBucketCap (measured against one counting pass over
// bins linear in the state: no faster here, so not kept).
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/block/block_radix_sort.hpp>
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

// The dense first position of every item; zero bucket counts; the overflow
// flag cleared.
__global__ __launch_bounds__(kThreads) void k_cdf_setup(const WorkItem *__restrict__ items, int n_items,
                                                        uint32_t *__restrict__ beg, uint32_t *__restrict__ bcount,
                                                        int nbuckets, uint32_t *__restrict__ flag) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n_items) beg[i] = (uint32_t)items[i].doff;
    if (i < nbuckets) bcount[i] = 0u;
    if (i == 0) *flag = 0u;
}

// Exclusive scan of one item's bucket counts (one block per item): each
// bucket's first dense output position and its count, for k_cdf_bsort; the
// counts cleared for the next step; a count above the capacity marks the
// sweep.
__global__ __launch_bounds__(kThreads) void k_cdf_bscan(const WorkItem *__restrict__ items,
                                                        uint32_t *__restrict__ bcount, uint2 *__restrict__ bmeta,
                                                        uint32_t *__restrict__ flag) {
    __shared__ uint32_t sh[kThreads];
    const WorkItem &W = items[blockIdx.x];
    uint32_t carry = 0;
    for (int c0 = 0; c0 < W.nbk; c0 += kThreads) {
        const int k = c0 + (int)threadIdx.x;
        const uint32_t v = k < W.nbk ? bcount[W.bbase + k] : 0u;
        if (v > (uint32_t)kCdfBucketCap) *flag = 1u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kThreads; off <<= 1) { // inclusive Hillis-Steele scan
            const uint32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < W.nbk) {
            bmeta[W.bbase + k] = make_uint2((uint32_t)W.doff + carry + sh[threadIdx.x] - v, v);
            bcount[W.bbase + k] = 0u;
        }
        carry += sh[kThreads - 1];
        __syncthreads();
    }
}

// Order key of a state: its bits mapped so that unsigned order is numeric
// order, with -0 taken as +0 (the library sort's convention: equal keys).
__device__ __forceinline__ uint32_t order_code(float u) {
    const uint32_t b = __float_as_uint(u == 0.0f ? 0.0f : u);
    return b ^ ((b >> 31) ? 0xffffffffu : 0x80000000u);
}
__device__ __forceinline__ uint64_t order_code(double u) {
    const uint64_t b = (uint64_t)__double_as_longlong(u == 0.0 ? 0.0 : u);
    return b ^ ((b >> 63) ? 0xffffffffffffffffull : 0x8000000000000000ull);
}

constexpr int kSortThreads = 256;
constexpr uint32_t kMaxTieRun = 32; // longer runs of equal states mark the sweep (redone by the library)

template <typename T, int ITEMS>
using BucketSorter = rocprim::block_radix_sort<decltype(order_code(T())), kSortThreads, ITEMS, uint32_t>;

// LDS of the bucket sort: the block radix sort's storage for either tile,
// then the sorted codes and staging slots; the bucket's smallest and largest
// codes before the sort.
template <typename T>
union BucketShared {
    using Code = decltype(order_code(T()));
    Code range[2];
    typename BucketSorter<T, kCdfTileSmall / kSortThreads>::storage_type small;
    typename BucketSorter<T, kCdfBucketCap / kSortThreads>::storage_type large;
    struct {
        Code code[kCdfBucketCap];
        uint32_t slot[kCdfBucketCap];
    } post;
};

// The n <= ITEMS * kSortThreads staged states of one bucket sorted by order
// code with a stable block radix sort over the bits in which the bucket's
// codes differ: code - min for the states, max - min + 1 for the padding
// (strictly last); the input order (the staging slots) only decides the
// order of equal codes, which the tie pass then sets: every run of equal
// codes ordered by the previous position (runs are short: states only tie by
// rounding once the noise has spread them; a run longer than kMaxTieRun
// marks the sweep).  Written with their labels from dst on.
template <typename T, int ITEMS, typename Storage>
__device__ __forceinline__ void sort_bucket(Storage &st, BucketShared<T> &sh, uint32_t n, uint32_t dst,
                                            const T *__restrict__ su, const uint32_t *__restrict__ sl,
                                            const uint32_t *__restrict__ sp, uint32_t *__restrict__ flag,
                                            T *__restrict__ ko, uint32_t *__restrict__ lo) {
    using Code = decltype(order_code(T()));
    Code keys[ITEMS];
    uint32_t vals[ITEMS];
    Code lmin = ~(Code)0, lmax = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        // striped, coalesced loads without a branch (every slot below
        // kCdfBucketCap is the bucket's own; those at or past n are not used)
        const uint32_t t = k * kSortThreads + threadIdx.x;
        const T a = su[t];
        keys[k] = order_code(a);
        vals[k] = t;
        lmin = t < n && keys[k] < lmin ? keys[k] : lmin;
        lmax = t < n && keys[k] > lmax ? keys[k] : lmax;
    }
    atomicMin(&sh.range[0], lmin);
    atomicMax(&sh.range[1], lmax);
    __syncthreads();
    const Code cmin = sh.range[0], span = sh.range[1] - sh.range[0];
    __syncthreads(); // (the sort storage overlays the range)
    if (n > 0 && span == ~(Code)0) { // no room above the largest key (a bucket across the whole range)
        if (threadIdx.x == 0) *flag = 1u;
        return;
    }
    const Code pad = span + 1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t t = k * kSortThreads + threadIdx.x;
        keys[k] = t < n ? keys[k] - cmin : pad;
    }
    unsigned nbits = 0;
    for (Code d = pad; d != 0; d >>= 1) ++nbits;
    BucketSorter<T, ITEMS>().sort_to_striped(keys, vals, st, 0u, nbits); // rank k * kSortThreads + t in thread t
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        sh.post.code[k * kSortThreads + threadIdx.x] = keys[k];
        sh.post.slot[k * kSortThreads + threadIdx.x] = vals[k];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i + 1 < n; i += kSortThreads) {
        const Code c = sh.post.code[i];
        if (sh.post.code[i + 1] != c || (i > 0 && sh.post.code[i - 1] == c)) continue;
        uint32_t e = i + 1; // the run [i, e]
        while (e + 1 < n && sh.post.code[e + 1] == c && e - i < kMaxTieRun) ++e;
        if (e - i >= kMaxTieRun) {
            *flag = 1u;
            continue;
        }
        for (uint32_t a = i + 1; a <= e; ++a) { // insertion sort of the run by previous position
            const uint32_t s = sh.post.slot[a], ps = sp[s];
            uint32_t q = a;
            while (q > i && sp[sh.post.slot[q - 1]] > ps) {
                sh.post.slot[q] = sh.post.slot[q - 1];
                --q;
            }
            sh.post.slot[q] = s;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < n; t += kSortThreads) {
        const uint32_t e = sh.post.slot[t];
        ko[dst + t] = su[e];
        lo[dst + t] = sl[e];
    }
}

// One bucket per block, sorted in the smaller tile when it fits (nearly
// always: the bucket stride leaves that margin), else in the full one; the
// result is the order of the stable library sort, at the item's positions
// (bmeta).
template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_cdf_bsort(const uint2 *__restrict__ bmeta, StageView<T> stage,
                                                            uint32_t *__restrict__ flag, T *__restrict__ ko,
                                                            uint32_t *__restrict__ lo) {
    using Code = decltype(order_code(T()));
    __shared__ BucketShared<T> sh;
    const uint2 meta = bmeta[blockIdx.x]; // (first dense output position, states)
    // The sweep is redone once any block has set the flag.  Other blocks of
    // this launch may set it while this one starts, so one thread reads it
    // and the whole block takes that one decision.
    __shared__ uint32_t skip;
    if (threadIdx.x == 0) skip = *flag;
    __syncthreads();
    if (skip) return;
    const uint32_t dst = meta.x, n = meta.y;
    if (n > (uint32_t)kCdfBucketCap) return; // cannot happen unflagged; keeps LDS indices in range
    const size_t s0 = (size_t)blockIdx.x * kCdfBucketCap; // the bucket's first staging slot
    if (threadIdx.x == 0) {
        sh.range[0] = ~(Code)0;
        sh.range[1] = 0;
    }
    __syncthreads();
    if (n <= (uint32_t)kCdfTileSmall) // (n is the same for the whole block)
        sort_bucket<T, kCdfTileSmall / kSortThreads>(sh.small, sh, n, dst, stage.u + s0, stage.lab + s0,
                                                     stage.pos + s0, flag, ko, lo);
    else
        sort_bucket<T, kCdfBucketCap / kSortThreads>(sh.large, sh, n, dst, stage.u + s0, stage.lab + s0,
                                                     stage.pos + s0, flag, ko, lo);
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
    const int cover = n_items > b.nbuckets ? n_items : b.nbuckets;
    hipLaunchKernelGGL(k_cdf_setup, dim3((cover + kThreads - 1) / kThreads), dim3(kThreads), 0, s, items, n_items,
                       b.seg_begin, b.bcount, b.nbuckets, b.flag);
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

hipError_t launch_cdf_buckets(int prec, const WorkItem *items, int n_items, const CdfBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_cdf_bscan, dim3(n_items), dim3(kThreads), 0, s, items, b.bcount, b.bmeta, b.flag);
    if (prec == 0)
        hipLaunchKernelGGL(k_cdf_bsort<double>, dim3(b.nbuckets), dim3(kSortThreads), 0, s, b.bmeta,
                           stage_view<double>(b.stage, b.nbuckets), b.flag, (double *)b.keys[1], b.lab[1]);
    else
        hipLaunchKernelGGL(k_cdf_bsort<float>, dim3(b.nbuckets), dim3(kSortThreads), 0, s, b.bmeta,
                           stage_view<float>(b.stage, b.nbuckets), b.flag, (float *)b.keys[1], b.lab[1]);
    return hipGetLastError();
}

hipError_t launch_cdf_sort(int prec, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s) {
    return prec == 0 ? sorted<double>(n_items, n, b, s) : sorted<float>(n_items, n, b, s);
}

} // namespace mcpr
