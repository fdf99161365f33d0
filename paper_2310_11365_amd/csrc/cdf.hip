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
// kCdfBucket, k_cdf_bscan turns the bucket counts into positions, and each
// bucket is sorted by (state, previous position), which is the order the
// stable library sort gives; the library sort then runs only on the first
// two steps.  (The first step's input may be a point mass, which splits
// nothing.)  Buckets stay near kCdfBucket states while the law changes
// little per step; one above kCdfBucketCap marks the sweep, whose remaining
// steps then do nothing and leave the particles untouched, and the host
// redoes the sweep with the library sort on its first 8 steps, then 32, then
// all of them.  A bucket of at most kCdfTileSmall states (nearly all) is
// sorted by one wavefront in its registers (k_cdf_wsort), the others by a
// whole block (k_cdf_bsort); both are bitonic networks.
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
// bucket's first dense output position and its count, for the bucket sort; the
// counts cleared for the next step; a count above the capacity marks the
// sweep; the block sort's list emptied.
__global__ __launch_bounds__(kThreads) void k_cdf_bscan(const WorkItem *__restrict__ items,
                                                        uint32_t *__restrict__ bcount, uint2 *__restrict__ bmeta,
                                                        uint32_t *__restrict__ defer, uint32_t *__restrict__ flag) {
    __shared__ uint32_t sh[kThreads];
    const WorkItem &W = items[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) defer[0] = 0u; // the block sort's list, filled by k_cdf_wsort
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
// A negative state's bits are negated (two's complement), a positive one's
// sign bit is set: -0 and +0 both give 2^31, and the map is monotone.
__device__ __forceinline__ uint32_t order_code(float u) {
    const uint32_t b = __float_as_uint(u), m = (uint32_t)((int32_t)b >> 31);
    return (b ^ (m | 0x80000000u)) - m;
}
__device__ __forceinline__ uint64_t order_code(double u) {
    const uint64_t b = (uint64_t)__double_as_longlong(u), m = (uint64_t)((int64_t)b >> 63);
    return (b ^ (m | 0x8000000000000000ull)) - m;
}

// Element idx of an array at a uniform base, addressed by a 32-bit byte
// offset (the base stays in scalar registers).
template <typename V>
__device__ __forceinline__ V ld_at(const V *base, uint32_t idx) {
    return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + idx * (uint32_t)sizeof(V));
}
template <typename V>
__device__ __forceinline__ void st_at(V *base, uint32_t idx, V v) {
    *reinterpret_cast<V *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(V)) = v;
}
// All ones when idx >= n (padding), else zero.
__device__ __forceinline__ uint32_t pad_mask(uint32_t idx, uint32_t n) {
    return ~(uint32_t)((int32_t)(idx - n) >> 31);
}

// ---------------------------------------------------------------------------
// Bucket sort: the staged states of every bucket ordered by (order code,
// previous position) and written with their labels at the bucket's dense
// positions.
//
// Keys.  A state's key packs a quantised code and its staging slot into one
// word, q << SB | slot with q = (code - min) >> s, where min is the bucket's
// smallest code and s the smallest shift that leaves every q below
// 2^(32 - SB) - 1 (the all-ones word is the padding, last).  q does not
// decrease with the code, so sorted keys order the states by code except
// inside runs of equal q: true ties, and codes that differ only in the
// dropped bits (s > 0: a bucket across zero or with a far outlier, every
// fp64 bucket), which are rare because at least 2^(31 - SB) quanta cover
// the bucket's codes.  Each such run is then ordered by (code, previous
// position) by the thread that holds its first element, which reads both
// from the staging area for the run's states only; a run longer than
// kMaxTieRun + 1 marks the sweep.
//
// Network.  A bitonic network over registers, in the variant whose every
// comparator is ascending (the first stage of each merge level compares an
// element with its mirror in the level's block, the others with the element
// j apart).  Element i is register i % E of thread i / E (lane-major):
// inside a thread a comparator is one v_min and one v_max; a partner in
// another lane arrives by a DPP permute where gfx950 has the pattern, the
// LDS crossbar's swizzle within 32 lanes, or ds_bpermute across the halves,
// and one v_med3 against 0 or all ones keeps the smaller or the larger;
// in the block sort a partner in another wavefront comes through LDS.  The
// input order is free (the keys are distinct), so the states load striped
// and coalesced; the sorted slots go through LDS to a striped order, so the
// output is written coalesced too.
//   wave sort   one wavefront per bucket of at most kCdfTileSmall states
//               (nearly all), kWaveElems keys per lane, SB = kWaveSlotBits;
//   block sort  one block per larger bucket (up to kCdfBucketCap; they
//               appear in the first steps of a sweep from a point mass),
//               kBlockElems keys per thread, SB = kBlockSlotBits.
constexpr uint32_t kMaxTieRun = 32;
constexpr int kWave = 64;
constexpr int kSortWaves = 4;
constexpr int kSortThreads = kSortWaves * kWave;
constexpr int kWaveElems = kCdfTileSmall / kWave;
constexpr int kBlockElems = kCdfBucketCap / kSortThreads;
constexpr int kWaveSlotBits = 11;
constexpr int kBlockSlotBits = 12;
static_assert((1 << kWaveSlotBits) == kCdfTileSmall && (1 << kBlockSlotBits) == kCdfBucketCap, "slot fields");
static_assert(kWaveElems == 32 && kBlockElems == 16, "sort shapes");

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// The value of lane (this lane ^ M).
template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    const int x = (int)v;
    if constexpr (M == 1)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true); // quad_perm [1,0,3,2]
    else if constexpr (M == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true); // quad_perm [2,3,0,1]
    else if constexpr (M == 3)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, true); // quad_perm [3,2,1,0]
    else if constexpr (M == 7)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true); // row_half_mirror
    else if constexpr (M == 8)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, true); // row_ror:8
    else if constexpr (M == 15)
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true); // row_mirror
    else if constexpr (M < 32)
        return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x1F | (M << 10)); // bitmask mode: xor M
    else
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ M) << 2, x);
}
template <int M>
__device__ __forceinline__ uint64_t lane_xor(uint64_t v) {
    return (uint64_t)lane_xor<M>((uint32_t)v) | ((uint64_t)lane_xor<M>((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ uint32_t lane_read(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((src & (kWave - 1)) << 2, (int)v);
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uniform(uint64_t v) {
    return (uint64_t)uniform((uint32_t)v) | ((uint64_t)uniform((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }
// the median of three (one v_med3_u32): min(a, b) for c = 0, max(a, b) for c = ~0
__device__ __forceinline__ uint32_t med3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    const uint32_t m = hi < c ? hi : c;
    return lo < m ? m : lo;
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The wavefront's smallest and largest code among its threads' valid ones.
template <typename Code>
__device__ __forceinline__ void wave_min_max(Code &mn, Code &mx) {
#define MCPR_WAVE_MINMAX(M)                                                                                         \
    {                                                                                                               \
        const Code a = lane_xor<M>(mn), c = lane_xor<M>(mx);                                                        \
        mn = a < mn ? a : mn;                                                                                       \
        mx = c > mx ? c : mx;                                                                                       \
    }
    MCPR_WAVE_MINMAX(1)
    MCPR_WAVE_MINMAX(2)
    MCPR_WAVE_MINMAX(4)
    MCPR_WAVE_MINMAX(8)
    MCPR_WAVE_MINMAX(16)
    MCPR_WAVE_MINMAX(32)
#undef MCPR_WAVE_MINMAX
}

// The smallest shift s with span >> s below 2^(32 - SB) - 1.
template <int SB, typename Code>
__device__ __forceinline__ int key_shift(Code span) {
    constexpr Code lim = ((Code)1 << (32 - SB)) - 1;
    int s = 0;
    while ((span >> s) >= lim) ++s;
    return s;
}

// Order of two staged states inside a run: (code, previous position).
template <typename T>
struct RunKey {
    decltype(order_code(T())) c;
    uint32_t p;
    __device__ __forceinline__ bool operator<(const RunKey &o) const { return c < o.c || (c == o.c && p < o.p); }
};
template <typename T>
__device__ __forceinline__ RunKey<T> run_key(const T *__restrict__ su, const uint32_t *__restrict__ sp, uint32_t slot) {
    return RunKey<T>{order_code(ld_at(su, slot)), ld_at(sp, slot)};
}

// E packed keys per thread.
template <int E>
struct Keys {
    uint32_t a[E];
    __device__ __forceinline__ void ce(int r, int p) {
        const uint32_t x = a[r], y = a[p];
        a[r] = x < y ? x : y;
        a[p] = x < y ? y : x;
    }
    // with lane ^ M: register r against the partner's register r (or E-1-r).
    // A DPP permute is a VALU operation and feeds its comparator at once; the
    // LDS crossbar's have latency, so they are issued kBatch at a time before
    // their comparators.
    template <int M, bool MIRROR>
    __device__ __forceinline__ void cross(bool lower) {
        const uint32_t sel = lower ? 0u : ~0u;
        constexpr bool kDpp = M == 1 || M == 2 || M == 3 || M == 7 || M == 8 || M == 15;
        constexpr int kBatch = kDpp ? 2 : 8;
        static_assert(E % kBatch == 0, "batches");
        if constexpr (MIRROR) {
            // pairs (r, E-1-r) together: each needs the other's value from the partner lane
#pragma unroll
            for (int r0 = 0; r0 < E / 2; r0 += kBatch / 2) {
                uint32_t b[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch / 2; ++j) {
                    b[2 * j] = lane_xor<M>(a[E - 1 - (r0 + j)]);
                    b[2 * j + 1] = lane_xor<M>(a[r0 + j]);
                }
#pragma unroll
                for (int j = 0; j < kBatch / 2; ++j) {
                    a[r0 + j] = med3(a[r0 + j], b[2 * j], sel);
                    a[E - 1 - (r0 + j)] = med3(a[E - 1 - (r0 + j)], b[2 * j + 1], sel);
                }
            }
        } else {
#pragma unroll
            for (int r0 = 0; r0 < E; r0 += kBatch) {
                uint32_t b[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch; ++j) b[j] = lane_xor<M>(a[r0 + j]);
#pragma unroll
                for (int j = 0; j < kBatch; ++j) a[r0 + j] = med3(a[r0 + j], b[j], sel);
            }
        }
    }
};

// LDS of the block sort: one key per element of the network, one pad word
// every kBlockElems (so that a store of every lane at once touches distinct
// banks).
__device__ __forceinline__ int bpad(int i) { return i + i / kBlockElems; }
constexpr int kBlockLds = kCdfBucketCap + kCdfBucketCap / kBlockElems;

// Stages whose partner (i ^ MASK) lies in another wavefront of the block.
struct BlockExchange {
    uint32_t *key;
    template <int MASK, int E>
    __device__ __forceinline__ void stage(Keys<E> &k) const {
        const int i0 = (int)threadIdx.x * E;
#pragma unroll
        for (int r = 0; r < E; ++r) key[bpad(i0 + r)] = k.a[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int i = i0 + r, p = i ^ MASK;
            k.a[r] = med3(k.a[r], key[bpad(p)], i < p ? 0u : ~0u);
        }
        __syncthreads();
    }
};
struct NoExchange {};

// Half-cleaner stages J, J/2, ..., 1 of a merge level.
template <int E, int J, typename X>
__device__ __forceinline__ void half_cleaners(Keys<E> &k, int lane, const X &x) {
    if constexpr (J >= 1) {
        if constexpr (J < E) {
#pragma unroll
            for (int r = 0; r < E; ++r)
                if ((r & J) == 0) k.ce(r, r | J);
        } else if constexpr (J < kWave * E) {
            k.template cross<J / E, false>((lane & (J / E)) == 0);
        } else {
            x.template stage<J>(k);
        }
        half_cleaners<E, J / 2>(k, lane, x);
    }
}

// Merge levels K, 2K, ..., N of a network over N elements.
template <int E, int N, int K, typename X>
__device__ __forceinline__ void bitonic_levels(Keys<E> &k, int lane, const X &x) {
    if constexpr (K <= N) {
        if constexpr (K <= E) {
#pragma unroll
            for (int r = 0; r < E; ++r)
                if ((r & (K / 2)) == 0) k.ce(r, r ^ (K - 1));
        } else if constexpr (K <= kWave * E) {
            k.template cross<K / E - 1, true>((lane & (K / (2 * E))) == 0);
        } else {
            x.template stage<K - 1>(k);
        }
        half_cleaners<E, K / 4>(k, lane, x);
        bitonic_levels<E, N, 2 * K>(k, lane, x);
    }
}

// The wave sort's network, run order and output for one bucket: the slots go
// to LDS in lane-major order (E + 2 halfwords per lane, so that a store of
// every lane at once touches distinct banks) with one word per lane marking
// which of its elements equal their successor's q; then the runs, and the
// slots read back striped.
template <int E, int SB, typename T>
__device__ __forceinline__ void wave_sort(Keys<E> &k, uint32_t n, uint32_t dst, int lane, uint16_t *__restrict__ xp,
                                          uint32_t *__restrict__ eqw, const T *__restrict__ su,
                                          const uint32_t *__restrict__ sl, const uint32_t *__restrict__ sp,
                                          uint32_t *__restrict__ flag, T *__restrict__ ko,
                                          uint32_t *__restrict__ lo) {
    constexpr int kRow = E + 2;
    constexpr uint32_t kMask = (1u << SB) - 1u;
    bitonic_levels<E, kWave * E, 2>(k, lane, NoExchange());
    const uint32_t e0 = (uint32_t)lane * E;
    uint32_t eqn = 0; // bit r: element e0 + r has the q of element e0 + r + 1 (both below n)
#pragma unroll
    for (int r = 0; r < E; ++r) {
        xp[lane * kRow + r] = (uint16_t)(k.a[r] & kMask);
        if (r + 1 < E && e0 + r + 1 < n && (k.a[r] >> SB) == (k.a[r + 1] >> SB)) eqn |= 1u << r;
    }
    {
        const uint32_t next = lane_read(k.a[0], lane + 1);
        if (e0 + E < n && (k.a[E - 1] >> SB) == (next >> SB)) eqn |= 1u << (E - 1);
    }
    eqw[lane] = eqn;
    const uint32_t eqp = lane_read(eqn >> (E - 1), lane - 1) & (lane > 0 ? 1u : 0u);
    uint32_t starts = eqn & ~((eqn << 1) | eqp); // first elements of runs
    wave_sync();
    if (wave_any(starts != 0)) {
        bool bad = false;
        while (starts) {
            const uint32_t a0 = e0 + (uint32_t)__builtin_ctz(starts);
            starts &= starts - 1;
            uint32_t a1 = a0; // the run [a0, a1]
            while ((eqw[a1 / E] >> (a1 % E)) & 1u) {
                if (a1 - a0 >= kMaxTieRun) {
                    bad = true;
                    break;
                }
                ++a1;
            }
            if (bad) break;
            for (uint32_t a = a0 + 1; a <= a1; ++a) { // insertion sort by (code, previous position)
                const uint16_t sa = xp[(a / E) * kRow + a % E];
                const RunKey<T> ka = run_key(su, sp, sa);
                uint32_t q = a;
                while (q > a0) {
                    const uint16_t sb = xp[((q - 1) / E) * kRow + (q - 1) % E];
                    if (!(ka < run_key(su, sp, sb))) break;
                    xp[(q / E) * kRow + q % E] = sb;
                    --q;
                }
                xp[(q / E) * kRow + q % E] = sa;
            }
        }
        if (wave_any(bad)) {
            if (lane == 0) *flag = 1u;
            return;
        }
        wave_sync();
    }
    // Slot reads and gathers are unconditional (every index stays in the
    // bucket's LDS row and staging slots; padding rows hold slots too), so
    // that they are all in flight together; only the stores are predicated.
    T *__restrict__ kd = ko + dst;
    uint32_t *__restrict__ ld = lo + dst;
    uint32_t slot[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = (uint32_t)(r * kWave + lane);
        slot[r] = xp[(e / E) * kRow + e % E];
    }
    T val[E];
    uint32_t lab[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        val[r] = ld_at(su, slot[r]);
        lab[r] = ld_at(sl, slot[r]);
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t e = (uint32_t)(r * kWave + lane);
        if (e < n) {
            st_at(kd, e, val[r]);
            st_at(ld, e, lab[r]);
        }
    }
}

// Wave sort: one bucket per wavefront, kSortWaves per block.  A bucket above
// kCdfTileSmall goes on the list of k_cdf_bsort.
template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_cdf_wsort(const uint2 *__restrict__ bmeta, int nbuckets,
                                                            StageView<T> stage, uint32_t *__restrict__ defer,
                                                            uint32_t *__restrict__ flag, T *__restrict__ ko,
                                                            uint32_t *__restrict__ lo) {
    using Code = decltype(order_code(T()));
    constexpr int E = kWaveElems, SB = kWaveSlotBits;
    __shared__ uint16_t xpose[kSortWaves][kWave * (E + 2)];
    __shared__ uint32_t eqwords[kSortWaves][kWave];
    const int wave = (int)(threadIdx.x / kWave), lane = lane_id();
    const int b = (int)blockIdx.x * kSortWaves + wave;
    // Every decision below is taken per wavefront (values made uniform with
    // readfirstlane) and no wavefront waits for another, so a wavefront may
    // leave early.  A sweep with the flag set is redone: its buckets stop.
    if (b >= nbuckets) return;
    if (uniform(*flag)) return;
    const uint2 meta = bmeta[b]; // (first dense output position, states)
    const uint32_t dst = uniform(meta.x), n = uniform(meta.y);
    if (n == 0) return;
    if (n > (uint32_t)kCdfTileSmall) {
        if (lane == 0) defer[1u + atomicAdd(&defer[0], 1u)] = (uint32_t)b;
        return;
    }
    const size_t s0 = (size_t)b * kCdfBucketCap; // the bucket's first staging slot
    const T *__restrict__ su = stage.u + s0;
    const uint32_t *__restrict__ sl = stage.lab + s0;
    const uint32_t *__restrict__ sp = stage.pos + s0;
    // striped, coalesced loads without a branch (every slot below
    // kCdfBucketCap is the bucket's own; those at or past n are padding)
    Code code[E];
#pragma unroll
    for (int r = 0; r < E; ++r) code[r] = order_code(ld_at(su, (uint32_t)(r * kWave + lane)));
    Code mn = ~(Code)0, mx = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const Code pad = (Code)(int32_t)pad_mask((uint32_t)(r * kWave + lane), n); // (sign-extended)
        const Code lo_c = code[r] | pad, hi_c = code[r] & ~pad;
        mn = lo_c < mn ? lo_c : mn;
        mx = hi_c > mx ? hi_c : mx;
    }
    wave_min_max(mn, mx);
    mn = uniform(mn);
    mx = uniform(mx);
    const int sh = key_shift<SB>(mx - mn);
    Keys<E> k;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t t = (uint32_t)(r * kWave + lane);
        k.a[r] = (((uint32_t)((code[r] - mn) >> sh) << SB) | t) | pad_mask(t, n);
    }
    wave_sort<E, SB>(k, n, dst, lane, xpose[wave], eqwords[wave], su, sl, sp, flag, ko, lo);
}

// Block sort of the buckets on k_cdf_wsort's list (rare: most steps have
// none), one bucket per block at a time over a fixed grid of kDeferBlocks.
// Every thread of a block reads the same words, so the branches are uniform.
constexpr int kDeferBlocks = 256;

template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_cdf_bsort(const uint2 *__restrict__ bmeta,
                                                            const uint32_t *__restrict__ defer, StageView<T> stage,
                                                            uint32_t *__restrict__ flag, T *__restrict__ ko,
                                                            uint32_t *__restrict__ lo) {
    using Code = decltype(order_code(T()));
    constexpr int E = kBlockElems, SB = kBlockSlotBits;
    constexpr uint32_t kMask = (1u << SB) - 1u;
    __shared__ uint32_t lk[kBlockLds];
    __shared__ Code red[2 * kSortWaves];
    __shared__ uint32_t skip, count;
    // one thread reads the flag and the list's length; the whole block takes that decision
    if (threadIdx.x == 0) {
        skip = *flag;
        count = defer[0];
    }
    __syncthreads();
    if (skip) return;
    const int tid = (int)threadIdx.x, wave = tid / kWave, lane = lane_id();
    for (uint32_t q = blockIdx.x; q < count; q += gridDim.x) {
        const uint32_t bw = defer[1u + q];
        const uint2 meta = bmeta[bw];
        const uint32_t n = meta.y, dst = meta.x;
        if (n > (uint32_t)kCdfBucketCap) continue; // cannot happen unflagged; keeps LDS indices in range
        const size_t s0 = (size_t)bw * kCdfBucketCap;
        const T *__restrict__ su = stage.u + s0;
        const uint32_t *__restrict__ sl = stage.lab + s0;
        const uint32_t *__restrict__ sp = stage.pos + s0;
        Code code[E];
        Code mn = ~(Code)0, mx = 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t t = (uint32_t)(r * kSortThreads + tid);
            code[r] = order_code(su[t]);
            if (t < n) {
                mn = code[r] < mn ? code[r] : mn;
                mx = code[r] > mx ? code[r] : mx;
            }
        }
        wave_min_max(mn, mx);
        if (lane == 0) {
            red[2 * wave] = mn;
            red[2 * wave + 1] = mx;
        }
        __syncthreads();
        mn = red[0];
        mx = red[1];
        for (int v = 1; v < kSortWaves; ++v) {
            mn = red[2 * v] < mn ? red[2 * v] : mn;
            mx = red[2 * v + 1] > mx ? red[2 * v + 1] : mx;
        }
        const int sh = key_shift<SB>(mx - mn);
        Keys<E> k;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t t = (uint32_t)(r * kSortThreads + tid);
            k.a[r] = t < n ? ((uint32_t)((code[r] - mn) >> sh) << SB) | t : ~0u;
        }
        bitonic_levels<E, kCdfBucketCap, 2>(k, lane, BlockExchange{lk});
#pragma unroll
        for (int r = 0; r < E; ++r) lk[bpad(tid * E + r)] = k.a[r];
        __syncthreads();
        for (uint32_t i = (uint32_t)tid; i + 1 < n; i += kSortThreads) {
            const uint32_t q = lk[bpad(i)] >> SB;
            if ((lk[bpad(i + 1)] >> SB) != q || (i > 0 && (lk[bpad(i - 1)] >> SB) == q)) continue;
            uint32_t e = i + 1; // the run [i, e]
            bool bad = false;
            while (e + 1 < n && (lk[bpad(e + 1)] >> SB) == q) {
                if (e - i >= kMaxTieRun) {
                    bad = true;
                    break;
                }
                ++e;
            }
            if (bad) {
                *flag = 1u;
                continue;
            }
            for (uint32_t a = i + 1; a <= e; ++a) { // insertion sort by (code, previous position)
                const uint32_t ea = lk[bpad(a)];
                const RunKey<T> ka = run_key(su, sp, ea & kMask);
                uint32_t p = a;
                while (p > i) {
                    const uint32_t eb = lk[bpad(p - 1)];
                    if (!(ka < run_key(su, sp, eb & kMask))) break;
                    lk[bpad(p)] = eb;
                    --p;
                }
                lk[bpad(p)] = ea;
            }
        }
        __syncthreads();
        // (unconditional gathers, predicated stores, as in the wave sort)
        uint32_t slot[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t t = (uint32_t)(r * kSortThreads + tid);
            slot[r] = t < n ? lk[bpad((int)t)] & kMask : 0u;
        }
        T val[E];
        uint32_t lab[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            val[r] = su[slot[r]];
            lab[r] = sl[slot[r]];
        }
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t t = (uint32_t)(r * kSortThreads + tid);
            if (t < n) {
                ko[dst + t] = val[r];
                lo[dst + t] = lab[r];
            }
        }
        __syncthreads(); // the LDS is reused by the next bucket
    }
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
    hipLaunchKernelGGL(k_cdf_bscan, dim3(n_items), dim3(kThreads), 0, s, items, b.bcount, b.bmeta, b.defer, b.flag);
    const dim3 grid((b.nbuckets + kSortWaves - 1) / kSortWaves);
    if (prec == 0) {
        const StageView<double> st = stage_view<double>(b.stage, b.nbuckets);
        hipLaunchKernelGGL(k_cdf_wsort<double>, grid, dim3(kSortThreads), 0, s, b.bmeta, b.nbuckets, st, b.defer,
                           b.flag, (double *)b.keys[1], b.lab[1]);
        hipLaunchKernelGGL(k_cdf_bsort<double>, dim3(kDeferBlocks), dim3(kSortThreads), 0, s, b.bmeta, b.defer, st,
                           b.flag, (double *)b.keys[1], b.lab[1]);
    } else {
        const StageView<float> st = stage_view<float>(b.stage, b.nbuckets);
        hipLaunchKernelGGL(k_cdf_wsort<float>, grid, dim3(kSortThreads), 0, s, b.bmeta, b.nbuckets, st, b.defer,
                           b.flag, (float *)b.keys[1], b.lab[1]);
        hipLaunchKernelGGL(k_cdf_bsort<float>, dim3(kDeferBlocks), dim3(kSortThreads), 0, s, b.bmeta, b.defer, st,
                           b.flag, (float *)b.keys[1], b.lab[1]);
    }
    return hipGetLastError();
}

hipError_t launch_cdf_sort(int prec, int n_items, uint32_t n, const CdfBuffers &b, hipStream_t s) {
    return prec == 0 ? sorted<double>(n_items, n, b, s) : sorted<float>(n_items, n, b, s);
}

} // namespace mcpr
