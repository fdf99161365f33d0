// kernels.hip -- CDNA4 (gfx950) kernels of the fine propagator, the restriction
// and the matching operator.
//
// Layout: each ensemble is a contiguous SoA array of P values (fp32 or fp64).
// A block of 256 threads owns one superchunk of 256*R quads; thread t handles
// quads Q = sc*256*R + r*256 + t, so every r-row of the block is one fully
// coalesced 4 KB (fp32) or 8 KB (fp64) read and write.  Philox counters are
// per quad, so the 4 normals of a quad come from one Philox call in registers.
//
// The per-step mean field (population mean and variance, eq. general_equation)
// is a reduction over the whole ensemble.  Each step kernel writes one fp64
// partial (sum of x - shift, sum of (x - shift)^2) per superchunk; the next
// step's blocks combine the partials of their ensemble in a fixed order at
// start-up (kernel boundaries order the data; no atomics, no fences, no
// spinning).  The shift of the sums is the previous step's mean, so the
// one-pass variance does not cancel.
#include <limits>

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"
#include "rng.hpp"

namespace mcpr {

// ----------------------------------------------------------------------------
// Reductions in the canonical order
// ----------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over the 256 threads of a block: butterfly per wave, then (w0+w1)+(w2+w3).
// lds must hold 4*N doubles.  Every thread receives the result.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[wave * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = (lds[k] + lds[N + k]) + (lds[2 * N + k] + lds[3 * N + k]);
    __syncthreads();
}

// Lane 0's value of wave_sum with the same additions in the same order, from
// DPP permutes, one swizzle and one readlane instead of LDS-crossbar shuffles
// (where many wavefronts reduce at once they queue on the crossbar: the
// resident sweep's sixteen wavefronts on one CU, the restriction's million
// blocks).
// At each level lane 0 reads a lane whose partial equals that of its xor
// partner: after the levels below o, the lanes of each aligned group of o
// hold equal partials (every addition is commutative), so the half-row
// mirror (lane 7 - i) stands for xor 4; row rotation by 8 is xor 8.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
// Lane 0's sum over lanes 0..15 (the levels of the xor butterfly inside a row).
__device__ __forceinline__ double row_sum_lane0(double v) {
    v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]: xor 1
    v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]: xor 2
    v += dpp_f64<0x141>(v); // row_half_mirror: a lane of the partner quad
    v += dpp_f64<0x128>(v); // row_ror:8: xor 8
    return v;
}
__device__ __forceinline__ double wave_sum_lane0(double v) {
    v = row_sum_lane0(v);
    {
        const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F); // xor 16 within 32 lanes
        const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
        v += __hiloint2double(hi, lo);
    }
    {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), 32);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 32);
        v += __hiloint2double(hi, lo);
    }
    return v;
}

// block_sum with the lane-0 wave sums (the same bits).
template <int N>
__device__ __forceinline__ void block_sum_dpp(double (&v)[N], double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum_lane0(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[wave * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = (lds[k] + lds[N + k]) + (lds[2 * N + k] + lds[3 * N + k]);
    __syncthreads();
}

template <int N>
__device__ __forceinline__ void block_minmax(double (&mn)[N], double (&mx)[N], double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        mn[k] = wave_min(mn[k]);
        mx[k] = wave_max(mx[k]);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            lds[wave * 2 * N + k] = mn[k];
            lds[wave * 2 * N + N + k] = mx[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        mn[k] = fmin(fmin(lds[k], lds[2 * N + k]), fmin(lds[4 * N + k], lds[6 * N + k]));
        mx[k] = fmax(fmax(lds[N + k], lds[3 * N + k]), fmax(lds[5 * N + k], lds[7 * N + k]));
    }
    __syncthreads();
}

// Mean and variance from shifted sums over n particles.
__device__ __forceinline__ void finish_moments(double s1, double s2, double shift, double n, double &mean,
                                               double &var) {
    const double a = s1 / n;
    mean = shift + a;
    var = s2 / n - a * a;
    if (var < 0.0) var = 0.0;
}

// Ensemble total of the per-superchunk partials (thread t: s = t, t+256, ...).
__device__ __forceinline__ void ensemble_sums(const double2 *__restrict__ part, int nsc, double &S1, double &S2,
                                              double *lds) {
    double v[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < nsc; s += kThreads) {
        const double2 p = part[s];
        v[0] += p.x;
        v[1] += p.y;
    }
    block_sum<2>(v, lds);
    S1 = v[0];
    S2 = v[1];
}

// ----------------------------------------------------------------------------
// Quad load / store (16-byte aligned arrays; the tail quad goes element-wise)
// ----------------------------------------------------------------------------
__device__ __forceinline__ void load_quad(const float *__restrict__ x, int64_t p, int64_t P, float v[4]) {
    if (p + 3 < P) {
        const float4 q = *reinterpret_cast<const float4 *>(x + p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (p + e < P) ? x[p + e] : 0.0f;
    }
}
__device__ __forceinline__ void load_quad(const double *__restrict__ x, int64_t p, int64_t P, double v[4]) {
    if (p + 3 < P) {
        const double2 a = *reinterpret_cast<const double2 *>(x + p);
        const double2 b = *reinterpret_cast<const double2 *>(x + p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (p + e < P) ? x[p + e] : 0.0;
    }
}
__device__ __forceinline__ void store_quad(float *__restrict__ x, int64_t p, int64_t P, const float v[4]) {
    if (p + 3 < P) {
        *reinterpret_cast<float4 *>(x + p) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (p + e < P) x[p + e] = v[e];
    }
}
__device__ __forceinline__ void store_quad(double *__restrict__ x, int64_t p, int64_t P, const double v[4]) {
    if (p + 3 < P) {
        *reinterpret_cast<double2 *>(x + p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2 *>(x + p + 2) = make_double2(v[2], v[3]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (p + e < P) x[p + e] = v[e];
    }
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

// region index: number of boundaries <= x (ties go to the upper region)
template <int NREG>
__device__ __forceinline__ int region_of(double x, const Splits &sp) {
    int g = 0;
#pragma unroll
    for (int i = 0; i < NREG - 1; ++i) g += (x >= sp.s[i]) ? 1 : 0;
    return g;
}

// ----------------------------------------------------------------------------
// Canonical leaf of the per-step sums: one quad, d_e = x_e - shift formed in
// fp64 from the state value and the shift (a value of the state type, so in
// fp32 the difference of the two widened values is exact unless their
// exponents are more than 29 apart):
//   q1 = (d0 + d1) + (d2 + d3),   q2 = fma(d3, d3, fma(d2, d2, fma(d1, d1, d0 * d0)))
// Absent particles have d = 0.  Every sum over particles is fp64 from the
// particle up, in fp32-state mode as well.
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double leaf_diff(T x, T shift) {
    return (double)x - (double)shift;
}
__device__ __forceinline__ void quad_leaf(const double d[4], double &q1, double &q2) {
    q1 = (d[0] + d[1]) + (d[2] + d[3]);
    q2 = fma(d[3], d[3], fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0])));
}

// Vector access to one quad through the global address space (full quads).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) f32x4 g_f32x4;
typedef __attribute__((address_space(1))) f64x2 g_f64x2;

template <bool NT>
__device__ __forceinline__ void gload_quad(const float *base, uint32_t q, float v[4]) {
    const g_f32x4 *p = ((const g_f32x4 *)(base)) + q;
    const f32x4 a = NT ? __builtin_nontemporal_load(p) : *p;
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
template <bool NT>
__device__ __forceinline__ void gload_quad(const double *base, uint32_t q, double v[4]) {
    const g_f64x2 *p = ((const g_f64x2 *)(base)) + 2 * q;
    const f64x2 a = NT ? __builtin_nontemporal_load(p) : p[0];
    const f64x2 b = NT ? __builtin_nontemporal_load(p + 1) : p[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <bool NT>
__device__ __forceinline__ void gstore_quad(float *base, uint32_t q, const float v[4]) {
    f32x4 a;
    a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
    g_f32x4 *p = ((g_f32x4 *)(base)) + q;
    if (NT) __builtin_nontemporal_store(a, p); else *p = a;
}
template <bool NT>
__device__ __forceinline__ void gstore_quad(double *base, uint32_t q, const double v[4]) {
    f64x2 a, b;
    a.x = v[0]; a.y = v[1]; b.x = v[2]; b.y = v[3];
    g_f64x2 *p = ((g_f64x2 *)(base)) + 2 * q;
    if (NT) {
        __builtin_nontemporal_store(a, p);
        __builtin_nontemporal_store(b, p + 1);
    } else {
        p[0] = a;
        p[1] = b;
    }
}

// ----------------------------------------------------------------------------
// Step-0 sums: shift = x[0] (a value of the ensemble itself, so the result
// depends on the ensemble only)
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sum_init(const WorkItem *__restrict__ items,
                                                       const int2 *__restrict__ blocks,
                                                       double2 *__restrict__ part_out,
                                                       double *__restrict__ shift_out) {
    __shared__ double lds[8];
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x);
    const int64_t P = W.P;
    const int R = W.R;
    const T shift = x[0];
    double a1 = 0.0, a2 = 0.0;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    const T *xs = x + base;
    if (base + (int64_t)4 * kThreads * R <= P) {
        for (int r = 0; r < R; ++r) {
            T v[4];
            double d[4];
            gload_quad<false>(xs, (uint32_t)(r * kThreads + threadIdx.x), v);
#pragma unroll
            for (int e = 0; e < 4; ++e) d[e] = leaf_diff(v[e], shift);
            double q1, q2;
            quad_leaf(d, q1, q2);
            a1 += q1;
            a2 += q2;
        }
    } else {
        for (int r = 0; r < R; ++r) {
            const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
            if (p < P) {
                T v[4];
                double d[4];
                load_quad(x, p, P, v);
#pragma unroll
                for (int e = 0; e < 4; ++e) d[e] = (p + e < P) ? leaf_diff(v[e], shift) : 0.0;
                double q1, q2;
                quad_leaf(d, q1, q2);
                a1 += q1;
                a2 += q2;
            }
        }
    }
    double sm[2] = {a1, a2};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) {
        part_out[W.part_off + bt.y] = make_double2(sm[0], sm[1]);
        if (bt.y == 0) shift_out[bt.x] = (double)shift;
    }
}

// ----------------------------------------------------------------------------
// One Euler-Maruyama step of every ensemble of the launch (eq. Euler_Maruyama
// with the X_n term):  x <- x + a(x, m_j, v_j) dt + b(x, m_j, v_j) sqrt(dt) z,
// evaluated as  x <- fma(b sqrt(dt), z, p(x))  with  p(x) = x + a(x) dt  a
// cubic in x (DEG 3) or, when a2 = a3 = 0, a line (DEG 1; bitwise the same).
// ----------------------------------------------------------------------------
template <typename T, int DEG>
__device__ __forceinline__ T em_update(T xv, T z, T c0, T c1, T c2, T c3, T e0, T e1) {
    const T pol = (DEG == 1) ? fmaT(c1, xv, c0) : fmaT(fmaT(fmaT(c3, xv, c2), xv, c1), xv, c0);
    return fmaT(fmaT(e1, xv, e0), z, pol);
}

// Coefficients of step j from its mean field: p(x) = x + a(x) dt as a
// polynomial (c0..c3), the diffusion times sqrt(dt) affine in x (e0, e1).
template <typename T>
struct StepCoef {
    T c0, c1, c2, c3, e0, e1;
};
// The inputs of step_coef that stay fixed through a sweep (the item's
// coefficients a0 a1 a2 a3 am av b0 b1 bm bv axs, dt and sqrt(dt)).
struct StepIn {
    double c[11];
    double dt, sdt;
};
__device__ __forceinline__ StepIn step_in(const WorkItem &W) {
    StepIn k;
#pragma unroll
    for (int i = 0; i < 11; ++i) k.c[i] = W.c[i];
    k.dt = W.dt;
    k.sdt = W.sdt;
    return k;
}
template <typename T>
__device__ __forceinline__ StepCoef<T> step_coef(const StepIn &W, double mean, double var) {
    const double dt = W.dt, sdt = W.sdt;
    StepCoef<T> k;
    k.c0 = (T)((W.c[0] + W.c[4] * mean + W.c[5] * var) * dt);
    k.c1 = (T)(1.0 + (W.c[1] + W.c[10] * (var + mean * mean)) * dt);
    k.c2 = (T)(W.c[2] * dt);
    k.c3 = (T)(W.c[3] * dt);
    k.e0 = (T)((W.c[6] + W.c[8] * mean + W.c[9] * var) * sdt);
    k.e1 = (T)(W.c[7] * sdt);
    return k;
}
template <typename T>
__device__ __forceinline__ StepCoef<T> step_coef(const WorkItem &W, double mean, double var) {
    return step_coef<T>(step_in(W), mean, var);
}

// Mean field of step j from the previous launch's partials: one block per item
// (the variant of the step kernel that does not combine in every block).
__global__ __launch_bounds__(kThreads) void k_combine(const WorkItem *__restrict__ items,
                                                      const double2 *__restrict__ part_in,
                                                      const double *__restrict__ shift_in,
                                                      double2 *__restrict__ mv_out) {
    __shared__ double lds[8];
    const WorkItem &W = items[blockIdx.x];
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    double mean, var;
    finish_moments(S1, S2, shift_in[blockIdx.x], (double)W.P, mean, var);
    if (threadIdx.x == 0) mv_out[blockIdx.x] = make_double2(mean, var);
}

// NT: non-temporal loads and stores of the state.  MV: the mean field comes
// from k_combine (mv_in) instead of each block combining the partials itself;
// both give the same bits (same order, same operations).
template <typename T, int DEG, bool NT, bool MV>
__global__ __launch_bounds__(kThreads) void k_em_step(const WorkItem *__restrict__ items,
                                                      const int2 *__restrict__ blocks, int32_t j,
                                                      const double2 *__restrict__ part_in,
                                                      const double *__restrict__ shift_in,
                                                      const double2 *__restrict__ mv_in,
                                                      double2 *__restrict__ part_out,
                                                      double *__restrict__ shift_out,
                                                      double2 *__restrict__ trace, int32_t m) {
    __shared__ double lds[8];
    const int2 bt = blocks[blockIdx.x];
    const int item = bt.x, sc = bt.y;
    const WorkItem &W = items[item];
    T *__restrict__ x = reinterpret_cast<T *>(W.x) + (int64_t)j * W.traj;
    T *__restrict__ y = x + W.traj; // the output state (the input itself when in place)
    const int64_t P = W.P;
    const int R = W.R;

    // a full superchunk's quads (R <= 4 per thread) do not depend on the mean
    // field: issue their loads before the combine so the two latencies overlap
    const int64_t base = (int64_t)sc * 4 * kThreads * R; // first particle of the superchunk
    const bool full = base + (int64_t)4 * kThreads * R <= P;
    T v[kMaxQuadsPerThread][4];
    if (full) {
#pragma unroll
        for (int g = 0; g < kMaxQuadsPerThread; ++g)
            if (g < R) gload_quad<NT>(x + base, (uint32_t)(g * kThreads + threadIdx.x), v[g]);
    }

    // mean field at the start of the step
    double mean, var;
    if (MV) {
        const double2 mvv = mv_in[item];
        mean = mvv.x;
        var = mvv.y;
    } else {
        double S1, S2;
        ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
        finish_moments(S1, S2, shift_in[item], (double)P, mean, var);
    }
    const T shift = (T)mean; // shift of this step's output sums, a value of the state type
    if (sc == 0 && threadIdx.x == 0) {
        shift_out[item] = (double)shift;
        if (trace) trace[(int64_t)item * (m + 1) + j] = make_double2(mean, var);
    }

    const StepCoef<T> kc = step_coef<T>(W, mean, var);
    const T c0 = kc.c0, c1 = kc.c1, c2 = kc.c2, c3 = kc.c3, e0 = kc.e0, e1 = kc.e1;
    const uint32_t step = (uint32_t)(W.step0 + j);
    const uint32_t inst = (uint32_t)W.inst;
    const uint32_t k0 = W.key0, k1 = W.key1;

    double a1 = 0.0, a2 = 0.0;
    if (full) {
        // full superchunk: 32-bit quad offsets, no per-quad checks
        T *ys = y + base;
        const uint32_t qb = (uint32_t)(base >> 2) + threadIdx.x;
#pragma unroll
        for (int g = 0; g < kMaxQuadsPerThread; ++g) {
            if (g < R) {
                const Words4 w = philox4x32_10(qb + (uint32_t)(g * kThreads), step, inst, 0u, k0, k1);
                T z[4];
                double d[4];
                box_muller4(w, z);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[g][e] = em_update<T, DEG>(v[g][e], z[e], c0, c1, c2, c3, e0, e1);
                    d[e] = leaf_diff(v[g][e], shift);
                }
                gstore_quad<NT>(ys, (uint32_t)(g * kThreads + threadIdx.x), v[g]);
                double q1, q2;
                quad_leaf(d, q1, q2);
                a1 += q1;
                a2 += q2;
            }
        }
    } else {
        // the ensemble's last superchunk: per-quad and per-particle bounds
        for (int r = 0; r < R; ++r) {
            const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
            if (p < P) {
                T v[4], z[4];
                double d[4];
                load_quad(x, p, P, v);
                const Words4 w = philox4x32_10((uint32_t)(p >> 2), step, inst, 0u, k0, k1);
                box_muller4(w, z);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = em_update<T, DEG>(v[e], z[e], c0, c1, c2, c3, e0, e1);
                    d[e] = (p + e < P) ? leaf_diff(v[e], shift) : 0.0;
                }
                store_quad(y, p, P, v);
                double q1, q2;
                quad_leaf(d, q1, q2);
                a1 += q1;
                a2 += q2;
            }
        }
    }
    double sm[2] = {a1, a2};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) part_out[W.part_off + sc] = make_double2(sm[0], sm[1]);
}

// ----------------------------------------------------------------------------
// Resident fine sweep of small ensembles (at most kResidentMaxP particles,
// canonical superchunks of one quad per thread): one block of
// kResidentThreads per ensemble keeps its particles in registers through all
// m steps of the sweep, so a step costs one block barrier instead of a
// launch.  Wavefront s of the block holds superchunk s, lane l its quads
// 256 s + 4 l + r (r = 0..3): the lane's four quad leaves are the leaves
// 4l .. 4l+3 of the superchunk's canonical tree, so the lane adds its two
// lowest levels, (u0 + u1) + (u2 + u3), and the wave's lane-0 sum adds the
// six above them -- the complete pairwise tree over the superchunk's 256
// thread sums, as the per-step launches form it (every addition is
// commutative, so the order of the two operands does not change a bit).
// Every wavefront that holds a superchunk then adds the ensemble tree itself
// (the same bits in each).  The sweep therefore gives the per-step launches'
// bits with a quarter of their reduction work per quad.
// The normals, which depend on the particle, the step and the instance only,
// are drawn for the whole sweep beforehand by k_sweep_normals (the
// transcendental work of every step in one launch wide enough to fill the
// chip) into z, laid out so that every load of the sweep is coalesced: item
// i's normal e of quad 256 s + 4 l + r at step j is
//   z[zoff_i + 1024 nsc_i j + 4 (64 nsc_i r + 64 s + l) + e].
// ----------------------------------------------------------------------------
constexpr int kResidentThreads = 64 * kResidentMaxSc;
static_assert(kResidentMaxP < kSmallEnsemble, "one quad per thread and superchunk");

// Quad index of (r, s, l) in one step's normals of an item with nsc superchunks.
__device__ __forceinline__ uint32_t resident_zquad(int r, int s, int l, int nsc) {
    return (uint32_t)(64 * nsc * r + 64 * s + l);
}

// grid (superchunk blocks of the launch, m): one quad per thread
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sweep_normals(const WorkItem *__restrict__ items,
                                                            const int2 *__restrict__ blocks, T *__restrict__ z) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const int32_t j = (int32_t)blockIdx.y;
    const uint32_t nq = (uint32_t)((W.P + 3) / 4);
    const int r = (int)threadIdx.x >> 6, l = (int)threadIdx.x & 63;
    const uint32_t q = (uint32_t)bt.y * kThreads + 4u * (uint32_t)l + (uint32_t)r;
    if (q >= nq) return;
    const Words4 w = philox4x32_10(q, (uint32_t)(W.step0 + j), (uint32_t)W.inst, 0u, W.key0, W.key1);
    T zz[4];
    box_muller4(w, zz);
    gstore_quad<false>(z + W.zoff + (int64_t)j * 4 * kThreads * W.nsc, resident_zquad(r, bt.y, l, W.nsc), zz);
}

// The lane's part of a superchunk's sums: the two lowest levels of the
// canonical tree over the thread sums of its four quads, which are 0.0 + the
// quad's leaf (0.0 past the ensemble).  The leaf q2 is never -0.0, so 0.0 + q2
// = q2; a tree over the q1 themselves differs from the tree over 0.0 + q1 at
// most by the sign of a zero result (a -0.0 where the canonical sum is +0.0),
// which the lane's final + 0.0 removes, so a1 and a2 carry the canonical bits.
// FULL: every particle of the lane's quads exists (all but the ensemble's
// last wavefront), so no test is made.
template <bool FULL, typename T>
__device__ __forceinline__ void resident_leaves(const T (&v)[4][4], T shift, uint32_t q0, uint32_t nq, int64_t P,
                                                double &a1, double &a2) {
    double u1[4], u2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t q = q0 + (uint32_t)r;
        if (FULL || q < nq) {
            double d[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) d[e] = leaf_diff(v[r][e], shift);
            if (!FULL && 4 * (int64_t)q + 4 > P) { // the ensemble's ragged last quad
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * (int64_t)q + e >= P) d[e] = 0.0;
            }
            quad_leaf(d, u1[r], u2[r]);
        } else {
            u1[r] = 0.0;
            u2[r] = 0.0;
        }
    }
    a1 = ((u1[0] + u1[1]) + (u1[2] + u1[3])) + 0.0;
    a2 = (u2[0] + u2[1]) + (u2[2] + u2[3]);
}

// One step of the lane's quads with normals zc, then its part of the sums
// (full: every particle of the wavefront's quads exists, which holds for all
// but the ensemble's last wavefront).
template <typename T, int DEG>
__device__ __forceinline__ void resident_advance(T (&v)[4][4], const T (&zc)[4][4], const T (&k)[6], T shift,
                                                 uint32_t q0, uint32_t nq, int64_t P, bool full, double &a1,
                                                 double &a2) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (q0 + r < nq) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[r][e] = em_update<T, DEG>(v[r][e], zc[r][e], k[0], k[1], k[2], k[3], k[4], k[5]);
        }
    if (full)
        resident_leaves<true>(v, shift, q0, nq, P, a1, a2);
    else
        resident_leaves<false>(v, shift, q0, nq, P, a1, a2);
}

// The per-step exchange of the resident block.  Wavefront s < nsc completes
// superchunk s's sums into ps[s]; after the one barrier every wavefront that
// holds a superchunk forms the ensemble sums, the mean field and the step
// coefficients itself (the same operations on the same values in every
// wavefront, so the same bits; no second barrier to publish them).  ps
// alternates between two buffers from one exchange to the next: a wavefront
// that starts writing exchange e + 1's sums may still find another reading
// exchange e's, but none can reach exchange e + 2 before every wavefront has
// passed the barrier of e + 1.  The ensemble sums follow the canonical tree:
// thread t of the 256-thread ensemble tree holds 0.0 + superchunk t's sums
// (t < nsc <= 16) and 0.0 beyond, so the wavefront tree over lanes 0..63 is
// the tree over lanes 0..15 (row_sum_lane0) plus two all-zero subtrees, and
// the three other wavefronts add (w0 + 0) + (0 + 0).
template <typename T>
struct ResidentField {
    double mean, var; // at the start of the next step
    T k[6];           // its c0 c1 c2 c3 e0 e1
};
static_assert(kResidentMaxSc <= 16, "the ensemble tree below covers 16 superchunks");
__device__ __forceinline__ double lane0_value(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 0);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 0);
    return __hiloint2double(hi, lo);
}
template <typename T>
__device__ __forceinline__ void resident_exchange(const StepIn &cin, double Pd, double a1, double a2, int nsc,
                                                  double shd, double (*ps)[2], ResidentField<T> &f) {
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    if (s < nsc) {
        const double w1 = wave_sum_lane0(a1), w2 = wave_sum_lane0(a2);
        if (lane == 0) {
            ps[s][0] = w1;
            ps[s][1] = w2;
        }
    }
    __syncthreads();
    if (s < nsc) {
        double t1 = 0.0, t2 = 0.0;
        if (lane < nsc) {
            t1 += ps[lane][0];
            t2 += ps[lane][1];
        }
        t1 = lane0_value(row_sum_lane0(t1));
        t2 = lane0_value(row_sum_lane0(t2));
        const double e1 = (t1 + 0.0) + 0.0, e2 = (t2 + 0.0) + 0.0; // lanes 16..31, then 32..63
        const double S1 = (e1 + 0.0) + (0.0 + 0.0), S2 = (e2 + 0.0) + (0.0 + 0.0);
        finish_moments(S1, S2, shd, Pd, f.mean, f.var);
        const StepCoef<T> k = step_coef<T>(cin, f.mean, f.var);
        f.k[0] = k.c0;
        f.k[1] = k.c1;
        f.k[2] = k.c2;
        f.k[3] = k.c3;
        f.k[4] = k.e0;
        f.k[5] = k.e1;
    }
}

// One block per item (in place, no trajectory).  Writes the final state, the
// last step's superchunk partials and shift (as the per-step launches leave
// them) and the trace entries 0..m-1.
template <typename T, int DEG>
__global__ __launch_bounds__(kResidentThreads) void k_em_sweep_resident(const WorkItem *__restrict__ items,
                                                                        const T *__restrict__ z, int32_t m,
                                                                        double2 *__restrict__ part_out,
                                                                        double *__restrict__ shift_out,
                                                                        double2 *__restrict__ trace) {
    __shared__ double psum[2][kResidentMaxSc][2];
    const WorkItem &W = items[blockIdx.x];
    T *__restrict__ x = reinterpret_cast<T *>(W.x);
    const int64_t P = W.P;
    const uint32_t nq = (uint32_t)((P + 3) / 4);
    const int nsc = W.nsc;
    // s is uniform in the wavefront: scalar branches on it
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), l = (int)threadIdx.x & 63;
    const uint32_t q0 = (uint32_t)s * kThreads + 4u * (uint32_t)l;
    const bool full = (int64_t)(s + 1) * 4 * kThreads <= P;
    const StepIn cin = step_in(W);
    const double Pd = (double)P;
    T v[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (q0 + r < nq) {
            load_quad(x, 4 * (int64_t)(q0 + r), P, v[r]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r][e] = (T)0;
        }
    }
    const T *__restrict__ zi = z + W.zoff;
    const int64_t zstep = (int64_t)4 * kThreads * nsc;
    // the step-0 sums, about x[0]
    const T shift0 = x[0];
    double a1, a2;
    resident_leaves<false>(v, shift0, q0, nq, P, a1, a2);
    double shd = (double)shift0;
    // The normals' loads are issued unconditionally, whole steps ahead of
    // their use, and no store is issued between them except every 64 steps,
    // so that the wait for one step's normals does not also wait for the
    // next step's (a conditional load or an interleaved store makes the
    // compiler wait for every load in flight).  A quad past the ensemble
    // reads an unused normal of its own superchunk, a wavefront past the
    // last superchunk superchunk 0's, the last step its own normals again.
    const int sz = s < nsc ? s : 0;
    T za[4][4], zb[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) gload_quad<false>(zi, resident_zquad(r, sz, l, nsc), za[r]);
    ResidentField<T> f = {}; // (wavefronts past the last superchunk keep these zeros)
    resident_exchange<T>(cin, Pd, a1, a2, nsc, shd, psum[0], f);
    // the trace entries of 64 steps, lane j % 64 of wavefront 0 holding step j's
    double tm = 0.0, tv = 0.0;
    // step j with its normals zc; the next step's normals go into zn, in
    // flight through this step's barrier
    auto step = [&](int32_t j, const T (&zc)[4][4], T (&zn)[4][4]) {
        const double mean = f.mean;
        if (trace && s == 0) {
            if (l == (j & 63)) {
                tm = mean;
                tv = f.var;
            }
            if ((j & 63) == 63 || j + 1 == m) {
                if (l <= (j & 63)) trace[(int64_t)blockIdx.x * (m + 1) + (j & ~63) + l] = make_double2(tm, tv);
            }
        }
        const T shift = (T)mean;
        T k[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) k[i] = f.k[i];
        {
            const T *__restrict__ zr = zi + (int64_t)(j + 1 < m ? j + 1 : j) * zstep;
#pragma unroll
            for (int r = 0; r < 4; ++r) gload_quad<false>(zr, resident_zquad(r, sz, l, nsc), zn[r]);
        }
        resident_advance<T, DEG>(v, zc, k, shift, q0, nq, P, full, a1, a2);
        shd = (double)shift;
        resident_exchange<T>(cin, Pd, a1, a2, nsc, shd, psum[(j + 1) & 1], f);
    };
    int32_t j = 0;
    for (; j + 1 < m; j += 2) {
        step(j, za, zb);
        step(j + 1, zb, za);
    }
    if (j < m) step(j, za, zb);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (q0 + r < nq) store_quad(x, 4 * (int64_t)(q0 + r), P, v[r]);
    if (threadIdx.x < (unsigned)nsc) {
        const double *pl = psum[m & 1][threadIdx.x]; // the last exchange's
        part_out[W.part_off + (int)threadIdx.x] = make_double2(pl[0], pl[1]);
    }
    if (threadIdx.x == 0) shift_out[blockIdx.x] = shd;
}

// ----------------------------------------------------------------------------
// Trigonometric mean field (plane rotator, Sec. 5.1): the drift
//   a(x) = a0 + a1 x + a2 x^2 + a3 x^3 + ksin sin x + kc (1/P) sum_q sin(X_q - x)
// with (1/P) sum_q sin(X_q - x) = S cos x - C sin x, S and C the population
// means of sin X and cos X.  The per-step mean field is (S, C): every launch
// writes per-superchunk partials (sum sin x, sum cos x) of its output in the
// canonical order (sin and cos in the state type, summed in fp64), and
// the next launch combines them.  wrap: x <- x - 2 pi floor(x / (2 pi)).
// ----------------------------------------------------------------------------
__device__ __forceinline__ void sincos_T(float x, float &s, float &c) {
    const float t = x * 0.15915494309189535f; // turns: v_sin_f32 / v_cos_f32 take sin(2 pi t)
    s = __builtin_amdgcn_sinf(t);
    c = __builtin_amdgcn_cosf(t);
}
__device__ __forceinline__ void sincos_T(double x, double &s, double &c) { sincos(x, &s, &c); }
__device__ __forceinline__ float wrap_T(float x) {
    const float tp = 6.28318530717958648f;
    return x - tp * floorf(x / tp);
}
__device__ __forceinline__ double wrap_T(double x) {
    const double tp = 6.283185307179586;
    return x - tp * floor(x / tp);
}

template <typename T>
__device__ __forceinline__ void trig_leaf(const T v[4], int64_t p, int64_t P, double &q1, double &q2) {
    T s[4], c[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        sincos_T(v[e], s[e], c[e]);
        if (p + e >= P) s[e] = c[e] = (T)0;
    }
    q1 = ((double)s[0] + (double)s[1]) + ((double)s[2] + (double)s[3]);
    q2 = ((double)c[0] + (double)c[1]) + ((double)c[2] + (double)c[3]);
}

// Step-0 trigonometric sums of each superchunk.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_sum_init_trig(const WorkItem *__restrict__ items,
                                                            const int2 *__restrict__ blocks,
                                                            double2 *__restrict__ part_out,
                                                            double *__restrict__ shift_out) {
    __shared__ double lds[8];
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x);
    const int64_t P = W.P;
    const int R = W.R;
    double a1 = 0.0, a2 = 0.0;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    for (int r = 0; r < R; ++r) {
        const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
        if (p < P) {
            T v[4];
            load_quad(x, p, P, v);
            double q1, q2;
            trig_leaf(v, p, P, q1, q2);
            a1 += q1;
            a2 += q2;
        }
    }
    double sm[2] = {a1, a2};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) {
        part_out[W.part_off + bt.y] = make_double2(sm[0], sm[1]);
        if (bt.y == 0) shift_out[bt.x] = 0.0;
    }
}

// One Euler-Maruyama step with the trigonometric mean field.
template <typename T, int DEG>
__global__ __launch_bounds__(kThreads) void k_em_step_trig(const WorkItem *__restrict__ items,
                                                           const int2 *__restrict__ blocks, int32_t j,
                                                           const double2 *__restrict__ part_in,
                                                           double2 *__restrict__ part_out,
                                                           double *__restrict__ shift_out,
                                                           double2 *__restrict__ trace, int32_t m) {
    __shared__ double lds[8];
    const int2 bt = blocks[blockIdx.x];
    const int item = bt.x, sc = bt.y;
    const WorkItem &W = items[item];
    T *__restrict__ x = reinterpret_cast<T *>(W.x) + (int64_t)j * W.traj;
    T *__restrict__ y = x + W.traj;
    const int64_t P = W.P;
    const int R = W.R;
    const int64_t base = (int64_t)sc * 4 * kThreads * R;
    T v[kMaxQuadsPerThread][4];
#pragma unroll
    for (int g = 0; g < kMaxQuadsPerThread; ++g) {
        const int64_t p = base + 4 * (int64_t)(g * kThreads + threadIdx.x);
        if (g < R && p < P) load_quad(x, p, P, v[g]);
    }
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    const double Sm = S1 / (double)P, Cm = S2 / (double)P;
    if (sc == 0 && threadIdx.x == 0) {
        shift_out[item] = 0.0;
        if (trace) trace[(int64_t)item * (m + 1) + j] = make_double2(Sm, Cm);
    }
    const double dt = W.dt, sdt = W.sdt;
    const T c0 = (T)(W.c[0] * dt);
    const T c1 = (T)(1.0 + W.c[1] * dt), c2 = (T)(W.c[2] * dt), c3 = (T)(W.c[3] * dt);
    const T ks = (T)((W.c[11] - W.c[12] * Cm) * dt), kcs = (T)(W.c[12] * Sm * dt);
    const T e0 = (T)(W.c[6] * sdt), e1 = (T)(W.c[7] * sdt);
    const uint32_t step = (uint32_t)(W.step0 + j);
    const uint32_t inst = (uint32_t)W.inst;
    double a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int g = 0; g < kMaxQuadsPerThread; ++g) {
        const int64_t p = base + 4 * (int64_t)(g * kThreads + threadIdx.x);
        if (g < R && p < P) {
            const Words4 w = philox4x32_10((uint32_t)(p >> 2), step, inst, 0u, W.key0, W.key1);
            T z[4], u[4];
            box_muller4(w, z);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T sx, cx;
                sincos_T(v[g][e], sx, cx);
                const T xv = v[g][e];
                const T pol0 = (DEG == 1) ? fmaT(c1, xv, c0) : fmaT(fmaT(fmaT(c3, xv, c2), xv, c1), xv, c0);
                const T pol = fmaT(kcs, cx, fmaT(ks, sx, pol0));
                u[e] = fmaT(fmaT(e1, v[g][e], e0), z[e], pol);
                if (W.wrap) u[e] = wrap_T(u[e]);
            }
            store_quad(y, p, P, u);
            double q1, q2;
            trig_leaf(u, p, P, q1, q2);
            a1 += q1;
            a2 += q2;
        }
    }
    double sm[2] = {a1, a2};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) part_out[W.part_off + sc] = make_double2(sm[0], sm[1]);
}

template <typename T>
__device__ __forceinline__ T normal_pick(const Words4 &w, int e);
template <>
__device__ __forceinline__ double normal_pick<double>(const Words4 &w, int e) { return normal_of(w, e); }
template <>
__device__ __forceinline__ float normal_pick<float>(const Words4 &w, int e) { return normal_of_f(w, e); }

// Sorted pairs of one item: separate key and label arrays, or packed pairs.
template <typename T, bool PACKED>
struct SortedView;
template <typename T>
struct SortedView<T, false> {
    const T *__restrict__ K;
    const uint32_t *__restrict__ L;
    __device__ __forceinline__ T key(int64_t r) const { return K[r]; }
    __device__ __forceinline__ uint32_t label(int64_t r) const { return L[r]; }
    __device__ __forceinline__ SortedView at(int64_t d) const { return SortedView{K + d, L + d}; }
};
template <typename T>
struct SortedView<T, true> {
    const KeyLabel<T> *__restrict__ S;
    __device__ __forceinline__ T key(int64_t r) const { return S[r].k; }
    __device__ __forceinline__ uint32_t label(int64_t r) const { return S[r].l; }
    __device__ __forceinline__ SortedView at(int64_t d) const { return SortedView{S + d}; }
};

// First (DIR < 0) or last (DIR > 0) position of the run of keys equal to v
// that contains position r of the ascending keys [0, P): doubling steps away
// from r while the key still equals v, then bisection of the last step.
template <int DIR, typename V, typename T>
__device__ __forceinline__ int64_t run_end(const V &S, int64_t P, int64_t r, T v) {
    int64_t known = r, step = 1;
    for (;;) {
        const int64_t probe = known + DIR * step;
        if (probe < 0 || probe >= P || S.key(probe) != v) break;
        known = probe;
        step <<= 1;
    }
    // S.key(known) == v; the position `step` beyond it is outside [0, P) or differs
    int64_t out = known + DIR * step;
    out = out < -1 ? -1 : (out > P ? P : out);
    while ((out - known) * DIR > 1) {
        const int64_t mid = known + (out - known) / 2;
        if (S.key(mid) == v)
            known = mid;
        else
            out = mid;
    }
    return known;
}

// Bucket of a new state u: the largest k in [0, nbk) with k == 0 or
// split(k) <= u, where split(k) is the sorted input's key at position
// k * kCdfBucket; searched from k0 (the bucket of the state's old position)
// by doubling steps, then bisection.
template <typename V, typename T>
__device__ __forceinline__ int bucket_of(const V &S, int nbk, int k0, T u) {
    auto ok = [&](int k) { return k == 0 || S.key((uint32_t)k * (uint32_t)kCdfBucket) <= u; };
    int lo, hi; // ok(lo), !ok(hi) (hi == nbk: past the end)
    if (ok(k0)) {
        lo = k0;
        int step = 1;
        while (lo + step < nbk && ok(lo + step)) {
            lo += step;
            step <<= 1;
        }
        hi = lo + step < nbk ? lo + step : nbk;
    } else {
        hi = k0;
        int step = 1;
        while (hi - step >= 1 && !ok(hi - step)) {
            hi -= step;
            step <<= 1;
        }
        lo = hi - step >= 1 ? hi - step : 0;
    }
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        if (ok(mid))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One Euler-Maruyama step with the empirical-CDF drift term acdf (1 - F_P(x)),
// taken in the ensemble's ascending order (the sorted pairs: state and label
// doff + p); the mean field of the input comes from k_combine.  Position r has sum_q H(x - X_q) = lo + (hi - lo + 1) / 2 for the
// run [lo, hi] of keys equal to its key (distinct neighbours: r + 1/2).
// Particle p's normal is normal p & 3 of Philox quad p >> 2, as in the
// particle-order steps.  The new state goes (mode 0) with its label to
// position r of keys[0] / lab[0], the next library sort's input; (mode 1)
// into its bucket, with a slot taken by one atomic per bucket and wave; or
// (mode 2, the last step of a sweep) to the particle's slot y[p], unless a
// bucket of the sweep overflowed (the sweep is then redone).  The (m, v)
// partials of the new states are summed in sorted order.
template <typename T, int DEG, bool PACKED>
__global__ __launch_bounds__(kThreads) void k_em_step_sorted(const WorkItem *__restrict__ items,
                                                             const int2 *__restrict__ blocks, int32_t j, int32_t mode,
                                                             const double2 *__restrict__ mv_in,
                                                             SortedView<T, PACKED> all, T *__restrict__ ko,
                                                             uint32_t *__restrict__ lo_out,
                                                             uint32_t *__restrict__ bcount, StageView<T> stage,
                                                             uint32_t *__restrict__ flag,
                                                             double2 *__restrict__ part_out,
                                                             double *__restrict__ shift_out,
                                                             double2 *__restrict__ trace, int32_t m) {
    // mode 1: a round's states (4 * kThreads neighbours in the previous
    // order) fall into buckets near the one of their first position; kWin
    // buckets around it are counted in LDS, reserved with one atomic each,
    // and the states grouped by bucket in LDS and copied out coalesced
    constexpr int kWin = 128, kBelow = 64, kRound = 4 * kThreads;
    static_assert(kWin == 2 * 64 && kWin <= kThreads, "one wave scans the window, two buckets per lane");
    __shared__ double lds[8];
    __shared__ uint32_t hist[kWin], hbase[kWin], lstart[kWin + 1];
    __shared__ T spl[kWin + 1]; // the window's splitters (-inf below bucket 1, +inf past the item)
    __shared__ T su[kRound];
    __shared__ uint32_t sl[kRound], sp[kRound];
    __shared__ uint8_t sw[kRound];
    // A doomed sweep (redone): skip its work, keep the input state.  Blocks
    // of this launch may set the flag while this one starts, so one thread
    // reads it and the whole block takes that one decision.
    if (mode != 0) {
        __shared__ uint32_t skip;
        if (threadIdx.x == 0) skip = *flag;
        __syncthreads();
        if (skip) return;
    }
    const int2 bt = blocks[blockIdx.x];
    const int item = bt.x, sc = bt.y;
    const WorkItem &W = items[item];
    T *__restrict__ y = reinterpret_cast<T *>(W.x);
    const SortedView<T, PACKED> S = all.at(W.doff); // this item's pairs
    // item-relative positions fit 32 bits (a launch holds fewer than 2^32 states)
    const uint32_t P = (uint32_t)W.P;
    const int R = W.R;
    const uint32_t base = (uint32_t)sc * 4u * kThreads * (uint32_t)R;
    if (mode == 1) {
        if (threadIdx.x < kWin) hist[threadIdx.x] = 0u;
        __syncthreads();
    }
    const double2 mvv = mv_in[item]; // the step's mean field, from k_combine
    const double mean = mvv.x, var = mvv.y;
    const T shift = (T)mean;
    if (sc == 0 && threadIdx.x == 0) {
        shift_out[item] = (double)shift;
        if (trace) trace[(int64_t)item * (m + 1) + j] = make_double2(mean, var);
    }
    const double dt = W.dt, sdt = W.sdt;
    const T c0 = (T)((W.c[0] + W.c[13]) * dt);
    const T c1 = (T)(1.0 + W.c[1] * dt), c2 = (T)(W.c[2] * dt), c3 = (T)(W.c[3] * dt);
    const T kf = (T)(-W.c[13] * dt / (double)P); // the CDF term: acdf dt (1 - cnt / P)
    const T e0 = (T)(W.c[6] * sdt), e1 = (T)(W.c[7] * sdt);
    const uint32_t step = (uint32_t)(W.step0 + j);
    const uint32_t inst = (uint32_t)W.inst;
    double a1 = 0.0, a2 = 0.0;
    for (int g = 0; g < R; ++g) {
        T uu[4];
        double d[4];
        uint32_t ll[4];
        int bb[4], loc[4];
        const uint32_t r0 = base + 4u * (uint32_t)g * kThreads; // the round's first position
        const int kc = ((int)(r0 / kCdfBucket) < W.nbk ? (int)(r0 / kCdfBucket) : W.nbk - 1) - kBelow;
        T vv[4], kb[4], ka[4];
        uint32_t lb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // the round's sorted pairs and their neighbours' keys, loaded
            // before the window's barrier; positions clamped into [0, P) so
            // that every load issues without a branch (the values of clamped
            // positions are not used)
            const uint32_t r = r0 + (uint32_t)e * kThreads + threadIdx.x;
            const uint32_t rc = r < P ? r : P - 1u;
            vv[e] = S.key(rc);
            lb[e] = S.label(rc);
            kb[e] = S.key(rc > 0u ? rc - 1u : 0u);
            ka[e] = S.key(rc + 1u < P ? rc + 1u : rc);
        }
        if (mode == 1) {
            if (threadIdx.x <= kWin) {
                const int k = kc + (int)threadIdx.x;
                spl[threadIdx.x] = k <= 0 ? -std::numeric_limits<T>::infinity()
                                          : (k >= W.nbk ? std::numeric_limits<T>::infinity()
                                                        : S.key((uint32_t)k * (uint32_t)kCdfBucket));
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // lane-contiguous positions: every load instruction reads 64 consecutive pairs
            const uint32_t r = base + (uint32_t)(4 * g + e) * kThreads + threadIdx.x;
            d[e] = 0.0;
            bb[e] = -1;
            if (r < P) {
                const T v = vv[e];
                const uint32_t lab = lb[e];
                int64_t lo = r, hi = r;
                if (r > 0 && kb[e] == v) lo = run_end<-1>(S, (int64_t)P, (int64_t)r, v);
                if (r + 1 < P && ka[e] == v) hi = run_end<1>(S, (int64_t)P, (int64_t)r, v);
                const T cnt = (T)((double)lo + 0.5 * (double)(hi - lo + 1));
                const uint32_t p = lab - (uint32_t)W.doff;
                const Words4 w = philox4x32_10((uint32_t)(p >> 2), step, inst, 0u, W.key0, W.key1);
                const T z = normal_pick<T>(w, (int)(p & 3));
                const T pol0 = (DEG == 1) ? fmaT(c1, v, c0) : fmaT(fmaT(fmaT(c3, v, c2), v, c1), v, c0);
                const T u = fmaT(fmaT(e1, v, e0), z, fmaT(kf, cnt, pol0));
                if (mode == 2) {
                    y[p] = u;
                } else if (mode == 0) {
                    ko[W.doff + r] = u;
                    lo_out[W.doff + r] = lab;
                } else {
                    // the largest w with spl[w] <= u (spl[w] nondecreasing), by
                    // halving steps in LDS; outside the window, a search of
                    // the item's splitters from the state's old bucket
                    int w = 0;
#pragma unroll
                    for (int step = kWin / 2; step > 0; step >>= 1)
                        if (spl[w + step] <= u) w += step;
                    if (spl[kWin] <= u) w = kWin;
                    if (spl[0] <= u && w < kWin) {
                        bb[e] = kc + w;
                    } else {
                        const int k0 = (int)(r / kCdfBucket) < W.nbk ? (int)(r / kCdfBucket) : W.nbk - 1;
                        bb[e] = bucket_of(S, W.nbk, k0, u);
                    }
                    uu[e] = u;
                    ll[e] = lab;
                }
                d[e] = leaf_diff(u, shift);
            }
        }
        double q1, q2;
        quad_leaf(d, q1, q2);
        a1 += q1;
        a2 += q2;
        if (mode == 1) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                loc[e] = -1;
                if (bb[e] >= 0 && bb[e] - kc >= 0 && bb[e] - kc < kWin) loc[e] = (int)atomicAdd(&hist[bb[e] - kc], 1u);
            }
            __syncthreads();
            if (threadIdx.x < kWin / 2) { // wave 0: offsets in the round, slots in the buckets
                const int k = 2 * (int)threadIdx.x; // this lane's buckets k, k + 1
                const uint32_t h0 = hist[k], h1 = hist[k + 1], h = h0 + h1;
                uint32_t incl = h;
#pragma unroll
                for (int off = 1; off < kWin / 2; off <<= 1) {
                    const uint32_t v = (uint32_t)__shfl_up((int)incl, off);
                    if ((int)threadIdx.x >= off) incl += v;
                }
                lstart[k] = incl - h;
                lstart[k + 1] = incl - h1;
                if (k + 2 == kWin) lstart[kWin] = incl;
                hbase[k] = h0 != 0u ? atomicAdd(&bcount[W.bbase + kc + k], h0) : 0u;
                hbase[k + 1] = h1 != 0u ? atomicAdd(&bcount[W.bbase + kc + k + 1], h1) : 0u;
                hist[k] = 0u; // for the next round
                hist[k + 1] = 0u;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (bb[e] < 0) continue;
                const uint32_t pos = base + (uint32_t)(4 * g + e) * kThreads + threadIdx.x;
                if (loc[e] >= 0) {
                    const int w = bb[e] - kc;
                    const uint32_t q = lstart[w] + (uint32_t)loc[e];
                    su[q] = uu[e];
                    sl[q] = ll[e];
                    sp[q] = pos;
                    sw[q] = (uint8_t)w;
                } else { // outside the window: a slot of its own
                    const int b = W.bbase + bb[e];
                    const uint32_t slot = atomicAdd(&bcount[b], 1u);
                    if (slot < (uint32_t)kCdfBucketCap) {
                        const size_t i = ((size_t)b << 12) + slot; // kCdfBucketCap == 4096
                        stage.u[i] = uu[e];
                        stage.lab[i] = ll[e];
                        stage.pos[i] = pos;
                    } else {
                        *flag = 1u;
                    }
                }
            }
            __syncthreads();
            const uint32_t total = lstart[kWin];
            for (uint32_t q = threadIdx.x; q < total; q += kThreads) {
                const int w = sw[q];
                const uint32_t slot = hbase[w] + (q - lstart[w]);
                if (slot < (uint32_t)kCdfBucketCap) {
                    const size_t i = ((size_t)(W.bbase + kc + w) << 12) + slot;
                    stage.u[i] = su[q];
                    stage.lab[i] = sl[q];
                    stage.pos[i] = sp[q];
                } else {
                    *flag = 1u;
                }
            }
            __syncthreads(); // before the next round reuses the LDS staging
        }
    }
    double sm[2] = {a1, a2};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) part_out[W.part_off + sc] = make_double2(sm[0], sm[1]);
}

// Trace entry m with the trigonometric mean field: the means of sin and cos.
__global__ __launch_bounds__(kThreads) void k_finish_trig(const WorkItem *__restrict__ items,
                                                          const double2 *__restrict__ part_in,
                                                          double2 *__restrict__ trace, int32_t m) {
    __shared__ double lds[8];
    const WorkItem &W = items[blockIdx.x];
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    if (threadIdx.x == 0)
        trace[(int64_t)blockIdx.x * (m + 1) + m] = make_double2(S1 / (double)W.P, S2 / (double)W.P);
}

// ----------------------------------------------------------------------------
// Quantity of interest: (1/P) sum Phi(x_p), Phi evaluated in fp64 (KIND 0: x,
// 1: x^2, 2: sin(x^2), the nonlinear QoI of the geometric Brownian motion
// example).  Per-superchunk partials in the canonical order, then one block
// per item forms the ensemble sum and divides by P.
// ----------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ double qoi_phi(double x) {
    return KIND == 0 ? x : (KIND == 1 ? x * x : sin(x * x));
}

template <typename T, int KIND>
__global__ __launch_bounds__(kThreads) void k_qoi_partials(const WorkItem *__restrict__ items,
                                                           const int2 *__restrict__ blocks,
                                                           double2 *__restrict__ part_out) {
    __shared__ double lds[8];
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x);
    const int64_t P = W.P;
    const int R = W.R;
    double a1 = 0.0;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    for (int r = 0; r < R; ++r) {
        const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
        if (p < P) {
            T v[4];
            load_quad(x, p, P, v);
            double f[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) f[e] = (p + e < P) ? qoi_phi<KIND>((double)v[e]) : 0.0;
            a1 += (f[0] + f[1]) + (f[2] + f[3]);
        }
    }
    double sm[2] = {a1, 0.0};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) part_out[W.part_off + bt.y] = make_double2(sm[0], 0.0);
}

__global__ __launch_bounds__(kThreads) void k_qoi_finish(const WorkItem *__restrict__ items,
                                                         const double2 *__restrict__ part_in,
                                                         double *__restrict__ out) {
    __shared__ double lds[8];
    const WorkItem &W = items[blockIdx.x];
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = S1 / (double)W.P;
}

// Moments of the final state of each ensemble (trace entry m): one block per item.
__global__ __launch_bounds__(kThreads) void k_finish(const WorkItem *__restrict__ items,
                                                     const double2 *__restrict__ part_in,
                                                     const double *__restrict__ shift_in,
                                                     double2 *__restrict__ trace, int32_t m) {
    __shared__ double lds[8];
    const WorkItem &W = items[blockIdx.x];
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    double mean, var;
    finish_moments(S1, S2, shift_in[blockIdx.x], (double)W.P, mean, var);
    if (threadIdx.x == 0) trace[(int64_t)blockIdx.x * (m + 1) + m] = make_double2(mean, var);
}

// ----------------------------------------------------------------------------
// Discrete adjoint of the fine propagator (pathwise gradients; not in the paper)
//
// Forward step s:  X_{s+1} = X_s + a(X_s, m_s, v_s) dt + b(X_s, m_s, v_s) sqrt(dt) z_s
// with m_s, v_s the population mean and variance of X_s.  With lambda_s =
// dL/dX_s (total derivative):
//   lambda_s = lambda_{s+1} (1 + a_x(X_s) dt + b_x sqrt(dt) z_s)
//            + g_m / P + 2 g_v (X_s - m_s) / P + [slice end] direct_s
//   g_m = sum_q lambda_{s+1}^q (a_m dt + b_m sqrt(dt) z_s^q)
//   g_v = sum_q lambda_{s+1}^q (a_v dt + b_v sqrt(dt) z_s^q)
//   dL/dtheta = sum_s sum_p lambda_{s+1}^p dX_{s+1}^p / dtheta   (theta = a0..bv)
// g_m and g_v need two ensemble sums of step s (sum lambda_{s+1}, sum
// lambda_{s+1} z_s); the launch of step s+1 forms them as partials while it
// writes lambda_{s+1}, exactly as the forward step forms the next mean field.
// lambda is fp64; X is the recomputed forward state (fp32 or fp64); z_s are the
// forward's own normals, regenerated.  Every sum uses the canonical order.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double adj_leaf(const double d[4]) { return (d[0] + d[1]) + (d[2] + d[3]); }

// The step's scalars from where they live on the device (uniform loads).
__device__ __forceinline__ AdjStep resolve_adj(const AdjRef &r) {
    AdjStep a{};
    a.step = r.step;
    a.zprev = r.zprev;
    a.grad = r.grad;
    if (r.mv) {
        const double2 t = *r.mv;
        a.m = t.x;
        a.v = t.y;
    }
    if (r.dl) {
        a.dm = r.dl[0] * r.invP;
        a.dv = 2.0 * r.dl[1] * r.invP;
        a.mdir = r.end->x;
    }
    return a;
}

// lambda_S = direct term at the final state; partials for step S-1.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_adj_init(const WorkItem *__restrict__ items,
                                                       const int2 *__restrict__ blocks, const T *__restrict__ xS,
                                                       double *__restrict__ lam, AdjRef ar,
                                                       double2 *__restrict__ part_out) {
    __shared__ double lds[8];
    const AdjStep a = resolve_adj(ar);
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const int64_t P = W.P;
    const int R = W.R;
    const double sdt = W.sdt;
    double s0 = 0.0, s1 = 0.0;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    for (int r = 0; r < R; ++r) {
        const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
        if (p < P) {
            T xv[4], z[4];
            load_quad(xS, p, P, xv);
            const Words4 w = philox4x32_10((uint32_t)(p >> 2), (uint32_t)(a.step - 1), (uint32_t)W.inst, 0u,
                                           W.key0, W.key1);
            box_muller4(w, z);
            double l[4], lz[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = p + e < P;
                l[e] = ok ? a.dm + a.dv * ((double)xv[e] - a.mdir) : 0.0;
                lz[e] = l[e] * (double)z[e];
                if (ok) lam[p + e] = l[e];
            }
            s0 += adj_leaf(l);
            s1 += adj_leaf(lz);
        }
    }
    (void)sdt;
    double sm[2] = {s0, s1};
    block_sum<2>(sm, lds);
    if (threadIdx.x == 0) part_out[W.part_off + bt.y] = make_double2(sm[0], sm[1]);
}

// Ensemble sums of each item's superchunk partials, one block per item (the
// adjoint step's combine for ensembles of many superchunks).
__global__ __launch_bounds__(kThreads) void k_item_sums(const WorkItem *__restrict__ items,
                                                        const double2 *__restrict__ part_in,
                                                        double2 *__restrict__ sums) {
    __shared__ double lds[8];
    const WorkItem &W = items[blockIdx.x];
    double S1, S2;
    ensemble_sums(part_in + W.part_off, W.nsc, S1, S2, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = make_double2(S1, S2);
}

// One backward step s: lambda_in = lambda_{s+1} -> lambda_out = lambda_s.
// acc: per-superchunk running gradient sums [nsc][10] (fp64, one writer each).
// PRE: the two ensemble sums come from k_item_sums instead of every block
// combining the partials itself (same order, same bits).
template <typename T, bool PRE>
__global__ __launch_bounds__(kThreads) void k_adj_step(const WorkItem *__restrict__ items,
                                                       const int2 *__restrict__ blocks, const T *__restrict__ xs_,
                                                       const double *__restrict__ lam_in,
                                                       double *__restrict__ lam_out, AdjRef ar,
                                                       const double2 *__restrict__ part_in,
                                                       const double2 *__restrict__ sums,
                                                       double2 *__restrict__ part_out, double *__restrict__ acc) {
    __shared__ double lds[4 * 8];
    const AdjStep a = resolve_adj(ar);
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const int64_t P = W.P;
    const int R = W.R;
    const double dt = W.dt, sdt = W.sdt;
    const double *c = W.c;
    // this thread's quads of the state and of lambda_{s+1}: loads issued
    // before the combine so that their latencies overlap
    constexpr int Q = kMaxQuadsPerThread;
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    T xq[Q][4];
    double lq[Q][4];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
        const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
        if (r < R && p < P) {
            load_quad(xs_, p, P, xq[r]);
            if (p + 3 < P) {
                const double2 l01 = *reinterpret_cast<const double2 *>(lam_in + p);
                const double2 l23 = *reinterpret_cast<const double2 *>(lam_in + p + 2);
                lq[r][0] = l01.x; lq[r][1] = l01.y; lq[r][2] = l23.x; lq[r][3] = l23.y;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) lq[r][e] = p + e < P ? lam_in[p + e] : 0.0;
            }
        }
    }

    // mean-field adjoint scalars of step s from the previous launch's partials
    double Sl, Slz;
    if (PRE) {
        const double2 sv = sums[bt.x];
        Sl = sv.x;
        Slz = sv.y;
    } else {
        ensemble_sums(part_in + W.part_off, W.nsc, Sl, Slz, lds);
    }
    const double gm = c[4] * dt * Sl + c[8] * sdt * Slz;
    const double gv = c[5] * dt * Sl + c[9] * sdt * Slz;
    const double c1 = gm / (double)P, c2 = 2.0 * gv / (double)P;

    double g[6] = {0, 0, 0, 0, 0, 0}; // sum l, lx, lx^2, lx^3, lz, lxz   (l = lambda_{s+1})
    double nx0 = 0.0, nx1 = 0.0;      // sum lambda_s, sum lambda_s z_{s-1}
#pragma unroll
    for (int r = 0; r < Q; ++r) {
        const int64_t p = base + 4 * (int64_t)(r * kThreads + threadIdx.x);
        if (r < R && p < P) {
            T z[4], zp[4];
            const T *xv = xq[r];
            const uint32_t q = (uint32_t)(p >> 2);
            const Words4 w = philox4x32_10(q, (uint32_t)a.step, (uint32_t)W.inst, 0u, W.key0, W.key1);
            box_muller4(w, z);
            if (a.zprev) {
                const Words4 w2 = philox4x32_10(q, (uint32_t)(a.step - 1), (uint32_t)W.inst, 0u, W.key0, W.key1);
                box_muller4(w2, zp);
            }
            double t0[4], t1[4], t2[4], t3[4], t4[4], t5[4], ln[4], lnz[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = p + e < P;
                const double x = (double)xv[e], zz = (double)z[e];
                const double l = lq[r][e];
                const double ax = c[1] + x * (2.0 * c[2] + 3.0 * c[3] * x);
                double lo = l * (1.0 + ax * dt + c[7] * sdt * zz) + c1 + c2 * (x - a.m);
                lo += a.dm + a.dv * (x - a.mdir);
                lo = ok ? lo : 0.0;
                if (ok) lam_out[p + e] = lo;
                t0[e] = l;
                t1[e] = l * x;
                t2[e] = l * x * x;
                t3[e] = l * x * x * x;
                t4[e] = l * zz;
                t5[e] = l * x * zz;
                ln[e] = lo;
                lnz[e] = a.zprev ? lo * (double)zp[e] : 0.0;
            }
            g[0] += adj_leaf(t0);
            g[1] += adj_leaf(t1);
            g[2] += adj_leaf(t2);
            g[3] += adj_leaf(t3);
            g[4] += adj_leaf(t4);
            g[5] += adj_leaf(t5);
            nx0 += adj_leaf(ln);
            nx1 += adj_leaf(lnz);
        }
    }
    double sm[8] = {g[0], g[1], g[2], g[3], g[4], g[5], nx0, nx1};
    block_sum<8>(sm, lds);
    if (threadIdx.x == 0) {
        part_out[W.part_off + bt.y] = make_double2(sm[6], sm[7]);
        if (a.grad) {
            double *ac = acc + (int64_t)(W.part_off + bt.y) * 10;
            ac[0] += dt * sm[0];
            ac[1] += dt * sm[1];
            ac[2] += dt * sm[2];
            ac[3] += dt * sm[3];
            ac[4] += dt * a.m * sm[0];
            ac[5] += dt * a.v * sm[0];
            ac[6] += sdt * sm[4];
            ac[7] += sdt * sm[5];
            ac[8] += sdt * a.m * sm[4];
            ac[9] += sdt * a.v * sm[4];
        }
    }
}

// The streaming ceiling of the step kernel's access pattern: every block
// reads its superchunk of 256 x 4 quads (non-temporal, all loads issued before
// any store), multiplies by a and writes it back in place.  No arithmetic of
// the method; a measurement of what the memory system sustains for it.
__global__ __launch_bounds__(kThreads) void k_stream_inplace(float *__restrict__ x, float a) {
    const uint32_t q0 = blockIdx.x * (uint32_t)(kThreads * kMaxQuadsPerThread) + threadIdx.x;
    float v[kMaxQuadsPerThread][4];
#pragma unroll
    for (int g = 0; g < kMaxQuadsPerThread; ++g) gload_quad<true>(x, q0 + (uint32_t)(g * kThreads), v[g]);
#pragma unroll
    for (int g = 0; g < kMaxQuadsPerThread; ++g) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[g][e] *= a;
        gstore_quad<true>(x, q0 + (uint32_t)(g * kThreads), v[g]);
    }
}

hipError_t launch_stream_inplace(float *x, int64_t n, hipStream_t s) {
    const int64_t per_block = (int64_t)4 * kThreads * kMaxQuadsPerThread;
    hipLaunchKernelGGL(k_stream_inplace, dim3((unsigned)(n / per_block)), dim3(kThreads), 0, s, x, 1.0f);
    return hipGetLastError();
}

// n doubles set to zero (a kernel, not a memset, so that it can be replayed from a graph).
__global__ __launch_bounds__(kThreads) void k_zero(double *__restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        x[i] = 0.0;
}

// Sum of the per-superchunk gradient accumulators of one item (one block).
__global__ __launch_bounds__(kThreads) void k_adj_reduce(const WorkItem *__restrict__ items,
                                                         const double *__restrict__ acc, double *__restrict__ out) {
    __shared__ double lds[4 * 10];
    const WorkItem &W = items[blockIdx.x];
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = threadIdx.x; s < W.nsc; s += kThreads)
#pragma unroll
        for (int k = 0; k < 10; ++k) v[k] += acc[(int64_t)(W.part_off + s) * 10 + k];
    block_sum<10>(v, lds);
    if (threadIdx.x < 10) out[(int64_t)blockIdx.x * 10 + threadIdx.x] = v[threadIdx.x];
}

// ----------------------------------------------------------------------------
// Region partials (restriction R, eq. multimodal_R).  MODE 0: the values
// themselves; MODE 1: the values after the matching map of their region (dry
// run of T), grouped by the region they came from.  NR = regions + 1 (the
// last entry is the whole ensemble).  Shift per (item, region).
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double apply_map(const RegionMap &mp, T xv, uint32_t q, int e, uint32_t inst,
                                            uint32_t k0, uint32_t k1);

template <>
__device__ __forceinline__ double apply_map<float>(const RegionMap &mp, float xv, uint32_t q, int e, uint32_t inst,
                                                   uint32_t k0, uint32_t k1) {
    if (mp.mode == 1) return (double)(float)fma(mp.scale, (double)xv - mp.from, mp.to);
    if (mp.mode == 2) {
        const Words4 w = philox4x32_10(q, (uint32_t)mp.boundary, inst, 3u, k0, k1);
        float z[4];
        box_muller4(w, z);
        return (double)(float)fma(mp.scale, (double)z[e], mp.to);
    }
    return (double)xv;
}
template <>
__device__ __forceinline__ double apply_map<double>(const RegionMap &mp, double xv, uint32_t q, int e, uint32_t inst,
                                                    uint32_t k0, uint32_t k1) {
    if (mp.mode == 1) return fma(mp.scale, xv - mp.from, mp.to);
    if (mp.mode == 2) {
        const Words4 w = philox4x32_10(q, (uint32_t)mp.boundary, inst, 3u, k0, k1);
        double z[4];
        box_muller4(w, z);
        return fma(mp.scale, z[e], mp.to);
    }
    return xv;
}

// Region partials of one superchunk, per region i < NREG (the whole-ensemble
// record is formed from the regions' in the combine).  FULL = false: count and
// sum of (y - shift_i) only (the first pass, which needs region means); FULL =
// true: also the sum of squares, min and max.
template <typename T, int NREG, int MODE, bool FULL>
__device__ __forceinline__ void region_accumulate(const T v[4], int64_t p, int64_t P, uint32_t Q, const WorkItem &W,
                                                  const Splits &sp, const RegionMap *mp, const double *sh,
                                                  double *acc, double *mn, double *mx, bool checked) {
    int g[4];
    double y[4];
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        ok[e] = !checked || (p + e < P);
        g[e] = region_of<NREG>((double)v[e], sp);
        if (MODE == 1) {
            RegionMap m0 = mp[0];
#pragma unroll
            for (int i = 1; i < NREG; ++i)
                if (g[e] == i) m0 = mp[i];
            y[e] = apply_map<T>(m0, v[e], Q, e, (uint32_t)W.inst, W.key0, W.key1);
        } else {
            y[e] = (double)v[e];
        }
    }
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
        double d[4], c[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool in = ok[e] && (NREG == 1 || g[e] == i);
            d[e] = in ? y[e] - sh[i] : 0.0;
            c[e] = in ? 1.0 : 0.0;
            if (FULL && in) {
                mn[i] = fmin(mn[i], y[e]);
                mx[i] = fmax(mx[i], y[e]);
            }
        }
        acc[3 * i] += (c[0] + c[1]) + (c[2] + c[3]);
        acc[3 * i + 1] += (d[0] + d[1]) + (d[2] + d[3]);
        if (FULL) acc[3 * i + 2] += (d[0] * d[0] + d[1] * d[1]) + (d[2] * d[2] + d[3] * d[3]);
    }
}

template <typename T, int NREG, int MODE, bool FULL>
__global__ __launch_bounds__(kThreads) void k_region_partials(const WorkItem *__restrict__ items,
                                                              const int2 *__restrict__ blocks,
                                                              const double *__restrict__ rshift, Splits sp,
                                                              const RegionMap *__restrict__ maps,
                                                              RegionPartial *__restrict__ rpart) {
    constexpr int NR = NREG + 1; // record stride (the whole-ensemble entry comes last)
    __shared__ double lds[4 * 3 * NREG + 8 * NREG];
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    const T *__restrict__ x = reinterpret_cast<const T *>(W.x);
    const int64_t P = W.P;
    const int R = W.R;
    double sh[NREG];
#pragma unroll
    for (int i = 0; i < NREG; ++i) sh[i] = rshift[(int64_t)bt.x * NR + i];
    RegionMap mp[NREG];
    if (MODE == 1) {
#pragma unroll
        for (int i = 0; i < NREG; ++i) mp[i] = maps[(int64_t)bt.x * NREG + i];
    }
    double acc[3 * NREG], mn[NREG], mx[NREG];
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
        acc[3 * i] = acc[3 * i + 1] = acc[3 * i + 2] = 0.0;
        mn[i] = __builtin_inf();
        mx[i] = -__builtin_inf();
    }
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R;
    if (base + (int64_t)4 * kThreads * R <= P) {
        // a full superchunk: every quad's load issued before the first is used
        const uint32_t qb = (uint32_t)(base >> 2) + threadIdx.x;
        T v[kMaxQuadsPerThread][4];
#pragma unroll
        for (int r = 0; r < kMaxQuadsPerThread; ++r)
            if (r < R) gload_quad<false>(x + base, (uint32_t)(r * kThreads + threadIdx.x), v[r]);
#pragma unroll
        for (int r = 0; r < kMaxQuadsPerThread; ++r)
            if (r < R)
                region_accumulate<T, NREG, MODE, FULL>(v[r], 0, P, qb + (uint32_t)(r * kThreads), W, sp, mp, sh, acc,
                                                       mn, mx, false);
    } else {
        for (int r = 0; r < R; ++r) {
            const int64_t Q = (base >> 2) + (int64_t)r * kThreads + threadIdx.x;
            const int64_t p = 4 * Q;
            if (p < P) {
                T v[4];
                load_quad(x, p, P, v);
                region_accumulate<T, NREG, MODE, FULL>(v, p, P, (uint32_t)Q, W, sp, mp, sh, acc, mn, mx, true);
            }
        }
    }
    block_sum_dpp<3 * NREG>(acc, lds);
    if (FULL) block_minmax<NREG>(mn, mx, lds);
    if (threadIdx.x == 0) {
        RegionPartial *out = rpart + (int64_t)(W.part_off + bt.y) * NREG;
#pragma unroll
        for (int i = 0; i < NREG; ++i) {
            RegionPartial rp;
            rp.cnt = acc[3 * i];
            rp.s1 = acc[3 * i + 1];
            rp.s2 = acc[3 * i + 2];
            rp.mn = mn[i];
            rp.mx = mx[i];
            out[i] = rp;
        }
    }
}

// One block per item: region partials -> records (regions, then the whole
// ensemble from the regions: total count, count-weighted mean, law of total
// variance, extreme min and max).  If rshift_next is set it receives the
// region means (the shifts of the second, full pass); the records then are
// not written.
template <int NREG, bool FULL>
__global__ __launch_bounds__(kThreads) void k_region_combine(const WorkItem *__restrict__ items,
                                                             const RegionPartial *__restrict__ rpart,
                                                             const double *__restrict__ rshift,
                                                             RegionStats *__restrict__ out,
                                                             double *__restrict__ rshift_next) {
    constexpr int NR = NREG + 1;
    __shared__ double lds[4 * 3 * NREG + 8 * NREG];
    const WorkItem &W = items[blockIdx.x];
    double acc[3 * NREG], mn[NREG], mx[NREG];
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
        acc[3 * i] = acc[3 * i + 1] = acc[3 * i + 2] = 0.0;
        mn[i] = __builtin_inf();
        mx[i] = -__builtin_inf();
    }
    for (int s = threadIdx.x; s < W.nsc; s += kThreads) {
        const RegionPartial *rp = rpart + (int64_t)(W.part_off + s) * NREG;
#pragma unroll
        for (int i = 0; i < NREG; ++i) {
            acc[3 * i] += rp[i].cnt;
            acc[3 * i + 1] += rp[i].s1;
            if (FULL) {
                acc[3 * i + 2] += rp[i].s2;
                mn[i] = fmin(mn[i], rp[i].mn);
                mx[i] = fmax(mx[i], rp[i].mx);
            }
        }
    }
    block_sum<3 * NREG>(acc, lds);
    if (FULL) block_minmax<NREG>(mn, mx, lds);
    if (threadIdx.x != 0) return;
    if (!FULL) {
#pragma unroll
        for (int i = 0; i < NREG; ++i) {
            const double sh = rshift[(int64_t)blockIdx.x * NR + i];
            const double mean = sh + acc[3 * i + 1] / acc[3 * i];
            rshift_next[(int64_t)blockIdx.x * NR + i] = (acc[3 * i] > 0.0 && isfinite(mean)) ? mean : sh;
        }
        return;
    }
    RegionStats st[NREG];
    int64_t ntot = 0;
    bool nonfinite = false;
    double gmin = __builtin_inf(), gmax = -__builtin_inf();
#pragma unroll
    for (int i = 0; i < NREG; ++i) {
        const double sh = rshift[(int64_t)blockIdx.x * NR + i];
        st[i].n = (int64_t)acc[3 * i];
        st[i].min = mn[i];
        st[i].max = mx[i];
        st[i].nonfinite = !(isfinite(acc[3 * i + 1]) && isfinite(acc[3 * i + 2]));
        st[i].reserved = 0;
        if (st[i].n == 0) {
            st[i].mean = 0.0;
            st[i].var = 0.0;
        } else if (mn[i] == mx[i]) {
            st[i].mean = mn[i];
            st[i].var = 0.0;
        } else {
            finish_moments(acc[3 * i + 1], acc[3 * i + 2], sh, acc[3 * i], st[i].mean, st[i].var);
        }
        ntot += st[i].n;
        nonfinite = nonfinite || st[i].nonfinite;
        gmin = fmin(gmin, mn[i]);
        gmax = fmax(gmax, mx[i]);
        out[(int64_t)blockIdx.x * NR + i] = st[i];
    }
    RegionStats g;
    g.n = ntot;
    g.min = gmin;
    g.max = gmax;
    g.nonfinite = nonfinite;
    g.reserved = 0;
    if (NREG == 1) {
        g.mean = st[0].mean;
        g.var = st[0].var;
    } else if (ntot == 0) {
        g.mean = 0.0;
        g.var = 0.0;
    } else if (gmin == gmax) {
        g.mean = gmin;
        g.var = 0.0;
    } else {
        double m = 0.0;
#pragma unroll
        for (int i = 0; i < NREG; ++i)
            if (st[i].n > 0) m += ((double)st[i].n / (double)ntot) * st[i].mean;
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < NREG; ++i)
            if (st[i].n > 0) {
                const double dm = st[i].mean - m;
                v += ((double)st[i].n / (double)ntot) * (st[i].var + dm * dm);
            }
        g.mean = m;
        g.var = v;
    }
    out[(int64_t)blockIdx.x * NR + NREG] = g;
}

// Shifts for the first restriction pass: the value the step sums were shifted
// by (after a fine step: the last step's mean) or x[0].
template <typename T, int NR>
__global__ void k_fill_shift(const WorkItem *__restrict__ items, int n_items, const double *__restrict__ shift,
                             double *__restrict__ rshift) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= n_items) return;
    const double s = shift ? shift[item] : (double)reinterpret_cast<const T *>(items[item].x)[0];
#pragma unroll
    for (int i = 0; i < NR; ++i) rshift[(int64_t)item * NR + i] = s;
}

// ----------------------------------------------------------------------------
// Matching T applied in place, per region (eq. multimodal_M)
// ----------------------------------------------------------------------------
template <typename T, int NREG>
__global__ __launch_bounds__(kThreads) void k_match_apply(const WorkItem *__restrict__ items,
                                                          const int2 *__restrict__ blocks, Splits sp,
                                                          const RegionMap *__restrict__ maps) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    T *__restrict__ x = reinterpret_cast<T *>(W.x);
    const T *__restrict__ xin = W.src ? reinterpret_cast<const T *>(W.src) : x;
    const int64_t P = W.P;
    const int R = W.R;
    RegionMap mp[NREG];
#pragma unroll
    for (int i = 0; i < NREG; ++i) mp[i] = maps[(int64_t)bt.x * NREG + i];
    auto map_quad = [&](T (&v)[4], int64_t Q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int g = region_of<NREG>((double)v[e], sp);
            RegionMap m0 = mp[0];
#pragma unroll
            for (int i = 1; i < NREG; ++i)
                if (g == i) m0 = mp[i];
            v[e] = (T)apply_map<T>(m0, v[e], (uint32_t)Q, e, (uint32_t)W.inst, W.key0, W.key1);
        }
    };
    const int64_t base = (int64_t)bt.y * 4 * kThreads * R; // first particle of the superchunk
    if (base + (int64_t)4 * kThreads * R <= P) {
        // a full superchunk: every quad's load issued before the first map
        T v[kMaxQuadsPerThread][4];
#pragma unroll
        for (int g = 0; g < kMaxQuadsPerThread; ++g)
            if (g < R) gload_quad<false>(xin + base, (uint32_t)(g * kThreads + threadIdx.x), v[g]);
#pragma unroll
        for (int g = 0; g < kMaxQuadsPerThread; ++g)
            if (g < R) {
                map_quad(v[g], (base >> 2) + g * kThreads + threadIdx.x);
                gstore_quad<false>(x + base, (uint32_t)(g * kThreads + threadIdx.x), v[g]);
            }
        return;
    }
    const int64_t qbase = (int64_t)bt.y * kThreads * R + threadIdx.x;
    for (int r = 0; r < R; ++r) {
        const int64_t Q = qbase + (int64_t)r * kThreads;
        const int64_t p = 4 * Q;
        if (p < P) {
            T v[4];
            load_quad(xin, p, P, v);
            map_quad(v, Q);
            store_quad(x, p, P, v);
        }
    }
}

// ----------------------------------------------------------------------------
// Initial law p0
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(const WorkItem *__restrict__ items,
                                                   const int2 *__restrict__ blocks) {
    const int2 bt = blocks[blockIdx.x];
    const WorkItem &W = items[bt.x];
    T *__restrict__ x = reinterpret_cast<T *>(W.x);
    const int64_t P = W.P;
    const int R = W.R;
    const int64_t qbase = (int64_t)bt.y * kThreads * R + threadIdx.x;
    for (int r = 0; r < R; ++r) {
        const int64_t Q = qbase + (int64_t)r * kThreads;
        const int64_t p = 4 * Q;
        if (p >= P) continue;
        T v[4];
        if (W.p0_kind == 2) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (T)W.p0[1];
        } else {
            const Words4 w = philox4x32_10((uint32_t)Q, 0u, (uint32_t)W.inst, 1u, W.key0, W.key1);
            T z[4];
            box_muller4(w, z);
            if (W.p0_kind == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (T)(W.p0[1] + W.p0[2] * (double)z[e]);
            } else {
                const Words4 pk = philox4x32_10((uint32_t)Q, 0u, (uint32_t)W.inst, 2u, W.key0, W.key1);
                const uint32_t pw[4] = {pk.w0, pk.w1, pk.w2, pk.w3};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool first = uniform_of(pw[e]) < W.p0[0];
                    const double mu = first ? W.p0[1] : W.p0[3];
                    const double sd = first ? W.p0[2] : W.p0[4];
                    v[e] = (T)(mu + sd * (double)z[e]);
                }
            }
        }
        store_quad(x, p, P, v);
    }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
hipError_t launch_sum_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, double2 *part_out,
                           double *shift_out, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_sum_init<double>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part_out, shift_out);
    else
        hipLaunchKernelGGL(k_sum_init<float>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part_out, shift_out);
    return hipGetLastError();
}

template <typename T, int DEG>
static void em_step_variant(int variant, const WorkItem *items, const int2 *blocks, int nblocks, int j,
                            const double2 *part_in, const double *shift_in, const double2 *mv, double2 *part_out,
                            double *shift_out, double2 *trace, int m, hipStream_t s) {
    switch (variant & 3) {
    case 0:
        hipLaunchKernelGGL((k_em_step<T, DEG, false, false>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           part_in, shift_in, mv, part_out, shift_out, trace, m);
        break;
    case 1:
        hipLaunchKernelGGL((k_em_step<T, DEG, true, false>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           part_in, shift_in, mv, part_out, shift_out, trace, m);
        break;
    case 2:
        hipLaunchKernelGGL((k_em_step<T, DEG, false, true>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           part_in, shift_in, mv, part_out, shift_out, trace, m);
        break;
    default:
        hipLaunchKernelGGL((k_em_step<T, DEG, true, true>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           part_in, shift_in, mv, part_out, shift_out, trace, m);
        break;
    }
}

hipError_t launch_em_step(int prec, int deg, int variant, const WorkItem *items, int n_items, const int2 *blocks,
                          int nblocks, int j, const double2 *part_in, const double *shift_in, double2 *mv,
                          double2 *part_out, double *shift_out, double2 *trace, int m, hipStream_t s) {
    if (variant & 2)
        hipLaunchKernelGGL(k_combine, dim3(n_items), dim3(kThreads), 0, s, items, part_in, shift_in, mv);
    if (prec == 0) {
        if (deg == 1)
            em_step_variant<double, 1>(variant, items, blocks, nblocks, j, part_in, shift_in, mv, part_out, shift_out,
                                       trace, m, s);
        else
            em_step_variant<double, 3>(variant, items, blocks, nblocks, j, part_in, shift_in, mv, part_out, shift_out,
                                       trace, m, s);
    } else {
        if (deg == 1)
            em_step_variant<float, 1>(variant, items, blocks, nblocks, j, part_in, shift_in, mv, part_out, shift_out,
                                      trace, m, s);
        else
            em_step_variant<float, 3>(variant, items, blocks, nblocks, j, part_in, shift_in, mv, part_out, shift_out,
                                      trace, m, s);
    }
    return hipGetLastError();
}

hipError_t launch_em_sweep_resident(int prec, int deg, const WorkItem *items, int n_items, const int2 *blocks,
                                    int nblocks, int m, void *z, double2 *part_out, double *shift_out,
                                    double2 *trace, hipStream_t s) {
    const dim3 gz(nblocks, m);
    if (prec == 0) {
        hipLaunchKernelGGL(k_sweep_normals<double>, gz, dim3(kThreads), 0, s, items, blocks, (double *)z);
        if (deg == 1)
            hipLaunchKernelGGL((k_em_sweep_resident<double, 1>), dim3(n_items), dim3(kResidentThreads), 0, s, items,
                               (const double *)z, m, part_out, shift_out, trace);
        else
            hipLaunchKernelGGL((k_em_sweep_resident<double, 3>), dim3(n_items), dim3(kResidentThreads), 0, s, items,
                               (const double *)z, m, part_out, shift_out, trace);
    } else {
        hipLaunchKernelGGL(k_sweep_normals<float>, gz, dim3(kThreads), 0, s, items, blocks, (float *)z);
        if (deg == 1)
            hipLaunchKernelGGL((k_em_sweep_resident<float, 1>), dim3(n_items), dim3(kResidentThreads), 0, s, items,
                               (const float *)z, m, part_out, shift_out, trace);
        else
            hipLaunchKernelGGL((k_em_sweep_resident<float, 3>), dim3(n_items), dim3(kResidentThreads), 0, s, items,
                               (const float *)z, m, part_out, shift_out, trace);
    }
    return hipGetLastError();
}

hipError_t launch_sum_init_trig(int prec, const WorkItem *items, const int2 *blocks, int nblocks,
                                double2 *part_out, double *shift_out, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_sum_init_trig<double>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part_out,
                           shift_out);
    else
        hipLaunchKernelGGL(k_sum_init_trig<float>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part_out,
                           shift_out);
    return hipGetLastError();
}

hipError_t launch_em_step_trig(int prec, int deg, const WorkItem *items, const int2 *blocks, int nblocks, int j,
                               const double2 *part_in, double2 *part_out, double *shift_out, double2 *trace, int m,
                               hipStream_t s) {
    if (prec == 0) {
        if (deg == 1)
            hipLaunchKernelGGL((k_em_step_trig<double, 1>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                               part_in, part_out, shift_out, trace, m);
        else
            hipLaunchKernelGGL((k_em_step_trig<double, 3>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                               part_in, part_out, shift_out, trace, m);
    } else {
        if (deg == 1)
            hipLaunchKernelGGL((k_em_step_trig<float, 1>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                               part_in, part_out, shift_out, trace, m);
        else
            hipLaunchKernelGGL((k_em_step_trig<float, 3>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                               part_in, part_out, shift_out, trace, m);
    }
    return hipGetLastError();
}

template <typename T, int DEG>
static void em_step_sorted(const WorkItem *items, const int2 *blocks, int nblocks, int j, int mode, bool packed,
                           const double2 *mv, const CdfBuffers &b, double2 *part_out, double *shift_out,
                           double2 *trace, int m, hipStream_t s) {
    if (packed) {
        SortedView<T, true> v{(const KeyLabel<T> *)b.kl[1]};
        hipLaunchKernelGGL((k_em_step_sorted<T, DEG, true>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           mode, mv, v, (T *)b.keys[0], b.lab[0], b.bcount, stage_view<T>(b.stage, b.nbuckets),
                           b.flag, part_out, shift_out, trace, m);
    } else {
        SortedView<T, false> v{(const T *)b.keys[1], b.lab[1]};
        hipLaunchKernelGGL((k_em_step_sorted<T, DEG, false>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, j,
                           mode, mv, v, (T *)b.keys[0], b.lab[0], b.bcount, stage_view<T>(b.stage, b.nbuckets),
                           b.flag, part_out, shift_out, trace, m);
    }
}

hipError_t launch_em_step_sorted(int prec, int deg, const WorkItem *items, int n_items, const int2 *blocks,
                                 int nblocks, int j, int mode, bool packed, const double2 *part_in,
                                 const double *shift_in, double2 *mv, const CdfBuffers &b, double2 *part_out,
                                 double *shift_out, double2 *trace, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(n_items), dim3(kThreads), 0, s, items, part_in, shift_in, mv);
    if (prec == 0) {
        if (deg == 1)
            em_step_sorted<double, 1>(items, blocks, nblocks, j, mode, packed, mv, b, part_out, shift_out, trace, m,
                                      s);
        else
            em_step_sorted<double, 3>(items, blocks, nblocks, j, mode, packed, mv, b, part_out, shift_out, trace, m,
                                      s);
    } else {
        if (deg == 1)
            em_step_sorted<float, 1>(items, blocks, nblocks, j, mode, packed, mv, b, part_out, shift_out, trace, m, s);
        else
            em_step_sorted<float, 3>(items, blocks, nblocks, j, mode, packed, mv, b, part_out, shift_out, trace, m, s);
    }
    return hipGetLastError();
}

hipError_t launch_finish_trig(const WorkItem *items, int n_items, const double2 *part_in, double2 *trace, int m,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_finish_trig, dim3(n_items), dim3(kThreads), 0, s, items, part_in, trace, m);
    return hipGetLastError();
}

template <typename T>
static void qoi_partials(int kind, const WorkItem *items, const int2 *blocks, int nblocks, double2 *part,
                         hipStream_t s) {
    if (kind == 0)
        hipLaunchKernelGGL((k_qoi_partials<T, 0>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part);
    else if (kind == 1)
        hipLaunchKernelGGL((k_qoi_partials<T, 1>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part);
    else
        hipLaunchKernelGGL((k_qoi_partials<T, 2>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, part);
}

hipError_t launch_qoi(int prec, int kind, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                      double2 *part, double *out, hipStream_t s) {
    if (prec == 0)
        qoi_partials<double>(kind, items, blocks, nblocks, part, s);
    else
        qoi_partials<float>(kind, items, blocks, nblocks, part, s);
    hipLaunchKernelGGL(k_qoi_finish, dim3(n_items), dim3(kThreads), 0, s, items, part, out);
    return hipGetLastError();
}

hipError_t launch_finish(const WorkItem *items, int n_items, const double2 *part_in, const double *shift_in,
                         double2 *trace, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(n_items), dim3(kThreads), 0, s, items, part_in, shift_in, trace, m);
    return hipGetLastError();
}

hipError_t launch_adj_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, const void *xS,
                           double *lam, const AdjRef &a, double2 *part_out, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_adj_init<double>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, (const double *)xS,
                           lam, a, part_out);
    else
        hipLaunchKernelGGL(k_adj_init<float>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks, (const float *)xS,
                           lam, a, part_out);
    return hipGetLastError();
}

template <typename T>
static void adj_step_variant(bool pre, const WorkItem *items, const int2 *blocks, int nblocks, const void *xs,
                             const double *lam_in, double *lam_out, const AdjRef &a, const double2 *part_in,
                             const double2 *sums, double2 *part_out, double *acc, hipStream_t s) {
    if (pre)
        hipLaunchKernelGGL((k_adj_step<T, true>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks,
                           (const T *)xs, lam_in, lam_out, a, part_in, sums, part_out, acc);
    else
        hipLaunchKernelGGL((k_adj_step<T, false>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks,
                           (const T *)xs, lam_in, lam_out, a, part_in, sums, part_out, acc);
}

hipError_t launch_adj_step(int prec, const WorkItem *items, int n_items, const int2 *blocks, int nblocks,
                           const void *xs, const double *lam_in, double *lam_out, const AdjRef &a,
                           const double2 *part_in, double2 *sums, double2 *part_out, double *acc, hipStream_t s) {
    if (sums) hipLaunchKernelGGL(k_item_sums, dim3(n_items), dim3(kThreads), 0, s, items, part_in, sums);
    if (prec == 0)
        adj_step_variant<double>(sums != nullptr, items, blocks, nblocks, xs, lam_in, lam_out, a, part_in, sums,
                                 part_out, acc, s);
    else
        adj_step_variant<float>(sums != nullptr, items, blocks, nblocks, xs, lam_in, lam_out, a, part_in, sums,
                                part_out, acc, s);
    return hipGetLastError();
}

hipError_t launch_zero(double *x, int64_t n, hipStream_t s) {
    const int64_t nb = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)(nb < 1024 ? (nb > 0 ? nb : 1) : 1024)), dim3(kThreads), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const WorkItem *items, int n_items, const double *acc, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce, dim3(n_items), dim3(kThreads), 0, s, items, acc, out);
    return hipGetLastError();
}

template <int NREG>
static void region_partials_nr(int prec, int mode, bool full, const WorkItem *items, const int2 *blocks, int nblocks,
                               const double *rshift, const Splits &sp, const RegionMap *maps, RegionPartial *rpart,
                               hipStream_t s) {
#define MCPR_RP(T, MODE, FULL)                                                                                     \
    hipLaunchKernelGGL((k_region_partials<T, NREG, MODE, FULL>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, \
                       rshift, sp, maps, rpart)
    if (prec == 0) {
        if (mode == 0) { if (full) MCPR_RP(double, 0, true); else MCPR_RP(double, 0, false); }
        else { if (full) MCPR_RP(double, 1, true); else MCPR_RP(double, 1, false); }
    } else {
        if (mode == 0) { if (full) MCPR_RP(float, 0, true); else MCPR_RP(float, 0, false); }
        else { if (full) MCPR_RP(float, 1, true); else MCPR_RP(float, 1, false); }
    }
#undef MCPR_RP
}

hipError_t launch_region_partials(int prec, int nr, int mode, bool full, const WorkItem *items, const int2 *blocks,
                                  int nblocks, const double *rshift, const Splits &sp, const RegionMap *maps,
                                  RegionPartial *rpart, hipStream_t s) {
    switch (nr - 1) {
    case 1: region_partials_nr<1>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 2: region_partials_nr<2>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 3: region_partials_nr<3>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 4: region_partials_nr<4>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 5: region_partials_nr<5>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 6: region_partials_nr<6>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 7: region_partials_nr<7>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    case 8: region_partials_nr<8>(prec, mode, full, items, blocks, nblocks, rshift, sp, maps, rpart, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NREG>
static void region_combine_nr(bool full, const WorkItem *items, int n_items, const RegionPartial *rpart,
                              const double *rshift, RegionStats *out, double *rshift_next, hipStream_t s) {
    if (full)
        hipLaunchKernelGGL((k_region_combine<NREG, true>), dim3(n_items), dim3(kThreads), 0, s, items, rpart, rshift,
                           out, rshift_next);
    else
        hipLaunchKernelGGL((k_region_combine<NREG, false>), dim3(n_items), dim3(kThreads), 0, s, items, rpart, rshift,
                           out, rshift_next);
}

hipError_t launch_region_combine(int nr, bool full, const WorkItem *items, int n_items, const RegionPartial *rpart,
                                 const double *rshift, RegionStats *out, double *rshift_next, hipStream_t s) {
    switch (nr - 1) {
    case 1: region_combine_nr<1>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 2: region_combine_nr<2>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 3: region_combine_nr<3>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 4: region_combine_nr<4>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 5: region_combine_nr<5>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 6: region_combine_nr<6>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 7: region_combine_nr<7>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    case 8: region_combine_nr<8>(full, items, n_items, rpart, rshift, out, rshift_next, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NR>
static void fill_shift_nr(int prec, const WorkItem *items, int n_items, const double *shift, double *rshift,
                          hipStream_t s) {
    const int nb = (n_items + 255) / 256;
    if (prec == 0)
        hipLaunchKernelGGL((k_fill_shift<double, NR>), dim3(nb), dim3(256), 0, s, items, n_items, shift, rshift);
    else
        hipLaunchKernelGGL((k_fill_shift<float, NR>), dim3(nb), dim3(256), 0, s, items, n_items, shift, rshift);
}

hipError_t launch_fill_shift(int prec, int nr, const WorkItem *items, int n_items, const double *shift, double *rshift,
                             hipStream_t s) {
    switch (nr) {
    case 2: fill_shift_nr<2>(prec, items, n_items, shift, rshift, s); break;
    case 3: fill_shift_nr<3>(prec, items, n_items, shift, rshift, s); break;
    case 4: fill_shift_nr<4>(prec, items, n_items, shift, rshift, s); break;
    case 5: fill_shift_nr<5>(prec, items, n_items, shift, rshift, s); break;
    case 6: fill_shift_nr<6>(prec, items, n_items, shift, rshift, s); break;
    case 7: fill_shift_nr<7>(prec, items, n_items, shift, rshift, s); break;
    case 8: fill_shift_nr<8>(prec, items, n_items, shift, rshift, s); break;
    case 9: fill_shift_nr<9>(prec, items, n_items, shift, rshift, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NREG>
static void match_nr(int prec, const WorkItem *items, const int2 *blocks, int nblocks, const Splits &sp,
                     const RegionMap *maps, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL((k_match_apply<double, NREG>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, sp, maps);
    else
        hipLaunchKernelGGL((k_match_apply<float, NREG>), dim3(nblocks), dim3(kThreads), 0, s, items, blocks, sp, maps);
}

hipError_t launch_match_apply(int prec, int nreg, const WorkItem *items, const int2 *blocks, int nblocks,
                              const Splits &sp, const RegionMap *maps, hipStream_t s) {
    switch (nreg) {
    case 1: match_nr<1>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 2: match_nr<2>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 3: match_nr<3>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 4: match_nr<4>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 5: match_nr<5>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 6: match_nr<6>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 7: match_nr<7>(prec, items, blocks, nblocks, sp, maps, s); break;
    case 8: match_nr<8>(prec, items, blocks, nblocks, sp, maps, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(int prec, const WorkItem *items, const int2 *blocks, int nblocks, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(k_init<double>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(nblocks), dim3(kThreads), 0, s, items, blocks);
    return hipGetLastError();
}

} // namespace mcpr
