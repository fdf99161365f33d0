// rng.hpp -- counter-based normals in registers (device code).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64 multiplies, key bumped by the Weyl constants between rounds.
// Box-Muller turns the four words into four standard normals.  The paper only
// requires that every iteration reuse the same numbers (Property "Exactness of
// MC-moments Parareal"); a counter-based generator gives that without storing
// any numbers: the counter is (quad, step, instance, tag).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mcpr {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Three-input XOR in one instruction: gfx950's v_bitop3_b32 with truth table
// 0x96 (the parity of the three inputs, whatever their order).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // round 0: the callers' counter words 1..3 and the key are uniform
        // across the wave, so plain XORs leave most of it to the scalar unit
        const uint32_t n0 = r == 0 ? ((uint32_t)(p1 >> 32) ^ c1 ^ k0) : xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = r == 0 ? ((uint32_t)(p0 >> 32) ^ c3 ^ k1) : xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

// fp64 normals: u = (w + 1/2) 2^-32 exactly; z = sqrt(-2 ln u0) (cos, sin)(2 pi u1)
__device__ __forceinline__ void box_muller4(const Words4 &w, double z[4]) {
    const double s = 2.3283064365386962890625e-10; // 2^-32
    const double u0 = ((double)w.w0 + 0.5) * s, u1 = ((double)w.w1 + 0.5) * s;
    const double u2 = ((double)w.w2 + 0.5) * s, u3 = ((double)w.w3 + 0.5) * s;
    const double r01 = sqrt(-2.0 * log(u0));
    const double r23 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    z[0] = r01 * c1;
    z[1] = r01 * s1;
    z[2] = r23 * c3;
    z[3] = r23 * s3;
}

// fp32 normals from the same words, on the transcendental units: v_log_f32 is
// log2, v_sin_f32 / v_cos_f32 take their argument in turns (sin(2 pi x)).
__device__ __forceinline__ void box_muller4(const Words4 &w, float z[4]) {
    const float s = 2.3283064365386963e-10f; // 2^-32
    const float h = 1.1641532182693481e-10f; // 2^-33
    const float u0 = fmaf((float)w.w0, s, h), u1 = fmaf((float)w.w1, s, h);
    const float u2 = fmaf((float)w.w2, s, h), u3 = fmaf((float)w.w3, s, h);
    const float m2ln2 = -1.3862943611198906f; // -2 ln 2
    const float r01 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    const float r23 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
    z[0] = r01 * __builtin_amdgcn_cosf(u1);
    z[1] = r01 * __builtin_amdgcn_sinf(u1);
    z[2] = r23 * __builtin_amdgcn_cosf(u3);
    z[3] = r23 * __builtin_amdgcn_sinf(u3);
}

// Normal e of the quad, by the same operations as box_muller4 (only its pair).
__device__ __forceinline__ double normal_of(const Words4 &w, int e) {
    const double s = 2.3283064365386962890625e-10; // 2^-32
    const uint32_t wa = e < 2 ? w.w0 : w.w2, wb = e < 2 ? w.w1 : w.w3;
    const double ua = ((double)wa + 0.5) * s, ub = ((double)wb + 0.5) * s;
    const double r = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincospi(2.0 * ub, &sn, &cs);
    return (e & 1) ? r * sn : r * cs;
}
__device__ __forceinline__ float normal_of_f(const Words4 &w, int e) {
    const float s = 2.3283064365386963e-10f; // 2^-32
    const float h = 1.1641532182693481e-10f; // 2^-33
    const uint32_t wa = e < 2 ? w.w0 : w.w2, wb = e < 2 ? w.w1 : w.w3;
    const float ua = fmaf((float)wa, s, h), ub = fmaf((float)wb, s, h);
    const float m2ln2 = -1.3862943611198906f; // -2 ln 2
    const float r = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(ua));
    return (e & 1) ? r * __builtin_amdgcn_sinf(ub) : r * __builtin_amdgcn_cosf(ub);
}

__device__ __forceinline__ double uniform_of(uint32_t w) {
    return ((double)w + 0.5) * 2.3283064365386962890625e-10;
}

} // namespace mcpr
