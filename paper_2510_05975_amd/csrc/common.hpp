// Device helpers shared by the gfx950 kernels of libcng.
//
// Keys: a candidate is the 64-bit word (float bits of D) << 32 | id.  D is a
// squared distance (>= +0), so unsigned comparison of keys is the
// lexicographic order on (D, id) used everywhere (ties go to the smaller id).
// Bit 63 (the sign bit of D) is free and marks "explored" inside a beam.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cng.h"

namespace cng {

constexpr uint32_t NONE = CNG_NONE;
constexpr uint64_t EXPL = 1ull << 63;
constexpr uint64_t KEY_INF = 0x7FFFFFFFFFFFFFFFull;

__device__ __forceinline__ uint64_t make_key(float D, uint32_t id)
{
    return ((uint64_t)__float_as_uint(D) << 32) | (uint64_t)id;
}
__device__ __forceinline__ uint64_t key_mask(uint64_t k) { return k & ~EXPL; }
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)k; }
__device__ __forceinline__ float key_dist(uint64_t k)
{
    return __uint_as_float((uint32_t)(k >> 32) & 0x7FFFFFFFu);
}

// Order of all LDS accesses of one wavefront across lanes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Butterfly over a group of G consecutive lanes (G a power of two <= 32):
// every lane ends with the sum in the order of the fixed reduction
// (offsets G/2 ... 1; the offsets 16 .. G of the 32-lane order would only add
// +0 to non-negative partial sums, which is exact).
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum_f64(double v)
{
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

// Partial sum of one lane for the fixed-order distance of two float4-chunked
// vectors: chunk r of lane gl covers elements (r*32 + gl)*4 .. +3.
__device__ __forceinline__ float chunk_fma(float4 a, float4 b, float acc)
{
    float t;
    t = a.x - b.x; acc = __builtin_fmaf(t, t, acc);
    t = a.y - b.y; acc = __builtin_fmaf(t, t, acc);
    t = a.z - b.z; acc = __builtin_fmaf(t, t, acc);
    t = a.w - b.w; acc = __builtin_fmaf(t, t, acc);
    return acc;
}

__device__ __forceinline__ double chunk_fma_f64(float4 a, float4 b, double acc)
{
    double t;
    t = (double)a.x - (double)b.x; acc = __builtin_fma(t, t, acc);
    t = (double)a.y - (double)b.y; acc = __builtin_fma(t, t, acc);
    t = (double)a.z - (double)b.z; acc = __builtin_fma(t, t, acc);
    t = (double)a.w - (double)b.w; acc = __builtin_fma(t, t, acc);
    return acc;
}

// Load chunk r of lane gl of a row (zeros past d).  VEC: d % 4 == 0 and rows
// 16-byte aligned, so a chunk is one dwordx4 load.
template <bool VEC>
__device__ __forceinline__ float4 load_chunk(const float *__restrict__ row, int d, int r, int gl)
{
    int i = (r * 32 + gl) * 4;
    if (VEC) {
        if (i < d) return *reinterpret_cast<const float4 *>(row + i);
        return make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        float4 v;
        v.x = i + 0 < d ? row[i + 0] : 0.f;
        v.y = i + 1 < d ? row[i + 1] : 0.f;
        v.z = i + 2 < d ? row[i + 2] : 0.f;
        v.w = i + 3 < d ? row[i + 3] : 0.f;
        return v;
    }
}

}  // namespace cng
