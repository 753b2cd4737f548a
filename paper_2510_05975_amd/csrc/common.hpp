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

// Lane exchange v[lane ^ OFF] within aligned groups of 32 lanes: DPP quad
// permutations for offsets 1 and 2, a DPP rotation of the 16-lane row by 8
// (lane i of a row takes lane (i + 8) mod 16 = i ^ 8) for offset 8,
// ds_swizzle (xor mode) for 4 and 16.
template <int OFF>
__device__ __forceinline__ float xor_lane(float v)
{
    const int x = __float_as_int(v);
    int r;
    if (OFF == 1) r = __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);       // quad_perm [1,0,3,2]
    else if (OFF == 2) r = __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else if (OFF == 8) r = __builtin_amdgcn_update_dpp(x, x, 0x128, 0xF, 0xF, false); // row_ror:8
    else r = __builtin_amdgcn_ds_swizzle(x, 0x1F | (OFF << 10));                      // and 0x1F, xor OFF
    return __int_as_float(r);
}

// a[l] + a[l ^ 16] for the lanes of even 16-lane rows and b[l] + b[l ^ 16] for
// those of odd rows, with one gfx950 row swap: it exchanges the odd rows of a
// with the even rows of b, after which the two registers hold, lane by lane,
// exactly the two addends (in some order; the sum is the same).
__device__ __forceinline__ float swap16_sum(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Fixed-order sums of UB vectors at once.  v[t] holds this lane's partial sum
// of vector t (lanes of a group of G, G <= 32, UB <= G).  Each step pairs lane
// l with lane l ^ off, the pairing of the butterfly, so every sum is the
// butterfly of one vector, bit for bit; but a step that still holds several
// vectors per lane sends half of them to the partner and keeps the other
// half (recursive halving), so the UB butterflies cost about UB exchanges in
// total instead of UB * log2(G).  On return, lanes
// [t * (G / UB), (t + 1) * (G / UB)) of the group hold the sum of vector t.
template <int G, int UB, int OFF, int N>
__device__ __forceinline__ void halve_step(float (&v)[UB], int gl)
{
    if constexpr (OFF == 16) {
        // lanes below 16 of a group keep vector j, the others vector j + N/2
        if constexpr (N > 1) {
#pragma unroll
            for (int j = 0; j < N / 2; ++j) v[j] = swap16_sum(v[j], v[j + N / 2]);
            halve_step<G, UB, 8, N / 2>(v, gl);
        } else {
            v[0] = swap16_sum(v[0], v[0]);
            halve_step<G, UB, 8, 1>(v, gl);
        }
    } else if constexpr (OFF >= 1) {
        if constexpr (N > 1) {
            const bool hi = (gl & OFF) != 0;
#pragma unroll
            for (int j = 0; j < N / 2; ++j) {
                const float keep = hi ? v[j + N / 2] : v[j];
                const float send = hi ? v[j] : v[j + N / 2];
                v[j] = keep + xor_lane<OFF>(send);
            }
            halve_step<G, UB, OFF / 2, N / 2>(v, gl);
        } else {
            v[0] = v[0] + xor_lane<OFF>(v[0]);
            halve_step<G, UB, OFF / 2, 1>(v, gl);
        }
    }
}

template <int G, int UB>
__device__ __forceinline__ void group_sums(float (&v)[UB], int gl)
{
    static_assert(UB <= G && G <= 32, "group_sums: UB <= G <= 32");
    halve_step<G, UB, G / 2, UB>(v, gl);
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

// Partial sum of one lane for the fixed-order dot product: chunk r of lane gl
// covers elements (r*32 + gl)*4 .. +3, acc = fma(a_i, b_i, acc) in order.
__device__ __forceinline__ float chunk_dot(float4 a, float4 b, float acc)
{
    acc = __builtin_fmaf(a.x, b.x, acc);
    acc = __builtin_fmaf(a.y, b.y, acc);
    acc = __builtin_fmaf(a.z, b.z, acc);
    acc = __builtin_fmaf(a.w, b.w, acc);
    return acc;
}

// fp8 score from the fixed-order dot product of the query with the E4M3
// values c of a stored vector, the query's squared norm qq (fixed order) and
// the vector's scale s and n2 = fl(fl(s s) dot(c, c)):
// fma(-2 s, dot, qq + n2), clamped at +0 (the dot form of |q - s c|^2).
__device__ __forceinline__ float fp8_score(float dot, float qq, float s, float n2)
{
    const float D = __builtin_fmaf(-2.0f * s, dot, qq + n2);
    return D > 0.0f ? D : 0.0f;
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


// ---- reduced-precision element codecs (bit-level; finite inputs)
// float32 -> bf16 bits, round to nearest even.
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// float32 -> OCP E4M3 code, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint8_t e4m3_encode(float v)
{
    const uint32_t u = __float_as_uint(v);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7FFFFFFFu;
    const float af = __uint_as_float(a);
    if (af >= 448.0f) return (uint8_t)(sign | 0x7Eu);
    int E = (int)(a >> 23) - 127;
    if (E < -6) {  // below the smallest normal 2^-6: multiples of 2^-9
        const float k = __builtin_rintf(af * 512.0f);
        return (uint8_t)(sign | (uint32_t)k);
    }
    uint32_t r = (a & 0x7FFFFFu) + 0x7FFFFu + (((a & 0x7FFFFFu) >> 20) & 1u);
    if (r & 0x800000u) {  // mantissa rounding carried into the exponent
        E += 1;
        r = 0;
    }
    const uint32_t mant = (r >> 20) & 7u;
    if (E > 8 || (E == 8 && mant == 7u)) return (uint8_t)(sign | 0x7Eu);
    return (uint8_t)(sign | ((uint32_t)(E + 7) << 3) | mant);
}

// E4M3 code -> float32 value (exact).
__device__ __forceinline__ float e4m3_value(uint32_t c)
{
    const uint32_t e = (c >> 3) & 0xFu, mt = c & 7u;
    float v = e == 0 ? (float)mt * 0x1p-9f : __uint_as_float(((e + 120u) << 23) | (mt << 20));
    return (c & 0x80u) ? -v : v;
}

// Chunk r of lane gl (elements (r*32 + gl)*4 .. +3) of a stored row, as
// float32 values.  ST 0: float32, 1: bf16, 2: fp8 E4M3 values (unscaled: the
// fp8 score applies the scale after the dot product).  VEC: d % 4 == 0 and
// the row base aligned to one chunk (one vector load).
template <int ST, bool VEC>
__device__ __forceinline__ float4 load_stored(const void *__restrict__ base, size_t row, int d, int r,
                                              int gl)
{
    const int i = (r * 32 + gl) * 4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ST == 0) {
        return load_chunk<VEC>(reinterpret_cast<const float *>(base) + row * (uint32_t)d, d, r, gl);
    } else if (ST == 1) {
        const uint16_t *p = reinterpret_cast<const uint16_t *>(base) + row * (uint32_t)d + i;
        if (VEC) {
            if (i < d) {
                const uint2 w = *reinterpret_cast<const uint2 *>(p);
                v = make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                                __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
            }
        } else {
            v.x = i + 0 < d ? bf16_value(p[0]) : 0.f;
            v.y = i + 1 < d ? bf16_value(p[1]) : 0.f;
            v.z = i + 2 < d ? bf16_value(p[2]) : 0.f;
            v.w = i + 3 < d ? bf16_value(p[3]) : 0.f;
        }
        return v;
    } else {
        const uint8_t *p = reinterpret_cast<const uint8_t *>(base) + row * (uint32_t)d + i;
        if (VEC) {
            if (i < d) {
                const uint32_t w = *reinterpret_cast<const uint32_t *>(p);
                v = make_float4(e4m3_value(w & 0xFFu), e4m3_value((w >> 8) & 0xFFu),
                                e4m3_value((w >> 16) & 0xFFu), e4m3_value(w >> 24));
            }
        } else {
            v.x = i + 0 < d ? e4m3_value(p[0]) : 0.f;
            v.y = i + 1 < d ? e4m3_value(p[1]) : 0.f;
            v.z = i + 2 < d ? e4m3_value(p[2]) : 0.f;
            v.w = i + 3 < d ? e4m3_value(p[3]) : 0.f;
        }
        return v;
    }
}

// Raw words of chunk r of lane gl of a stored row (no use of the loaded value,
// so a batch of these loads stays in flight together); decode_chunk turns them
// into the float32 values.  VEC layout only (d % 4 == 0, aligned rows).
template <int ST> struct RawChunk;
template <> struct RawChunk<0> { typedef float4 type; };
template <> struct RawChunk<1> { typedef uint2 type; };
template <> struct RawChunk<2> { typedef uint32_t type; };

template <int ST, bool GUARD = true>
__device__ __forceinline__ typename RawChunk<ST>::type load_raw(const void *__restrict__ base, size_t row,
                                                                int d, int r, int gl)
{
    typedef typename RawChunk<ST>::type T;
    const int i = (r * 32 + gl) * 4;
    if (GUARD && i >= d) return T{};  // without GUARD the caller knows every chunk is in the row
    if (ST == 0) return *reinterpret_cast<const T *>(reinterpret_cast<const float *>(base) + row * (uint32_t)d + i);
    if (ST == 1) return *reinterpret_cast<const T *>(reinterpret_cast<const uint16_t *>(base) + row * (uint32_t)d + i);
    return *reinterpret_cast<const T *>(reinterpret_cast<const uint8_t *>(base) + row * (uint32_t)d + i);
}

__device__ __forceinline__ float4 decode_chunk(float4 w) { return w; }
__device__ __forceinline__ float4 decode_chunk(uint2 w)
{
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                       __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
}
// fp8: the gfx950 conversion instruction widens two E4M3 codes per call
// (exact E4M3 values, unscaled).
__device__ __forceinline__ float4 decode_chunk(uint32_t w)
{
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    return make_float4(lo[0], lo[1], hi[0], hi[1]);
}

// Bitonic sort of n (power of two) 64-bit keys in LDS by one wavefront.
__device__ inline void wave_sort(uint64_t *k, int n)
{
    const int lane = lane_id();
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_sync();
            for (int t = lane; t < n / 2; t += 64) {
                int i = 2 * t - (t & (stride - 1));
                int j = i + stride;
                bool up = (i & size) == 0;
                uint64_t a = k[i], b = k[j];
                if ((a > b) == up) {
                    k[i] = b;
                    k[j] = a;
                }
            }
        }
    }
    wave_sync();
}

}  // namespace cng
