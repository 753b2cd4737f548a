// Reduced-precision vector storage for the precision form of the search:
//   bf16: round to nearest even (8 significant bits);
//   fp8:  OCP E4M3 (exponent bias 7, largest finite 448, subnormal step 2^-9),
//         one float32 scale per vector s = max|x| / 448 (1 for a zero vector),
//         code = E4M3 rounding of x / s, ties to even, saturating at +-448;
//         the stored element stands for decode(code) * s (one float32 product).
//         Beside s each vector keeps n2 = fl(fl(s s) dot(c, c)), c the E4M3
//         values, dot the fixed-order dot product: the search scores fp8
//         vectors in the dot form fma(-2 s, dot(q, c), dot(q, q) + n2).
// Finite inputs are assumed.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

__global__ void quant_bf16(const float *__restrict__ x, int64_t total, uint16_t *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) out[t] = bf16_bits(x[t]);
}

// One wavefront per vector; sn [n x 2] receives (s, n2).
__global__ __launch_bounds__(256) void quant_fp8(const float *__restrict__ x, int64_t n, int d,
                                                 uint8_t *__restrict__ out, float *__restrict__ sn)
{
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (p >= n) return;
    const float *row = x + (size_t)p * d;
    float m = 0.f;
    for (int i = lane; i < d; i += 64) m = __builtin_fmaxf(m, __builtin_fabsf(row[i]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = __builtin_fmaxf(m, __shfl_xor(m, off, 64));
    const float s = m > 0.f ? m / 448.0f : 1.0f;
    for (int i = lane; i < d; i += 64) out[(size_t)p * d + i] = e4m3_encode(row[i] / s);
    // dot(c, c) in the fixed order: lane l < 32 takes elements (r*32 + l)*4 .. +3
    // for r = 0, 1, ... in increasing order, then the 16-8-4-2-1 butterfly
    float acc = 0.f;
    if (lane < 32) {
        for (int i0 = lane * 4; i0 < d; i0 += 128)
            for (int j = 0; j < 4 && i0 + j < d; ++j) {
                const float c = e4m3_value(e4m3_encode(row[i0 + j] / s));
                acc = __builtin_fmaf(c, c, acc);
            }
    }
    acc = group_sum<32>(acc);
    if (lane == 0) {
        const float ss = s * s;
        sn[2 * p] = s;
        sn[2 * p + 1] = ss * acc;
    }
}

}  // namespace

size_t quantized_bytes(int64_t n, int d, int dtype)
{
    return dtype == 1 ? (size_t)n * d * 2 : dtype == 2 ? (size_t)n * d : (size_t)n * d * 4;
}

hipError_t launch_quantize(const float *x, int64_t n, int d, int dtype, void *out, float *scales,
                           hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    if (dtype == 1) {
        const int64_t total = n * d;
        hipLaunchKernelGGL(quant_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, x,
                           total, (uint16_t *)out);
    } else {
        hipLaunchKernelGGL(quant_fp8, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, x, n, d,
                           (uint8_t *)out, scales);
    }
    return hipGetLastError();
}

}  // namespace cng
