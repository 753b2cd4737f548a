// Learned entry point: a multilayer perceptron d -> H -> H -> K (ReLU) maps a
// query to scores over K graph entry nodes; softmax cross-entropy against the
// entry that the plain search itself found best; Adam updates.  Not part of
// the paper (which starts every search at one navigating node, Algorithm 3);
// the navigating node stays the fallback when the network is not confident.
//
// Every matrix product runs on the matrix cores, one wavefront per 32 x 32
// output tile: bf16 inputs (v_mfma_f32_32x32x16_bf16) or float32 inputs
// (v_mfma_f32_32x32x2f32, used for gradient checks), float32 accumulation.
// Operands are read through strides, so transposed products need no copies.
// Prediction packs the weights and inputs to bf16 once and runs the same
// products on 16-byte fragment loads.
// Parameters, gradients and Adam moments are float32.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t as0, as1;  // A(i, k) = A[ri(i) * as0 + rk(k) * as1]
    const uint32_t *ri, *rk;  // optional index maps of A's first / second index
    const float *B;
    int64_t bs0, bs1;  // B(k, j) = B[k * bs0 + j * bs1]
    float *C;          // C[i * N + j]
    const float *bias; // optional, per column
    const float *mask; // optional: C(i, j) *= (mask[i * N + j] > 0)
    int relu;
};

__device__ __forceinline__ __bf16 to_bf16(float f)
{
    uint16_t b = bf16_bits(f);
    return __builtin_bit_cast(__bf16, b);
}

__device__ __forceinline__ int64_t aidx(const GemmArgs &g, int i, int k)
{
    const int64_t ii = g.ri ? (int64_t)g.ri[i] : i, kk = g.rk ? (int64_t)g.rk[k] : k;
    return ii * g.as0 + kk * g.as1;
}

template <bool BF16>
__global__ __launch_bounds__(64) void gemm_kernel(GemmArgs g)
{
    const int lane = lane_id();
    const int tilesN = (g.N + 31) / 32;
    const int ti = blockIdx.x / tilesN, tj = blockIdx.x % tilesN;
    const int i0 = ti * 32, j0 = tj * 32;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int ia = i0 + (lane & 31), jb = j0 + (lane & 31);
    const bool iok = ia < g.M, jok = jb < g.N;
    if (BF16) {
        // rows of A contiguous (forward products): two 16-byte loads per lane
        // and k step
        const bool avec = g.rk == nullptr && g.as1 == 1 && (g.K & 15) == 0 && (g.as0 & 3) == 0 &&
                          ((uintptr_t)g.A & 15) == 0;
        if (avec) {
            const float *arow = g.A + (iok ? (g.ri ? (int64_t)g.ri[ia] : ia) * g.as0 : 0);
            for (int k0 = 0; k0 < g.K; k0 += 16) {
                const int kb = k0 + (lane >> 5) * 8;
                float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
                if (iok) {
                    a0 = *reinterpret_cast<const float4 *>(arow + kb);
                    a1 = *reinterpret_cast<const float4 *>(arow + kb + 4);
                }
                bf16x8 av, bv;
                av[0] = to_bf16(a0.x); av[1] = to_bf16(a0.y); av[2] = to_bf16(a0.z); av[3] = to_bf16(a0.w);
                av[4] = to_bf16(a1.x); av[5] = to_bf16(a1.y); av[6] = to_bf16(a1.z); av[7] = to_bf16(a1.w);
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    bv[t] = to_bf16(jok ? g.B[(int64_t)(kb + t) * g.bs0 + jb * g.bs1] : 0.f);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
        } else {
            for (int k0 = 0; k0 < g.K; k0 += 16) {
                bf16x8 av, bv;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int k = k0 + (lane >> 5) * 8 + t;
                    const bool kok = k < g.K;
                    av[t] = to_bf16(iok && kok ? g.A[aidx(g, ia, k)] : 0.f);
                    bv[t] = to_bf16(jok && kok ? g.B[k * g.bs0 + jb * g.bs1] : 0.f);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
        }
    } else {
        for (int k0 = 0; k0 < g.K; k0 += 2) {
            const int k = k0 + (lane >> 5);
            const bool kok = k < g.K;
            const float av = iok && kok ? g.A[aidx(g, ia, k)] : 0.f;
            const float bv = jok && kok ? g.B[k * g.bs0 + jb * g.bs1] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + (lane & 31);
        if (i < g.M && j < g.N) {
            float v = acc[r];
            if (g.bias) v = v + g.bias[j];
            if (g.relu) v = v > 0.f ? v : 0.f;
            if (g.mask && !(g.mask[(int64_t)i * g.N + j] > 0.f)) v = 0.f;
            g.C[(int64_t)i * g.N + j] = v;
        }
    }
}

// Batch-deep products with few output tiles (the weight gradients): each of
// the GEMM_SPLIT waves of a workgroup accumulates one contiguous k range of the
// tile, and wave 0 adds the shares in wave order (a fixed order) before the
// same epilogue as gemm_kernel.
constexpr int GEMM_SPLIT = 8;

template <bool BF16>
__global__ __launch_bounds__(64 * GEMM_SPLIT) void gemm_splitk_kernel(GemmArgs g)
{
    __shared__ float part[GEMM_SPLIT - 1][16][64];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int tilesN = (g.N + 31) / 32;
    const int ti = blockIdx.x / tilesN, tj = blockIdx.x % tilesN;
    const int i0 = ti * 32, j0 = tj * 32;
    const int ia = i0 + (lane & 31), jb = j0 + (lane & 31);
    const bool iok = ia < g.M, jok = jb < g.N;
    constexpr int KS = BF16 ? 16 : 2;  // k per matrix instruction
    const int per = ((g.K + KS - 1) / KS + GEMM_SPLIT - 1) / GEMM_SPLIT * KS;
    const int kbeg = w * per, kend = (w + 1) * per < g.K ? (w + 1) * per : g.K;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    if (BF16) {
        for (int k0 = kbeg; k0 < kend; k0 += 16) {
            bf16x8 av, bv;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int k = k0 + (lane >> 5) * 8 + t;
                const bool kok = k < kend;
                av[t] = to_bf16(iok && kok ? g.A[aidx(g, ia, k)] : 0.f);
                bv[t] = to_bf16(jok && kok ? g.B[k * g.bs0 + jb * g.bs1] : 0.f);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
    } else {
        for (int k0 = kbeg; k0 < kend; k0 += 2) {
            const int k = k0 + (lane >> 5);
            const bool kok = k < kend;
            const float av = iok && kok ? g.A[aidx(g, ia, k)] : 0.f;
            const float bv = jok && kok ? g.B[k * g.bs0 + jb * g.bs1] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
        }
    }
    if (w > 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) part[w - 1][r][lane] = acc[r];
    }
    __syncthreads();
    if (w != 0) return;
    for (int q = 0; q < GEMM_SPLIT - 1; ++q) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += part[q][r][lane];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = j0 + (lane & 31);
        if (i < g.M && j < g.N) {
            float v = acc[r];
            if (g.bias) v = v + g.bias[j];
            if (g.relu) v = v > 0.f ? v : 0.f;
            if (g.mask && !(g.mask[(int64_t)i * g.N + j] > 0.f)) v = 0.f;
            g.C[(int64_t)i * g.N + j] = v;
        }
    }
}

// splitk: a batch-deep product (weight gradient); with fewer than 128 output
// tiles its k range is shared by the waves of a workgroup
hipError_t gemm(const GemmArgs &g, bool bf16, hipStream_t st, bool splitk = false)
{
    const unsigned tiles = (unsigned)(((g.M + 31) / 32) * ((g.N + 31) / 32));
    if (splitk && tiles < 128) {
        if (bf16) hipLaunchKernelGGL(gemm_splitk_kernel<true>, dim3(tiles), dim3(64 * GEMM_SPLIT), 0, st, g);
        else hipLaunchKernelGGL(gemm_splitk_kernel<false>, dim3(tiles), dim3(64 * GEMM_SPLIT), 0, st, g);
        return hipGetLastError();
    }
    if (bf16) hipLaunchKernelGGL(gemm_kernel<true>, dim3(tiles), dim3(64), 0, st, g);
    else hipLaunchKernelGGL(gemm_kernel<false>, dim3(tiles), dim3(64), 0, st, g);
    return hipGetLastError();
}

// Softmax cross-entropy per row (one wavefront per row): loss[i] and
// dZ = (softmax(Z) - onehot(label)) / B.
__global__ __launch_bounds__(256) void softmax_xent(const float *__restrict__ Z, const uint32_t *__restrict__ lab,
                                                    const uint32_t *__restrict__ idx, int B, int K,
                                                    float *__restrict__ dZ, float *__restrict__ loss)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (i >= B) return;
    const float *z = Z + i * K;
    float m = -__builtin_inff();
    for (int j = lane; j < K; j += 64) m = __builtin_fmaxf(m, z[j]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = __builtin_fmaxf(m, __shfl_xor(m, off, 64));
    float s = 0.f;
    for (int j = lane; j < K; j += 64) s += expf(z[j] - m);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const uint32_t y = lab[idx ? idx[i] : i];  // a label >= K contributes no target
    const float inv = 1.f / s;
    for (int j = lane; j < K; j += 64) {
        const float p = expf(z[j] - m) * inv;
        dZ[i * K + j] = (p - (j == (int)y ? 1.f : 0.f)) / (float)B;
    }
    if (lane == 0) loss[i] = y < (uint32_t)K ? (m + logf(s)) - z[y] : 0.f;
}

// Column sums (bias gradients), one thread per column, rows in order.
// Column sums of X [B x N] (the bias gradients): a workgroup of 16 waves owns
// 64 columns (lane = column); wave w sums rows w, w + 16, ..., and the 16
// partial sums are added in wave order (a fixed order: the same bits on every
// run).
constexpr int COLSUM_WAVES = 16;
__global__ __launch_bounds__(64 * COLSUM_WAVES) void colsum(const float *__restrict__ X, int B, int N,
                                                           float *__restrict__ out)
{
    __shared__ float part[COLSUM_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (j < N) {
#pragma unroll 8
        for (int i = w; i < B; i += COLSUM_WAVES) s += X[(int64_t)i * N + j];
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N) {
        float t = 0.f;
        for (int k = 0; k < COLSUM_WAVES; ++k) t += part[k][lane];
        out[j] = t;
    }
}

// Mean of x [n] in float64: strided partial sums per thread, then a fixed tree.
__global__ __launch_bounds__(256) void mean_of(const float *__restrict__ x, int n, float *__restrict__ out)
{
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(part[0] / n);
}

// Input affine of the network: out[i * d + c] = (X[row(i) * d + c] - mean[c]) / scale
// in float32 (row(i) = idx[i], or i without an index map).
__global__ void standardize_rows(const float *__restrict__ X, const uint32_t *__restrict__ idx,
                                 int B, int d, const float *__restrict__ mean,
                                 const float *__restrict__ scale, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * d) return;
    const int64_t i = t / d, c = t % d;
    const int64_t r = idx ? (int64_t)idx[i] : i;
    out[t] = (X[r * d + c] - mean[c]) / scale[0];
}

// Statistics of the training inputs: per-column sums of a block of STAT_ROWS
// rows in float64 (rows in order), then the block sums in block order.
constexpr int STAT_ROWS = 4096;
__global__ __launch_bounds__(256) void column_block_sums(const float *__restrict__ X, int64_t n, int d,
                                                         double *__restrict__ part)
{
    const int64_t r0 = (int64_t)blockIdx.x * STAT_ROWS;
    const int64_t r1 = r0 + STAT_ROWS < n ? r0 + STAT_ROWS : n;
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)X[r * d + c];
        part[(int64_t)blockIdx.x * d + c] = s;
    }
}

__global__ void column_means(const double *__restrict__ part, int nb, int64_t n, int d,
                             float *__restrict__ mean)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * d + c];
    mean[c] = (float)(s / (double)n);
}

// Sum of squared deviations from the (float32) column means, per row block.
__global__ __launch_bounds__(256) void block_sq_dev(const float *__restrict__ X, int64_t n, int d,
                                                    const float *__restrict__ mean,
                                                    double *__restrict__ part)
{
    __shared__ double red[256];
    const int64_t r0 = (int64_t)blockIdx.x * STAT_ROWS;
    const int64_t r1 = r0 + STAT_ROWS < n ? r0 + STAT_ROWS : n;
    double s = 0.0;
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        const double m = (double)mean[c];
        for (int64_t r = r0; r < r1; ++r) {
            const double t = (double)X[r * d + c] - m;
            s += t * t;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void rms_scale(const double *__restrict__ part, int nb, int64_t n, int d,
                          float *__restrict__ scale)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    const double r = sqrt(s / ((double)n * d));
    scale[0] = r > 1e-12 ? (float)r : 1e-12f;
}

__global__ void adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                     float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                     float c1, float c2)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    w[t] = w[t] - lr * (mt / c1) / (__builtin_sqrtf(vt / c2) + eps);
}

// Entry choice: argmax of the scores (ties to the lower index) and its softmax
// probability; below theta the navigating node is used instead.
// ---- prediction-only products on packed bf16 operands
// out[r * cols + c] = bf16(src[r * s0 + c * s1]): inputs row by row, weights
// transposed so that a column's k values are contiguous.
__global__ void pack_bf16(const float *__restrict__ src, int64_t rows, int cols, int64_t s0,
                          int64_t s1, uint16_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    const int64_t r = t / cols, c = t % cols;
    out[t] = bf16_bits(src[r * s0 + c * s1]);
}

// out[i * d + c] = bf16((X[i * d + c] - mean[c]) / scale), or bf16(X) without
// an input affine: the first layer's operand, rounded as gemm_kernel rounds it.
__global__ void pack_inputs(const float *__restrict__ X, int64_t B, int d,
                            const float *__restrict__ mean, const float *__restrict__ scale,
                            uint16_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * d) return;
    const float v = X[t];
    out[t] = bf16_bits(mean ? (v - mean[t % d]) / scale[0] : v);
}

// C = A Bt^T + bias with A [M x K] and Bt [N x K] bf16 (K a multiple of 16):
// the same bf16 operands, k order and matrix instruction as gemm_kernel, so
// the float32 results are identical; every fragment is one 16-byte load.  A
// wave computes 32 x (32 NJ) outputs (the A fragment serves NJ products);
// RELU writes relu(C) rounded to bf16 (the next layer's operand), otherwise C
// is written in float32.
template <int NJ, bool RELU>
__global__ __launch_bounds__(256) void gemm_packed(const uint16_t *__restrict__ A,
                                                   const uint16_t *__restrict__ Bt, int M, int N,
                                                   int K, const float *__restrict__ bias,
                                                   float *__restrict__ Cf, uint16_t *__restrict__ Cb)
{
    const int lane = lane_id();
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tilesN = (N + 32 * NJ - 1) / (32 * NJ);
    if (tile >= (int64_t)((M + 31) / 32) * tilesN) return;
    const int i0 = (int)(tile / tilesN) * 32, j0 = (int)(tile % tilesN) * 32 * NJ;
    const int ia = i0 + (lane & 31) < M ? i0 + (lane & 31) : M - 1;
    const uint16_t *arow = A + (int64_t)ia * K + (lane >> 5) * 8;
    const uint16_t *brow[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int jb = j0 + j * 32 + (lane & 31);
        brow[j] = Bt + (int64_t)(jb < N ? jb : N - 1) * K + (lane >> 5) * 8;
    }
    floatx16 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = floatx16{};
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(arow + k0);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(brow[j] + k0);
            acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int c = j0 + j * 32 + (lane & 31);
            if (i < M && c < N) {
                float v = acc[j][r] + bias[c];
                if (RELU) {
                    v = v > 0.f ? v : 0.f;
                    Cb[(int64_t)i * N + c] = bf16_bits(v);
                } else {
                    Cf[(int64_t)i * N + c] = v;
                }
            }
        }
}

__global__ __launch_bounds__(256) void predict_entry(const float *__restrict__ Z, int B, int K,
                                                     const uint32_t *__restrict__ entries,
                                                     uint32_t fallback, float theta,
                                                     uint32_t *__restrict__ out,
                                                     float *__restrict__ conf)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (i >= B) return;
    const float *z = Z + i * K;
    float m = -__builtin_inff();
    int am = 0x7FFFFFFF;
    for (int j = lane; j < K; j += 64)
        if (z[j] > m) {
            m = z[j];
            am = j;
        }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float om = __shfl_xor(m, off, 64);
        const int oa = __shfl_xor(am, off, 64);
        if (om > m || (om == m && oa < am)) {
            m = om;
            am = oa;
        }
    }
    float s = 0.f;
    for (int j = lane; j < K; j += 64) s += expf(z[j] - m);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const float p = 1.f / s;
        if (conf) conf[i] = p;
        out[i] = (am < K && p >= theta) ? entries[am] : fallback;
    }
}

}  // namespace

// ---------------------------------------------------------------- host side
MlpShape::MlpShape(int d_, int H_, int K_) : d(d_), H(H_), K(K_)
{
    oW1 = 0;
    ob1 = oW1 + (int64_t)d * H;
    oW2 = ob1 + H;
    ob2 = oW2 + (int64_t)H * H;
    oW3 = ob2 + H;
    ob3 = oW3 + (int64_t)H * K;
    total = ob3 + K;
}

static size_t mlp_base_floats(const MlpShape &s, int B)
{
    // H1, H2, Z, dZ, dH2, dH1, loss, then the standardized inputs [B x d]
    return ((size_t)B * s.H * 4 + (size_t)B * s.K * 2 + (size_t)B + 64 + 3) / 4 * 4 +
           ((size_t)B * s.d + 3) / 4 * 4;
}

static float *std_inputs(const MlpShape &s, float *ws, int B)
{
    return ws + ((size_t)B * s.H * 4 + (size_t)B * s.K * 2 + (size_t)B + 64 + 3) / 4 * 4;
}

size_t mlp_stats_workspace_bytes(int64_t n, int d)
{
    const int64_t nb = (n + STAT_ROWS - 1) / STAT_ROWS;
    return (size_t)nb * d * 8 + (size_t)nb * 8 + 256;
}

hipError_t mlp_input_stats(const float *X, int64_t n, int d, float *mean, float *scale, void *ws,
                           hipStream_t st)
{
    const int nb = (int)((n + STAT_ROWS - 1) / STAT_ROWS);
    double *part = (double *)ws;
    double *part2 = part + (size_t)nb * d;
    hipLaunchKernelGGL(column_block_sums, dim3(nb), dim3(256), 0, st, X, n, d, part);
    hipLaunchKernelGGL(column_means, dim3((d + 255) / 256), dim3(256), 0, st, part, nb, n, d, mean);
    hipLaunchKernelGGL(block_sq_dev, dim3(nb), dim3(256), 0, st, X, n, d, mean, part2);
    hipLaunchKernelGGL(rms_scale, dim3(1), dim3(64), 0, st, part2, nb, n, d, scale);
    return hipGetLastError();
}

// The first layer's input: X itself, or its standardized rows in the workspace.
static const float *first_input(const MlpShape &s, const float *X, const uint32_t *&idx, int B,
                                const float *mean, const float *scale, float *ws, hipStream_t st)
{
    if (!mean) return X;
    float *Xs = std_inputs(s, ws, B);
    const int64_t t = (int64_t)B * s.d;
    hipLaunchKernelGGL(standardize_rows, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, X, idx,
                       B, s.d, mean, scale, Xs);
    idx = nullptr;
    return Xs;
}

size_t mlp_workspace_floats(const MlpShape &s, int B)
{
    // then, for prediction, packed bf16 weights (transposed) and inputs
    const size_t halves = (size_t)s.d * s.H + (size_t)s.H * s.H + (size_t)s.K * s.H + (size_t)B * s.d;
    return mlp_base_floats(s, B) + (halves + 1) / 2 + 64;
}

static GemmArgs mk(int M, int N, int K, const float *A, int64_t as0, int64_t as1, const float *B,
                   int64_t bs0, int64_t bs1, float *C, const float *bias, const float *mask, int relu,
                   const uint32_t *ri = nullptr, const uint32_t *rk = nullptr)
{
    GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.as0 = as0; g.as1 = as1; g.ri = ri; g.rk = rk;
    g.B = B; g.bs0 = bs0; g.bs1 = bs1;
    g.C = C; g.bias = bias; g.mask = mask; g.relu = relu;
    return g;
}

hipError_t mlp_forward(const MlpShape &s, const float *P, const float *X, const uint32_t *idx, int B,
                       bool bf16, float *ws, float *Z_out, hipStream_t st, const float *mean,
                       const float *scale)
{
    X = first_input(s, X, idx, B, mean, scale, ws, st);
    float *H1 = ws, *H2 = H1 + (size_t)B * s.H;
    float *Z = Z_out ? Z_out : H2 + (size_t)B * s.H * 3;
    hipError_t e;
    e = gemm(mk(B, s.H, s.d, X, s.d, 1, P + s.oW1, s.H, 1, H1, P + s.ob1, nullptr, 1, idx), bf16, st);
    if (e != hipSuccess) return e;
    e = gemm(mk(B, s.H, s.H, H1, s.H, 1, P + s.oW2, s.H, 1, H2, P + s.ob2, nullptr, 1), bf16, st);
    if (e != hipSuccess) return e;
    return gemm(mk(B, s.K, s.H, H2, s.H, 1, P + s.oW3, s.K, 1, Z, P + s.ob3, nullptr, 0), bf16, st);
}

hipError_t mlp_gradients(const MlpShape &s, const float *P, const float *X, const uint32_t *lab,
                         const uint32_t *idx, int B, bool bf16, float *ws, float *G,
                         float *loss_mean, hipStream_t st, const float *mean, const float *scale)
{
    float *H1 = ws, *H2 = H1 + (size_t)B * s.H;
    float *dH2 = H2 + (size_t)B * s.H, *dH1 = dH2 + (size_t)B * s.H;
    float *Z = dH1 + (size_t)B * s.H, *dZ = Z + (size_t)B * s.K, *loss = dZ + (size_t)B * s.K;
    const uint32_t *lab_idx = idx;  // labels stay indexed by the batch's rows
    X = first_input(s, X, idx, B, mean, scale, ws, st);
    hipError_t e = mlp_forward(s, P, X, idx, B, bf16, ws, Z, st, nullptr, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(softmax_xent, dim3((B + 3) / 4), dim3(256), 0, st, Z, lab, lab_idx, B, s.K, dZ, loss);
    if (loss_mean) hipLaunchKernelGGL(mean_of, dim3(1), dim3(256), 0, st, loss, B, loss_mean);
    // layer 3: dW3 = H2^T dZ, db3 = colsum dZ, dH2 = (dZ W3^T) * (H2 > 0)
    e = gemm(mk(s.H, s.K, B, H2, 1, s.H, dZ, s.K, 1, G + s.oW3, nullptr, nullptr, 0), bf16, st, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum, dim3((s.K + 63) / 64), dim3(64 * COLSUM_WAVES), 0, st, dZ, B, s.K, G + s.ob3);
    e = gemm(mk(B, s.H, s.K, dZ, s.K, 1, P + s.oW3, 1, s.K, dH2, nullptr, H2, 0), bf16, st);
    if (e != hipSuccess) return e;
    // layer 2
    e = gemm(mk(s.H, s.H, B, H1, 1, s.H, dH2, s.H, 1, G + s.oW2, nullptr, nullptr, 0), bf16, st, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum, dim3((s.H + 63) / 64), dim3(64 * COLSUM_WAVES), 0, st, dH2, B, s.H, G + s.ob2);
    e = gemm(mk(B, s.H, s.H, dH2, s.H, 1, P + s.oW2, 1, s.H, dH1, nullptr, H1, 0), bf16, st);
    if (e != hipSuccess) return e;
    // layer 1
    e = gemm(mk(s.d, s.H, B, X, 1, s.d, dH1, s.H, 1, G + s.oW1, nullptr, nullptr, 0, nullptr, idx),
             bf16, st, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum, dim3((s.H + 63) / 64), dim3(64 * COLSUM_WAVES), 0, st, dH1, B, s.H, G + s.ob1);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpShape &s, float *P, const float *G, float *M1, float *M2, int step,
                    float lr, float b1, float b2, float eps, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam, dim3((unsigned)((s.total + 255) / 256)), dim3(256), 0, st, P, G, M1, M2,
                       s.total, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// hidden [2 x B x H] = the activations as the next product reads them:
// float32 values, rounded to bf16 first when `round` is set.
__global__ void widen_hidden(const float *__restrict__ Hf, const uint16_t *__restrict__ Hb,
                             int64_t m, int round, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    if (Hb) out[t] = __uint_as_float((uint32_t)Hb[t] << 16);
    else out[t] = round ? __uint_as_float((uint32_t)bf16_bits(Hf[t]) << 16) : Hf[t];
}

// Scores Z [B x K] of the queries.  bf16: on packed operands (every operand
// rounded to bf16 once, as gemm_kernel rounds it on load) when d and H are
// multiples of 16, else through mlp_forward.  hidden (optional): the two
// hidden layers as the next products read them.
hipError_t mlp_scores(const MlpShape &s, const float *P, const float *X, int B, bool bf16,
                      float *ws, float *Z, hipStream_t st, const float *mean, const float *scale,
                      float *hidden)
{
    const int64_t bh = (int64_t)B * s.H;
    auto widen = [&](const float *Hf, const uint16_t *Hb, float *out) {
        hipLaunchKernelGGL(widen_hidden, dim3((unsigned)((bh + 255) / 256)), dim3(256), 0, st, Hf, Hb,
                           bh, bf16 ? 1 : 0, out);
    };
    hipError_t e = hipSuccess;
    if (bf16 && s.d % 16 == 0 && s.H % 16 == 0 && B > 0) {
        // packed operands: bf16 activations in the H1 / H2 areas, weights and
        // inputs after the training areas (every part 16-byte aligned)
        uint16_t *H1b = reinterpret_cast<uint16_t *>(ws);
        uint16_t *H2b = reinterpret_cast<uint16_t *>(ws + (size_t)B * s.H);
        uint16_t *W1t = reinterpret_cast<uint16_t *>(ws + mlp_base_floats(s, B));
        uint16_t *W2t = W1t + (size_t)s.d * s.H;
        uint16_t *W3t = W2t + (size_t)s.H * s.H;
        uint16_t *Xb = W3t + ((size_t)s.K * s.H + 7) / 8 * 8;
        auto pack = [&](const float *src, int64_t rows, int cols, int64_t s0, int64_t s1, uint16_t *dst) {
            const int64_t t = rows * cols;
            hipLaunchKernelGGL(pack_bf16, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, src, rows,
                               cols, s0, s1, dst);
        };
        pack(P + s.oW1, s.H, s.d, 1, s.H, W1t);  // W1 (k, j) = W1[k * H + j]
        pack(P + s.oW2, s.H, s.H, 1, s.H, W2t);
        pack(P + s.oW3, s.K, s.H, 1, s.K, W3t);  // W3 (k, j) = W3[k * K + j]
        const int64_t tx = (int64_t)B * s.d;
        hipLaunchKernelGGL(pack_inputs, dim3((unsigned)((tx + 255) / 256)), dim3(256), 0, st, X,
                           (int64_t)B, s.d, mean, scale, Xb);
        auto grid = [&](int N) {
            const int64_t tiles = (int64_t)((B + 31) / 32) * ((N + 127) / 128);
            return dim3((unsigned)((tiles + 3) / 4));
        };
        hipLaunchKernelGGL((gemm_packed<4, true>), grid(s.H), dim3(256), 0, st, Xb, W1t, B, s.H, s.d,
                           P + s.ob1, nullptr, H1b);
        hipLaunchKernelGGL((gemm_packed<4, true>), grid(s.H), dim3(256), 0, st, H1b, W2t, B, s.H, s.H,
                           P + s.ob2, nullptr, H2b);
        hipLaunchKernelGGL((gemm_packed<4, false>), grid(s.K), dim3(256), 0, st, H2b, W3t, B, s.K, s.H,
                           P + s.ob3, Z, nullptr);
        if (hidden) {
            widen(nullptr, H1b, hidden);
            widen(nullptr, H2b, hidden + bh);
        }
        e = hipGetLastError();
    } else {
        e = mlp_forward(s, P, X, nullptr, B, bf16, ws, Z, st, mean, scale);
        if (e == hipSuccess && hidden) {
            widen(ws, nullptr, hidden);
            widen(ws + bh, nullptr, hidden + bh);
            e = hipGetLastError();
        }
    }
    return e;
}

hipError_t mlp_predict(const MlpShape &s, const float *P, const float *X, int B, bool bf16,
                       const uint32_t *entries, uint32_t fallback, float theta, float *ws,
                       uint32_t *out, float *conf, hipStream_t st, const float *mean,
                       const float *scale)
{
    float *Z = ws + (size_t)B * s.H * 2;
    hipError_t e = mlp_scores(s, P, X, B, bf16, ws, Z, st, mean, scale, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(predict_entry, dim3((B + 3) / 4), dim3(256), 0, st, Z, B, s.K, entries,
                       fallback, theta, out, conf);
    return hipGetLastError();
}

}  // namespace cng
