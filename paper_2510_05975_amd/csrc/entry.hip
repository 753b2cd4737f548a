// Entry point of the graph (Algorithm 3, phase 1: the navigating node is the
// point found nearest to the centroid of P).  Computed exactly here:
//   centroid c = float64 mean; each thread sums one dimension of one block of
//   4096 points sequentially, then one thread per dimension adds the block
//   sums in block order and divides by n;
//   entry = argmin over points of (squared float64 distance to c summed
//   sequentially over dimensions with fused multiply-adds, id).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

constexpr int64_t BLOCK_PTS = 4096;

__global__ void block_sums(const float *__restrict__ x, int64_t n, int d, int64_t nb,
                           double *__restrict__ blk)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * d) return;
    int64_t b = t / d;
    int i = (int)(t % d);
    int64_t p0 = b * BLOCK_PTS, p1 = p0 + BLOCK_PTS < n ? p0 + BLOCK_PTS : n;
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) s += (double)x[(size_t)p * d + i];
    blk[(size_t)b * d + i] = s;
}

__global__ void centroid(const double *__restrict__ blk, int64_t nb, int d, int64_t n,
                         double *__restrict__ c)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d) return;
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s += blk[(size_t)b * d + i];
    c[i] = s / (double)n;
}

struct DKey {
    double D;
    uint32_t id;
};

__device__ __forceinline__ bool dkey_less(DKey a, DKey b)
{
    return a.D < b.D || (a.D == b.D && a.id < b.id);
}

__device__ DKey block_min(DKey k)
{
    __shared__ double sD[256];
    __shared__ uint32_t sI[256];
    sD[threadIdx.x] = k.D;
    sI[threadIdx.x] = k.id;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            DKey o{sD[threadIdx.x + off], sI[threadIdx.x + off]};
            DKey m{sD[threadIdx.x], sI[threadIdx.x]};
            if (dkey_less(o, m)) {
                sD[threadIdx.x] = o.D;
                sI[threadIdx.x] = o.id;
            }
        }
        __syncthreads();
    }
    return DKey{sD[0], sI[0]};
}

__global__ __launch_bounds__(256) void nearest_partial(const float *__restrict__ x, int64_t n, int d,
                                                       const double *__restrict__ c,
                                                       double *__restrict__ pD,
                                                       uint32_t *__restrict__ pI)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    DKey k{__builtin_inf(), NONE};
    if (p < n) {
        const float *row = x + (size_t)p * d;
        double acc = 0.0;
        for (int i = 0; i < d; ++i) {
            double t = (double)row[i] - c[i];
            acc = __builtin_fma(t, t, acc);
        }
        k = DKey{acc, (uint32_t)p};
    }
    DKey m = block_min(k);
    if (threadIdx.x == 0) {
        pD[blockIdx.x] = m.D;
        pI[blockIdx.x] = m.id;
    }
}

__global__ __launch_bounds__(256) void nearest_final(const double *__restrict__ pD,
                                                     const uint32_t *__restrict__ pI, int64_t m,
                                                     uint32_t *__restrict__ entry)
{
    DKey k{__builtin_inf(), NONE};
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        DKey o{pD[j], pI[j]};
        if (dkey_less(o, k)) k = o;
    }
    DKey r = block_min(k);
    if (threadIdx.x == 0) *entry = r.id;
}

}  // namespace

size_t entry_workspace_bytes(int64_t n, int d)
{
    int64_t nb = (n + BLOCK_PTS - 1) / BLOCK_PTS;
    int64_t np = (n + 255) / 256;
    size_t b = (size_t)nb * d * 8 + (size_t)d * 8 + (size_t)np * 8 + (size_t)np * 4;
    return (b + 255) & ~(size_t)255;
}

hipError_t launch_entry(const float *points, int64_t n, int d, uint32_t *entry, void *ws,
                        hipStream_t stream)
{
    int64_t nb = (n + BLOCK_PTS - 1) / BLOCK_PTS;
    int64_t np = (n + 255) / 256;
    double *blk = (double *)ws;
    double *c = blk + (size_t)nb * d;
    double *pD = c + d;
    uint32_t *pI = (uint32_t *)(pD + np);
    int64_t tt = nb * d;
    hipLaunchKernelGGL(block_sums, dim3((unsigned)((tt + 255) / 256)), dim3(256), 0, stream, points,
                       n, d, nb, blk);
    hipLaunchKernelGGL(centroid, dim3((d + 255) / 256), dim3(256), 0, stream, blk, nb, d, n, c);
    hipLaunchKernelGGL(nearest_partial, dim3((unsigned)np), dim3(256), 0, stream, points, n, d, c,
                       pD, pI);
    hipLaunchKernelGGL(nearest_final, dim3(1), dim3(256), 0, stream, pD, pI, np, entry);
    return hipGetLastError();
}

}  // namespace cng
