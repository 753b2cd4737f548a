// k-means (Lloyd) for the entry nodes of the learned entry point.  The
// assignment step is the exact candidate stage with one candidate (nearest
// centre by (D, id)); the update sums assigned points with float atomics (the
// summation order is not fixed, so centres may differ in the last bits between
// runs: k-means is an input to the learned part, not a pinned result).  Empty
// clusters keep their centre.  Entry node j = the point nearest centre j.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

__global__ void gather_rows(const float *__restrict__ x, int d, const uint32_t *__restrict__ ids,
                            int K, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)K * d) return;
    out[t] = x[(size_t)ids[t / d] * d + t % d];
}

__global__ void zero_f(float *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.f;
}

__global__ void accumulate(const float *__restrict__ x, int64_t n, int d,
                           const uint32_t *__restrict__ assign, float *sums, float *counts)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * d) return;
    const int64_t p = t / d;
    const int i = (int)(t % d);
    const uint32_t c = assign[p];
    atomicAdd(&sums[(size_t)c * d + i], x[t]);
    if (i == 0) atomicAdd(&counts[c], 1.f);
}

__global__ void finalize(const float *__restrict__ sums, const float *__restrict__ counts, int K,
                         int d, float *__restrict__ centers)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)K * d) return;
    const float c = counts[t / d];
    if (c > 0.f) centers[t] = sums[t] / c;
}

__global__ void map_ids(const uint32_t *__restrict__ idx, int64_t m, const uint32_t *__restrict__ table,
                        uint32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const uint32_t j = idx[t];
    out[t] = j == NONE ? NONE : table[j];
}

}  // namespace

hipError_t gather_points(const float *x, int d, const uint32_t *ids, int64_t m, float *out,
                         hipStream_t st)
{
    const int64_t t = m * d;
    if (t == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, x, d, ids,
                       (int)m, out);
    return hipGetLastError();
}

hipError_t map_through(const uint32_t *idx, int64_t m, const uint32_t *table, uint32_t *out,
                       hipStream_t st)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(map_ids, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, idx, m, table, out);
    return hipGetLastError();
}

size_t kmeans_workspace_bytes(int64_t n, int d, int K)
{
    KnnPlan a = knn_plan(n, K, d, 1, 0), b = knn_plan(K, n, d, 1, 0);
    size_t knn = a.bytes > b.bytes ? a.bytes : b.bytes;
    return align256(knn) + align256((size_t)n * 4) * 2 + align256((size_t)K * d * 4) +
           align256((size_t)K * 4) * 2;
}

hipError_t run_kmeans(const float *points, int64_t n, int d, int K, int iters,
                      const uint32_t *init_ids, float *centers, uint32_t *entries, void *ws,
                      hipStream_t st)
{
    KnnPlan pa = knn_plan(n, K, d, 1, 0), pb = knn_plan(K, n, d, 1, 0);
    unsigned char *w = (unsigned char *)ws;
    void *kws = w;
    w += align256(pa.bytes > pb.bytes ? pa.bytes : pb.bytes);
    uint32_t *assign = (uint32_t *)w;
    w += align256((size_t)n * 4);
    float *aD = (float *)w;
    w += align256((size_t)n * 4);
    float *sums = (float *)w;
    w += align256((size_t)K * d * 4);
    float *counts = (float *)w;
    w += align256((size_t)K * 4);
    float *eD = (float *)w;
    const int64_t kd = (int64_t)K * d, nd = n * d;
    hipLaunchKernelGGL(gather_rows, dim3((unsigned)((kd + 255) / 256)), dim3(256), 0, st, points, d,
                       init_ids, K, centers);
    hipError_t e;
    for (int it = 0; it < iters; ++it) {
        e = launch_knn(points, n, centers, K, d, 1, 0, pa, assign, aD, kws, st, nullptr, nullptr, nullptr);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(zero_f, dim3((unsigned)((kd + 255) / 256)), dim3(256), 0, st, sums, kd);
        hipLaunchKernelGGL(zero_f, dim3((K + 255) / 256), dim3(256), 0, st, counts, (int64_t)K);
        hipLaunchKernelGGL(accumulate, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, points, n,
                           d, assign, sums, counts);
        hipLaunchKernelGGL(finalize, dim3((unsigned)((kd + 255) / 256)), dim3(256), 0, st, sums, counts,
                           K, d, centers);
    }
    e = launch_knn(centers, K, points, n, d, 1, 0, pb, entries, eD, kws, st, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace cng
