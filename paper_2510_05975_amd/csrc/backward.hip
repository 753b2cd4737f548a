// Algorithm 3, phase 3: backward edges with lazy pruning (Section 4.3).
//
// Every edge (u, v) of the pruned graph adds the reverse edge (v, u).  The
// candidate set of a point p is its out-neighbours together with the sources
// of the edges into it (a set), ordered by (D, id) and cut to its Cb nearest;
// if it holds more than R points it is pruned once (Algorithm 2 with cap R, or
// Algorithm 4 with adaptive alpha), otherwise it becomes p's row as it is.
// Every decision reads the graph as it was before the phase.
//
// Device steps: in-degrees (atomics), an exclusive scan into offsets, the
// sources scattered into per-point lists (their order within a list is free:
// the candidate sets are sorted by key), one wavefront per point to form its
// candidate set (distances in the fixed order, an LDS buffer cut back to the
// best Cb keys whenever it fills, a final bitonic sort), then the pruning
// kernel over the candidate lists, copying lists of at most R points.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

__global__ void clear_u32(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// in-degree of every point over the rows (a row ends at its first NONE or id >= n)
__global__ void count_in(const uint32_t *__restrict__ adj, int64_t n, int W, uint32_t *indeg)
{
    const int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (u >= n) return;
    const uint32_t *row = adj + (size_t)u * W;
    bool alive = true;
    for (int s0 = 0; s0 < W && alive; s0 += 64) {
        const int s = s0 + lane;
        const uint32_t v = s < W ? row[s] : NONE;
        const bool ok = s < W && v != NONE && (int64_t)v < n;
        const uint64_t bad = ballot(!ok && s < W);
        // valid entries are those before the first invalid one
        const int first_bad = bad ? __builtin_ctzll(bad) : 64;
        if (ok && lane < first_bad) atomicAdd(&indeg[v], 1u);
        if (bad) alive = false;
    }
}

// exclusive scan of n 32-bit counts into 64-bit offsets, in blocks of 1024
constexpr int SCAN_B = 1024;

__global__ __launch_bounds__(SCAN_B) void scan_local(const uint32_t *__restrict__ cnt, int64_t n,
                                                     int64_t *off, int64_t *block_tot)
{
    __shared__ int64_t s[SCAN_B];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + t;
    const int64_t v = i < n ? (int64_t)cnt[i] : 0;
    s[t] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_B; o <<= 1) {
        const int64_t add = t >= o ? s[t - o] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    if (i < n) off[i] = s[t] - v;
    if (t == SCAN_B - 1) block_tot[blockIdx.x] = s[t];
}

// one workgroup: exclusive scan of the block totals, sequentially in chunks
__global__ __launch_bounds__(SCAN_B) void scan_totals(int64_t *tot, int64_t nb, int64_t *grand)
{
    __shared__ int64_t s[SCAN_B];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_B) {
        const int64_t i = b0 + t;
        const int64_t v = i < nb ? tot[i] : 0;
        s[t] = v;
        __syncthreads();
        for (int o = 1; o < SCAN_B; o <<= 1) {
            const int64_t add = t >= o ? s[t - o] : 0;
            __syncthreads();
            s[t] += add;
            __syncthreads();
        }
        if (i < nb) tot[i] = carry + s[t] - v;
        __syncthreads();
        if (t == SCAN_B - 1) carry += s[t];
        __syncthreads();
    }
    if (t == 0) *grand = carry;
}

__global__ void scan_add(int64_t *off, int64_t n, const int64_t *block_off, const int64_t *grand)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) off[i] += block_off[i / SCAN_B];
    if (i == n) off[n] = *grand;
}

// sources of the edges into every point
__global__ void scatter_src(const uint32_t *__restrict__ adj, int64_t n, int W,
                            const int64_t *__restrict__ off, uint32_t *cursor, uint32_t *src)
{
    const int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (u >= n) return;
    const uint32_t *row = adj + (size_t)u * W;
    bool alive = true;
    for (int s0 = 0; s0 < W && alive; s0 += 64) {
        const int s = s0 + lane;
        const uint32_t v = s < W ? row[s] : NONE;
        const bool ok = s < W && v != NONE && (int64_t)v < n;
        const uint64_t bad = ballot(!ok && s < W);
        const int first_bad = bad ? __builtin_ctzll(bad) : 64;
        if (ok && lane < first_bad) {
            const uint32_t pos = atomicAdd(&cursor[v], 1u);
            src[off[v] + pos] = (uint32_t)u;
        }
        if (bad) alive = false;
    }
}

struct GatherArgs {
    const float *points;
    int64_t n;
    int d;
    const uint32_t *adj;
    int W;
    const int64_t *off;
    const uint32_t *src;
    int Cb, CBX;
    uint32_t *cand;  // [n x Cb], NONE padded
    float *candD;    // [n x Cb], +inf padded
};

// One wave per point: its candidate set, ascending by (D, id), cut to Cb.
template <int G, int RND, bool VEC>
__global__ __launch_bounds__(256) void gather_candidates(GatherArgs a)
{
    constexpr int NG = 64 / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    const int64_t p = (int64_t)blockIdx.x * 4 + wave;
    if (p >= a.n) return;
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem) + (size_t)wave * a.CBX;
    uint32_t *own = reinterpret_cast<uint32_t *>(reinterpret_cast<uint64_t *>(smem) + 4 * (size_t)a.CBX) +
                    (size_t)wave * a.W;
    const int d = a.d;

    // own row (its entries before the first NONE or id >= n)
    int nown = 0;
    {
        const uint32_t *row = a.adj + (size_t)p * a.W;
        bool alive = true;
        for (int s0 = 0; s0 < a.W && alive; s0 += 64) {
            const int s = s0 + lane;
            const uint32_t v = s < a.W ? row[s] : NONE;
            const bool ok = s < a.W && v != NONE && (int64_t)v < a.n;
            const uint64_t bad = ballot(!ok && s < a.W);
            const int first_bad = bad ? __builtin_ctzll(bad) : 64;
            if (ok && lane < first_bad) own[s] = v;
            nown += bad ? first_bad : (a.W - s0 < 64 ? a.W - s0 : 64);
            if (bad) alive = false;
        }
    }
    wave_sync();
    const int64_t s0 = a.off[p];
    const int64_t total = nown + (a.off[p + 1] - s0);

    const float *xp = a.points + (size_t)p * (uint32_t)d;
    float4 xr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) xr[r] = load_chunk<VEC>(xp, d, r, gl);

    int fill = 0;
    uint64_t thr = ~0ull;
    for (int64_t b = 0; b < total; b += NG) {
        const int64_t e = b + grp;
        uint32_t id = NONE;
        bool valid = e < total;
        if (valid) {
            if (e < nown) {
                id = own[e];
            } else {
                id = a.src[s0 + (e - nown)];
                // a source that is also an out-neighbour (u -> p and p -> u) counts once
                for (int t = 0; t < nown; ++t)
                    if (own[t] == id) valid = false;
            }
        }
        float4 yr[RND];
        if (valid) {
            const float *y = a.points + (size_t)id * (uint32_t)d;
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = load_chunk<VEC>(y, d, r, gl);
        } else {
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r) acc = chunk_fma(xr[r], yr[r], acc);
        acc = group_sum<G>(acc);
        const uint64_t key = make_key(acc, id);
        const bool take = valid && gl == 0 && key < thr;
        const uint64_t tm = ballot(take);
        if (take) buf[fill + __popcll(tm & ((1ull << lane) - 1ull))] = key;
        fill += __popcll(tm);
        if (fill + NG > a.CBX) {  // full: keep the best Cb (fill > CBX - NG >= Cb here)
            wave_sync();
            for (int t = fill + lane; t < a.CBX; t += 64) buf[t] = ~0ull;
            wave_sort(buf, a.CBX);
            fill = a.Cb;
            thr = buf[a.Cb - 1];
        }
    }
    int np = 1;
    while (np < fill) np <<= 1;
    wave_sync();
    for (int t = fill + lane; t < np; t += 64) buf[t] = ~0ull;
    wave_sync();
    wave_sort(buf, np);
    const int m = fill < a.Cb ? fill : a.Cb;
    for (int t = lane; t < a.Cb; t += 64) {
        a.cand[(size_t)p * a.Cb + t] = t < m ? key_id(buf[t]) : NONE;
        a.candD[(size_t)p * a.Cb + t] = t < m ? key_dist(buf[t]) : __builtin_inff();
    }
}

using GatherFn = void (*)(GatherArgs);

template <bool VEC>
GatherFn pick_gather(int d)
{
    if (d <= 32) return gather_candidates<8, 1, VEC>;
    if (d <= 64) return gather_candidates<16, 1, VEC>;
    const int rnd = (d + 127) / 128;
    if (rnd <= 1) return gather_candidates<32, 1, VEC>;
    if (rnd <= 2) return gather_candidates<32, 2, VEC>;
    if (rnd <= 4) return gather_candidates<32, 4, VEC>;
    if (rnd <= 8) return gather_candidates<32, 8, VEC>;
    if (rnd <= 16) return gather_candidates<32, 16, VEC>;
    return gather_candidates<32, 32, VEC>;
}

}  // namespace

size_t backward_workspace_bytes(int64_t n, int W)
{
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    return align256((size_t)n * 4) * 2 + align256((size_t)(n + 1) * 8) +
           align256((size_t)(nb + 1) * 8) + align256((size_t)n * W * 4) + 256;
}

hipError_t run_backward(const float *points, int64_t n, int d, uint32_t *adj, int W, int R, int Cb,
                        double alpha, double alpha_max, double alpha_step, double tau,
                        uint32_t *cand, float *candD, void *ws, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    unsigned char *w = (unsigned char *)ws;
    uint32_t *indeg = (uint32_t *)w;
    w += align256((size_t)n * 4);
    uint32_t *cursor = (uint32_t *)w;
    w += align256((size_t)n * 4);
    int64_t *off = (int64_t *)w;
    w += align256((size_t)(n + 1) * 8);
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    int64_t *btot = (int64_t *)w;  // nb block totals, then the grand total
    w += align256((size_t)(nb + 1) * 8);
    uint32_t *src = (uint32_t *)w;

    const unsigned g256 = (unsigned)((n + 255) / 256);
    const unsigned gw = (unsigned)((n + 3) / 4);  // one wave per point
    hipLaunchKernelGGL(clear_u32, dim3(g256), dim3(256), 0, stream, indeg, n);
    hipLaunchKernelGGL(clear_u32, dim3(g256), dim3(256), 0, stream, cursor, n);
    hipLaunchKernelGGL(count_in, dim3(gw), dim3(256), 0, stream, adj, n, W, indeg);
    hipLaunchKernelGGL(scan_local, dim3((unsigned)nb), dim3(SCAN_B), 0, stream, indeg, n, off, btot);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(SCAN_B), 0, stream, btot, nb, btot + nb);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, stream, off,
                       n, btot, btot + nb);
    hipLaunchKernelGGL(scatter_src, dim3(gw), dim3(256), 0, stream, adj, n, W, off, cursor, src);

    const int CBX = next_pow2(Cb + 64);
    GatherArgs ga{points, n, d, adj, W, off, src, Cb, CBX, cand, candD};
    const bool vec = (d % 4 == 0) && ((uintptr_t)points % 16 == 0);
    GatherFn fn = vec ? pick_gather<true>(d) : pick_gather<false>(d);
    const unsigned lds = (unsigned)(4 * (size_t)CBX * 8 + 4 * (size_t)W * 4);
    hipLaunchKernelGGL(fn, dim3(gw), dim3(256), lds, stream, ga);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // rows are rewritten only after every candidate set has been read from them
    return launch_prune(points, n, d, cand, candD, Cb, R, W, alpha, tau, adj, stream, R, alpha_max,
                        alpha_step);
}

}  // namespace cng
