// Connectivity (Algorithm 3, phase 4): make every point reachable from the
// entry.  The paper adds edges from the traversal tree of s to every point it
// misses, as NSG does; the reading implemented here works in rounds on a
// snapshot of the graph so that the searches of one round run as one batch:
//   U = points not reachable from the entry (breadth-first search on the GPU);
//   A = the smallest id of every strongly connected component of the
//       subgraph U induces that no edge from another component of U enters
//       (its source components: every point of U is reachable from one), in
//       id order; found on the host (Tarjan's algorithm on U's rows);
//   every p in A is searched from the entry with beam Lc (the batched beam
//   search kernel, query = point p) and gets the first result, by (D, id),
//   whose row has a free slot in the snapshot; if none has one, the reachable
//   point with a free slot nearest to p;
//   attachments are applied in increasing p by one thread: t_p's row gets p in
//   its first free slot, unless an earlier p of the round filled it (then p
//   waits for the next round).
// Rows have spare slots beyond the pruning cap for exactly these edges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

constexpr int SEG = 1024;       // points per block in the ordered compaction
constexpr int64_t BATCH = 65536; // searches per launch

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Counters {
    uint32_t next;      // BFS next-frontier size
    uint32_t nA;        // |U| (then |A|)
    uint32_t nfb;       // points that need the nearest-free fallback
    uint32_t attached;  // points attached this round
    uint32_t cap_err;   // 1 if some point found no row with room
    uint32_t pad[3];
    unsigned long long fb_key;  // (D, id) of the nearest free point
};

__global__ void fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void start_bfs(uint32_t *reached, uint32_t *frontier, uint32_t entry, Counters *c)
{
    reached[entry] = 1;
    frontier[0] = entry;
    c->next = 0;
}

__device__ __forceinline__ int row_len(const uint32_t *row, int W, int64_t n)
{
    int g = 0;
    while (g < W && row[g] != NONE && (int64_t)row[g] < n) ++g;
    return g;
}

__global__ void bfs_expand(const uint32_t *__restrict__ adj, int W, int64_t n,
                           const uint32_t *__restrict__ frontier, uint32_t fsize,
                           uint32_t *__restrict__ reached, uint32_t *__restrict__ next, Counters *c)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= fsize) return;
    const uint32_t *row = adj + (size_t)frontier[i] * W;
    for (int g = 0; g < W; ++g) {
        uint32_t v = row[g];
        if (v == NONE || (int64_t)v >= n) break;
        if (reached[v] == 0 && atomicExch(&reached[v], 1u) == 0u) next[atomicAdd(&c->next, 1u)] = v;
    }
}

__global__ void reset_next(Counters *c) { c->next = 0; }

__global__ void round_init(Counters *c)
{
    {
        c->nA = 0;
        c->nfb = 0;
        c->attached = 0;
        c->cap_err = 0;
        c->fb_key = ~0ull;
    }
}

// Points of U (listed in id order by count_A / scan_segments / scatter_A).
__device__ __forceinline__ bool in_A(const uint32_t *reached, int64_t p) { return !reached[p]; }

__global__ __launch_bounds__(256) void count_A(const uint32_t *__restrict__ reached, int64_t n,
                                               uint32_t *__restrict__ segcnt)
{
    __shared__ uint32_t s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SEG;
    uint32_t k = 0;
    for (int j = threadIdx.x; j < SEG; j += 256) {
        int64_t p = base + j;
        if (p < n && in_A(reached, p)) ++k;
    }
    atomicAdd(&s, k);
    __syncthreads();
    if (threadIdx.x == 0) segcnt[blockIdx.x] = s;
}

// Exclusive scan of the segment counts by one block; total into c->nA.
__global__ __launch_bounds__(1024) void scan_segments(uint32_t *segcnt, int64_t nseg, Counters *c)
{
    __shared__ uint32_t buf[1024];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nseg; b0 += 1024) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < nseg ? segcnt[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            uint32_t t = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nseg) segcnt[i] = carry + buf[threadIdx.x] - v;
        uint32_t tot = buf[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) c->nA = carry;
}

// Ordered write of A: each block scans its segment (256 threads x 4 points).
__global__ __launch_bounds__(256) void scatter_A(const uint32_t *__restrict__ reached, int64_t n,
                                                 const uint32_t *__restrict__ segoff,
                                                 uint32_t *__restrict__ A)
{
    __shared__ uint32_t buf[256];
    int64_t base = (int64_t)blockIdx.x * SEG + (int64_t)threadIdx.x * 4;
    uint32_t f[4], k = 0;
    for (int j = 0; j < 4; ++j) {
        int64_t p = base + j;
        f[j] = (p < n && in_A(reached, p)) ? 1u : 0u;
        k += f[j];
    }
    buf[threadIdx.x] = k;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t t = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t o = segoff[blockIdx.x] + buf[threadIdx.x] - k;
    for (int j = 0; j < 4; ++j)
        if (f[j]) A[o++] = (uint32_t)(base + j);
}

__global__ void degrees(const uint32_t *__restrict__ adj, int W, int64_t n, uint32_t *__restrict__ deg)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) deg[t] = (uint32_t)row_len(adj + (size_t)t * W, W, n);
}

// Rows of the points U[u0 .. u0 + cnt) into out [cnt x W].
__global__ void gather_u_rows(const uint32_t *__restrict__ U, int64_t u0, int64_t cnt,
                              const uint32_t *__restrict__ adj, int W, uint32_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * W) return;
    const int64_t i = t / W;
    out[t] = adj[(size_t)U[u0 + i] * W + (t % W)];
}

// First beam entry whose row has room (snapshot degrees); else queue a fallback.
__global__ void pick_targets(const uint32_t *__restrict__ beam, int Lc, int64_t cnt,
                             const uint32_t *__restrict__ deg, int W, int64_t off,
                             uint32_t *__restrict__ T, uint32_t *__restrict__ fb, Counters *c)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    uint32_t t = NONE;
    for (int j = 0; j < Lc; ++j) {
        uint32_t v = beam[(size_t)i * Lc + j];
        if (v == NONE) break;
        if (deg[v] < (uint32_t)W) {
            t = v;
            break;
        }
    }
    T[off + i] = t;
    if (t == NONE) fb[atomicAdd(&c->nfb, 1u)] = (uint32_t)(off + i);
}

// Nearest reachable point with room to point p: (D, id) minimum over the grid.
template <int G, int RND, bool VEC>
__global__ __launch_bounds__(256) void nearest_free(const float *__restrict__ pts, int64_t n, int d,
                                                   uint32_t p, const uint32_t *__restrict__ reached,
                                                   const uint32_t *__restrict__ deg, int W,
                                                   Counters *c)
{
    constexpr int NG = 64 / G;
    const int lane = lane_id(), grp = lane / G, gl = lane % G;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const float *xp = pts + (size_t)p * (uint32_t)d;
    float4 xr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) xr[r] = load_chunk<VEC>(xp, d, r, gl);
    for (int64_t w0 = wave * NG; w0 < n; w0 += nwaves * NG) {
        const int64_t w = w0 + grp;
        const bool cand = w < n && reached[w] && deg[w] < (uint32_t)W;
        float acc = 0.f;
        if (cand) {
            const float *y = pts + (size_t)w * (uint32_t)d;
#pragma unroll
            for (int r = 0; r < RND; ++r) acc = chunk_fma(xr[r], load_chunk<VEC>(y, d, r, gl), acc);
        }
        acc = group_sum<G>(acc);
        if (cand && gl == 0) atomicMin(&c->fb_key, (unsigned long long)make_key(acc, (uint32_t)w));
    }
}

__global__ void take_fallback(uint32_t *T, uint32_t a, Counters *c)
{
    T[a] = c->fb_key == ~0ull ? NONE : (uint32_t)(c->fb_key & 0xFFFFFFFFull);
    c->fb_key = ~0ull;
}

// Apply the round's attachments in increasing p (A is in id order).
__global__ void apply_attach(const uint32_t *__restrict__ A, const uint32_t *__restrict__ T,
                             uint32_t nA, uint32_t *adj, int W, uint32_t *deg, uint32_t *reached,
                             uint32_t *frontier, Counters *c)
{
    uint32_t k = 0;
    for (uint32_t a = 0; a < nA; ++a) {
        uint32_t p = A[a], t = T[a];
        if (t == NONE) {
            c->cap_err = 1;
            break;
        }
        if (deg[t] >= (uint32_t)W) continue;
        adj[(size_t)t * W + deg[t]] = p;
        deg[t] += 1;
        reached[p] = 1;
        frontier[k++] = p;
    }
    c->attached = k;
}

using NearestFn = void (*)(const float *, int64_t, int, uint32_t, const uint32_t *,
                           const uint32_t *, int, Counters *);

template <bool VEC>
NearestFn pick_nf(int d)
{
    if (d <= 32) return nearest_free<8, 1, VEC>;
    if (d <= 64) return nearest_free<16, 1, VEC>;
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return nearest_free<32, 1, VEC>;
    if (rnd <= 2) return nearest_free<32, 2, VEC>;
    if (rnd <= 4) return nearest_free<32, 4, VEC>;
    if (rnd <= 8) return nearest_free<32, 8, VEC>;
    if (rnd <= 16) return nearest_free<32, 16, VEC>;
    return nearest_free<32, 32, VEC>;
}

struct Ws {
    uint32_t *reached, *f0, *f1, *deg, *A, *T, *fb, *segcnt, *beam, *entry;
    float *beamD;
    Counters *c;
};

Ws carve(void *ws, int64_t n, int W, int Lc)
{
    unsigned char *w = (unsigned char *)ws;
    Ws s;
    auto take = [&](size_t b) {
        void *p = w;
        w += align256(b);
        return p;
    };
    s.reached = (uint32_t *)take((size_t)n * 4);
    s.f0 = (uint32_t *)take((size_t)n * 4);
    s.f1 = (uint32_t *)take((size_t)n * 4);
    s.deg = (uint32_t *)take((size_t)n * 4);
    s.A = (uint32_t *)take((size_t)n * 4);
    s.T = (uint32_t *)take((size_t)n * 4);
    s.fb = (uint32_t *)take((size_t)n * 4);
    s.segcnt = (uint32_t *)take((size_t)((n + SEG - 1) / SEG + 1) * 4);
    int64_t b = n < BATCH ? n : BATCH;
    // the beams of a search batch, and the rows of a chunk of U
    s.beam = (uint32_t *)take((size_t)b * (Lc > W ? Lc : W) * 4);
    s.beamD = (float *)take((size_t)b * Lc * 4);
    s.entry = (uint32_t *)take(4);
    s.c = (Counters *)take(sizeof(Counters));
    return s;
}

hipError_t read_counters(Counters *h, Counters *d, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(h, d, sizeof(Counters), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// Breadth-first expansion from `frontier` (size fsize); returns points added.
hipError_t bfs(const uint32_t *adj, int W, int64_t n, Ws &s, uint32_t *frontier, uint32_t fsize,
               hipStream_t st, int64_t *added)
{
    uint32_t *cur = frontier, *nxt = cur == s.f0 ? s.f1 : s.f0;
    int64_t total = 0;
    Counters h;
    while (fsize > 0) {
        hipLaunchKernelGGL(reset_next, dim3(1), dim3(1), 0, st, s.c);
        hipLaunchKernelGGL(bfs_expand, dim3((fsize + 255) / 256), dim3(256), 0, st, adj, W, n, cur,
                           fsize, s.reached, nxt, s.c);
        hipError_t e = read_counters(&h, s.c, st);
        if (e != hipSuccess) return e;
        fsize = h.next;
        total += fsize;
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    *added = total;
    return hipSuccess;
}

// A of a round, on the host: U (ascending) with its rows (rows[i * W ..] is
// the row of U[i]).  Tarjan's strongly connected components (1972), with an
// explicit stack of (point, next edge); a component is a source when no edge
// from another component of U enters it; A = the smallest id of each source
// component, ascending.
std::vector<uint32_t> source_component_mins(const std::vector<uint32_t> &U,
                                            const std::vector<uint32_t> &rows, int W, int64_t n)
{
    const size_t m = U.size();
    // the subgraph on U as compressed rows of local indices
    std::vector<size_t> first(m + 1, 0);
    std::vector<uint32_t> to;
    to.reserve(m * 2);
    for (size_t i = 0; i < m; ++i) {
        for (int g = 0; g < W; ++g) {
            const uint32_t v = rows[i * (size_t)W + g];
            if (v == NONE || (int64_t)v >= n) break;
            const auto it = std::lower_bound(U.begin(), U.end(), v);
            if (it != U.end() && *it == v) to.push_back((uint32_t)(it - U.begin()));
        }
        first[i + 1] = to.size();
    }
    std::vector<int64_t> order(m, -1), low(m, 0);
    std::vector<int64_t> comp(m, -1);
    std::vector<char> open(m, 0);
    std::vector<uint32_t> pending;                       // points of unfinished components
    std::vector<std::pair<uint32_t, size_t>> path;       // (point, next edge)
    int64_t clock = 0, ncomp = 0;
    for (size_t r = 0; r < m; ++r) {
        if (order[r] >= 0) continue;
        order[r] = low[r] = clock++;
        pending.push_back((uint32_t)r);
        open[r] = 1;
        path.emplace_back((uint32_t)r, first[r]);
        while (!path.empty()) {
            const uint32_t u = path.back().first;
            const size_t e = path.back().second;
            if (e < first[u + 1]) {
                path.back().second = e + 1;
                const uint32_t v = to[e];
                if (order[v] < 0) {
                    order[v] = low[v] = clock++;
                    pending.push_back(v);
                    open[v] = 1;
                    path.emplace_back(v, first[v]);
                } else if (open[v]) {
                    low[u] = std::min(low[u], order[v]);
                }
                continue;
            }
            if (low[u] == order[u]) {  // u roots a component
                uint32_t w;
                do {
                    w = pending.back();
                    pending.pop_back();
                    open[w] = 0;
                    comp[w] = ncomp;
                } while (w != u);
                ++ncomp;
            }
            path.pop_back();
            if (!path.empty()) low[path.back().first] = std::min(low[path.back().first], low[u]);
        }
    }
    std::vector<char> entered((size_t)ncomp, 0), taken((size_t)ncomp, 0);
    for (size_t u = 0; u < m; ++u)
        for (size_t e = first[u]; e < first[u + 1]; ++e)
            if (comp[to[e]] != comp[u]) entered[(size_t)comp[to[e]]] = 1;
    std::vector<uint32_t> A;
    for (size_t i = 0; i < m; ++i) {
        const size_t c = (size_t)comp[i];
        if (entered[c] || taken[c]) continue;
        taken[c] = 1;
        A.push_back(U[i]);
    }
    return A;
}

}  // namespace

size_t connect_workspace_bytes(int64_t n, int W, int Lc)
{
    int64_t b = n < BATCH ? n : BATCH;
    return align256((size_t)n * 4) * 7 + align256((size_t)((n + SEG - 1) / SEG + 1) * 4) +
           align256((size_t)b * (Lc > W ? Lc : W) * 4) + align256((size_t)b * Lc * 4) + align256(4) +
           align256(sizeof(Counters));
}

hipError_t run_connect(const float *points, int64_t n, int d, uint32_t *adj, int W,
                       uint32_t entry_host, int Lc, int vlog2, void *ws, hipStream_t st,
                       int64_t *rounds, int64_t *added, int *capacity_error)
{
    Ws s = carve(ws, n, W, Lc);
    *rounds = 0;
    *added = 0;
    *capacity_error = 0;
    const unsigned gb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_u32, dim3(gb), dim3(256), 0, st, s.reached, n, 0u);
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(1), 0, st, s.entry, (int64_t)1, entry_host);
    hipLaunchKernelGGL(start_bfs, dim3(1), dim3(1), 0, st, s.reached, s.f0, entry_host, s.c);
    int64_t reached = 1, got = 0;
    hipError_t e = bfs(adj, W, n, s, s.f0, 1, st, &got);
    if (e != hipSuccess) return e;
    reached += got;
    const bool vec = (d % 4 == 0) && ((uintptr_t)points % 16 == 0);
    NearestFn nf = vec ? pick_nf<true>(d) : pick_nf<false>(d);
    Counters h;
    const int64_t nseg = (n + SEG - 1) / SEG;
    // row lengths; apply_attach keeps them current (it is the only writer of
    // adj from here on)
    hipLaunchKernelGGL(degrees, dim3(gb), dim3(256), 0, st, adj, W, n, s.deg);
    while (reached < n) {
        ++*rounds;
        hipLaunchKernelGGL(round_init, dim3(1), dim3(1), 0, st, s.c);
        // U in id order into s.A, |U| into c->nA
        hipLaunchKernelGGL(count_A, dim3((unsigned)nseg), dim3(256), 0, st, s.reached, n, s.segcnt);
        hipLaunchKernelGGL(scan_segments, dim3(1), dim3(1024), 0, st, s.segcnt, nseg, s.c);
        hipLaunchKernelGGL(scatter_A, dim3((unsigned)nseg), dim3(256), 0, st, s.reached, n, s.segcnt, s.A);
        e = read_counters(&h, s.c, st);
        if (e != hipSuccess) return e;
        if (h.nA == 0) break;  // the device sees every point reached
        if (*rounds > n) return hipErrorUnknown;  // each round attaches a point: cannot happen
        // U and its rows to the host (rows in chunks through the beam buffer)
        std::vector<uint32_t> Uh(h.nA), rows((size_t)h.nA * W);
        e = hipMemcpyAsync(Uh.data(), s.A, (size_t)h.nA * 4, hipMemcpyDeviceToHost, st);
        for (int64_t u0 = 0; e == hipSuccess && u0 < (int64_t)h.nA; u0 += BATCH) {
            const int64_t cnt = (int64_t)h.nA - u0 < BATCH ? (int64_t)h.nA - u0 : BATCH;
            hipLaunchKernelGGL(gather_u_rows, dim3((unsigned)((cnt * W + 255) / 256)), dim3(256), 0, st, s.A,
                               u0, cnt, adj, W, s.beam);
            e = hipMemcpyAsync(rows.data() + (size_t)u0 * W, s.beam, (size_t)cnt * W * 4,
                               hipMemcpyDeviceToHost, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        const std::vector<uint32_t> Ah = source_component_mins(Uh, rows, W, n);
        e = hipMemcpyAsync(s.A, Ah.data(), Ah.size() * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        const uint32_t nA = (uint32_t)Ah.size();
        for (int64_t off = 0; off < nA; off += BATCH) {
            const int64_t cnt = nA - off < BATCH ? nA - off : BATCH;
            SearchArgs sa{};
            sa.points = points;
            sa.vecs = points;
            sa.scales = nullptr;
            sa.store = 0;
            sa.n = n;
            sa.d = d;
            sa.adj = adj;
            sa.W = W;
            sa.queries = nullptr;
            sa.query_ids = s.A + off;
            sa.nq = cnt;
            sa.k = Lc;
            sa.Leff = Lc;
            sa.entries = s.entry;
            sa.per_query_entry = 0;
            sa.ids = s.beam;
            sa.dists = s.beamD;
            sa.hops = nullptr;
            sa.ndc = nullptr;
            sa.vlog2 = vlog2 ? vlog2 : search_default_vlog2(Lc, cnt, 0);
            e = launch_search(sa, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(pick_targets, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                               s.beam, Lc, cnt, s.deg, W, off, s.T, s.fb, s.c);
        }
        e = read_counters(&h, s.c, st);
        if (e != hipSuccess) return e;
        if (h.nfb > 0) {
            // rare: read which points need the nearest-free fallback
            uint32_t *fbh = new uint32_t[h.nfb];
            uint32_t *Ah = new uint32_t[h.nfb];
            e = hipMemcpyAsync(fbh, s.fb, (size_t)h.nfb * 4, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            for (uint32_t i = 0; e == hipSuccess && i < h.nfb; ++i) {
                e = hipMemcpyAsync(&Ah[i], s.A + fbh[i], 4, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) break;
                hipLaunchKernelGGL(nf, dim3(1024), dim3(256), 0, st, points, n, d, Ah[i], s.reached,
                                   s.deg, W, s.c);
                hipLaunchKernelGGL(take_fallback, dim3(1), dim3(1), 0, st, s.T, fbh[i], s.c);
            }
            delete[] fbh;
            delete[] Ah;
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(apply_attach, dim3(1), dim3(1), 0, st, s.A, s.T, nA, adj, W, s.deg,
                           s.reached, s.f0, s.c);
        e = read_counters(&h, s.c, st);
        if (e != hipSuccess) return e;
        if (h.cap_err) {
            *capacity_error = 1;
            return hipSuccess;
        }
        *added += h.attached;
        reached += h.attached;
        e = bfs(adj, W, n, s, s.f0, h.attached, st, &got);
        if (e != hipSuccess) return e;
        reached += got;
    }
    return hipGetLastError();
}

}  // namespace cng
