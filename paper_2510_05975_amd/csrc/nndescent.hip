// Sub-quadratic candidate lists (Algorithm 3, phases 1-2, Section 4.1):
//
// Phase 1: an approximate K-NN graph G0 by NN-descent in synchronous rounds.
// A point's list starts as the K nearest by (D, id) of K SplitMix64 draws
// (output p K + j of the stream with the build's seed, mod n), itself
// excluded; every round replaces each list by the K nearest of itself and the
// lists of its members (neighbours of neighbours), all read from the lists as
// they were when the round began; rounds stop when one changes nothing.
//   One wavefront per point: its list is a sorted key array in LDS (the beam
//   structure of the search, merge_keys), the members' rows are read with one
//   coalesced load each, unseen candidates go through the search's visited
//   table and gather_dists.  A candidate v from member u is skipped when
//   neither u is new in p's list nor v new in u's list: then v was a
//   candidate of p in the round before, was not kept, and cannot be kept now
//   (p's K-th key only decreases), so the lists are those of the full union.
//
// Phase 2: every point's local-neighbour set is the C nearest (D, id), itself
// excluded, of the points that beam-search(G0, x_p, s, L, C + 1) evaluates
// together with p's own G0 row: the search's first C + 1 results (with
// squared distances) merged with the row.
#include <hip/hip_runtime.h>

#include <utility>

#include "beam.hpp"

namespace cng {

namespace {

using namespace beam;

// SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator:
// output i of the stream with seed s is mix(s + (i + 1) * golden gamma).
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct NndArgs {
    const float *points;
    int64_t n;
    int d;
    int K;
    uint64_t seed;
    const uint32_t *pid;   // previous lists [n x K] (NONE padded, ascending (D, id))
    const float *pD;       // their squared distances
    const uint8_t *pnew;   // previous "new" flags [n x K]
    uint32_t *nid;         // next lists
    float *nD;             // next squared distances
    uint8_t *nnew;         // next flags: entry not in the previous list of the point
    unsigned int *changed; // points whose list changed
    int vlog2;
};

constexpr int NND_VLOG2 = 11;

__host__ __device__ constexpr size_t nnd_lds_per_wave(int vlog2)
{
    // list (64 keys), merge scratch (64 keys), distances and ids of a batch
    // (64 + 64), the old ids (64), the visited table
    return 64 * 8 + 64 * 8 + 64 * 4 + 64 * 4 + 64 * 4 + ((size_t)4 << vlog2);
}

// One wavefront per point: the start (round 0, from the draws) or one round.
// The visited table never reports an id it has not seen; if it forgets one,
// the id's distance is computed again and merge_keys drops the equal key.
template <int G, int RND, bool VEC, int UB, bool START>
__global__ __launch_bounds__(256) void nnd_kernel(NndArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (p >= a.n) return;
    unsigned char *base = smem + (size_t)wave * nnd_lds_per_wave(a.vlog2);
    uint64_t *qa = reinterpret_cast<uint64_t *>(base);
    uint64_t *tmp = qa + 64;
    float *dsc = reinterpret_cast<float *>(tmp + 64);
    uint32_t *cid = reinterpret_cast<uint32_t *>(dsc + 64);
    uint32_t *old = cid + 64;
    uint32_t *vis = old + 64;
    const int d = a.d, K = a.K;
    const int gl = lane % G;
    const float *xp = a.points + (size_t)p * (uint32_t)d;
    float4 qr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) qr[r] = load_chunk<VEC>(xp, d, r, gl);
    for (int i = lane; i < (1 << a.vlog2); i += 64) vis[i] = NONE;
    wave_sync();
    if (lane == 0) visit(vis, a.vlog2, (uint32_t)p);
    wave_sync();

    // scores the ids v of the lanes with `cand` set (p excluded, each unseen
    // id once) and merges them into the list
    int qn = 0;
    auto offer = [&](uint32_t v, bool cand) {
        const bool fresh = cand && v != (uint32_t)p && visit(vis, a.vlog2, v);
        const uint64_t fm = ballot(fresh);
        const int m = __popcll(fm);
        if (m == 0) return;
        if (fresh) cid[__popcll(fm & ((1ull << lane) - 1ull))] = v;
        wave_sync();
        gather_dists<G, RND, VEC, UB, 0>(a.points, nullptr, d, cid, m, qr, dsc);
        wave_sync();
        const uint64_t kc = lane < m ? make_key(dsc[lane], cid[lane]) : KEY_INF;
        qn = merge_keys<1>(qa, qn, K, tmp, kc, lane < m);
    };

    if (START) {
        // the K draws (repeats and p dropped)
        const uint32_t v = lane < K ? (uint32_t)(splitmix_at(a.seed, (uint64_t)p * K + lane) %
                                                 (uint64_t)a.n)
                                    : NONE;
        offer(v, lane < K);
    } else {
        // the point's own list (keys from the stored distances), its ids seen
        const uint32_t u0 = lane < K ? a.pid[(size_t)p * K + lane] : NONE;
        const bool ok0 = u0 != NONE;
        qn = __popcll(ballot(ok0));
        old[lane] = u0;
        if (ok0) {
            qa[lane] = make_key(a.pD[(size_t)p * K + lane], u0);
            visit(vis, a.vlog2, u0);
        }
        const uint64_t newm = ballot(ok0 && a.pnew[(size_t)p * K + lane] != 0);
        wave_sync();
        // the members' lists, in list order
        const int m0 = qn;
        for (int j = 0; j < m0; ++j) {
            const uint32_t u = old[j];
            const bool unew = (newm >> j) & 1ull;
            const uint32_t v = lane < K ? a.pid[(size_t)u * K + lane] : NONE;
            const bool vnew = lane < K && a.pnew[(size_t)u * K + lane] != 0;
            offer(v, v != NONE && (unew || vnew));
        }
    }
    // the new list and its flags (entries that were not in the old list)
    bool isnew = false;
    uint32_t id = NONE;
    float Dv = __builtin_inff();
    if (lane < qn) {
        id = key_id(qa[lane]);
        Dv = key_dist(qa[lane]);
        isnew = true;
        if (!START)
            for (int j = 0; j < K; ++j) isnew = isnew && old[j] != id;
    }
    if (lane < K) {
        a.nid[(size_t)p * K + lane] = id;
        a.nD[(size_t)p * K + lane] = Dv;
        a.nnew[(size_t)p * K + lane] = isnew ? 1 : 0;
    }
    const uint64_t anynew = ballot(isnew);
    if (!START && lane == 0 && anynew != 0) atomicAdd(a.changed, 1u);
}

using NndFn = void (*)(NndArgs);

template <int G, int RND, bool VEC, bool START>
NndFn nnd_fn()
{
    constexpr int UB = G == 32 ? (RND >= 16 ? 1 : 16 / RND) : G / 2;
    return nnd_kernel<G, RND, VEC, UB, START>;
}

template <bool VEC, bool START>
NndFn pick_nnd(int d)
{
    if (d <= 32) return nnd_fn<8, 1, VEC, START>();
    if (d <= 64) return nnd_fn<16, 1, VEC, START>();
    const int rnd = (d + 127) / 128;
    if (rnd <= 1) return nnd_fn<32, 1, VEC, START>();
    if (rnd <= 2) return nnd_fn<32, 2, VEC, START>();
    if (rnd <= 4) return nnd_fn<32, 4, VEC, START>();
    if (rnd <= 8) return nnd_fn<32, 8, VEC, START>();
    if (rnd <= 16) return nnd_fn<32, 16, VEC, START>();
    return nnd_fn<32, 32, VEC, START>();
}

// Phase 2 merge: row p of the search result (k = C + 1 entries, squared
// distances) and p's G0 row, p and repeats dropped, the first C by (D, id).
// One wavefront per point; C + 1 + K <= 256 keys in LDS, bitonic sort.
__global__ __launch_bounds__(256) void pool_kernel(int64_t p0, int64_t np, int C, const uint32_t *sid,
                                                   const float *sD, const uint32_t *g0,
                                                   const float *g0D, int K, uint32_t *cand,
                                                   float *candD)
{
    __shared__ uint64_t keys[4][256];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * 4 + wave;
    if (i >= np) return;
    const int64_t p = p0 + i;
    uint64_t *k = keys[wave];
    const int ns = C + 1;
    for (int e = lane; e < 256; e += 64) {
        uint64_t key = ~0ull;
        if (e < ns) {
            const uint32_t v = sid[(size_t)i * ns + e];
            if (v != NONE && v != (uint32_t)p) key = make_key(sD[(size_t)i * ns + e], v);
        } else if (e < ns + K) {
            const uint32_t v = g0[(size_t)p * K + (e - ns)];
            if (v != NONE && v != (uint32_t)p) key = make_key(g0D[(size_t)p * K + (e - ns)], v);
        }
        k[e] = key;
    }
    wave_sort(k, 256);
    // drop repeats (equal keys are adjacent), keep the first C
    int w = 0;
    for (int e0 = 0; e0 < 256 && w < C; e0 += 64) {
        const int e = e0 + lane;
        const uint64_t key = k[e];
        const bool keep = key != ~0ull && (e == 0 || k[e - 1] != key);
        const uint64_t bm = ballot(keep);
        const int pos = w + __popcll(bm & ((1ull << lane) - 1ull));
        if (keep && pos < C) {
            cand[(size_t)p * C + pos] = key_id(key);
            candD[(size_t)p * C + pos] = key_dist(key);
        }
        w += __popcll(bm);
    }
    for (int e = (w < C ? w : C) + lane; e < C; e += 64) {
        cand[(size_t)p * C + e] = NONE;
        candD[(size_t)p * C + e] = __builtin_inff();
    }
}

}  // namespace

size_t nndescent_workspace_bytes(int64_t n, int K)
{
    const size_t a = ((size_t)n * K * 4 + 255) & ~(size_t)255;
    const size_t f = ((size_t)n * K + 255) & ~(size_t)255;
    return 3 * a + 2 * f + 256;
}

hipError_t run_nndescent(const float *points, int64_t n, int d, int K, uint64_t seed, int rounds,
                         uint32_t *ids, float *D, void *ws, hipStream_t st, int *rounds_run)
{
    const size_t a = ((size_t)n * K * 4 + 255) & ~(size_t)255;
    const size_t f = ((size_t)n * K + 255) & ~(size_t)255;
    unsigned char *w = (unsigned char *)ws;
    uint32_t *ids2 = (uint32_t *)w;
    float *D2 = (float *)(w + a);
    uint8_t *fl1 = (uint8_t *)(w + 2 * a);
    uint8_t *fl2 = (uint8_t *)(w + 2 * a + f);
    unsigned int *changed = (unsigned int *)(w + 2 * a + 2 * f);
    const bool vec = (d % 4 == 0) && ((uintptr_t)points % 16 == 0);
    const int wpb = 4;
    const unsigned blocks = (unsigned)((n + wpb - 1) / wpb);
    const unsigned lds = (unsigned)(wpb * nnd_lds_per_wave(NND_VLOG2));
    NndArgs na{points, n, d, K, seed, nullptr, nullptr, nullptr, ids, D, fl1, changed, NND_VLOG2};
    NndFn f0 = vec ? pick_nnd<true, true>(d) : pick_nnd<false, true>(d);
    hipLaunchKernelGGL(f0, dim3(blocks), dim3(64 * wpb), lds, st, na);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    NndFn fr = vec ? pick_nnd<true, false>(d) : pick_nnd<false, false>(d);
    // the current lists alternate between (ids, D, fl1) and (ids2, D2, fl2)
    uint32_t *cur_id = ids, *nxt_id = ids2;
    float *cur_D = D, *nxt_D = D2;
    uint8_t *cur_f = fl1, *nxt_f = fl2;
    int r = 0;
    while (r < rounds) {
        unsigned int h = 0;
        e = hipMemsetAsync(changed, 0, 4, st);
        if (e != hipSuccess) return e;
        NndArgs ra{points, n, d, K, seed, cur_id, cur_D, cur_f, nxt_id, nxt_D, nxt_f, changed, NND_VLOG2};
        hipLaunchKernelGGL(fr, dim3(blocks), dim3(64 * wpb), lds, st, ra);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&h, changed, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        ++r;
        std::swap(cur_id, nxt_id);
        std::swap(cur_D, nxt_D);
        std::swap(cur_f, nxt_f);
        if (h == 0) break;
    }
    if (cur_id != ids) {
        e = hipMemcpyAsync(ids, cur_id, (size_t)n * K * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(D, cur_D, (size_t)n * K * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    if (rounds_run) *rounds_run = r;
    return hipSuccess;
}

size_t graph_candidates_workspace_bytes(int64_t n, int C)
{
    const int64_t chunk = n < (1 << 20) ? n : (1 << 20);
    return ((size_t)chunk * (C + 1) * 4 + 255) / 256 * 256 * 2 + 256;
}

hipError_t run_graph_candidates(const float *points, int64_t n, int d, const uint32_t *g0,
                                const float *g0D, int K, uint32_t s_host, int L, int C,
                                uint32_t *cand, float *candD, void *ws, hipStream_t st)
{
    const int64_t chunk = n < (1 << 20) ? n : (1 << 20);
    const size_t ob = ((size_t)chunk * (C + 1) * 4 + 255) / 256 * 256;
    unsigned char *w = (unsigned char *)ws;
    uint32_t *sid = (uint32_t *)w;
    float *sD = (float *)(w + ob);
    uint32_t *entry = (uint32_t *)(w + 2 * ob);
    hipError_t e = hipMemcpyAsync(entry, &s_host, 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const int Leff = L > C + 1 ? L : C + 1;
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t np = n - p0 < chunk ? n - p0 : chunk;
        SearchArgs a{};
        a.points = points;
        a.vecs = points;
        a.store = 0;
        a.n = n;
        a.d = d;
        a.adj = g0;
        a.W = K;
        a.queries = points + (size_t)p0 * d;
        a.nq = np;
        a.k = C + 1;
        a.Leff = Leff;
        a.entries = entry;
        a.per_query_entry = 0;
        a.ids = sid;
        a.dists = sD;
        a.vlog2 = search_default_vlog2(Leff, np, 0);
        a.out_sq = 1;
        e = launch_search(a, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pool_kernel, dim3((unsigned)((np + 3) / 4)), dim3(256), 0, st, p0, np, C,
                           sid, sD, g0, g0D, K, cand, candD);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(st);
}

}  // namespace cng
