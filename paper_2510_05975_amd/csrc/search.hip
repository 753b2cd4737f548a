// Batched beam search over a proximity graph: Algorithm 1 of the paper
// (beam-search(G, q, s, L, k), Section 2.2), one wavefront per query.
//
// Per wavefront, in LDS:
//   beam   L_eff keys (D, id), ascending; bit 63 of a key marks the point as
//          explored (the set E of Algorithm 1); merged in place (every lane
//          reads its old entries into registers before any entry is written);
//   vis    an open-addressing table of ids whose distance was computed.  It
//          never reports an id it has not seen, so skipping those ids leaves
//          the beam identical to Algorithm 1 at every step (a point that left
//          or never entered the beam cannot re-enter: the beam's L-th key only
//          decreases).  When a probe sequence is full an old id is overwritten;
//          that costs a repeated distance evaluation, never a different result.
// Per hop: the row of the first unexplored point is read with one coalesced
// load, unseen neighbours are compacted, their vectors are gathered with one
// dwordx4 per lane per 128 dimensions (G lanes per vector, 64/G vectors per
// instruction, all loads of a batch in flight together) and reduced with a
// lane butterfly in the fixed order, then merged into the beam by rank.
//
// Precision form: the gathered vectors may be stored in bf16 or fp8-E4M3 (one
// float32 scale per vector).  They are widened to the float32 values they
// stand for and scored in the same fixed order; when the beam has converged
// its L entries are re-scored from the float32 vectors and sorted, and the
// first k are returned (exact float32 distances).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

constexpr int PROBES = 8;

__device__ __forceinline__ bool visit(uint32_t *vis, int vlog2, uint32_t id)
{
    const uint32_t mask = (1u << vlog2) - 1u;
    const uint32_t h = (id * 0x9E3779B1u) >> (32 - vlog2);
    for (int t = 0; t < PROBES; ++t) {
        uint32_t slot = (h + (uint32_t)t) & mask;
        uint32_t cur = vis[slot];
        if (cur == id) return false;
        if (cur == NONE) {
            uint32_t old = atomicCAS(&vis[slot], NONE, id);
            if (old == NONE) return true;
            if (old == id) return false;
        }
    }
    // every probed slot holds another id: forget the one at h
    return atomicExch(&vis[h], id) != id;
}

// First index e < qn of the beam whose key is not explored, or -1.
template <int QS>
__device__ __forceinline__ int first_unexplored(const uint64_t *beam, int qn)
{
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < QS; ++j) {
        int e = j * 64 + lane;
        bool un = e < qn && !(beam[e] & EXPL);
        uint64_t m = ballot(un);
        if (m) return j * 64 + (__ffsll((unsigned long long)m) - 1);
        if ((j + 1) * 64 >= qn) break;
    }
    return -1;
}

// Number of entries of sorted arr[0..cnt) that are < key.
__device__ __forceinline__ int lower_bound_keys(const uint64_t *arr, int cnt, uint64_t key)
{
    int lo = 0, hi = cnt;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (key_mask(arr[mid]) < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Fixed-order squared distances of the stored vectors cid[0..m) to the
// query (chunks qr, this lane's share) into dsc[0..m).  Group grp of G lanes
// takes vectors b + t * NG + grp for t < UB; all loads of a batch are issued
// before any sum (a batch's trip count is uniform across the wavefront), then
// the UB sums are formed together by group_sums.
template <int G, int RND, bool VEC, int UB, int ST>
__device__ __forceinline__ void gather_dists(const void *__restrict__ vecs, const float *__restrict__ scales,
                                             int d, const uint32_t *cid, int m, const float4 (&qr)[RND],
                                             float *dsc, int part = 0, int parts = 1)
{
    constexpr int NG = 64 / G;
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    // batches part, part + parts, ... of the list (several waves may share it)
    for (int b = part * NG * UB; b < m; b += parts * NG * UB) {
        // Loads only: nothing in a guarded block uses a loaded value, so no
        // wait separates the loads of a batch.  A group past the end of the
        // list re-reads vector b and its sum is never written.
        float acc[UB];
        if (VEC) {
            typename RawChunk<ST>::type raw[UB][RND];
            float sc[UB];
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                if (b + t * NG < m) {  // uniform: some group still has a vector
                    const int c = b + t * NG + grp;
                    const uint32_t id = cid[c < m ? c : b];
                    sc[t] = ST == 2 ? scales[id] : 1.f;
#pragma unroll
                    for (int r = 0; r < RND; ++r) raw[t][r] = load_raw<ST>(vecs, id, d, r, gl);
                } else {
                    sc[t] = 0.f;
#pragma unroll
                    for (int r = 0; r < RND; ++r) raw[t][r] = typename RawChunk<ST>::type{};
                }
            }
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                acc[t] = 0.f;
#pragma unroll
                for (int r = 0; r < RND; ++r) acc[t] = chunk_fma(decode_chunk(raw[t][r], sc[t]), qr[r], acc[t]);
            }
        } else {
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                acc[t] = 0.f;
                if (b + t * NG < m) {
                    const int c = b + t * NG + grp;
                    const uint32_t id = cid[c < m ? c : b];
                    const float sc = ST == 2 ? scales[id] : 1.f;
#pragma unroll
                    for (int r = 0; r < RND; ++r)
                        acc[t] = chunk_fma(load_stored<ST, VEC>(vecs, id, d, r, gl, sc), qr[r], acc[t]);
                }
            }
        }
        group_sums<G, UB>(acc, gl);
        constexpr int SPAN = G / UB;  // lanes holding one vector's sum
        const int t = gl / SPAN;
        const int c = b + t * NG + grp;
        if (gl % SPAN == 0 && c < m) dsc[c] = acc[0];
    }
}

struct WaveLds {
    uint64_t *qa, *tmp;
    float *dsc;
    uint32_t *cid, *vis;
    int *ctl;  // cooperative searches: the list length handed to the helper waves
};

__host__ __device__ constexpr size_t wave_lds_bytes(int qcap, int vlog2)
{
    return (size_t)qcap * 8 + 64 * 8 + 64 * 4 + 64 * 4 + ((size_t)4 << vlog2);
}

// One query.  G lanes per vector, RND float4 rounds per lane, QS beam slots per lane.
// COOP > 1: the query's wave is the first of a workgroup of COOP waves; the
// others (coop_helper) compute a share of every distance batch.  Each batch
// costs the workgroup two barriers, matched one for one by the helpers.
template <int G, int RND, bool VEC, int QS, int UB, int ST, int COOP = 1>
__device__ void beam_query(const SearchArgs a, int64_t qi, WaveLds s)
{
    const int lane = lane_id();
    const int gl = lane % G;
    const int d = a.d;
    const int Leff = a.Leff;

    const float *qv = a.query_ids ? a.points + (size_t)a.query_ids[qi] * d : a.queries + (size_t)qi * d;
    float4 qr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) qr[r] = load_chunk<VEC>(qv, d, r, gl);

    for (int i = lane; i < (1 << a.vlog2); i += 64) s.vis[i] = NONE;
    wave_sync();

    const uint32_t s0 = a.entries[a.per_query_entry ? qi : 0];
    if ((int64_t)s0 >= a.n) {  // invalid entry: nothing is reachable
        for (int e = lane; e < a.k; e += 64) {
            a.ids[(size_t)qi * a.k + e] = NONE;
            a.dists[(size_t)qi * a.k + e] = __builtin_inff();
        }
        if (lane == 0) {
            if (a.hops) a.hops[qi] = 0;
            if (a.ndc) a.ndc[qi] = 0;
        }
        return;
    }
    {
        const float sc0 = ST == 2 ? a.scales[s0] : 1.f;
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r)
            acc = chunk_fma(load_stored<ST, VEC>(a.vecs, s0, d, r, gl, sc0), qr[r], acc);
        acc = group_sum<G>(acc);
        if (lane == 0) {
            s.qa[0] = make_key(acc, s0);
            visit(s.vis, a.vlog2, s0);
        }
    }
    wave_sync();
    int qn = 1;
    uint32_t hops = 0, ndc = 1;
    uint64_t *qa = s.qa;

    for (;;) {
        const int f = first_unexplored<QS>(qa, qn);
        if (f < 0) break;
        const uint32_t u = key_id(qa[f]);
        wave_sync();
        if (lane == 0) qa[f] |= EXPL;
        ++hops;
        const uint32_t *row = a.adj + (size_t)u * a.W;
        for (int c0 = 0; c0 < a.W; c0 += 64) {
            // ---- neighbours of u*: coalesced row load, cut at the first sentinel
            uint32_t v = c0 + lane < a.W ? row[c0 + lane] : NONE;
            bool ok = v != NONE && (int64_t)v < a.n;
            uint64_t bad = ballot(!ok);
            int cut = bad ? (__ffsll((unsigned long long)bad) - 1) : 64;
            ok = ok && lane < cut;
            // ---- visited filter + compaction
            bool fresh = ok && visit(s.vis, a.vlog2, v);
            uint64_t fm = ballot(fresh);
            int m = __popcll(fm);
            if (fresh) {
                int slot = __popcll(fm & ((1ull << lane) - 1ull));
                s.cid[slot] = v;
            }
            wave_sync();
            // ---- distances: G lanes per vector, NG vectors per instruction
            if constexpr (COOP > 1) {
                if (lane == 0) s.ctl[0] = m;
                __syncthreads();  // the list and its length are visible to the helpers
                gather_dists<G, RND, VEC, UB, ST>(a.vecs, a.scales, d, s.cid, m, qr, s.dsc, 0, COOP);
                __syncthreads();  // every share of the distances is in dsc
            } else {
                gather_dists<G, RND, VEC, UB, ST>(a.vecs, a.scales, d, s.cid, m, qr, s.dsc);
            }
            wave_sync();
            ndc += (uint32_t)m;
            // ---- merge the m new keys into the beam (Algorithm 1: union, keep the L closest)
            bool val = lane < m;
            uint64_t kc = val ? make_key(s.dsc[lane], s.cid[lane]) : KEY_INF;
            if (qn == Leff) val = val && kc < key_mask(qa[Leff - 1]);
            int lb = 0;
            if (val) {
                lb = lower_bound_keys(qa, qn, kc);
                // an id the visited table forgot may still be in the beam: same key, drop it
                if (lb < qn && key_mask(qa[lb]) == kc) val = false;
            }
            uint64_t sm = ballot(val);
            int ns = __popcll(sm);
            if (ns > 0) {
                int rank = 0;
                uint64_t it = sm;
                while (it) {
                    int j = __ffsll((unsigned long long)it) - 1;
                    it &= it - 1;
                    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kc, j);
                    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(kc >> 32), j);
                    uint64_t kj = ((uint64_t)hi << 32) | lo;
                    rank += kj < kc ? 1 : 0;
                }
                if (val) s.tmp[rank] = kc;
                uint64_t old[QS];
#pragma unroll
                for (int j = 0; j < QS; ++j) {
                    int e = j * 64 + lane;
                    old[j] = e < qn ? qa[e] : 0;
                }
                wave_sync();  // every old entry is in registers before any write
                const int nqn = qn + ns < Leff ? qn + ns : Leff;
#pragma unroll
                for (int j = 0; j < QS; ++j) {
                    int e = j * 64 + lane;
                    if (e < qn) {
                        int np = e + lower_bound_keys(s.tmp, ns, key_mask(old[j]));
                        if (np < Leff) qa[np] = old[j];
                    }
                }
                if (val && lb + rank < Leff) qa[lb + rank] = kc;
                wave_sync();
                qn = nqn;
            }
            if (cut < 64) break;
        }
    }

    if (ST != 0) {
        // ---- re-rank the converged beam with the float32 vectors
        for (int b0 = 0; b0 < qn; b0 += 64) {
            const int cnt = qn - b0 < 64 ? qn - b0 : 64;
            if (lane < cnt) s.cid[lane] = key_id(qa[b0 + lane]);
            wave_sync();
            gather_dists<G, RND, VEC, UB, 0>(a.points, nullptr, d, s.cid, cnt, qr, s.dsc);
            wave_sync();
            if (lane < cnt) qa[b0 + lane] = make_key(s.dsc[lane], key_id(qa[b0 + lane]));
            wave_sync();
        }
        int np = 1;
        while (np < qn) np <<= 1;
        for (int e = qn + lane; e < np; e += 64) qa[e] = ~0ull;
        wave_sort(qa, np);
    }

    // ---- outputs: the first k of the beam
    for (int e = lane; e < a.k; e += 64) {
        uint32_t id = NONE;
        float dist = __builtin_inff();
        if (e < qn) {
            uint64_t ke = qa[e];
            id = key_id(ke);
            dist = __builtin_sqrtf(key_dist(ke));
        }
        a.ids[(size_t)qi * a.k + e] = id;
        a.dists[(size_t)qi * a.k + e] = dist;
    }
    if (lane == 0) {
        if (a.hops) a.hops[qi] = hops;
        if (a.ndc) a.ndc[qi] = ndc;
    }
}

template <int G, int RND, bool VEC, int QS, int UB, int ST>
__global__ __launch_bounds__(256) void search_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * wpb + wave;
    if (qi >= a.nq) return;  // waves never synchronise with each other
    const int qcap = 64 * QS;
    unsigned char *base = smem + (size_t)wave * wave_lds_bytes(qcap, a.vlog2);
    WaveLds s;
    s.qa = reinterpret_cast<uint64_t *>(base);
    s.tmp = s.qa + qcap;
    s.dsc = reinterpret_cast<float *>(s.tmp + 64);
    s.cid = reinterpret_cast<uint32_t *>(s.dsc + 64);
    s.vis = s.cid + 64;
    beam_query<G, RND, VEC, QS, UB, ST>(a, qi, s);
}

// Waves per workgroup of the cooperative search (one query per workgroup).
constexpr int COOPW = 8;

// One query per workgroup of COOPW waves: wave 0 runs the search, the others
// compute their share of each distance batch.  For launches of few queries
// with long vectors, where a hop waits on several rounds of vector loads.
template <int G, int RND, bool VEC, int QS, int UB>
__global__ __launch_bounds__(64 * COOPW) void search_coop_kernel(SearchArgs a)
{
    constexpr int COOP = COOPW;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6;
    const int64_t qi = blockIdx.x;  // the grid has exactly nq workgroups
    const int qcap = 64 * QS;
    WaveLds s;
    s.qa = reinterpret_cast<uint64_t *>(smem);
    s.tmp = s.qa + qcap;
    s.dsc = reinterpret_cast<float *>(s.tmp + 64);
    s.cid = reinterpret_cast<uint32_t *>(s.dsc + 64);
    s.vis = s.cid + 64;
    s.ctl = reinterpret_cast<int *>(s.vis + ((size_t)1 << a.vlog2));
    if (wave == 0) {
        beam_query<G, RND, VEC, QS, UB, 0, COOP>(a, qi, s);
        if (lane_id() == 0) s.ctl[0] = -1;
        __syncthreads();  // releases the helpers
        return;
    }
    const int gl = lane_id() % G;
    const float *qv = a.query_ids ? a.points + (size_t)a.query_ids[qi] * a.d : a.queries + (size_t)qi * a.d;
    float4 qr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) qr[r] = load_chunk<VEC>(qv, a.d, r, gl);
    for (;;) {
        __syncthreads();  // a list from wave 0, or the end of the search
        const int m = s.ctl[0];
        if (m < 0) break;
        gather_dists<G, RND, VEC, UB, 0>(a.vecs, a.scales, a.d, s.cid, m, qr, s.dsc, wave, COOP);
        __syncthreads();
    }
}

using KernelFn = void (*)(SearchArgs);

template <int G, int RND, bool VEC, int ST, int UBX = 0>
KernelFn pick_qs(int qs)
{
    constexpr int UB = UBX ? UBX : G == 32 ? (RND >= 16 ? 1 : 16 / RND) : G / 2;
    switch (qs) {
    case 1: return search_kernel<G, RND, VEC, 1, UB, ST>;
    case 2: return search_kernel<G, RND, VEC, 2, UB, ST>;
    case 4: return search_kernel<G, RND, VEC, 4, UB, ST>;
    default: return search_kernel<G, RND, VEC, 8, UB, ST>;
    }
}

// deep: a launch of few queries leaves the GPU mostly idle, so float32
// searches with 257 <= d <= 1024 take twice the vectors per load batch (more
// registers, half the memory round trips per hop).
template <bool VEC, int ST>
KernelFn pick_kernel(int d, int qs, bool deep)
{
    if (d <= 32) return pick_qs<8, 1, VEC, ST>(qs);
    if (d <= 64) return pick_qs<16, 1, VEC, ST>(qs);
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return pick_qs<32, 1, VEC, ST>(qs);
    if (rnd <= 2) return pick_qs<32, 2, VEC, ST>(qs);
    if constexpr (ST == 0) {
        if (deep && rnd > 2 && rnd <= 4) return pick_qs<32, 4, VEC, ST, 8>(qs);
        if (deep && rnd > 4 && rnd <= 8) return pick_qs<32, 8, VEC, ST, 4>(qs);
    }
    if (rnd <= 4) return pick_qs<32, 4, VEC, ST>(qs);
    if (rnd <= 8) return pick_qs<32, 8, VEC, ST>(qs);
    if (rnd <= 16) return pick_qs<32, 16, VEC, ST>(qs);
    return pick_qs<32, 32, VEC, ST>(qs);
}

template <int G, int RND, bool VEC, int UB>
KernelFn pick_coop_qs(int qs)
{
    switch (qs) {
    case 1: return search_coop_kernel<G, RND, VEC, 1, UB>;
    case 2: return search_coop_kernel<G, RND, VEC, 2, UB>;
    case 4: return search_coop_kernel<G, RND, VEC, 4, UB>;
    default: return search_coop_kernel<G, RND, VEC, 8, UB>;
    }
}

// float32, 257 <= d <= 1024 (rnd 3 .. 8), with the deep load batches
template <bool VEC>
KernelFn pick_coop(int rnd, int qs)
{
    return rnd <= 4 ? pick_coop_qs<32, 4, VEC, 8>(qs) : pick_coop_qs<32, 8, VEC, 4>(qs);
}

template <bool VEC>
KernelFn pick_store(int d, int qs, int st, bool deep)
{
    return st == 1 ? pick_kernel<VEC, 1>(d, qs, deep) : st == 2 ? pick_kernel<VEC, 2>(d, qs, deep)
                                                                 : pick_kernel<VEC, 0>(d, qs, deep);
}


// ---------------------------------------------------------------- serving loop
// A persistent grid: every wavefront claims work items in order from a ring
// that the host fills (coherent pinned host memory), runs the beam search of
// one query with that item's k and L, writes the results to pinned host
// memory and marks the item done with a system-scope release store.  The host
// publishes items by advancing `tail` (release); a wave whose claimed item is
// not yet published sleeps and re-checks `tail` and `stop`, and leaves after
// `idle_limit` empty checks, so every wave ends even if the host goes away.
__device__ __forceinline__ uint64_t sys_load_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t sys_load_u32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int G, int RND, bool VEC, int QS, int UB, int ST>
__global__ __launch_bounds__(256) void serve_kernel(ServeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int qcap = 64 * QS;
    const size_t per_wave = wave_lds_bytes(qcap, a.base.vlog2) + (size_t)a.base.d * 4 + 16;
    unsigned char *base = smem + (size_t)wave * per_wave;
    WaveLds s;
    s.qa = reinterpret_cast<uint64_t *>(base);
    s.tmp = s.qa + qcap;
    s.dsc = reinterpret_cast<float *>(s.tmp + 64);
    s.cid = reinterpret_cast<uint32_t *>(s.dsc + 64);
    s.vis = s.cid + 64;
    float *qbuf = reinterpret_cast<float *>(s.vis + ((size_t)1 << a.base.vlog2));
    uint32_t *ebuf = reinterpret_cast<uint32_t *>(qbuf + a.base.d);
    (void)wpb;

    uint32_t idle = 0;
    for (;;) {
        uint64_t t = 0;
        if (lane == 0) t = atomicAdd(a.head, 1ull);
        t = ((uint64_t)__shfl((uint32_t)(t >> 32), 0, 64) << 32) | __shfl((uint32_t)t, 0, 64);
        for (;;) {  // wait until item t is published
            // Only the wave holding the oldest unpublished item reads host
            // memory; it copies tail / stop into device memory (mirror[0] /
            // mirror[1]) where the other waves wait without crossing the bus.
            int state = 0;  // 1: ready, 2: leave, 3: keep waiting as the poller
            if (lane == 0) {
                // relaxed checks (an acquire at agent scope would invalidate
                // this CU's vector L1 on every check, under the searches of the
                // other waves); the acquire fence follows once the item is there
                uint64_t seen = __hip_atomic_load(&a.mirror[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seen > t) {
                    state = 1;
                } else if (__hip_atomic_load(&a.mirror[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    state = 2;
                } else {
                    if (seen == t) {  // this wave is next in line: poll the host
                        const uint64_t tail = sys_load_u64(&a.ring->tail);
                        if (tail > seen) {
                            atomicMax(reinterpret_cast<unsigned long long *>(&a.mirror[0]),
                                      (unsigned long long)tail);
                            state = 1;
                        } else if (sys_load_u64(&a.ring->stop) != 0) {
                            __hip_atomic_store(&a.mirror[1], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            state = 2;
                        }
                    }
                    if (state == 0 && ++idle > a.idle_limit) state = 2;
                    if (state == 0 && seen == t) state = 3;
                }
            }
            state = __shfl(state, 0, 64);
            if (state == 1) {
                __atomic_thread_fence(__ATOMIC_ACQUIRE);  // pairs with the publisher's release
                break;
            }
            if (state == 2) return;
            // The poller re-reads the host soon; every other wave backs off
            // longer, so that idle waves do not crowd the mirror's cache line
            // while searches run.
            if (state == 3) __builtin_amdgcn_s_sleep(16);
            else __builtin_amdgcn_s_sleep(127);
        }
        idle = 0;
        const uint64_t slot = t % a.cap;
        const ServeItem *item = a.items + slot;
        // item fields and the query vector, read through to host memory
        uint32_t f[1] = {0};
        if (lane < 4) f[0] = sys_load_u32(reinterpret_cast<const uint32_t *>(item) + lane);
        const uint32_t k = (uint32_t)__shfl((int)f[0], 1, 64);
        const uint32_t L = (uint32_t)__shfl((int)f[0], 2, 64);
        const uint32_t entry = (uint32_t)__shfl((int)f[0], 3, 64);
        const float *qsrc = a.payload + slot * (uint64_t)a.base.d;
        for (int i = lane; i < a.base.d; i += 64)
            qbuf[i] = __uint_as_float(sys_load_u32(reinterpret_cast<const uint32_t *>(qsrc) + i));
        if (lane == 0) ebuf[0] = entry;
        wave_sync();
        SearchArgs q = a.base;
        q.queries = qbuf;
        q.query_ids = nullptr;
        q.nq = 1;
        q.k = (int)k;
        q.Leff = (int)(L > k ? L : k);
        q.entries = ebuf;
        q.per_query_entry = 0;
        q.ids = a.out_ids + slot * (uint64_t)a.max_k;
        q.dists = a.out_dists + slot * (uint64_t)a.max_k;
        q.hops = nullptr;
        q.ndc = nullptr;
        if (q.k >= 1 && q.k <= a.max_k && q.Leff <= qcap) beam_query<G, RND, VEC, QS, UB, ST>(q, 0, s);
        wave_sync();
        __threadfence_system();
        if (lane == 0) __hip_atomic_store(&a.done[slot], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

using ServeFn = void (*)(ServeArgs);

template <int G, int RND, int ST>
ServeFn serve_fn()
{
    constexpr int UB = G == 32 ? (RND >= 16 ? 1 : 16 / RND) : G / 2;
    return serve_kernel<G, RND, true, 4, UB, ST>;
}

template <int ST>
ServeFn pick_serve(int d)
{
    if (d <= 32) return serve_fn<8, 1, ST>();
    if (d <= 64) return serve_fn<16, 1, ST>();
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return serve_fn<32, 1, ST>();
    if (rnd <= 2) return serve_fn<32, 2, ST>();
    return serve_fn<32, 4, ST>();
}
}  // namespace

// Measured on 1M x 128 (beam 48..128): a 1024-slot table beats larger ones,
// whose LDS cost in occupancy outweighs the distance evaluations they save.
size_t search_lds_per_wave(int Leff, int vlog2)
{
    int qs = Leff <= 64 ? 1 : Leff <= 128 ? 2 : Leff <= 256 ? 4 : 8;
    return wave_lds_bytes(64 * qs, vlog2);
}

// Visited-table slots (log2) of a launch of nq queries over vectors stored as
// `store` (0 float32, 1 bf16, 2 fp8) when the caller leaves them open.  With
// more queries than the GPU holds at once, 1024 slots, or 2048 for float32 up
// to L = 128: a small LDS share keeps more waves resident, and longer or
// lighter (reduced-precision) searches need that most (measured, 1M x 128 and
// 10M x 128 with 10k queries: float32 2048 slots 1-2 % faster than 1024 at
// L = 64 .. 96, 1024 slots 3 % to 74 % faster than 2048 or 4096 at
// L = 144 .. 512; bf16 at L = 80 17 % slower with 2048 than with 1024; 512
// slots slower everywhere).  When every query's wave fits at once, the largest
// table up to 8192 slots that still lets them all be resident: fewer forgotten
// vectors to read again (1M x 960, 1000 queries, L = 352: 8192 slots 9 %
// faster than 4096).
int search_default_vlog2(int Leff, int64_t nq, int store)
{
    const size_t lds_cu = 160 * 1024;
    for (int vl = 13; vl > 10; --vl) {
        const size_t wg = 4 * search_lds_per_wave(Leff, vl);  // 4 waves per workgroup
        int64_t waves = wg > lds_cu ? 0 : 4 * (int64_t)(lds_cu / wg);
        if (waves > 32) waves = 32;
        if (256 * waves >= nq) return vl;
    }
    return store == 0 && Leff <= 128 ? 11 : 10;
}

hipError_t launch_search(const SearchArgs &a, hipStream_t stream)
{
    if (a.nq == 0) return hipSuccess;
    const int qs = a.Leff <= 64 ? 1 : a.Leff <= 128 ? 2 : a.Leff <= 256 ? 4 : 8;
    const size_t vbytes = a.store == 1 ? 8 : a.store == 2 ? 4 : 16;  // one stored chunk
    const bool vec = (a.d % 4 == 0) && ((uintptr_t)a.points % 16 == 0) &&
                     ((uintptr_t)a.vecs % vbytes == 0) &&
                     (a.query_ids || (uintptr_t)a.queries % 16 == 0);
    const bool deep = a.nq <= 1024;
    const int rnd = (a.d + 127) / 128;
    if (a.store == 0 && a.nq <= 256 && rnd > 2 && rnd <= 8) {
        // few float32 queries with long vectors: COOPW waves per query
        KernelFn cf = vec ? pick_coop<true>(rnd, qs) : pick_coop<false>(rnd, qs);
        SearchArgs b = a;
        while (b.vlog2 > 6 && wave_lds_bytes(64 * qs, b.vlog2) + 16 > 64 * 1024) --b.vlog2;
        hipLaunchKernelGGL(cf, dim3((unsigned)a.nq), dim3(64 * COOPW),
                           (unsigned)(wave_lds_bytes(64 * qs, b.vlog2) + 16), stream, b);
        return hipGetLastError();
    }
    KernelFn fn = vec ? pick_store<true>(a.d, qs, a.store, deep) : pick_store<false>(a.d, qs, a.store, deep);
    // the visited table may be shrunk to keep a wave within 64 KB of LDS
    // (it only changes how often a distance is recomputed, never the results)
    SearchArgs b = a;
    while (b.vlog2 > 6 && wave_lds_bytes(64 * qs, b.vlog2) > 64 * 1024) --b.vlog2;
    const size_t per_wave = wave_lds_bytes(64 * qs, b.vlog2);
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * per_wave > 64 * 1024) wpb >>= 1;
    const int64_t blocks = (a.nq + wpb - 1) / wpb;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * wpb), (unsigned)(wpb * per_wave),
                       stream, b);
    return hipGetLastError();
}

size_t serve_lds_per_wave(int d, int vlog2)
{
    return wave_lds_bytes(256, vlog2) + (size_t)d * 4 + 16;
}

// The persistent serving grid: `waves` wavefronts, 4 per workgroup.  Needs
// d % 4 == 0, d <= 512, beams up to 256 entries (one template per storage).
hipError_t launch_serve(const ServeArgs &a, int waves, hipStream_t stream)
{
    ServeFn fn = a.base.store == 1 ? pick_serve<1>(a.base.d)
               : a.base.store == 2 ? pick_serve<2>(a.base.d) : pick_serve<0>(a.base.d);
    const size_t per_wave = serve_lds_per_wave(a.base.d, a.base.vlog2);
    const int wpb = 4;
    const unsigned blocks = (unsigned)((waves + wpb - 1) / wpb);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * wpb), (unsigned)(wpb * per_wave), stream, a);
    return hipGetLastError();
}

}  // namespace cng
