// Device side of the beam search, Algorithm 1 of the paper (beam-search(G, q,
// s, L, k), Section 2.2): one wavefront runs one query.  Shared by the batched
// search kernels (search.hip) and the persistent serving loop (serve_kernel.hip).
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
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {
namespace beam {

constexpr int PROBES = 8;

// Marks id visited; false if it was.  The lanes of one call must hold distinct
// ids: when every probed slot holds another id, the home slot is overwritten
// (the old id is forgotten and may be scored again, which merge_keys
// tolerates), and three lanes meeting there, two of them with the same id,
// would each be told their id is new.
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

// Scores of the stored vectors cid[0..m) against the query (chunks qr, this
// lane's share) into dsc[0..m): the fixed-order squared distance for float32
// and bf16 storage; for fp8 storage the fixed-order dot product with the E4M3
// values, turned into the dot-form score with the query's squared norm qq and
// the vector's (s, n2) (scales holds the pairs).  Group grp of G lanes takes
// vectors b + t * NG + grp for t < UB; all loads of a batch are issued before
// any sum (a batch's trip count is uniform across the wavefront), then the UB
// sums are formed together by group_sums.

// The raw chunks of a batch (VEC layout); slots that no group fills this
// batch (b + t * NG >= m, uniform) are zeros.  GUARD: lanes past d load
// nothing (zeros); without it every chunk lies in the row (d == RND * 4 * G),
// so no lane is masked off around a load.
template <bool GUARD, int NG, int RND, int UB, int ST>
__device__ __forceinline__ void load_batch(typename RawChunk<ST>::type (&raw)[UB][RND],
                                           const void *__restrict__ vecs, const uint32_t (&ids)[UB], int d,
                                           int gl, int b, int m)
{
#pragma unroll
    for (int t = 0; t < UB; ++t) {
        if (b + t * NG < m) {  // uniform: some group still has a vector
#pragma unroll
            for (int r = 0; r < RND; ++r) raw[t][r] = load_raw<ST, GUARD>(vecs, ids[t], d, r, gl);
        } else {
#pragma unroll
            for (int r = 0; r < RND; ++r) raw[t][r] = typename RawChunk<ST>::type{};
        }
    }
}

// PADDED: the 64 entries of cid past m repeat cid[0], so a group past the
// end of the list reads its entry as it is instead of a clamped one (and
// loads the lines of a vector that another group loads too).
template <int G, int RND, bool VEC, int UB, int ST, bool PADDED = false>
__device__ __forceinline__ void gather_dists(const void *__restrict__ vecs, const float *__restrict__ scales,
                                             int d, const uint32_t *cid, int m, const float4 (&qr)[RND],
                                             float *dsc, float qq = 0.f, int part = 0, int parts = 1)
{
    constexpr int NG = 64 / G;
    constexpr int SPAN = G / UB;  // lanes holding one vector's sum after group_sums
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    const int tw = gl / SPAN;     // the vector whose sum this lane ends up holding
    const float2 *sn2 = reinterpret_cast<const float2 *>(scales);
    // batches part, part + parts, ... of the list (several waves may share it)
    for (int b = part * NG * UB; b < m; b += parts * NG * UB) {
        const int cw = b + tw * NG + grp;
        float2 sn = make_float2(0.f, 0.f);
        if (ST == 2 && gl % SPAN == 0 && cw < m) sn = sn2[cid[cw]];
        // Loads only: nothing in a guarded block uses a loaded value, so no
        // wait separates the loads of a batch.  A group past the end of the
        // list re-reads vector b (PADDED: vector 0) and its sum is never
        // written.
        float acc[UB];
        if (VEC) {
            // the batch's ids first (LDS reads, one wait for all of them)
            uint32_t ids[UB];
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                const int c = b + t * NG + grp;
                ids[t] = cid[PADDED || c < m ? c : b];
            }
            typename RawChunk<ST>::type raw[UB][RND];
            if constexpr (PADDED) {
                // every slot loads (its id is valid) and every lane loads
                // (lanes past d from the row's start); a lane past d keeps
                // its partial sum unchanged in that round, as a zero chunk
                // would leave it
#pragma unroll
                for (int t = 0; t < UB; ++t)
#pragma unroll
                    for (int r = 0; r < RND; ++r)
                        raw[t][r] = load_raw<ST, false>(vecs, ids[t], d, (r * 32 + gl) * 4 < d ? r : 0,
                                                        (r * 32 + gl) * 4 < d ? gl : 0);
                // fp8, and bf16 batches of 4 or more vectors of several rounds:
                // every load issued before any arithmetic (the compiler would
                // otherwise reuse loaded registers for later addresses and wait;
                // measured, 1M x 960, 1000 queries at L = 352: fp8 3.51 -> 3.26 ms,
                // bf16 with 4-vector batches 8.7 -> 4.0 ms; float32, and bf16 at
                // d = 128, 1-2 % slower with it)
                if constexpr (ST == 2 || (ST == 1 && RND > 1 && UB >= 4)) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < UB; ++t) {
                    acc[t] = 0.f;
#pragma unroll
                    for (int r = 0; r < RND; ++r) {
                        const float nv = ST == 2 ? chunk_dot(decode_chunk(raw[t][r]), qr[r], acc[t])
                                                 : chunk_fma(decode_chunk(raw[t][r]), qr[r], acc[t]);
                        acc[t] = (r * 32 + gl) * 4 < d ? nv : acc[t];
                    }
                }
            } else {
                load_batch<true, NG, RND, UB, ST>(raw, vecs, ids, d, gl, b, m);
#pragma unroll
                for (int t = 0; t < UB; ++t) {
                    acc[t] = 0.f;
#pragma unroll
                    for (int r = 0; r < RND; ++r) {
                        if (ST == 2) acc[t] = chunk_dot(decode_chunk(raw[t][r]), qr[r], acc[t]);
                        else acc[t] = chunk_fma(decode_chunk(raw[t][r]), qr[r], acc[t]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                acc[t] = 0.f;
                if (b + t * NG < m) {
                    const int c = b + t * NG + grp;
                    const uint32_t id = cid[c < m ? c : b];
#pragma unroll
                    for (int r = 0; r < RND; ++r) {
                        const float4 v = load_stored<ST, VEC>(vecs, id, d, r, gl);
                        acc[t] = ST == 2 ? chunk_dot(v, qr[r], acc[t]) : chunk_fma(v, qr[r], acc[t]);
                    }
                }
            }
        }
        group_sums<G, UB>(acc, gl);
        if (gl % SPAN == 0 && cw < m) dsc[cw] = ST == 2 ? fp8_score(acc[0], qq, sn.x, sn.y) : acc[0];
    }
}

// Merges the keys of the lanes with val set (distinct among themselves) into
// the ascending list qa[0..qn) of at most cap entries: the union, cut to the
// cap smallest (Algorithm 1's beam update).  A key equal to an entry is
// dropped (an id that a forgetful visited table let through twice).  Explored
// bits (bit 63) of the entries are kept and ignored in the order.  Returns the
// new length.  tmp: 64 keys of LDS scratch.
template <int QS>
__device__ __forceinline__ int merge_keys(uint64_t *qa, int qn, int cap, uint64_t *tmp, uint64_t kc,
                                          bool val)
{
    const int lane = lane_id();
    if (qn == cap) val = val && kc < key_mask(qa[cap - 1]);
    int lb = 0;
    if (val) {
        lb = lower_bound_keys(qa, qn, kc);
        if (lb < qn && key_mask(qa[lb]) == kc) val = false;
    }
    const uint64_t sm = ballot(val);
    const int ns = __popcll(sm);
    if (ns == 0) return qn;
    int rank = 0;
    uint64_t it = sm;
    while (it) {
        const int j = __ffsll((unsigned long long)it) - 1;
        it &= it - 1;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kc, j);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(kc >> 32), j);
        const uint64_t kj = ((uint64_t)hi << 32) | lo;
        rank += kj < kc ? 1 : 0;
    }
    if (val) tmp[rank] = kc;
    uint64_t old[QS];
#pragma unroll
    for (int j = 0; j < QS; ++j) {
        const int e = j * 64 + lane;
        old[j] = e < qn ? qa[e] : 0;
    }
    wave_sync();  // every old entry is in registers before any write
    const int nqn = qn + ns < cap ? qn + ns : cap;
#pragma unroll
    for (int j = 0; j < QS; ++j) {
        const int e = j * 64 + lane;
        if (e < qn) {
            const int np = e + lower_bound_keys(tmp, ns, key_mask(old[j]));
            if (np < cap) qa[np] = old[j];
        }
    }
    if (val && lb + rank < cap) qa[lb + rank] = kc;
    wave_sync();
    return nqn;
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
    // fp8 storage: the query's squared norm (fixed-order dot product)
    float qq = 0.f;
    if (ST == 2) {
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r) acc = chunk_dot(qr[r], qr[r], acc);
        qq = group_sum<G>(acc);
    }
    {
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            const float4 v = load_stored<ST, VEC>(a.vecs, s0, d, r, gl);
            acc = ST == 2 ? chunk_dot(v, qr[r], acc) : chunk_fma(v, qr[r], acc);
        }
        acc = group_sum<G>(acc);
        if (ST == 2) {
            const float2 sn = reinterpret_cast<const float2 *>(a.scales)[s0];
            acc = fp8_score(acc, qq, sn.x, sn.y);
        }
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
            // entries past the list repeat its first id (gather_dists, PADDED)
            if (m > 0 && lane >= m)
                s.cid[lane] = (uint32_t)__builtin_amdgcn_readlane((int)v, __ffsll((unsigned long long)fm) - 1);
            wave_sync();
            // ---- distances: G lanes per vector, NG vectors per instruction
            if constexpr (COOP > 1) {
                if (lane == 0) s.ctl[0] = m;
                __syncthreads();  // the list and its length are visible to the helpers
                gather_dists<G, RND, VEC, UB, ST>(a.vecs, a.scales, d, s.cid, m, qr, s.dsc, qq, 0, COOP);
                __syncthreads();  // every share of the distances is in dsc
            } else {
                gather_dists<G, RND, VEC, UB, ST, true>(a.vecs, a.scales, d, s.cid, m, qr, s.dsc, qq);
            }
            wave_sync();
            ndc += (uint32_t)m;
            // ---- merge the m new keys into the beam (Algorithm 1: union, keep the L closest)
            const uint64_t kc = lane < m ? make_key(s.dsc[lane], s.cid[lane]) : KEY_INF;
            qn = merge_keys<QS>(qa, qn, Leff, s.tmp, kc, lane < m);
            if (cut < 64) break;
        }
    }

    if (ST != 0) {
        // ---- re-rank the converged beam with the float32 vectors
        for (int b0 = 0; b0 < qn; b0 += 64) {
            const int cnt = qn - b0 < 64 ? qn - b0 : 64;
            s.cid[lane] = key_id(qa[b0 + (lane < cnt ? lane : 0)]);
            wave_sync();
            // float32 rows take 2 (bf16) or 4 (fp8) times the registers of
            // stored ones: a batch of as many registers, but at least two
            // vectors per group (measured, 1M x 128 at L = 80: bf16 0.996 ->
            // 0.972 ms, fp8 0.938 -> 0.921 ms; 1M x 960 at L = 352, bf16 with
            // one vector per group instead of two 4.74 -> 5.79 ms)
            constexpr int UBS = ST == 1 ? UB / 2 : UB / 4;
            constexpr int UBR = UB < 2 ? 1 : UBS > 2 ? UBS : 2;
            gather_dists<G, RND, VEC, UBR, 0, true>(a.points, nullptr, d, s.cid, cnt, qr, s.dsc);
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
            dist = a.out_sq ? key_dist(ke) : __builtin_sqrtf(key_dist(ke));
        }
        a.ids[(size_t)qi * a.k + e] = id;
        a.dists[(size_t)qi * a.k + e] = dist;
    }
    if (lane == 0) {
        if (a.hops) a.hops[qi] = hops;
        if (a.ndc) a.ndc[qi] = ndc;
    }
}

}  // namespace beam
}  // namespace cng
