// Edge pruning (Definition 2, Eq. (1)) with the pruning procedure of
// Algorithm 2 applied to every point's candidate list, one wavefront per point.
//
// Candidates arrive ascending by (D, id) (Algorithm 2, line 1, done by the
// candidate stage).  For candidate u the wave evaluates D(u, v) for every
// already kept v, G lanes per pair, 64/G pairs per instruction, all loads of a
// batch in flight together; u is dropped as soon as one pair satisfies
//     sqrt(D(p,u)) > alpha * sqrt(D(u,v)) + (alpha + 1) * tau      (strict).
// The comparison is made in float32.  When |lhs - rhs| <= 1e-6 * lhs the pair
// is re-decided from float64 distances of the same reduction order.  At most R
// candidates are kept (stopping there equals keeping the R closest of the full
// shortcut set, since a decision only looks at earlier kept points).
// Three kernels make the same decisions: prune_reg_kernel (d <= 128, R <= 32,
// C <= 128: kept vectors in registers; 1M x 128, R = 32: 11 ms against 33 ms
// for prune_kernel, adaptive alpha 0.9 .. 1.6: 92 ms against 192 ms for the
// table kernel), prune_kernel (fixed alpha otherwise; candidates taken in
// pairs, so that one read of the kept rows from L2 serves two of them: 1M x
// 960, R = 48, C = 192: 653 -> 381 ms) and prune_adaptive_kernel (adaptive
// alpha otherwise).
#include <hip/hip_runtime.h>

#include <cmath>

#include "beam.hpp"

namespace cng {

namespace {

struct PruneArgs {
    const float *points;
    int64_t n;
    int d;
    const uint32_t *cand;
    const float *candD;
    int C, R, W;
    double alpha, tau;
    uint32_t *adj;
    int copy_upto;  // > 0: a list of at most this many candidates is copied, not pruned
    // Algorithm 4: passes i = 0 .. iters-1 with alpha_i = alpha + i * alpha_step;
    // the first whose kept set reaches R/2 stands (iters = 1: fixed alpha)
    int iters;
    double alpha_step;
};

template <int G, int RND, bool VEC>
__device__ __forceinline__ double dist_f64_group(const float *__restrict__ x,
                                                 const float *__restrict__ y, int d, int gl)
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < RND; ++r)
        acc = chunk_fma_f64(load_chunk<VEC>(x, d, r, gl), load_chunk<VEC>(y, d, r, gl), acc);
    return group_sum_f64<G>(acc);
}

// Lazy pruning (Section 4.3): with copy_upto > 0 a list of at most copy_upto
// candidates becomes point p's row as it is.  Returns true if it did.
__device__ __forceinline__ bool copy_short_list(const PruneArgs &a, int64_t p)
{
    if (!(a.copy_upto > 0 &&
          (a.C <= a.copy_upto || a.cand[(size_t)p * a.C + a.copy_upto] == NONE)))
        return false;
    const int lane = lane_id();
    uint32_t *out = a.adj + (size_t)p * a.W;
    bool alive = true;
    for (int s0 = 0; s0 < a.W; s0 += 64) {
        const int s = s0 + lane;
        uint32_t u = s < a.C && s < a.copy_upto ? a.cand[(size_t)p * a.C + s] : NONE;
        const bool ok = alive && u != NONE && (int64_t)u < a.n;
        const uint64_t bad = ballot(!ok);
        const int first_bad = bad ? __builtin_ctzll(bad) : 64;
        if (s < a.W) out[s] = ok && lane < first_bad ? u : NONE;
        if (bad) alive = false;
    }
    return true;
}

template <int G, int RND, bool VEC, int UB>
__global__ __launch_bounds__(256) void prune_kernel(PruneArgs a)
{
    constexpr int NG = 64 / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    const int64_t p = (int64_t)blockIdx.x * wpb + wave;
    if (p >= a.n) return;
    uint32_t *S = reinterpret_cast<uint32_t *>(smem) + (size_t)wave * a.R;
    const int d = a.d;

    if (copy_short_list(a, p)) return;
    const float ta = (float)a.tau;
    const float *xp = a.points + (size_t)p * (uint32_t)d;

    int ns = 0;
    for (int it = 0; it < a.iters; ++it) {
    const double alpha = a.iters > 1 ? a.alpha + it * a.alpha_step : a.alpha;
    const float al = (float)alpha;
    const float cterm = (al + 1.0f) * ta;
    ns = 0;
    // the decision of Eq. (1) for a candidate (lhs = its distance to p, xu its
    // row) against a kept point (summed squared distance acc, id v): float32
    // unless near a tie, then float64 (the same for the whole group)
    auto decide = [&](float lhs, float acc, const float *xu, uint32_t v) -> bool {
        const float dist = __builtin_sqrtf(acc);
        const float rhs = al * dist + cterm;
        if (__builtin_fabsf(lhs - rhs) <= 1e-6f * lhs) {
            const float *xv = a.points + (size_t)v * (uint32_t)d;
            const double a64 = __builtin_sqrt(dist_f64_group<G, RND, VEC>(xp, xu, d, gl));
            const double b64 = __builtin_sqrt(dist_f64_group<G, RND, VEC>(xu, xv, d, gl));
            return a64 > alpha * b64 + (alpha + 1.0) * a.tau;
        }
        return lhs > rhs;
    };
    // Candidates in pairs: both are compared with each batch of kept points
    // (one read of the kept rows serves two candidates); the second is then
    // compared with the first if the first was kept, so each sees exactly the
    // points kept before it.
    for (int j = 0; j < a.C && ns < a.R; j += 2) {
        const uint32_t u0 = a.cand[(size_t)p * a.C + j];
        if (u0 == NONE || (int64_t)u0 >= a.n) break;
        const uint32_t c1 = j + 1 < a.C ? a.cand[(size_t)p * a.C + j + 1] : NONE;
        const bool has1 = c1 != NONE && (int64_t)c1 < a.n;
        const uint32_t u1 = has1 ? c1 : u0;
        const float lhs0 = __builtin_sqrtf(a.candD[(size_t)p * a.C + j]);
        const float lhs1 = has1 ? __builtin_sqrtf(a.candD[(size_t)p * a.C + j + 1]) : 0.f;
        const float *xu0 = a.points + (size_t)u0 * (uint32_t)d;
        const float *xu1 = a.points + (size_t)u1 * (uint32_t)d;
        float4 ur0[RND], ur1[RND];
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            ur0[r] = load_chunk<VEC>(xu0, d, r, gl);
            ur1[r] = load_chunk<VEC>(xu1, d, r, gl);
        }
        bool pr0 = false, pr1 = !has1;
        for (int b = 0; b < ns && !(pr0 && pr1); b += NG * UB) {
            float4 vr[UB][RND];
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                int c = b + t * NG + grp;
                if (c < ns) {
                    const float *xv = a.points + (size_t)S[c] * (uint32_t)d;
#pragma unroll
                    for (int r = 0; r < RND; ++r) vr[t][r] = load_chunk<VEC>(xv, d, r, gl);
                } else {
#pragma unroll
                    for (int r = 0; r < RND; ++r) vr[t][r] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
            bool hit0 = false, hit1 = false;
#pragma unroll
            for (int t = 0; t < UB; ++t) {
                float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
                for (int r = 0; r < RND; ++r) {
                    acc0 = chunk_fma(ur0[r], vr[t][r], acc0);
                    acc1 = chunk_fma(ur1[r], vr[t][r], acc1);
                }
                acc0 = group_sum<G>(acc0);
                acc1 = group_sum<G>(acc1);
                const int c = b + t * NG + grp;
                if (c < ns) {
                    const uint32_t v = S[c];
                    if (!pr0) hit0 = hit0 || (decide(lhs0, acc0, xu0, v) && gl == 0);
                    if (!pr1) hit1 = hit1 || (decide(lhs1, acc1, xu1, v) && gl == 0);
                }
            }
            pr0 = pr0 || ballot(hit0) != 0;
            pr1 = pr1 || ballot(hit1) != 0;
        }
        bool kept0 = false;
        if (!pr0) {
            wave_sync();
            if (lane == 0) S[ns] = u0;
            wave_sync();
            ++ns;
            kept0 = true;
        }
        if (!has1 || ns >= a.R) {
            if (j + 1 < a.C && !has1) break;  // the list ends at j + 1
            continue;
        }
        if (!pr1 && kept0) {
            // the second against the first, now kept
            float acc = 0.f;
#pragma unroll
            for (int r = 0; r < RND; ++r) acc = chunk_fma(ur1[r], ur0[r], acc);
            acc = group_sum<G>(acc);
            pr1 = ballot(decide(lhs1, acc, xu1, u0) && gl == 0) != 0;
        }
        if (!pr1) {
            wave_sync();
            if (lane == 0) S[ns] = u1;
            wave_sync();
            ++ns;
        }
    }
    if (2 * ns >= a.R) break;
    }
    uint32_t *out = a.adj + (size_t)p * a.W;
    for (int s = lane; s < a.W; s += 64) out[s] = s < ns ? S[s] : NONE;
}

// Algorithm 4 with the distance reuse of Section 4.3: the alpha passes run one
// after the other as in prune_kernel, but the distance of a pair (u, v) of
// candidates is kept in an LDS table (keyed by the two list positions) once
// evaluated, so each pair is computed once across the passes: a later pass
// only looks its pairs up.  Per candidate u the kept points are taken in
// batches of 64 pairs: cached pairs are decided first (u may be pruned without
// computing anything), the missing distances are then computed G lanes per
// pair (gather_dists, the fixed order) and entered in the table.  Every
// decision is the comparison of prune_kernel on the same float32 distance
// (near-ties re-decided from float64 distances, by the whole wave), so the
// kept sets are those of running each pass alone.  The table may forget
// (bounded probing, overwrite): a forgotten pair is computed again, to the
// same bits.
constexpr int MAX_PASSES = 1024;
constexpr int PAIR_LOG2 = 10;  // table slots per wave

__host__ __device__ constexpr size_t adaptive_lds_per_wave(int R, int C)
{
    // the table (key << 32 | distance bits), a batch's ids and distances, kept
    // ids and positions, the candidate list (ids and distances)
    return ((size_t)8 << PAIR_LOG2) + 64 * 8 + (size_t)R * 8 + (size_t)C * 8;
}

__device__ __forceinline__ uint32_t pair_slot(uint32_t key, int t)
{
    return ((key * 0x9E3779B1u) >> (32 - PAIR_LOG2)) + (uint32_t)t & ((1u << PAIR_LOG2) - 1u);
}

template <int G, int RND, bool VEC, int UB>
__global__ __launch_bounds__(256) void prune_adaptive_kernel(PruneArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int gl = lane % G;
    const int64_t p = (int64_t)blockIdx.x * wpb + wave;
    if (p >= a.n) return;
    if (copy_short_list(a, p)) return;
    unsigned char *base = smem + (size_t)wave * adaptive_lds_per_wave(a.R, a.C);
    // table entries hold key << 32 | float bits of the distance, so that an
    // entry is written whole (one 64-bit store or atomic)
    unsigned long long *tab = reinterpret_cast<unsigned long long *>(base);  // [2^PAIR_LOG2]
    uint32_t *cid = reinterpret_cast<uint32_t *>(tab + (1 << PAIR_LOG2));  // [64]
    float *dsc = reinterpret_cast<float *>(cid + 64);               // [64]
    uint32_t *Sid = reinterpret_cast<uint32_t *>(dsc + 64);         // [R]
    uint32_t *Spos = Sid + a.R;                                     // [R]
    uint32_t *cand = Spos + a.R;                                    // [C] this point's list
    float *lhsv = reinterpret_cast<float *>(cand + a.C);            // [C] its sqrt(D(p, u))
    const int d = a.d;
    constexpr unsigned long long EMPTY = ~0ull;
    for (int i = lane; i < (1 << PAIR_LOG2); i += 64) tab[i] = EMPTY;
    // the candidate list, read once for all passes
    for (int j = lane; j < a.C; j += 64) {
        cand[j] = a.cand[(size_t)p * a.C + j];
        lhsv[j] = __builtin_sqrtf(a.candD[(size_t)p * a.C + j]);
    }
    wave_sync();
    const float ta = (float)a.tau;
    const float *xp = a.points + (size_t)p * (uint32_t)d;

    int ns = 0;
    for (int it = 0; it < a.iters; ++it) {
        const double alpha = a.alpha + it * a.alpha_step;
        const float al = (float)alpha;
        const float cterm = (al + 1.0f) * ta;
        ns = 0;
        for (int j = 0; j < a.C && ns < a.R; ++j) {
            const uint32_t u = cand[j];
            if (u == NONE || (int64_t)u >= a.n) break;
            const float lhs = lhsv[j];
            const float band = 1e-6f * lhs;
            const float *xu = a.points + (size_t)u * (uint32_t)d;
            bool have_u = false;
            float4 ur[RND];
            bool pruned = false;
            for (int b = 0; b < ns && !pruned; b += 64) {
                const int t = b + lane;
                const bool valid = t < ns;
                // look the pair (j, position of kept point t) up
                const uint32_t key = valid ? ((uint32_t)j << 16) | Spos[t] : NONE;
                float bd = 0.f;
                bool hit = false;
                if (valid) {
                    for (int q = 0; q < 8; ++q) {
                        const unsigned long long e = tab[pair_slot(key, q)];
                        if ((uint32_t)(e >> 32) == key) {
                            bd = __uint_as_float((uint32_t)e);
                            hit = true;
                            break;
                        }
                        if (e == EMPTY) break;
                    }
                }
                // decisions of the cached pairs (float32 unless near a tie)
                bool tie = false, dec = false;
                if (hit) {
                    const float rhs = al * bd + cterm;
                    tie = __builtin_fabsf(lhs - rhs) <= band;
                    dec = !tie && lhs > rhs;
                }
                if (ballot(dec)) {
                    pruned = true;
                    break;
                }
                // the missing distances, G lanes per pair
                const bool miss = valid && !hit;
                const uint64_t mm = ballot(miss);
                const int m = __popcll(mm);
                if (m > 0) {
                    if (!have_u) {
#pragma unroll
                        for (int r = 0; r < RND; ++r) ur[r] = load_chunk<VEC>(xu, d, r, gl);
                        have_u = true;
                    }
                    const int slot = __popcll(mm & ((1ull << lane) - 1ull));
                    if (miss) cid[slot] = Sid[t];
                    wave_sync();
                    beam::gather_dists<G, RND, VEC, UB, 0>(a.points, nullptr, d, cid, m, ur, dsc);
                    wave_sync();
                    if (miss) {
                        bd = __builtin_sqrtf(dsc[slot]);
                        // enter it (overwrite the home slot when the probes are full)
                        const unsigned long long ent = ((unsigned long long)key << 32) | __float_as_uint(bd);
                        bool placed = false;
                        for (int q = 0; q < 8 && !placed; ++q) {
                            const unsigned long long old = atomicCAS(&tab[pair_slot(key, q)], EMPTY, ent);
                            placed = old == EMPTY || (uint32_t)(old >> 32) == key;
                        }
                        if (!placed) atomicExch(&tab[pair_slot(key, 0)], ent);
                        const float rhs = al * bd + cterm;
                        tie = __builtin_fabsf(lhs - rhs) <= band;
                        dec = !tie && lhs > rhs;
                    }
                    wave_sync();
                    if (ballot(dec)) {
                        pruned = true;
                        break;
                    }
                }
                // near-ties: re-decided from float64 distances, one pair at a
                // time by the whole wave
                uint64_t tm = ballot(tie);
                while (tm && !pruned) {
                    const int l = __builtin_ctzll(tm);
                    tm &= tm - 1;
                    const uint32_t v = Sid[b + l];
                    const float *xv = a.points + (size_t)v * (uint32_t)d;
                    const double a64 = __builtin_sqrt(dist_f64_group<G, RND, VEC>(xp, xu, d, gl));
                    const double b64 = __builtin_sqrt(dist_f64_group<G, RND, VEC>(xu, xv, d, gl));
                    pruned = a64 > alpha * b64 + (alpha + 1.0) * a.tau;
                }
            }
            if (!pruned) {
                wave_sync();
                if (lane == 0) {
                    Sid[ns] = u;
                    Spos[ns] = (uint32_t)j;
                }
                wave_sync();
                ++ns;
            }
        }
        if (2 * ns >= a.R) break;
    }
    uint32_t *out = a.adj + (size_t)p * a.W;
    for (int s2 = lane; s2 < a.W; s2 += 64) out[s2] = s2 < ns ? Sid[s2] : NONE;
}

// Fixed and adaptive pruning with the kept points' vectors in registers: for
// d <= 128 (float4 chunks, 32 lanes per vector), R <= 32 and C <= 128.  Lane
// group g (lanes 32g .. 32g+31) holds kept points 2q + g in kv[q], so a
// candidate u is compared with every kept point by one chunk product per kept
// pair per lane and one recursive-halving reduction (group_sums: each sum is
// the fixed-order butterfly of one pair, bit for bit; with d <= 64 the upper
// lanes add exact zeros).  Only the candidate vectors are read from memory, a
// block of REG_AHEAD candidates ahead.  Decisions are those of prune_kernel:
// float32 unless near a tie, then float64 (from the registers).  The passes of
// Algorithm 4 run one after the other and recompute their pairs: evaluating
// several alpha values in one sweep over a shared set of kept vectors (the
// union of the passes' kept sets) was measured slower, its union outgrowing
// the registers of one wave (1M x 128: 144 ms for pairs of passes, 192 ms for
// fours, 95 ms one at a time).
constexpr int REG_KEPT = 32, REG_CAND = 128, REG_AHEAD = 2;

// Squared distances of candidate u (chunk ur) to the kept points 2q + g, q <
// UB: on return the lanes gl % (32 / UB) == 0 of group g hold kept point
// 2 * (gl / (32 / UB)) + g.
template <int UB>
__device__ __forceinline__ float reg_sums(const float4 &ur, const float4 (&kv)[REG_KEPT / 2], int gl)
{
    float acc[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) acc[q] = chunk_fma(ur, kv[q], 0.f);
    group_sums<32, UB>(acc, gl);
    return acc[0];
}

template <bool VEC>
__global__ __launch_bounds__(256) void prune_reg_kernel(PruneArgs a)
{
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int g = lane >> 5, gl = lane & 31;
    const int64_t p = (int64_t)blockIdx.x * wpb + wave;
    if (p >= a.n) return;
    if (copy_short_list(a, p)) return;
    const int d = a.d;
    const float ta = (float)a.tau;
    // the candidate list in registers: lane l holds entries l and l + 64, with
    // sqrt(D(p, u)); the list ends at its first invalid entry
    const uint32_t *cl = a.cand + (size_t)p * a.C;
    const float *cd = a.candD + (size_t)p * a.C;
    const uint32_t c0 = lane < a.C ? cl[lane] : NONE;
    const uint32_t c1 = lane + 64 < a.C ? cl[lane + 64] : NONE;
    const float l0 = lane < a.C ? __builtin_sqrtf(cd[lane]) : 0.f;
    const float l1 = lane + 64 < a.C ? __builtin_sqrtf(cd[lane + 64]) : 0.f;
    int len;
    {
        const uint64_t b0 = ballot(!(c0 != NONE && (int64_t)c0 < a.n));
        const uint64_t b1 = ballot(!(c1 != NONE && (int64_t)c1 < a.n));
        len = b0 ? __builtin_ctzll(b0) : 64 + (b1 ? __builtin_ctzll(b1) : 64);
        if (len > a.C) len = a.C;
    }
    auto cand_at = [&](int j) -> uint32_t {
        return (uint32_t)(j < 64 ? __builtin_amdgcn_readlane((int)c0, j)
                                 : __builtin_amdgcn_readlane((int)c1, j - 64));
    };
    auto lhs_at = [&](int j) -> float {
        return __int_as_float(j < 64 ? __builtin_amdgcn_readlane(__float_as_int(l0), j)
                                     : __builtin_amdgcn_readlane(__float_as_int(l1), j - 64));
    };
    // Lane gl's chunk of a row, loaded unconditionally (lanes past d read the
    // row's first chunk and mask it when it is used): no load sits in a
    // divergent branch, so a use waits for its own loads only.
    const bool in_d = gl * 4 < d;
    auto raw_chunk = [&](uint32_t id) -> float4 {
        return *reinterpret_cast<const float4 *>(a.points + (size_t)id * (uint32_t)d + (in_d ? gl * 4 : 0));
    };
    auto masked = [&](float4 v) -> float4 { return in_d ? v : make_float4(0.f, 0.f, 0.f, 0.f); };
    // candidate j's chunk; past the list, point p's own (a valid row)
    auto fetch = [&](int j) -> float4 { return raw_chunk(j < len ? cand_at(j) : (uint32_t)p); };
    const float4 xpr = masked(raw_chunk((uint32_t)p));

    float4 kv[REG_KEPT / 2];
#pragma unroll
    for (int q = 0; q < REG_KEPT / 2; ++q) kv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t sid = NONE;  // lane t: the t-th kept point
    int ns = 0;
    for (int it = 0; it < a.iters; ++it) {
        const double alpha = a.iters > 1 ? a.alpha + it * a.alpha_step : a.alpha;
        const float al = (float)alpha;
        const float cterm = (al + 1.0f) * ta;
        ns = 0;
        // candidates in blocks of REG_AHEAD: the next block's loads are issued
        // when a block starts and have the whole block's work to arrive
        float4 cur[REG_AHEAD], nxt[REG_AHEAD];
#pragma unroll
        for (int k = 0; k < REG_AHEAD; ++k) cur[k] = fetch(k);
        bool go = len > 0;
        for (int jb = 0; go; jb += REG_AHEAD) {
#pragma unroll
            for (int k = 0; k < REG_AHEAD; ++k) nxt[k] = fetch(jb + REG_AHEAD + k);
#pragma unroll
            for (int k = 0; k < REG_AHEAD; ++k) {
                const int j = jb + k;
                if (!go || j >= len || ns >= a.R) {
                    go = false;
                    break;
                }
                const uint32_t u = cand_at(j);
                const float lhs = lhs_at(j);
                const float4 ur = masked(cur[k]);
                bool pruned = false;
                if (ns > 0) {
                    const int nh = (ns + 1) >> 1;  // kept slots in use per lane group
                    float sum;
                    int span;
                    if (nh <= 2) {
                        sum = reg_sums<2>(ur, kv, gl);
                        span = 16;
                    } else if (nh <= 4) {
                        sum = reg_sums<4>(ur, kv, gl);
                        span = 8;
                    } else if (nh <= 8) {
                        sum = reg_sums<8>(ur, kv, gl);
                        span = 4;
                    } else {
                        sum = reg_sums<16>(ur, kv, gl);
                        span = 2;
                    }
                    const int t = 2 * (gl / span) + g;  // this lane's kept point
                    bool dec = false, tie = false;
                    if (gl % span == 0 && t < ns) {
                        const float dist = __builtin_sqrtf(sum);
                        const float ab = al * dist;
                        const float rhs = ab + cterm;
                        tie = __builtin_fabsf(lhs - rhs) <= 1e-6f * lhs;
                        dec = !tie && lhs > rhs;
                    }
                    pruned = ballot(dec) != 0;
                    uint64_t tm = pruned ? 0ull : ballot(tie);
                    // near-ties: float64 distances from the registers (the
                    // order of dist_f64_group), one pair at a time
                    while (tm && !pruned) {
                        const int l = __builtin_ctzll(tm);
                        tm &= tm - 1;
                        const int tt = 2 * ((l & 31) / span) + (l >> 5);
                        const double a64 = __builtin_sqrt(group_sum_f64<32>(chunk_fma_f64(xpr, ur, 0.0)));
                        double b2 = 0.0;
#pragma unroll
                        for (int q = 0; q < REG_KEPT / 2; ++q)
                            if (q == (tt >> 1)) b2 = chunk_fma_f64(ur, kv[q], 0.0);  // uniform
                        b2 = group_sum_f64<32>(b2);  // group tt & 1 holds the pair
                        b2 = __shfl(b2, (tt & 1) * 32, 64);
                        const double b64 = __builtin_sqrt(b2);
                        // every lane holds the same values: the ballot makes
                        // the decision visibly uniform
                        pruned = ballot(a64 > alpha * b64 + (alpha + 1.0) * a.tau) != 0;
                    }
                }
                if (!pruned) {
                    const int q0 = ns >> 1;
                    const bool mine = g == (ns & 1);
#pragma unroll
                    for (int q = 0; q < REG_KEPT / 2; ++q) {
                        if (q == q0) {  // uniform
                            kv[q].x = mine ? ur.x : kv[q].x;
                            kv[q].y = mine ? ur.y : kv[q].y;
                            kv[q].z = mine ? ur.z : kv[q].z;
                            kv[q].w = mine ? ur.w : kv[q].w;
                        }
                    }
                    if (lane == ns) sid = u;
                    ++ns;
                }
            }
#pragma unroll
            for (int k = 0; k < REG_AHEAD; ++k) cur[k] = nxt[k];
        }
        if (2 * ns >= a.R) break;
    }
    uint32_t *out = a.adj + (size_t)p * a.W;
    for (int s2 = lane; s2 < a.W; s2 += 64) out[s2] = s2 < ns ? sid : NONE;
}

using PruneFn = void (*)(PruneArgs);

template <int G, int RND, bool VEC>
PruneFn prune_fn()
{
    constexpr int UB = G == 32 ? (RND >= 8 ? 1 : 8 / RND) : 4;
    return prune_kernel<G, RND, VEC, UB>;
}

template <int G, int RND, bool VEC>
PruneFn adaptive_fn()
{
    constexpr int UB = G == 32 ? (RND >= 8 ? 1 : 8 / RND) : 4;
    return prune_adaptive_kernel<G, RND, VEC, UB>;
}

template <bool VEC>
PruneFn pick_adaptive(int d)
{
    if (d <= 32) return adaptive_fn<8, 1, VEC>();
    if (d <= 64) return adaptive_fn<16, 1, VEC>();
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return adaptive_fn<32, 1, VEC>();
    if (rnd <= 2) return adaptive_fn<32, 2, VEC>();
    if (rnd <= 4) return adaptive_fn<32, 4, VEC>();
    if (rnd <= 8) return adaptive_fn<32, 8, VEC>();
    if (rnd <= 16) return adaptive_fn<32, 16, VEC>();
    return adaptive_fn<32, 32, VEC>();
}

template <bool VEC>
PruneFn pick_prune(int d)
{
    if (d <= 32) return prune_fn<8, 1, VEC>();
    if (d <= 64) return prune_fn<16, 1, VEC>();
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return prune_fn<32, 1, VEC>();
    if (rnd <= 2) return prune_fn<32, 2, VEC>();
    if (rnd <= 4) return prune_fn<32, 4, VEC>();
    if (rnd <= 8) return prune_fn<32, 8, VEC>();
    if (rnd <= 16) return prune_fn<32, 16, VEC>();
    return prune_fn<32, 32, VEC>();
}

}  // namespace

int adaptive_iters(double alpha0, double alpha_max, double alpha_step)
{
    if (!(alpha_step > 0.0)) return 1;
    return (int)std::floor((alpha_max - alpha0) / alpha_step + 1e-9) + 1;
}

hipError_t launch_prune(const float *points, int64_t n, int d, const uint32_t *cand,
                        const float *candD, int C, int R, int W, double alpha, double tau,
                        uint32_t *adj, hipStream_t stream, int copy_upto, double alpha_max,
                        double alpha_step)
{
    if (n == 0) return hipSuccess;
    const int iters = adaptive_iters(alpha, alpha_max, alpha_step);
    PruneArgs a{points, n, d, cand, candD, C, R, W, alpha, tau, adj, copy_upto, iters,
                alpha_step};
    const bool vec = (d % 4 == 0) && ((uintptr_t)points % 16 == 0);
    if (vec && d <= 128 && R <= REG_KEPT && C <= REG_CAND) {
        const int wpb = 4;
        hipLaunchKernelGGL(prune_reg_kernel<true>, dim3((unsigned)((n + wpb - 1) / wpb)), dim3(64 * wpb),
                           0, stream, a);
        return hipGetLastError();
    }
    const size_t lds_wave = adaptive_lds_per_wave(R, C);
    if (iters > 1 && iters <= MAX_PASSES && lds_wave <= 64 * 1024) {
        // as many waves per workgroup (up to 4) as 64 KB of LDS holds
        int wpa = 4;
        while (wpa > 1 && (size_t)wpa * lds_wave > 64 * 1024) wpa >>= 1;
        PruneFn fn = vec ? pick_adaptive<true>(d) : pick_adaptive<false>(d);
        hipLaunchKernelGGL(fn, dim3((unsigned)((n + wpa - 1) / wpa)), dim3(64 * wpa),
                           (unsigned)(wpa * lds_wave), stream, a);
        return hipGetLastError();
    }
    const int wpb = 4;
    const int64_t blocks = (n + wpb - 1) / wpb;
    PruneFn fn = vec ? pick_prune<true>(d) : pick_prune<false>(d);
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * wpb), (unsigned)(wpb * R * 4), stream, a);
    return hipGetLastError();
}

}  // namespace cng
