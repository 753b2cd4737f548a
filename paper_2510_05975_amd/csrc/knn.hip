// Exact candidate lists: for every row x the C columns y nearest by (D, id),
// D in the fixed reduction order.  This stands in for the local-neighbour set
// V of Algorithm 3 (phases 1-2), computed exactly.
//
// Stage 1, filter (MFMA): a workgroup owns a block of rows and sweeps all
// column tiles.  For each pair it computes F = |y|^2 - 2 x.y on the matrix
// cores (float32 accumulate) and appends (F, id) to the row's band when F is at
// most the row threshold.  Three forms: bf16 inputs for small-integer data
// (exact), bf16 hi/lo pairs for other data (three products per k step), float32
// inputs for the rest (larger integers, extreme magnitudes).  The bf16 forms
// keep a wave's row fragments in registers for d <= 128 (filter_bf16) and
// stream them through k otherwise (filter_wide).  Whenever a band could
// overflow on the next tile it is compacted: cut to F <= F_C + 2E, where F_C
// is the C-th smallest F so far and E bounds |F - (D - |x|^2)| for every
// column of this row (the product and norm rounding of the filter plus the
// rounding of D itself).  Any point of the exact top C then satisfies
// F <= F_C + 2E, so the band always contains it.  With small-integer data every
// quantity is an exact integer and E = 0.  Self-joins with d <= 128 sweep the
// columns in a locality order (see the locality order section below).
// Stage 2, rerank: D is recomputed for the band in the fixed order and the top
// C by (D, id) is selected by a bitonic sort.
// Stage 3: rows whose band overflowed are recomputed exhaustively.
#include <hip/hip_runtime.h>

#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace cng {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 32, APAD = 4;
constexpr int NT = 256;  // threads of the filter workgroup

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t fkey(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unfkey(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

// Smallest float >= v.
__device__ __forceinline__ float float_up(double v)
{
    float f = (float)v;
    if ((double)f < v) {
        uint32_t u = __float_as_uint(f);
        if (f > 0.f) u += 1;
        else if (f < 0.f) u -= 1;
        else u = 1;  // +0 -> smallest subnormal
        f = __uint_as_float(u);
    }
    return f;
}

// ---------------------------------------------------------------- prep
struct PrepOut {
    uint32_t max_norm_bits;  // max |y| over columns (float bits, >= 0)
    uint32_t all_int;        // 1 while every value seen is an integer
    uint32_t max_abs_bits;   // max |value| (float bits)
    uint32_t any_neg;        // 1 if a value < 0
    uint32_t overflow;       // rows recomputed exhaustively
    uint32_t pad[3];
};

// Squared norms of columns (any order: part of the filter's error bound),
// norms of rows, and the small-integer test.
__global__ void prep_cols(const float *__restrict__ y, int64_t nc, int d, float *__restrict__ ny,
                          PrepOut *st)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool isint = true, neg = false;
    float mabs = 0.f, nrm = 0.f;
    if (c < nc) {
        const float *row = y + (size_t)c * d;
        float s = 0.f;
        for (int i = 0; i < d; ++i) {
            float v = row[i];
            s = __builtin_fmaf(v, v, s);
            isint = isint && (v == __builtin_rintf(v));
            neg = neg || v < 0.f;
            mabs = __builtin_fmaxf(mabs, __builtin_fabsf(v));
        }
        ny[c] = s;
        nrm = __builtin_sqrtf(s);
    }
    if (!isint) atomicAnd(&st->all_int, 0u);
    if (neg) atomicOr(&st->any_neg, 1u);
    atomicMax(&st->max_abs_bits, __float_as_uint(mabs));
    atomicMax(&st->max_norm_bits, __float_as_uint(nrm));
}

__global__ void prep_rows(const float *__restrict__ x, int64_t nr, int d, float *__restrict__ xn,
                          PrepOut *st)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool isint = true, neg = false;
    float mabs = 0.f;
    if (r < nr) {
        const float *row = x + (size_t)r * d;
        double s = 0.0;
        for (int i = 0; i < d; ++i) {
            float v = row[i];
            s += (double)v * (double)v;
            isint = isint && (v == __builtin_rintf(v));
            neg = neg || v < 0.f;
            mabs = __builtin_fmaxf(mabs, __builtin_fabsf(v));
        }
        xn[r] = float_up(__builtin_sqrt(s) * (1.0 + 1e-12));
    }
    if (!isint) atomicAnd(&st->all_int, 0u);
    if (neg) atomicOr(&st->any_neg, 1u);
    atomicMax(&st->max_abs_bits, __float_as_uint(mabs));
}

// Per-row error bound E = kappa * (|x| + max|y|)^2 (0 in exact-integer mode).
__global__ void row_bounds(const float *__restrict__ xn, int64_t nr, const PrepOut *st, double kappa,
                           int exact, float *__restrict__ E)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    if (exact) {
        E[r] = 0.f;
        return;
    }
    double my = (double)__uint_as_float(st->max_norm_bits) * (1.0 + 1e-6);
    double s = (double)xn[r] + my;
    E[r] = float_up(kappa * s * s);
}

// ---------------------------------------------------------------- filter
struct FilterArgs {
    const float *rows;
    int64_t nr, r0;  // rows r0 .. r0 + chunk handled by this launch
    int64_t chunk;
    const float *cols;
    int64_t nc;
    int d;
    int C;
    int exclude_self;
    const float *ny;
    const float *E;  // indexed by global row
    int CB;
    float *bandF;    // [chunk x CB]
    uint32_t *bandI;
    int *cnt;        // [chunk]; -1 = overflowed
    PrepOut *st;
    // bf16 filters, self-joins in locality order (nullable): the end of each of
    // the ncells cells in the order (cell c spans cell_ends[c - 1] ..
    // cell_ends[c]).  A workgroup then starts its column sweep at the first
    // tile of the cell holding its middle row, where the nearest columns of
    // its rows are, and wraps around.
    const uint32_t *cell_ends;
    int ncells;
    // filter_wide: column tiles t0 .. t1 - 1 in this launch (t1 = 0: all), the
    // rows' thresholds carried from one launch to the next in thrG [chunk]
    // (the counts in cnt)
    int64_t t0, t1;
    float *thrG;
};

// First column tile of a workgroup's sweep (see FilterArgs::cell_ends).
__device__ __forceinline__ int64_t first_tile(const FilterArgs &a, int64_t row0, int rows, int bn)
{
    if (!a.cell_ends) return 0;
    int64_t mid = row0 + rows / 2;
    if (mid > a.nc - 1) mid = a.nc - 1;
    // the cell of mid: the first c with cell_ends[c] > mid
    int lo = 0, hi = a.ncells - 1;
    while (lo < hi) {
        const int md = (lo + hi) / 2;
        if ((int64_t)a.cell_ends[md] > mid) hi = md;
        else lo = md + 1;
    }
    const int64_t start = lo > 0 ? (int64_t)a.cell_ends[lo - 1] : 0;
    return start / bn;
}

struct FilterLds {
    float *As, *Bs, *thr, *erow;
    int *cnt;
    uint64_t *sort;  // 4 x CB: per wave the keys, then the ids, of a band
    uint32_t *hist;  // 4 x 256
};

// Compact the band of chunk row lr (one wave): find the C-th smallest F
// exactly (radix select over the order-preserving 32-bit keys, 8 bits per
// round), set the threshold to F_C + 2E and keep the entries at or below it
// (in any order: the rerank sorts).  A band that could not take another tile
// of `bn` columns is marked overflowed (cnt = -1, threshold -inf): that row is
// recomputed exhaustively.  After the last tile a band may stay large (no
// further appends follow).
// `keys` is the wave's LDS scratch: CB words of order-preserving keys and,
// with STAGE, CB more words with the ids of the band.  STAGE issues the loads
// of 8 entries per lane before the first is used and reads only LDS after
// that (measured: 262144 x 960 candidate search 0.665 -> 0.637 s), without it
// the entries are read in steps of 64 and the ids again when kept (10M x 128:
// 26.8 s against 30.9 s staged).
template <bool STAGE>
__device__ void compact_band(const FilterArgs &a, int64_t lr, float *thr_slot, int *cnt_slot,
                             float erow, uint32_t *keys, uint32_t *hist, bool last, int bn)
{
    const int lane = lane_id();
    float *bF = a.bandF + (size_t)lr * a.CB;
    uint32_t *bI = a.bandI + (size_t)lr * a.CB;
    uint32_t *ids = STAGE ? keys + a.CB : bI;
    int c = *cnt_slot;
    if (c > a.CB) c = a.CB;
    int keep = c;
    float thr = *thr_slot;
    // the row's own column (appended by the bf16 filter of a self-join) gets
    // the key ~0u: above every threshold, so it is never kept
    const uint32_t self = a.exclude_self ? (uint32_t)(a.r0 + lr) : NONE;
    int real = 0;
    if constexpr (STAGE) {
        for (int e0 = 0; e0 < c; e0 += 8 * 64) {
            uint32_t ib[8];
            float fb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + lane;
                ib[u] = e < c ? bI[e] : NONE;
                fb[u] = e < c ? bF[e] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 64 + lane;
                const bool ok = e < c && ib[u] != self;
                if (e < c) {
                    keys[e] = ok ? fkey(fb[u]) : ~0u;
                    ids[e] = ib[u];
                }
                real += __popcll(ballot(ok));
            }
        }
        wave_sync();
    } else {
        for (int e0 = 0; e0 < c; e0 += 64) {
            const int e = e0 + lane;
            bool ok = false;
            if (e < c) {
                ok = bI[e] != self;
                keys[e] = ok ? fkey(bF[e]) : ~0u;
            }
            real += __popcll(ballot(ok));
        }
    }
    if (real < c && real < a.C) {
        // too few to cut: drop the row's own column only
        int out = 0;
        for (int e0 = 0; e0 < c; e0 += 64) {
            const int e = e0 + lane;
            const bool in = e < c && keys[e] != ~0u;
            const uint32_t id = in ? ids[e] : 0u;
            const uint64_t bm = ballot(in);
            const int p = out + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
            if (in) {
                bF[p] = unfkey(keys[e]);
                bI[p] = id;
            }
            out += __popcll(bm);
        }
        keep = out;
    } else if (c >= a.C) {
        uint32_t prefix = 0, pmask = 0;
        uint32_t k = (uint32_t)a.C;  // rank (1-based) among the keys matching the prefix
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int b = lane; b < 256; b += 64) hist[b] = 0;
            wave_sync();
            for (int e = lane; e < c; e += 64) {
                const uint32_t kk = keys[e];
                if ((kk & pmask) == prefix) atomicAdd(&hist[(kk >> shift) & 255u], 1u);
            }
            wave_sync();
            // lane l holds buckets 4l .. 4l+3; inclusive scan of their sums
            const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                           h3 = hist[4 * lane + 3];
            const uint32_t s = h0 + h1 + h2 + h3;
            uint32_t incl = s;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const uint32_t excl = incl - s;
            const uint64_t m = ballot(excl < k && k <= incl);
            const int L = __builtin_ctzll(m);
            uint32_t before = excl;
            int b = 4 * lane;
            if (before + h0 < k) {
                before += h0;
                ++b;
                if (before + h1 < k) {
                    before += h1;
                    ++b;
                    if (before + h2 < k) {
                        before += h2;
                        ++b;
                    }
                }
            }
            b = __builtin_amdgcn_readlane(b, L);
            before = (uint32_t)__builtin_amdgcn_readlane((int)before, L);
            k -= before;
            prefix |= (uint32_t)b << shift;
            pmask |= 255u << shift;
            wave_sync();
        }
        thr = float_up((double)unfkey(prefix) + 2.0 * (double)erow);
        const uint32_t tk = fkey(thr);
        // keep entries with key <= tk, in place (writes never pass the reads)
        int out = 0;
        for (int e0 = 0; e0 < c; e0 += 64) {
            const int e = e0 + lane;
            const bool in = e < c && keys[e] <= tk;
            const uint32_t id = in ? ids[e] : 0u;
            const uint64_t bm = ballot(in);
            const int p = out + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
            if (in) {
                bF[p] = unfkey(keys[e]);
                bI[p] = id;
            }
            out += __popcll(bm);
        }
        keep = out;
    }
    wave_sync();
    if (lane == 0) {
        if (!last && keep > a.CB - bn) {
            *cnt_slot = -1;
            *thr_slot = -__builtin_inff();
        } else {
            *cnt_slot = keep;
            *thr_slot = thr;
        }
    }
}

template <bool VEC>
__device__ __forceinline__ void load_tile(const float *__restrict__ src, int64_t nrows, int64_t row0,
                                          int d, int k0, float *__restrict__ dst)
{
    // BM x BK floats, stored k-major: dst[k * (BM + APAD) + row]
    for (int f = threadIdx.x; f < BM * BK / 4; f += NT) {
        int row = f / (BK / 4), kq = f % (BK / 4);
        int64_t gr = row0 + row;
        int k = k0 + kq * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gr < nrows) {
            const float *p = src + (size_t)gr * d + k;
            if (VEC) {
                if (k < d) v = *reinterpret_cast<const float4 *>(p);
            } else {
                v.x = k + 0 < d ? p[0] : 0.f;
                v.y = k + 1 < d ? p[1] : 0.f;
                v.z = k + 2 < d ? p[2] : 0.f;
                v.w = k + 3 < d ? p[3] : 0.f;
            }
        }
        dst[(kq * 4 + 0) * (BM + APAD) + row] = v.x;
        dst[(kq * 4 + 1) * (BM + APAD) + row] = v.y;
        dst[(kq * 4 + 2) * (BM + APAD) + row] = v.z;
        dst[(kq * 4 + 3) * (BM + APAD) + row] = v.w;
    }
}

template <bool VEC>
__global__ __launch_bounds__(NT) void filter_f32(FilterArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    FilterLds s;
    s.As = reinterpret_cast<float *>(smem);
    s.Bs = s.As + BK * (BM + APAD);
    s.thr = s.Bs + BK * (BN + APAD);
    s.erow = s.thr + BM;
    s.cnt = reinterpret_cast<int *>(s.erow + BM);
    s.sort = reinterpret_cast<uint64_t *>(s.cnt + BM + 2);  // +2 keeps 8-byte alignment slack
    s.sort = reinterpret_cast<uint64_t *>(((uintptr_t)s.sort + 7) & ~(uintptr_t)7);
    s.hist = reinterpret_cast<uint32_t *>(s.sort + (size_t)(NT / 64) * a.CB);

    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t row0 = a.r0 + (int64_t)blockIdx.x * BM;  // global first row
    const int64_t rend = a.r0 + a.chunk < a.nr ? a.r0 + a.chunk : a.nr;

    for (int li = threadIdx.x; li < BM; li += NT) {
        int64_t gi = row0 + li;
        bool live = gi < rend;
        s.thr[li] = live ? __builtin_inff() : -__builtin_inff();
        s.erow[li] = live ? a.E[gi] : 0.f;
        s.cnt[li] = 0;
    }
    __syncthreads();

    for (int64_t col0 = 0; col0 < a.nc; col0 += BN) {
        floatx16 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

        for (int k0 = 0; k0 < a.d; k0 += BK) {
            load_tile<VEC>(a.rows, rend, row0, a.d, k0, s.As);
            load_tile<VEC>(a.cols, a.nc, col0, a.d, k0, s.Bs);
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < BK; kk += 2) {
                const int k = kk + (lane >> 5);
                float af[2], bf[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) af[i] = s.As[k * (BM + APAD) + wr * 64 + i * 32 + (lane & 31)];
#pragma unroll
                for (int j = 0; j < 2; ++j) bf[j] = s.Bs[k * (BN + APAD) + wc * 64 + j * 32 + (lane & 31)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
            __syncthreads();
        }

        // ---- epilogue: threshold test and append
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t gj = col0 + wc * 64 + j * 32 + (lane & 31);
            if (gj >= a.nc) continue;
            const float nyj = a.ny[gj];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int li = wr * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int64_t gi = row0 + li;
                    if (gi >= rend || (a.exclude_self && gi == gj)) continue;
                    const float F = nyj - 2.0f * acc[i][j][r];
                    if (F <= s.thr[li]) {
                        int pos = atomicAdd(&s.cnt[li], 1);
                        if (pos < a.CB) {
                            const size_t o = (size_t)(gi - a.r0) * a.CB + pos;
                            a.bandF[o] = F;
                            a.bandI[o] = (uint32_t)gj;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // ---- compaction of rows that could overflow on the next tile
        const bool last = col0 + BN >= a.nc;
        for (int li = wave; li < BM; li += NT / 64) {
            const int c = s.cnt[li];
            const bool need = c >= 0 && (last ? c > a.C : c > a.CB - BN);
            if (need)
                compact_band<false>(a, (int64_t)blockIdx.x * BM + li, &s.thr[li], &s.cnt[li], s.erow[li],
                             reinterpret_cast<uint32_t *>(s.sort + (size_t)wave * a.CB),
                             s.hist + wave * 256, last, BN);
        }
        __syncthreads();
    }
    for (int li = threadIdx.x; li < BM; li += NT) {
        int64_t gi = row0 + li;
        if (gi < rend) {
            a.cnt[gi - a.r0] = s.cnt[li];
            if (s.cnt[li] < 0) atomicAdd(&a.st->overflow, 1u);
        }
    }
}

// ---------------------------------------------------------------- bf16 filter
// Used when every value is a small integer (see launch_knn): the bf16 copies
// are then exact, every product and partial sum is an integer below 2^24 and
// the float32 accumulation of the matrix cores is exact, so E = 0.
// A workgroup owns 256 rows (64 per wave, kept in registers as MFMA A
// fragments) and sweeps column tiles of 64 through double-buffered LDS.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM2 = 256, BN2 = 64;

__device__ __forceinline__ uint16_t to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

// Output element t of an n-row bf16 copy with K values per row -> (row r, value
// k): row-major [n x K] when blk = 0, else k-blocked [K / blk][n][blk] (the
// streamed filter reads blk values of many rows per stage, and in this layout
// they are whole, contiguous cache lines).  K is a multiple of blk.
__device__ __forceinline__ void copy_pos(int64_t t, int64_t n, int K, int blk, int64_t &r, int &k)
{
    if (blk) {
        const int64_t nb = n * blk, kb = t / nb, rem = t - kb * nb;
        r = rem / blk;
        k = (int)(kb * blk + rem % blk);
    } else {
        r = t / K;
        k = (int)(t % K);
    }
}

// x [n x d] float32 -> bf16 copy, zero padded to K values per row; row r of the
// copy is row order[r] of x (order may be null: the identity)
__global__ void to_bf16_padded(const float *__restrict__ x, int64_t n, int d, int K, int blk,
                               uint16_t *__restrict__ out, const uint32_t *__restrict__ order)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * K) return;
    int64_t r;
    int k;
    copy_pos(t, n, K, blk, r, k);
    if (order) r = order[r];
    out[t] = k < d ? to_bf16_rne(x[(size_t)r * d + k]) : (uint16_t)0;
}

// x [n x d] float32 -> hi = bf16(x), lo = bf16(x - hi), laid out as above, zero
// padded (x - hi is exact in float32); rows in `order` as above
__global__ void to_bf16_split(const float *__restrict__ x, int64_t n, int d, int K, int blk,
                              uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                              const uint32_t *__restrict__ order)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * K) return;
    int64_t r;
    int k;
    copy_pos(t, n, K, blk, r, k);
    if (order) r = order[r];
    const float v = k < d ? x[(size_t)r * d + k] : 0.f;
    const uint16_t h = to_bf16_rne(v);
    hi[t] = h;
    lo[t] = to_bf16_rne(v - __uint_as_float((uint32_t)h << 16));
}

// bf16 copies: [n x K] for filter_bf16, k-blocked [K / KCW][n][KCW] for filter_wide
struct FilterBf16Args {
    FilterArgs f;
    const uint16_t *rows16;    // nr rows
    const uint16_t *cols16;    // nc rows
    const uint16_t *rows16lo;  // split mode: bf16 of x - hi, nr rows
    const uint16_t *cols16lo;  // nc rows
};

// LDS-only barrier: the band stores of the epilogue need not be complete here
// (they are read only by compaction, which is preceded by a full barrier).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Per-lane thresholds of the 32 rows of this wave that the lane's accumulator
// elements belong to (the 32x32 MFMA output layout).
__device__ __forceinline__ void load_thr(float (&th)[2][16], const float *thr)
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            th[i][r] = thr[wave * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
}

// Epilogue of a column tile of NJ blocks of 32 for the wave's 64 rows: F =
// |y|^2 - 2 x.y against the row thresholds.  One compare per element gives a
// wave mask per (row pair, column block); appends (rare once the thresholds
// have settled) take positions from the register counts (mypos: next free band
// slot of row wave * 64 + lane): a popcount per row and a prefix count per lane.
// A row's own column (self-joins) is appended like any other and dropped by the
// compaction and the rerank.  One column block per instantiation, so that every
// accumulator index is a constant however many blocks a tile has.
// Thresholds come from th (registers) or, with thr_lds set, straight from LDS.
template <int J, int NJ>
__device__ __forceinline__ void append_block(const FilterArgs &a, const floatx16 (&acc)[2][NJ],
                                             const float (&ny)[NJ], const float (&th)[2][16],
                                             const float *thr_lds, int64_t col0, int trig,
                                             uint32_t &mypos, bool &wflag)
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        // The 16 elements of a lane first decide together whether any of them
        // is at or below its threshold: the least F - t of the lane (exact in
        // sign; a NaN F, past the last column, drops out of the minimum), one
        // ballot and one branch for the block instead of one per element.
        float Fv[16], tv[16];
        float g = __builtin_inff();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            Fv[r] = __builtin_fmaf(-2.0f, acc[i][J][r], ny[J]);
            tv[r] = thr_lds ? thr_lds[wave * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)]
                            : th[i][r];
            g = __builtin_fminf(g, Fv[r] - tv[r]);
        }
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(g <= 0.0f) == 0, 1)) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float F = Fv[r];
            const float t = tv[r];
            const uint64_t m = __builtin_amdgcn_ballot_w64(F <= t);
            if (__builtin_expect(m != 0, 0)) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // lanes 32h .. 32h+31 hold row ro of this wave
                    const int ro = i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                    const uint64_t hm = m & (h ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull);
                    if (hm) {
                        // a row holds at most CB - 32 NJ entries when a tile
                        // starts and takes at most 32 NJ in it: every slot
                        // taken here is below CB
                        const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)mypos, ro);
                        const uint32_t o = base + __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(hm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0u));
                        if ((hm >> lane) & 1ull) {
                            a.bandF[o] = F;
                            a.bandI[o] = (uint32_t)(col0 + J * 32 + (lane & 31));
                        }
                        const uint32_t nb = base + (uint32_t)__popcll(hm);
                        wflag |= (int)(base & (uint32_t)(a.CB - 1)) + __popcll(hm) > trig;
                        asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(mypos) : "s"(nb), "i"(ro));
                    }
                }
            }
        }
    }
}

template <int NJ, int... J>
__device__ __forceinline__ bool append_blocks(const FilterArgs &a, const floatx16 (&acc)[2][NJ],
                                              const float (&ny)[NJ], const float (&th)[2][16],
                                              const float *thr_lds, int64_t col0, int trig,
                                              uint32_t &mypos, std::integer_sequence<int, J...>)
{
    bool wflag = false;
    (append_block<J, NJ>(a, acc, ny, th, thr_lds, col0, trig, mypos, wflag), ...);
    return wflag;
}

// Returns whether a band of this wave passed the compaction trigger.
template <int NJ>
__device__ __forceinline__ bool append_tile(const FilterArgs &a, const floatx16 (&acc)[2][NJ],
                                            const float (&ny)[NJ], const float (&th)[2][16],
                                            const float *thr_lds, int64_t col0, int trig,
                                            uint32_t &mypos)
{
    return append_blocks<NJ>(a, acc, ny, th, thr_lds, col0, trig, mypos,
                             std::make_integer_sequence<int, NJ>{});
}

// After a tile (every thread of the workgroup): the barrier that publishes the
// next column tile; then a wave one of whose bands passed the trigger (and
// every wave after the last tile) compacts its own rows' bands that need it:
// only that wave appends to them, so no other wave has to wait for it here
// (measured: 262144 x 960 candidate search 0.633 -> 0.605 s against a
// workgroup-wide compaction step; neutral at d = 128).  An overflowed row
// (count -1) keeps the OVERFLOWED marker and takes nothing more.
constexpr uint32_t OVERFLOWED = 0xFFFFFFFFu;

template <int BN, bool STAGE>
__device__ __forceinline__ void settle_bands(const FilterArgs &a, bool wflag, bool last, int *cnt,
                                             float *thr, const float *erow, uint32_t *keys,
                                             uint32_t *hist, uint32_t rowstart, uint32_t &mypos,
                                             float (&th)[2][16])
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int trig = a.CB - BN;
    lds_barrier();
    if (wflag || last) {  // uniform across the wave
        // this wave's band stores complete before its lanes read them back
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        cnt[wave * 64 + lane] = mypos == OVERFLOWED ? -1 : (int)(mypos - rowstart);
        wave_sync();
        for (int li = wave * 64; li < wave * 64 + 64; ++li) {
            const int c = cnt[li];
            const bool need = c >= 0 && (last ? c > a.C : c > trig);
            if (need)
                compact_band<STAGE>(a, (int64_t)blockIdx.x * BM2 + li, &thr[li], &cnt[li], erow[li],
                                    keys + (size_t)wave * (STAGE ? 2 : 1) * a.CB, hist + wave * 256,
                                    last, BN);
        }
        wave_sync();
        {
            const int c = cnt[wave * 64 + lane];
            mypos = c < 0 ? OVERFLOWED : rowstart + (uint32_t)c;
        }
        load_thr(th, thr);
    }
    if (last) __syncthreads();  // every row's final count is in LDS
}

// SPLIT (general float data): every value is the sum of two bf16 numbers,
// hi = bf16(x) and lo = bf16(x - hi), and x.y is taken as hi.hi + hi.lo + lo.hi
// on the matrix cores (the dropped parts are below 3.1 * 2^-16 |x_k||y_k| per
// element; the band margin E accounts for them).
template <int KS, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SPLIT ? 1 : 2, SPLIT ? 1 : 2)))
void filter_bf16(FilterBf16Args A)
{
    constexpr int K = 16 * KS;
    constexpr int BSTR = K + 8;  // bf16 elements per LDS column row (16 B pad: no bank conflicts)
    constexpr int NP = SPLIT ? 2 : 1;  // parts per value in LDS: hi (and lo)
    const FilterArgs &a = A.f;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *Bs = reinterpret_cast<uint16_t *>(smem);                 // 2 x NP x BN2 x BSTR
    float *nys = reinterpret_cast<float *>(Bs + 2 * NP * BN2 * BSTR);  // 2 x BN2 column norms
    float *thr = nys + 2 * BN2;                                     // BM2
    float *erow = thr + BM2;
    int *cnt = reinterpret_cast<int *>(erow + BM2);                // band counts, during compaction
    uint32_t *hist = reinterpret_cast<uint32_t *>(cnt + BM2);       // 4 x 256
    uint32_t *keys = hist + 4 * 256;                                // 4 x CB

    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row0 = a.r0 + (int64_t)blockIdx.x * BM2;
    const int64_t rend = a.r0 + a.chunk < a.nr ? a.r0 + a.chunk : a.nr;
    for (int li = threadIdx.x; li < BM2; li += 256) {
        int64_t gi = row0 + li;
        bool live = gi < rend;
        // a dead row never takes a column: every F is finite or NaN
        thr[li] = live ? __builtin_inff() : -__builtin_inff();
        erow[li] = live ? a.E[gi] : 0.f;
        cnt[li] = 0;
    }
    // Next free band slot of row wave * 64 + lane, as an offset into the band
    // arrays (a pass holds at most 2^28 entries).  A wave alone appends to its
    // 64 rows, so these live in a register, read and written per row by lane
    // index, and go through LDS (as counts) only around compactions.
    const uint32_t rowstart = (uint32_t)(blockIdx.x * BM2 + wave * 64 + lane) * (uint32_t)a.CB;
    // compaction once a band could not take another whole tile (measured: an
    // earlier cut, at half the capacity, costs more than the appends it saves)
    const int trig = a.CB - BN2;
    uint32_t mypos = rowstart;

    // A fragments of this wave's 64 rows: [row block][k step] (hi, and lo)
    bf16x8 af[2][KS], al[2][SPLIT ? KS : 1];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t gi = row0 + wave * 64 + i * 32 + (lane & 31);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const size_t o = (size_t)gi * K + ks * 16 + (lane >> 5) * 8;
            af[i][ks] = gi < rend ? *reinterpret_cast<const bf16x8 *>(A.rows16 + o) : bf16x8{};
            if constexpr (SPLIT)
                al[i][ks] = gi < rend ? *reinterpret_cast<const bf16x8 *>(A.rows16lo + o) : bf16x8{};
        }
    }

    // B tile loader: BN2 columns x K bf16 = BN2 * K / 8 chunks of 16 B, plus the
    // columns' squared norms (NaN past the last column: F is then NaN and never
    // at or below a threshold)
    constexpr int CHUNKS = BN2 * K / 8;
    static_assert(CHUNKS % 256 == 0, "K is padded to a multiple of 32");
    constexpr int PER_T = CHUNKS / 256;
    // Loads are unconditional (columns past the end are clamped to the last
    // one; their F is NaN through the norm), so no register is cleared while
    // a load may be in flight.
    u32x4 pre[NP][PER_T];
    float pny = 0.f;
    bool pdead = false;
    auto fetch = [&](int64_t col0) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int col = c / (K / 8), kc = c % (K / 8);
            int64_t gj = col0 + col;
            gj = gj < a.nc ? gj : a.nc - 1;
            pre[0][i] = *reinterpret_cast<const u32x4 *>(A.cols16 + (size_t)gj * K + kc * 8);
            if constexpr (SPLIT)
                pre[NP - 1][i] = *reinterpret_cast<const u32x4 *>(A.cols16lo + (size_t)gj * K + kc * 8);
        }
        if (threadIdx.x < BN2) {
            const int64_t gj = col0 + threadIdx.x;
            pdead = gj >= a.nc;
            pny = a.ny[pdead ? a.nc - 1 : gj];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int part = 0; part < NP; ++part)
#pragma unroll
            for (int i = 0; i < PER_T; ++i) {
                const int c = threadIdx.x + 256 * i;
                const int col = c / (K / 8), kc = c % (K / 8);
                *reinterpret_cast<u32x4 *>(Bs + ((size_t)buf * NP + part) * BN2 * BSTR + col * BSTR +
                                           kc * 8) = pre[part][i];
            }
        if (threadIdx.x < BN2) nys[buf * BN2 + threadIdx.x] = pdead ? __builtin_nanf("") : pny;
    };

    const int64_t ntiles = (a.nc + BN2 - 1) / BN2;
    int64_t col0 = first_tile(a, row0, BM2, BN2) * BN2;
    fetch(col0);
    stash(0);
    __syncthreads();
    // per-lane thresholds of the 32 rows this lane sees (refreshed after compactions)
    float th[2][16];
    load_thr(th, thr);

    int buf = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const bool more = t + 1 < ntiles;
        const int64_t next0 = col0 + BN2 < ntiles * BN2 ? col0 + BN2 : 0;
        if (more) fetch(next0);
        constexpr int NJ = BN2 / 32;  // column blocks of a tile
        floatx16 acc[2][NJ];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
        const uint16_t *Bb = Bs + (size_t)buf * NP * BN2 * BSTR + (lane & 31) * BSTR + (lane >> 5) * 8;
        const uint16_t *Bl = Bb + (NP - 1) * BN2 * BSTR;  // lo part (split mode)
        // B fragments one k step ahead of the matrix instructions
        bf16x8 b[NJ], l[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            b[j] = *reinterpret_cast<const bf16x8 *>(Bb + j * 32 * BSTR);
            l[j] = b[j];
            if constexpr (SPLIT) l[j] = *reinterpret_cast<const bf16x8 *>(Bl + j * 32 * BSTR);
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 nb[NJ], nl[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                nb[j] = b[j];
                nl[j] = l[j];
                if (ks + 1 < KS) {
                    nb[j] = *reinterpret_cast<const bf16x8 *>(Bb + j * 32 * BSTR + (ks + 1) * 16);
                    if constexpr (SPLIT)
                        nl[j] = *reinterpret_cast<const bf16x8 *>(Bl + j * 32 * BSTR + (ks + 1) * 16);
                }
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][ks], b[j], acc[i][j], 0, 0, 0);
            if constexpr (SPLIT) {
#pragma unroll
                for (int j = 0; j < NJ; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][ks], l[j], acc[i][j], 0, 0, 0);
#pragma unroll
                for (int j = 0; j < NJ; ++j)
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i][ks], b[j], acc[i][j], 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                b[j] = nb[j];
                l[j] = nl[j];
            }
        }
        // next tile into the other buffer now: its loads were issued a whole
        // matrix phase ago, and waiting for them later would also wait for the
        // band stores of the epilogue
        if (more) stash(buf ^ 1);
        float nyv[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) nyv[j] = nys[buf * BN2 + j * 32 + (lane & 31)];
        const bool wflag = append_tile<NJ>(a, acc, nyv, th, nullptr, col0, trig, mypos);
        settle_bands<BN2, false>(a, wflag, !more, cnt, thr, erow, keys, hist, rowstart, mypos, th);
        buf ^= 1;
        col0 = next0;
    }
    for (int li = threadIdx.x; li < BM2; li += 256) {
        int64_t gi = row0 + li;
        if (gi < rend) {
            a.cnt[gi - a.r0] = cnt[li];
            if (cnt[li] < 0) atomicAdd(&a.st->overflow, 1u);
        }
    }
}

size_t filter_bf16_lds_bytes(int K, int CB, bool split)
{
    return (size_t)2 * (split ? 2 : 1) * BN2 * (K + 8) * 2 + (size_t)2 * BN2 * 4 +
           (size_t)BM2 * 4 * 3 + (size_t)4 * 256 * 4 + (size_t)4 * CB * 4;
}

// ---------------------------------------------------------------- wide bf16 filter
// For d > 128 the fragments of a wave's rows over the whole k range no longer
// fit in registers, so both operands stream through k in stages of KC values
// (the row length K is a multiple of 2 KC).  A workgroup owns 256 rows (64 per
// wave, as in filter_bf16) and sweeps column tiles of BNW.  Only its own wave
// reads a row fragment, so each wave loads its rows straight from global memory
// into registers; the column tile, read by all four waves, goes through LDS.
// Both are double-buffered one stage ahead: stages alternate between buffer
// pairs 0 and 1, and the prefetch issued in a tile's last stage is the next
// tile's first.  Same forms (exact bf16, split hi / lo) and the same epilogue as
// filter_bf16.
template <int KC, int BNW, bool SPLIT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void filter_wide(FilterBf16Args A, int K)
{
    constexpr int KSS = KC / 16;            // k steps per stage
    constexpr int NP = SPLIT ? 2 : 1;       // parts per value: hi (and lo)
    constexpr int BSTR = KC + 8;            // LDS row of a column: 16 B pad against bank conflicts
    constexpr int CPR = KC / 8;             // 16-byte chunks per column, part and stage
    constexpr int PER_T = NP * BNW * CPR / 256;
    static_assert(PER_T * 256 == NP * BNW * CPR, "whole chunks per thread");
    constexpr int NJ = BNW / 32;
    const FilterArgs &a = A.f;
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *Bs = reinterpret_cast<uint16_t *>(smem);  // 2 x NP x BNW x BSTR
    float *thr = reinterpret_cast<float *>(Bs + 2 * NP * BNW * BSTR);
    float *erow = thr + BM2;
    int *cnt = reinterpret_cast<int *>(erow + BM2);
    uint32_t *hist = reinterpret_cast<uint32_t *>(cnt + BM2);  // 4 x 256
    uint32_t *keys = hist + 4 * 256;                          // 4 x 2 CB

    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int64_t row0 = a.r0 + (int64_t)blockIdx.x * BM2;
    const int64_t rend = a.r0 + a.chunk < a.nr ? a.r0 + a.chunk : a.nr;
    const int64_t ntiles = (a.nc + BNW - 1) / BNW;
    // this launch's tiles; the band state of a later launch's rows comes from
    // the one before (bands, counts and thresholds in global memory)
    const int64_t tb = a.t1 > 0 ? a.t0 : 0, te = a.t1 > 0 ? a.t1 : ntiles;
    const bool final_launch = te == ntiles;
    // thread li owns row li here and in the band positions below
    const uint32_t rowstart = (uint32_t)(blockIdx.x * BM2 + wave * 64 + lane) * (uint32_t)a.CB;
    const int trig = a.CB - BNW;
    uint32_t mypos = rowstart;
    {
        const int li = threadIdx.x;
        const int64_t gi = row0 + li;
        const bool live = gi < rend;
        int c = 0;
        float t = live ? __builtin_inff() : -__builtin_inff();
        if (live && tb > 0) {
            c = a.cnt[gi - a.r0];
            t = a.thrG[gi - a.r0];
        }
        thr[li] = t;
        erow[li] = live ? a.E[gi] : 0.f;
        cnt[li] = c;
        mypos = c < 0 ? OVERFLOWED : rowstart + (uint32_t)c;
    }

    // The bf16 copies are k-blocked, [K / KC][rows][KC]: stage k0 of row g
    // starts at k0 * rows + g * KC.  Element offsets of this lane's row
    // fragments within a stage; rows past the end read the last row (a dead
    // row never takes a column), so every load is unconditional.
    size_t aoff[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        int64_t gi = row0 + wave * 64 + i * 32 + (lane & 31);
        gi = gi < rend ? gi : rend - 1;
        aoff[i] = (size_t)gi * KC + (lane >> 5) * 8;
    }
    bf16x8 a0[2][KSS][NP], a1[2][KSS][NP];
    auto fetch_a = [&](bf16x8 (&dst)[2][KSS][NP], int k0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int ks = 0; ks < KSS; ++ks) {
                const size_t o = (size_t)k0 * a.nr + aoff[i] + ks * 16;
                dst[i][ks][0] = *reinterpret_cast<const bf16x8 *>(A.rows16 + o);
                if constexpr (SPLIT) dst[i][ks][NP - 1] = *reinterpret_cast<const bf16x8 *>(A.rows16lo + o);
            }
    };
    // column tile stage: columns past the end read the last column (their F
    // is NaN through the norm)
    u32x4 pre[PER_T];
    auto fetch_b = [&](int64_t col0, int k0) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int part = c / (BNW * CPR), cc = c % (BNW * CPR);
            const int col = cc / CPR, kc = cc % CPR;
            int64_t gj = col0 + col;
            gj = gj < a.nc ? gj : a.nc - 1;
            const uint16_t *src = (SPLIT && part) ? A.cols16lo : A.cols16;
            pre[i] = *reinterpret_cast<const u32x4 *>(src + (size_t)k0 * a.nc + (size_t)gj * KC + kc * 8);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int c = threadIdx.x + 256 * i;
            const int part = c / (BNW * CPR), cc = c % (BNW * CPR);
            const int col = cc / CPR, kc = cc % CPR;
            *reinterpret_cast<u32x4 *>(Bs + ((size_t)(buf * NP + part) * BNW + col) * BSTR + kc * 8) =
                pre[i];
        }
    };
    floatx16 acc[2][NJ];
    auto stage = [&](int buf, const bf16x8 (&af)[2][KSS][NP]) {
        const uint16_t *Bb = Bs + (size_t)buf * NP * BNW * BSTR + (lane & 31) * BSTR + (lane >> 5) * 8;
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(Bb + j * 32 * BSTR + ks * 16);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][ks][0], bh, acc[i][j], 0, 0, 0);
                if constexpr (SPLIT) {
                    const bf16x8 bl =
                        *reinterpret_cast<const bf16x8 *>(Bb + (BNW + j * 32) * BSTR + ks * 16);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][ks][0], bl, acc[i][j], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i][ks][NP - 1], bh, acc[i][j], 0, 0, 0);
                }
            }
        }
    };

    const int S = K / KC;  // even
    int64_t col0 = tb * BNW;
    fetch_a(a0, 0);
    fetch_b(col0, 0);
    stash(0);
    __syncthreads();
    float th[2][16];
    load_thr(th, thr);
    for (int64_t t = tb; t < te; ++t) {
        const bool more_tiles = t + 1 < te;
        const int64_t next0 = col0 + BNW;
        float nyv[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int64_t gj = col0 + j * 32 + (lane & 31);
            nyv[j] = a.ny[gj < a.nc ? gj : a.nc - 1];
            if (gj >= a.nc) nyv[j] = __builtin_nanf("");
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = floatx16{};
        for (int s = 0; s < S; s += 2) {
            // stage s from buffers 0; stage s + 1 (same tile: S is even) into buffers 1
            fetch_a(a1, (s + 1) * KC);
            fetch_b(col0, (s + 1) * KC);
            // keep the loads ahead of the matrix phase (the scheduler would
            // otherwise sink them next to their first use)
            __builtin_amdgcn_sched_barrier(0);
            stage(0, a0);
            stash(1);
            lds_barrier();
            // stage s + 1 from buffers 1; stage s + 2, or the next tile's first, into buffers 0
            const bool in_tile = s + 2 < S;
            const bool more = in_tile || more_tiles;
            if (more) {
                // split form: the next tile's first row fragments are loaded
                // after the epilogue, since held across it they were spilled
                // (1M x 960: 232 -> 91 spilled registers, 6.87 -> 6.83 s)
                if (in_tile || !SPLIT) fetch_a(a0, in_tile ? (s + 2) * KC : 0);
                fetch_b(in_tile ? col0 : next0, in_tile ? (s + 2) * KC : 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            stage(1, a1);
            if (more) stash(0);
            lds_barrier();
        }
        const bool wflag = append_tile<NJ>(a, acc, nyv, th, thr, col0, trig, mypos);
        settle_bands<BNW, true>(a, wflag, !more_tiles && final_launch, cnt, thr, erow, keys, hist,
                                rowstart, mypos, th);
        if constexpr (SPLIT)
            if (more_tiles) fetch_a(a0, 0);
        col0 = next0;
    }
    if (!final_launch) {
        // counts back into LDS (the settle after the last tile left them in
        // the register positions), then state to global memory for the next launch
        cnt[threadIdx.x] = mypos == OVERFLOWED ? -1 : (int)(mypos - rowstart);
        __syncthreads();
    }
    for (int li = threadIdx.x; li < BM2; li += 256) {
        int64_t gi = row0 + li;
        if (gi < rend) {
            a.cnt[gi - a.r0] = cnt[li];
            a.thrG[gi - a.r0] = thr[li];
            if (final_launch && cnt[li] < 0) atomicAdd(&a.st->overflow, 1u);
        }
    }
}

// Stage depth, tile width and occupancy of the wide filter (measured at
// 262144 x 960: 32 / 256 / 1 wave per SIMD 0.67 s; 32 / 128 / 1 0.73 s;
// 16 / 128 / 2 1.55 s)
constexpr int KCW = 32;   // k values per stage
constexpr int BNW = 256;  // columns per tile
constexpr int WPEW = 1;   // waves per SIMD
// column tiles per launch of the wide filter (1M x 960 candidate search: one
// launch per pass 7.30 s, 16 or 64 tiles per launch 6.99 s, 4 tiles 7.40 s)
constexpr int64_t WIDE_TILES = 16;

size_t filter_wide_lds_bytes(int CB, bool split)
{
    return (size_t)2 * (split ? 2 : 1) * BNW * (KCW + 8) * 2 + (size_t)BM2 * 4 * 3 +
           (size_t)4 * 256 * 4 + (size_t)4 * CB * 8;
}

// ---------------------------------------------------------------- rerank
struct RerankArgs {
    const float *rows;
    int64_t r0, chunk, nr;
    const float *cols;
    int64_t nc;
    int d, C, CB;
    const float *bandF;
    const uint32_t *bandI;
    const int *cnt;
    uint32_t *ids;  // [nr x C]
    float *D;
    int exclude_self;  // self-join: a band may hold the row's own column
    // self-joins in locality order: row and band positions -> point ids
    // (nullptr: positions are ids)
    const uint32_t *order;
};

template <int G, int RND, bool VEC>
__global__ __launch_bounds__(256) void rerank_kernel(RerankArgs a)
{
    constexpr int NG = 64 / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    const int64_t lr = (int64_t)blockIdx.x * 4 + wave;
    const int64_t gp = a.r0 + lr;
    if (lr >= a.chunk || gp >= a.nr) return;
    const int c = a.cnt[lr];
    if (c < 0) return;  // exhaustive path
    const int64_t gi = a.order ? (int64_t)a.order[gp] : gp;
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem) + (size_t)wave * a.CB;
    const float *x = a.rows + (size_t)gi * (uint32_t)a.d;
    float4 xr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) xr[r] = load_chunk<VEC>(x, a.d, r, gl);
    const uint32_t *bI = a.bandI + (size_t)lr * a.CB;
    const uint32_t self = a.exclude_self ? (uint32_t)gi : NONE;
    int nself = 0;
    for (int b = 0; b < c; b += NG) {
        const int e = b + grp;
        float4 yr[RND];
        uint32_t id = NONE;
        bool is_self = false;
        if (e < c) {
            id = a.order ? a.order[bI[e]] : bI[e];
            is_self = id == self;
            if (is_self) id = 0;  // its key is replaced below
            const float *y = a.cols + (size_t)id * (uint32_t)a.d;
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = load_chunk<VEC>(y, a.d, r, gl);
        } else {
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r) acc = chunk_fma(xr[r], yr[r], acc);
        acc = group_sum<G>(acc);
        nself += __popcll(ballot(gl == 0 && is_self));
        if (gl == 0 && e < c) buf[e] = is_self ? ~0ull : make_key(acc, id);
    }
    int np = 1;
    while (np < c) np <<= 1;
    wave_sync();
    for (int e = c + lane; e < np; e += 64) buf[e] = ~0ull;
    wave_sync();
    wave_sort(buf, np);
    const int cv = c - nself;  // the row's own column sorted last
    for (int e = lane; e < a.C; e += 64) {
        uint32_t id = NONE;
        float dd = __builtin_inff();
        if (e < cv) {
            id = key_id(buf[e]);
            dd = key_dist(buf[e]);
        }
        a.ids[(size_t)gi * a.C + e] = id;
        a.D[(size_t)gi * a.C + e] = dd;
    }
}

// ---------------------------------------------------------------- exhaustive
// One wave per row whose band overflowed: every column, exact keys, an LDS
// buffer of CB keys cut back to the best C whenever it fills.
template <int G, int RND, bool VEC>
__global__ __launch_bounds__(256) void exhaustive_kernel(RerankArgs a, int exclude_self, int CBX)
{
    constexpr int NG = 64 / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int grp = lane / G, gl = lane % G;
    const int64_t lr = (int64_t)blockIdx.x * 4 + wave;
    const int64_t gp = a.r0 + lr;
    if (lr >= a.chunk || gp >= a.nr) return;
    if (a.cnt[lr] >= 0) return;
    const int64_t gi = a.order ? (int64_t)a.order[gp] : gp;
    // CBX (a power of two) >= C + 64: room for one more batch after a cut to C
    uint64_t *buf = reinterpret_cast<uint64_t *>(smem) + (size_t)wave * CBX;
    const float *x = a.rows + (size_t)gi * (uint32_t)a.d;
    float4 xr[RND];
#pragma unroll
    for (int r = 0; r < RND; ++r) xr[r] = load_chunk<VEC>(x, a.d, r, gl);
    int fill = 0;
    uint64_t thr = ~0ull;
    for (int64_t b = 0; b < a.nc; b += NG) {
        const int64_t col = b + grp;
        float4 yr[RND];
        const bool in = col < a.nc && !(exclude_self && col == gi);
        if (in) {
            const float *y = a.cols + (size_t)col * (uint32_t)a.d;
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = load_chunk<VEC>(y, a.d, r, gl);
        } else {
#pragma unroll
            for (int r = 0; r < RND; ++r) yr[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < RND; ++r) acc = chunk_fma(xr[r], yr[r], acc);
        acc = group_sum<G>(acc);
        const uint64_t key = make_key(acc, (uint32_t)col);
        const bool take = in && gl == 0 && key < thr;
        const uint64_t tm = ballot(take);
        if (take) buf[fill + __popcll(tm & ((1ull << lane) - 1ull))] = key;
        fill += __popcll(tm);
        if (fill + NG > CBX) {  // full: keep the best C (fill > CBX - NG >= C here)
            wave_sync();
            for (int e = fill + lane; e < CBX; e += 64) buf[e] = ~0ull;
            wave_sort(buf, CBX);
            fill = a.C;
            thr = buf[a.C - 1];
        }
    }
    int np = 1;
    while (np < fill) np <<= 1;
    wave_sync();
    for (int e = fill + lane; e < np; e += 64) buf[e] = ~0ull;
    wave_sync();
    wave_sort(buf, np);
    for (int e = lane; e < a.C; e += 64) {
        uint32_t id = NONE;
        float dd = __builtin_inff();
        if (e < fill) {
            id = key_id(buf[e]);
            dd = key_dist(buf[e]);
        }
        a.ids[(size_t)gi * a.C + e] = id;
        a.D[(size_t)gi * a.C + e] = dd;
    }
}

}  // namespace

// ---------------------------------------------------------------- locality order
// Self-joins (d <= 128) sweep their columns in an order where a row's nearest
// columns sit near its own position: every point goes to the cell of its nearest sample
// point (K samples at evenly spaced ids), points are grouped by cell (in any
// order within a cell), and a workgroup starts its sweep at its own cell.
// The thresholds of its rows then settle within the first tiles instead of
// over the whole sweep, which saves band appends and compactions.  The
// candidate lists do not depend on the order: the band rule holds for any
// sweep order, and the rerank maps positions back to point ids.
__global__ void gather_rows(const float *__restrict__ x, int d, int64_t step, int K,
                            float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)K * d) return;
    const int64_t k = t / d;
    out[t] = x[(size_t)(k * step) * d + (t % d)];
}

// (a point without a label, which finite data never has, joins cell 0)
__global__ void cell_hist(const uint32_t *__restrict__ label, int64_t n, int K, uint32_t *hist)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&hist[label[i] < (uint32_t)K ? label[i] : 0u], 1u);
}

// In-place exclusive scan of K <= 8192 counts, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void cell_scan(uint32_t *hist, int K)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t v[8], sum = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = t * 8 + j;
        v[j] = i < K ? hist[i] : 0u;
        sum += v[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = t * 8 + j;
        if (i < K) hist[i] = run;
        run += v[j];
    }
}

__global__ void cell_scatter(const uint32_t *__restrict__ label, int64_t n, int K, uint32_t *cursor,
                             uint32_t *__restrict__ order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) order[atomicAdd(&cursor[label[i] < (uint32_t)K ? label[i] : 0u], 1u)] = (uint32_t)i;
}

__global__ void gather_f32(const float *__restrict__ src, const uint32_t *__restrict__ order,
                           int64_t n, float *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[order[i]];
}

// ---------------------------------------------------------------- host side
namespace {

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

__global__ void zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void init_prep(PrepOut *st)
{
    st->max_norm_bits = 0;
    st->all_int = 1;
    st->max_abs_bits = 0;
    st->any_neg = 0;
    st->overflow = 0;
}

using RerankFn = void (*)(RerankArgs);
using ExhFn = void (*)(RerankArgs, int, int);

template <int G, int RND, bool VEC>
void pick_gr(RerankFn &r, ExhFn &e)
{
    r = rerank_kernel<G, RND, VEC>;
    e = exhaustive_kernel<G, RND, VEC>;
}

template <bool VEC>
void pick_rerank(int d, RerankFn &r, ExhFn &e)
{
    if (d <= 32) return pick_gr<8, 1, VEC>(r, e);
    if (d <= 64) return pick_gr<16, 1, VEC>(r, e);
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return pick_gr<32, 1, VEC>(r, e);
    if (rnd <= 2) return pick_gr<32, 2, VEC>(r, e);
    if (rnd <= 4) return pick_gr<32, 4, VEC>(r, e);
    if (rnd <= 8) return pick_gr<32, 8, VEC>(r, e);
    if (rnd <= 16) return pick_gr<32, 16, VEC>(r, e);
    return pick_gr<32, 32, VEC>(r, e);
}

// Row length of the bf16 copies: whole k steps of 16 in an even count for
// filter_bf16 (d <= 128), whole stage pairs for filter_wide.
int bf16_row_len(int d)
{
    return d <= 128 ? (d + 31) / 32 * 32 : (d + 2 * KCW - 1) / (2 * KCW) * (2 * KCW);
}

size_t filter_lds_bytes(int CB)
{
    size_t b = (size_t)BK * (BM + APAD) * 4 * 2 + (size_t)BM * 4 * 2 + (size_t)(BM + 2) * 4;
    b = (b + 15) & ~(size_t)15;
    return b + (size_t)(NT / 64) * CB * 8 + (size_t)(NT / 64) * 256 * 4;
}

}  // namespace

// Locality order of self-joins: from this many points on, for d <= 128, with
// about 1024 points per cell.  Measured on the 1M x 128 integer workload: 2430
// band appends and 6.5 compactions per row without the order, 1530 and 3.7
// with it (candidate stage 0.51 -> 0.46 s); cells of 4096 to 16384 points gain
// nothing more (a row's 128 nearest neighbours reach far beyond its cell in
// this intrinsic dimension), and at d = 960 the order does not pay for itself.
// Sweeps start at the first tile of the workgroup's cell: 0.437 -> 0.419 s
// against a start half a cell before the workgroup's rows (which often lies in
// the previous cell, an unrelated one); sweeping the tiles of the 6, 12 or 24
// cells with the nearest sample points first instead gained nothing more
// (0.417, 0.434, 0.437 s).
constexpr int64_t ORDER_MIN = 2048;
constexpr int ORDER_MAX_D = 128;

int order_cells(int64_t n)
{
    int64_t K = n / 1024;
    return (int)(K < 2 ? 2 : K > 8192 ? 8192 : K);
}

KnnPlan knn_plan(int64_t nr, int64_t nc, int d, int C, int band, int64_t pass_rows)
{
    KnnPlan p{};
    int CB = band > 0 ? next_pow2(band) : next_pow2(2 * C + (d > 128 ? BNW : BN));
    if (CB < 64) CB = 64;
    // a band takes a whole column tile of the filter before its first cut
    if (d > 128 && CB < BNW) CB = BNW;
    p.band = CB;
    // band bytes per pass: one pass when the whole band fits in 4 GiB, passes
    // of 1 GiB otherwise (measured: 1M x 128 in one pass of 4 GiB 6 % faster
    // than four of 1 GiB; 10M x 128 in ten passes of 4 GiB 2 % slower than
    // 39 of 1 GiB; 1M x 960 in one pass of 8 GiB 3 % slower than eight)
    const int64_t rows_pad = (nr + BM2 - 1) / BM2 * BM2;
    const size_t budget = (size_t)rows_pad * CB * 8 <= ((size_t)4 << 30) ? (size_t)4 << 30
                                                                          : (size_t)1 << 30;
    int64_t chunk = pass_rows > 0 ? pass_rows : (int64_t)(budget / ((size_t)CB * 8));
    chunk = chunk / BM * BM;
    if (chunk < BM) chunk = BM;
    int64_t nr_pad = (nr + BM - 1) / BM * BM;
    if (chunk > nr_pad) chunk = nr_pad;
    chunk = (chunk + BM2 - 1) / BM2 * BM2;  // whole workgroups of either filter
    p.chunk_rows = chunk;
    p.bytes = align256((size_t)nc * 4) + align256((size_t)nr * 4) * 2 + align256(sizeof(PrepOut)) +
              align256((size_t)chunk * CB * 4) * 2 + align256((size_t)chunk * 4) * 2;
    {  // bf16 copies (hi and lo parts) for the matrix-core filters
        const int K = bf16_row_len(d);
        p.bytes += (align256((size_t)nc * K * 2) + align256((size_t)nr * K * 2)) * 2;
    }
    if (nr == nc && nr >= ORDER_MIN && d <= ORDER_MAX_D) {
        // order, labels, label distances, permuted bounds and norms, samples,
        // cell counts, and the cell assignment's own workspace
        const int K = order_cells(nr);
        const KnnPlan in = knn_plan(nr, K, d, 1, d <= 128 ? 2 * BN2 : 2 * BNW);
        p.order_K = K;
        p.inner_chunk = in.chunk_rows;
        p.inner_band = in.band;
        p.inner_bytes = in.bytes;
        p.bytes += align256((size_t)nr * 4) * 5 + align256((size_t)K * d * 4) +
                   align256((size_t)(K + 1) * 4) + in.bytes;
    }
    return p;
}

hipError_t launch_knn(const float *rows, int64_t nr, const float *cols, int64_t nc, int d, int C,
                      int exclude_self, const KnnPlan &plan, uint32_t *ids, float *D, void *ws,
                      hipStream_t stream, int64_t *overflow_rows, int *exact_int, int *dtype)
{
    unsigned char *w = (unsigned char *)ws;
    float *ny = (float *)w;
    w += align256((size_t)nc * 4);
    float *xn = (float *)w;
    w += align256((size_t)nr * 4);
    float *E = (float *)w;
    w += align256((size_t)nr * 4);
    PrepOut *st = (PrepOut *)w;
    w += align256(sizeof(PrepOut));
    const int CB = plan.band;
    float *bandF = (float *)w;
    w += align256((size_t)plan.chunk_rows * CB * 4);
    uint32_t *bandI = (uint32_t *)w;
    w += align256((size_t)plan.chunk_rows * CB * 4);
    int *cnt = (int *)w;
    w += align256((size_t)plan.chunk_rows * 4);
    float *thrG = (float *)w;  // row thresholds between the wide filter's launches
    w += align256((size_t)plan.chunk_rows * 4);
    const int K16 = bf16_row_len(d);
    uint16_t *cols16 = (uint16_t *)w;
    w += align256((size_t)nc * K16 * 2);
    uint16_t *rows16 = (uint16_t *)w;
    w += align256((size_t)nr * K16 * 2);
    uint16_t *cols16lo = (uint16_t *)w;
    w += align256((size_t)nc * K16 * 2);
    uint16_t *rows16lo = (uint16_t *)w;
    w += align256((size_t)nr * K16 * 2);  // the locality order's arrays follow

    hipLaunchKernelGGL(init_prep, dim3(1), dim3(1), 0, stream, st);
    hipLaunchKernelGGL(prep_cols, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream, cols, nc,
                       d, ny, st);
    hipLaunchKernelGGL(prep_rows, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, stream, rows, nr,
                       d, xn, st);
    PrepOut h;
    hipError_t e = hipMemcpyAsync(&h, st, sizeof(PrepOut), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    // exact small-integer mode: every partial sum of the filter and of D is an
    // integer below 2^24, so both are exact and the band needs no margin
    const double M = (double)__builtin_bit_cast(float, h.max_abs_bits);
    const double lim = 16777216.0;
    bool exact = h.all_int != 0 &&
                 (h.any_neg ? 4.0 * d * M * M <= lim : 2.0 * d * M * M <= lim);
    // bf16 holds every integer of magnitude <= 256 exactly
    const bool use_bf16 = exact && M <= 256.0;
    // other data: hi / lo bf16 parts, three products per k step.  Within this
    // range of magnitudes no part is subnormal where it matters and no squared
    // norm overflows; outside it the float32 filter runs.
    const bool use_split = !use_bf16 && !exact && M >= 0x1p-60 && M <= 0x1p60;
    const bool wide = d > 128;
    if (exact_int) *exact_int = exact ? 1 : 0;
    if (dtype) *dtype = use_bf16 ? 1 : use_split ? 2 : 0;
    const bool self = rows == cols && nr == nc;
    // E = kappa (|x| + max|y|)^2 bounds |F - (D - |x|^2)| (module comment).  The
    // split filter adds 2d more float32 roundings per pair and the dropped
    // lo.lo and rounding parts of the bf16 pairs (< 3.1 * 2^-16 |x||y|).
    const double kappa = use_split ? (12.0 * d + 40.0) * 5.9604644775390625e-8 + 4.0 * 1.52587890625e-5
                                   : (6.0 * d + 40.0) * 5.9604644775390625e-8;  // (6d + 40) * 2^-24
    hipLaunchKernelGGL(row_bounds, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, stream, xn, nr,
                       st, kappa, exact ? 1 : 0, E);

    // locality order of a self-join (bf16 filters only)
    const bool ordered = self && plan.order_K > 0 && (use_bf16 || use_split);
    const uint32_t *ord = nullptr, *cell_ends = nullptr;
    const float *Ef = E, *nyf = ny;
    if (ordered) {
        const int K = plan.order_K;
        unsigned char *o = w;
        uint32_t *order = (uint32_t *)o;
        o += align256((size_t)nr * 4);
        uint32_t *label = (uint32_t *)o;
        o += align256((size_t)nr * 4);
        float *labelD = (float *)o;
        o += align256((size_t)nr * 4);
        float *Ep = (float *)o;
        o += align256((size_t)nr * 4);
        float *nyp = (float *)o;
        o += align256((size_t)nr * 4);
        float *samples = (float *)o;
        o += align256((size_t)K * d * 4);
        uint32_t *cursor = (uint32_t *)o;
        o += align256((size_t)(K + 1) * 4);
        const int64_t tk = (int64_t)K * d;
        hipLaunchKernelGGL(gather_rows, dim3((unsigned)((tk + 255) / 256)), dim3(256), 0, stream,
                           cols, d, nc / K, K, samples);
        KnnPlan ip{};
        ip.chunk_rows = plan.inner_chunk;
        ip.band = plan.inner_band;
        ip.bytes = plan.inner_bytes;
        e = launch_knn(cols, nc, samples, K, d, 1, 0, ip, label, labelD, o, stream, nullptr, nullptr,
                       nullptr);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(zero_u32, dim3((unsigned)((K + 256) / 256)), dim3(256), 0, stream, cursor,
                           (int64_t)K + 1);
        const unsigned gn = (unsigned)((nr + 255) / 256);
        hipLaunchKernelGGL(cell_hist, dim3(gn), dim3(256), 0, stream, label, nr, K, cursor);
        hipLaunchKernelGGL(cell_scan, dim3(1), dim3(1024), 0, stream, cursor, K);
        hipLaunchKernelGGL(cell_scatter, dim3(gn), dim3(256), 0, stream, label, nr, K, cursor, order);
        hipLaunchKernelGGL(gather_f32, dim3(gn), dim3(256), 0, stream, E, order, nr, Ep);
        hipLaunchKernelGGL(gather_f32, dim3(gn), dim3(256), 0, stream, ny, order, nr, nyp);
        ord = order;
        cell_ends = cursor;  // after the scatter, cursor[c] is the end of cell c
        Ef = Ep;
        nyf = nyp;
    }
    if (use_bf16 || use_split) {
        const int64_t tc = nc * K16, tr = nr * K16;
        const int blk = wide ? KCW : 0;  // the streamed filter reads k-blocked copies
        if (use_bf16) {
            hipLaunchKernelGGL(to_bf16_padded, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0,
                               stream, cols, nc, d, K16, blk, cols16, ord);
            if (!self)
                hipLaunchKernelGGL(to_bf16_padded, dim3((unsigned)((tr + 255) / 256)), dim3(256), 0,
                                   stream, rows, nr, d, K16, blk, rows16, nullptr);
        } else {
            hipLaunchKernelGGL(to_bf16_split, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0,
                               stream, cols, nc, d, K16, blk, cols16, cols16lo, ord);
            if (!self)
                hipLaunchKernelGGL(to_bf16_split, dim3((unsigned)((tr + 255) / 256)), dim3(256), 0,
                                   stream, rows, nr, d, K16, blk, rows16, rows16lo, nullptr);
        }
        if (self) {
            rows16 = cols16;
            rows16lo = cols16lo;
        }
    }

    const bool vec = (d % 4 == 0) && ((uintptr_t)rows % 16 == 0) && ((uintptr_t)cols % 16 == 0);
    RerankFn rfn;
    ExhFn efn;
    if (vec) pick_rerank<true>(d, rfn, efn);
    else pick_rerank<false>(d, rfn, efn);
    const size_t flds = filter_lds_bytes(CB);
    for (int64_t r0 = 0; r0 < nr; r0 += plan.chunk_rows) {
        const int64_t chunk = nr - r0 < plan.chunk_rows ? nr - r0 : plan.chunk_rows;
        FilterArgs fa{rows, nr, r0, chunk, cols, nc, d, C, exclude_self, nyf, Ef, CB, bandF, bandI, cnt, st,
                      cell_ends, ordered ? plan.order_K : 0};
        if ((use_bf16 || use_split) && wide) {
            // the column sweep in launches of WIDE_TILES column tiles: the
            // workgroups in flight then work on the same columns, which the
            // L2 of each XCD serves to all of them
            const unsigned blocks = (unsigned)((chunk + BM2 - 1) / BM2);
            const unsigned lds = (unsigned)filter_wide_lds_bytes(CB, use_split);
            const int64_t ntw = (nc + BNW - 1) / BNW;
            for (int64_t t0 = 0; t0 < ntw; t0 += WIDE_TILES) {
                fa.t0 = t0;
                fa.t1 = t0 + WIDE_TILES < ntw ? t0 + WIDE_TILES : ntw;
                fa.thrG = thrG;
                FilterBf16Args fb{fa, rows16, cols16, rows16lo, cols16lo};
                if (use_split) hipLaunchKernelGGL((filter_wide<KCW, BNW, true, WPEW>), dim3(blocks), dim3(256), lds, stream, fb, K16);
                else hipLaunchKernelGGL((filter_wide<KCW, BNW, false, WPEW>), dim3(blocks), dim3(256), lds, stream, fb, K16);
            }
        } else if (use_bf16 || use_split) {
            FilterBf16Args fb{fa, rows16, cols16, rows16lo, cols16lo};
            const unsigned blocks = (unsigned)((chunk + BM2 - 1) / BM2);
            const unsigned lds = (unsigned)filter_bf16_lds_bytes(K16, CB, use_split);
            if (use_split) {
                switch (K16 / 32) {
                case 1: hipLaunchKernelGGL((filter_bf16<2, true>), dim3(blocks), dim3(256), lds, stream, fb); break;
                case 2: hipLaunchKernelGGL((filter_bf16<4, true>), dim3(blocks), dim3(256), lds, stream, fb); break;
                case 3: hipLaunchKernelGGL((filter_bf16<6, true>), dim3(blocks), dim3(256), lds, stream, fb); break;
                default: hipLaunchKernelGGL((filter_bf16<8, true>), dim3(blocks), dim3(256), lds, stream, fb); break;
                }
            } else {
                switch (K16 / 32) {
                case 1: hipLaunchKernelGGL((filter_bf16<2, false>), dim3(blocks), dim3(256), lds, stream, fb); break;
                case 2: hipLaunchKernelGGL((filter_bf16<4, false>), dim3(blocks), dim3(256), lds, stream, fb); break;
                case 3: hipLaunchKernelGGL((filter_bf16<6, false>), dim3(blocks), dim3(256), lds, stream, fb); break;
                default: hipLaunchKernelGGL((filter_bf16<8, false>), dim3(blocks), dim3(256), lds, stream, fb); break;
                }
            }
        } else {
            const unsigned fblocks = (unsigned)((chunk + BM - 1) / BM);
            if (vec) hipLaunchKernelGGL(filter_f32<true>, dim3(fblocks), dim3(NT), (unsigned)flds, stream, fa);
            else hipLaunchKernelGGL(filter_f32<false>, dim3(fblocks), dim3(NT), (unsigned)flds, stream, fa);
        }
        RerankArgs ra{rows, r0, chunk, nr, cols, nc, d, C, CB, bandF, bandI, cnt, ids, D, exclude_self, ord};
        const unsigned rblocks = (unsigned)((chunk + 3) / 4);
        hipLaunchKernelGGL(rfn, dim3(rblocks), dim3(256), (unsigned)(4 * CB * 8), stream, ra);
        const int CBX = next_pow2(2 * C + 64 > CB ? 2 * C + 64 : CB);
        hipLaunchKernelGGL(efn, dim3(rblocks), dim3(256), (unsigned)(4 * CBX * 8), stream, ra,
                           exclude_self, CBX);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&h, st, sizeof(PrepOut), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(stream);
    if (overflow_rows) *overflow_rows = h.overflow;
    return e;
}

}  // namespace cng
