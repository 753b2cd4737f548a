// Batched beam search over a proximity graph: the launch interfaces of
// Algorithm 1 (the per-query device code is in beam.hpp).
#include <hip/hip_runtime.h>

#include "beam.hpp"

namespace cng {

namespace {

using namespace beam;

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
        gather_dists<G, RND, VEC, UB, 0>(a.vecs, a.scales, a.d, s.cid, m, qr, s.dsc, 0.f, wave, COOP);
        __syncthreads();
    }
}

using KernelFn = void (*)(SearchArgs);

// Vectors per lane group in one load batch for 32-lane groups: the batch's raw
// words (UB x RND chunks of W words: 4 for float32, 1 for fp8) kept within
// BUDGET registers, at most 16.  bf16 batches are sized as float32 ones
// (measured, 1M x 960 with 1000 queries at L = 352: twice the bf16 batch,
// 4.7 -> 8.8 ms per launch; fp8 batches of 8 vectors instead of 2, 5.25 ->
// 3.50 ms, of 16 vectors 5.05 ms).
template <int RND, int ST, int BUDGET>
constexpr int batch_ub()
{
    constexpr int w = RND * (ST == 2 ? 1 : 4);
    return w >= BUDGET ? 1 : BUDGET / w > 16 ? 16 : BUDGET / w;
}

template <int G, int RND, bool VEC, int ST, int UBX = 0>
KernelFn pick_qs(int qs)
{
    constexpr int UB = UBX ? UBX : G == 32 ? batch_ub<RND, ST, 64>() : G / 2;
    switch (qs) {
    case 1: return search_kernel<G, RND, VEC, 1, UB, ST>;
    case 2: return search_kernel<G, RND, VEC, 2, UB, ST>;
    case 4: return search_kernel<G, RND, VEC, 4, UB, ST>;
    default: return search_kernel<G, RND, VEC, 8, UB, ST>;
    }
}

// deep: a launch of few queries leaves the GPU mostly idle, so float32 and
// bf16 searches with 257 <= d <= 1024 give a load batch twice the registers
// (more vectors per batch, half the memory round trips per hop; 1M x 960,
// 1000 queries at L = 352: bf16 4.7 -> 4.0 ms with the loads kept ahead of
// the arithmetic), fp8 ones keep 64.
template <bool VEC, int ST>
KernelFn pick_kernel(int d, int qs, bool deep)
{
    constexpr int DEEP_REGS = ST == 2 ? 64 : 128;
    if (d <= 32) return pick_qs<8, 1, VEC, ST>(qs);
    if (d <= 64) return pick_qs<16, 1, VEC, ST>(qs);
    int rnd = (d + 127) / 128;
    if (rnd <= 1) return pick_qs<32, 1, VEC, ST>(qs);
    if (rnd <= 2) return pick_qs<32, 2, VEC, ST>(qs);
    if (deep && rnd > 2 && rnd <= 4) return pick_qs<32, 4, VEC, ST, batch_ub<4, ST, DEEP_REGS>()>(qs);
    if (deep && rnd > 4 && rnd <= 8) return pick_qs<32, 8, VEC, ST, batch_ub<8, ST, DEEP_REGS>()>(qs);
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

}  // namespace cng
