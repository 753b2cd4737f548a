// The persistent serving loop's device side (continuous batching of beam
// searches; the host side is serve.hip).
#include <hip/hip_runtime.h>

#include "beam.hpp"

namespace cng {

namespace {

using namespace beam;

// ---------------------------------------------------------------- serving loop
// A persistent grid: every wavefront claims work items in order (item t sits
// at ring position t % rc, in coherent pinned host memory), runs the beam
// search of one query with that item's k and L, writes the results into the
// request's place in the pinned arena and marks the item done with a
// system-scope release store.  The host publishes items by advancing `tail`
// (release); a wave whose claimed item is not yet published sleeps and
// re-checks `tail` and `stop`, and leaves after `idle_limit` empty checks, so
// every wave ends even if the host goes away (the host then launches a fresh
// grid).  A claimed item whose position holds another item number (it was
// retired and the position reused) or that is already done (a fresh grid
// resumes at the oldest incomplete item) is skipped.
__device__ __forceinline__ uint64_t sys_load_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t sys_load_u32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void serve_reset_kernel(unsigned long long *head, uint64_t *mirror, uint64_t first,
                                   uint64_t seen)
{
    if (threadIdx.x == 0) {
        *head = first;
        mirror[0] = seen;
        mirror[1] = 0;
    }
}

template <int G, int RND, bool VEC, int QS, int UB, int ST>
__global__ __launch_bounds__(256) void serve_kernel(ServeArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
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
        const uint64_t pos = t % a.rc;
        // the item's eight words, read through to host memory
        uint32_t f = 0;
        if (lane < 8) f = sys_load_u32(reinterpret_cast<const uint32_t *>(a.items + pos) + lane);
        const uint32_t tag_lo = (uint32_t)__shfl((int)f, 0, 64);
        const uint32_t tag_hi = (uint32_t)__shfl((int)f, 1, 64);
        const uint32_t k = (uint32_t)__shfl((int)f, 2, 64);
        const uint32_t L = (uint32_t)__shfl((int)f, 3, 64);
        const uint32_t entry = (uint32_t)__shfl((int)f, 4, 64);
        const uint32_t qoff = (uint32_t)__shfl((int)f, 5, 64);
        const uint32_t ioff = (uint32_t)__shfl((int)f, 6, 64);
        const uint32_t doff = (uint32_t)__shfl((int)f, 7, 64);
        uint64_t dn = 0;
        if (lane == 0) dn = sys_load_u64(&a.done[pos]);
        dn = ((uint64_t)__shfl((uint32_t)(dn >> 32), 0, 64) << 32) | __shfl((uint32_t)dn, 0, 64);
        if ((((uint64_t)tag_hi << 32) | tag_lo) != t || dn == t + 1) continue;  // retired or done
        uint32_t *words = reinterpret_cast<uint32_t *>(a.arena);
        const uint32_t *qsrc = words + qoff;
        for (int i = lane; i < a.base.d; i += 64) qbuf[i] = __uint_as_float(sys_load_u32(qsrc + i));
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
        q.ids = words + ioff;
        q.dists = reinterpret_cast<float *>(words + doff);
        q.hops = nullptr;
        q.ndc = nullptr;
        if (q.k >= 1 && q.k <= (int)a.max_k && q.Leff <= qcap) beam_query<G, RND, VEC, QS, UB, ST>(q, 0, s);
        wave_sync();
        __threadfence_system();
        if (lane == 0) __hip_atomic_store(&a.done[pos], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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

size_t serve_lds_per_wave(int d, int vlog2)
{
    return wave_lds_bytes(256, vlog2) + (size_t)d * 4 + 16;
}

// The persistent serving grid: `waves` wavefronts, 4 per workgroup.  Needs
// d % 4 == 0, d <= 512, beams up to 256 entries (one template per storage).
hipError_t launch_serve_reset(unsigned long long *head, uint64_t *mirror, uint64_t first,
                              uint64_t seen, hipStream_t stream)
{
    hipLaunchKernelGGL(serve_reset_kernel, dim3(1), dim3(64), 0, stream, head, mirror, first, seen);
    return hipGetLastError();
}

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
