// Host side of the serving loop: a persistent search grid fed through a ring
// of item descriptors in coherent pinned host memory (see serve_kernel).
//
// Requests carry 1..n queries with their own k and beam L.  Each query is one
// item; the items of a request are published together at consecutive ring
// positions.  What a request holds while in flight is its footprint in the
// pinned arena: its query vectors (d floats each) and its result space (k ids
// and k distances per query), nq * (4d + 8k) bytes.  Admission is by that
// footprint: the request takes the first free range of the arena that holds
// it (first fit, anywhere), so a long request that is still in flight blocks
// nothing but its own bytes.  A request that does not fit now is refused
// (CNG_ECAPACITY) and the client retries after polling, while the device keeps
// working on everything already admitted: requests that arrive later join the
// running grid as memory frees up.  The per-query beam state (up to 256 keys
// and the visited table) lives in the LDS of the wave that runs the query.
//
// The grid leaves by itself after a long time without work.  Submit and poll
// notice an ended grid and launch a fresh one, which starts at the oldest
// item not yet complete; items that are already complete, or whose position
// has been reused, are skipped by the kernel (it checks the item's tag and
// done word), so nothing is run twice into live memory.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/cng.h"
#include "kernels.hpp"

namespace cng {
void set_error(const char *msg);  // api.hip
}

struct cng_server {
    hipStream_t stream = nullptr;
    cng::ServeArgs args{};
    int waves = 0;
    cng::ServeRing *ring = nullptr;  // host pointers (same memory as args' device pointers)
    cng::ServeItem *items = nullptr;
    unsigned char *arena = nullptr;
    uint64_t *done = nullptr;
    uint64_t rc = 0;                 // ring positions
    uint64_t next_t = 0, next_req = 1;
    uint64_t arena_bytes = 0, arena_used = 0;
    int d = 0, max_k = 0, maxL = 256;
    uint32_t entry = 0;
    std::vector<uint8_t> busy;       // ring position holds an item not yet retired
    std::map<uint64_t, uint64_t> free_ranges;  // arena offset -> length
    struct Req {
        uint64_t t0, off, len;
        int nq, k;
    };
    std::unordered_map<uint64_t, Req> reqs;
    bool running = false;
    cng_serve_stats stats{};
};

namespace {

cng_status err(cng_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
cng_status err(cng_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    cng::set_error(buf);
    return s;
}

template <typename T>
hipError_t pinned(T **host, T **dev, size_t count)
{
    hipError_t e = hipHostMalloc((void **)host, count * sizeof(T), hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) return e;
    std::memset((void *)*host, 0, count * sizeof(T));
    return hipHostGetDevicePointer((void **)dev, (void *)*host, 0);
}

void release_all(cng_server *s)
{
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->items) (void)hipHostFree(s->items);
    if (s->arena) (void)hipHostFree(s->arena);
    if (s->done) (void)hipHostFree(s->done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
}

constexpr uint64_t ARENA_ALIGN = 64;

uint64_t footprint(int nq, int d, int k)
{
    const uint64_t b = (uint64_t)nq * ((uint64_t)d * 4 + (uint64_t)k * 8);
    return (b + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
}

// First free range of the arena that holds len bytes; UINT64_MAX if none.
uint64_t arena_alloc(cng_server *s, uint64_t len)
{
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
        if (it->second < len) continue;
        const uint64_t off = it->first, rest = it->second - len;
        s->free_ranges.erase(it);
        if (rest) s->free_ranges[off + len] = rest;
        s->arena_used += len;
        return off;
    }
    return UINT64_MAX;
}

void arena_free(cng_server *s, uint64_t off, uint64_t len)
{
    s->arena_used -= len;
    auto nx = s->free_ranges.lower_bound(off);
    if (nx != s->free_ranges.end() && off + len == nx->first) {  // merge with the next range
        len += nx->second;
        nx = s->free_ranges.erase(nx);
    }
    if (nx != s->free_ranges.begin()) {  // merge with the previous range
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += len;
            return;
        }
    }
    s->free_ranges[off] = len;
}

// Launch the persistent grid, starting at item `head`; items below `seen`
// count as published.
cng_status launch(cng_server *s, uint64_t head, uint64_t seen)
{
    cng::ServeArgs &a = s->args;
    hipError_t e = cng::launch_serve_reset(a.head, a.mirror, head, seen, s->stream);
    if (e == hipSuccess) e = cng::launch_serve(a, s->waves, s->stream);
    if (e != hipSuccess) {
        s->running = false;
        return err(CNG_EDEVICE, "serve launch: %s", hipGetErrorString(e));
    }
    s->stats.launches++;
    s->running = true;
    return CNG_OK;
}

// A grid that has left (after a long idle time) is replaced by a fresh one
// that starts at the oldest item not yet complete.
cng_status ensure_grid(cng_server *s)
{
    hipError_t q = hipStreamQuery(s->stream);
    if (q == hipErrorNotReady) return CNG_OK;
    if (q != hipSuccess) {
        s->running = false;
        return err(CNG_EDEVICE, "serving grid failed: %s", hipGetErrorString(q));
    }
    uint64_t head = s->next_t;
    for (const auto &kv : s->reqs) {
        const cng_server::Req &r = kv.second;
        for (int i = 0; i < r.nq; ++i) {
            const uint64_t t = r.t0 + i;
            if (t < head && __atomic_load_n(&s->done[t % s->rc], __ATOMIC_ACQUIRE) != t + 1) head = t;
        }
    }
    return launch(s, head, s->next_t);
}

}  // namespace

extern "C" {

size_t cng_serve_workspace_size(void) { return 256; }

cng_status cng_serve_start(const cng_serve_config *c, void *workspace, size_t ws_bytes,
                           cng_server **out)
{
    if (!c || !out) return err(CNG_EINVAL, "NULL argument");
    if (!c->points || !c->vecs || !c->adj) return err(CNG_EINVAL, "NULL graph array");
    if (c->n < 1 || c->n > 2147483646 || c->d < 4 || c->d > 512 || c->d % 4)
        return err(CNG_EUNSUPPORTED, "serving needs 1 <= n < 2^31, d in [4, 512] and d %% 4 == 0");
    if (c->dtype < 0 || c->dtype > 2 || (c->dtype == 2 && !c->scales)) return err(CNG_EINVAL, "bad dtype/scales");
    if (c->W < 1 || c->W > 256) return err(CNG_EUNSUPPORTED, "W out of range");
    if ((int64_t)c->entry >= c->n) return err(CNG_EINVAL, "entry >= n");
    if (c->max_k < 1 || c->max_k > 256) return err(CNG_EUNSUPPORTED, "max_k must be in [1, 256]");
    if (c->visited_log2 != 0 && (c->visited_log2 < 6 || c->visited_log2 > 13))
        return err(CNG_EINVAL, "visited_log2 must be 0 or in [6, 13]");
    if (c->waves < 0 || c->capacity < 0 || c->arena_bytes < 0 || c->idle_checks < 0)
        return err(CNG_EINVAL, "waves, capacity, arena_bytes and idle_checks must be >= 0");
    if (c->arena_bytes > 0 && (uint64_t)c->arena_bytes < footprint(1, c->d, 1))
        return err(CNG_EINVAL, "arena_bytes smaller than one query");
    if ((uint64_t)c->arena_bytes > (16ull << 30)) return err(CNG_EUNSUPPORTED, "arena_bytes above 16 GiB");
    if (!workspace || ws_bytes < cng_serve_workspace_size()) return err(CNG_ENOMEM, "workspace too small");
    const size_t va = c->dtype == 1 ? 8 : c->dtype == 2 ? 4 : 16;
    if ((uintptr_t)c->points % 16 || (uintptr_t)c->vecs % va) return err(CNG_EINVAL, "vectors must be aligned");

    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int waves = c->waves > 0 ? c->waves : 4 * cus;
    const uint64_t rc = c->capacity > 0 ? (uint64_t)c->capacity : 16ull * waves;
    const uint64_t arena = c->arena_bytes > 0 ? (uint64_t)c->arena_bytes
                                              : 4ull * waves * footprint(1, c->d, c->max_k);
    if (arena > (16ull << 30)) return err(CNG_EUNSUPPORTED, "arena_bytes above 16 GiB");

    cng_server *s = new (std::nothrow) cng_server();
    if (!s) return err(CNG_ENOMEM, "host allocation failed");
    s->rc = rc;
    s->waves = waves;
    s->d = c->d;
    s->max_k = c->max_k;
    s->entry = c->entry;
    s->arena_bytes = arena;
    s->busy.assign((size_t)rc, 0);
    s->free_ranges[0] = arena;
    cng::ServeArgs &a = s->args;
    cng::ServeRing *dring;
    cng::ServeItem *ditems;
    unsigned char *darena;
    uint64_t *ddone;
    hipError_t e = pinned(&s->ring, &dring, 1);
    if (e == hipSuccess) e = pinned(&s->items, &ditems, (size_t)rc);
    if (e == hipSuccess) e = pinned(&s->arena, &darena, (size_t)arena);
    if (e == hipSuccess) e = pinned(&s->done, &ddone, (size_t)rc);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        release_all(s);
        delete s;
        return err(CNG_EDEVICE, "serve start: %s", hipGetErrorString(e));
    }
    a.base.points = c->points;
    a.base.vecs = c->vecs;
    a.base.scales = c->scales;
    a.base.store = c->dtype;
    a.base.n = c->n;
    a.base.d = c->d;
    a.base.adj = c->adj;
    a.base.W = c->W;
    if (c->visited_log2) {
        a.base.vlog2 = c->visited_log2;
    } else {
        // the persistent grid keeps its waves resident anyway: the largest
        // table (up to 8192 slots) whose workgroups still fit the LDS of a
        // compute unit, so that fewer forgotten vectors are read again
        const int64_t wg_per_cu = ((int64_t)waves + 4 * cus - 1) / (4 * cus);
        int vl = 13;
        while (vl > 10 && (size_t)wg_per_cu * 4 * cng::serve_lds_per_wave(c->d, vl) > 160 * 1024) --vl;
        a.base.vlog2 = vl;
    }
    a.ring = dring;
    a.items = ditems;
    a.rc = rc;
    a.arena = darena;
    a.done = ddone;
    a.head = (unsigned long long *)workspace;
    a.mirror = (uint64_t *)workspace + 2;
    a.max_k = (uint32_t)c->max_k;
    a.idle_limit = c->idle_checks > 0 ? (uint32_t)c->idle_checks : 1u << 21;  // seconds of quiet
    s->stats.arena_bytes = (int64_t)arena;
    cng_status st = launch(s, 0, 0);
    if (st != CNG_OK) {
        (void)hipStreamSynchronize(s->stream);
        release_all(s);
        delete s;
        return st;
    }
    *out = s;
    return CNG_OK;
}

cng_status cng_serve_submit(cng_server *s, const float *queries_host, int32_t nq, int32_t k,
                            int32_t L, const uint32_t *entries_host, uint64_t *req_host)
{
    if (!s) return err(CNG_EINVAL, "NULL server");
    if (!queries_host || !req_host) return err(CNG_EINVAL, "NULL argument");
    if (nq < 1 || (uint64_t)nq > s->rc) return err(CNG_EINVAL, "nq=%d must be in [1, capacity]", nq);
    if (k < 1 || k > s->max_k) return err(CNG_EINVAL, "k=%d must be in [1, max_k]", k);
    if (L < 1 || (L > k ? L : k) > s->maxL) return err(CNG_EUNSUPPORTED, "max(L, k) must be <= 256");
    if (entries_host)
        for (int i = 0; i < nq; ++i)
            if ((int64_t)entries_host[i] >= s->args.base.n) return err(CNG_EINVAL, "entry %u >= n", entries_host[i]);
    const uint64_t len = footprint(nq, s->d, k);
    if (len > s->arena_bytes) return err(CNG_EINVAL, "request of %llu bytes exceeds the arena", (unsigned long long)len);
    for (int i = 0; i < nq; ++i)
        if (s->busy[(s->next_t + i) % s->rc]) {
            s->stats.refused++;
            return err(CNG_ECAPACITY, "not admitted: ring positions still held by unretired items");
        }
    const uint64_t off = arena_alloc(s, len);
    if (off == UINT64_MAX) {
        s->stats.refused++;
        return err(CNG_ECAPACITY, "not admitted: no free arena range of %llu bytes", (unsigned long long)len);
    }
    cng_status st = ensure_grid(s);
    if (st != CNG_OK) {
        arena_free(s, off, len);
        return st;
    }
    const uint64_t req = s->next_req++;
    const uint64_t qbase = off, ibase = off + (uint64_t)nq * s->d * 4, dbase = ibase + (uint64_t)nq * k * 4;
    std::memcpy(s->arena + qbase, queries_host, (size_t)nq * s->d * 4);
    for (int i = 0; i < nq; ++i) {
        const uint64_t t = s->next_t + i, p = t % s->rc;
        s->busy[p] = 1;
        cng::ServeItem &it = s->items[p];
        it.tag_lo = (uint32_t)t;
        it.tag_hi = (uint32_t)(t >> 32);
        it.k = (uint32_t)k;
        it.L = (uint32_t)L;
        it.entry = entries_host ? entries_host[i] : s->entry;
        it.qoff = (uint32_t)((qbase + (uint64_t)i * s->d * 4) / 4);
        it.ioff = (uint32_t)((ibase + (uint64_t)i * k * 4) / 4);
        it.doff = (uint32_t)((dbase + (uint64_t)i * k * 4) / 4);
    }
    s->reqs[req] = cng_server::Req{s->next_t, off, len, nq, k};
    s->next_t += nq;
    s->stats.submitted++;
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&s->ring->tail, s->next_t, __ATOMIC_RELEASE);
    *req_host = req;
    return CNG_OK;
}

cng_status cng_serve_poll(cng_server *s, uint64_t req, uint32_t *ids_host, float *dists_host,
                          int32_t *done_host)
{
    if (!s || !done_host) return err(CNG_EINVAL, "NULL argument");
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return err(CNG_EINVAL, "unknown request %llu", (unsigned long long)req);
    const cng_server::Req r = it->second;
    for (int i = 0; i < r.nq; ++i) {
        const uint64_t t = r.t0 + i;
        if (__atomic_load_n(&s->done[t % s->rc], __ATOMIC_ACQUIRE) != t + 1) {
            *done_host = 0;
            return ensure_grid(s);
        }
    }
    const uint64_t ibase = r.off + (uint64_t)r.nq * s->d * 4, dbase = ibase + (uint64_t)r.nq * r.k * 4;
    if (ids_host) std::memcpy(ids_host, s->arena + ibase, (size_t)r.nq * r.k * 4);
    if (dists_host) std::memcpy(dists_host, s->arena + dbase, (size_t)r.nq * r.k * 4);
    for (int i = 0; i < r.nq; ++i) s->busy[(r.t0 + i) % s->rc] = 0;
    arena_free(s, r.off, r.len);
    s->reqs.erase(it);
    s->stats.completed++;
    *done_host = 1;
    return CNG_OK;
}

cng_status cng_serve_get_stats(cng_server *s, cng_serve_stats *out)
{
    if (!s || !out) return err(CNG_EINVAL, "NULL argument");
    *out = s->stats;
    out->arena_used = (int64_t)s->arena_used;
    out->running = hipStreamQuery(s->stream) == hipErrorNotReady ? 1 : 0;
    out->in_flight = (int64_t)s->reqs.size();
    return CNG_OK;
}

cng_status cng_serve_stop(cng_server *s)
{
    if (!s) return err(CNG_EINVAL, "NULL server");
    __atomic_store_n(&s->ring->stop, 1ull, __ATOMIC_RELEASE);
    hipError_t e = hipStreamSynchronize(s->stream);
    release_all(s);
    delete s;
    if (e != hipSuccess) return err(CNG_EDEVICE, "serve stop: %s", hipGetErrorString(e));
    return CNG_OK;
}

}  // extern "C"
