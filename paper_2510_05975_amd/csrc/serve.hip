// Host side of the serving loop: a persistent search grid fed through rings
// in coherent pinned host memory (see serve_kernel).  Requests carry 1..cap
// queries with their own k and beam L.  Admission: a request takes as many
// consecutive ring slots as it has queries; each slot holds one query's vector
// and result space, so the slots bound both the queries in flight and their
// memory.  A request that does not fit is refused (CNG_ECAPACITY) and the
// client retries after polling, while the device keeps working on everything
// already admitted: requests that arrive later join the running grid as slots
// free up.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
    cng::ServeRing *ring = nullptr;  // host pointers (same memory as args' device pointers)
    cng::ServeItem *items = nullptr;
    float *payload = nullptr;
    uint32_t *out_ids = nullptr;
    float *out_dists = nullptr;
    uint64_t *done = nullptr;
    uint64_t cap = 0, next_t = 0, next_req = 1;
    int d = 0, max_k = 0, maxL = 256;
    uint32_t entry = 0;
    std::vector<uint64_t> owner;  // item t occupying each slot, or FREE
    struct Req {
        uint64_t t0;
        int nq, k;
    };
    std::unordered_map<uint64_t, Req> reqs;
    bool running = false;
};

namespace {

constexpr uint64_t FREE = ~0ull;

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
    if (s->payload) (void)hipHostFree(s->payload);
    if (s->out_ids) (void)hipHostFree(s->out_ids);
    if (s->out_dists) (void)hipHostFree(s->out_dists);
    if (s->done) (void)hipHostFree(s->done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
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
    if (!workspace || ws_bytes < cng_serve_workspace_size()) return err(CNG_ENOMEM, "workspace too small");
    const size_t va = c->dtype == 1 ? 8 : c->dtype == 2 ? 4 : 16;
    if ((uintptr_t)c->points % 16 || (uintptr_t)c->vecs % va) return err(CNG_EINVAL, "vectors must be aligned");

    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int waves = c->waves > 0 ? c->waves : 4 * cus;
    const int cap = c->capacity > 0 ? c->capacity : 4 * waves;

    cng_server *s = new (std::nothrow) cng_server();
    if (!s) return err(CNG_ENOMEM, "host allocation failed");
    s->cap = (uint64_t)cap;
    s->d = c->d;
    s->max_k = c->max_k;
    s->entry = c->entry;
    s->owner.assign((size_t)cap, FREE);
    cng::ServeArgs &a = s->args;
    cng::ServeRing *dring;
    cng::ServeItem *ditems;
    float *dpay, *ddist;
    uint32_t *dids;
    uint64_t *ddone;
    hipError_t e = pinned(&s->ring, &dring, 1);
    if (e == hipSuccess) e = pinned(&s->items, &ditems, (size_t)cap);
    if (e == hipSuccess) e = pinned(&s->payload, &dpay, (size_t)cap * c->d);
    if (e == hipSuccess) e = pinned(&s->out_ids, &dids, (size_t)cap * c->max_k);
    if (e == hipSuccess) e = pinned(&s->out_dists, &ddist, (size_t)cap * c->max_k);
    if (e == hipSuccess) e = pinned(&s->done, &ddone, (size_t)cap);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, 64, s->stream);
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
    a.cap = (uint64_t)cap;
    a.payload = dpay;
    a.out_ids = dids;
    a.out_dists = ddist;
    a.done = ddone;
    a.head = (unsigned long long *)workspace;
    a.mirror = (uint64_t *)workspace + 2;
    a.max_k = (uint32_t)c->max_k;
    a.idle_limit = 1u << 21;  // some seconds without work end the grid
    e = cng::launch_serve(a, waves, s->stream);
    if (e != hipSuccess) {
        release_all(s);
        delete s;
        return err(CNG_EDEVICE, "serve launch: %s", hipGetErrorString(e));
    }
    s->running = true;
    *out = s;
    return CNG_OK;
}

cng_status cng_serve_submit(cng_server *s, const float *queries_host, int32_t nq, int32_t k,
                            int32_t L, const uint32_t *entries_host, uint64_t *req_host)
{
    if (!s || !s->running) return err(CNG_EINVAL, "server not running");
    if (!queries_host || !req_host) return err(CNG_EINVAL, "NULL argument");
    if (nq < 1 || (uint64_t)nq > s->cap) return err(CNG_EINVAL, "nq=%d must be in [1, capacity]", nq);
    if (k < 1 || k > s->max_k) return err(CNG_EINVAL, "k=%d must be in [1, max_k]", k);
    if (L < 1 || (L > k ? L : k) > s->maxL) return err(CNG_EUNSUPPORTED, "max(L, k) must be <= 256");
    for (int i = 0; i < nq; ++i)
        if (s->owner[(s->next_t + i) % s->cap] != FREE)
            return err(CNG_ECAPACITY, "not admitted: ring slots busy");
    const uint64_t req = s->next_req++;
    for (int i = 0; i < nq; ++i) {
        const uint64_t t = s->next_t + i, slot = t % s->cap;
        s->owner[slot] = t;
        cng::ServeItem &it = s->items[slot];
        it.req = (uint32_t)req;
        it.k = (uint32_t)k;
        it.L = (uint32_t)L;
        it.entry = entries_host ? entries_host[i] : s->entry;
        std::memcpy(s->payload + slot * s->d, queries_host + (size_t)i * s->d, (size_t)s->d * 4);
    }
    s->reqs[req] = cng_server::Req{s->next_t, nq, k};
    s->next_t += nq;
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
        if (__atomic_load_n(&s->done[t % s->cap], __ATOMIC_ACQUIRE) != t + 1) {
            *done_host = 0;
            if (hipStreamQuery(s->stream) != hipErrorNotReady) {
                s->running = false;
                return err(CNG_EDEVICE, "the serving grid has ended");
            }
            return CNG_OK;
        }
    }
    for (int i = 0; i < r.nq; ++i) {
        const uint64_t slot = (r.t0 + i) % s->cap;
        if (ids_host) std::memcpy(ids_host + (size_t)i * r.k, s->out_ids + slot * s->max_k, (size_t)r.k * 4);
        if (dists_host) std::memcpy(dists_host + (size_t)i * r.k, s->out_dists + slot * s->max_k, (size_t)r.k * 4);
        s->owner[slot] = FREE;
    }
    s->reqs.erase(it);
    *done_host = 1;
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
