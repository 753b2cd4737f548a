// C ABI of libcng: argument validation, workspace layout and the build
// pipeline (Algorithm 3 with exact candidates and fixed alpha):
//   entry point -> exact candidate lists -> pruning (Algorithm 2, Eq. (1))
//   -> connectivity (phase 4).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>

#include "../../include/cng.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

cng_status fail(cng_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
cng_status fail(cng_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

}  // namespace

namespace cng {
void set_error(const char *msg) { g_err = msg; }
}  // namespace cng

namespace {

cng_status ok()
{
    g_err.clear();
    return CNG_OK;
}

cng_status hip_fail(hipError_t e, const char *where)
{
    return fail(CNG_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int64_t MAX_N = 2147483646;  // ids are uint32 with bit 31 never set
constexpr int MAX_W = 256;
constexpr int MAX_LEFF = 512;

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

cng_status check_points(const void *p, int64_t n, int32_t d, int64_t nmin)
{
    if (n < nmin || n > MAX_N) return fail(CNG_EINVAL, "n=%lld out of range [%lld, %lld]", (long long)n, (long long)nmin, (long long)MAX_N);
    if (d < 1 || d > 4096) return fail(CNG_EINVAL, "d=%d out of range [1, 4096]", d);
    if (!p) return fail(CNG_EINVAL, "points is NULL");
    return CNG_OK;
}

cng_status check_adaptive(double alpha0, double alpha_max, double alpha_step)
{
    if (alpha_step == 0.0) return CNG_OK;
    if (!(alpha_step > 0.0) || !std::isfinite(alpha_step)) return fail(CNG_EINVAL, "alpha_step must be finite and >= 0");
    if (!(alpha_max >= alpha0) || !std::isfinite(alpha_max)) return fail(CNG_EINVAL, "alpha_max must be finite and >= alpha");
    if ((alpha_max - alpha0) / alpha_step > 1023.0) return fail(CNG_EUNSUPPORTED, "more than 1024 alpha passes");
    return CNG_OK;
}

struct BuildSizes {
    int Ceff, W, Lc;
    bool graph;             // CNG_BUILD_GRAPH_CANDIDATES
    int gK, gRounds, gL;    // its K-NN graph degree, rounds and beam width
    cng::KnnPlan knn;
    size_t cand_ids, cand_D, g0, entry, connect, backward, total;
};

cng_status build_sizes(int64_t n, int32_t d, const cng_build_params *p, BuildSizes *z)
{
    cng_status s = check_points((const void *)1, n, d, 2);
    if (s != CNG_OK) return s;
    if (!p) return fail(CNG_EINVAL, "params is NULL");
    if (p->R < 1) return fail(CNG_EINVAL, "R=%d must be >= 1", p->R);
    if (p->extra < 0) return fail(CNG_EINVAL, "extra=%d must be >= 0", p->extra);
    if (p->R + p->extra > MAX_W) return fail(CNG_EUNSUPPORTED, "row width R+extra=%d exceeds %d", p->R + p->extra, MAX_W);
    if (p->C < 1) return fail(CNG_EINVAL, "C=%d must be >= 1", p->C);
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(CNG_EINVAL, "alpha must be finite and > 0");
    if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) return fail(CNG_EINVAL, "tau must be finite and >= 0");
    s = check_adaptive(p->alpha, p->alpha_max, p->alpha_step);
    if (s != CNG_OK) return s;
    if (p->Lc < 0) return fail(CNG_EINVAL, "Lc=%d must be >= 0", p->Lc);
    if (p->band < 0 || p->band > 2048) return fail(CNG_EUNSUPPORTED, "band=%d must be in [0, 2048]", p->band);
    if (p->visited_log2 != 0 && (p->visited_log2 < 6 || p->visited_log2 > 14))
        return fail(CNG_EINVAL, "visited_log2=%d must be 0 or in [6, 14]", p->visited_log2);
    z->Ceff = (int64_t)p->C > n - 1 ? (int)(n - 1) : p->C;
    // the automatic band (2C plus a column tile, to a power of two) must fit the
    // largest band the kernels take, 2048 entries
    if (p->band == 0 && 2 * z->Ceff + 256 > 2048)
        return fail(CNG_EUNSUPPORTED, "C=%d exceeds 896 (pass a band of up to 2048)", p->C);
    z->W = p->R + p->extra;
    z->Lc = p->Lc > 0 ? p->Lc : z->Ceff;
    if (z->Lc > MAX_LEFF) return fail(CNG_EUNSUPPORTED, "Lc=%d exceeds %d", z->Lc, MAX_LEFF);
    if (p->pass_rows < 0) return fail(CNG_EINVAL, "pass_rows=%d must be >= 0", p->pass_rows);
    z->graph = (p->flags & CNG_BUILD_GRAPH_CANDIDATES) != 0;
    z->gK = p->knn_K > 0 ? p->knn_K : 32;
    z->gRounds = p->knn_rounds > 0 ? p->knn_rounds : 12;
    z->gL = p->cand_L > 0 ? p->cand_L : z->Ceff;
    if (z->graph) {
        if (p->knn_K < 0 || z->gK > 64) return fail(CNG_EUNSUPPORTED, "knn_K=%d must be in [0, 64]", p->knn_K);
        if ((int64_t)z->gK > n - 1) z->gK = (int)(n - 1);
        if (p->knn_rounds < 0 || p->cand_L < 0) return fail(CNG_EINVAL, "knn_rounds and cand_L must be >= 0");
        if (z->Ceff + 1 + z->gK > 256) return fail(CNG_EUNSUPPORTED, "C + 1 + knn_K exceeds 256");
        if ((z->gL > z->Ceff + 1 ? z->gL : z->Ceff + 1) > MAX_LEFF) return fail(CNG_EUNSUPPORTED, "cand_L exceeds %d", MAX_LEFF);
    }
    z->cand_ids = align256((size_t)n * z->Ceff * 4);
    z->cand_D = align256((size_t)n * z->Ceff * 4);
    z->entry = align256(cng::entry_workspace_bytes(n, d));
    z->connect = align256(cng::connect_workspace_bytes(n, z->W, z->Lc));
    z->backward = (p->flags & CNG_BUILD_BACKWARD) ? align256(cng::backward_workspace_bytes(n, z->W)) : 0;
    size_t scratch = z->entry;
    if (z->graph) {
        z->knn = cng::KnnPlan{};
        z->g0 = align256((size_t)n * z->gK * 4) * 2;  // the K-NN graph: ids and D
        const size_t a = align256(cng::nndescent_workspace_bytes(n, z->gK));
        const size_t b = align256(cng::graph_candidates_workspace_bytes(n, z->Ceff));
        if (a > scratch) scratch = a;
        if (b > scratch) scratch = b;
    } else {
        z->knn = cng::knn_plan(n, n, d, z->Ceff, p->band, p->pass_rows);
        z->g0 = 0;
        if (z->knn.bytes > scratch) scratch = z->knn.bytes;
    }
    if (z->connect > scratch) scratch = z->connect;
    if (z->backward > scratch) scratch = z->backward;
    z->total = z->cand_ids + z->cand_D + z->g0 + align256(scratch);
    return CNG_OK;
}

}  // namespace

extern "C" {

const char *cng_last_error(void) { return g_err.c_str(); }

const char *cng_version(void) { return "cng-gfx950 0.1"; }

cng_status cng_build_workspace_size(int64_t n, int32_t d, const cng_build_params *p, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    BuildSizes z;
    cng_status s = build_sizes(n, d, p, &z);
    if (s != CNG_OK) return s;
    *bytes = z.total;
    return ok();
}

cng_status cng_build(const float *points, int64_t n, int32_t d, const cng_build_params *p,
                     uint32_t *adj, uint32_t *entry, void *workspace, size_t ws_bytes, void *stream,
                     cng_build_stats *stats)
{
    BuildSizes z;
    cng_status s = check_points(points, n, d, 2);
    if (s != CNG_OK) return s;
    s = build_sizes(n, d, p, &z);
    if (s != CNG_OK) return s;
    if (!adj || !entry) return fail(CNG_EINVAL, "adj/entry is NULL");
    if (!workspace || ws_bytes < z.total)
        return fail(CNG_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, z.total);
    hipStream_t st = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)workspace;
    uint32_t *cand = (uint32_t *)w;
    float *candD = (float *)(w + z.cand_ids);
    uint32_t *g0 = (uint32_t *)(w + z.cand_ids + z.cand_D);
    float *g0D = (float *)(w + z.cand_ids + z.cand_D + z.g0 / 2);
    void *scratch = w + z.cand_ids + z.cand_D + z.g0;
    cng_build_stats local{};
    cng_build_stats *S = stats ? stats : &local;
    std::memset(S, 0, sizeof *S);
    hipError_t e;
    const double t0 = now_ms();

    e = cng::launch_entry(points, n, d, entry, scratch, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "entry point");
    uint32_t entry_h = 0;
    e = hipMemcpyAsync(&entry_h, entry, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "entry point");
    const double t1 = now_ms();

    int64_t ovf = 0;
    int exact = 0, dtype = 0;
    double tg = t1;
    int rounds_run = 0;
    if (z.graph) {
        // phases 1-2: NN-descent graph, then each point's candidates from a
        // beam search on it
        e = cng::run_nndescent(points, n, d, z.gK, p->knn_seed, z.gRounds, g0, g0D, scratch, st,
                               &rounds_run);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "nn-descent");
        tg = now_ms();
        e = cng::run_graph_candidates(points, n, d, g0, g0D, z.gK, entry_h, z.gL, z.Ceff, cand,
                                      candD, scratch, st);
        if (e != hipSuccess) return hip_fail(e, "graph candidates");
        dtype = -1;
    } else {
        e = cng::launch_knn(points, n, points, n, d, z.Ceff, 1, z.knn, cand, candD, scratch, st, &ovf,
                            &exact, &dtype);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "candidates");
    }
    const double t2 = now_ms();

    e = cng::launch_prune(points, n, d, cand, candD, z.Ceff, p->R, z.W, p->alpha, p->tau, adj, st, 0,
                          p->alpha_max, p->alpha_step);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "prune");
    const double t3 = now_ms();

    // phase 3: the candidate arrays (n x Ceff) are free again and hold the
    // candidate sets of the backward-edge phase
    if (p->flags & CNG_BUILD_BACKWARD) {
        e = cng::run_backward(points, n, d, adj, z.W, p->R, z.Ceff, p->alpha, p->alpha_max,
                              p->alpha_step, p->tau, cand, candD, scratch, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "backward edges");
    }
    const double t3b = now_ms();

    int64_t rounds = 0, added = 0;
    if (p->flags & CNG_BUILD_CONNECT) {
        int cap = 0;
        const int vl = p->visited_log2;  // 0: chosen per round by the batch size
        e = cng::run_connect(points, n, d, adj, z.W, entry_h, z.Lc, vl, scratch, st, &rounds, &added, &cap);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "connect");
        if (cap) return fail(CNG_ECAPACITY, "connectivity: no reachable row has a free slot");
    }
    const double t4 = now_ms();
    S->ms_entry = t1 - t0;
    S->ms_candidates = t2 - t1;
    S->ms_prune = t3 - t2;
    S->ms_backward = t3b - t3;
    S->ms_connect = t4 - t3b;
    S->ms_total = t4 - t0;
    S->connect_rounds = rounds;
    S->connect_added = added;
    S->overflow_rows = ovf;
    S->exact_integer = exact;
    S->filter_dtype = dtype;
    S->ms_knn_graph = z.graph ? tg - t1 : 0.0;
    S->knn_rounds_run = rounds_run;
    return ok();
}

cng_status cng_nndescent_workspace_size(int64_t n, int32_t K, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (n < 1 || n > MAX_N) return fail(CNG_EINVAL, "n out of range");
    if (K < 1 || K > 64) return fail(CNG_EUNSUPPORTED, "K=%d must be in [1, 64]", K);
    *bytes = cng::nndescent_workspace_bytes(n, K);
    return ok();
}

cng_status cng_nndescent(const float *points, int64_t n, int32_t d, int32_t K, uint64_t seed,
                         int32_t rounds, uint32_t *ids, float *D, void *workspace, size_t ws_bytes,
                         void *stream, int32_t *rounds_host)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    size_t need = 0;
    s = cng_nndescent_workspace_size(n, K, &need);
    if (s != CNG_OK) return s;
    if (rounds < 0) return fail(CNG_EINVAL, "rounds must be >= 0");
    if (!ids || !D) return fail(CNG_EINVAL, "NULL array argument");
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    int rr = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = cng::run_nndescent(points, n, d, K, seed, rounds, ids, D, workspace, st, &rr);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "nn-descent");
    if (rounds_host) *rounds_host = rr;
    return ok();
}

cng_status cng_graph_candidates_workspace_size(int64_t n, int32_t C, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (n < 1 || n > MAX_N || C < 1) return fail(CNG_EINVAL, "n or C out of range");
    *bytes = cng::graph_candidates_workspace_bytes(n, C);
    return ok();
}

cng_status cng_graph_candidates(const float *points, int64_t n, int32_t d, const uint32_t *g0,
                                const float *g0D, int32_t K, uint32_t entry, int32_t L, int32_t C,
                                uint32_t *cand, float *candD, void *workspace, size_t ws_bytes,
                                void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    size_t need = 0;
    s = cng_graph_candidates_workspace_size(n, C, &need);
    if (s != CNG_OK) return s;
    if (K < 1 || K > MAX_W) return fail(CNG_EINVAL, "K out of range");
    if (L < 1) return fail(CNG_EINVAL, "L must be >= 1");
    if (C + 1 + K > 256) return fail(CNG_EUNSUPPORTED, "C + 1 + K exceeds 256");
    if ((L > C + 1 ? L : C + 1) > MAX_LEFF) return fail(CNG_EUNSUPPORTED, "max(L, C + 1) exceeds %d", MAX_LEFF);
    if ((int64_t)entry >= n) return fail(CNG_EINVAL, "entry %u >= n", entry);
    if (!g0 || !g0D || !cand || !candD) return fail(CNG_EINVAL, "NULL array argument");
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::run_graph_candidates(points, n, d, g0, g0D, K, entry, L, C, cand, candD,
                                             workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph candidates");
    return ok();
}

size_t cng_entry_workspace_size(int64_t n, int32_t d)
{
    if (n < 1 || d < 1) return 0;
    return cng::entry_workspace_bytes(n, d);
}

cng_status cng_entry_point(const float *points, int64_t n, int32_t d, uint32_t *entry,
                           void *workspace, size_t ws_bytes, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (!entry) return fail(CNG_EINVAL, "entry is NULL");
    if (!workspace || ws_bytes < cng::entry_workspace_bytes(n, d))
        return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::launch_entry(points, n, d, entry, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "entry point");
    return ok();
}

cng_status cng_knn_workspace_size(int64_t nr, int64_t nc, int32_t d, int32_t C, int32_t band,
                                  int64_t pass_rows, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (nr < 0 || nr > MAX_N || nc < 1 || nc > MAX_N) return fail(CNG_EINVAL, "nr/nc out of range");
    if (d < 1 || d > 4096) return fail(CNG_EINVAL, "d out of range");
    if (C < 1) return fail(CNG_EINVAL, "C must be >= 1");
    if (band < 0 || band > 2048) return fail(CNG_EUNSUPPORTED, "band must be in [0, 2048]");
    if (pass_rows < 0) return fail(CNG_EINVAL, "pass_rows must be >= 0");
    int Ce = C;
    if (band == 0 && 2 * Ce + 256 > 2048) return fail(CNG_EUNSUPPORTED, "C=%d exceeds 896 (pass a band of up to 2048)", C);
    *bytes = cng::knn_plan(nr, nc, d, Ce, band, pass_rows).bytes;
    return ok();
}

cng_status cng_knn(const float *rows, int64_t nr, const float *cols, int64_t nc, int32_t d, int32_t C,
                   int32_t exclude_self, int32_t band, int64_t pass_rows, uint32_t *ids, float *D,
                   void *workspace, size_t ws_bytes, void *stream, int64_t *overflow_rows_host)
{
    size_t need = 0;
    cng_status s = cng_knn_workspace_size(nr, nc, d, C, band, pass_rows, &need);
    if (s != CNG_OK) return s;
    if (!rows || !cols || !ids || !D) return fail(CNG_EINVAL, "NULL array argument");
    if (exclude_self && (rows != cols || nr != nc)) return fail(CNG_EINVAL, "exclude_self needs rows == cols");
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    if (nr == 0) return ok();
    cng::KnnPlan plan = cng::knn_plan(nr, nc, d, C, band, pass_rows);
    int64_t ovf = 0;
    int exact = 0, dtype = 0;
    hipError_t e = cng::launch_knn(rows, nr, cols, nc, d, C, exclude_self ? 1 : 0, plan, ids, D,
                                   workspace, (hipStream_t)stream, &ovf, &exact, &dtype);
    if (e != hipSuccess) return hip_fail(e, "knn");
    if (overflow_rows_host) *overflow_rows_host = ovf;
    return ok();
}

cng_status cng_prune(const float *points, int64_t n, int32_t d, const uint32_t *cand,
                     const float *candD, int32_t C, int32_t R, int32_t W, double alpha, double tau,
                     uint32_t *adj, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (!cand || !candD || !adj) return fail(CNG_EINVAL, "NULL array argument");
    if (C < 1 || R < 1 || W < R) return fail(CNG_EINVAL, "need C >= 1, R >= 1, W >= R");
    if (W > MAX_W) return fail(CNG_EUNSUPPORTED, "W=%d exceeds %d", W, MAX_W);
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(CNG_EINVAL, "alpha must be finite and > 0");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(CNG_EINVAL, "tau must be finite and >= 0");
    hipError_t e = cng::launch_prune(points, n, d, cand, candD, C, R, W, alpha, tau, adj, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "prune");
    return ok();
}

cng_status cng_backward_workspace_size(int64_t n, int32_t W, int32_t Cb, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (n < 1 || n > MAX_N || W < 1 || W > MAX_W) return fail(CNG_EINVAL, "n/W out of range");
    if (Cb < 1 || Cb > 448) return fail(CNG_EUNSUPPORTED, "Cb=%d must be in [1, 448]", Cb);
    *bytes = align256((size_t)n * Cb * 4) * 2 + cng::backward_workspace_bytes(n, W);
    return ok();
}

cng_status cng_backward(const float *points, int64_t n, int32_t d, uint32_t *adj, int32_t W,
                        int32_t R, int32_t Cb, double alpha, double alpha_max, double alpha_step,
                        double tau, void *workspace, size_t ws_bytes, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    size_t need = 0;
    s = cng_backward_workspace_size(n, W, Cb, &need);
    if (s != CNG_OK) return s;
    if (!adj) return fail(CNG_EINVAL, "adj is NULL");
    if (R < 1 || R > W) return fail(CNG_EINVAL, "need 1 <= R <= W");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(CNG_EINVAL, "alpha must be finite and > 0");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(CNG_EINVAL, "tau must be finite and >= 0");
    s = check_adaptive(alpha, alpha_max, alpha_step);
    if (s != CNG_OK) return s;
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    unsigned char *w = (unsigned char *)workspace;
    uint32_t *cand = (uint32_t *)w;
    float *candD = (float *)(w + align256((size_t)n * Cb * 4));
    void *rest = w + align256((size_t)n * Cb * 4) * 2;
    hipError_t e = cng::run_backward(points, n, d, adj, W, R, Cb, alpha, alpha_max, alpha_step, tau,
                                     cand, candD, rest, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "backward edges");
    return ok();
}

cng_status cng_prune_adaptive(const float *points, int64_t n, int32_t d, const uint32_t *cand,
                              const float *candD, int32_t C, int32_t R, int32_t W, double alpha0,
                              double alpha_max, double alpha_step, double tau, uint32_t *adj,
                              void *stream)
{
    if (!(alpha_step > 0.0)) return fail(CNG_EINVAL, "alpha_step must be > 0");
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (!cand || !candD || !adj) return fail(CNG_EINVAL, "NULL array argument");
    if (C < 1 || R < 1 || W < R) return fail(CNG_EINVAL, "need C >= 1, R >= 1, W >= R");
    if (W > MAX_W) return fail(CNG_EUNSUPPORTED, "W=%d exceeds %d", W, MAX_W);
    if (!(alpha0 > 0.0) || !std::isfinite(alpha0)) return fail(CNG_EINVAL, "alpha0 must be finite and > 0");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(CNG_EINVAL, "tau must be finite and >= 0");
    s = check_adaptive(alpha0, alpha_max, alpha_step);
    if (s != CNG_OK) return s;
    hipError_t e = cng::launch_prune(points, n, d, cand, candD, C, R, W, alpha0, tau, adj,
                                     (hipStream_t)stream, 0, alpha_max, alpha_step);
    if (e != hipSuccess) return hip_fail(e, "prune");
    return ok();
}

cng_status cng_connect_workspace_size(int64_t n, int32_t W, int32_t Lc, size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (n < 1 || n > MAX_N || W < 1 || W > MAX_W || Lc < 1 || Lc > MAX_LEFF)
        return fail(CNG_EINVAL, "n/W/Lc out of range");
    *bytes = cng::connect_workspace_bytes(n, W, Lc);
    return ok();
}

cng_status cng_connect(const float *points, int64_t n, int32_t d, uint32_t *adj, int32_t W,
                       uint32_t entry, int32_t Lc, int32_t visited_log2, void *workspace,
                       size_t ws_bytes, void *stream, int64_t *rounds_host, int64_t *added_host)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    size_t need = 0;
    s = cng_connect_workspace_size(n, W, Lc, &need);
    if (s != CNG_OK) return s;
    if (!adj) return fail(CNG_EINVAL, "adj is NULL");
    if ((int64_t)entry >= n) return fail(CNG_EINVAL, "entry %u >= n", entry);
    if (visited_log2 != 0 && (visited_log2 < 6 || visited_log2 > 14)) return fail(CNG_EINVAL, "visited_log2 out of range");
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    int64_t rounds = 0, added = 0;
    int cap = 0;
    const int vl = visited_log2;  // 0: chosen per round by the batch size
    hipError_t e = cng::run_connect(points, n, d, adj, W, entry, Lc, vl, workspace, st, &rounds, &added, &cap);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "connect");
    if (rounds_host) *rounds_host = rounds;
    if (added_host) *added_host = added;
    if (cap) return fail(CNG_ECAPACITY, "connectivity: no reachable row has a free slot");
    return ok();
}

static cng_status search_impl(const float *points, const void *vecs, int32_t dtype,
                              const float *scales, int64_t n, int32_t d, const uint32_t *adj,
                              int32_t W, const float *queries, int64_t nq, int32_t k, int32_t L,
                              const uint32_t *entries, int64_t n_entries, uint32_t *ids,
                              float *dists, uint32_t *hops, uint32_t *ndc, int32_t visited_log2,
                              void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (dtype < 0 || dtype > 2) return fail(CNG_EINVAL, "dtype=%d must be 0, 1 or 2", dtype);
    if (!vecs) return fail(CNG_EINVAL, "vecs is NULL");
    if (dtype == 2 && !scales) return fail(CNG_EINVAL, "fp8 storage needs scales");
    if (s != CNG_OK) return s;
    if (W < 1) return fail(CNG_EINVAL, "W=%d must be >= 1", W);
    if (W > MAX_W) return fail(CNG_EUNSUPPORTED, "W=%d exceeds %d", W, MAX_W);
    if (nq < 0 || nq > MAX_N) return fail(CNG_EINVAL, "nq out of range");
    if (k < 1 || L < 1) return fail(CNG_EINVAL, "k and L must be >= 1");
    const int Leff = L > k ? L : k;
    if (Leff > MAX_LEFF) return fail(CNG_EUNSUPPORTED, "max(L, k)=%d exceeds %d", Leff, MAX_LEFF);
    if (n_entries != 1 && n_entries != nq) return fail(CNG_EINVAL, "n_entries must be 1 or nq");
    if (visited_log2 != 0 && (visited_log2 < 6 || visited_log2 > 14)) return fail(CNG_EINVAL, "visited_log2 out of range");
    if (nq == 0) return ok();
    if (!adj || !queries || !entries || !ids || !dists) return fail(CNG_EINVAL, "NULL array argument");
    cng::SearchArgs a{};
    a.points = points;
    a.vecs = vecs;
    a.scales = scales;
    a.store = dtype;
    a.n = n;
    a.d = d;
    a.adj = adj;
    a.W = W;
    a.queries = queries;
    a.query_ids = nullptr;
    a.nq = nq;
    a.k = k;
    a.Leff = Leff;
    a.entries = entries;
    a.per_query_entry = n_entries == nq && nq > 1 ? 1 : (n_entries == 1 ? 0 : 1);
    a.ids = ids;
    a.dists = dists;
    a.hops = hops;
    a.ndc = ndc;
    a.vlog2 = visited_log2 ? visited_log2 : cng::search_default_vlog2(Leff, nq, a.store);
    hipError_t e = cng::launch_search(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "search");
    return ok();
}

cng_status cng_search(const float *points, int64_t n, int32_t d, const uint32_t *adj, int32_t W,
                      const float *queries, int64_t nq, int32_t k, int32_t L,
                      const uint32_t *entries, int64_t n_entries, uint32_t *ids, float *dists,
                      uint32_t *hops, uint32_t *ndc, int32_t visited_log2, void *stream)
{
    return search_impl(points, points, 0, nullptr, n, d, adj, W, queries, nq, k, L, entries,
                       n_entries, ids, dists, hops, ndc, visited_log2, stream);
}

cng_status cng_search_quantized(const float *points, const void *vecs, int32_t dtype,
                                const float *scales, int64_t n, int32_t d, const uint32_t *adj,
                                int32_t W, const float *queries, int64_t nq, int32_t k, int32_t L,
                                const uint32_t *entries, int64_t n_entries, uint32_t *ids,
                                float *dists, uint32_t *hops, uint32_t *ndc, int32_t visited_log2,
                                void *stream)
{
    return search_impl(points, vecs, dtype, scales, n, d, adj, W, queries, nq, k, L, entries,
                       n_entries, ids, dists, hops, ndc, visited_log2, stream);
}

size_t cng_quantized_bytes(int64_t n, int32_t d, int32_t dtype)
{
    if (n < 0 || d < 1 || dtype < 0 || dtype > 2) return 0;
    return cng::quantized_bytes(n, d, dtype);
}

cng_status cng_quantize(const float *points, int64_t n, int32_t d, int32_t dtype, void *vecs,
                        float *scales, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (dtype != 1 && dtype != 2) return fail(CNG_EINVAL, "dtype=%d must be 1 (bf16) or 2 (fp8)", dtype);
    if (!vecs || (dtype == 2 && !scales)) return fail(CNG_EINVAL, "NULL output");
    hipError_t e = cng::launch_quantize(points, n, d, dtype, vecs, scales, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "quantize");
    return ok();
}

// ---------------------------------------------------------------- learned entry point

size_t cng_kmeans_workspace_size(int64_t n, int32_t d, int32_t K)
{
    if (n < 1 || d < 1 || K < 1) return 0;
    return cng::kmeans_workspace_bytes(n, d, K);
}

cng_status cng_kmeans(const float *points, int64_t n, int32_t d, int32_t K, int32_t iters,
                      const uint32_t *init_ids, float *centers, uint32_t *entries, void *workspace,
                      size_t ws_bytes, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    if (K < 1 || K > n) return fail(CNG_EINVAL, "K=%d must be in [1, n]", K);
    if (iters < 0) return fail(CNG_EINVAL, "iters must be >= 0");
    if (!init_ids || !centers || !entries) return fail(CNG_EINVAL, "NULL array argument");
    if (!workspace || ws_bytes < cng::kmeans_workspace_bytes(n, d, K))
        return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::run_kmeans(points, n, d, K, iters, init_ids, centers, entries, workspace,
                                   (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "kmeans");
    return ok();
}

static cng_status check_mlp(int32_t d, int32_t H, int32_t K, int32_t B, int32_t precision)
{
    if (d < 1 || d > 4096 || H < 1 || H > 8192 || K < 1 || K > 65536)
        return fail(CNG_EINVAL, "MLP shape d=%d H=%d K=%d out of range", d, H, K);
    if (B < 1) return fail(CNG_EINVAL, "batch B=%d must be >= 1", B);
    if (precision != 0 && precision != 1) return fail(CNG_EINVAL, "precision must be 0 (fp32) or 1 (bf16)");
    return CNG_OK;
}

int64_t cng_mlp_param_count(int32_t d, int32_t H, int32_t K)
{
    if (d < 1 || H < 1 || K < 1) return 0;
    return cng::MlpShape(d, H, K).total;
}

size_t cng_mlp_workspace_size(int32_t d, int32_t H, int32_t K, int32_t B)
{
    if (d < 1 || H < 1 || K < 1 || B < 1) return 0;
    return cng::mlp_workspace_floats(cng::MlpShape(d, H, K), B) * 4;
}

static cng_status check_affine(const float *x_mean, const float *x_scale)
{
    if ((x_mean == nullptr) != (x_scale == nullptr))
        return fail(CNG_EINVAL, "x_mean and x_scale must both be given or both be NULL");
    return CNG_OK;
}

size_t cng_mlp_input_stats_workspace_size(int64_t n, int32_t d)
{
    if (n < 1 || d < 1) return 0;
    return cng::mlp_stats_workspace_bytes(n, d);
}

cng_status cng_mlp_input_stats(const float *X, int64_t n, int32_t d, float *x_mean, float *x_scale,
                               void *workspace, size_t ws_bytes, void *stream)
{
    cng_status s = check_points(X, n, d, 1);
    if (s != CNG_OK) return s;
    if (!x_mean || !x_scale) return fail(CNG_EINVAL, "NULL array argument");
    if (!workspace || ws_bytes < cng::mlp_stats_workspace_bytes(n, d)) return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::mlp_input_stats(X, n, d, x_mean, x_scale, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp input stats");
    return ok();
}

cng_status cng_mlp_gradients(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                             const float *x_mean, const float *x_scale, const uint32_t *labels,
                             const uint32_t *batch_ids, int32_t B, int32_t precision, float *grads,
                             float *loss, void *workspace, size_t ws_bytes, void *stream)
{
    cng_status s = check_mlp(d, H, K, B, precision);
    if (s != CNG_OK) return s;
    s = check_affine(x_mean, x_scale);
    if (s != CNG_OK) return s;
    if (!params || !X || !labels || !grads) return fail(CNG_EINVAL, "NULL array argument");
    cng::MlpShape sh(d, H, K);
    if (!workspace || ws_bytes < cng::mlp_workspace_floats(sh, B) * 4) return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::mlp_gradients(sh, params, X, labels, batch_ids, B, precision == 1,
                                      (float *)workspace, grads, loss, (hipStream_t)stream, x_mean,
                                      x_scale);
    if (e != hipSuccess) return hip_fail(e, "mlp gradients");
    return ok();
}

cng_status cng_mlp_adam(float *params, const float *grads, float *m1, float *m2, int32_t d,
                        int32_t H, int32_t K, int32_t step, float lr, float beta1, float beta2,
                        float eps, void *stream)
{
    cng_status s = check_mlp(d, H, K, 1, 0);
    if (s != CNG_OK) return s;
    if (!params || !grads || !m1 || !m2) return fail(CNG_EINVAL, "NULL array argument");
    if (step < 1) return fail(CNG_EINVAL, "step must be >= 1");
    hipError_t e = cng::mlp_adam(cng::MlpShape(d, H, K), params, grads, m1, m2, step, lr, beta1,
                                 beta2, eps, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp adam");
    return ok();
}

cng_status cng_mlp_logits(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                          const float *x_mean, const float *x_scale, int32_t B, int32_t precision,
                          float *logits, float *hidden, void *workspace, size_t ws_bytes,
                          void *stream)
{
    cng_status s = check_mlp(d, H, K, B, precision);
    if (s != CNG_OK) return s;
    s = check_affine(x_mean, x_scale);
    if (s != CNG_OK) return s;
    if (!params || !X || !logits) return fail(CNG_EINVAL, "NULL array argument");
    cng::MlpShape sh(d, H, K);
    if (!workspace || ws_bytes < cng::mlp_workspace_floats(sh, B) * 4) return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::mlp_scores(sh, params, X, B, precision == 1, (float *)workspace, logits,
                                   (hipStream_t)stream, x_mean, x_scale, hidden);
    if (e != hipSuccess) return hip_fail(e, "mlp logits");
    return ok();
}

cng_status cng_entry_predict(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                             const float *x_mean, const float *x_scale, int32_t B, int32_t precision,
                             const uint32_t *entries, uint32_t fallback, float theta,
                             uint32_t *out_entry, float *out_conf, void *workspace, size_t ws_bytes,
                             void *stream)
{
    cng_status s = check_mlp(d, H, K, B, precision);
    if (s != CNG_OK) return s;
    s = check_affine(x_mean, x_scale);
    if (s != CNG_OK) return s;
    if (!params || !X || !entries || !out_entry) return fail(CNG_EINVAL, "NULL array argument");
    cng::MlpShape sh(d, H, K);
    if (!workspace || ws_bytes < cng::mlp_workspace_floats(sh, B) * 4) return fail(CNG_ENOMEM, "workspace too small");
    hipError_t e = cng::mlp_predict(sh, params, X, B, precision == 1, entries, fallback, theta,
                                    (float *)workspace, out_entry, out_conf, (hipStream_t)stream,
                                    x_mean, x_scale);
    if (e != hipSuccess) return hip_fail(e, "entry predict");
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free prediction
// A fixed device array holds the scratch memory of cng_entry_predict_noalloc.
// In host code `scratch` only names the symbol: its device address, one per
// GPU, comes from hipGetSymbolAddress on the first call on that device (with
// that device current) and is kept in scratch_ptr.
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static cng_status device_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(CNG_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return CNG_OK;
}

extern "C" {

size_t cng_entry_predict_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

cng_status cng_entry_predict_noalloc(const float *params, int32_t d, int32_t H, int32_t K,
                                     const float *X, const float *x_mean, const float *x_scale,
                                     int32_t B, int32_t precision, const uint32_t *entries,
                                     uint32_t fallback, float theta, uint32_t *out_entry,
                                     float *out_conf, void *stream)
{
    cng_status s = check_mlp(d, H, K, B, precision);
    if (s != CNG_OK) return s;
    s = check_affine(x_mean, x_scale);
    if (s != CNG_OK) return s;
    if (!params || !X || !entries || !out_entry) return fail(CNG_EINVAL, "NULL array argument");
    cng::MlpShape sh(d, H, K);
    const size_t need = cng::mlp_workspace_floats(sh, B) * 4;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(CNG_EUNSUPPORTED, "scratch of %zu bytes needed, the static array holds %zu", need,
                    NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    s = device_scratch(&ws);
    if (s != CNG_OK) return s;
    hipError_t e = cng::mlp_predict(sh, params, X, B, precision == 1, entries, fallback, theta,
                                    (float *)ws, out_entry, out_conf, (hipStream_t)stream, x_mean,
                                    x_scale);
    if (e != hipSuccess) return hip_fail(e, "entry predict (no allocation)");
    return ok();
}

cng_status cng_entry_labels_workspace_size(int64_t n, int32_t d, int64_t nq, int32_t K,
                                           size_t *bytes)
{
    if (!bytes) return fail(CNG_EINVAL, "bytes is NULL");
    if (n < 1 || d < 1 || nq < 0 || K < 1) return fail(CNG_EINVAL, "sizes out of range");
    cng::KnnPlan p = cng::knn_plan(nq, K, d, 1, 0);
    *bytes = align256(p.bytes) + align256((size_t)nq * d * 4) + align256((size_t)K * d * 4) +
             align256((size_t)nq * 4) * 3;
    return ok();
}

cng_status cng_entry_labels(const float *points, int64_t n, int32_t d, const uint32_t *adj, int32_t W,
                            uint32_t nav, const float *queries, int64_t nq, int32_t L,
                            const uint32_t *entries, int32_t K, uint32_t *labels, void *workspace,
                            size_t ws_bytes, void *stream)
{
    cng_status s = check_points(points, n, d, 1);
    if (s != CNG_OK) return s;
    size_t need = 0;
    s = cng_entry_labels_workspace_size(n, d, nq, K, &need);
    if (s != CNG_OK) return s;
    if (!adj || !queries || !entries || !labels) return fail(CNG_EINVAL, "NULL array argument");
    if ((int64_t)nav >= n) return fail(CNG_EINVAL, "navigating node %u >= n", nav);
    if (L < 1 || L > MAX_LEFF) return fail(CNG_EUNSUPPORTED, "L out of range");
    if (W < 1 || W > MAX_W) return fail(CNG_EUNSUPPORTED, "W out of range");
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace too small");
    if (nq == 0) return ok();
    hipStream_t st = (hipStream_t)stream;
    cng::KnnPlan p = cng::knn_plan(nq, K, d, 1, 0);
    unsigned char *w = (unsigned char *)workspace;
    void *kws = w;
    w += align256(p.bytes);
    float *found = (float *)w;
    w += align256((size_t)nq * d * 4);
    float *evec = (float *)w;
    w += align256((size_t)K * d * 4);
    uint32_t *top = (uint32_t *)w;
    w += align256((size_t)nq * 4);
    float *topd = (float *)w;
    w += align256((size_t)nq * 4);
    uint32_t *nav_dev = (uint32_t *)w;
    hipError_t e = hipMemcpyAsync(nav_dev, &nav, 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "labels");
    // 1. plain float32 search from the navigating node: the best point found
    cng::SearchArgs a{};
    a.points = points; a.vecs = points; a.scales = nullptr; a.store = 0;
    a.n = n; a.d = d; a.adj = adj; a.W = W; a.queries = queries; a.query_ids = nullptr; a.nq = nq;
    a.k = 1; a.Leff = L; a.entries = nav_dev; a.per_query_entry = 0;
    a.ids = top; a.dists = topd; a.hops = nullptr; a.ndc = nullptr;
    a.vlog2 = cng::search_default_vlog2(L, nq, 0);
    e = cng::launch_search(a, st);
    // 2. label = entry node nearest to that point, by (D, index)
    if (e == hipSuccess) e = cng::gather_points(points, d, top, nq, found, st);
    if (e == hipSuccess) e = cng::gather_points(points, d, entries, K, evec, st);
    if (e == hipSuccess)
        e = cng::launch_knn(found, nq, evec, K, d, 1, 0, p, labels, topd, kws, st, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "labels");
    return ok();
}

cng_status cng_nearest_centre_entry(const float *queries, int64_t nq, int32_t d, const float *centers,
                                    int32_t K, const uint32_t *entries, uint32_t *out_entry,
                                    void *workspace, size_t ws_bytes, void *stream)
{
    if (nq < 0 || d < 1 || K < 1) return fail(CNG_EINVAL, "sizes out of range");
    if (!queries || !centers || !entries || !out_entry) return fail(CNG_EINVAL, "NULL array argument");
    cng::KnnPlan p = cng::knn_plan(nq, K, d, 1, 0);
    const size_t need = align256(p.bytes) + align256((size_t)nq * 4) * 2;
    if (!workspace || ws_bytes < need) return fail(CNG_ENOMEM, "workspace of %zu bytes < %zu", ws_bytes, need);
    if (nq == 0) return ok();
    hipStream_t st = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)workspace;
    uint32_t *j = (uint32_t *)(w + align256(p.bytes));
    float *jd = (float *)(w + align256(p.bytes) + align256((size_t)nq * 4));
    hipError_t e = cng::launch_knn(queries, nq, centers, K, d, 1, 0, p, j, jd, w, st, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = cng::map_through(j, nq, entries, out_entry, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "nearest centre");
    return ok();
}

size_t cng_nearest_centre_workspace_size(int64_t nq, int32_t d, int32_t K)
{
    if (nq < 0 || d < 1 || K < 1) return 0;
    cng::KnnPlan p = cng::knn_plan(nq, K, d, 1, 0);
    return align256(p.bytes) + align256((size_t)nq * 4) * 2;
}

}  // extern "C"
