// Internal launch interfaces of the gfx950 kernels (host side of libcng).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cng {

struct SearchArgs {
    const float *points;       // float32 vectors (queries by id, final re-rank)
    const void *vecs;          // stored vectors that are scored (== points for float32)
    const float *scales;       // fp8 per-vector scales (store 2)
    int store;                 // 0 float32, 1 bf16, 2 fp8-E4M3
    int64_t n;
    int d;
    const uint32_t *adj;
    int W;
    const float *queries;      // [nq x d], or nullptr when query_ids is set
    const uint32_t *query_ids; // optional: query i is points[query_ids[i]]
    int64_t nq;
    int k, Leff;
    const uint32_t *entries;
    int per_query_entry;
    uint32_t *ids;
    float *dists;
    uint32_t *hops, *ndc;
    int vlog2;
    int out_sq;                // dists receive the squared distances D instead of sqrt(D)
};

hipError_t launch_search(const SearchArgs &a, hipStream_t stream);

// serving loop (persistent kernel; ring and results in coherent pinned host memory)
struct ServeRing {
    uint64_t tail;  // items published by the host
    uint64_t stop;  // non-zero: leave the loop
    uint64_t pad[6];
};
struct ServeItem {   // read by the device as eight uint32 words
    uint32_t tag_lo, tag_hi;  // the item number t this position holds
    uint32_t k, L;            // results wanted and beam width
    uint32_t entry;           // entry point of the search
    uint32_t qoff;            // query vector: arena word offset (d floats)
    uint32_t ioff, doff;      // result ids / distances: arena word offsets (k each)
};
struct ServeArgs {
    SearchArgs base;            // graph, vectors, storage, visited table size
    ServeRing *ring;
    const ServeItem *items;     // [rc] ring of item descriptors, item t at t % rc
    uint64_t rc;
    unsigned char *arena;       // query vectors and results of the requests in flight
    uint64_t *done;             // [rc]: t + 1 once item t is complete
    unsigned long long *head;   // device memory: next item to claim
    uint64_t *mirror;           // device memory: [0] last tail seen, [1] stop seen
    uint32_t max_k;
    uint32_t idle_limit;
};
// head = first item to claim, mirror = {seen, 0}: before a (re)launch
hipError_t launch_serve_reset(unsigned long long *head, uint64_t *mirror, uint64_t first,
                              uint64_t seen, hipStream_t stream);
hipError_t launch_serve(const ServeArgs &a, int waves, hipStream_t stream);
size_t serve_lds_per_wave(int d, int vlog2);
int search_default_vlog2(int Leff, int64_t nq, int store);
size_t search_lds_per_wave(int Leff, int vlog2);

// reduced-precision storage
size_t quantized_bytes(int64_t n, int d, int dtype);
hipError_t launch_quantize(const float *x, int64_t n, int d, int dtype, void *out, float *scales,
                           hipStream_t stream);

// entry point (centroid rule)
size_t entry_workspace_bytes(int64_t n, int d);
hipError_t launch_entry(const float *points, int64_t n, int d, uint32_t *entry, void *ws,
                        hipStream_t stream);

// exact candidates
struct KnnPlan {
    int64_t chunk_rows;   // rows per pass
    int band;             // per-row band capacity
    size_t bytes;         // workspace bytes
    // self-joins: cells of the locality order (0: none) and the plan of the
    // cell assignment (a candidate search with C = 1 against the cell samples)
    int order_K;
    int64_t inner_chunk;
    int inner_band;
    size_t inner_bytes;
};
// pass_rows > 0 caps the rows of one filter pass (rounded to whole
// workgroups); 0 sizes passes from the band memory budget
KnnPlan knn_plan(int64_t nr, int64_t nc, int d, int C, int band, int64_t pass_rows = 0);
hipError_t launch_knn(const float *rows, int64_t nr, const float *cols, int64_t nc, int d, int C,
                      int exclude_self, const KnnPlan &plan, uint32_t *ids, float *D, void *ws,
                      hipStream_t stream, int64_t *overflow_rows, int *exact_int, int *dtype);

// sub-quadratic candidates: NN-descent K-NN graph and a beam search on it
size_t nndescent_workspace_bytes(int64_t n, int K);
hipError_t run_nndescent(const float *points, int64_t n, int d, int K, uint64_t seed, int rounds,
                         uint32_t *ids, float *D, void *ws, hipStream_t st, int *rounds_run);
size_t graph_candidates_workspace_bytes(int64_t n, int C);
hipError_t run_graph_candidates(const float *points, int64_t n, int d, const uint32_t *g0,
                                const float *g0D, int K, uint32_t s_host, int L, int C,
                                uint32_t *cand, float *candD, void *ws, hipStream_t st);

// pruning; with copy_upto > 0 a list of at most copy_upto candidates becomes
// the row unpruned; alpha_step > 0: adaptive alpha (Algorithm 4) from alpha to
// alpha_max
hipError_t launch_prune(const float *points, int64_t n, int d, const uint32_t *cand,
                        const float *candD, int C, int R, int W, double alpha, double tau,
                        uint32_t *adj, hipStream_t stream, int copy_upto = 0,
                        double alpha_max = 0.0, double alpha_step = 0.0);
int adaptive_iters(double alpha0, double alpha_max, double alpha_step);

// backward edges with lazy pruning (Algorithm 3, phase 3); cand / candD hold
// n x Cb entries of scratch
size_t backward_workspace_bytes(int64_t n, int W);
hipError_t run_backward(const float *points, int64_t n, int d, uint32_t *adj, int W, int R, int Cb,
                        double alpha, double alpha_max, double alpha_step, double tau,
                        uint32_t *cand, float *candD, void *ws, hipStream_t stream);

// connectivity
size_t connect_workspace_bytes(int64_t n, int W, int Lc);
hipError_t run_connect(const float *points, int64_t n, int d, uint32_t *adj, int W,
                       uint32_t entry_host, int Lc, int vlog2, void *ws, hipStream_t stream,
                       int64_t *rounds, int64_t *added, int *capacity_error);

// learned entry point: MLP d -> H -> H -> K
struct MlpShape {
    int d, H, K;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, total;  // offsets into the parameter vector
    MlpShape(int d_, int H_, int K_);
};
size_t mlp_workspace_floats(const MlpShape &s, int B);
// mean [d] / scale [1] (device, both or neither): the network's input is
// (x - mean) / scale, applied in float32 before the first layer
hipError_t mlp_forward(const MlpShape &s, const float *P, const float *X, const uint32_t *idx, int B,
                       bool bf16, float *ws, float *Z_out, hipStream_t st,
                       const float *mean = nullptr, const float *scale = nullptr);
hipError_t mlp_gradients(const MlpShape &s, const float *P, const float *X, const uint32_t *lab,
                         const uint32_t *idx, int B, bool bf16, float *ws, float *G,
                         float *loss_mean, hipStream_t st, const float *mean = nullptr,
                         const float *scale = nullptr);
hipError_t mlp_adam(const MlpShape &s, float *P, const float *G, float *M1, float *M2, int step,
                    float lr, float b1, float b2, float eps, hipStream_t st);
hipError_t mlp_scores(const MlpShape &s, const float *P, const float *X, int B, bool bf16,
                      float *ws, float *Z, hipStream_t st, const float *mean = nullptr,
                      const float *scale = nullptr, float *hidden = nullptr);
hipError_t mlp_predict(const MlpShape &s, const float *P, const float *X, int B, bool bf16,
                       const uint32_t *entries, uint32_t fallback, float theta, float *ws,
                       uint32_t *out, float *conf, hipStream_t st, const float *mean = nullptr,
                       const float *scale = nullptr);
size_t mlp_stats_workspace_bytes(int64_t n, int d);
hipError_t mlp_input_stats(const float *X, int64_t n, int d, float *mean, float *scale, void *ws,
                           hipStream_t st);

// k-means (entry nodes of the learned entry point)
size_t kmeans_workspace_bytes(int64_t n, int d, int K);
hipError_t run_kmeans(const float *points, int64_t n, int d, int K, int iters,
                      const uint32_t *init_ids, float *centers, uint32_t *entries, void *ws,
                      hipStream_t st);

hipError_t gather_points(const float *x, int d, const uint32_t *ids, int64_t m, float *out,
                         hipStream_t st);
hipError_t map_through(const uint32_t *idx, int64_t m, const uint32_t *table, uint32_t *out,
                       hipStream_t st);

}  // namespace cng
