/*
 * cng.h -- C ABI of the MI355X (gfx950) alpha-CNG library (libcng.so).
 *
 * The library builds an alpha-convergent neighbourhood graph with a fixed alpha
 * and searches it, following Li, Yan, Lu, "Fast-Convergent Proximity Graphs
 * for Approximate Nearest Neighbor Search":
 *   - edge pruning rule: Definition 2, Eq. (1); pruning procedure: Algorithm 2;
 *   - construction framework: Algorithm 3 (entry point, candidate lists,
 *     pruning, connectivity), with exact candidate lists in place of the
 *     approximate K-NN graph and a fixed alpha (the paper's Fixed-alpha-CNG);
 *   - beam search: Algorithm 1.
 *
 * Conventions (all entry points):
 *   - Array pointers are DEVICE pointers unless the name ends in _host.  The
 *     caller owns every buffer; the library never allocates device memory.
 *     Scratch memory is passed in as `workspace` (size from *_workspace_size).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *     enqueue work and return, except where a function says it synchronises.
 *   - Vectors are row-major float32, n rows of d contiguous values.
 *   - Distances: Euclidean.  Ordering uses the squared distance D computed in
 *     a fixed order (element i goes to lane (i/4) mod 32, lanes accumulate with
 *     fused multiply-adds in increasing i, then a 16-8-4-2-1 butterfly); ties
 *     in D are broken by the smaller id.  Returned distances are sqrt(D).
 *   - An adjacency is n rows of W uint32 ids.  A row's out-neighbours are the
 *     entries before its first CNG_NONE (or first id >= n); the rest is padding.
 *     A row lists an id at most once (the builders' rows do): a search marks
 *     a row's ids visited together, and an id repeated within one row may be
 *     taken twice once its visited table is full, leaving a damaged beam.
 *   - Arguments are validated before any launch.  On a non-OK status nothing
 *     was launched (EINVAL/EUNSUPPORTED) or outputs are undefined (EDEVICE);
 *     cng_last_error() gives a message.  No C++ exception crosses the ABI.
 *   - Not thread-safe on one stream; distinct streams are independent.
 */
#ifndef CNG_H
#define CNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CNG_OK = 0,
    CNG_EINVAL = -1,       /* an argument is out of range or inconsistent */
    CNG_ENOMEM = -2,       /* workspace too small */
    CNG_EDEVICE = -3,      /* a HIP call failed */
    CNG_EUNSUPPORTED = -4, /* valid but outside what the kernels implement (e.g. L > 512) */
    CNG_ECAPACITY = -5     /* connectivity could not attach a point: no row has a free slot */
} cng_status;

#define CNG_NONE 0xFFFFFFFFu

/* Build flags */
#define CNG_BUILD_CONNECT 1u  /* run the connectivity phase (Algorithm 3, phase 4) */
#define CNG_BUILD_BACKWARD 2u /* backward edges with lazy pruning (Algorithm 3, phase 3) */
#define CNG_BUILD_GRAPH_CANDIDATES 4u /* sub-quadratic candidates (Algorithm 3, phases 1-2):
                                         an NN-descent K-NN graph and a beam search on it,
                                         instead of the exact C nearest neighbours */

typedef struct {
    int32_t R;           /* out-degree cap of pruning (Algorithm 2 keeps at most R), >= 1 */
    int32_t extra;       /* spare slots per row for connectivity edges; row width W = R + extra */
    int32_t C;           /* candidate-list size (the local-neighbour set V), clamped to n - 1;
                            up to 896 with the automatic band (larger with an explicit band of
                            up to 2048 entries; C above the band sends rows to the exhaustive
                            recomputation) */
    double alpha;        /* alpha of Eq. (1), > 0 */
    double tau;          /* tau of Eq. (1), >= 0 */
    uint32_t flags;      /* CNG_BUILD_* */
    int32_t Lc;          /* beam width of the connectivity searches (0 = C) */
    int32_t band;        /* per-row capacity of the candidate filter, <= 2048, rounded up to a
                            power of two (0 = automatic) */
    int32_t visited_log2;/* log2 of the search visited-table slots (0 = automatic) */
    double alpha_max;    /* adaptive alpha (Algorithm 4): largest alpha tried, >= alpha */
    double alpha_step;   /* adaptive alpha step; 0 = fixed alpha (Algorithm 2 alone) */
    int32_t pass_rows;   /* rows per pass of the candidate filter, >= 0 (0 = sized from a band
                            memory budget); rounded up to whole workgroups of 256 rows.  Only
                            splits the work: candidate lists do not depend on it */
    /* CNG_BUILD_GRAPH_CANDIDATES (see cng_nndescent, cng_graph_candidates): */
    int32_t knn_K;       /* degree of the K-NN graph, 1..64 (0 = 32); C + 1 + knn_K <= 256 */
    int32_t knn_rounds;  /* most NN-descent rounds (0 = 12) */
    int32_t cand_L;      /* beam width of the candidate searches (0 = C), <= 512 */
    uint64_t knn_seed;   /* seed of the NN-descent start (SplitMix64 stream) */
} cng_build_params;

typedef struct {
    double ms_entry, ms_candidates, ms_prune, ms_connect, ms_total; /* stage wall times */
    int64_t connect_rounds;    /* rounds of the connectivity phase */
    int64_t connect_added;     /* edges added by the connectivity phase */
    int64_t overflow_rows;     /* candidate rows recomputed exhaustively (filter band full) */
    int32_t exact_integer;     /* 1 if the filter ran in exact small-integer mode */
    int32_t filter_dtype;      /* 0 = fp32 MFMA filter, 1 = bf16 MFMA filter */
    double ms_backward;        /* wall time of the backward-edge phase (0 if not run) */
    double ms_knn_graph;       /* CNG_BUILD_GRAPH_CANDIDATES: NN-descent part of ms_candidates */
    int32_t knn_rounds_run;    /* NN-descent rounds run */
} cng_build_stats;

/* ------------------------------------------------------------------ build */

/* Bytes of device workspace cng_build needs for n points of dimension d. */
cng_status cng_build_workspace_size(int64_t n, int32_t d, const cng_build_params *p,
                                    size_t *bytes_host);

/* Build the graph (Algorithm 3 with exact candidates and fixed alpha).
 *   points  [n x d] float32;  2 <= n < 2^31 - 1, 1 <= d <= 4096.
 *   adj     [n x (R + extra)] uint32 output, CNG_NONE padded.  Columns 0..R-1
 *           hold the pruned out-neighbours in increasing (D, id) (after the
 *           backward-edge phase, if flagged); further columns only receive
 *           connectivity edges.
 *   entry   [1] uint32 output: the point nearest the centroid (search entry).
 *   stats_host  optional (NULL allowed).
 * Synchronises `stream` (the connectivity phase is iterative) and returns
 * when adj and entry are final. */
cng_status cng_build(const float *points, int64_t n, int32_t d, const cng_build_params *p,
                     uint32_t *adj, uint32_t *entry, void *workspace, size_t workspace_bytes,
                     void *stream, cng_build_stats *stats_host);

/* Stage: entry point (Algorithm 3, phase 1: the point nearest to the centroid
 * of P).  The centroid is the float64 mean (sequential sums inside blocks of
 * 4096 points, then over the block sums); the entry minimises the float64
 * squared distance to it (sequential over dimensions), ties to the smaller id.
 * workspace >= cng_entry_workspace_size(n, d). */
size_t cng_entry_workspace_size(int64_t n, int32_t d);
cng_status cng_entry_point(const float *points, int64_t n, int32_t d, uint32_t *entry,
                           void *workspace, size_t workspace_bytes, void *stream);

/* Stage: exact candidate lists.  For every row r of `rows` [nr x d], the C
 * columns of `cols` [nc x d] nearest by (D, id), ascending; with exclude_self
 * (requires rows == cols, nr == nc) column r is skipped for row r.  Missing
 * entries (C > available columns) are CNG_NONE / +inf.  band: per-row capacity
 * of the filter (0 = automatic, as in cng_build_params: then C <= 896, else
 * CNG_EUNSUPPORTED); pass_rows: rows per
 * filter pass (0 = automatic), results do not depend on it.
 *   ids [nr x C] uint32, D [nr x C] float32 squared distances (fixed order).
 * Replaces the approximate K-NN graph + beam-search candidates of Algorithm 3
 * (phases 1-2) by the exact C nearest neighbours. */
cng_status cng_knn_workspace_size(int64_t nr, int64_t nc, int32_t d, int32_t C, int32_t band,
                                  int64_t pass_rows, size_t *bytes_host);
cng_status cng_knn(const float *rows, int64_t nr, const float *cols, int64_t nc, int32_t d,
                   int32_t C, int32_t exclude_self, int32_t band, int64_t pass_rows, uint32_t *ids,
                   float *D, void *workspace, size_t workspace_bytes, void *stream,
                   int64_t *overflow_rows_host);

/* Stage: approximate K-NN graph by NN-descent (Algorithm 3, phase 1).
 * Synchronous rounds: a point's list starts as the K nearest by (D, id) of
 * the distinct points splitmix64(seed, p K + j) mod n, j < K, other than p
 * (output i of the SplitMix64 stream with seed s is the SplitMix64 mix of
 * s + (i + 1) 0x9E3779B97F4A7C15); each round replaces every list by the K
 * nearest of itself and the lists of its members, all read from the lists as
 * they were when the round began.  Stops after `rounds` rounds or after a
 * round that changed no list (rounds_host: rounds run).
 *   ids [n x K] uint32 ascending (D, id), CNG_NONE padded; D [n x K] float32.
 *   1 <= K <= 64.  Synchronises `stream`. */
cng_status cng_nndescent_workspace_size(int64_t n, int32_t K, size_t *bytes_host);
cng_status cng_nndescent(const float *points, int64_t n, int32_t d, int32_t K, uint64_t seed,
                         int32_t rounds, uint32_t *ids, float *D, void *workspace,
                         size_t workspace_bytes, void *stream, int32_t *rounds_host);

/* Stage: local-neighbour sets from a graph (Algorithm 3, phase 2).  For every
 * point p the C nearest by (D, id), p excluded, of the points that
 * beam-search(G0, x_p, s, L, C + 1) evaluates together with p's own row of
 * G0 (the pool of the NSG framework: it keeps the K-NN neighbours where G0
 * does not lead from s to p).  G0: g0 [n x K] with distances g0D (as
 * cng_nndescent returns them).  cand [n x C], candD [n x C] as cng_knn.
 * C + 1 + K <= 256, max(L, C + 1) <= 512.  Synchronises `stream`. */
cng_status cng_graph_candidates_workspace_size(int64_t n, int32_t C, size_t *bytes_host);
cng_status cng_graph_candidates(const float *points, int64_t n, int32_t d, const uint32_t *g0,
                                const float *g0D, int32_t K, uint32_t entry, int32_t L, int32_t C,
                                uint32_t *cand, float *candD, void *workspace,
                                size_t workspace_bytes, void *stream);

/* Stage: pruning (Algorithm 2 with Eq. (1), fixed alpha, at most R kept).
 *   cand [n x C] candidate ids of every point, ascending by (D, id), CNG_NONE
 *        terminated; candD [n x C] their squared distances as returned by
 *        cng_knn.  adj [n x W] output, W >= R.
 * A candidate u is dropped iff an already kept v satisfies
 *   sqrt(D(p,u)) > alpha * sqrt(D(u,v)) + (alpha + 1) * tau   (strict),
 * evaluated in float32; when the two sides differ by at most 1e-6 relative the
 * comparison is re-decided from float64 distances. */
cng_status cng_prune(const float *points, int64_t n, int32_t d, const uint32_t *cand,
                     const float *candD, int32_t C, int32_t R, int32_t W, double alpha,
                     double tau, uint32_t *adj, void *stream);

/* Stage: adaptive local pruning (Algorithm 4, Section 4.2) with the rule of
 * cng_prune.  For every point the pruning runs with alpha_i = alpha0 + i *
 * alpha_step, i = 0, 1, ... while alpha_i <= alpha_max (with 1e-9 of slack in
 * units of the step); the first pass whose kept set holds at least R/2 points
 * stands (else the pass at alpha_max), and it keeps at most R points (its R
 * closest).  alpha_step > 0, alpha_max >= alpha0; at most 1024 passes. */
cng_status cng_prune_adaptive(const float *points, int64_t n, int32_t d, const uint32_t *cand,
                              const float *candD, int32_t C, int32_t R, int32_t W, double alpha0,
                              double alpha_max, double alpha_step, double tau, uint32_t *adj,
                              void *stream);

/* Stage: backward edges with lazy pruning (Algorithm 3, phase 3; Section 4.3)
 * in place on adj [n x W] (rows end at their first CNG_NONE).  Every edge
 * (u, v) adds the reverse edge (v, u).  The candidate set of p is its row
 * together with the sources of its in-edges (a set), ordered by (D, id) with D
 * in the fixed order, and cut to its Cb nearest (the paper bounds candidate
 * sets by C).  A set of more than R points is pruned once as in cng_prune
 * (alpha_step = 0) or cng_prune_adaptive (alpha_step > 0, alpha from alpha to
 * alpha_max), at most R kept; a smaller one becomes p's row as it is.  All
 * sets are formed from the rows as they were before the call.
 *   1 <= R <= W <= 256, 1 <= Cb <= 448.
 * workspace >= cng_backward_workspace_size(n, W, Cb); enqueued on `stream`. */
cng_status cng_backward_workspace_size(int64_t n, int32_t W, int32_t Cb, size_t *bytes_host);
cng_status cng_backward(const float *points, int64_t n, int32_t d, uint32_t *adj, int32_t W,
                        int32_t R, int32_t Cb, double alpha, double alpha_max,
                        double alpha_step, double tau, void *workspace,
                        size_t workspace_bytes, void *stream);

/* Stage: connectivity (Algorithm 3, phase 4) in place on adj [n x W].
 * Rounds on a snapshot of the graph: let U be the points unreachable from
 * `entry`; A = points of U without an in-edge from U (or the smallest id of U
 * if none); each p in A is searched from `entry` with beam Lc and attached to
 * the first result (by (D, id)) whose row has a free slot (else the nearest
 * reachable point with a free slot); attachments are applied in increasing p,
 * a p whose target filled up earlier in the round waits for the next round.
 * Synchronises `stream`.  CNG_ECAPACITY if no reachable row has room. */
cng_status cng_connect_workspace_size(int64_t n, int32_t W, int32_t Lc, size_t *bytes_host);
cng_status cng_connect(const float *points, int64_t n, int32_t d, uint32_t *adj, int32_t W,
                       uint32_t entry, int32_t Lc, int32_t visited_log2, void *workspace,
                       size_t workspace_bytes, void *stream, int64_t *rounds_host,
                       int64_t *added_host);

/* ------------------------------------------------------------------ search */

/* Batched beam search (Algorithm 1), one wavefront per query.
 *   points [n x d], adj [n x W], queries [nq x d].
 *   entries [n_entries]: n_entries == 1 (shared) or nq (one per query).
 *   k >= 1; L >= 1; the beam keeps L_eff = max(L, k) <= 512 entries.
 *   ids [nq x k] uint32, dists [nq x k] float32 (sqrt of D): the first k of
 *   the final beam; CNG_NONE / +inf when fewer points were reached.
 *   hops [nq], ndc [nq]: optional (NULL allowed): explored points and
 *   distance evaluations per query.
 *   visited_log2: log2 of the per-query visited-table slots in LDS, 6..14
 *   (0 = automatic: the largest of 2^11 .. 2^13 slots with which every query
 *   of the launch can be resident on the GPU at once, else 2^10, or 2^11 for
 *   float32 vectors up to L = 128).  The table
 *   may forget old entries when full; results do not depend on it, only ndc
 *   and speed do.
 * Requires W <= 256 and d <= 4096. */
cng_status cng_search(const float *points, int64_t n, int32_t d, const uint32_t *adj, int32_t W,
                      const float *queries, int64_t nq, int32_t k, int32_t L,
                      const uint32_t *entries, int64_t n_entries, uint32_t *ids, float *dists,
                      uint32_t *hops, uint32_t *ndc, int32_t visited_log2, void *stream);

/* ------------------------------------------------------------------ precision form */

typedef enum {
    CNG_F32 = 0,      /* float32 */
    CNG_BF16 = 1,     /* bfloat16, round to nearest even */
    CNG_FP8_E4M3 = 2  /* OCP fp8 E4M3 codes with one float32 scale per vector */
} cng_dtype;

/* Bytes of the stored copy of n vectors of dimension d in `dtype`. */
size_t cng_quantized_bytes(int64_t n, int32_t d, int32_t dtype);

/* Reduced-precision copy of points [n x d] float32 for scoring in the search.
 *   CNG_BF16:     vecs [n x d] uint16 bf16 bits, each element rounded to nearest even.
 *   CNG_FP8_E4M3: vecs [n x d] uint8 codes and scales [n x 2] float32 pairs
 *                 (s, n2); per vector s = max|x| / 448 (1 if the vector is
 *                 zero), code = E4M3 value nearest x / s (ties to even,
 *                 saturating at +-448), an element stands for value(code) * s;
 *                 n2 = fl(fl(s s) dot(c, c)) with c the E4M3 values and dot the
 *                 fixed-order dot product (the distance's lanes and butterfly,
 *                 fused multiply-adds of products).
 * Finite inputs; enqueues and returns. */
cng_status cng_quantize(const float *points, int64_t n, int32_t d, int32_t dtype, void *vecs,
                        float *scales, void *stream);

/* Beam search (Algorithm 1) scoring the stored copy `vecs` (dtype as above),
 * then the converged beam of L_eff entries is re-ranked with float32
 * distances to `points` and the first k are returned: ids and dists are the
 * float32-exact values for the returned points.  bf16: the fixed-order
 * squared distance of the widened values.  fp8 (scales = the (s, n2) pairs of
 * cng_quantize): the dot form D = fma(-2 s, dot(q, c), fl(dot(q, q) + n2)),
 * clamped at +0, with float32 accumulation.  hops/ndc count the
 * reduced-precision search only.  Other arguments as cng_search.  dtype
 * CNG_F32 (vecs == points) is plain search. */
cng_status cng_search_quantized(const float *points, const void *vecs, int32_t dtype,
                                const float *scales, int64_t n, int32_t d, const uint32_t *adj,
                                int32_t W, const float *queries, int64_t nq, int32_t k, int32_t L,
                                const uint32_t *entries, int64_t n_entries, uint32_t *ids,
                                float *dists, uint32_t *hops, uint32_t *ndc, int32_t visited_log2,
                                void *stream);

/* ------------------------------------------------------------------ learned entry point */
/* Not in the paper, which starts every search at one navigating node (the
 * point nearest the centroid, Algorithm 3).  A multilayer perceptron
 * d -> H -> H -> K (ReLU hidden layers) scores K entry nodes for a query; the
 * navigating node remains the fallback when the top softmax probability is
 * below a threshold.  Parameters: one float32 vector, in this order:
 * W1 [d x H], b1 [H], W2 [H x H], b2 [H], W3 [H x K], b3 [K] (row-major,
 * y = x W + b).  precision 0: float32 matrix-core products; 1: bf16 inputs,
 * float32 accumulation. */

/* k-means (Lloyd) over points: centres start at points[init_ids[j]]
 * (init_ids [K], device), `iters` rounds of assignment (nearest centre by
 * (D, index)) and mean update (float atomics: not bit-reproducible).
 * entries [K] = point nearest each final centre.  Synchronises `stream`. */
size_t cng_kmeans_workspace_size(int64_t n, int32_t d, int32_t K);
cng_status cng_kmeans(const float *points, int64_t n, int32_t d, int32_t K, int32_t iters,
                      const uint32_t *init_ids, float *centers, uint32_t *entries, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Training labels from the plain search itself: for each query, the best
 * point of a float32 beam search (beam L, from the navigating node `nav`)
 * and then the index (0..K-1) of the entry node nearest to that point.
 * labels [nq] uint32.  Synchronises `stream`. */
cng_status cng_entry_labels_workspace_size(int64_t n, int32_t d, int64_t nq, int32_t K,
                                           size_t *bytes_host);
cng_status cng_entry_labels(const float *points, int64_t n, int32_t d, const uint32_t *adj, int32_t W,
                            uint32_t nav, const float *queries, int64_t nq, int32_t L,
                            const uint32_t *entries, int32_t K, uint32_t *labels, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Number of parameters and workspace bytes for batch B. */
int64_t cng_mlp_param_count(int32_t d, int32_t H, int32_t K);
size_t cng_mlp_workspace_size(int32_t d, int32_t H, int32_t K, int32_t B);

/* Input standardisation of the network.  The calls below that take x_mean
 * [d] and x_scale [1] (device floats; both NULL: raw inputs) feed the first
 * layer with (x - x_mean) / x_scale, computed in float32 per element.
 * cng_mlp_input_stats gives the training set's statistics: x_mean = the
 * column means (float64 sums over blocks of 4096 rows in order, then over the
 * blocks), x_scale = the root-mean-square deviation from x_mean over all
 * n * d elements (float64, at least 1e-12). */
size_t cng_mlp_input_stats_workspace_size(int64_t n, int32_t d);
cng_status cng_mlp_input_stats(const float *X, int64_t n, int32_t d, float *x_mean, float *x_scale,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Softmax cross-entropy gradients of a batch: rows batch_ids[0..B) of X
 * [* x d] (batch_ids may be NULL: rows 0..B-1) with labels[row] in [0, K).
 * grads [param_count]; loss (device float, may be NULL) = mean loss.
 * precision 1: every matrix product rounds both operands to bf16 (nearest
 * even) and accumulates in float32; 0: float32 operands.  On return the
 * workspace begins with the step's float32 intermediates, in this order:
 * H1 [B x H], H2 [B x H] (hidden activations after ReLU), dH2 [B x H],
 * dH1 [B x H] (their gradients, masked by the ReLU), Z [B x K] (logits),
 * dZ [B x K] (softmax minus one-hot, over B), loss [B]. */
cng_status cng_mlp_gradients(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                             const float *x_mean, const float *x_scale, const uint32_t *labels,
                             const uint32_t *batch_ids, int32_t B, int32_t precision, float *grads,
                             float *loss, void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (bias-corrected, step >= 1) on params with moments m1, m2. */
cng_status cng_mlp_adam(float *params, const float *grads, float *m1, float *m2, int32_t d,
                        int32_t H, int32_t K, int32_t step, float lr, float beta1, float beta2,
                        float eps, void *stream);

/* Scores: logits [B x K] for X [B x d], computed as cng_entry_predict
 * computes them (precision 1: the standardised input, the weights and each
 * hidden activation after its ReLU are rounded to bf16, products accumulate
 * in float32, biases are added in float32).  hidden (may be NULL):
 * [2 x B x H] float32, the two hidden layers' activations as the following
 * products read them (bf16 values in precision 1). */
cng_status cng_mlp_logits(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                          const float *x_mean, const float *x_scale, int32_t B, int32_t precision,
                          float *logits, float *hidden, void *workspace, size_t workspace_bytes,
                          void *stream);

/* Entry choice per query: entries[argmax] (ties to the lower index) if its
 * softmax probability is >= theta, else `fallback`.  out_entry [B] uint32,
 * out_conf [B] float (may be NULL). */
cng_status cng_entry_predict(const float *params, int32_t d, int32_t H, int32_t K, const float *X,
                             const float *x_mean, const float *x_scale, int32_t B, int32_t precision,
                             const uint32_t *entries, uint32_t fallback, float theta,
                             uint32_t *out_entry, float *out_conf, void *workspace,
                             size_t workspace_bytes, void *stream);

/* cng_entry_predict without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Its scratch memory is a fixed device
 * array of cng_entry_predict_noalloc_max_bytes() bytes (16 MiB) that the
 * library holds on every GPU it runs on until the process ends; the call
 * allocates nothing.  Shapes whose scratch (cng_mlp_workspace_size(d, H, K,
 * B)) exceeds it are refused with CNG_EUNSUPPORTED.  Every call on one GPU
 * uses that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race; calls in order on one stream do not.  Nothing in the array
 * needs to start at zero.  Outputs and arguments as cng_entry_predict. */
size_t cng_entry_predict_noalloc_max_bytes(void);
cng_status cng_entry_predict_noalloc(const float *params, int32_t d, int32_t H, int32_t K,
                                     const float *X, const float *x_mean, const float *x_scale,
                                     int32_t B, int32_t precision, const uint32_t *entries,
                                     uint32_t fallback, float theta, uint32_t *out_entry,
                                     float *out_conf, void *stream);

/* Ablation baseline without a network: entries[index of the nearest centre]. */
size_t cng_nearest_centre_workspace_size(int64_t nq, int32_t d, int32_t K);
cng_status cng_nearest_centre_entry(const float *queries, int64_t nq, int32_t d, const float *centers,
                                    int32_t K, const uint32_t *entries, uint32_t *out_entry,
                                    void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ serving */
/* Continuous batching on the device (not in the paper).  cng_serve_start
 * launches a persistent grid of `waves` wavefronts on a stream of its own;
 * each wavefront repeatedly takes the next queued query (in submission
 * order), runs the beam search of cng_search / cng_search_quantized with that
 * query's k and L, and publishes the result.  Requests submitted while others
 * run join the same grid as memory frees up.
 *
 * Admission is by footprint.  A request of nq queries with k results each
 * holds nq * (4 d + 8 k) bytes (rounded up to 64) of a pinned arena while it
 * is in flight (its query vectors and its result space) plus nq positions of
 * the item ring; it is admitted into the first free range of the arena that
 * holds it, wherever that is, so an earlier request that is still in flight
 * blocks only its own bytes.  cng_serve_submit refuses (CNG_ECAPACITY) a
 * request that does not fit now; poll completed requests and retry.  Each
 * query's beam (max(L, k) <= 256 keys) and visited table live in the LDS of
 * the wave that runs it.  Results of a query do not depend on what else is
 * in flight.
 *
 * The grid leaves by itself after `idle_checks` empty polls (default 2^21,
 * some seconds); the next submit or poll launches a fresh grid that resumes
 * at the oldest incomplete item.  A server is used from one host thread. */
typedef struct cng_server cng_server;

typedef struct {
    const float *points;    /* [n x d] float32 (re-rank / plain scoring) */
    const void *vecs;       /* stored vectors scored by the search (== points for CNG_F32) */
    int32_t dtype;          /* cng_dtype of vecs */
    const float *scales;    /* fp8 (s, n2) pairs of cng_quantize, or NULL */
    int64_t n;
    int32_t d;              /* 4..512, multiple of 4 */
    const uint32_t *adj;    /* [n x W] */
    int32_t W;
    uint32_t entry;         /* default entry point */
    int32_t waves;          /* persistent wavefronts (0: 4 per compute unit) */
    int32_t capacity;       /* item ring positions = most queries in flight (0: 16 x waves) */
    int32_t max_k;          /* largest k of any request, <= 256 */
    int32_t visited_log2;   /* 6..13; 0: the largest of 2^10 .. 2^13 slots whose
                               workgroups of 4 waves fit the LDS of a compute unit */
    int64_t arena_bytes;    /* pinned bytes for the footprints of requests in flight
                               (0: 4 x waves queries of 4 d + 8 max_k bytes); <= 16 GiB */
    int32_t idle_checks;    /* empty polls after which the grid leaves (0: 2^21) */
} cng_serve_config;

typedef struct {
    int64_t launches;       /* grids launched (1 + relaunches after an idle exit) */
    int64_t submitted;      /* requests admitted */
    int64_t completed;      /* requests retired by cng_serve_poll */
    int64_t refused;        /* submits refused with CNG_ECAPACITY */
    int64_t in_flight;      /* admitted, not yet retired */
    int64_t arena_bytes;    /* arena size */
    int64_t arena_used;     /* bytes held by requests in flight */
    int32_t running;        /* 1 while a grid is on the device */
} cng_serve_stats;

/* Device workspace (bytes) the server keeps for its lifetime. */
size_t cng_serve_workspace_size(void);
cng_status cng_serve_start(const cng_serve_config *cfg, void *workspace, size_t workspace_bytes,
                           cng_server **server_host);
/* Queue a request: queries_host [nq x d] float32, results k per query, beam L
 * (max(L, k) <= 256); entries_host [nq] optional per-query entry points.
 * Writes the request id.  CNG_ECAPACITY: not admitted now, nothing queued. */
cng_status cng_serve_submit(cng_server *server, const float *queries_host, int32_t nq, int32_t k,
                            int32_t L, const uint32_t *entries_host, uint64_t *req_host);
/* done_host = 1 once every query of the request is complete; then ids_host /
 * dists_host [nq x k] (may be NULL) receive the results and the request is
 * retired (its footprint is free again).  done_host = 0 while pending. */
cng_status cng_serve_poll(cng_server *server, uint64_t req, uint32_t *ids_host, float *dists_host,
                          int32_t *done_host);
/* Counters of the server (host memory). */
cng_status cng_serve_get_stats(cng_server *server, cng_serve_stats *stats_host);
/* End the grid and release the server. */
cng_status cng_serve_stop(cng_server *server);

/* ------------------------------------------------------------------ misc */

/* Message of the last non-OK status on the calling thread ("" if none). */
const char *cng_last_error(void);

/* Library version string. */
const char *cng_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CNG_H */
