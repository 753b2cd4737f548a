/*
 * CPU oracle for the alpha-CNG hot path (Li, Yan, Lu: "Fast-Convergent
 * Proximity Graphs for Approximate Nearest Neighbor Search").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no source, header or table with this file.
 *
 * Plain, slow, scalar code: every function follows the paper's definition or
 * algorithm in the paper's order, with OpenMP only across independent rows or
 * queries (results do not depend on the thread count).
 *
 * Two arithmetic modes:
 *   ORC_FP64 (0): every distance and decision in double precision.
 *   ORC_FP32 (1): the fixed-reduction-order single-precision arithmetic that the
 *                 GPU path must reproduce bit for bit (see orc_dist_f32).
 *
 * Readings of points where the paper is silent (tie order, tau, centroid,
 * connectivity edges) are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NONE 0xFFFFFFFFu
#define ORC_FP64 0
#define ORC_FP32 1

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ECAPACITY = -5 };

/* ------------------------------------------------------------------------- */
/* Distances (paper Section 2.1: a metric; here Euclidean L2).  Ordering keys   */
/* use the squared distance D; delta = sqrt(D) is used where the rule needs     */
/* the metric itself (the additive tau term of Eq. (1)).                        */
/* ------------------------------------------------------------------------- */

/* Fixed-order single-precision squared distance.
 * Element i belongs to lane l = (i/4) mod 32 and round r = i/128.  Each lane
 * accumulates its elements in increasing i with a fused multiply-add
 * (acc = fma(t, t, acc), t = x_i - y_i, acc starting at +0).  The 32 lane sums
 * are then combined by a butterfly: for off = 16, 8, 4, 2, 1 every lane l
 * replaces its value with value[l] + value[l ^ off]; the result is lane 0. */
float orc_dist_f32(const float *x, const float *y, int d)
{
    float acc[32];
    for (int l = 0; l < 32; ++l) acc[l] = 0.0f;
    for (int i = 0; i < d; ++i) {
        int l = (i / 4) % 32;
        float t = x[i] - y[i];
        acc[l] = fmaf(t, t, acc[l]);
    }
    for (int off = 16; off >= 1; off /= 2) {
        float next[32];
        for (int l = 0; l < 32; ++l) next[l] = acc[l] + acc[l ^ off];
        for (int l = 0; l < 32; ++l) acc[l] = next[l];
    }
    return acc[0];
}

/* The same order in double precision (inputs widened exactly). */
double orc_dist_f64(const float *x, const float *y, int d)
{
    double acc[32];
    for (int l = 0; l < 32; ++l) acc[l] = 0.0;
    for (int i = 0; i < d; ++i) {
        int l = (i / 4) % 32;
        double t = (double)x[i] - (double)y[i];
        acc[l] = fma(t, t, acc[l]);
    }
    for (int off = 16; off >= 1; off /= 2) {
        double next[32];
        for (int l = 0; l < 32; ++l) next[l] = acc[l] + acc[l ^ off];
        for (int l = 0; l < 32; ++l) acc[l] = next[l];
    }
    return acc[0];
}

/* Fixed-order single-precision dot product: the lanes and butterfly of
 * orc_dist_f32 with acc = fma(x_i, y_i, acc) (the precision form's fp8 score
 * is built from it). */
float orc_dot_f32(const float *x, const float *y, int d)
{
    float acc[32];
    for (int l = 0; l < 32; ++l) acc[l] = 0.0f;
    for (int i = 0; i < d; ++i) {
        int l = (i / 4) % 32;
        acc[l] = fmaf(x[i], y[i], acc[l]);
    }
    for (int off = 16; off >= 1; off /= 2) {
        float next[32];
        for (int l = 0; l < 32; ++l) next[l] = acc[l] + acc[l ^ off];
        for (int l = 0; l < 32; ++l) acc[l] = next[l];
    }
    return acc[0];
}

static double dist_mode(const float *x, const float *y, int d, int mode)
{
    return mode == ORC_FP32 ? (double)orc_dist_f32(x, y, d) : orc_dist_f64(x, y, d);
}

/* delta from D: correctly rounded square root in the mode's precision. */
static double delta_mode(double D, int mode)
{
    return mode == ORC_FP32 ? (double)sqrtf((float)D) : sqrt(D);
}

/* Strict total order on (D, id): ties in distance go to the smaller id.  The
 * paper gives no tie rule (Alg. 1 argmin, Alg. 2 sort); this pins one. */
static int key_less(double Da, uint32_t ia, double Db, uint32_t ib)
{
    return Da < Db || (Da == Db && ia < ib);
}

typedef struct { double D; uint32_t id; } orc_key;

static int cmp_key(const void *a, const void *b)
{
    const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
    if (key_less(x->D, x->id, y->D, y->id)) return -1;
    if (key_less(y->D, y->id, x->D, x->id)) return 1;
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------------- */
/* Exact candidates: for each row the C nearest columns by (D, id).            */
/* Stands in for the local-neighbour set V of Section 4.1 (Alg. 3 phases 1-2), */
/* computed exactly.  With exclude_self, column r is skipped for row r (the    */
/* point itself); exact duplicates of it at D = 0 are kept.                    */
/* ------------------------------------------------------------------------- */
int orc_knn(const float *rows, int64_t nr, const float *cols, int64_t nc, int d, int C,
            int exclude_self, int mode, uint32_t *ids, double *Dout)
{
    if (nr < 0 || nc < 0 || d < 1 || C < 1) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        orc_key *best = (orc_key *)malloc(sizeof(orc_key) * (size_t)(C + 1));
        if (!best) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nr; ++r) {
            if (!best) continue;
            int cnt = 0;
            const float *x = rows + (size_t)r * d;
            for (int64_t c = 0; c < nc; ++c) {
                if (exclude_self && c == r) continue;
                double D = dist_mode(x, cols + (size_t)c * d, d, mode);
                uint32_t id = (uint32_t)c;
                if (cnt == C && !key_less(D, id, best[C - 1].D, best[C - 1].id)) continue;
                /* insertion into the sorted list of the best C so far */
                int pos = cnt < C ? cnt : C - 1;
                while (pos > 0 && key_less(D, id, best[pos - 1].D, best[pos - 1].id)) {
                    best[pos] = best[pos - 1];
                    --pos;
                }
                best[pos].D = D;
                best[pos].id = id;
                if (cnt < C) ++cnt;
            }
            for (int j = 0; j < C; ++j) {
                ids[(size_t)r * C + j] = j < cnt ? best[j].id : ORC_NONE;
                Dout[(size_t)r * C + j] = j < cnt ? best[j].D : INFINITY;
            }
        }
        free(best);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Edge pruning rule (Definition 2, Eq. (1)): candidate u of point p is pruned */
/* by an already selected out-neighbour v iff                                  */
/*        delta(p,u) > alpha * delta(u,v) + (alpha + 1) * tau.                 */
/* The inequality is strict, so an exact tie keeps u.                          */
/* In FP32 mode the decision is taken in single precision unless the two sides */
/* are within 1e-6 (relative to delta(p,u)); such near-ties are re-decided     */
/* from double-precision distances.                                            */
/* ------------------------------------------------------------------------- */
static int orc_prunes(const float *pts, int d, uint32_t p, uint32_t u, uint32_t v,
                      double Dpu, double alpha, double tau, int mode)
{
    const float *xp = pts + (size_t)p * d, *xu = pts + (size_t)u * d, *xv = pts + (size_t)v * d;
    if (mode == ORC_FP64) {
        double a = sqrt(Dpu);
        double b = sqrt(orc_dist_f64(xu, xv, d));
        double lhs_b = alpha * b;
        double c = (alpha + 1.0) * tau;
        return a > lhs_b + c;
    }
    float a = sqrtf((float)Dpu);
    float b = sqrtf(orc_dist_f32(xu, xv, d));
    float al = (float)alpha, ta = (float)tau;
    float c = (al + 1.0f) * ta;
    float ab = al * b;
    float rhs = ab + c;
    float diff = fabsf(a - rhs);
    float band = 1e-6f * a;
    if (diff <= band) {
        double a64 = sqrt(orc_dist_f64(xp, xu, d));
        double b64 = sqrt(orc_dist_f64(xu, xv, d));
        double ab64 = alpha * b64;
        double c64 = (alpha + 1.0) * tau;
        return a64 > ab64 + c64;
    }
    return a > rhs;
}

/* Alg. 2 on one candidate list V (ascending by (D, id)): keep u unless an
 * earlier kept v prunes it, stopping once R are kept.  Returns the count. */
static int prune_sorted(const float *pts, int d, uint32_t p, const orc_key *V, int nv, int R,
                        double alpha, double tau, int mode, uint32_t *S)
{
    int ns = 0;
    for (int j = 0; j < nv && ns < R; ++j) {
        int pruned = 0;
        for (int s = 0; s < ns && !pruned; ++s)
            pruned = orc_prunes(pts, d, p, V[j].id, S[s], V[j].D, alpha, tau, mode);
        if (!pruned) S[ns++] = V[j].id;
    }
    return ns;
}

/* Alg. 4 adaptive-pruning(p, V, M, alpha0, alpha_max, dalpha) on a sorted V:
 * alpha_i = alpha0 + i * dalpha for i = 0, 1, ... while alpha_i <= alpha_max
 * (up to 1e-9 of slack, so that alpha_max itself is reached despite rounding);
 * the first alpha_i whose shortcut set holds at least M/2 points ends the
 * loop (else the last one stands), and the M closest points of that set are
 * returned (the pruning stops once M are kept).  dalpha <= 0: one pass with
 * alpha0 (fixed alpha). */
static int prune_select(const float *pts, int d, uint32_t p, const orc_key *V, int nv, int M,
                        double alpha0, double alpha_max, double dalpha, double tau, int mode,
                        uint32_t *S)
{
    if (!(dalpha > 0.0)) return prune_sorted(pts, d, p, V, nv, M, alpha0, tau, mode, S);
    const int h = (int)floor((alpha_max - alpha0) / dalpha + 1e-9);
    int ns = 0;
    for (int i = 0; i <= h; ++i) {
        ns = prune_sorted(pts, d, p, V, nv, M, alpha0 + i * dalpha, tau, mode, S);
        if (2 * ns >= M) break;
    }
    return ns;
}

/* Alg. 2 pruning(p, V, alpha) on the candidate list of every point, keeping at
 * most R out-neighbours, written into rows of width W >= R (padded with
 * ORC_NONE; slots beyond R are spare slots for connectivity edges).  Stopping once R are kept equals returning the R
 * closest points of the full shortcut set (the decision for u only involves
 * earlier kept points).  Candidate lists are re-sorted by (D, id) first
 * (Alg. 2 line 1); entries equal to ORC_NONE end a list. */
int orc_prune_adaptive(const float *pts, int64_t n, int d, const uint32_t *cand,
                       const double *candD, int C, int R, int W, double alpha, double alpha_max,
                       double dalpha, double tau, int mode, uint32_t *adj)
{
    if (n < 1 || d < 1 || C < 1 || R < 1 || W < R || !(alpha > 0.0) || !(tau >= 0.0))
        return ORC_EINVAL;
    if (dalpha > 0.0 && !(alpha_max >= alpha)) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        orc_key *V = (orc_key *)malloc(sizeof(orc_key) * (size_t)C);
        uint32_t *S = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)R);
        if (!V || !S) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < n; ++p) {
            if (!V || !S) continue;
            int nv = 0;
            for (int j = 0; j < C; ++j) {
                uint32_t u = cand[(size_t)p * C + j];
                if (u == ORC_NONE) break;
                V[nv].id = u;
                V[nv].D = candD[(size_t)p * C + j];
                ++nv;
            }
            qsort(V, (size_t)nv, sizeof(orc_key), cmp_key);
            int ns = prune_select(pts, d, (uint32_t)p, V, nv, R, alpha, alpha_max, dalpha, tau,
                                  mode, S);
            for (int s = 0; s < W; ++s) adj[(size_t)p * W + s] = s < ns ? S[s] : ORC_NONE;
        }
        free(V);
        free(S);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

int orc_prune(const float *pts, int64_t n, int d, const uint32_t *cand, const double *candD,
              int C, int R, int W, double alpha, double tau, int mode, uint32_t *adj)
{
    return orc_prune_adaptive(pts, n, d, cand, candD, C, R, W, alpha, alpha, 0.0, tau, mode, adj);
}

/* ------------------------------------------------------------------------- */
/* Alg. 3 phase 3: backward edges with lazy pruning (Section 4.3).  For every  */
/* edge (u, v) of the pruned graph the reverse edge (v, u) is added.  Each      */
/* point's candidate set V is its out-neighbours together with the sources of  */
/* the edges into it (a set), ordered by (D, id).  The paper bounds candidate  */
/* sets by C; here V is cut to its Cb nearest.  A point with |V| > R is pruned  */
/* once over V (Alg. 2 with cap R, or Alg. 4 when dalpha > 0); otherwise V     */
/* itself becomes its row (in (D, id)                                           */
/* order; the order of a row does not change Alg. 1).  Every decision reads    */
/* the graph as it was before this phase.  Rows have width W >= R.             */
/* ------------------------------------------------------------------------- */
int orc_backward(const float *pts, int64_t n, int d, uint32_t *adj, int R, int W, int Cb,
                 double alpha, double alpha_max, double dalpha, double tau, int mode)
{
    if (n < 1 || d < 1 || R < 1 || W < R || Cb < 1 || !(alpha > 0.0) || !(tau >= 0.0))
        return ORC_EINVAL;
    if (dalpha > 0.0 && !(alpha_max >= alpha)) return ORC_EINVAL;
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    uint32_t *out = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * W);
    uint32_t *src = NULL;
    int rc = ORC_OK;
    if (!off || !cur || !out) { rc = ORC_ENOMEM; goto done; }
    /* sources of the edges into every point, in increasing source order */
    for (int64_t u = 0; u < n; ++u)
        for (int s = 0; s < W; ++s) {
            uint32_t v = adj[(size_t)u * W + s];
            if (v == ORC_NONE || (int64_t)v >= n) break;
            off[v + 1]++;
        }
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    src = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    if (!src) { rc = ORC_ENOMEM; goto done; }
    for (int64_t v = 0; v < n; ++v) cur[v] = off[v];
    for (int64_t u = 0; u < n; ++u)
        for (int s = 0; s < W; ++s) {
            uint32_t v = adj[(size_t)u * W + s];
            if (v == ORC_NONE || (int64_t)v >= n) break;
            src[cur[v]++] = (uint32_t)u;
        }
    int fail = 0;
#pragma omp parallel
    {
        int64_t cap = 0;
        orc_key *V = NULL;
        uint32_t *S = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)R);
        if (!S) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < n; ++p) {
            if (!S) continue;
            int64_t need = W + (off[p + 1] - off[p]);
            if (need > cap) {
                free(V);
                cap = need;
                V = (orc_key *)malloc(sizeof(orc_key) * (size_t)cap);
                if (!V) {
                    cap = 0;
#pragma omp atomic write
                    fail = 1;
                    continue;
                }
            }
            const float *xp = pts + (size_t)p * d;
            int64_t nv = 0;
            for (int s = 0; s < W; ++s) {
                uint32_t v = adj[(size_t)p * W + s];
                if (v == ORC_NONE || (int64_t)v >= n) break;
                V[nv].id = v;
                V[nv].D = dist_mode(xp, pts + (size_t)v * d, d, mode);
                ++nv;
            }
            for (int64_t e = off[p]; e < off[p + 1]; ++e) {
                V[nv].id = src[e];
                V[nv].D = dist_mode(xp, pts + (size_t)src[e] * d, d, mode);
                ++nv;
            }
            qsort(V, (size_t)nv, sizeof(orc_key), cmp_key);
            /* a set: an id seen twice (u -> p and p -> u) has equal keys, adjacent */
            int64_t m = 0;
            for (int64_t j = 0; j < nv; ++j)
                if (m == 0 || V[j].id != V[m - 1].id) V[m++] = V[j];
            if (m > Cb) m = Cb;
            uint32_t *row = out + (size_t)p * W;
            int ns;
            if (m <= R) {
                for (int64_t j = 0; j < m; ++j) S[j] = V[j].id;
                ns = (int)m;
            } else {
                ns = prune_select(pts, d, (uint32_t)p, V, (int)m, R, alpha, alpha_max, dalpha,
                                  tau, mode, S);
            }
            for (int s = 0; s < W; ++s) row[s] = s < ns ? S[s] : ORC_NONE;
        }
        free(V);
        free(S);
    }
    if (fail) { rc = ORC_ENOMEM; goto done; }
    memcpy(adj, out, sizeof(uint32_t) * (size_t)n * W);
done:
    free(off); free(cur); free(out); free(src);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Entry point.  Alg. 3 uses the point found nearest to the centroid of P      */
/* (the mean of all points).  Here it is found exactly: the centroid is the    */
/* double-precision mean, summed sequentially inside blocks of 4096 points and */
/* then sequentially over the block sums; the entry is the point minimising    */
/* (squared distance in double, summed sequentially over dimensions, id).      */
/* ------------------------------------------------------------------------- */
uint32_t orc_medoid(const float *pts, int64_t n, int d)
{
    const int64_t B = 4096;
    double *tot = (double *)calloc((size_t)d, sizeof(double));
    double *blk = (double *)calloc((size_t)d, sizeof(double));
    if (!tot || !blk || n < 1) { free(tot); free(blk); return ORC_NONE; }
    for (int64_t a = 0; a < n; a += B) {
        int64_t b = a + B < n ? a + B : n;
        for (int i = 0; i < d; ++i) blk[i] = 0.0;
        for (int64_t p = a; p < b; ++p)
            for (int i = 0; i < d; ++i) blk[i] += (double)pts[(size_t)p * d + i];
        for (int i = 0; i < d; ++i) tot[i] += blk[i];
    }
    for (int i = 0; i < d; ++i) tot[i] = tot[i] / (double)n;
    double bestD = INFINITY;
    uint32_t best = ORC_NONE;
    for (int64_t p = 0; p < n; ++p) {
        double acc = 0.0;
        for (int i = 0; i < d; ++i) {
            double t = (double)pts[(size_t)p * d + i] - tot[i];
            acc = fma(t, t, acc);
        }
        if (key_less(acc, (uint32_t)p, bestD, best)) { bestD = acc; best = (uint32_t)p; }
    }
    free(tot);
    free(blk);
    return best;
}

/* ------------------------------------------------------------------------- */
/* Beam search, Alg. 1 beam-search(G, q, s, L, k), taken literally:            */
/*   Q <- {s}; E <- {}                                                         */
/*   while Q \ E is not empty:                                                 */
/*       u* <- the element of Q \ E with the smallest (D, id)                  */
/*       Q <- Q united with every out-neighbour v of u*                        */
/*       keep the L smallest of Q;  E <- E with u*                             */
/*   return the k smallest of Q                                                */
/* L is raised to k when k > L.  A row's out-neighbours are its entries before */
/* the first ORC_NONE or out-of-range id.  hops = |E|; ndc counts the distinct */
/* points whose distance to q was evaluated (the entry included).              */
/* ------------------------------------------------------------------------- */
/* How a beam search scores a point v against the query q:
 *   canonical: D(q, x_v) of the mode (pts = the vectors searched);
 *   fp8 form (scales != NULL, float32): pts = the E4M3 values c_v (unscaled),
 *   s_v = scales[v], n2_v = n2[v] = fl(fl(s_v s_v) dot(c_v, c_v)), and
 *     D = fma(-2 s_v, dot(q, c_v), fl(dot(q, q) + n2_v)), clamped at +0,
 *   the dot form of |q - s_v c_v|^2 with float32 accumulation. */
typedef struct {
    const float *pts;
    const float *scales;
    const float *n2;
    int mode;
} orc_scorer;

static double score_point(const orc_scorer *sc, const float *q, float qq, uint32_t v, int d)
{
    const float *x = sc->pts + (size_t)v * d;
    if (!sc->scales) return dist_mode(q, x, d, sc->mode);
    const float s = sc->scales[v];
    const float dot = orc_dot_f32(q, x, d);
    const float base = qq + sc->n2[v];
    const float D = fmaf(-2.0f * s, dot, base);
    return D > 0.0f ? (double)D : 0.0;
}

typedef struct {
    double *D;
    uint32_t *id;
    unsigned char *expl;
    unsigned char *seen; /* n bytes */
    uint32_t *touched;   /* ids marked in seen (to clear) */
    size_t ntouched, cap_touched;
} orc_beam;

static int beam_init(orc_beam *b, int64_t n, int cap)
{
    b->D = (double *)malloc(sizeof(double) * (size_t)cap);
    b->id = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    b->expl = (unsigned char *)malloc((size_t)cap);
    b->seen = (unsigned char *)calloc((size_t)n, 1);
    b->cap_touched = 1024;
    b->touched = (uint32_t *)malloc(sizeof(uint32_t) * b->cap_touched);
    b->ntouched = 0;
    return b->D && b->id && b->expl && b->seen && b->touched;
}

static void beam_free(orc_beam *b)
{
    free(b->D); free(b->id); free(b->expl); free(b->seen); free(b->touched);
}

static int beam_mark_seen(orc_beam *b, uint32_t v)
{
    if (b->seen[v]) return 0;
    b->seen[v] = 1;
    if (b->ntouched == b->cap_touched) {
        size_t nc = b->cap_touched * 2;
        uint32_t *t = (uint32_t *)realloc(b->touched, sizeof(uint32_t) * nc);
        if (!t) return -1;
        b->touched = t;
        b->cap_touched = nc;
    }
    b->touched[b->ntouched++] = v;
    return 1;
}

static void beam_clear_seen(orc_beam *b)
{
    for (size_t i = 0; i < b->ntouched; ++i) b->seen[b->touched[i]] = 0;
    b->ntouched = 0;
}

/* One query.  Returns the final Q size (<= Leff); Q is left in b. */
static int beam_one(orc_beam *b, const orc_scorer *sc, int64_t n, int d, const uint32_t *adj, int R,
                    const float *q, uint32_t s, int Leff, uint32_t *hops, uint32_t *ndc,
                    uint32_t *trace, int trace_cap, int *trace_len)
{
    int qn = 1, h = 0;
    uint32_t nd = 0;
    const float qq = sc->scales ? orc_dot_f32(q, q, d) : 0.0f;
    b->D[0] = score_point(sc, q, qq, s, d);
    b->id[0] = s;
    b->expl[0] = 0;
    if (beam_mark_seen(b, s) > 0) ++nd;
    for (;;) {
        int i = 0;
        while (i < qn && b->expl[i]) ++i; /* Q is kept sorted: first unexplored */
        if (i == qn) break;
        uint32_t u = b->id[i];
        if (trace && h < trace_cap) trace[h] = u;
        ++h;
        for (int j = 0; j < R; ++j) {
            uint32_t v = adj[(size_t)u * R + j];
            if (v == ORC_NONE || (int64_t)v >= n) break;
            int inq = 0;
            for (int t = 0; t < qn; ++t)
                if (b->id[t] == v) { inq = 1; break; }
            if (inq) continue; /* set union */
            double Dv = score_point(sc, q, qq, v, d);
            if (beam_mark_seen(b, v) > 0) ++nd;
            int pos = qn;
            while (pos > 0 && key_less(Dv, v, b->D[pos - 1], b->id[pos - 1])) {
                b->D[pos] = b->D[pos - 1];
                b->id[pos] = b->id[pos - 1];
                b->expl[pos] = b->expl[pos - 1];
                --pos;
            }
            b->D[pos] = Dv;
            b->id[pos] = v;
            b->expl[pos] = 0;
            ++qn;
        }
        if (qn > Leff) qn = Leff; /* keep the L closest */
        /* mark u* explored (it may have been cut by the truncation) */
        for (int t = 0; t < qn; ++t)
            if (b->id[t] == u) { b->expl[t] = 1; break; }
    }
    beam_clear_seen(b);
    if (hops) *hops = (uint32_t)h;
    if (ndc) *ndc = nd;
    if (trace_len) *trace_len = h;
    return qn;
}

int orc_search(const float *pts, int64_t n, int d, const uint32_t *adj, int R,
               const float *queries, int64_t nq, int k, int L,
               const uint32_t *entries, int64_t n_entries, int mode,
               uint32_t *ids, double *dists, uint32_t *hops, uint32_t *ndc)
{
    if (n < 1 || d < 1 || R < 1 || k < 1 || L < 1 || nq < 0) return ORC_EINVAL;
    if (n_entries != 1 && n_entries != nq) return ORC_EINVAL;
    for (int64_t e = 0; e < n_entries; ++e)
        if ((int64_t)entries[e] >= n) return ORC_EINVAL;
    int Leff = L > k ? L : k;
    int cap = Leff + R + 1;
    int fail = 0;
#pragma omp parallel
    {
        orc_beam b;
        int ok = beam_init(&b, n, cap);
        if (!ok) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nq; ++i) {
            if (!ok) continue;
            uint32_t s = entries[n_entries == 1 ? 0 : i];
            uint32_t h = 0, nd = 0;
            const orc_scorer sc = {pts, NULL, NULL, mode};
            int qn = beam_one(&b, &sc, n, d, adj, R, queries + (size_t)i * d, s, Leff, &h, &nd,
                              NULL, 0, NULL);
            for (int j = 0; j < k; ++j) {
                ids[(size_t)i * k + j] = j < qn ? b.id[j] : ORC_NONE;
                dists[(size_t)i * k + j] = j < qn ? delta_mode(b.D[j], mode) : INFINITY;
            }
            if (hops) hops[i] = h;
            if (ndc) ndc[i] = nd;
        }
        beam_free(&b);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Single query with the sequence of hop vertices u* (Lemma 5 checks). */
int orc_search_trace(const float *pts, int64_t n, int d, const uint32_t *adj, int R,
                     const float *q, int k, int L, uint32_t entry, int mode,
                     uint32_t *ids, double *dists, uint32_t *trace, int trace_cap, int *trace_len)
{
    if (n < 1 || d < 1 || R < 1 || k < 1 || L < 1 || (int64_t)entry >= n) return ORC_EINVAL;
    int Leff = L > k ? L : k;
    orc_beam b;
    if (!beam_init(&b, n, Leff + R + 1)) { beam_free(&b); return ORC_ENOMEM; }
    const orc_scorer sc = {pts, NULL, NULL, mode};
    int qn = beam_one(&b, &sc, n, d, adj, R, q, entry, Leff, NULL, NULL, trace, trace_cap,
                      trace_len);
    for (int j = 0; j < k; ++j) {
        ids[j] = j < qn ? b.id[j] : ORC_NONE;
        dists[j] = j < qn ? delta_mode(b.D[j], mode) : INFINITY;
    }
    beam_free(&b);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Reduced-precision storage (the precision form of the search: vectors kept  */
/* in bf16 or in fp8-E4M3 with one float32 scale per vector, candidates scored */
/* from them, the final beam re-ranked with the float32 vectors).  These       */
/* return the float32 value each stored element stands for.                    */
/* ------------------------------------------------------------------------- */

/* Nearest bfloat16 (8 significant bits), ties to even. */
float orc_round_bf16(float x)
{
    if (x == 0.0f || !isfinite(x)) return x;
    if (fabsf(x) < 0x1p-126f) return ldexpf(rintf(ldexpf(x, 133)), -133); /* subnormal step */
    int e;
    float m = frexpf(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
    return ldexpf(rintf(ldexpf(m, 8)), e - 8);
}

/* Nearest OCP fp8-E4M3 value (4 significant bits, exponent bias 7, no
 * infinities, largest finite 448, subnormal step 2^-9), ties to even,
 * saturating at +-448. */
float orc_round_e4m3(float v)
{
    float a = fabsf(v), r;
    if (!(a == a)) return v;
    if (a >= 448.0f) r = 448.0f;
    else if (a < 0x1p-6f) r = ldexpf(rintf(ldexpf(a, 9)), -9);
    else {
        int e;
        float m = frexpf(a, &e);
        r = ldexpf(rintf(ldexpf(m, 4)), e - 4);
        if (r > 448.0f) r = 448.0f;
    }
    return copysignf(r, v);
}

/* Per-vector fp8 scale: s = max|x| / 448 (1 for an all-zero vector). */
float orc_fp8_scale(const float *x, int d)
{
    float m = 0.0f;
    for (int i = 0; i < d; ++i) m = fmaxf(m, fabsf(x[i]));
    return m > 0.0f ? m / 448.0f : 1.0f;
}

/* dtype 1: bf16, 2: fp8-E4M3 with per-vector scale.  out [n x d] holds the
 * float32 values the stored vectors represent (fp8: code value times scale). */
int orc_dequantized(const float *pts, int64_t n, int d, int dtype, float *out, float *scales)
{
    if (n < 0 || d < 1 || (dtype != 1 && dtype != 2)) return ORC_EINVAL;
    for (int64_t p = 0; p < n; ++p) {
        const float *x = pts + (size_t)p * d;
        float *o = out + (size_t)p * d;
        if (dtype == 1) {
            for (int i = 0; i < d; ++i) o[i] = orc_round_bf16(x[i]);
        } else {
            float sc = orc_fp8_scale(x, d);
            if (scales) scales[p] = sc;
            for (int i = 0; i < d; ++i) {
                float scaled = x[i] / sc;
                o[i] = orc_round_e4m3(scaled) * sc;
            }
        }
    }
    return ORC_OK;
}

/* Beam search scored by `sc`, then, when rpts is given, the final beam (all
 * of its L entries) is re-ranked by distances to the float32 vectors rpts and
 * the first k returned. */
static int search_scored(const orc_scorer *sc, const float *rpts, int64_t n, int d,
                         const uint32_t *adj, int R, const float *queries, int64_t nq, int k, int L,
                         const uint32_t *entries, int64_t n_entries, int mode, uint32_t *ids,
                         double *dists, uint32_t *hops, uint32_t *ndc);

/* Beam search over `spts` (the stored, possibly reduced-precision vectors, by
 * the canonical distance), with the re-rank of search_scored. */
int orc_search_rerank(const float *spts, const float *rpts, int64_t n, int d, const uint32_t *adj,
                      int R, const float *queries, int64_t nq, int k, int L,
                      const uint32_t *entries, int64_t n_entries, int mode, uint32_t *ids,
                      double *dists, uint32_t *hops, uint32_t *ndc)
{
    const orc_scorer sc = {spts, NULL, NULL, mode};
    return search_scored(&sc, rpts, n, d, adj, R, queries, nq, k, L, entries, n_entries, mode, ids,
                         dists, hops, ndc);
}

/* fp8 form of the stored vectors: per vector the scale s = max|x| / 448 (1
 * for a zero vector), the E4M3 values c_i = e4m3(x_i / s) (unscaled) and
 * n2 = fl(fl(s s) dot(c, c)) (fixed-order dot). */
int orc_fp8_encode(const float *pts, int64_t n, int d, float *cvals, float *scales, float *n2)
{
    if (n < 0 || d < 1) return ORC_EINVAL;
    for (int64_t p = 0; p < n; ++p) {
        const float *x = pts + (size_t)p * d;
        float *c = cvals + (size_t)p * d;
        const float sc = orc_fp8_scale(x, d);
        for (int i = 0; i < d; ++i) c[i] = orc_round_e4m3(x[i] / sc);
        scales[p] = sc;
        const float ss = sc * sc;
        n2[p] = ss * orc_dot_f32(c, c, d);
    }
    return ORC_OK;
}

/* The fp8 score of one stored vector (c, s, n2) against q (see orc_scorer). */
float orc_fp8_score(const float *q, const float *c, float s, float n2, int d)
{
    const orc_scorer sc = {c, &s, &n2, ORC_FP32};
    return (float)score_point(&sc, q, orc_dot_f32(q, q, d), 0, d);
}

/* Beam search scored by the fp8 dot form (float32), the final beam re-ranked
 * with the float32 vectors rpts. */
int orc_search_fp8(const float *cvals, const float *scales, const float *n2, const float *rpts,
                   int64_t n, int d, const uint32_t *adj, int R, const float *queries, int64_t nq,
                   int k, int L, const uint32_t *entries, int64_t n_entries, uint32_t *ids,
                   double *dists, uint32_t *hops, uint32_t *ndc)
{
    if (!scales || !n2) return ORC_EINVAL;
    const orc_scorer sc = {cvals, scales, n2, ORC_FP32};
    return search_scored(&sc, rpts, n, d, adj, R, queries, nq, k, L, entries, n_entries, ORC_FP32,
                         ids, dists, hops, ndc);
}

static int search_scored(const orc_scorer *sc, const float *rpts, int64_t n, int d,
                         const uint32_t *adj, int R, const float *queries, int64_t nq, int k, int L,
                         const uint32_t *entries, int64_t n_entries, int mode, uint32_t *ids,
                         double *dists, uint32_t *hops, uint32_t *ndc)
{
    if (n < 1 || d < 1 || R < 1 || k < 1 || L < 1 || nq < 0) return ORC_EINVAL;
    if (n_entries != 1 && n_entries != nq) return ORC_EINVAL;
    for (int64_t e = 0; e < n_entries; ++e)
        if ((int64_t)entries[e] >= n) return ORC_EINVAL;
    int Leff = L > k ? L : k;
    int cap = Leff + R + 1;
    int fail = 0;
#pragma omp parallel
    {
        orc_beam b;
        int ok = beam_init(&b, n, cap);
        orc_key *rk = (orc_key *)malloc(sizeof(orc_key) * (size_t)cap);
        if (!ok || !rk) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nq; ++i) {
            if (!ok || !rk) continue;
            const float *q = queries + (size_t)i * d;
            uint32_t s = entries[n_entries == 1 ? 0 : i];
            uint32_t h = 0, nd = 0;
            int qn = beam_one(&b, sc, n, d, adj, R, q, s, Leff, &h, &nd, NULL, 0, NULL);
            for (int j = 0; j < qn; ++j) {
                rk[j].id = b.id[j];
                rk[j].D = rpts ? dist_mode(q, rpts + (size_t)b.id[j] * d, d, mode) : b.D[j];
            }
            qsort(rk, (size_t)qn, sizeof(orc_key), cmp_key);
            for (int j = 0; j < k; ++j) {
                ids[(size_t)i * k + j] = j < qn ? rk[j].id : ORC_NONE;
                dists[(size_t)i * k + j] = j < qn ? delta_mode(rk[j].D, mode) : INFINITY;
            }
            if (hops) hops[i] = h;
            if (ndc) ndc[i] = nd;
        }
        beam_free(&b);
        free(rk);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Connectivity (Alg. 3 phase 4).  The paper only says that edges are added   */
/* from the traversal tree of s so that every point is reachable.  Reading,    */
/* in rounds on a fixed snapshot of the graph:                                 */
/*   Reach <- points reachable from s.  If Reach = P: done.                    */
/*   U <- P \ Reach.  On the subgraph that U induces, take the strongly        */
/*   connected components that no edge from the rest of U enters (the source   */
/*   components: every point of U is reachable from one of them), and let A   */
/*   be the smallest id of each, in id order.  (A point of U without an       */
/*   in-edge from U is a source component of its own.)                        */
/*   For every p in A: run beam-search(G, x_p, s, Lc, Lc) on the snapshot and */
/*   let t_p be the first point of its result (by (D, id)) whose row has a     */
/*   free slot; if none has one, the reached point with a free slot nearest to */
/*   x_p by (D, id); if no reached point has a free slot: capacity error.      */
/*   Then, in increasing p, append p to row t_p if that row still has a free   */
/*   slot (a p that finds it full waits for the next round).                   */
/* Rows have width W here (pruned edges plus spare slots); a row's out-degree  */
/* is the number of entries before its first ORC_NONE.  The paper's phase 4   */
/* follows NSG, whose tree growth adds edges regardless of the degree cap;     */
/* the spare slots give those edges room without touching pruned edges.        */
/* ------------------------------------------------------------------------- */
static int row_degree(const uint32_t *adj, int R, uint32_t t)
{
    int g = 0;
    while (g < R && adj[(size_t)t * R + g] != ORC_NONE) ++g;
    return g;
}

/* A of a connectivity round: the smallest id of every source component of the
 * subgraph induced by the unreached points (Tarjan's algorithm, 1972, run
 * iteratively).  Work arrays of n entries: idx, low, comp (int64), stk, cs
 * (uint32), cpos (int), flag (bytes: on the stack / component not a source /
 * component taken).  Returns |A|. */
static int64_t source_components(const uint32_t *adj, int64_t n, int R, const unsigned char *reached,
                                 uint32_t *A, int64_t *idx, int64_t *low, int64_t *comp,
                                 uint32_t *stk, uint32_t *cs, int *cpos, unsigned char *flag)
{
    const unsigned char ONSTACK = 1, NOTSRC = 2, TAKEN = 4;
    for (int64_t v = 0; v < n; ++v) { idx[v] = -1; flag[v] = 0; comp[v] = -1; }
    int64_t counter = 0, ncomp = 0, sp = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (reached[r] || idx[r] >= 0) continue;
        /* depth-first search from r over unreached points; cs holds the path,
         * cpos the next edge of each point on it */
        int64_t csp = 0;
        cs[csp] = (uint32_t)r; cpos[csp] = 0; ++csp;
        idx[r] = low[r] = counter++;
        stk[sp++] = (uint32_t)r; flag[r] |= ONSTACK;
        while (csp > 0) {
            const uint32_t u = cs[csp - 1];
            int j = cpos[csp - 1];
            int descended = 0;
            while (j < R) {
                const uint32_t v = adj[(size_t)u * R + j];
                if (v == ORC_NONE || (int64_t)v >= n) { j = R; break; }
                ++j;
                if (reached[v]) continue;
                if (idx[v] < 0) {
                    cpos[csp - 1] = j;
                    idx[v] = low[v] = counter++;
                    stk[sp++] = v; flag[v] |= ONSTACK;
                    cs[csp] = v; cpos[csp] = 0; ++csp;
                    descended = 1;
                    break;
                }
                if (flag[v] & ONSTACK) low[u] = low[u] < idx[v] ? low[u] : idx[v];
            }
            if (descended) continue;
            /* u is done: close its component if it is a root, then return */
            if (low[u] == idx[u]) {
                uint32_t w;
                do {
                    w = stk[--sp];
                    flag[w] &= (unsigned char)~ONSTACK;
                    comp[w] = ncomp;
                } while (w != u);
                ++ncomp;
            }
            --csp;
            if (csp > 0) {
                const uint32_t parent = cs[csp - 1];
                low[parent] = low[parent] < low[u] ? low[parent] : low[u];
            }
        }
    }
    /* components entered by an edge from another component of U; flags of
     * components are kept at the index of the component */
    for (int64_t v = 0; v < n; ++v) flag[v] = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (reached[u]) continue;
        for (int j = 0; j < R; ++j) {
            const uint32_t v = adj[(size_t)u * R + j];
            if (v == ORC_NONE || (int64_t)v >= n) break;
            if (!reached[v] && comp[v] != comp[u]) flag[comp[v]] |= NOTSRC;
        }
    }
    int64_t nA = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (reached[v]) continue;
        const int64_t c = comp[v];
        if (flag[c] & (NOTSRC | TAKEN)) continue;
        flag[c] |= TAKEN;
        A[nA++] = (uint32_t)v;
    }
    return nA;
}

static void bfs_mark(const uint32_t *adj, int64_t n, int R, unsigned char *reached, uint32_t *stack,
                     uint32_t src)
{
    if (reached[src]) return;
    int64_t top = 0;
    reached[src] = 1;
    stack[top++] = src;
    while (top > 0) {
        uint32_t u = stack[--top];
        for (int j = 0; j < R; ++j) {
            uint32_t v = adj[(size_t)u * R + j];
            if (v == ORC_NONE || (int64_t)v >= n) break;
            if (!reached[v]) { reached[v] = 1; stack[top++] = v; }
        }
    }
}

int orc_connect(const float *pts, int64_t n, int d, uint32_t *adj, int R, uint32_t entry, int Lc,
                int mode, int64_t *n_added, int64_t *n_rounds)
{
    if (n < 1 || d < 1 || R < 1 || Lc < 1 || (int64_t)entry >= n) return ORC_EINVAL;
    unsigned char *reached = (unsigned char *)calloc((size_t)n, 1);
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *A = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *low = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *comp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    uint32_t *cs = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int *cpos = (int *)malloc(sizeof(int) * (size_t)n);
    unsigned char *flag = (unsigned char *)malloc((size_t)n);
    int rc = ORC_OK;
    int64_t added = 0, rounds = 0;
    if (!reached || !stack || !A || !T || !deg || !idx || !low || !comp || !cs || !cpos || !flag) {
        rc = ORC_ENOMEM;
        goto done;
    }
    bfs_mark(adj, n, R, reached, stack, entry);
    for (;;) {
        int64_t any = 0;
        for (int64_t w = 0; w < n && !any; ++w) any = !reached[w];
        if (!any) break; /* everything reachable */
        ++rounds;
        const int64_t nA = source_components(adj, n, R, reached, A, idx, low, comp, stack, cs, cpos, flag);
        for (int64_t t = 0; t < n; ++t) deg[t] = row_degree(adj, R, (uint32_t)t);
        int fail = 0;
#pragma omp parallel
        {
            orc_beam b;
            int ok = beam_init(&b, n, Lc + R + 1);
            if (!ok) {
#pragma omp atomic write
                fail = ORC_ENOMEM;
            }
#pragma omp for schedule(dynamic, 1)
            for (int64_t a = 0; a < nA; ++a) {
                if (!ok) continue;
                uint32_t p = A[a];
                const float *xp = pts + (size_t)p * d;
                const orc_scorer sc = {pts, NULL, NULL, mode};
                int qn = beam_one(&b, &sc, n, d, adj, R, xp, entry, Lc, NULL, NULL, NULL, 0, NULL);
                uint32_t t = ORC_NONE;
                for (int j = 0; j < qn; ++j)
                    if (deg[b.id[j]] < R) { t = b.id[j]; break; }
                if (t == ORC_NONE) { /* nearest reached point with room */
                    double bD = INFINITY;
                    for (int64_t w = 0; w < n; ++w) {
                        if (!reached[w] || deg[w] >= R) continue;
                        double D = dist_mode(xp, pts + (size_t)w * d, d, mode);
                        if (key_less(D, (uint32_t)w, bD, t)) { bD = D; t = (uint32_t)w; }
                    }
                }
                T[a] = t;
            }
            beam_free(&b);
        }
        if (fail) { rc = fail; goto done; }
        for (int64_t a = 0; a < nA; ++a) {
            uint32_t p = A[a], t = T[a];
            if (t == ORC_NONE) { rc = ORC_ECAPACITY; goto done; }
            if (deg[t] >= R) continue; /* taken earlier in this round: retry */
            adj[(size_t)t * R + deg[t]] = p;
            deg[t]++;
            ++added;
        }
        /* reach(s) grows by what the new edges expose */
        memset(reached, 0, (size_t)n);
        bfs_mark(adj, n, R, reached, stack, entry);
    }
done:
    if (n_added) *n_added = added;
    if (n_rounds) *n_rounds = rounds;
    free(reached); free(stack); free(A); free(T); free(deg);
    free(idx); free(low); free(comp); free(cs); free(cpos); free(flag);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Alg. 3 phases 1-2 with sub-quadratic candidates (Section 4.1): an           */
/* approximate K-NN graph G0, then each point's local-neighbour set from a     */
/* beam search on G0.                                                          */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea and Flood, 2014) used as a counter-based generator:
 * output i of the stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15),
 * mix(z) = z3 ^ (z3 >> 31) with z1 = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9,
 * z2 = z1, z3 = (z2 ^ (z2 >> 27)) * 0x94D049BB133111EB. */
uint64_t orc_splitmix(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int cmp_u32(const void *a, const void *b)
{
    const uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

/* The K nearest (D, id) of the distinct ids in ids[0..m) other than p, into
 * out / outD (ORC_NONE / +inf padded).  ids is reordered. */
static void top_k_of(const float *pts, int d, uint32_t p, uint32_t *ids, int64_t m, int K, int mode,
                     orc_key *tmp, uint32_t *out, double *outD)
{
    qsort(ids, (size_t)m, sizeof(uint32_t), cmp_u32);
    int64_t nt = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (ids[i] == p || ids[i] == ORC_NONE || (i > 0 && ids[i] == ids[i - 1])) continue;
        tmp[nt].id = ids[i];
        tmp[nt].D = dist_mode(pts + (size_t)p * d, pts + (size_t)ids[i] * d, d, mode);
        ++nt;
    }
    qsort(tmp, (size_t)nt, sizeof(orc_key), cmp_key);
    for (int j = 0; j < K; ++j) {
        out[j] = j < nt ? tmp[j].id : ORC_NONE;
        outD[j] = j < nt ? tmp[j].D : INFINITY;
    }
}

/* Phase 1: approximate K-NN graph G0 by NN-descent in synchronous rounds.
 * Start: the list of p is the K nearest by (D, id) of the distinct points
 * orc_splitmix(seed, p K + j) mod n (j < K) other than p.  Round: every list
 * becomes the K nearest by (D, id) of itself together with the lists of its
 * members (neighbours of neighbours), p excluded, all read from the lists as
 * they were when the round began.  Stops after `rounds` rounds or after a
 * round that changed no list.  knn / knnD [n x K] (NONE / +inf padded). */
int orc_nndescent(const float *pts, int64_t n, int d, int K, uint64_t seed, int rounds, int mode,
                  uint32_t *knn, double *knnD, int *rounds_run)
{
    if (n < 1 || d < 1 || K < 1 || rounds < 0) return ORC_EINVAL;
    const int64_t cap = (int64_t)K + (int64_t)K * K;
    uint32_t *prev = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * K);
    if (!prev) return ORC_ENOMEM;
    int fail = 0;
#pragma omp parallel
    {
        uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
        orc_key *tmp = (orc_key *)malloc(sizeof(orc_key) * (size_t)cap);
        if (!ids || !tmp) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < n; ++p) {
            if (!ids || !tmp) continue;
            for (int j = 0; j < K; ++j)
                ids[j] = (uint32_t)(orc_splitmix(seed, (uint64_t)p * K + j) % (uint64_t)n);
            top_k_of(pts, d, (uint32_t)p, ids, K, K, mode, tmp, knn + (size_t)p * K,
                     knnD + (size_t)p * K);
        }
        free(ids);
        free(tmp);
    }
    int r = 0;
    while (!fail && r < rounds) {
        memcpy(prev, knn, sizeof(uint32_t) * (size_t)n * K);
        int64_t changed = 0;
#pragma omp parallel
        {
            uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
            orc_key *tmp = (orc_key *)malloc(sizeof(orc_key) * (size_t)cap);
            if (!ids || !tmp) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(dynamic, 64) reduction(+ : changed)
            for (int64_t p = 0; p < n; ++p) {
                if (!ids || !tmp) continue;
                int64_t m = 0;
                const uint32_t *own = prev + (size_t)p * K;
                for (int j = 0; j < K; ++j) {
                    const uint32_t u = own[j];
                    ids[m++] = u;
                    if (u == ORC_NONE) continue;
                    for (int i = 0; i < K; ++i) ids[m++] = prev[(size_t)u * K + i];
                }
                uint32_t *out = knn + (size_t)p * K;
                top_k_of(pts, d, (uint32_t)p, ids, m, K, mode, tmp, out, knnD + (size_t)p * K);
                for (int j = 0; j < K; ++j)
                    if (out[j] != own[j]) { ++changed; break; }
            }
            free(ids);
            free(tmp);
        }
        ++r;
        if (changed == 0) break;
    }
    free(prev);
    if (rounds_run) *rounds_run = r;
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Phase 2: the local-neighbour set of every point from G0 (rows of width Kg,
 * NONE terminated): the C nearest (D, id), p excluded, of the points that
 * beam-search(G0, x_p, s, L, C + 1) evaluates together with p's own G0 row
 * (the pool of the NSG framework the paper follows; it keeps a point's K-NN
 * neighbours when G0 does not lead from s to it, as between clusters).  With a
 * beam of max(L, C + 1) entries the nearest evaluated points are the first of
 * its final beam (an evaluated point leaves the beam, or never enters it,
 * only for nearer ones).  cand / candD [n x C] (NONE / +inf padded). */
int orc_graph_candidates(const float *pts, int64_t n, int d, const uint32_t *g0, int Kg, uint32_t s,
                         int L, int C, int mode, uint32_t *cand, double *candD)
{
    if (n < 1 || d < 1 || Kg < 1 || C < 1 || L < 1 || (int64_t)s >= n) return ORC_EINVAL;
    const int Leff = L > C + 1 ? L : C + 1;
    int fail = 0;
#pragma omp parallel
    {
        orc_beam b;
        int ok = beam_init(&b, n, Leff + Kg + 1);
        orc_key *pool = (orc_key *)malloc(sizeof(orc_key) * (size_t)(Leff + Kg));
        if (!ok || !pool) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < n; ++p) {
            if (!ok || !pool) continue;
            const orc_scorer sc = {pts, NULL, NULL, mode};
            const float *xp = pts + (size_t)p * d;
            int qn = beam_one(&b, &sc, n, d, g0, Kg, xp, s, Leff, NULL, NULL, NULL, 0, NULL);
            int m = 0;
            for (int j = 0; j < qn; ++j) {
                pool[m].id = b.id[j];
                pool[m].D = b.D[j];
                ++m;
            }
            for (int j = 0; j < Kg; ++j) {
                const uint32_t v = g0[(size_t)p * Kg + j];
                if (v == ORC_NONE || (int64_t)v >= n) break;
                pool[m].id = v;
                pool[m].D = dist_mode(xp, pts + (size_t)v * d, d, mode);
                ++m;
            }
            qsort(pool, (size_t)m, sizeof(orc_key), cmp_key);
            int w = 0;
            for (int j = 0; j < m && w < C; ++j) {
                if (pool[j].id == (uint32_t)p) continue;
                if (j > 0 && pool[j].id == pool[j - 1].id) continue;  /* equal keys are adjacent */
                cand[(size_t)p * C + w] = pool[j].id;
                candD[(size_t)p * C + w] = pool[j].D;
                ++w;
            }
            for (; w < C; ++w) {
                cand[(size_t)p * C + w] = ORC_NONE;
                candD[(size_t)p * C + w] = INFINITY;
            }
        }
        beam_free(&b);
        free(pool);
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Whole build: entry point, exact candidates, pruning of each candidate list  */
/* (Alg. 2 with cap R and fixed alpha, or Alg. 4's adaptive alpha when         */
/* dalpha > 0), optionally backward edges with lazy pruning (phase 3, the same */
/* pruning), then connectivity.  Rows have width R + extra; the extra slots    */
/* only ever hold connectivity edges.                                           */
/* ------------------------------------------------------------------------- */
int orc_build_ex(const float *pts, int64_t n, int d, int R, int extra, int C, double alpha,
                 double alpha_max, double dalpha, double tau, int mode, int connect, int backward,
                 int Lc, int knn_K, uint64_t knn_seed, int knn_rounds, int cand_L, uint32_t *adj,
                 uint32_t *entry, int64_t *n_added)
{
    if (n < 2 || d < 1 || R < 1 || extra < 0 || C < 1) return ORC_EINVAL;
    int W = R + extra;
    int Ce = (int64_t)C > n - 1 ? (int)(n - 1) : C;
    uint32_t *cand = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * Ce);
    double *cD = (double *)malloc(sizeof(double) * (size_t)n * Ce);
    uint32_t *g0 = NULL;
    double *g0D = NULL;
    int rc = ORC_OK;
    if (!cand || !cD) { rc = ORC_ENOMEM; goto out; }
    *entry = orc_medoid(pts, n, d);
    if (knn_K > 0) {
        /* phases 1-2: NN-descent graph, candidates from a beam search on it */
        g0 = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * knn_K);
        g0D = (double *)malloc(sizeof(double) * (size_t)n * knn_K);
        if (!g0 || !g0D) { rc = ORC_ENOMEM; goto out; }
        rc = orc_nndescent(pts, n, d, knn_K, knn_seed, knn_rounds, mode, g0, g0D, NULL);
        if (rc) goto out;
        rc = orc_graph_candidates(pts, n, d, g0, knn_K, *entry, cand_L, Ce, mode, cand, cD);
    } else {
        rc = orc_knn(pts, n, pts, n, d, Ce, 1, mode, cand, cD);
    }
    if (rc) goto out;
    rc = orc_prune_adaptive(pts, n, d, cand, cD, Ce, R, W, alpha, alpha_max, dalpha, tau, mode,
                            adj);
    if (rc) goto out;
    if (backward) rc = orc_backward(pts, n, d, adj, R, W, Ce, alpha, alpha_max, dalpha, tau, mode);
    if (rc) goto out;
    if (n_added) *n_added = 0;
    if (connect) rc = orc_connect(pts, n, d, adj, W, *entry, Lc > 0 ? Lc : Ce, mode, n_added, NULL);
out:
    free(cand);
    free(cD);
    free(g0);
    free(g0D);
    return rc;
}

int orc_build(const float *pts, int64_t n, int d, int R, int extra, int C, double alpha,
              double alpha_max, double dalpha, double tau, int mode, int connect, int backward,
              int Lc, uint32_t *adj, uint32_t *entry, int64_t *n_added)
{
    return orc_build_ex(pts, n, d, R, extra, C, alpha, alpha_max, dalpha, tau, mode, connect,
                        backward, Lc, 0, 0, 0, 0, adj, entry, n_added);
}
