/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for min-plus APSP.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant generator with the HIP path.
 *
 * Conventions (paper: "The Floyd-Warshall Algorithm Re-implemented Using
 * 3D-Tensors and Hardware Acceleration", arXiv 2310.03983):
 *   - a cost matrix is n x n, row = source vertex, column = target vertex,
 *     stored row-major with a leading dimension ld >= n (Sec. 3.1 describes
 *     H with rows indexing the "from" vertex and columns the "to" vertex);
 *   - the diagonal is 0 (Sec. 3.4, self-loops get zero cost);
 *   - a missing edge is INF: 2^30 for int32, +inf for floating point.
 *     The paper does not fix INF or say what happens on overflow; the
 *     reading used here is saturating addition, a (+) b = min(a + b, INF),
 *     evaluated in 64-bit so that it can never wrap.
 *
 * Every routine below is a direct transcription of a definition; none is
 * blocked, fused or reordered.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>

/* binary32 sums below must be rounded once, to binary32 (no excess precision). */
_Static_assert(FLT_EVAL_METHOD == 0, "oracle needs FLT_EVAL_METHOD == 0");

#define ORACLE_INF_I32 ((int64_t)1 << 30)

static int64_t sat_add_i32(int64_t a, int64_t b) {
    int64_t s = a + b;
    return s < ORACLE_INF_I32 ? s : ORACLE_INF_I32;
}

/* ------------------------------------------------------------------------
 * O1: Floyd-Warshall (Sec. 2, Eq. 1):
 *   d^{k+1}[i,j] = min(d^k[i,j], d^k[i,k] + d^k[k,j]),  k = 0 .. n-1.
 * Updating d in place is the textbook form: during pass k, row k and column
 * k do not change because d[k][k] = 0, so every read of d[i][k] / d[k][j]
 * sees the pass-k value.  The optional OpenMP split is over i only, inside
 * one k, which is exactly the data-parallel reading of Eq. 1.
 * ---------------------------------------------------------------------- */
void oracle_fw_i32(int64_t n, int32_t *d, int64_t ld, int nthreads)
{
    for (int64_t k = 0; k < n; ++k) {
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t dik = d[i * ld + k];
            for (int64_t j = 0; j < n; ++j) {
                int64_t via = sat_add_i32(dik, d[k * ld + j]);
                if (via < d[i * ld + j]) d[i * ld + j] = (int32_t)via;
            }
        }
    }
}

/* Passes k0 .. k1-1 of the same recurrence, in place: after passes 0 .. k-1
 * from W, d[i][j] is the shortest i -> j distance over paths whose
 * intermediate vertices all lie below k (the invariant behind Eq. 1).  Used
 * to time a bounded sample of the full triple loop (every pass does exactly
 * n^2 updates). */
void oracle_fw_i32_steps(int64_t n, int32_t *d, int64_t ld, int64_t k0, int64_t k1, int nthreads)
{
    for (int64_t k = k0; k < k1 && k < n; ++k) {
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t dik = d[i * ld + k];
            for (int64_t j = 0; j < n; ++j) {
                int64_t via = sat_add_i32(dik, d[k * ld + j]);
                if (via < d[i * ld + j]) d[i * ld + j] = (int32_t)via;
            }
        }
    }
}

void oracle_fw_f64(int64_t n, double *d, int64_t ld, int nthreads)
{
    for (int64_t k = 0; k < n; ++k) {
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double dik = d[i * ld + k];
            for (int64_t j = 0; j < n; ++j) {
                double via = dik + d[k * ld + j];
                if (via < d[i * ld + j]) d[i * ld + j] = via;
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * O6: min-plus product (Sec. 3, Eq. 2), accumulating form:
 *   C[i][j] <- min(C[i][j], min_k (A[i][k] (+) B[k][j]))
 * With C pre-filled with INF this is exactly Eq. 2 (Z = X (min,+) Y).
 * A is m x k (lda), B is k x n (ldb), C is m x n (ldc), all row-major.
 * int32: saturating add in 64-bit.  fp32: each term is one IEEE binary32
 * addition (round to nearest even; C's float + float on x86-64/SSE rounds
 * once), and min is exact, so the result is unique.
 * ---------------------------------------------------------------------- */
void oracle_minplus_i32(int64_t m, int64_t n, int64_t kk,
                        const int32_t *A, int64_t lda,
                        const int32_t *B, int64_t ldb,
                        int32_t *C, int64_t ldc)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t best = C[i * ldc + j];
            for (int64_t k = 0; k < kk; ++k) {
                int64_t t = sat_add_i32(A[i * lda + k], B[k * ldb + j]);
                if (t < best) best = t;
            }
            C[i * ldc + j] = (int32_t)best;
        }
}

void oracle_minplus_f32(int64_t m, int64_t n, int64_t kk,
                        const float *A, int64_t lda,
                        const float *B, int64_t ldb,
                        float *C, int64_t ldc)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            float best = C[i * ldc + j];
            for (int64_t k = 0; k < kk; ++k) {
                float t = A[i * lda + k] + B[k * ldb + j];
                if (t < best) best = t;
            }
            C[i * ldc + j] = best;
        }
}

/* ------------------------------------------------------------------------
 * O2: Dijkstra's algorithm from a list of sources (binary heap with lazy
 * deletion).  Independent of Eq. 1: it is used to check the FW oracle and,
 * at large n, to check sampled rows of a GPU result.
 * Edges are the off-diagonal entries below INF (int32) or finite (float).
 * int32 weights: distances in int64, clamped to INF at the end (the
 * saturating reading above).  fp32 weights: promoted to double.
 * ---------------------------------------------------------------------- */
typedef struct { double key; int64_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *sz, double key, int64_t v)
{
    int64_t i = (*sz)++;
    h[i].key = key; h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, int64_t *sz)
{
    heap_item top = h[0];
    h[0] = h[--(*sz)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *sz && h[l].key < h[s].key) s = l;
        if (r < *sz && h[r].key < h[s].key) s = r;
        if (s == i) break;
        heap_item t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

/* Compressed adjacency built from the dense matrix (weights kept as double,
 * which represents every int32 weight and every binary32 weight exactly). */
typedef struct { int64_t *start; int64_t *to; double *w; } adjacency;

static int build_adjacency_i32(int64_t n, const int32_t *W, int64_t ld, adjacency *g)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (i != j && (int64_t)W[i * ld + j] < ORACLE_INF_I32) ++m;
    g->start = malloc(sizeof(int64_t) * (n + 1));
    g->to = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    g->w = malloc(sizeof(double) * (m > 0 ? m : 1));
    if (!g->start || !g->to || !g->w) return -1;
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        g->start[i] = e;
        for (int64_t j = 0; j < n; ++j)
            if (i != j && (int64_t)W[i * ld + j] < ORACLE_INF_I32) {
                g->to[e] = j; g->w[e] = (double)W[i * ld + j]; ++e;
            }
    }
    g->start[n] = e;
    return 0;
}

static int build_adjacency_f32(int64_t n, const float *W, int64_t ld, adjacency *g)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (i != j && isfinite(W[i * ld + j])) ++m;
    g->start = malloc(sizeof(int64_t) * (n + 1));
    g->to = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    g->w = malloc(sizeof(double) * (m > 0 ? m : 1));
    if (!g->start || !g->to || !g->w) return -1;
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        g->start[i] = e;
        for (int64_t j = 0; j < n; ++j)
            if (i != j && isfinite(W[i * ld + j])) {
                g->to[e] = j; g->w[e] = (double)W[i * ld + j]; ++e;
            }
    }
    g->start[n] = e;
    return 0;
}

static void free_adjacency(adjacency *g) { free(g->start); free(g->to); free(g->w); }

/* Single-source shortest paths; dist[v] = +inf when unreachable. */
static int dijkstra_one(int64_t n, const adjacency *g, int64_t src, double *dist)
{
    int64_t m = g->start[n];
    heap_item *h = malloc(sizeof(heap_item) * (m + 1));
    char *done = calloc(n, 1);
    if (!h || !done) { free(h); free(done); return -1; }
    for (int64_t v = 0; v < n; ++v) dist[v] = INFINITY;
    int64_t sz = 0;
    dist[src] = 0.0;
    heap_push(h, &sz, 0.0, src);
    while (sz > 0) {
        heap_item it = heap_pop(h, &sz);
        if (done[it.v]) continue;
        done[it.v] = 1;
        for (int64_t e = g->start[it.v]; e < g->start[it.v + 1]; ++e) {
            int64_t u = g->to[e];
            double nd = it.key + g->w[e];
            if (nd < dist[u]) { dist[u] = nd; heap_push(h, &sz, nd, u); }
        }
    }
    free(h); free(done);
    return 0;
}

/* out: nsrc x n int32 rows, min(distance, INF). Returns 0 on success. */
int oracle_dijkstra_i32(int64_t n, const int32_t *W, int64_t ld,
                        int64_t nsrc, const int64_t *src, int32_t *out, int nthreads)
{
    adjacency g;
    if (build_adjacency_i32(n, W, ld, &g)) { free_adjacency(&g); return -1; }
    int err = 0;
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 1) reduction(|:err)
    for (int64_t s = 0; s < nsrc; ++s) {
        double *dist = malloc(sizeof(double) * (n > 0 ? n : 1));
        if (!dist || dijkstra_one(n, &g, src[s], dist)) { err |= 1; free(dist); continue; }
        for (int64_t v = 0; v < n; ++v) {
            /* int32 weights are exact in double and every path sum here is
             * far below 2^53, so the double distance is the exact integer. */
            double d = dist[v];
            out[s * n + v] = (d >= (double)ORACLE_INF_I32) ? (int32_t)ORACLE_INF_I32 : (int32_t)d;
        }
        free(dist);
    }
    free_adjacency(&g);
    return err ? -1 : 0;
}

/* fp32 weights promoted to double; out: nsrc x n doubles (+inf unreachable). */
int oracle_dijkstra_f64(int64_t n, const float *W, int64_t ld,
                        int64_t nsrc, const int64_t *src, double *out, int nthreads)
{
    adjacency g;
    if (build_adjacency_f32(n, W, ld, &g)) { free_adjacency(&g); return -1; }
    int err = 0;
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 1) reduction(|:err)
    for (int64_t s = 0; s < nsrc; ++s) {
        if (dijkstra_one(n, &g, src[s], out + s * n)) err |= 1;
    }
    free_adjacency(&g);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * O5: Bellman optimality certificate for int32 APSP with weights >= 1.
 * D equals min(true distance, INF) exactly when
 *   (1) D[i][i] = 0 and 0 <= D[i][j] <= INF;
 *   (2) for every edge (i,k) and every j:  D[i][j] <= min(w_ik + D[k][j], INF);
 *   (3) every D[i][j] < INF with i != j has an edge (i,k) with
 *       w_ik + D[k][j] == D[i][j].
 * (2) bounds D above by every path length, (3) with strictly positive
 * weights follows tight edges along a strictly decreasing walk to j, which
 * bounds D below by a real walk length.  Rows [row0, row1) are checked;
 * the return value is the number of violated conditions (0 = certified).
 * ---------------------------------------------------------------------- */
int64_t oracle_certificate_i32(int64_t n, const int32_t *W, int64_t ldw,
                               const int32_t *D, int64_t ldd,
                               int64_t row0, int64_t row1, int nthreads)
{
    int64_t bad = 0;
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 1) reduction(+:bad)
    for (int64_t i = row0; i < row1; ++i) {
        char *tight = calloc(n > 0 ? n : 1, 1);
        if (!tight) { ++bad; continue; }
        if (D[i * ldd + i] != 0) ++bad;
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = D[i * ldd + j];
            if (v < 0 || v > ORACLE_INF_I32) ++bad;
        }
        for (int64_t k = 0; k < n; ++k) {
            int64_t w = W[i * ldw + k];
            if (k == i || w >= ORACLE_INF_I32) continue;
            for (int64_t j = 0; j < n; ++j) {
                int64_t via = sat_add_i32(w, D[k * ldd + j]);
                int64_t dij = D[i * ldd + j];
                if (dij > via) ++bad;
                if (dij < ORACLE_INF_I32 && w + (int64_t)D[k * ldd + j] == dij) tight[j] = 1;
            }
        }
        for (int64_t j = 0; j < n; ++j)
            if (j != i && (int64_t)D[i * ldd + j] < ORACLE_INF_I32 && !tight[j]) ++bad;
        free(tight);
    }
    return bad;
}

/* ------------------------------------------------------------------------
 * Last-hop predecessors (Sec. 2: pred[i][j] is the vertex before j on the
 * current i -> j path; Sec. 3.1 obtains it with an argmin over the
 * intermediate index).  Written out from that definition: for i != j,
 *   P[i][j] = the smallest v != j minimising D[i][v] (+) W[v][j]
 * provided that minimum is below INF; otherwise (i == j, or j unreachable)
 * P[i][j] = -1.  With D = APSP(W) and positive costs, W[v][j] is the last
 * edge of a shortest i -> j path exactly when D[i][v] + W[v][j] = D[i][j].
 * ---------------------------------------------------------------------- */
void oracle_predecessors_i32(int64_t n, const int32_t *D, int64_t ldd, const int32_t *W, int64_t ldw,
                             int32_t *P, int64_t ldp, int nthreads)
{
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t best = ORACLE_INF_I32;
            int64_t arg = -1;
            for (int64_t v = 0; v < n; ++v) {
                if (v == j) continue;
                int64_t t = sat_add_i32(D[i * ldd + v], W[v * ldw + j]);
                if (t < best) { best = t; arg = v; }
            }
            P[i * ldp + j] = (i == j || best >= ORACLE_INF_I32) ? -1 : (int32_t)arg;
        }
}
