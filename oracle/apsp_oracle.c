/*
 * Host oracle for all-pairs shortest-path lengths (Schoeneman & Zola,
 * "Solving All-Pairs Shortest-Paths Problem in Large Graphs Using Apache
 * Spark", arXiv:1902.04446).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * Problem (paper Sec. 3, Preliminaries): an undirected weighted graph with no
 * negative cycles, vertices indexed 0..n-1, adjacency matrix A with
 * A_ij = A_ji = w_ij; the output is the length (only) of a shortest path
 * between every pair.  Because the graph is undirected, a negative edge would
 * itself be a negative cycle (u->v->u), so every weight is >= 0.
 *
 * Representation used here (the paper names no element type or sentinel):
 *   int32 input  : entries in [0, 2^30]; 2^30 (or anything above it) means
 *                  "no edge".  Computed in int64, so no sum can overflow;
 *                  final lengths >= 2^30 are reported as 2^30.
 *   fp32 input   : entries in [0, +inf]; +inf means "no edge".  Computed in
 *                  fp64 (every fp32 value converts exactly).
 *   diagonal     : the empty path, length 0, whatever the input holds.
 *
 * Functions and the passage each follows:
 *   orc_fw_steps_i64 / _f64   classic Floyd-Warshall (Sec. 3 cites the
 *                             textbook algorithm; Table 1 FloydWarshall)
 *   orc_apsp_i32 / _f32       input normalisation + the triple loop above
 *   orc_dijkstra_csr_*        Dijkstra from chosen sources, an independent
 *                             algorithm for the same definition (Sec. 3
 *                             names the textbook APSP alternatives)
 *   orc_brute_*               minimum over all simple paths (definition
 *                             itself; tiny n only)
 *   orc_blocked_u32 / _f32    the three-phase blocked method (Sec. 4.4 and
 *                             Sec. 4.5, Algorithms 3 and 4; Table 1 MinPlus,
 *                             MatProd, MatMin) in the element type of the
 *                             device path, with phase products taken on the
 *                             values before the phase starts
 *   orc_minplus_*             the min-plus product of Table 1 (MatProd)
 *   orc_squaring_*            repeated min-plus squaring (Sec. 4.2,
 *                             Algorithm 1) in the device element type
 *   orc_bellman_*             Bellman optimality residual, a certificate that
 *                             characterises the distance matrix when w > 0
 *
 * Mutation hooks: compiling with -DORC_MUTANT=<m> plants one plausible
 * mistake in the Floyd-Warshall triple loop (see orc_fw_steps_*).  The test
 * suite builds such variants to show that its pins catch them; the default
 * build has ORC_MUTANT = 0 and no mistake.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

#define ORC_INF_I64 ((int64_t)1 << 30)

int orc_mutant(void) { return ORC_MUTANT; }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Classic Floyd-Warshall, steps k0..k1-1, on a dense row-major n x n matrix. */
/* Row k and column k do not change during step k when D_kk = 0 and all     */
/* entries are >= 0, so the rows i may be split over threads.               */
/* ------------------------------------------------------------------------ */
void orc_fw_steps_i64(int64_t *D, int64_t n, int64_t k0, int64_t k1, int threads)
{
    if (threads < 1) threads = 1;
#if ORC_MUTANT == 3
    if (k1 > k0) k1 -= 1; /* mutant: last pivot skipped */
#endif
    for (int64_t k = k0; k < k1; ++k) {
        const int64_t *rowk = D + k * n;
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t *rowi = D + i * n;
#if ORC_MUTANT == 1
            const int64_t dik = D[k * n + i]; /* mutant: transposed operand */
#else
            const int64_t dik = rowi[k];
#endif
            for (int64_t j = 0; j < n; ++j) {
#if ORC_MUTANT == 2
                const int64_t c = dik + rowk[j] + 1; /* mutant: spurious term */
#else
                const int64_t c = dik + rowk[j];
#endif
                if (c < rowi[j]) rowi[j] = c;
            }
        }
    }
}

void orc_fw_steps_f64(double *D, int64_t n, int64_t k0, int64_t k1, int threads)
{
    if (threads < 1) threads = 1;
#if ORC_MUTANT == 3
    if (k1 > k0) k1 -= 1;
#endif
    for (int64_t k = k0; k < k1; ++k) {
        const double *rowk = D + k * n;
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double *rowi = D + i * n;
#if ORC_MUTANT == 1
            const double dik = D[k * n + i];
#else
            const double dik = rowi[k];
#endif
            for (int64_t j = 0; j < n; ++j) {
#if ORC_MUTANT == 2
                const double c = dik + rowk[j] + 1.0;
#else
                const double c = dik + rowk[j];
#endif
                if (c < rowi[j]) rowi[j] = c;
            }
        }
    }
}

/* Loop order k innermost is the classic wrong Floyd-Warshall; it is only   */
/* reachable as mutant 4 and exists so the pins can be shown to catch it.   */
#if ORC_MUTANT == 4
static void orc_wrong_order_i64(int64_t *D, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t k = 0; k < n; ++k) {
                const int64_t c = D[i * n + k] + D[k * n + j];
                if (c < D[i * n + j]) D[i * n + j] = c;
            }
}
static void orc_wrong_order_f64(double *D, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t k = 0; k < n; ++k) {
                const double c = D[i * n + k] + D[k * n + j];
                if (c < D[i * n + j]) D[i * n + j] = c;
            }
}
#endif

/* Input normalisation for the int32 representation: copy, map entries at  */
/* or above 2^30 to 2^30, set the diagonal to 0.                            */
void orc_prepare_i32(const int32_t *W, int64_t n, int64_t ldw, int64_t *D)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = W[i * ldw + j];
            if (v > ORC_INF_I64) v = ORC_INF_I64;
            D[i * n + j] = v;
        }
#if ORC_MUTANT != 5
    for (int64_t i = 0; i < n; ++i) D[i * n + i] = 0;
#endif
}

void orc_prepare_f32(const float *W, int64_t n, int64_t ldw, double *D)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) D[i * n + j] = (double)W[i * ldw + j];
#if ORC_MUTANT != 5
    for (int64_t i = 0; i < n; ++i) D[i * n + i] = 0.0;
#endif
}

void orc_clamp_i64(int64_t *D, int64_t count)
{
    for (int64_t t = 0; t < count; ++t)
        if (D[t] > ORC_INF_I64) D[t] = ORC_INF_I64;
}

/* Full APSP: int32 weights in, int64 lengths out (n x n, dense). */
void orc_apsp_i32(const int32_t *W, int64_t n, int64_t ldw, int64_t *D, int threads)
{
    orc_prepare_i32(W, n, ldw, D);
#if ORC_MUTANT == 4
    (void)threads;
    orc_wrong_order_i64(D, n);
#else
    orc_fw_steps_i64(D, n, 0, n, threads);
#endif
    orc_clamp_i64(D, n * n);
}

/* Full APSP: fp32 weights in, fp64 lengths out. */
void orc_apsp_f32(const float *W, int64_t n, int64_t ldw, double *D, int threads)
{
    orc_prepare_f32(W, n, ldw, D);
#if ORC_MUTANT == 4
    (void)threads;
    orc_wrong_order_f64(D, n);
#else
    orc_fw_steps_f64(D, n, 0, n, threads);
#endif
}

/* ------------------------------------------------------------------------ */
/* Dijkstra from a list of sources over a CSR adjacency (both directions of */
/* every undirected edge present).  Binary heap with lazy deletion.         */
/* ------------------------------------------------------------------------ */
typedef struct { double key; int64_t v; } orc_hent;

static void heap_push(orc_hent *h, int64_t *sz, double key, int64_t v)
{
    int64_t c = (*sz)++;
    h[c].key = key; h[c].v = v;
    while (c > 0) {
        int64_t p = (c - 1) / 2;
        if (h[p].key <= h[c].key) break;
        orc_hent t = h[p]; h[p] = h[c]; h[c] = t;
        c = p;
    }
}

static orc_hent heap_pop(orc_hent *h, int64_t *sz)
{
    orc_hent top = h[0];
    h[0] = h[--(*sz)];
    int64_t c = 0;
    for (;;) {
        int64_t l = 2 * c + 1, r = l + 1, m = c;
        if (l < *sz && h[l].key < h[m].key) m = l;
        if (r < *sz && h[r].key < h[m].key) m = r;
        if (m == c) break;
        orc_hent t = h[m]; h[m] = h[c]; h[c] = t;
        c = m;
    }
    return top;
}

/* Core: weights in double (exact for int32 and fp32 inputs; int sums stay  */
/* below 2^53 for any n here, so the int path is exact too).                */
static void dijkstra_one(const int64_t *indptr, const int64_t *indices, const double *w,
                         int64_t n, int64_t s, double *dist, orc_hent *heap, char *done)
{
    for (int64_t v = 0; v < n; ++v) { dist[v] = INFINITY; done[v] = 0; }
    int64_t sz = 0;
    dist[s] = 0.0;
    heap_push(heap, &sz, 0.0, s);
    while (sz > 0) {
        orc_hent e = heap_pop(heap, &sz);
        if (done[e.v]) continue;
        done[e.v] = 1;
        for (int64_t t = indptr[e.v]; t < indptr[e.v + 1]; ++t) {
            const int64_t u = indices[t];
            const double c = e.key + w[t];
            if (c < dist[u]) { dist[u] = c; heap_push(heap, &sz, c, u); }
        }
    }
}

/* fp64 lengths; +inf where unreachable. */
void orc_dijkstra_csr_f64(const int64_t *indptr, const int64_t *indices, const double *w,
                          int64_t n, const int64_t *src, int64_t nsrc, double *out, int threads)
{
    if (threads < 1) threads = 1;
#pragma omp parallel num_threads(threads)
    {
        const int64_t nnz = indptr[n];
        orc_hent *heap = (orc_hent *)malloc(sizeof(orc_hent) * (size_t)(nnz + n + 1));
        char *done = (char *)malloc((size_t)n + 1);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < nsrc; ++t)
            dijkstra_one(indptr, indices, w, n, src[t], out + t * n, heap, done);
        free(heap);
        free(done);
    }
}

/* int64 lengths from integer weights; lengths >= 2^30 reported as 2^30.   */
void orc_dijkstra_csr_i64(const int64_t *indptr, const int64_t *indices, const int64_t *wi,
                          int64_t n, const int64_t *src, int64_t nsrc, int64_t *out, int threads)
{
    const int64_t nnz = indptr[n];
    double *w = (double *)malloc(sizeof(double) * (size_t)(nnz + 1));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(nsrc * n + 1));
    for (int64_t t = 0; t < nnz; ++t) w[t] = (double)wi[t];
    orc_dijkstra_csr_f64(indptr, indices, w, n, src, nsrc, tmp, threads);
    for (int64_t t = 0; t < nsrc * n; ++t) {
        const double d = tmp[t];
        out[t] = (d >= (double)ORC_INF_I64) ? ORC_INF_I64 : (int64_t)d;
    }
    free(w);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Brute force: minimum weight over all simple paths s -> t (n <= 10).     */
/* With non-negative weights a shortest walk can be shortened to a simple  */
/* path, so this is the definition itself.  W is a dense n x n matrix in   */
/* double with +inf for "no edge"; the diagonal of W is ignored.           */
/* ------------------------------------------------------------------------ */
static void brute_dfs(const double *W, int64_t n, int64_t v, int64_t t, double len,
                      uint32_t visited, double *best)
{
    if (v == t) { if (len < *best) *best = len; return; }
    for (int64_t u = 0; u < n; ++u) {
        if (u == v || (visited >> u) & 1u) continue;
        const double w = W[v * n + u];
        if (isinf(w)) continue;
        brute_dfs(W, n, u, t, len + w, visited | (1u << u), best);
    }
}

int orc_brute_f64(const double *W, int64_t n, double *out)
{
    if (n > 10) return -1;
    for (int64_t s = 0; s < n; ++s)
        for (int64_t t = 0; t < n; ++t) {
            double best = INFINITY;
            if (s == t) best = 0.0;
            else brute_dfs(W, n, s, t, 0.0, 1u << s, &best);
            out[s * n + t] = best;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Min-plus product (Table 1, MatProd): C_ij = min_k A_ik + B_kj, and the   */
/* fused MatMin of MinPlus: C_ij = min(C_ij, min_k A_ik + B_kj).            */
/* ------------------------------------------------------------------------ */
void orc_minplus_acc_f32(const float *A, int64_t lda, const float *B, int64_t ldb,
                         float *C, int64_t ldc, int64_t m, int64_t nn, int64_t kk)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < nn; ++j) {
            float best = C[i * ldc + j];
            for (int64_t k = 0; k < kk; ++k) {
                const float c = A[i * lda + k] + B[k * ldb + j];
                if (c < best) best = c;
            }
            C[i * ldc + j] = best;
        }
}

void orc_minplus_acc_u32(const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
                         uint32_t *C, int64_t ldc, int64_t m, int64_t nn, int64_t kk)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < nn; ++j) {
            uint32_t best = C[i * ldc + j];
            for (int64_t k = 0; k < kk; ++k) {
                const uint32_t c = A[i * lda + k] + B[k * ldb + j];
                if (c < best) best = c;
            }
            C[i * ldc + j] = best;
        }
}

/* ------------------------------------------------------------------------ */
/* Repeated squaring (Sec. 4.2, Algorithm 1): X <- X (x) X, `steps` times,  */
/* on a prepared n x n matrix (diagonal 0).  Each product is taken whole    */
/* into a temporary (every entry from the same X), then copied back.        */
/* ------------------------------------------------------------------------ */
#define ORC_SQUARING_BODY(T)                                                    \
    T *Y = (T *)malloc(sizeof(T) * (size_t)(n * n + 1));                       \
    for (int64_t st = 0; st < steps; ++st) {                                   \
        for (int64_t i = 0; i < n; ++i)                                        \
            for (int64_t j = 0; j < n; ++j) {                                  \
                T best = X[i * n + 0] + X[0 * n + j];                          \
                for (int64_t k = 1; k < n; ++k) {                              \
                    const T c = X[i * n + k] + X[k * n + j];                   \
                    if (c < best) best = c;                                    \
                }                                                              \
                Y[i * n + j] = best;                                           \
            }                                                                  \
        memcpy(X, Y, sizeof(T) * (size_t)(n * n));                             \
    }                                                                          \
    free(Y);

void orc_squaring_u32(uint32_t *X, int64_t n, int64_t steps)
{
    if (n < 1) return;
    ORC_SQUARING_BODY(uint32_t)
}

void orc_squaring_f32(float *X, int64_t n, int64_t steps)
{
    if (n < 1) return;
    ORC_SQUARING_BODY(float)
}

/* ------------------------------------------------------------------------ */
/* Three-phase blocked Floyd-Warshall (Sec. 4.4/4.5, Algorithms 3 and 4),  */
/* rounds r0..r1-1 with round width b, in place on a prepared n x n matrix */
/* (diagonal 0, every entry in [0, 2^30] for the integer form).            */
/*                                                                         */
/* Round r, K = [r*b, min(r*b+b, n)):                                      */
/*  phase 1  Floyd-Warshall on the diagonal block D[K,K] (Table 1,         */
/*           FloydWarshall), pivots k in K ascending;                      */
/*  phase 2  row panel    D[K,j] = min(D[K,j], (D[K,K] (x) D[K,j])) and    */
/*           column panel D[i,K] = min(D[i,K], (D[i,K] (x) D[K,K])) for    */
/*           i, j outside K (MinPlus = MatProd then MatMin); the product   */
/*           reads the panel as it was when phase 2 began;                 */
/*  phase 3  D[i,j] = min(D[i,j], (D[i,K] (x) D[K,j])) for i, j outside K  */
/*           (ListUnpack pairs the column-panel block of block-row I with  */
/*           the row-panel block of block-column J).                       */
/* Because phase 2 and 3 products are taken element by element, how the    */
/* columns outside K are grouped into blocks does not change the result.   */
/* The integer form computes in uint32: every entry stays <= 2^30, so a    */
/* sum of two is <= 2^31 and cannot wrap.                                  */
/* ------------------------------------------------------------------------ */
#define ORC_BLOCKED_BODY(T)                                                         \
    for (int64_t r = r0; r < r1; ++r) {                                             \
        const int64_t kb = r * b;                                                   \
        if (kb >= n) break;                                                         \
        const int64_t ke = (kb + b < n) ? kb + b : n;                               \
        const int64_t w = ke - kb;                                                  \
        /* phase 1 */                                                               \
        for (int64_t k = kb; k < ke; ++k)                                           \
            for (int64_t i = kb; i < ke; ++i)                                       \
                for (int64_t j = kb; j < ke; ++j) {                                 \
                    const T c = D[i * n + k] + D[k * n + j];                        \
                    if (c < D[i * n + j]) D[i * n + j] = c;                         \
                }                                                                   \
        /* phase 2, row panel: old copy of rows K, then product with D[K,K] */      \
        T *rows = (T *)malloc(sizeof(T) * (size_t)(w * n));                         \
        memcpy(rows, D + kb * n, sizeof(T) * (size_t)(w * n));                      \
        for (int64_t i = kb; i < ke; ++i)                                           \
            for (int64_t j = 0; j < n; ++j) {                                       \
                if (j >= kb && j < ke) continue;                                    \
                T best = rows[(i - kb) * n + j];                                    \
                for (int64_t k = kb; k < ke; ++k) {                                 \
                    const T c = D[i * n + k] + rows[(k - kb) * n + j];              \
                    if (c < best) best = c;                                         \
                }                                                                   \
                D[i * n + j] = best;                                                \
            }                                                                       \
        free(rows);                                                                 \
        /* phase 2, column panel: old copy of columns K */                          \
        T *cols = (T *)malloc(sizeof(T) * (size_t)(n * w));                         \
        for (int64_t i = 0; i < n; ++i)                                             \
            for (int64_t k = kb; k < ke; ++k) cols[i * w + (k - kb)] = D[i * n + k]; \
        for (int64_t i = 0; i < n; ++i) {                                           \
            if (i >= kb && i < ke) continue;                                        \
            for (int64_t j = kb; j < ke; ++j) {                                     \
                T best = cols[i * w + (j - kb)];                                    \
                for (int64_t k = kb; k < ke; ++k) {                                 \
                    const T c = cols[i * w + (k - kb)] + D[k * n + j];              \
                    if (c < best) best = c;                                         \
                }                                                                   \
                D[i * n + j] = best;                                                \
            }                                                                       \
        }                                                                           \
        free(cols);                                                                 \
        /* phase 3: operands are panel entries, which phase 3 does not write */     \
        for (int64_t i = 0; i < n; ++i) {                                           \
            if (i >= kb && i < ke) continue;                                        \
            for (int64_t j = 0; j < n; ++j) {                                       \
                if (j >= kb && j < ke) continue;                                    \
                T best = D[i * n + j];                                              \
                for (int64_t k = kb; k < ke; ++k) {                                 \
                    const T c = D[i * n + k] + D[k * n + j];                        \
                    if (c < best) best = c;                                         \
                }                                                                   \
                D[i * n + j] = best;                                                \
            }                                                                       \
        }                                                                           \
    }

void orc_blocked_u32(uint32_t *D, int64_t n, int64_t b, int64_t r0, int64_t r1)
{
    if (b < 1) return;
    ORC_BLOCKED_BODY(uint32_t)
}

void orc_blocked_f32(float *D, int64_t n, int64_t b, int64_t r0, int64_t r1)
{
    if (b < 1) return;
    ORC_BLOCKED_BODY(float)
}

/* ------------------------------------------------------------------------ */
/* Bellman certificate.  For w > 0 and D_ii = 0, the shortest-path matrix  */
/* is the unique matrix with D_ij = min over neighbours k of i of          */
/* (w_ik + D_kj) for every i != j.  Over the given rows, returns the       */
/* largest relative residual |D_ij - min_k(w_ik + D_kj)| / D_ij (inf       */
/* entries must match exactly: a mismatch returns +inf), computed in fp64. */
/* D is fp32 with leading dimension ldd; the graph is a CSR (both          */
/* directions).                                                             */
/* ------------------------------------------------------------------------ */
double orc_bellman_residual_f32(const float *D, int64_t ldd, int64_t n, const int64_t *indptr,
                                const int64_t *indices, const double *w, const int64_t *rows,
                                int64_t nrows, int threads)
{
    double worst = 0.0;
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) reduction(max : worst) schedule(dynamic, 4)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            const double dij = (double)D[i * ldd + j];
            if (j == i) {
                if (dij != 0.0) worst = INFINITY;
                continue;
            }
            double best = INFINITY;
            for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
                const double c = w[e] + (double)D[indices[e] * ldd + j];
                if (c < best) best = c;
            }
            double res;
            if (isinf(best) || isinf(dij)) res = (isinf(best) && isinf(dij)) ? 0.0 : INFINITY;
            else res = fabs(dij - best) / (dij > 0 ? dij : 1.0);
            if (res > worst) worst = res;
        }
    }
    return worst;
}

/* Integer form: number of entries (over the given rows) that violate the  */
/* certificate exactly, with sums saturated at 2^30.                        */
int64_t orc_bellman_violations_i32(const int32_t *D, int64_t ldd, int64_t n, const int64_t *indptr,
                                   const int64_t *indices, const int64_t *w, const int64_t *rows,
                                   int64_t nrows, int threads)
{
    int64_t bad = 0;
    if (threads < 1) threads = 1;
#pragma omp parallel for num_threads(threads) reduction(+ : bad) schedule(dynamic, 4)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int64_t j = 0; j < n; ++j) {
            const int64_t dij = D[i * ldd + j];
            if (j == i) { bad += (dij != 0); continue; }
            int64_t best = ORC_INF_I64;
            for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
                int64_t c = w[e] + (int64_t)D[indices[e] * ldd + j];
                if (c > ORC_INF_I64) c = ORC_INF_I64;
                if (c < best) best = c;
            }
            bad += (best != dij);
        }
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Rows of the Floyd-Warshall state after the first K pivots (Sec. 3: the  */
/* classic loop stopped after k = 0 .. K-1; a blocked solver reaches this   */
/* state after K / b rounds), for a graph given as adjacency lists, so no   */
/* n x n matrix is needed.  Entry (i, j) of that state is the least length  */
/* over i -> j paths whose intermediate vertices all lie in {0 .. K-1}.     */
/* Such a path is the edge (i, j) itself, or                                */
/*     edge i -> a,  a shortest a -> b path inside {0 .. K-1},  edge b -> j */
/* with a, b < K, where a = i (i < K) and b = j (j < K) stand for the      */
/* empty first or last edge.  The a -> b lengths come from the classic      */
/* loop on the subgraph induced by {0 .. K-1}.  fp64; +inf = no path.       */
/* ------------------------------------------------------------------------ */
void orc_fw_prefix_rows_f64(const int64_t *indptr, const int64_t *indices, const double *w,
                            int64_t n, int64_t K, const int64_t *rows, int64_t nrows, double *out,
                            int threads)
{
    if (threads < 1) threads = 1;
    if (K > n) K = n;
    double *dk = (double *)malloc(sizeof(double) * (size_t)(K * K + 1));
    for (int64_t t = 0; t < K * K; ++t) dk[t] = INFINITY;
    for (int64_t a = 0; a < K; ++a) {
        dk[a * K + a] = 0.0;
        for (int64_t e = indptr[a]; e < indptr[a + 1]; ++e) {
            const int64_t b = indices[e];
            if (b < K && b != a && w[e] < dk[a * K + b]) dk[a * K + b] = w[e];
        }
    }
    for (int64_t k = 0; k < K; ++k)
        for (int64_t a = 0; a < K; ++a) {
            const double dak = dk[a * K + k];
            for (int64_t b = 0; b < K; ++b) {
                const double c = dak + dk[k * K + b];
                if (c < dk[a * K + b]) dk[a * K + b] = c;
            }
        }
#pragma omp parallel num_threads(threads)
    {
        double *tb = (double *)malloc(sizeof(double) * (size_t)(K + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < nrows; ++t) {
            const int64_t i = rows[t];
            double *o = out + t * n;
            for (int64_t j = 0; j < n; ++j) o[j] = INFINITY;
            o[i] = 0.0;
            for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
                if (indices[e] != i && w[e] < o[indices[e]]) o[indices[e]] = w[e];
            /* tb[b]: least i -> b length with every vertex after i in {0..K-1} */
            for (int64_t b = 0; b < K; ++b) tb[b] = (i < K) ? dk[i * K + b] : INFINITY;
            for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
                const int64_t a = indices[e];
                if (a >= K || a == i) continue;
                for (int64_t b = 0; b < K; ++b) {
                    const double c = w[e] + dk[a * K + b];
                    if (c < tb[b]) tb[b] = c;
                }
            }
            for (int64_t b = 0; b < K; ++b) {
                if (isinf(tb[b])) continue;
                if (tb[b] < o[b]) o[b] = tb[b];
                for (int64_t e = indptr[b]; e < indptr[b + 1]; ++e) {
                    const int64_t j = indices[e];
                    const double c = tb[b] + w[e];
                    if (j != i && c < o[j]) o[j] = c;
                }
            }
        }
        free(tb);
    }
    free(dk);
}
