/*
 * CPU oracle for the fork-processing pattern (FPP): plain, sequential
 * reference implementations of the single-source queries that an FPP launches
 * (Algorithm 1; Definition 2.2).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product library links or calls this file.  It shares no code with the GPU
 * path.
 *
 * Graph: directed multigraph in CSR (Section 2.1: an undirected graph is two
 * directed edges), row_ptr uint64[V+1], col uint32[E], weight uint32[E] or
 * NULL (unit weights).  Duplicate edges and self-loops are allowed.
 *
 * Queries follow the paper's three FPP query kinds (Section 3, supported
 * queries; Section 4.1 names the sequential algorithms it reuses):
 *   SSSP  - Dijkstra with a binary heap (lazy deletion); int32 distances,
 *           INT32_MAX = unreachable.
 *   BFS   - FIFO queue; int32 hop levels, INT32_MAX = unreachable.
 *   PPR   - sequential forward push in fp64, and fp64 power iteration for the
 *           exact personalised PageRank vector it approximates.
 * Multiple queries run one per OpenMP thread: the paper's inter-query
 * parallel baseline with one thread per query (Introduction, t = 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_INF 0x7fffffff

/* ------------------------------------------------------------ binary heap */
typedef struct { uint64_t key; uint32_t v; } hent;
typedef struct { hent *a; size_t n, cap; } heap;

static void hpush(heap *h, uint64_t key, uint32_t v) {
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (hent *)realloc(h->a, h->cap * sizeof(hent));
    }
    size_t i = h->n++;
    while (i > 0) {
        size_t par = (i - 1) / 2;
        if (h->a[par].key <= key) break;
        h->a[i] = h->a[par];
        i = par;
    }
    h->a[i].key = key;
    h->a[i].v = v;
}

static hent hpop(heap *h) {
    hent top = h->a[0];
    hent last = h->a[--h->n];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        uint64_t mk = last.key;
        if (l < h->n && h->a[l].key < mk) { m = l; mk = h->a[l].key; }
        if (r < h->n && h->a[r].key < mk) { m = r; }
        if (m == i) break;
        h->a[i] = h->a[m];
        i = m;
    }
    if (h->n) h->a[i] = last;
    return top;
}

/*
 * Dijkstra from src.  Returns 0, or -1 if a finite distance does not fit in
 * int32 (never the case for the workloads used here).  *relax_out (optional)
 * receives the number of edges scanned: the work of the sequential algorithm.
 */
int or_dijkstra(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                const uint32_t *w, uint32_t src, int32_t *dist_out,
                uint64_t *relax_out) {
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * nv);
    for (uint32_t v = 0; v < nv; ++v) d[v] = UINT64_MAX;
    heap h = {0};
    uint64_t scanned = 0;
    d[src] = 0;
    hpush(&h, 0, src);
    while (h.n) {
        hent t = hpop(&h);
        if (t.key != d[t.v]) continue; /* stale entry */
        for (uint64_t e = row_ptr[t.v]; e < row_ptr[t.v + 1]; ++e) {
            uint64_t nd = t.key + (w ? w[e] : 1u);
            uint32_t u = col[e];
            ++scanned;
            if (nd < d[u]) {
                d[u] = nd;
                hpush(&h, nd, u);
            }
        }
    }
    int rc = 0;
    for (uint32_t v = 0; v < nv; ++v) {
        if (d[v] == UINT64_MAX) dist_out[v] = OR_INF;
        else if (d[v] >= (uint64_t)OR_INF) { dist_out[v] = OR_INF; rc = -1; }
        else dist_out[v] = (int32_t)d[v];
    }
    if (relax_out) *relax_out = scanned;
    free(d);
    free(h.a);
    return rc;
}

/* BFS levels from src (FIFO queue). */
int or_bfs(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
           uint32_t src, int32_t *level_out, uint64_t *relax_out) {
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nv);
    for (uint32_t v = 0; v < nv; ++v) level_out[v] = OR_INF;
    size_t qh = 0, qt = 0;
    uint64_t scanned = 0;
    level_out[src] = 0;
    q[qt++] = src;
    while (qh < qt) {
        uint32_t v = q[qh++];
        int32_t nl = level_out[v] + 1;
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t u = col[e];
            ++scanned;
            if (level_out[u] == OR_INF) {
                level_out[u] = nl;
                q[qt++] = u;
            }
        }
    }
    if (relax_out) *relax_out = scanned;
    free(q);
    return 0;
}

/*
 * Sequential forward push for PPR (non-lazy), fp64, FIFO order.
 * A vertex u is active while r[u] > 0 and r[u] >= thr(u), where
 * thr(u) = eps (mode 0, absolute) or eps * outdeg(u) (mode 1, degree-scaled).
 * Pushing u: p[u] += alpha*r[u]; every out-edge (u,v) gets
 * (1-alpha)*r[u]/outdeg(u) added to r[v] (once per parallel edge); r[u] = 0.
 * At a vertex without out-edges the (1-alpha) share is dropped, matching the
 * substochastic walk used by or_ppr_power.  *pushes_out receives the number
 * of edge pushes performed.
 */
int or_forward_push(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                    uint32_t src, double alpha, double eps, int mode,
                    double *p, double *r, uint64_t *pushes_out) {
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nv);
    unsigned char *inq = (unsigned char *)calloc(nv, 1);
    memset(p, 0, sizeof(double) * nv);
    memset(r, 0, sizeof(double) * nv);
    size_t head = 0, count = 0; /* ring of at most nv entries */
    uint64_t pushes = 0;
    r[src] = 1.0;
#define THR(u) (mode ? eps * (double)(row_ptr[(u) + 1] - row_ptr[(u)]) : eps)
    if (r[src] >= THR(src)) {
        q[0] = src;
        count = 1;
        inq[src] = 1;
    }
    while (count) {
        uint32_t u = q[head];
        head = (head + 1) % nv;
        --count;
        inq[u] = 0;
        double m = r[u];
        if (!(m > 0.0 && m >= THR(u))) continue;
        r[u] = 0.0;
        p[u] += alpha * m;
        uint64_t deg = row_ptr[u + 1] - row_ptr[u];
        if (deg == 0) continue;
        double share = (1.0 - alpha) * m / (double)deg;
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t v = col[e];
            r[v] += share;
            ++pushes;
            if (!inq[v] && r[v] >= THR(v)) {
                q[(head + count) % nv] = v;
                ++count;
                inq[v] = 1;
            }
        }
    }
#undef THR
    if (pushes_out) *pushes_out = pushes;
    free(q);
    free(inq);
    return 0;
}

/*
 * Personalised PageRank by power iteration, fp64:
 *   pi = alpha * sum_k ((1-alpha) P^T)^k x0,  P = D_out^{-1} A (rows of
 *   dangling vertices are zero),
 * for an arbitrary start vector x0 (x0 = e_s gives PPR(s); by linearity
 * x0 = e_s - r gives PPR(e_s) - PPR(r)).  Iterates until the L1 norm of the
 * current term is below tol, which bounds the dropped tail.  Returns the
 * number of iterations.
 */
int or_ppr_power(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                 double alpha, const double *x0, double tol, int max_iter,
                 double *pi) {
    double *y = (double *)malloc(sizeof(double) * nv);
    double *z = (double *)malloc(sizeof(double) * nv);
    memcpy(y, x0, sizeof(double) * nv);
    memset(pi, 0, sizeof(double) * nv);
    int it = 0;
    for (; it < max_iter; ++it) {
        double norm = 0.0;
        for (uint32_t v = 0; v < nv; ++v) {
            pi[v] += alpha * y[v];
            norm += fabs(y[v]);
        }
        if (norm < tol) break;
        memset(z, 0, sizeof(double) * nv);
        for (uint32_t u = 0; u < nv; ++u) {
            if (y[u] == 0.0) continue;
            uint64_t deg = row_ptr[u + 1] - row_ptr[u];
            if (deg == 0) continue;
            double share = (1.0 - alpha) * y[u] / (double)deg;
            for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) z[col[e]] += share;
        }
        double *t = y; y = z; z = t;
    }
    free(y);
    free(z);
    return it;
}

/*
 * Optimality certificate for single-source shortest distances with positive
 * integer weights (unit weights when w == NULL, i.e. BFS levels):
 *   d[src] = 0;  for every edge (u,v,w) with d[u] finite: d[v] <= d[u] + w;
 *   every v != src with finite d[v] has an in-edge (u,v,w) with
 *   d[u] + w == d[v].
 * With w >= 1 these three facts hold only for the exact distance vector.
 * Returns 0 when the certificate holds, otherwise a positive code naming the
 * first violated condition (1, 2 or 3).
 */
int or_sp_certificate(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                      const uint32_t *w, uint32_t src, const int32_t *d) {
    if (d[src] != 0) return 1;
    unsigned char *wit = (unsigned char *)calloc(nv, 1);
    int rc = 0;
    for (uint32_t u = 0; u < nv && !rc; ++u) {
        if (d[u] == OR_INF) continue;
        if (d[u] < 0) { rc = 2; break; }
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t nd = (int64_t)d[u] + (int64_t)(w ? w[e] : 1u);
            uint32_t v = col[e];
            int64_t dv = d[v] == OR_INF ? INT64_MAX : (int64_t)d[v];
            if (dv > nd) { rc = 2; break; }
            if (dv == nd) wit[v] = 1;
        }
    }
    for (uint32_t v = 0; v < nv && !rc; ++v)
        if (v != src && d[v] != OR_INF && !wit[v]) rc = 3;
    free(wit);
    return rc;
}

/* ------------------------------------------------- many queries (t = 1) */
int or_sssp_many(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                 const uint32_t *w, uint32_t nsrc, const uint32_t *srcs,
                 int32_t *out, uint64_t *relax, int nthreads) {
    int rc = 0;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(|:rc)
    for (int64_t i = 0; i < (int64_t)nsrc; ++i)
        rc |= or_dijkstra(nv, row_ptr, col, w, srcs[i], out + (size_t)i * nv,
                          relax ? relax + i : NULL);
    return rc;
}

int or_bfs_many(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                uint32_t nsrc, const uint32_t *srcs, int32_t *out,
                uint64_t *relax, int nthreads) {
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < (int64_t)nsrc; ++i)
        or_bfs(nv, row_ptr, col, srcs[i], out + (size_t)i * nv, relax ? relax + i : NULL);
    return 0;
}

int or_push_many(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                 uint32_t nsrc, const uint32_t *srcs, double alpha, double eps,
                 int mode, double *p, double *r, uint64_t *pushes, int nthreads) {
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < (int64_t)nsrc; ++i)
        or_forward_push(nv, row_ptr, col, srcs[i], alpha, eps, mode,
                        p + (size_t)i * nv, r + (size_t)i * nv,
                        pushes ? pushes + i : NULL);
    return 0;
}

int or_ppr_power_many(uint32_t nv, const uint64_t *row_ptr, const uint32_t *col,
                      double alpha, uint32_t nvec, const double *x0, double tol,
                      int max_iter, double *pi, int nthreads) {
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < (int64_t)nvec; ++i)
        or_ppr_power(nv, row_ptr, col, alpha, x0 + (size_t)i * nv, tol, max_iter,
                     pi + (size_t)i * nv);
    return 0;
}
