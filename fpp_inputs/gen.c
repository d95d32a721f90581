/*
 * Seeded synthetic workload generators: R-MAT edge lists, 2D grid graphs,
 * integer edge weights, and a stable counting-sort CSR builder.
 *
 * This file holds no part of the fork-processing method: it only produces the
 * graphs that both the CPU oracle and the GPU path consume.  All randomness
 * comes from one counter-based generator (the SplitMix64 finaliser of Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014), so edge i of a graph is the same whatever the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Counter-based draw: stream `seed`, counter `ctr`. */
static inline uint64_t draw(uint64_t seed, uint64_t ctr) {
    return mix64(mix64(seed) ^ (ctr * 0xD1B54A32D192ED03ull));
}

/* uniform double in [0,1) with 53 random bits */
static inline double unif(uint64_t seed, uint64_t ctr) {
    return (double)(draw(seed, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): for each of `ne` edges choose one
 * quadrant per bit level with probabilities (a, b, c, 1-a-b-c), most
 * significant bit first, no noise.  Row bit -> source, column bit -> target.
 */
void fi_rmat_edges(int scale, uint64_t ne, double a, double b, double c,
                   uint64_t seed, uint32_t *src, uint32_t *dst) {
    const double ab = a + b, abc = a + b + c;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)ne; ++i) {
        uint32_t s = 0, t = 0;
        for (int l = 0; l < scale; ++l) {
            double u = unif(seed, (uint64_t)i * 64u + (uint64_t)l);
            uint32_t rb, cb;
            if (u < a) { rb = 0; cb = 0; }
            else if (u < ab) { rb = 0; cb = 1; }
            else if (u < abc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            s = (s << 1) | rb;
            t = (t << 1) | cb;
        }
        src[i] = s;
        dst[i] = t;
    }
}

/* Integer weights uniform on [lo, hi] (inclusive), one per counter value,
 * by Lemire's multiply-shift range reduction of a 32-bit draw. */
void fi_uniform_weights(uint64_t n, uint32_t lo, uint32_t hi, uint64_t seed,
                        const uint64_t *ctr_of /* may be NULL: counter = index */,
                        uint32_t *out) {
    const uint64_t range = (uint64_t)hi - (uint64_t)lo + 1u;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t ctr = ctr_of ? ctr_of[i] : (uint64_t)i;
        uint64_t r32 = draw(seed, ctr) >> 32;
        out[i] = lo + (uint32_t)((r32 * range) >> 32);
    }
}

/*
 * 4-neighbour grid of rows x cols vertices, id = r*cols + c, both directions
 * of every undirected edge.  Writes the CSR directly (neighbours in the order
 * up, left, right, down, i.e. ascending id) and, for each directed edge, the
 * id of its undirected edge so that both directions can share one weight.
 */
void fi_grid_csr(uint32_t rows, uint32_t cols, uint64_t *row_ptr,
                 uint32_t *col, uint64_t *undirected_id) {
    const uint64_t nh = (uint64_t)rows * (cols - 1u); /* horizontal edges */
    uint64_t e = 0;
    row_ptr[0] = 0;
    for (uint32_t r = 0; r < rows; ++r) {
        for (uint32_t c = 0; c < cols; ++c) {
            uint64_t v = (uint64_t)r * cols + c;
            if (r > 0) { /* vertical edge between (r-1,c) and (r,c) */
                col[e] = (uint32_t)(v - cols);
                undirected_id[e] = nh + (uint64_t)(r - 1) * cols + c;
                ++e;
            }
            if (c > 0) { /* horizontal edge between (r,c-1) and (r,c) */
                col[e] = (uint32_t)(v - 1);
                undirected_id[e] = (uint64_t)r * (cols - 1u) + (c - 1);
                ++e;
            }
            if (c + 1 < cols) {
                col[e] = (uint32_t)(v + 1);
                undirected_id[e] = (uint64_t)r * (cols - 1u) + c;
                ++e;
            }
            if (r + 1 < rows) {
                col[e] = (uint32_t)(v + cols);
                undirected_id[e] = nh + (uint64_t)r * cols + c;
                ++e;
            }
            row_ptr[v + 1] = e;
        }
    }
}

/*
 * Stable counting sort of an edge list by source into CSR.  Edges of one
 * source keep their generation order; duplicates and self-loops are kept.
 * perm[k] = index in the input list of the k-th CSR edge (may be NULL).
 */
void fi_build_csr(uint32_t nv, uint64_t ne, const uint32_t *src,
                  const uint32_t *dst, uint64_t *row_ptr, uint32_t *col,
                  uint64_t *perm) {
    memset(row_ptr, 0, sizeof(uint64_t) * ((size_t)nv + 1));
    for (uint64_t i = 0; i < ne; ++i) row_ptr[src[i] + 1]++;
    for (uint32_t v = 0; v < nv; ++v) row_ptr[v + 1] += row_ptr[v];
    uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nv);
    memcpy(cur, row_ptr, sizeof(uint64_t) * (size_t)nv);
    for (uint64_t i = 0; i < ne; ++i) {
        uint64_t k = cur[src[i]]++;
        col[k] = dst[i];
        if (perm) perm[k] = i;
    }
    free(cur);
}
