// Sweep cuts of PPR results: the NCP application (Sections 2 and 6.1), gfx950.
//
// The paper builds NCP from one PPR per seed and keeps, per cluster size, the
// least conductance; it does not print the sweep.  Reading used (shared with
// the CPU oracle's documentation):
//   * the graph is read as undirected: each directed edge is one undirected
//     edge, d(v) = out-degree + in-degree, total volume 2|E|;
//   * the sweep visits the vertices with p[v] > 0 and d(v) > 0 in decreasing
//     fp32 p[v] / d(v), equal keys in increasing internal position;
//   * prefix S_k: cut = edges with exactly one endpoint in S_k, vol = sum of
//     d, conductance = cut / min(vol, 2|E| - vol) (undefined when 0).
//
// k_sweep: one workgroup per query, up to SW_K prefixes.
//   1. radix select (4 passes of 8 bits over the key bits of all vertices)
//      finds the SW_K-th largest key T;
//   2. keys above T, and the first keys equal to T in position order, are
//      collected and sorted in LDS (bitonic, key descending, position
//      ascending);
//   3. each thread takes one swept vertex u (rank i) and counts its incident
//      edges (out-edges and in-edges) to vertices of smaller rank: u adds
//      d(u) - self-loop entries - 2 * (edges into S_i) to the cut;
//   4. block scans give cut and volume of every prefix; the least
//      conductance overall and per size range [2^j, 2^(j+1)) are kept.
#include "fork_dev.h"
#include "fork_util.h"

namespace fk {

constexpr int SW_NT = 1024;      // threads per query (one swept vertex each)
constexpr int SW_K = 1024;       // most prefixes per query
constexpr int SW_H = 2048;       // rank table slots
constexpr int SW_BUCKETS = 11;   // size ranges [2^j, 2^(j+1)), j < 11 covers 1..1024
static_assert(SW_K == SW_NT, "one swept vertex per thread");

struct SweepOut {
    uint32_t support, swept, best_size, flags;
    double best_conductance;
    unsigned long long best_cut, best_volume;
    double size_min[SW_BUCKETS];
};

struct SweepShared {
    unsigned long long sel[SW_K];   // (key << 32) | ~position, sorted descending
    uint32_t tie[SW_K];             // positions whose key equals the cut-off
    uint32_t hkey[SW_H], hval[SW_H];
    uint32_t hist[256];
    unsigned long long wsum[SW_NT / WAVE], wsum2[SW_NT / WAVE];
    unsigned long long bmin[SW_BUCKETS];
    unsigned long long best;        // (conductance bits << ... ) see below
    uint32_t nsel, ntie, need, prefix, support, bucket;
};

__device__ __forceinline__ uint32_t sweep_key(const float* p, const uint32_t* sdeg, uint32_t v) {
    const float x = p[v];
    const uint32_t d = sdeg[v];
    return (x > 0.f && d > 0) ? __float_as_uint(x / (float)d) : 0u;
}

// Inclusive block scan of 64-bit values (SW_NT threads).
__device__ __forceinline__ unsigned long long block_scan64(unsigned long long v, unsigned long long* wsum) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        unsigned long long y = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v += y;
    }
    if (lane == WAVE - 1) wsum[w] = v;
    __syncthreads();
    unsigned long long before = 0;
    for (uint32_t k = 0; k < w; ++k) before += wsum[k];
    __syncthreads();
    return v + before;
}

__device__ __forceinline__ int32_t rank_of(const SweepShared& S, uint32_t u) {
    uint32_t h = (uint32_t)(((unsigned long long)(u * 0x9E3779B1u) * SW_H) >> 32);
    for (int i = 0; i < SW_H; ++i) {
        const uint32_t k = S.hkey[h];
        if (k == u) return (int32_t)S.hval[h];
        if (k == 0xffffffffu) return -1;
        h = h + 1 == (uint32_t)SW_H ? 0u : h + 1;
    }
    return -1;
}

__global__ __launch_bounds__(SW_NT) void k_sweep(const uint32_t* state, const unsigned long long* qoff, uint32_t nv,
                                                 const uint32_t* rowptr, const uint32_t* col, const uint32_t* rrow,
                                                 const uint32_t* rcol, const uint32_t* sdeg,
                                                 unsigned long long total_vol, uint32_t max_size, SweepOut* out) {
    __shared__ SweepShared S;
    const uint32_t t = threadIdx.x, q = blockIdx.x;
    const float* p = (const float*)(state + qoff[q]);
    const uint32_t K = max_size < (uint32_t)SW_K ? max_size : (uint32_t)SW_K;
    // support size
    if (t == 0) { S.support = 0; S.nsel = 0; S.ntie = 0; S.prefix = 0; S.need = 0; }
    __syncthreads();
    {
        uint32_t c = 0;
        for (uint32_t v = t; v < nv; v += SW_NT) c += sweep_key(p, sdeg, v) != 0u;
        if (c) atomicAdd(&S.support, c);
    }
    __syncthreads();
    const uint32_t support = S.support;
    const bool all = support <= K;
    // radix select of the K-th largest key (when the support is larger)
    uint32_t T = 1u, mask = 0u;
    if (!all) {
        if (t == 0) S.need = K;
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (uint32_t b = t; b < 256; b += SW_NT) S.hist[b] = 0;
            __syncthreads();
            const uint32_t pre = S.prefix;
            for (uint32_t v = t; v < nv; v += SW_NT) {
                const uint32_t k = sweep_key(p, sdeg, v);
                if (k && (k & mask) == pre) atomicAdd(&S.hist[(k >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (t == 0) {
                uint32_t need = S.need, b = 255;
                for (;; --b) {
                    const uint32_t h = S.hist[b];
                    if (h >= need || b == 0) break;
                    need -= h;
                }
                S.need = need;
                S.prefix = pre | (b << shift);
            }
            mask |= 255u << shift;
            __syncthreads();
        }
        T = S.prefix;  // the K-th largest key; S.need of the keys equal to T are taken
    }
    // collect: every key above T (all of the support when it fits), and the ties at T
    for (uint32_t v0 = 0; v0 < nv; v0 += SW_NT) {
        const uint32_t v = v0 + t;
        const uint32_t k = v < nv ? sweep_key(p, sdeg, v) : 0u;
        const bool above = k != 0u && (all || k > T);
        const bool tie = !all && k == T && k != 0u;
        if (above) {
            const uint32_t i = atomicAdd(&S.nsel, 1u);
            if (i < (uint32_t)SW_K) S.sel[i] = ((unsigned long long)k << 32) | (0xffffffffu - v);
        }
        if (tie) {
            const uint32_t i = atomicAdd(&S.ntie, 1u);
            if (i < (uint32_t)SW_K) S.tie[i] = v;
        }
    }
    __syncthreads();
    const uint32_t ntie = S.ntie, nabove = S.nsel;
    const bool overflow = !all && ntie > (uint32_t)SW_K;
    if (overflow) {  // more equal keys at the cut-off than the tie list holds: no result
        if (t == 0) {
            SweepOut o{};
            o.support = support;
            o.flags = 1u;
            o.best_conductance = __longlong_as_double(0x7ff0000000000000ll);
            for (int j = 0; j < SW_BUCKETS; ++j) o.size_min[j] = o.best_conductance;
            out[q] = o;
        }
        return;
    }
    if (!all) {
        // ties in position order: sort the tie list ascending (bitonic over SW_K, padding last)
        if (t >= ntie) S.tie[t] = 0xffffffffu;
        __syncthreads();
        for (uint32_t k = 2; k <= (uint32_t)SW_K; k <<= 1)
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                const uint32_t l = t ^ j;
                if (l > t) {
                    const uint32_t a = S.tie[t], b = S.tie[l];
                    const bool up = (t & k) == 0;
                    if ((a > b) == up) { S.tie[t] = b; S.tie[l] = a; }
                }
                __syncthreads();
            }
        const uint32_t need = S.need;
        if (t < need) S.sel[nabove + t] = ((unsigned long long)T << 32) | (0xffffffffu - S.tie[t]);
        __syncthreads();
    }
    const uint32_t n = all ? support : K;
    // sort the selection descending (key, then position ascending via ~position)
    if (t >= n) S.sel[t] = 0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= (uint32_t)SW_K; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            const uint32_t l = t ^ j;
            if (l > t) {
                const unsigned long long a = S.sel[t], b = S.sel[l];
                const bool down = (t & k) == 0;
                if ((a < b) == down) { S.sel[t] = b; S.sel[l] = a; }
            }
            __syncthreads();
        }
    // rank table
    for (uint32_t i = t; i < (uint32_t)SW_H; i += SW_NT) S.hkey[i] = 0xffffffffu;
    __syncthreads();
    const uint32_t u = t < n ? 0xffffffffu - (uint32_t)S.sel[t] : 0u;
    if (t < n) {
        uint32_t h = (uint32_t)(((unsigned long long)(u * 0x9E3779B1u) * SW_H) >> 32);
        while (atomicCAS(&S.hkey[h], 0xffffffffu, u) != 0xffffffffu) h = h + 1 == (uint32_t)SW_H ? 0u : h + 1;
        S.hval[h] = t;
    }
    __syncthreads();
    // cut change and volume of swept vertex t
    unsigned long long dcut = 0, dvol = 0;
    if (t < n) {
        uint32_t self = 0, joined = 0;
        for (uint32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            const uint32_t w = col[e];
            if (w == u) { ++self; continue; }
            const int32_t r = rank_of(S, w);
            joined += (r >= 0 && (uint32_t)r < t) ? 1u : 0u;
        }
        for (uint32_t e = rrow[u]; e < rrow[u + 1]; ++e) {
            const uint32_t x = rcol[e];
            if (x == u) { ++self; continue; }
            const int32_t r = rank_of(S, x);
            joined += (r >= 0 && (uint32_t)r < t) ? 1u : 0u;
        }
        const uint32_t d = sdeg[u];
        dvol = d;
        dcut = (unsigned long long)(d - self) - 2ull * joined;  // may wrap: the scan below is modular
    }
    const unsigned long long cut = block_scan64(dcut, S.wsum);
    const unsigned long long vol = block_scan64(dvol, S.wsum2);
    // conductance of prefix t + 1; non-negative doubles compare like their bits
    unsigned long long key = ~0ull;
    if (t < n) {
        const unsigned long long den = vol < total_vol - vol ? vol : total_vol - vol;
        if (den > 0) key = (unsigned long long)__double_as_longlong((double)cut / (double)den);
    }
    if (t < (uint32_t)SW_BUCKETS) S.bmin[t] = ~0ull;
    if (t == 0) S.best = ~0ull;
    __syncthreads();
    if (key != ~0ull) {
        atomicMin(&S.bmin[31 - __clz(t + 1)], key);
        atomicMin(&S.best, key);
    }
    __syncthreads();
    // smallest prefix reaching the best conductance
    if (t == 0) S.bucket = 0xffffffffu;
    __syncthreads();
    if (key != ~0ull && key == S.best) atomicMin(&S.bucket, t);
    __syncthreads();
    const uint32_t bt = S.bucket;
    if (t == bt) {
        out[q].best_size = t + 1;
        out[q].best_cut = cut;
        out[q].best_volume = vol;
        out[q].best_conductance = __longlong_as_double((long long)key);
    }
    if (t == 0) {
        out[q].support = support;
        out[q].swept = n;
        out[q].flags = 0u;
        if (bt == 0xffffffffu) {
            out[q].best_size = 0;
            out[q].best_cut = 0;
            out[q].best_volume = 0;
            out[q].best_conductance = __longlong_as_double(0x7ff0000000000000ll);
        }
    }
    if (t < (uint32_t)SW_BUCKETS)
        out[q].size_min[t] = S.bmin[t] == ~0ull ? __longlong_as_double(0x7ff0000000000000ll)
                                                : __longlong_as_double((long long)S.bmin[t]);
}

// In-degrees (for the reverse adjacency) and the reverse adjacency itself.
__global__ void k_indeg(const uint32_t* col, unsigned long long ne, uint32_t* indeg) {
    for (unsigned long long e = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; e < ne;
         e += (unsigned long long)gridDim.x * blockDim.x)
        atomicAdd(&indeg[col[e]], 1u);
}
// In-edges: rcol[k] = source of in-edge k, reid[k] = its index among the
// out-edges (for its weight).
__global__ void k_rfill(const uint32_t* rowptr, const uint32_t* col, uint32_t nv, const uint32_t* rrow,
                        uint32_t* cursor, uint32_t* rcol, uint32_t* reid) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nv; u += gridDim.x * blockDim.x)
        for (uint32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            const uint32_t w = col[e];
            const uint32_t k = rrow[w] + atomicAdd(&cursor[w], 1u);
            rcol[k] = u;
            reid[k] = e;
        }
}
__global__ void k_sdeg(const uint32_t* rowptr, const uint32_t* rrow, uint32_t nv, uint32_t* sdeg) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < nv; u += gridDim.x * blockDim.x)
        sdeg[u] = (rowptr[u + 1] - rowptr[u]) + (rrow[u + 1] - rrow[u]);
}

hipError_t launch_indeg(const uint32_t* col, unsigned long long ne, uint32_t* indeg, hipStream_t s) {
    if (ne) hipLaunchKernelGGL(k_indeg, dim3(2048), dim3(256), 0, s, col, ne, indeg);
    return hipGetLastError();
}
hipError_t launch_rfill(const uint32_t* rowptr, const uint32_t* col, uint32_t nv, const uint32_t* rrow,
                        uint32_t* cursor, uint32_t* rcol, uint32_t* reid, hipStream_t s) {
    hipLaunchKernelGGL(k_rfill, dim3(2048), dim3(256), 0, s, rowptr, col, nv, rrow, cursor, rcol, reid);
    return hipGetLastError();
}
hipError_t launch_sdeg(const uint32_t* rowptr, const uint32_t* rrow, uint32_t nv, uint32_t* sdeg, hipStream_t s) {
    hipLaunchKernelGGL(k_sdeg, dim3(2048), dim3(256), 0, s, rowptr, rrow, nv, sdeg);
    return hipGetLastError();
}
hipError_t launch_sweep(const uint32_t* state, const unsigned long long* qoff, uint32_t nq, uint32_t nv,
                        const uint32_t* rowptr, const uint32_t* col, const uint32_t* rrow, const uint32_t* rcol,
                        const uint32_t* sdeg, unsigned long long total_vol, uint32_t max_size, void* out,
                        hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep, dim3(nq), dim3(SW_NT), 0, s, state, qoff, nv, rowptr, col, rrow, rcol, sdeg,
                       total_vol, max_size, (SweepOut*)out);
    return hipGetLastError();
}
size_t sweep_out_bytes() { return sizeof(SweepOut); }

// ------------------------------------------------------------ betweenness
// Brandes' accumulation over resident BFS or SSSP queries (the BC application
// of Sections 2 and 6.1: many BFSs from sampled sources, then dependencies;
// on a weighted graph the same with SSSP).  The shortest-path DAG of a source
// holds the edges (u, v) with value(u) + w(u, v) = value(v), w = 1 for BFS.
// One workgroup per query, in three steps:
//   1. counting sort of the reached vertices by value (BFS level or SSSP
//      distance; per-query scratch).  With weights >= 1 a DAG edge raises the
//      value by at least one, so the vertices of one value are independent;
//   2. path counts sigma in order of increasing value: sigma(v) = sum over
//      DAG in-edges (u, v) of sigma(u).  Counts grow exponentially with depth
//      (a 2048 x 2048 grid has about 10^1230 corner-to-corner paths), so each
//      is kept as its natural logarithm, summed as log-sum-exp around the
//      largest term;
//   3. dependencies in order of decreasing value: delta(v) = sum over DAG
//      out-edges (v, w) of sigma(v) / sigma(w) * (1 + delta(w)), the ratio
//      taken as exp of the difference of logarithms (at most 1: sigma(w)
//      includes sigma(v)); every vertex but the source adds delta(v) to bc[v].
constexpr int BC_NT = 1024;
constexpr uint32_t BC_LMAX = 65536;  // values a query's reached vertices may span (the scratch size)

struct BcScratch {
    uint32_t* order;     // [nq][nv] vertices by value
    uint32_t* lstart;    // [nq][BC_LMAX + 2] value starts (then fill cursors)
    double* lsig;        // [nq][nv] ln sigma
    double* delta;       // [nq][nv]
};

__device__ __forceinline__ uint32_t bc_weight(const void* w, uint32_t wb, uint32_t e) {
    return wb == 0 ? 1u : wb == 1 ? ((const uint8_t*)w)[e] : wb == 2 ? ((const uint16_t*)w)[e] : ((const uint32_t*)w)[e];
}

__global__ __launch_bounds__(BC_NT) void k_bc(const uint32_t* state, const unsigned long long* qoff, const uint32_t* src,
                                             const uint32_t* qweighted, uint32_t nv, const uint32_t* rowptr,
                                             const uint32_t* col, const void* w, uint32_t wb, const uint32_t* rrow,
                                             const uint32_t* rcol, const uint32_t* reid, BcScratch sc, double* bc,
                                             uint32_t* err) {
    const uint32_t t = threadIdx.x, q = blockIdx.x;
    const uint32_t* val = state + qoff[q];
    const uint32_t qwb = qweighted[q] ? wb : 0u;  // BFS: unit steps
    uint32_t* order = sc.order + (unsigned long long)q * nv;
    uint32_t* ls = sc.lstart + (unsigned long long)q * (BC_LMAX + 2);
    double* lsig = sc.lsig + (unsigned long long)q * nv;
    double* delta = sc.delta + (unsigned long long)q * nv;
    __shared__ uint32_t s_max, s_bad;
    __shared__ uint32_t s_w[BC_NT / WAVE];
    if (t == 0) { s_max = 0; s_bad = 0; }
    for (uint32_t i = t; i < BC_LMAX + 2; i += BC_NT) ls[i] = 0;
    __syncthreads();
    // 1. value histogram
    for (uint32_t v = t; v < nv; v += BC_NT) {
        const uint32_t l = val[v];
        delta[v] = 0.0;
        if (l == INF) continue;
        if (l >= BC_LMAX) { s_bad = 1; continue; }
        atomicAdd(&ls[l + 1], 1u);
        atomicMax(&s_max, l);
    }
    __syncthreads();
    if (s_bad) {
        if (t == 0) atomicOr(err, 1u);
        return;
    }
    const uint32_t L = s_max;  // largest value
    // exclusive prefix over values 0..L (ls[l] = start of value l), chunked by the block
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 <= L + 1; b0 += BC_NT) {
        const uint32_t i = b0 + t;
        uint32_t x = i <= L + 1 ? ls[i] : 0u;
        const uint32_t lane = t & (WAVE - 1), wv = t / WAVE;
        uint32_t incl = wscan_incl(x, lane);
        if (lane == WAVE - 1) s_w[wv] = incl;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (uint32_t k = 0; k < BC_NT / WAVE; ++k) { before += k < wv ? s_w[k] : 0u; tot += s_w[k]; }
        __syncthreads();
        if (i <= L + 1) ls[i] = carry + before + incl;  // inclusive over shifted counts = start of value i
        carry += tot;
        __syncthreads();
    }
    // scatter: ls[l] (the start of value l) is value l's fill cursor, so it
    // ends as the end of value l; value l then spans [ls[l - 1], ls[l]) (from 0 for l = 0)
    for (uint32_t v = t; v < nv; v += BC_NT) {
        const uint32_t l = val[v];
        if (l == INF) continue;
        order[atomicAdd(&ls[l], 1u)] = v;
    }
    __syncthreads();
    // 2. ln sigma (the source: ln 1 = 0)
    if (t == 0) lsig[src[q]] = 0.0;
    __syncthreads();
    for (uint32_t l = 1; l <= L; ++l) {
        const uint32_t b = ls[l - 1], e = ls[l];
        for (uint32_t i = b + t; i < e; i += BC_NT) {
            const uint32_t v = order[i];
            // log-sum-exp over the DAG in-edges: the largest term first, then the sum around it
            double m = -INFINITY;
            for (uint32_t k = rrow[v]; k < rrow[v + 1]; ++k) {
                const uint32_t u = rcol[k];
                const uint32_t du = val[u];
                if (du != INF && (unsigned long long)du + bc_weight(w, qwb, reid[k]) == l) m = fmax(m, lsig[u]);
            }
            double sum = 0.0;
            for (uint32_t k = rrow[v]; k < rrow[v + 1]; ++k) {
                const uint32_t u = rcol[k];
                const uint32_t du = val[u];
                if (du != INF && (unsigned long long)du + bc_weight(w, qwb, reid[k]) == l) sum += exp(lsig[u] - m);
            }
            lsig[v] = m + log(sum);  // every reached vertex but the source has a DAG in-edge
        }
        __syncthreads();
    }
    // 3. delta
    for (int l = (int)L - 1; l >= 0; --l) {
        const uint32_t b = l ? ls[l - 1] : 0u, e = ls[l];
        for (uint32_t i = b + t; i < e; i += BC_NT) {
            const uint32_t v = order[i];
            double a = 0.0;
            const double sv = lsig[v];
            for (uint32_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
                const uint32_t x = col[k];
                const uint32_t dx = val[x];
                if (dx != INF && (unsigned long long)l + bc_weight(w, qwb, k) == dx)
                    a += exp(sv - lsig[x]) * (1.0 + delta[x]);
            }
            delta[v] = a;
        }
        __syncthreads();
    }
    const uint32_t s0 = src[q];
    for (uint32_t v = t; v < nv; v += BC_NT)
        if (v != s0 && val[v] != INF && delta[v] != 0.0) atomicAdd(&bc[v], delta[v]);
}

hipError_t launch_bc(const uint32_t* state, const unsigned long long* qoff, const uint32_t* src,
                     const uint32_t* qweighted, uint32_t nq, uint32_t nv, const uint32_t* rowptr, const uint32_t* col,
                     const void* w, uint32_t wb, const uint32_t* rrow, const uint32_t* rcol, const uint32_t* reid,
                     uint32_t* order, uint32_t* lstart, double* lsig, double* delta, double* bc, uint32_t* err,
                     hipStream_t s) {
    if (nq == 0) return hipSuccess;
    BcScratch sc{order, lstart, lsig, delta};
    hipLaunchKernelGGL(k_bc, dim3(nq), dim3(BC_NT), 0, s, state, qoff, src, qweighted, nv, rowptr, col, w, wb, rrow,
                       rcol, reid, sc, bc, err);
    return hipGetLastError();
}
uint32_t bc_level_cap() { return BC_LMAX; }

}  // namespace fk
