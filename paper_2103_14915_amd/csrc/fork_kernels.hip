// Scheduling and set-up kernels of the buffered fork-processing pass (gfx950).
//
// One pass of Algorithm 2 on the GPU:
//   k_select    -- ScheduleNextPart: score every partition from its buffer
//                  summary (Section 5.2 priority functor, or FIFO / random /
//                  max-ops / learned score) and pick the best kmax partitions.
//   k_worklist  -- detach the buffers of the picked partitions, one work item
//                  per (partition, query) with buffered operations
//                  (query-centric consolidation, Section 4.2; buckets keyed
//                  by query, the K = |Q| case of Appendix B.1).
//   k_process   -- IntraPartProcess, in fork_pass.hip.
// Also: free-ring set-up, InitBuffers (source operations) and per-query
// result digests.
#include "fork_sched.h"

namespace fk {

// ------------------------------------------------------------ scheduling
constexpr int SEL_THREADS = 1024;
constexpr int SEL_CACHE = 4096;

__global__ __launch_bounds__(SEL_THREADS) void k_select(GraphDev g, BufDev B, PassCfg cfg) {
    __shared__ unsigned long long s_key[SEL_CACHE];
    __shared__ unsigned int s_qn[SEL_CACHE];
    select_body<SEL_THREADS>(g, B, cfg, s_key, s_qn, SEL_CACHE);
}

__global__ __launch_bounds__(256) void k_worklist(BufDev B, QueryDev Q, PassCfg cfg) {
    const uint32_t j = blockIdx.x;
    if (B.ctl->err || j >= B.ctl->nsel) return;
    worklist_one(B, Q, cfg, j, blockIdx.y * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_qmin(BufDev B, QueryDev Q, uint32_t np) {
    qmin_one(B, Q, np, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_psum(BufDev B, QueryDev Q, PassCfg cfg) { psum_one(B, Q, cfg, blockIdx.x); }

// ------------------------------------------------------------ wave setup
__global__ void k_fill64(unsigned long long* p, unsigned long long n, unsigned long long v) {
    unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (unsigned long long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_ring_init(uint32_t* ring, unsigned long long nch) {
    unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < nch; i += (unsigned long long)gridDim.x * blockDim.x) ring[i] = (uint32_t)i;
}

// Initial operations (InitBuffers of Algorithm 2): query q's source operation
// goes to the buffer of the source's partition; chunk q holds it.
__global__ void k_seed(GraphDev g, QueryDev Q, BufDev B, const uint32_t* src) {
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q.nq) return;
    uint32_t s = src[q];
    uint32_t P = g.vpart[s >> g.pshift];
    uint32_t t = Q.qtype[q];
    uint32_t val = t == Q_PPR ? __float_as_uint(1.0f) : 0u;
    B.chunks[(unsigned long long)q * CH] = make_uint2(s, val);
    unsigned long long b = (unsigned long long)P * Q.qc + q;
    B.bhead[b] = (int32_t)q;
    B.btw[b] = ((unsigned long long)q << 32) | 1ull;  // chunk q is the tail, one slot used
    B.bcnt[b] = CH;
    B.bval[b] = t == Q_PPR ? ~__float_as_uint(1.0f) : 0u;
    B.bfirst[b] = 0;
}

// Per-query digest of the final state (one block per query).  orig (NULL
// for the identity) maps the internal vertex numbering to the caller's ids,
// which the hash is defined on.
__global__ __launch_bounds__(256) void k_digest(QueryDev Q, uint32_t nv, unsigned long long* out /*[nq*6]*/,
                                                const uint32_t* orig) {
    const uint32_t q = blockIdx.x;
    if (q >= Q.nq) return;
    const uint32_t t = Q.qtype[q];
    const unsigned long long off = Q.qoff[q];
    __shared__ unsigned long long s_cnt, s_sum, s_hash;
    __shared__ double s_f0, s_f1;
    __shared__ unsigned int s_fmax;
    if (threadIdx.x == 0) { s_cnt = s_sum = s_hash = 0; s_f0 = s_f1 = 0; s_fmax = 0; }
    __syncthreads();
    unsigned long long cnt = 0, sum = 0, hash = 0;
    double f0 = 0, f1 = 0;
    float fmax = 0.f;
    if (t == Q_PPR) {
        const float* p = (const float*)(Q.state + off);
        const float* r = p + nv;
        for (uint32_t v = threadIdx.x; v < nv; v += blockDim.x) {
            float pv = p[v];
            cnt += pv > 0.f;
            f0 += pv;
            f1 += r[v];
            fmax = pv > fmax ? pv : fmax;
        }
    } else {
        const uint32_t* d = Q.state + off;
        for (uint32_t v = threadIdx.x; v < nv; v += blockDim.x) {
            uint32_t x = d[v];
            if (x != INF) {
                ++cnt;
                sum += x;
                hash += mix64(((unsigned long long)(orig ? orig[v] : v) << 32) | x);
            }
        }
    }
    atomicAdd(&s_cnt, cnt);
    atomicAdd(&s_sum, sum);
    atomicAdd(&s_hash, hash);
    atomicAdd(&s_f0, f0);
    atomicAdd(&s_f1, f1);
    atomicMax(&s_fmax, __float_as_uint(fmax));
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long* o = out + (unsigned long long)q * 6;
        o[0] = s_cnt;
        o[1] = s_sum;
        o[2] = s_hash;
        double fm = (double)__uint_as_float(s_fmax);
        o[3] = __double_as_longlong(s_f0);
        o[4] = __double_as_longlong(s_f1);
        o[5] = __double_as_longlong(fm);
    }
}

// A result vector in the caller's numbering: dst[v] = src[pos[v]], with pos
// the internal position of vertex v.
__global__ void k_gather(const uint32_t* src, const uint32_t* pos, uint32_t* dst, uint32_t nv) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x)
        dst[v] = src[pos[v]];
}

// ------------------------------------------------------------ certified PPR
// Residual mass ||r||_1 of each listed PPR query, in fp64 (one block per
// query).  It bounds the L1 distance of p from the PPR vector, since that
// distance is ||PPR(r)||_1 <= ||r||_1 by the push invariant.
__global__ __launch_bounds__(256) void k_rnorm(QueryDev Q, uint32_t nv, const uint32_t* qs, uint32_t n, double* out) {
    const uint32_t i = blockIdx.x;
    if (i >= n) return;
    const uint32_t q = qs[i];
    __shared__ double s_f;
    if (threadIdx.x == 0) s_f = 0;
    __syncthreads();
    double f = 0;
    if (q < Q.nq && Q.qtype[q] == Q_PPR) {
        const float* r = (const float*)(Q.state + Q.qoff[q]) + nv;
        for (uint32_t v = threadIdx.x; v < nv; v += blockDim.x) f += r[v];
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) f += __shfl_xor(f, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_f, f);
    __syncthreads();
    if (threadIdx.x == 0) out[i] = s_f;
}

// Opens a refinement pass: work items for the (partition, query) pairs
// lo .. lo+n-1 of the np x |qs| grid (pair i = j*np + P, query qs[j]), each
// marked RESCAN, dealt round-robin over the per-XCD lists.  Also does what
// k_select does for a pass: the pass number, the pool bound, the list heads
// and the items per partition (approximate here; it only sizes yield
// heuristic 1's edge budget).
__global__ __launch_bounds__(256) void k_rescan_items(BufDev B, uint32_t np, const uint32_t* qs,
                                                      unsigned long long lo, uint32_t n) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) {
        const unsigned long long i = lo + k;
        Item* it = &B.items[(unsigned long long)(k % NXCD) * B.item_cap + k / NXCD];
        it->part = (uint32_t)(i % np);
        it->q = qs[i / np];
        it->rest = RESCAN;
        it->nch = 0;
    }
    if (k < np) B.pn[k] = (n + np - 1) / np;
    if (blockIdx.x == 0 && threadIdx.x < NXCD) {
        B.ctl->nitems[threadIdx.x] = (n + NXCD - 1 - threadIdx.x) / NXCD;
        B.ctl->next[threadIdx.x] = 0;
    }
    if (k == 0) {
        B.ctl->pass += 1;
        B.ctl->avail_end = B.ctl->ring_tail;
    }
}

}  // namespace fk

// ------------------------------------------------------------ launchers
namespace fk {
hipError_t launch_select(const GraphDev& g, const BufDev& B, const PassCfg& cfg, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(SEL_THREADS), 0, s, g, B, cfg);
    return hipGetLastError();
}
hipError_t launch_worklist(const BufDev& B, const QueryDev& Q, const PassCfg& cfg, hipStream_t s) {
    dim3 grid(cfg.kmax, (Q.nq + 255) / 256);
    hipLaunchKernelGGL(k_worklist, grid, dim3(256), 0, s, B, Q, cfg);
    return hipGetLastError();
}
hipError_t launch_summaries(const GraphDev& g, const BufDev& B, const QueryDev& Q, const PassCfg& cfg, hipStream_t s) {
    hipLaunchKernelGGL(k_qmin, dim3((Q.nq + 255) / 256), dim3(256), 0, s, B, Q, g.np);
    hipLaunchKernelGGL(k_psum, dim3(g.np), dim3(256), 0, s, B, Q, cfg);
    return hipGetLastError();
}
hipError_t launch_fill64(unsigned long long* p, unsigned long long n, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill64, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_ring_init(uint32_t* ring, unsigned long long nch, hipStream_t s) {
    hipLaunchKernelGGL(k_ring_init, dim3(1024), dim3(256), 0, s, ring, nch);
    return hipGetLastError();
}
hipError_t launch_seed(const GraphDev& g, const QueryDev& Q, const BufDev& B, const uint32_t* src, hipStream_t s) {
    hipLaunchKernelGGL(k_seed, dim3((Q.nq + 255) / 256), dim3(256), 0, s, g, Q, B, src);
    return hipGetLastError();
}
hipError_t launch_rnorm(const QueryDev& Q, uint32_t nv, const uint32_t* qs, uint32_t n, double* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rnorm, dim3(n), dim3(256), 0, s, Q, nv, qs, n, out);
    return hipGetLastError();
}
// n pairs starting at lo; the caller keeps n <= NXCD * item_cap and
// lo + n <= np * |qs|.
hipError_t launch_rescan_items(const BufDev& B, uint32_t np, const uint32_t* qs, unsigned long long lo, uint32_t n,
                               hipStream_t s) {
    if (n == 0 || n > (unsigned long long)NXCD * B.item_cap) return hipErrorInvalidValue;
    const uint32_t m = n > np ? n : np;
    hipLaunchKernelGGL(k_rescan_items, dim3((m + 255) / 256), dim3(256), 0, s, B, np, qs, lo, n);
    return hipGetLastError();
}
hipError_t launch_digest(const QueryDev& Q, uint32_t nv, unsigned long long* out, const uint32_t* orig,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_digest, dim3(Q.nq), dim3(256), 0, s, Q, nv, out, orig);
    return hipGetLastError();
}
hipError_t launch_gather(const uint32_t* src, const uint32_t* pos, uint32_t* dst, uint32_t nv, hipStream_t s) {
    const uint32_t blocks = (nv + 255) / 256 < 4096u ? (nv + 255) / 256 : 4096u;
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, src, pos, dst, nv);
    return hipGetLastError();
}
}  // namespace fk
