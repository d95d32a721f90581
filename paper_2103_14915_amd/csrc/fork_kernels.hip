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
#include "fork_util.h"

namespace fk {

// ------------------------------------------------------------ scheduling
__device__ __forceinline__ uint32_t ordf(float f) {  // order-preserving float -> u32
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int SEL_THREADS = 1024;

__global__ __launch_bounds__(SEL_THREADS) void k_select(GraphDev g, BufDev B, PassCfg cfg) {
    __shared__ unsigned int s_u[8];
    __shared__ float s_f[4];
    __shared__ unsigned long long s_cnt;
    __shared__ unsigned int s_nsel;
    __shared__ unsigned long long s_pend;
    Ctl* ctl = B.ctl;
    const uint32_t np = g.np;
    const uint32_t tid = threadIdx.x;
    if (ctl->err) {  // a failed pass ends the run: select nothing
        if (tid == 0) { ctl->nsel = 0; ctl->pending_parts = 0; }
        return;
    }
    const uint32_t pass = ctl->pass + 1;
    if (tid == 0) {
        s_u[0] = INF; s_u[1] = 0; s_u[2] = INF; s_u[3] = 0; s_u[4] = 0;
        s_f[0] = 3.4e38f; s_f[1] = 0.f;
        s_nsel = 0;
        s_pend = 0;
    }
    __syncthreads();
    // global ranges for normalising mixed-type priorities
    uint32_t npend = 0;
    unsigned long long pend_ops = 0;
    for (uint32_t P = tid; P < np; P += SEL_THREADS) {
        uint32_t cnt = B.pcount[P];
        if (!cnt) continue;
        ++npend;
        pend_ops += cnt;
        uint32_t sp = B.pbest_sp[P], lv = B.pbest_lv[P];
        float pr = __uint_as_float(B.pbest_pr[P]);
        if (sp < INF) { atomicMin(&s_u[0], sp); atomicMax(&s_u[1], sp); }
        if (lv < INF) { atomicMin(&s_u[2], lv); atomicMax(&s_u[3], lv); }
        if (pr > 0.f) { atomicMin((unsigned int*)&s_f[0], __float_as_uint(pr)); atomicMax((unsigned int*)&s_f[1], __float_as_uint(pr)); }
    }
    atomicAdd(&s_u[4], npend);
    atomicAdd(&s_pend, pend_ops);
    __syncthreads();
    const uint32_t gsp0 = s_u[0], gsp1 = s_u[1], glv0 = s_u[2], glv1 = s_u[3];
    const float gpr0 = s_f[0], gpr1 = s_f[1];
    const uint32_t total_pend = s_u[4];
    // key: (priority << 16 | partition) -- smaller is better, unique
    auto key_of = [&](uint32_t P) -> unsigned long long {
        uint32_t cnt = B.pcount[P];
        if (!cnt) return ~0ull;
        uint32_t k;
        switch (cfg.sched) {
        case S_FIFO: k = B.pfirst[P]; break;
        case S_MAXOPS: k = ~cnt; break;
        case S_RANDOM: k = (uint32_t)mix64(((unsigned long long)cfg.seed << 40) ^ ((unsigned long long)pass << 20) ^ P); break;
        case S_LEARNED: k = ~ordf(B.score[P]); break;
        default: {
            uint32_t sp = B.pbest_sp[P], lv = B.pbest_lv[P];
            float pr = __uint_as_float(B.pbest_pr[P]);
            if (!cfg.mixed) {
                if (sp < INF) k = sp;
                else if (lv < INF) k = lv;
                else k = ~__float_as_uint(pr);
            } else {
                float best = 2.f;
                if (sp < INF) best = fminf(best, (float)(sp - gsp0) / (float)(gsp1 - gsp0 + 1u));
                if (lv < INF) best = fminf(best, (float)(lv - glv0) / (float)(glv1 - glv0 + 1u));
                if (pr > 0.f) best = fminf(best, (gpr1 - pr) / (gpr1 - gpr0 + 1e-30f));
                k = __float_as_uint(best);
            }
        }
        }
        return ((unsigned long long)k << 16) | P;
    };
    const uint32_t kmax = cfg.kmax;
    unsigned long long thresh = ~0ull;  // select keys < thresh
    if (total_pend > kmax) {
        // binary search the smallest t such that count(key <= t) >= kmax
        unsigned long long lo = 0, hi = (1ull << 48);
        while (lo < hi) {
            unsigned long long mid = lo + ((hi - lo) >> 1);
            if (tid == 0) s_cnt = 0;
            __syncthreads();
            uint32_t cnt = 0;
            for (uint32_t P = tid; P < np; P += SEL_THREADS) cnt += key_of(P) <= mid;
            if (cnt) atomicAdd(&s_cnt, (unsigned long long)cnt);
            __syncthreads();
            unsigned long long tot = s_cnt;
            __syncthreads();
            if (tot >= kmax) hi = mid; else lo = mid + 1;
        }
        thresh = lo + 1;
    }
    for (uint32_t P = tid; P < np; P += SEL_THREADS) {
        unsigned long long k = key_of(P);
        if (k != ~0ull && k < thresh) {
            uint32_t j = atomicAdd(&s_nsel, 1u);
            if (j < kmax) B.sel[j] = P;
        }
    }
    __syncthreads();
    uint32_t nsel = s_nsel < kmax ? s_nsel : kmax;
    for (uint32_t j = tid; j < nsel; j += SEL_THREADS) {
        uint32_t P = B.sel[j];
        B.pcount[P] = 0;
        B.pbest_sp[P] = INF;
        B.pbest_lv[P] = INF;
        B.pbest_pr[P] = 0;
        B.pfirst[P] = INF;
        B.plast[P] = pass;
        B.pvisits[P] += 1;
        B.pn[P] = 0;
    }
    if (tid < NXCD) { ctl->nitems[tid] = 0; ctl->next[tid] = 0; }
    if (tid == 0) {
        ctl->nsel = nsel;
        ctl->pending_parts = total_pend;
        ctl->pending_ops = s_pend;
        ctl->avail_end = ctl->ring_tail;
        ctl->pass = pass;
        if (nsel) ctl->c_passes_nonempty += 1;
    }
}

__global__ __launch_bounds__(256) void k_worklist(BufDev B, QueryDev Q) {
    Ctl* ctl = B.ctl;
    const uint32_t j = blockIdx.x;
    if (ctl->err || j >= ctl->nsel) return;
    const uint32_t P = B.sel[j];
    const uint32_t x = j % NXCD;
    const uint32_t q = blockIdx.y * 256 + threadIdx.x;
    const uint32_t lane = lane_id();
    bool has = false;
    int32_t h = -1;
    unsigned long long b = (unsigned long long)P * Q.qc + q;
    if (q < Q.nq) { h = B.bhead[b]; has = h >= 0; }
    unsigned long long mask = wballot(has);
    uint32_t n = __popcll(mask);
    if (!n) return;
    uint32_t base = 0;
    if (lane == 0) { base = dev_add(&ctl->nitems[x], n); dev_add(&B.pn[P], n); }
    base = __shfl(base, 0);
    if (has) {
        uint32_t pos = base + rank_in(mask);
        if (pos < B.item_cap) {
            Item it;
            it.part = P;
            it.q = q;
            it.head = h;
            it.count = 0;
            B.items[(unsigned long long)x * B.item_cap + pos] = it;
            B.bhead[b] = -1;
            B.btail[b] = -1;
        } else {
            dev_or(&ctl->err, (uint32_t)ERR_ITEMS);
        }
    }
}

// ------------------------------------------------------------ wave setup
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
    B.ccount[q] = 1;
    B.cnext[q] = -1;
    unsigned long long b = (unsigned long long)P * Q.qc + q;
    B.bhead[b] = (int32_t)q;
    B.btail[b] = (int32_t)q;
    dev_add(&B.pcount[P], 1u);
    dev_min(&B.pfirst[P], 0u);
    if (t == Q_PPR) dev_max(&B.pbest_pr[P], __float_as_uint(1.0f));
    else if (t == Q_BFS) dev_min(&B.pbest_lv[P], 0u);
    else dev_min(&B.pbest_sp[P], 0u);
}

// Per-query digest of the final state (one block per query).
__global__ __launch_bounds__(256) void k_digest(QueryDev Q, uint32_t nv, unsigned long long* out /*[nq*6]*/) {
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
                hash += mix64(((unsigned long long)v << 32) | x);
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

}  // namespace fk

// ------------------------------------------------------------ launchers
namespace fk {
hipError_t launch_select(const GraphDev& g, const BufDev& B, const PassCfg& cfg, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(SEL_THREADS), 0, s, g, B, cfg);
    return hipGetLastError();
}
hipError_t launch_worklist(const BufDev& B, const QueryDev& Q, uint32_t kmax, hipStream_t s) {
    dim3 grid(kmax, (Q.nq + 255) / 256);
    hipLaunchKernelGGL(k_worklist, grid, dim3(256), 0, s, B, Q);
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
hipError_t launch_digest(const QueryDev& Q, uint32_t nv, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_digest, dim3(Q.nq), dim3(256), 0, s, Q, nv, out);
    return hipGetLastError();
}
}  // namespace fk
