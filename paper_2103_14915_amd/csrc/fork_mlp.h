// Learned partition scheduler, device side: normalisation statistics,
// partition features from buffer statistics, and the 16 -> 64 -> 64 -> 1 MLP
// that scores partitions in place of the priority functor (Section 5.2 scores
// a partition by the best priority among its buffered operations).
#pragma once
#include "fork_util.h"

namespace fk {

// Global ranges used to normalise per-partition statistics.
struct GStat {
    unsigned int sp_min, sp_max, lv_min, lv_max;
    unsigned int pr_min, pr_max;  // float bits of positive masses
    unsigned int nparts;          // partitions with pending operations
    unsigned int pad;
    unsigned long long ops;       // pending operations
};

// Normalisation ranges over all partitions (one block).
__device__ inline void gstat_body(const GraphDev& g, const BufDev& B, GStat* out) {
    __shared__ GStat s;
    if (threadIdx.x == 0) {
        s.sp_min = INF; s.sp_max = 0; s.lv_min = INF; s.lv_max = 0;
        s.pr_min = 0x7f7fffffu; s.pr_max = 0; s.nparts = 0; s.ops = 0;
    }
    __syncthreads();
    for (uint32_t P = threadIdx.x; P < g.np; P += blockDim.x) {
        uint32_t cnt = B.pcount[P];
        if (!cnt) continue;
        atomicAdd(&s.nparts, 1u);
        atomicAdd(&s.ops, (unsigned long long)cnt);
        uint32_t sp = B.pbest_sp[P], lv = B.pbest_lv[P], pr = B.pbest_pr[P];
        if (sp < INF) { atomicMin(&s.sp_min, sp); atomicMax(&s.sp_max, sp); }
        if (lv < INF) { atomicMin(&s.lv_min, lv); atomicMax(&s.lv_max, lv); }
        if (pr) { atomicMin(&s.pr_min, pr); atomicMax(&s.pr_max, pr); }
    }
    __syncthreads();
    if (threadIdx.x == 0) *out = s;
}

// Feature vector of partition P (16 fp32 values): buffer size, ready share,
// best SSSP distance / BFS level / PPR mass relative to the global range and
// their presence flags, recency, visits, partition size, age of the oldest
// buffered operation, and the share and count of its buffers that hold their
// query's dist_min.
__device__ inline void partition_features(const GraphDev& g, const BufDev& B, const GStat& s, uint32_t pass, uint32_t P,
                                   float* x) {
    uint32_t cnt = B.pcount[P];
    uint32_t sp = B.pbest_sp[P], lv = B.pbest_lv[P];
    float pr = __uint_as_float(B.pbest_pr[P]);
    float prmin = __uint_as_float(s.pr_min), prmax = __uint_as_float(s.pr_max);
    float fp = (float)(pass + 1);
    uint32_t v0 = g.pstart[P], v1 = g.pstart[P + 1];
    float ep = (float)(g.rowptr[v1] - g.rowptr[v0]);
    x[0] = log1pf((float)cnt) * 0.125f;
    x[1] = (float)B.pready[P] / (float)(B.pqn[P] ? B.pqn[P] : 1u);  // share of its buffers that are ready
    x[2] = sp < INF ? (float)(sp - s.sp_min) / (float)(s.sp_max - s.sp_min + 1u) : 1.f;
    x[3] = sp < INF ? 1.f : 0.f;
    x[4] = lv < INF ? (float)(lv - s.lv_min) / (float)(s.lv_max - s.lv_min + 1u) : 1.f;
    x[5] = lv < INF ? 1.f : 0.f;
    x[6] = pr > 0.f ? (log2f(prmax) - log2f(pr)) / (log2f(prmax) - log2f(prmin) + 1.f) : 1.f;
    x[7] = pr > 0.f ? 1.f : 0.f;
    x[8] = (float)(pass - B.plast[P]) / fp;
    x[9] = log1pf((float)B.pvisits[P]) * 0.125f;
    x[10] = log1pf(ep) * 0.0625f;
    x[11] = (float)(v1 - v0) / (float)VPMAX;
    uint32_t pf = B.pfirst[P];
    x[12] = pf < INF ? (float)(pass - pf) / fp : 0.f;
    // buffers holding their query's dist_min: visiting them is what advances
    // the queries' heuristic-2 windows
    x[13] = (float)B.pqmin[P] / (float)(B.pqn[P] ? B.pqn[P] : 1u);
    x[14] = log1pf((float)B.pqmin[P]) * 0.125f;
    x[15] = pr > 0.f ? fminf(1.f, pr * 1e3f) : 0.f;
}


// y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for one feature vector; w is the
// flat parameter vector (LDS or global).
__device__ __forceinline__ float mlp_forward(const float* w, const float* x) {
    const float* W1 = w;
    const float* b1 = W1 + MLP_H * MLP_IN;
    const float* W2 = b1 + MLP_H;
    const float* b2 = W2 + MLP_H * MLP_H;
    const float* W3 = b2 + MLP_H;
    const float* b3 = W3 + MLP_H;
    float h1[MLP_H];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float a = b1[o];
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) a = fmaf(W1[o * MLP_IN + i], x[i], a);
        h1[o] = a > 0.f ? a : 0.f;
    }
    float y = b3[0];
    for (int o = 0; o < MLP_H; ++o) {
        float a = b2[o];
#pragma unroll
        for (int i = 0; i < MLP_H; ++i) a = fmaf(W2[o * MLP_H + i], h1[i], a);
        a = a > 0.f ? a : 0.f;
        y = fmaf(W3[o], a, y);
    }
    return y;
}

}  // namespace fk
