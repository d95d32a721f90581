// Scheduling device code shared by the per-pass kernels and the persistent
// kernel: partition selection (ScheduleNextPart of Algorithm 2, Section 5.2)
// and buffer detachment into work items.
#pragma once
#include "fork_util.h"

namespace fk {

// ------------------------------------------------------------ scheduling
__device__ __forceinline__ uint32_t ordf(float f) {  // order-preserving float -> u32
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}


// ScheduleNextPart for one pass, run by one block of NTH threads.  The keys
// and buffer counts of up to cache_cap partitions are kept in s_key / s_qn.
template <int NTH>
__device__ void select_body(const GraphDev& g, const BufDev& B, const PassCfg& cfg, unsigned long long* s_key,
                            unsigned int* s_qn, uint32_t cache_cap) {
    __shared__ unsigned int s_u[8];
    __shared__ float s_f[4];
    __shared__ unsigned long long s_cnt;
    __shared__ unsigned int s_nsel;
    __shared__ unsigned long long s_pend;
    Ctl* ctl = B.ctl;
    const uint32_t np = g.np;
    const uint32_t tid = threadIdx.x;
    if (ctl->err) {  // a failed pass ends the run: select nothing
        if (tid == 0) { ctl->nsel = 0; ctl->pending_parts = 0; ctl->stop = 1u; }
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
    for (uint32_t P = tid; P < np; P += NTH) {
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
        if (!cnt || !B.pready[P]) return ~0ull;
        uint32_t k;
        switch (cfg.sched) {
        case S_FIFO: k = B.pfirst[P]; break;
        case S_MAXOPS: k = ~cnt; break;
        case S_RANDOM: k = (uint32_t)mix64(((unsigned long long)cfg.seed << 40) ^ ((unsigned long long)pass << 20) ^ P); break;
        // learned: partitions holding some query's dist_min first (they carry
        // heuristic 2's progress), each class in the network's score order
        case S_LEARNED: k = ((B.pqmin[P] ? 0u : 1u) << 31) | (~ordf(B.score[P]) >> 1); break;
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
    // keys (and buffer counts) of up to SEL_CACHE partitions are kept in LDS
    const bool cached = np <= cache_cap;
    if (cached) {
        for (uint32_t P = tid; P < np; P += NTH) {
            s_key[P] = key_of(P);
            s_qn[P] = B.pready[P];
        }
        __syncthreads();
    }
    auto key_at = [&](uint32_t P) -> unsigned long long { return cached ? s_key[P] : key_of(P); };
    auto qn_at = [&](uint32_t P) -> uint32_t { return cached ? s_qn[P] : B.pready[P]; };
    const uint32_t kmax = cfg.kmax;
    const uint32_t target = cfg.target_items;
    // Take partitions in priority order until kmax of them, or until their
    // buffers hold at least `target` work items (enough to fill the GPU).
    unsigned long long items_all = 0;
    if (target) {
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        uint32_t it = 0;
        for (uint32_t P = tid; P < np; P += NTH) it += B.pcount[P] ? B.pready[P] : 0u;
        if (it) atomicAdd(&s_cnt, (unsigned long long)it);
        __syncthreads();
        items_all = s_cnt;
        __syncthreads();
    }
    unsigned long long thresh = ~0ull;  // select keys < thresh
    if (total_pend > kmax || (target && items_all > target)) {
        // binary search the smallest t whose prefix {key <= t} meets the limit
        unsigned long long lo = 0, hi = (1ull << 48);
        while (lo < hi) {
            unsigned long long mid = lo + ((hi - lo) >> 1);
            if (tid == 0) { s_cnt = 0; s_pend = 0; }
            __syncthreads();
            uint32_t cnt = 0, it = 0;
            for (uint32_t P = tid; P < np; P += NTH)
                if (key_at(P) <= mid) { ++cnt; it += qn_at(P); }
            if (cnt) atomicAdd(&s_cnt, (unsigned long long)cnt);
            if (it) atomicAdd(&s_pend, (unsigned long long)it);
            __syncthreads();
            unsigned long long tot = s_cnt, tit = s_pend;
            __syncthreads();
            if (tot >= kmax || (target && tit >= target)) hi = mid; else lo = mid + 1;
        }
        thresh = lo + 1;
    }
    if (tid == 0) s_pend = 0;
    __syncthreads();
    for (uint32_t P = tid; P < np; P += NTH) {
        uint32_t cnt = B.pcount[P];
        if (cnt) atomicAdd(&s_pend, (unsigned long long)cnt);
    }
    __syncthreads();
    for (uint32_t P = tid; P < np; P += NTH) {
        unsigned long long k = key_at(P);
        if (k != ~0ull && k < thresh) {
            uint32_t j = atomicAdd(&s_nsel, 1u);
            if (j < kmax) B.sel[j] = P;
        }
    }
    __syncthreads();
    uint32_t nsel = s_nsel < kmax ? s_nsel : kmax;
    unsigned long long sel_edges = 0;
    for (uint32_t j = tid; j < nsel; j += NTH) {
        uint32_t P = B.sel[j];
        B.plast[P] = pass;
        B.pvisits[P] += 1;
        B.pn[P] = 0;
        sel_edges += g.rowptr[g.pstart[P + 1]] - g.rowptr[g.pstart[P]];
    }
    if (sel_edges) atomicAdd(&ctl->c_sel_edges, sel_edges);
    if (tid < NXCD) { ctl->nitems[tid] = 0; ctl->next[tid] = 0; }
    if (tid == 0) {
        ctl->nsel = nsel;
        ctl->pending_parts = total_pend;
        ctl->pending_ops = s_pend;
        ctl->stop = total_pend == 0 ? 1u : 0u;
        ctl->avail_end = ctl->ring_tail;
        ctl->pass = pass;
        if (nsel) ctl->c_passes_nonempty += 1;
    }
}

// Detach the buffer of (selected partition j, query q) into a work item.
// Lanes of one wave must share j (one reservation per wave).
__device__ __forceinline__ void worklist_one(const BufDev& B, const QueryDev& Q, const PassCfg& cfg, uint32_t j,
                                             uint32_t q) {
    Ctl* ctl = B.ctl;
    const uint32_t P = B.sel[j];
    const uint32_t x = j % NXCD;
    const uint32_t lane = lane_id();
    bool has = false;
    int32_t h = -1, o = -1;
    unsigned long long b = (unsigned long long)P * Q.qc + q;
    if (q < Q.nq) {
        h = B.bhead[b];
        o = B.bover[b];
        has = (h >= 0 || o >= 0) && bucket_ready(B.bval[b], Q.qtype[q], B.qmin[q], cfg);
    }
    unsigned long long mask = wballot(has);
    uint32_t n = __popcll(mask);
    if (!n) return;
    uint32_t base = 0;
    if (lane == 0) { base = dev_add(&ctl->nitems[x], n); dev_add(&B.pn[P], n); }
    base = __shfl(base, 0);
    if (has) {
        uint32_t pos = base + rank_in(mask);
        if (pos < B.item_cap) {
            // close the tail: record its fill and splice the overflow list after it
            const unsigned long long w = B.btw[b];
            uint32_t tl = 0xffffffffu, tf = 0;
            // chunk ids out of range mean a damaged buffer: the item is left
            // empty and the run stops with the consistency error
            bool bad = (unsigned long long)h >= B.nch && h >= 0;
            bad |= (unsigned long long)o >= B.nch && o >= 0;
            if (h >= 0 && !bad) {
                tl = (uint32_t)(w >> 32);
                tf = (uint32_t)w < (uint32_t)CH ? (uint32_t)w : (uint32_t)CH;
                if (tl < B.nch) {
                    B.ccount[tl] = tf;
                    B.cnext[tl] = o;
                } else {
                    bad = true;
                }
            }
            Item* it = &B.items[(unsigned long long)x * B.item_cap + pos];
            int32_t cur = (h >= 0 ? h : o);
            uint32_t n = 0;
            while (!bad && cur >= 0 && n < (uint32_t)ICH) {
                if ((unsigned long long)cur >= B.nch) { bad = true; break; }
                const bool is_tail = (uint32_t)cur == tl;
                it->ch[n++] = make_uint2((uint32_t)cur, is_tail ? tf : B.ccount[cur]);
                cur = is_tail ? o : B.cnext[cur];
            }
            if (bad) {
                dev_or(&ctl->err, (uint32_t)ERR_CORRUPT);
                n = 0;
                cur = -1;
            }
            it->part = P;
            it->q = q;
            it->nch = n;
            it->rest = cur;
            B.bhead[b] = -1;
            B.bover[b] = -1;
            B.btw[b] = BTW_EMPTY;
            B.bval[b] = 0xffffffffu;
            B.bcnt[b] = 0;
        } else {
            dev_or(&ctl->err, (uint32_t)ERR_ITEMS);
        }
    }
}

// Per query: its best buffered SSSP/BFS value over all partitions (the
// dist_min of heuristic 2, Section 5.1).
__device__ __forceinline__ void qmin_one(const BufDev& B, const QueryDev& Q, uint32_t np, uint32_t q) {
    if (q >= Q.nq) return;
    uint32_t m = 0xffffffffu;
    if (Q.qtype[q] != Q_PPR)
        for (uint32_t P = 0; P < np; ++P) {
            unsigned long long b = (unsigned long long)P * Q.qc + q;
            if (B.bcnt[b]) { uint32_t v = B.bval[b]; m = v < m ? v : m; }
        }
    B.qmin[q] = m;
}

// Partition summary from its buffers (one block): buffered operations, best
// SSSP distance / BFS level / PPR mass, non-empty and ready buffers, age of
// the oldest buffer.  These are what the priority functor and the learned
// scorer read.
__device__ inline void psum_one(const BufDev& B, const QueryDev& Q, const PassCfg& cfg, uint32_t P) {
    __shared__ unsigned long long s_cnt;
    __shared__ unsigned int s_sp, s_lv, s_pr, s_ne, s_rd, s_first, s_hm;
    if (threadIdx.x == 0) { s_cnt = 0; s_sp = INF; s_lv = INF; s_pr = 0; s_ne = 0; s_rd = 0; s_first = INF; s_hm = 0; }
    __syncthreads();
    unsigned long long cnt = 0;
    uint32_t sp = INF, lv = INF, pr = 0, ne = 0, rd = 0, first = INF, hm = 0;
    for (uint32_t q = threadIdx.x; q < Q.nq; q += blockDim.x) {
        unsigned long long b = (unsigned long long)P * Q.qc + q;
        uint32_t cb = B.bcnt[b];
        if (!cb) continue;
        uint32_t v = B.bval[b], t = Q.qtype[q];
        cnt += cb;
        ++ne;
        if (t == Q_PPR) { uint32_t m = ~v; pr = m > pr ? m : pr; }
        else if (t == Q_BFS) lv = v < lv ? v : lv;
        else sp = v < sp ? v : sp;
        rd += bucket_ready(v, t, B.qmin[q], cfg);
        hm += (t != Q_PPR && v == B.qmin[q]) ? 1u : 0u;  // this buffer holds the query's dist_min
        uint32_t f = B.bfirst[b];
        first = f < first ? f : first;
    }
    if (cnt) atomicAdd(&s_cnt, cnt);
    if (sp < INF) atomicMin(&s_sp, sp);
    if (lv < INF) atomicMin(&s_lv, lv);
    if (pr) atomicMax(&s_pr, pr);
    if (ne) atomicAdd(&s_ne, ne);
    if (rd) atomicAdd(&s_rd, rd);
    if (first < INF) atomicMin(&s_first, first);
    if (hm) atomicAdd(&s_hm, hm);
    __syncthreads();
    if (threadIdx.x == 0) {
        B.pcount[P] = s_cnt > 0xffffffffull ? 0xffffffffu : (uint32_t)s_cnt;
        B.pbest_sp[P] = s_sp;
        B.pbest_lv[P] = s_lv;
        B.pbest_pr[P] = s_pr;
        B.pqn[P] = s_ne;
        B.pready[P] = s_rd;
        B.pfirst[P] = s_first;
        B.pqmin[P] = s_hm;
    }
    __syncthreads();
}

}  // namespace fk
