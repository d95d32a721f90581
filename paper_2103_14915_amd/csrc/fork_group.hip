// The query-grouped engine (gfx950): the fork-processing pattern with the
// queries of one type taken 64 at a time, one query per lane of a wave.
//
// Mapping of the paper's design (Sections 3-5) onto the GPU:
//   * state is kept vertex-major per group: the 64 queries' values of a
//     vertex are one 256-byte row, so a visit reads each out-edge once for
//     all 64 queries (the fork sharing of Section 4.1) and every state access
//     of a wave is one coalesced row;
//   * the buffer of a (partition, group) pair holds the consolidated pending
//     operations <q, v, val> of Section 4.2: at most one per (query, vertex),
//     with the minimum distance (SSSP/BFS) or the summed residual (PPR).  Its
//     values live in the state rows, combined there at once by device atomics
//     (min, or add), and its membership is a 64-bit lane mask per vertex plus
//     a bitmap of the vertices with pending lanes.  An update to another
//     partition marks the target pending and counts the activation in that
//     pair's summary (count, best value, age), which the scheduler reads;
//   * a visit of (P, g) moves P's pending bits into LDS and works through
//     them in rounds (Algorithm 2's IntraPartProcess), expanding every
//     pending lane of a vertex together; activations inside P join the next
//     round, the rest wait for their partition's visit.  Heuristic 2 of
//     Section 5.1 holds back lanes beyond the group's window, heuristic 1
//     ends the visit after an edge budget; held-back work stays pending.
#include "fork_sched.h"

namespace fk {

constexpr int GW = 64;        // queries per group (one per lane)
constexpr int GNTMAX = 1024;  // threads per workgroup: 256, 512 or 1024 (chosen at launch)
constexpr int GNWMAX = GNTMAX / WAVE;
constexpr int RCAP = 512;     // vertices per round
constexpr uint32_t GPVMAX = 16384;  // largest partition the grouped engine visits
constexpr int LBW = GPVMAX / 32;     // local pending bitmap words
constexpr int UNR = 8;        // edges in flight per wave step (and marking lanes)
constexpr int BAT = 4;        // round vertices per wave whose row loads are issued together
static_assert(UNR <= WAVE && RCAP % 256 == 0, "task layout");

// Per round vertex and lane, what its out-edges carry: SSSP/BFS the lane's
// value when the vertex was filtered (a snapshot: the value can only have
// dropped since, which the vertex's new pending mark covers), PPR the share
// each out-edge receives.  Kept in LDS so that the edge tasks read no source
// row from memory.
union GCtxShare {
    uint32_t sd[RCAP][GW];
    float share[RCAP][GW];
};

// Block counters (LDS), added by one lane per wave from ballot counts.
enum { K_EDGES, K_INTRA, K_IMPROVED, K_VPUSH, K_ACT, K_EDGES_PPR, K_VPUSH_PPR, K_VTASK, K_ROUNDS, K_TASKS,
       K_T_GATHER, K_T_TAKE, K_T_FILTER, K_T_TASKS, K_T_YIELD, NCNT };

struct GShared {
    uint32_t lbits[LBW];              // pending vertices of the partition (local ids)
    uint32_t rv[RCAP];                // round: vertex (local id)
    unsigned long long rm[RCAP];      // round: lanes taken, then lanes expanding
    uint32_t rnt[RCAP];               // round: expanding out-edges of the vertex, then its first flat edge
    uint32_t rdeg[RCAP];              // round: out-degree of the vertex
    uint32_t nr, next;
    uint32_t lmin[GW];                // per lane: least pending value of the round (SSSP/BFS)
    uint32_t wred[GNWMAX];
    unsigned long long edges;         // lane-edges of the visit so far
    unsigned long long itpos;
    unsigned long long cnt[NCNT];
    unsigned long long tk;            // start of the current visit phase (thread 0)
    Item it;
};

// Wave-uniform count n added to block counter k (call from every lane of a wave).
__device__ __forceinline__ void gcount(GShared& S, int k, uint32_t n) {
    if (lane_id() == 0 && n) atomicAdd(&S.cnt[k], (unsigned long long)n);
}

// Entry `lane` of vertex u's row in a group's state block.  Byte offsets are
// 32-bit: the grouped engine takes graphs of at most 2^24 vertices.
__device__ __forceinline__ uint32_t* rowp(uint32_t* base, uint32_t u, uint32_t lane) {
    return (uint32_t*)((char*)base + (u * (uint32_t)(GW * 4) + lane * 4u));
}
__device__ __forceinline__ float* rowf(float* base, uint32_t u, uint32_t lane) {
    return (float*)((char*)base + (u * (uint32_t)(GW * 4) + lane * 4u));
}

// The rows of a group's state block as a buffer resource (gfx9 raw buffer,
// no stride): a lane whose byte offset lies beyond the block reads 0 and
// touches no memory, so a wave loads rows for its active lanes only without a
// branch around the load (a branch would make the compiler wait for each load
// in turn).
constexpr uint32_t ROW_NONE = 0xfffffffcu;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(uint32_t* base, uint32_t nv) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(nv * (uint32_t)(GW * 4)), 0x00020000);
}
__device__ __forceinline__ uint32_t row_off(uint32_t u, uint32_t lane) { return u * (uint32_t)(GW * 4) + lane * 4u; }

__device__ __forceinline__ unsigned long long gpend_take(unsigned long long* p) {
    return __hip_atomic_exchange(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t fresh_load(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Make this thread's earlier device atomics visible before what follows (a
// barrier then lets other threads of the block act on them).
__device__ __forceinline__ void mem_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

struct GCtx {
    GraphDev g;
    GroupDev G;
    BufDev B;
    uint32_t P, grp, qt, v0, nvp, pass;
    uint32_t* st;          // group state rows (SSSP/BFS dist, PPR r)
    float* pp;             // PPR p rows
    float alpha, eps;      // this lane's query
    uint32_t mode;
    uint32_t win;          // heuristic-2 bound: lanes with value > win wait (INF: none)
    uint32_t bwin;         // batch width inside a visit: a lane expands values in [lmin, lmin + bwin)
};

// Mark lanes `bits` of vertex u (global id) pending in the group.  Called by
// one lane.  val: the activation's priority (SSSP/BFS distance; PPR ~residual
// bits).  Returns true for a new activation registered in another partition.
//
// Split in two so that a caller can overlap the wait for the mask's old value
// with other work: gmark_begin sets the lanes in the mask and returns its old
// value, gmark_end registers the activation from it.
__device__ __forceinline__ unsigned long long gmark_begin(GCtx& c, uint32_t u, unsigned long long bits) {
    return dev_or(&c.G.pend[(unsigned long long)c.grp * c.g.nv + u], bits);
}
__device__ __forceinline__ bool gmark_end(GCtx& c, GShared& S, uint32_t u, unsigned long long old, uint32_t val) {
    const uint32_t ul = u - c.v0;
    if (ul < c.nvp) {
        if (!old) atomicOr(&S.lbits[ul >> 5], 1u << (ul & 31));
        return false;
    }
    const uint32_t Pu = c.g.vpart[u >> c.g.pshift];
    const unsigned long long pi = (unsigned long long)Pu * c.G.ng + c.grp;
    // only the mask's old value is waited for (it orders the mask before the
    // bitmap bit that announces it); the rest are fire-and-forget atomics
    if (!old) {
        dev_or(&c.G.bits[(unsigned long long)c.grp * c.G.bw + (u >> 5)], 1u << (u & 31));
        dev_add(&c.G.icnt[pi], 1u);
        dev_min(&c.G.ifirst[pi], c.pass);
    }
    dev_min(&c.G.ibest[pi], val);
    return !old;
}
__device__ __forceinline__ bool gmark(GCtx& c, GShared& S, uint32_t u, unsigned long long bits, uint32_t val) {
    return gmark_end(c, S, u, gmark_begin(c, u, bits), val);
}

// Re-register vertex vloc of the visited partition as pending in the pair's
// summary (work held back by a yield).  Called by one lane.
__device__ __forceinline__ void gkeep(GCtx& c, uint32_t vloc, uint32_t val) {
    const uint32_t u = c.v0 + vloc;
    const unsigned long long pi = (unsigned long long)c.P * c.G.ng + c.grp;
    dev_or(&c.G.bits[(unsigned long long)c.grp * c.G.bw + (u >> 5)], 1u << (u & 31));
    dev_add(&c.G.icnt[pi], 1u);
    dev_min(&c.G.ibest[pi], val);
    dev_min(&c.G.ifirst[pi], c.pass);
}

template <class T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o; o >>= 1) { T t = __shfl_xor(v, o); v = t < v ? t : v; }
    return v;
}

// Build the next round from the local bitmap: up to `cap` vertices, their
// pending lanes taken from the global masks (one vertex per thread, so the
// exchanges are in flight together) and their degrees.  Returns the round size.
__device__ uint32_t gtake_round(GCtx& c, GShared& S, uint32_t cap) {
    const uint32_t t = threadIdx.x;
    if (t == 0) S.nr = 0;
    __syncthreads();
    const uint32_t nw = (c.nvp + 31) / 32;
    for (uint32_t w0 = 0; w0 < nw; w0 += blockDim.x) {
        const uint32_t w = w0 + t;
        uint32_t word = w < nw ? S.lbits[w] : 0u;
        // how many of this word's vertices fit in the round
        const uint32_t cnt = __popc(word);
        if (cnt) {
            const uint32_t at = atomicAdd(&S.nr, cnt);
            const uint32_t room = at >= cap ? 0u : (cap - at < cnt ? cap - at : cnt);
            for (uint32_t k = 0; k < room; ++k) {
                const uint32_t b = __ffs(word) - 1;
                word &= word - 1;
                S.rv[at + k] = w * 32 + b;
            }
            S.lbits[w] = word;  // what did not fit stays for a later round
        }
        __syncthreads();
        const bool full = S.nr >= cap;
        __syncthreads();
        if (full) break;
    }
    const uint32_t nr = S.nr < cap ? S.nr : cap;
    for (uint32_t k = t; k < nr; k += blockDim.x) {
        const uint32_t v = c.v0 + S.rv[k];
        S.rm[k] = gpend_take(&c.G.pend[(unsigned long long)c.grp * c.g.nv + v]);
        S.rdeg[k] = c.g.rowptr[v + 1] - c.g.rowptr[v];
    }
    __syncthreads();
    return nr;
}

// SSSP / BFS, first half of a round: each lane's least pending value among
// the round's vertices (the start of its batch window, Section 4.2's
// Dijkstra order taken in batches as in Delta-stepping).
__device__ void ground_min(GCtx& c, GShared& S, uint32_t nr) {
    const uint32_t t = threadIdx.x, lane = lane_id(), wv = t / WAVE, nwv = blockDim.x / WAVE;
    if (t < (uint32_t)GW) S.lmin[t] = INF;
    __syncthreads();
    uint32_t m = INF;
    for (uint32_t k0 = wv; k0 < nr; k0 += nwv * BAT) {
        uint32_t d[BAT];
#pragma unroll
        for (int i = 0; i < BAT; ++i) {
            const uint32_t k = k0 + i * nwv;
            const bool a = k < nr && ((S.rm[k] >> lane) & 1ull);
            d[i] = a ? fresh_load(rowp(c.st, c.v0 + S.rv[k], lane)) : INF;
        }
#pragma unroll
        for (int i = 0; i < BAT; ++i) m = d[i] < m ? d[i] : m;
    }
    if (m < INF) atomicMin(&S.lmin[lane], m);
    __syncthreads();
}

// Exclusive prefix sum over the block of one value per thread.
__device__ __forceinline__ uint32_t gblock_excl(GShared& S, uint32_t v, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wscan_incl(v, lane);
    if (lane == 63) S.wred[wid] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    const int nwv = (int)(blockDim.x / WAVE);
    for (int w = 0; w < nwv; ++w) {
        const uint32_t x = S.wred[w];
        before += (w < (int)wid) ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// Number the round's out-edges: S.rnt[k] holds vertex k's expanding out-edge
// count on entry and the index of its first edge in the round's flat edge
// list on return.  Returns the round's edge total.
__device__ uint32_t gnumber_edges(GShared& S, uint32_t nr) {
    constexpr uint32_t PERMAX = RCAP / 256;  // entries per thread with the smallest workgroup
    const uint32_t per = (RCAP + blockDim.x - 1) / blockDim.x;
    const uint32_t t = threadIdx.x;
    uint32_t x[PERMAX];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < PERMAX; ++k) {
        const uint32_t i = t * per + k;
        x[k] = (k < per && i < nr) ? S.rnt[i] : 0u;
        sum += x[k];
    }
    uint32_t total = 0;
    uint32_t run = gblock_excl(S, sum, &total);
#pragma unroll
    for (uint32_t k = 0; k < PERMAX; ++k) {
        const uint32_t i = t * per + k;
        if (k < per && i < nr) S.rnt[i] = run;
        run += x[k];
    }
    __syncthreads();
    return total;
}

// Round vertex of flat edge f: the last k with rnt[k] <= f.
__device__ __forceinline__ uint32_t gedge_vertex(const GShared& S, uint32_t nr, uint32_t f) {
    uint32_t lo = 0, hi = nr;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (S.rnt[mid] <= f) lo = mid; else hi = mid;
    }
    return lo;
}

// SSSP / BFS, second step of a round: per vertex (one wave each), the lanes
// that expand now.  Lanes beyond the group's heuristic-2 window wait in the
// pair's buffer for a later pass; lanes beyond their batch window go back to
// the partition's pending set for a later round of this visit.
__device__ void gfilter_sp(GCtx& c, GShared& S, GCtxShare& SH, uint32_t nr) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE, nwv = blockDim.x / WAVE;
    const uint32_t lo = S.lmin[lane];
    const unsigned long long hi_ = (unsigned long long)lo + c.bwin;
    const uint32_t hi = hi_ >= INF ? INF : (uint32_t)hi_;
    uint32_t n_push = 0, n_vt = 0;
    for (uint32_t k0 = wv; k0 < nr; k0 += nwv * BAT) {
        uint32_t d[BAT];
#pragma unroll
        for (int i = 0; i < BAT; ++i) {
            const uint32_t k = k0 + i * nwv;
            const bool a = k < nr && ((S.rm[k] >> lane) & 1ull);
            d[i] = a ? fresh_load(rowp(c.st, c.v0 + S.rv[k], lane)) : INF;
        }
#pragma unroll
        for (int i = 0; i < BAT; ++i) {
            const uint32_t k = k0 + i * nwv;
            if (k >= nr) break;
            const uint32_t vloc = S.rv[k];
            const uint32_t v = c.v0 + vloc;
            bool act = (S.rm[k] >> lane) & 1ull;
            const bool late = act && d[i] > c.win;
            const unsigned long long lm = wballot(late);
            if (lm) {
                const uint32_t dl = wave_min(late ? d[i] : 0xffffffffu);
                if (lane == 0) {
                    dev_or(&c.G.pend[(unsigned long long)c.grp * c.g.nv + v], lm);
                    gkeep(c, vloc, dl);
                }
                act = act && !late;
            }
            const bool later = act && d[i] >= hi;
            const unsigned long long lr = wballot(later);
            if (lr && lane == 0) {
                // back to the partition's pending set; the fence below orders the
                // mask before the next round takes it
                dev_or(&c.G.pend[(unsigned long long)c.grp * c.g.nv + v], lr);
                atomicOr(&S.lbits[vloc >> 5], 1u << (vloc & 31));
            }
            act = act && !later;
            const unsigned long long am = wballot(act);
            SH.sd[k][lane] = d[i];
            n_push += (uint32_t)__popcll(am);
            n_vt += am ? 1u : 0u;
            if (lane == 0) {
                S.rm[k] = am;
                S.rnt[k] = am ? S.rdeg[k] : 0u;
            }
        }
    }
    gcount(S, K_VPUSH, n_push);
    gcount(S, K_VTASK, n_vt);
    mem_release();
    __syncthreads();
}

// PPR, second step of a round: per vertex (one wave each), take the pending
// lanes' residuals, push those at or above their threshold into p and keep
// the share each out-edge receives (Section 4.1's push).
__device__ void gfilter_ppr(GCtx& c, GShared& S, GCtxShare& SH, uint32_t nr) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE, nwv = blockDim.x / WAVE;
    uint32_t n_push = 0, n_vt = 0, n_act = 0;
    for (uint32_t k0 = wv; k0 < nr; k0 += nwv * BAT) {
        float rx[BAT];
#pragma unroll
        for (int i = 0; i < BAT; ++i) {
            const uint32_t k = k0 + i * nwv;
            const bool mine = k < nr && ((S.rm[k] >> lane) & 1ull);
            rx[i] = mine ? __hip_atomic_exchange(rowf((float*)c.st, c.v0 + S.rv[k], lane), 0.f, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                         : 0.f;
        }
#pragma unroll
        for (int i = 0; i < BAT; ++i) {
            const uint32_t k = k0 + i * nwv;
            if (k >= nr) break;
            const uint32_t v = c.v0 + S.rv[k];
            const uint32_t deg = S.rdeg[k];
            const bool mine = (S.rm[k] >> lane) & 1ull;
            const float rv = rx[i];
            const float thr = c.mode ? c.eps * (float)deg : c.eps;
            const bool push = mine && ppr_active(rv, thr);
            bool back = false;
            if (mine && !push && rv != 0.f) {
                // below the threshold after all: give the residual back (it may cross with what arrived)
                const float old = __hip_atomic_fetch_add(rowf((float*)c.st, v, lane), rv, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                back = !ppr_active(old, thr) && ppr_active(old + rv, thr);
            }
            const unsigned long long bk = wballot(back);
            bool newact = false;
            if (bk && lane == 0) newact = gmark(c, S, v, bk, 0u);
            n_act += newact ? 1u : 0u;
            const unsigned long long pm = wballot(push);
            n_push += (uint32_t)__popcll(pm);
            n_vt += pm ? 1u : 0u;
            float share = 0.f;
            if (push) {
                __hip_atomic_fetch_add(rowf(c.pp, v, lane), c.alpha * rv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (deg) share = (1.f - c.alpha) * rv / (float)deg;
            }
            SH.share[k][lane] = share;
            if (lane == 0) {
                S.rm[k] = deg ? pm : 0ull;
                S.rnt[k] = pm ? deg : 0u;
            }
        }
    }
    n_act = __shfl(n_act, 0);
    gcount(S, K_ACT, n_act);
    gcount(S, K_VPUSH, n_push);
    gcount(S, K_VPUSH_PPR, n_push);
    gcount(S, K_VTASK, n_vt);
    __syncthreads();
}

// Third step of a round: the edge tasks, shared by the block's waves.  A task
// is 64 consecutive edges of the round's flat edge list (the expanding
// vertices' out-edges one after another, so low-degree vertices share a
// task): lane j finds edge j's source vertex and loads its target (and
// weight).  Then UNR edges at a time, every query lane that expands the
// edge's source relaxes (SSSP/BFS: atomic min of the target row's entry) or
// pushes to (PPR: atomic add of its share) the target, and the lanes
// 0..UNR-1 mark the newly pending targets in parallel.
//
// SSSP/BFS steps are software-pipelined: a step's atomic minima are issued,
// then the next step's row loads, and only then are the minima's old values
// waited for.  Whether a lane improved a target is still decided by the
// value its own atomic returned, so the marks are what the unpipelined loop
// makes.
template <int WB, bool ppr>
__device__ void gtasks(GCtx& c, GShared& S, GCtxShare& SH, uint32_t nr, uint32_t nedge) {
    const uint32_t lane = lane_id();
    const uint32_t ntask = (nedge + GW - 1) / GW;
    // counts of this wave's tasks: wave-uniform, or per lane (summed at the end)
    uint32_t n_imp = 0, n_act = 0, n_tasks = 0;
    uint32_t n_lane_edges = 0, n_lane_intra = 0;
    // the mark begun in the previous step (one per lane 0..UNR-1): target,
    // priority and the mask's old value, finished while the next step's
    // memory operations are in flight
    bool pm_on = false;
    uint32_t pm_u = 0, pm_val = 0;
    unsigned long long pm_old = 0;
    // SSSP/BFS: the marks a step decided, begun during the next step
    unsigned long long mk_bits = 0;
    uint32_t mk_u = 0, mk_val = 0;
    const __amdgpu_buffer_rsrc_t rsrc = row_rsrc(c.st, c.g.nv);
    for (;;) {
        uint32_t task = 0;
        if (lane == 0) task = atomicAdd(&S.next, 1u);
        task = (uint32_t)__builtin_amdgcn_readfirstlane((int)task);
        if (task >= ntask) break;
        ++n_tasks;
        const uint32_t f = task * GW + lane;
        const uint32_t cnt = nedge - task * GW < (uint32_t)GW ? nedge - task * GW : (uint32_t)GW;
        // edge `lane` of this task: its round vertex, target and weight
        uint32_t myk = 0, myu = 0, myw = 1u;
        float mythr = 0.f;
        if (lane < cnt) {
            myk = gedge_vertex(S, nr, f);
            const uint32_t v = c.v0 + S.rv[myk];
            const uint32_t e = c.g.rowptr[v] + (f - S.rnt[myk]);
            myu = c.g.col[e];
            if constexpr (!ppr) {
                if (WB != 0 && c.qt != Q_BFS) myw = edge_w<WB>(c.g.w, e);
            }
            if constexpr (ppr) mythr = (float)(c.g.rowptr[myu + 1] - c.g.rowptr[myu]);  // degree, scaled per lane below
        }
        uint32_t kprev = 0xffffffffu, dprev = INF;
        float sprev = 0.f;
        bool aprev = false;
        // Step j0's edges: targets u (wave-uniform), this lane's value through
        // each edge x (SSSP/BFS: distance; PPR: the pushed share's bits), and
        // the masks actm (bit j: this lane relaxes / pushes along edge j0 + j)
        // and imask (bit j: edge j0 + j stays in the partition).  Edge j0 + j's
        // source, target and weight are the same for every lane: they are read
        // from lane j0 + j into scalar registers.
        auto gather = [&](uint32_t j0, uint32_t (&u)[UNR], uint32_t (&x)[UNR], uint32_t& actm, uint32_t& imask) {
            actm = 0;
            imask = 0;
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const uint32_t fj = j0 + j;
                const bool ok = fj < cnt;
                const uint32_t kj = (uint32_t)__builtin_amdgcn_readlane((int)myk, (int)(fj & (GW - 1)));
                u[j] = (uint32_t)__builtin_amdgcn_readlane((int)myu, (int)(fj & (GW - 1)));
                if (ok && kj != kprev) {  // a new source vertex (uniform): its mask and this lane's value
                    kprev = kj;
                    const unsigned long long m = S.rm[kj];
                    aprev = (m >> lane) & 1ull;
                    if constexpr (ppr) sprev = SH.share[kj][lane];
                    else dprev = aprev ? SH.sd[kj][lane] : INF;
                }
                actm |= (ok && aprev) ? (1u << j) : 0u;
                imask |= (ok && u[j] - c.v0 < c.nvp) ? (1u << j) : 0u;
                if constexpr (ppr) {
                    x[j] = __float_as_uint(sprev);
                } else {
                    const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)myw, (int)(fj & (GW - 1)));
                    const uint32_t sum = dprev + w;  // dprev < INF: no wrap unless the path is too long
                    x[j] = (sum < dprev || sum >= INF) ? INF - 1 : sum;
                }
            }
        };
        if constexpr (ppr) {
            for (uint32_t j0 = 0; j0 < cnt; j0 += UNR) {
                uint32_t u[UNR], x[UNR], y[UNR];  // y: the target's residual before the push (float bits)
                uint32_t actm, imask;
                gather(j0, u, x, actm, imask);
                n_lane_edges += (uint32_t)__popc(actm);
                n_lane_intra += (uint32_t)__popc(actm & imask);
#pragma unroll
                for (int j = 0; j < UNR; ++j)
                    y[j] = ((actm >> j) & 1u) ? __float_as_uint(__hip_atomic_fetch_add(
                                                    rowf((float*)c.st, u[j], lane), __uint_as_float(x[j]),
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                              : 0u;
                if (pm_on) { pm_on = false; n_act += gmark_end(c, S, pm_u, pm_old, pm_val) ? 1u : 0u; }
                // lane j marks the target of edge j0 + j for every lane that crossed its threshold
                unsigned long long mine_bits = 0;
                uint32_t mine_val = 0, mine_u = 0;
#pragma unroll
                for (int j = 0; j < UNR; ++j) {
                    const bool act = (actm >> j) & 1u;
                    const float du = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mythr),
                                                                              (int)((j0 + j) & (GW - 1))));
                    const float thu = c.mode ? c.eps * du : c.eps;
                    const float old = __uint_as_float(y[j]);
                    const float nr_ = old + __uint_as_float(x[j]);
                    const bool hit = act && !ppr_active(old, thu) && ppr_active(nr_, thu);
                    const uint32_t val = ~__float_as_uint(nr_);
                    const unsigned long long bm = wballot(hit);
                    if (bm) {  // uniform
                        const uint32_t vj = (uint32_t)__builtin_amdgcn_readlane((int)val, __ffsll(bm) - 1);
                        if (lane == (uint32_t)j) { mine_bits = bm; mine_val = vj; mine_u = u[j]; }
                    }
                }
                if (mine_bits) {
                    pm_old = gmark_begin(c, mine_u, mine_bits);
                    pm_u = mine_u;
                    pm_val = mine_val;
                    pm_on = true;
                }
            }
        } else {
            // step A is the one being relaxed, step B the next one, whose row
            // loads are in flight meanwhile
            uint32_t uA[UNR], xA[UNR], yA[UNR], actA, imA;
            gather(0, uA, xA, actA, imA);
#pragma unroll
            for (int j = 0; j < UNR; ++j)
                yA[j] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, ((actA >> j) & 1u) ? row_off(uA[j], lane) : ROW_NONE,
                                                             0, 0);
            for (uint32_t j0 = 0; j0 < cnt; j0 += UNR) {
                n_lane_edges += (uint32_t)__popc(actA);
                n_lane_intra += (uint32_t)__popc(actA & imA);
                // y: the target's value; then the old value at this lane's atomic min (0: none made).
                // Which minima to make is decided for the whole step first (the empty asm keeps the
                // mask opaque), so that every row load of the step is waited for before the first
                // atomic is issued: a wait for one load issued after an atomic would wait for the
                // atomic too.
                uint32_t amask = 0;
#pragma unroll
                for (int j = 0; j < UNR; ++j) amask |= (((actA >> j) & 1u) && xA[j] < yA[j]) ? (1u << j) : 0u;
                asm volatile("" : "+v"(amask));
#pragma unroll
                for (int j = 0; j < UNR; ++j)
                    yA[j] = ((amask >> j) & 1u) ? dev_min(rowp(c.st, uA[j], lane), xA[j]) : 0u;
                // the previous step's marks, begun now that this step's minima are in flight
                if (mk_bits) {
                    pm_old = gmark_begin(c, mk_u, mk_bits);
                    pm_u = mk_u;
                    pm_val = mk_val;
                    pm_on = true;
                    mk_bits = 0;
                }
                uint32_t uB[UNR], xB[UNR], yB[UNR], actB = 0, imB = 0;
                const bool more = j0 + UNR < cnt;  // uniform
                if (more) {
                    gather(j0 + UNR, uB, xB, actB, imB);
#pragma unroll
                    for (int j = 0; j < UNR; ++j)
                        yB[j] = __builtin_amdgcn_raw_buffer_load_b32(
                            rsrc, ((actB >> j) & 1u) ? row_off(uB[j], lane) : ROW_NONE, 0, 0);
                }
                if (pm_on) { pm_on = false; n_act += gmark_end(c, S, pm_u, pm_old, pm_val) ? 1u : 0u; }
                // lane j will mark the target of edge j0 + j for every lane that lowered it
#pragma unroll
                for (int j = 0; j < UNR; ++j) {
                    const bool hit = xA[j] < yA[j];  // yA[j] = 0 where no atomic was made
                    const unsigned long long bm = wballot(hit);
                    if (bm) {  // uniform
                        const uint32_t vj = (uint32_t)__builtin_amdgcn_readlane((int)xA[j], __ffsll(bm) - 1);
                        if (lane == (uint32_t)j) { mk_bits = bm; mk_val = vj; mk_u = uA[j]; }
                        n_imp += (uint32_t)__popcll(bm);
                    }
                }
                if (more) {
#pragma unroll
                    for (int j = 0; j < UNR; ++j) {
                        uA[j] = uB[j];
                        xA[j] = xB[j];
                        yA[j] = yB[j];
                    }
                    actA = actB;
                    imA = imB;
                }
            }
        }
    }
    if (pm_on) n_act += gmark_end(c, S, pm_u, pm_old, pm_val) ? 1u : 0u;
    if (mk_bits) n_act += gmark(c, S, mk_u, mk_bits, mk_val) ? 1u : 0u;
    // n_act counted per lane (lanes 0..UNR-1 mark), and the lane-edges
    uint32_t n_edges = n_lane_edges, n_intra = n_lane_intra;
    for (int o = 32; o; o >>= 1) {
        n_act += __shfl_xor(n_act, o);
        n_edges += __shfl_xor(n_edges, o);
        n_intra += __shfl_xor(n_intra, o);
    }
    gcount(S, K_EDGES, n_edges);
    if constexpr (ppr) gcount(S, K_EDGES_PPR, n_edges);
    gcount(S, K_INTRA, n_intra);
    gcount(S, K_IMPROVED, n_imp);
    gcount(S, K_ACT, n_act);
    gcount(S, K_TASKS, n_tasks);
    if (lane == 0 && n_edges) atomicAdd(&S.edges, (unsigned long long)n_edges);
}

// One visit of the (partition, group) pair of S.it.
template <int WB>
__device__ void gvisit(GCtx& c, GShared& S, GCtxShare& SH, const PassCfg& cfg) {
    const uint32_t t = threadIdx.x;
    const uint32_t lane = lane_id();
    c.qt = c.G.gtype[c.grp];
    c.v0 = c.g.pstart[c.P];
    c.nvp = c.g.pstart[c.P + 1] - c.v0;
    const unsigned long long off = c.G.goff[c.grp];
    c.st = c.G.state + off;
    c.pp = (float*)(c.G.state + off + (unsigned long long)c.g.nv * GW);
    c.alpha = c.G.lalpha[c.grp * GW + lane];
    c.eps = c.G.leps[c.grp * GW + lane];
    c.mode = c.G.lmode[c.grp * GW + lane];
    c.win = INF;
    c.bwin = c.qt == Q_BFS ? cfg.win_lv : cfg.win_sp;
    if (c.bwin == 0) c.bwin = INF;
    if (cfg.gate && c.qt != Q_PPR) {
        const unsigned long long d = c.qt == Q_BFS ? cfg.yld_lv : cfg.yld_sp;
        const unsigned long long w = (unsigned long long)c.G.gmin[c.grp] + d;
        c.win = d == 0 ? INF : (w >= INF ? INF : (uint32_t)w);
    }
    // time of the visit's phases, read by thread 0 between barriers (10 ns ticks)
    if (t == 0) S.tk = wall_clock64();
    auto phase = [&](int k) {
        if (t == 0) {
            const unsigned long long now = wall_clock64();
            S.cnt[k] += now - S.tk;
            S.tk = now;
        }
    };
    // the pair's pending vertices: global bitmap -> LDS
    const uint32_t nw = (c.nvp + 31) / 32;
    for (uint32_t w = t; w < nw; w += blockDim.x) {
        const uint32_t u0 = c.v0 + w * 32;  // first vertex of local word w
        // the partition starts on a multiple of 2^pshift, which may not be a
        // multiple of 32: gather the 32 bits from up to two global words
        const uint32_t gw = u0 >> 5, sh = u0 & 31;
        const uint32_t lim = c.nvp - w * 32 < 32 ? c.nvp - w * 32 : 32;
        const uint32_t want = lim == 32 ? 0xffffffffu : ((1u << lim) - 1u);
        uint32_t* base = c.G.bits + (unsigned long long)c.grp * c.G.bw;
        uint32_t lo = 0, hi = 0;
        const uint32_t m_lo = want << sh;
        if (m_lo) lo = atomicAnd(&base[gw], ~m_lo) & m_lo;
        if (sh) {
            const uint32_t m_hi = want >> (32 - sh);
            if (m_hi) hi = atomicAnd(&base[gw + 1], ~m_hi) & m_hi;
        }
        S.lbits[w] = (lo >> sh) | (sh ? (hi << (32 - sh)) : 0u);
    }
    if (t == 0) S.edges = 0;
    __syncthreads();
    phase(K_T_GATHER);
    unsigned long long budget = 0;
    if (cfg.mu > 0.f) {
        const uint32_t np_items = c.B.pn[c.P];
        const float e_p = (float)(c.g.rowptr[c.v0 + c.nvp] - c.g.rowptr[c.v0]) * (float)GW;
        const float bgt = cfg.mu * e_p / (float)(np_items ? np_items : 1u);
        budget = bgt < 16384.f ? 16384ull : (unsigned long long)bgt;
    }
    const bool ppr = c.qt == Q_PPR;
    for (;;) {
        const uint32_t nr = gtake_round(c, S, (uint32_t)RCAP);
        phase(K_T_TAKE);
        if (nr == 0) break;
        if (ppr) {
            gfilter_ppr(c, S, SH, nr);
        } else {
            ground_min(c, S, nr);
            gfilter_sp(c, S, SH, nr);
        }
        const uint32_t nedge = gnumber_edges(S, nr);
        if (t == 0) { S.next = 0; S.cnt[K_ROUNDS] += 1; }
        __syncthreads();
        phase(K_T_FILTER);
        if (ppr) gtasks<WB, true>(c, S, SH, nr, nedge);
        else gtasks<WB, false>(c, S, SH, nr, nedge);
        __syncthreads();
        phase(K_T_TASKS);
        if (budget && S.edges >= budget) break;
    }
    __syncthreads();
    // yield: what is still pending in the partition stays in the pair's buffer
    for (uint32_t w = t; w < nw; w += blockDim.x) {
        uint32_t word = S.lbits[w];
        while (word) {
            const uint32_t b = __ffs(word) - 1;
            word &= word - 1;
            const uint32_t vloc = w * 32 + b;
            const uint32_t u = c.v0 + vloc;
            // priority of the held-back vertex: its best pending value (PPR: highest priority)
            uint32_t val = 0u;
            if (c.qt != Q_PPR) {
                const unsigned long long m = __hip_atomic_load(&c.G.pend[(unsigned long long)c.grp * c.g.nv + u],
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                val = 0xffffffffu;
                for (unsigned long long mm = m; mm; mm &= mm - 1) {
                    const uint32_t l = __ffsll(mm) - 1;
                    const uint32_t x = fresh_load(rowp(c.st, u, l));
                    val = x < val ? x : val;
                }
            }
            gkeep(c, vloc, val);
        }
        S.lbits[w] = 0u;
    }
    __syncthreads();
    phase(K_T_YIELD);
}

template <int WB>
__global__ __launch_bounds__(GNTMAX) void k_gprocess(GraphDev g, GroupDev G, BufDev B, PassCfg cfg) {
    __shared__ GShared S;
    __shared__ GCtxShare SH;
    GCtx c;
    c.g = g;
    c.G = G;
    c.B = B;
    const uint32_t t = threadIdx.x;
    if (t < (uint32_t)NCNT) S.cnt[t] = 0;
    const uint32_t xcd = blockIdx.x % NXCD;
    c.pass = B.ctl->pass;
    unsigned long long items = 0;
    for (;;) {
        if (t == 0) {
            unsigned long long pos = ~0ull;
            if (!__hip_atomic_load(&B.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                for (uint32_t k = 0; k < NXCD; ++k) {
                    const uint32_t x = (xcd + k) % NXCD;
                    uint32_t n = B.ctl->nitems[x];
                    n = n < B.item_cap ? n : B.item_cap;
                    if (__hip_atomic_load(&B.ctl->next[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
                    const uint32_t idx = dev_add(&B.ctl->next[x], 1u);
                    if (idx < n) { pos = (unsigned long long)x * B.item_cap + idx; break; }
                }
            }
            S.itpos = pos;
        }
        __syncthreads();
        const unsigned long long pos = S.itpos;
        if (pos == ~0ull) break;
        if (t == 0) { S.it.part = B.items[pos].part; S.it.q = B.items[pos].q; }
        __syncthreads();
        c.P = S.it.part;
        c.grp = S.it.q;
        ++items;
        gvisit<WB>(c, S, SH, cfg);
    }
    // counters
    __syncthreads();
    if (t < (uint32_t)NCNT && S.cnt[t]) {
        Ctl* k = B.ctl;
        unsigned long long* d = t == K_EDGES ? &k->c_edges : t == K_INTRA ? &k->c_intra
                              : t == K_IMPROVED ? &k->c_improved : t == K_VPUSH ? &k->c_vpush
                              : t == K_ACT ? &k->c_act : t == K_EDGES_PPR ? &k->c_edges_ppr
                              : t == K_VPUSH_PPR ? &k->c_vpush_ppr : t == K_VTASK ? &k->c_vtask
                              : t == K_ROUNDS ? &k->c_rounds : t == K_TASKS ? &k->c_tasks
                              : &k->c_tphase[t - K_T_GATHER];
        dev_add(d, S.cnt[t]);
    }
    if (t == 0 && items) dev_add(&B.ctl->c_items, items);
}

// Per group: its best pending SSSP/BFS value over all partitions (the
// query-global dist_min of heuristic 2, taken over the group's queries).
__global__ void k_gmin(GroupDev G, uint32_t np) {
    const uint32_t grp = blockIdx.x * blockDim.x + threadIdx.x;
    if (grp >= G.ng) return;
    uint32_t m = 0xffffffffu;
    if (G.gtype[grp] != Q_PPR)
        for (uint32_t P = 0; P < np; ++P) {
            const unsigned long long pi = (unsigned long long)P * G.ng + grp;
            if (G.icnt[pi]) m = G.ibest[pi] < m ? G.ibest[pi] : m;
        }
    G.gmin[grp] = m;
}

// Partition summaries from the pairs' summaries, in the form the scheduler
// (select step, learned scorer) reads: pending activations, best SSSP
// distance / BFS level / PPR residual, pairs pending and ready, age.
__global__ __launch_bounds__(256) void k_gsum(GroupDev G, BufDev B, PassCfg cfg) {
    const uint32_t P = blockIdx.x;
    __shared__ unsigned long long s_cnt;
    __shared__ unsigned int s_sp, s_lv, s_pr, s_ne, s_rd, s_first, s_hm;
    if (threadIdx.x == 0) { s_cnt = 0; s_sp = INF; s_lv = INF; s_pr = 0; s_ne = 0; s_rd = 0; s_first = INF; s_hm = 0; }
    __syncthreads();
    unsigned long long cnt = 0;
    uint32_t sp = INF, lv = INF, pr = 0, ne = 0, rd = 0, first = INF, hm = 0;
    for (uint32_t grp = threadIdx.x; grp < G.ng; grp += blockDim.x) {
        const unsigned long long pi = (unsigned long long)P * G.ng + grp;
        const uint32_t cb = G.icnt[pi];
        if (!cb) continue;
        const uint32_t v = G.ibest[pi], t = G.gtype[grp];
        cnt += cb;
        ++ne;
        if (t == Q_PPR) { const uint32_t m = ~v; pr = m > pr ? m : pr; }
        else if (t == Q_BFS) lv = v < lv ? v : lv;
        else sp = v < sp ? v : sp;
        rd += bucket_ready(v, t, G.gmin[grp], cfg);
        hm += (t != Q_PPR && v == G.gmin[grp]) ? 1u : 0u;
        const uint32_t f = G.ifirst[pi];
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
}

// Detach the ready pairs of the selected partitions into work items.
__global__ __launch_bounds__(256) void k_gworklist(BufDev B, GroupDev G, PassCfg cfg) {
    const uint32_t j = blockIdx.x;
    Ctl* ctl = B.ctl;
    if (ctl->err || j >= ctl->nsel) return;
    const uint32_t P = B.sel[j];
    const uint32_t x = j % NXCD;
    const uint32_t grp = blockIdx.y * 256 + threadIdx.x;
    bool has = false;
    unsigned long long pi = 0;
    if (grp < G.ng) {
        pi = (unsigned long long)P * G.ng + grp;
        has = G.icnt[pi] && bucket_ready(G.ibest[pi], G.gtype[grp], G.gmin[grp], cfg);
    }
    const unsigned long long mask = wballot(has);
    const uint32_t n = __popcll(mask);
    if (!n) return;
    uint32_t base = 0;
    if (lane_id() == 0) { base = dev_add(&ctl->nitems[x], n); dev_add(&B.pn[P], n); }
    base = __shfl(base, 0);
    if (has) {
        const uint32_t pos = base + rank_in(mask);
        if (pos < B.item_cap) {
            Item* it = &B.items[(unsigned long long)x * B.item_cap + pos];
            it->part = P;
            it->q = grp;
            it->nch = 0;
            it->rest = -1;
            G.icnt[pi] = 0;
            G.ibest[pi] = 0xffffffffu;
            G.ifirst[pi] = 0xffffffffu;
        } else {
            dev_or(&ctl->err, (uint32_t)ERR_ITEMS);
        }
    }
}

// Sources: lane l of group g starts at src[g*64 + l] (0xffffffff: unused lane).
__global__ void k_gseed(GraphDev g, GroupDev G, const uint32_t* src) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= G.ng * GW) return;
    const uint32_t grp = i / GW, lane = i % GW, s = src[i];
    if (s >= g.nv) return;
    uint32_t* st = G.state + G.goff[grp];
    const bool ppr = G.gtype[grp] == Q_PPR;
    if (ppr) ((float*)st)[(unsigned long long)s * GW + lane] = 1.0f;
    else st[(unsigned long long)s * GW + lane] = 0u;
    dev_or(&G.pend[(unsigned long long)grp * g.nv + s], 1ull << lane);
    dev_or(&G.bits[(unsigned long long)grp * G.bw + (s >> 5)], 1u << (s & 31));
    const uint32_t P = g.vpart[s >> g.pshift];
    const unsigned long long pi = (unsigned long long)P * G.ng + grp;
    dev_add(&G.icnt[pi], 1u);
    dev_min(&G.ibest[pi], ppr ? ~__float_as_uint(1.0f) : 0u);
    dev_min(&G.ifirst[pi], 0u);
}

// Group state (vertex-major rows of 64 lanes) -> per-query vectors.  One
// block transposes a tile of 64 vertices x 64 lanes of one group.
__global__ __launch_bounds__(256) void k_gout(GroupDev G, uint32_t nv, uint32_t* out, const unsigned long long* qoff,
                                              const uint32_t* lq) {
    __shared__ uint32_t tile[GW][GW + 1];
    const uint32_t grp = blockIdx.y, v0 = blockIdx.x * GW;
    const bool ppr = G.gtype[grp] == Q_PPR;
    const uint32_t* src = G.state + G.goff[grp];
    for (int part = 0; part < (ppr ? 2 : 1); ++part) {
        // PPR: part 0 = p (the second block of the group state), part 1 = r
        const uint32_t* s = src + (ppr && part == 0 ? (unsigned long long)nv * GW : 0ull);
        for (uint32_t i = threadIdx.x; i < GW * GW; i += blockDim.x) {
            const uint32_t dv = i / GW, l = i % GW;
            tile[dv][l] = v0 + dv < nv ? s[(unsigned long long)(v0 + dv) * GW + l] : 0u;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < GW * GW; i += blockDim.x) {
            const uint32_t l = i / GW, dv = i % GW;
            const uint32_t q = lq[grp * GW + l];
            if (q != 0xffffffffu && v0 + dv < nv)
                out[qoff[q] + (ppr && part == 1 ? nv : 0u) + v0 + dv] = tile[dv][l];
        }
        __syncthreads();
    }
}

// Digests of a wave's queries straight from the group rows (for waves whose
// vectors are not kept, so that they need no transpose): the definition of
// k_digest per lane.  One block sums a chunk of vertices of one group, its
// four waves reduced in LDS; then one lane per query adds to the query's
// digest (SSSP/BFS count, sum, hash; PPR count of p > 0, sum p, sum r, max p).
// `out` starts zeroed.
constexpr uint32_t GDCHUNK = 16384;
__global__ __launch_bounds__(256) void k_gdigest(GroupDev G, uint32_t nv, const uint32_t* lq, unsigned long long* out,
                                                 const uint32_t* orig) {
    const uint32_t grp = blockIdx.y, v0 = blockIdx.x * GDCHUNK;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t v1 = nv - v0 < GDCHUNK ? nv : v0 + GDCHUNK;
    const bool ppr = G.gtype[grp] == Q_PPR;
    const uint32_t* st = G.state + G.goff[grp];
    unsigned long long cnt = 0, sum = 0, hash = 0;
    double f0 = 0, f1 = 0;
    float fmax = 0.f;
    if (ppr) {
        const float* r = (const float*)st;
        const float* p = (const float*)(st + (unsigned long long)nv * GW);
        for (uint32_t v = v0 + wv; v < v1; v += 4) {
            const float pv = p[(unsigned long long)v * GW + lane];
            cnt += pv > 0.f;
            f0 += pv;
            f1 += r[(unsigned long long)v * GW + lane];
            fmax = pv > fmax ? pv : fmax;
        }
    } else {
        for (uint32_t v = v0 + wv; v < v1; v += 4) {
            const uint32_t x = st[(unsigned long long)v * GW + lane];
            if (x != INF) {
                ++cnt;
                sum += x;
                hash += mix64(((unsigned long long)(orig ? orig[v] : v) << 32) | x);
            }
        }
    }
    __shared__ unsigned long long s_u[3][4][GW];
    __shared__ double s_d[2][4][GW];
    __shared__ float s_m[4][GW];
    s_u[0][wv][lane] = cnt; s_u[1][wv][lane] = sum; s_u[2][wv][lane] = hash;
    s_d[0][wv][lane] = f0; s_d[1][wv][lane] = f1; s_m[wv][lane] = fmax;
    __syncthreads();
    if (wv != 0) return;
    const uint32_t q = lq[grp * GW + lane];
    if (q == 0xffffffffu) return;
    for (int w = 1; w < 4; ++w) {
        cnt += s_u[0][w][lane]; sum += s_u[1][w][lane]; hash += s_u[2][w][lane];
        f0 += s_d[0][w][lane]; f1 += s_d[1][w][lane];
        fmax = s_m[w][lane] > fmax ? s_m[w][lane] : fmax;
    }
    unsigned long long* o = out + (unsigned long long)q * 6;
    if (cnt) { atomicAdd(&o[0], cnt); atomicAdd(&o[1], sum); atomicAdd(&o[2], hash); }
    if (ppr) {
        atomicAdd((double*)&o[3], f0);
        atomicAdd((double*)&o[4], f1);
        // non-negative doubles order as their bit patterns
        atomicMax(&o[5], (unsigned long long)__double_as_longlong((double)fmax));
    }
}

// ------------------------------------------------------------ launchers
hipError_t launch_gdigest(const GroupDev& G, uint32_t nv, const uint32_t* lq, unsigned long long* out,
                          const uint32_t* orig, hipStream_t s) {
    hipLaunchKernelGGL(k_gdigest, dim3((nv + GDCHUNK - 1) / GDCHUNK, G.ng), dim3(256), 0, s, G, nv, lq, out, orig);
    return hipGetLastError();
}
hipError_t launch_gprocess(const GraphDev& g, const GroupDev& G, const BufDev& B, const PassCfg& cfg, uint32_t blocks,
                           uint32_t nth, hipStream_t s) {
    if (nth != 256 && nth != 512 && nth != 1024) return hipErrorInvalidValue;
    switch (g.wbytes) {
    case 0: hipLaunchKernelGGL((k_gprocess<0>), dim3(blocks), dim3(nth), 0, s, g, G, B, cfg); break;
    case 1: hipLaunchKernelGGL((k_gprocess<1>), dim3(blocks), dim3(nth), 0, s, g, G, B, cfg); break;
    case 2: hipLaunchKernelGGL((k_gprocess<2>), dim3(blocks), dim3(nth), 0, s, g, G, B, cfg); break;
    default: hipLaunchKernelGGL((k_gprocess<4>), dim3(blocks), dim3(nth), 0, s, g, G, B, cfg); break;
    }
    return hipGetLastError();
}
const void* gprocess_kernel_ptr(int wbytes) {
    switch (wbytes) {
    case 0: return (const void*)k_gprocess<0>;
    case 1: return (const void*)k_gprocess<1>;
    case 2: return (const void*)k_gprocess<2>;
    default: return (const void*)k_gprocess<4>;
    }
}
hipError_t launch_gsummaries(const GraphDev& g, const GroupDev& G, const BufDev& B, const PassCfg& cfg, hipStream_t s) {
    hipLaunchKernelGGL(k_gmin, dim3((G.ng + 255) / 256), dim3(256), 0, s, G, g.np);
    hipLaunchKernelGGL(k_gsum, dim3(g.np), dim3(256), 0, s, G, B, cfg);
    return hipGetLastError();
}
hipError_t launch_gworklist(const BufDev& B, const GroupDev& G, const PassCfg& cfg, hipStream_t s) {
    dim3 grid(cfg.kmax, (G.ng + 255) / 256);
    hipLaunchKernelGGL(k_gworklist, grid, dim3(256), 0, s, B, G, cfg);
    return hipGetLastError();
}
hipError_t launch_gseed(const GraphDev& g, const GroupDev& G, const uint32_t* src, hipStream_t s) {
    hipLaunchKernelGGL(k_gseed, dim3((G.ng * GW + 255) / 256), dim3(256), 0, s, g, G, src);
    return hipGetLastError();
}
hipError_t launch_gout(const GroupDev& G, uint32_t nv, uint32_t* out, const unsigned long long* qoff, const uint32_t* lq,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_gout, dim3((nv + GW - 1) / GW, G.ng), dim3(256), 0, s, G, nv, out, qoff, lq);
    return hipGetLastError();
}
int gprocess_threads() { return GNTMAX; }
size_t group_dev_bytes() { return sizeof(GroupDev); }

}  // namespace fk
