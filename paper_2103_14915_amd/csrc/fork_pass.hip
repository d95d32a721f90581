// IntraPartProcess on gfx950: one workgroup processes one (partition, query)
// work item at a time (Algorithm 2, the body of the parallel-for over the
// queries of the scheduled partition).
//
// Mapping of the paper's cache design onto the MI355X:
//   * the scheduled partition's edges are read from L2, shared by the
//     workgroups of the XCD that process other queries of the same partition
//     (the paper keeps the partition in the LLC shared by all cores);
//   * the query's state slice for the partition (distances, or PPR
//     residuals) is staged in LDS for the whole visit, so every relaxation
//     inside the partition is an LDS atomic (the paper keeps the query's
//     state in contiguous memory owned by one thread, Section 4.2);
//   * one workgroup owns the slice, so no other workgroup touches it during
//     the pass; lanes combine concurrent updates with LDS atomics.
// Inside the visit, work is taken in priority order (Section 4.2): SSSP in
// distance windows [lo, lo + win) smallest first (Dijkstra order, batched),
// BFS level by level, PPR by pushing every vertex above its threshold.
// Yielding (Section 5.1): heuristic 2 stops once the window start passes the
// first value plus a range; heuristic 1 stops after an edge budget.  The
// unfinished frontier is retained as operations in the partition's own buffer.
// Operations for other partitions are staged in LDS, consolidated per target
// vertex (min value / summed mass), grouped by target partition and appended
// to the target buffers with one chunk reservation per flush (Algorithm 2:
// send after processing; Appendix B.1: reserve a range, then copy).
#include <hip/hip_cooperative_groups.h>

#include "fork_mlp.h"
#include "fork_sched.h"

namespace fk {

constexpr int NT = 256;           // threads per workgroup
constexpr int NW = NT / WAVE;     // waves per workgroup
constexpr int FCAP = 1024;        // frontier capacity (two buffers)
static_assert((uint32_t)FCAP >= CERT_MAX_PART || FORK_CERT_MAX_PART > 1024u, "a certified refinement fits the frontier");
constexpr int BCAP = 512;         // vertices expanded per batch
constexpr int SCAP = 512;         // staged outgoing operations
constexpr int CCAP = 128;         // chunk ids gathered per consume round
// Free chunks each workgroup keeps for itself: chunks freed by consume are
// reused by the same workgroup's next flush without touching the pool's ring
// counters (two single-address atomics per item otherwise).  A flush needs at
// most one fresh chunk per run plus SCAP/CH, so STASH >= SCAP + SCAP/CH + 1.
constexpr int STASH = 640;
constexpr int REFILL = 32;        // chunks taken from the ring per refill when the pool is not low
static_assert(STASH >= SCAP + SCAP / 256 + 1, "a flush must fit in the stash");
static_assert(CCAP <= NT && ICH <= CCAP, "one thread per chunk of a consume round");
constexpr int SE = (SCAP + NT - 1) / NT;

struct PassShared {
    uint32_t fq[2][FCAP];         // frontier (partition-local ids), double-buffered
    uint32_t bv[BCAP];            // batch vertex
    uint32_t bval[BCAP];          // batch distance, or PPR share (float bits)
    uint32_t brow[BCAP];          // batch first edge
    uint32_t bpre[BCAP];          // batch exclusive degree prefix
    unsigned long long sk[SCAP];  // staged ops (vertex << 32 | value)
    uint32_t tp[SCAP];            // target partition of compacted staged op
    int32_t rt[SCAP];             // per run: tail chunk (-1: none)
    uint32_t rp[SCAP];            // per run: slot | taken << 9 | fresh-chunk base << 18
    uint32_t rbest[SCAP];         // per run: best value (SSSP/BFS min value, PPR ~mass)
    int32_t clist[CCAP];          // chunk ids of the consume round
    uint32_t ccnt[CCAP];          // their valid ops
    uint32_t cpre[CCAP];          // exclusive prefix of ccnt
    uint32_t stash[STASH];        // free chunks owned by this workgroup
    uint32_t nstash, nrefill;
    uint32_t nspill;              // activated vertices this item retained (frontier full)
    uint32_t wred[NW];
    uint32_t nf, nk, nb, ns, ncl, cur;
    int32_t chnext;
    unsigned long long base, itpos;
    Item it;
};

// -------------------------------------------------------- block helpers

// Exclusive prefix sum over the block; *total gets the sum.
__device__ __forceinline__ uint32_t block_excl(PassShared& S, uint32_t v, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = wscan_incl(v, lane);
    if (lane == 63) S.wred[wid] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t x = S.wred[w];
        before += (w < (int)wid) ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__device__ __forceinline__ uint32_t block_min(PassShared& S, uint32_t v) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wmin(v);
    if (lane == 0) S.wred[wid] = v;
    __syncthreads();
    uint32_t r = S.wred[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = S.wred[w] < r ? S.wred[w] : r;
    __syncthreads();
    return r;
}

// Exclusive max-scan over the block (0 for thread 0).
__device__ __forceinline__ uint32_t block_max_excl(PassShared& S, uint32_t v) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = wscan_max_incl(v, lane);
    if (lane == 63) S.wred[wid] = incl;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        if (w < (int)wid) before = S.wred[w] > before ? S.wred[w] : before;
    __syncthreads();
    uint32_t ex = __shfl_up(incl, 1);
    if (lane == 0) ex = 0;
    return ex > before ? ex : before;
}

// Position in an LDS list for lanes with `want` (one LDS atomic per wave).
__device__ __forceinline__ uint32_t block_append(bool want, uint32_t* counter) {
    unsigned long long mask = wballot(want);
    uint32_t n = __popcll(mask);
    uint32_t base = 0;
    if ((threadIdx.x & 63) == 0 && n) base = atomicAdd(counter, n);
    base = __shfl(base, 0);
    return base + rank_in(mask);
}

__device__ __forceinline__ bool tas(uint32_t* bits, uint32_t v) {
    uint32_t bit = 1u << (v & 31);
    return !(atomicOr(&bits[v >> 5], bit) & bit);
}

struct ItemCtx {
    GraphDev g;
    QueryDev Q;
    BufDev B;
    uint32_t P, q, qt, v0, nvp, pass, mode;
    uint32_t qlo;       // query's best buffered value at the start of the pass (INF: unknown)
    float alpha, eps;
    uint32_t* gstate;   // global state of the query (dist, or r for PPR)
    float* gp;          // PPR p
    uint32_t* st;       // LDS slice: values by vertex (dense) or by hash slot
    uint32_t* hkeys;    // hashed slice: vertex of each slot (EMPTY_KEY if free)
    uint32_t hn;        // hashed slice: number of slots (0: dense slice)
    uint32_t* bits;     // LDS in-frontier flags (by vertex)
    // per-thread counters
    unsigned long long c_edges, c_intra, c_improved, c_emitted, c_consumed, c_vpush, c_chunks, c_pruned;
    unsigned long long c_edges_ppr, c_vpush_ppr, c_spill;
    // per-item usefulness (trace runs): work units whose value was final / all
    float it_useful, it_work;
    const uint32_t* gfinal;  // final state of the query (trace runs), else NULL
};

// LDS slice entries are fetched on first touch, so a visit moves HBM traffic
// in proportion to the vertices it touches, not to the partition size.
constexpr uint32_t UNLOADED = 0xffffffffu;  // no distance or residual has this value

constexpr uint32_t EMPTY_KEY = 0xffffffffu;
constexpr int MAXPROBE = 32;

// Where vertex vloc's value lives during the visit, fetched on first touch.
// Dense slice: st[vloc].  Hashed slice (for partitions whose visits touch few
// of their vertices): an LDS open-addressing table; a vertex whose probe path
// is full stays in global memory for the whole visit (slots are never freed
// during a visit, so every thread reaches the same decision).
//
// In the hashed form a slot's key word also carries the vertex's frontier
// flag (FRONT), so no per-vertex flag array is needed and the table can use
// that LDS.  A vertex kept in global memory has no flag: it may enter the
// frontier more than once, which repeats no update (a second SSSP expansion
// finds no shorter path, a second PPR push finds its residual already taken).
constexpr uint32_t FRONT = 0x80000000u;

// LDS index of vertex vloc's value for this visit (claimed on first touch), or
// -1 when it stays in global memory.
__device__ __forceinline__ int32_t slot_index(const ItemCtx& c, uint32_t vloc) {
    if (!c.hn) return (int32_t)vloc;
    // Fibonacci hashing: the top bits of vloc * 2^32/phi pick the home slot
    uint32_t h = (uint32_t)(((unsigned long long)(vloc * 0x9E3779B1u) * c.hn) >> 32);
    for (int i = 0; i < MAXPROBE; ++i) {
        uint32_t k = c.hkeys[h];
        if (k == EMPTY_KEY) k = atomicCAS(&c.hkeys[h], EMPTY_KEY, vloc);
        if (k == EMPTY_KEY || (k & ~FRONT) == vloc) return (int32_t)h;
        h = h + 1 == c.hn ? 0u : h + 1;
    }
    return -1;
}

// Pointer to vertex vloc's value, fetched from global memory on first touch.
__device__ __forceinline__ uint32_t* slot_at(const ItemCtx& c, int32_t idx, uint32_t vloc) {
    if (idx < 0) return c.gstate + c.v0 + vloc;
    if (c.st[idx] == UNLOADED) atomicCAS(&c.st[idx], UNLOADED, c.gstate[c.v0 + vloc]);
    return &c.st[idx];
}

__device__ __forceinline__ uint32_t* slot(const ItemCtx& c, uint32_t vloc) {
    return slot_at(c, slot_index(c, vloc), vloc);
}

// Frontier flag of vertex vloc (slot idx): set it, returning whether it was clear.
__device__ __forceinline__ bool front_set(const ItemCtx& c, int32_t idx, uint32_t vloc) {
    if (!c.hn) return tas(c.bits, vloc);
    if (idx < 0) return true;
    return !(atomicOr(&c.hkeys[idx], FRONT) & FRONT);
}
__device__ __forceinline__ void front_clear(const ItemCtx& c, uint32_t vloc) {
    if (!c.hn) {
        atomicAnd(&c.bits[vloc >> 5], ~(1u << (vloc & 31)));
        return;
    }
    const int32_t idx = slot_index(c, vloc);
    if (idx >= 0) atomicAnd(&c.hkeys[idx], ~FRONT);
}

// Value reads and updates through a slot: LDS instructions for the dense
// slice, flat (LDS or L2) atomics for the hashed one.
__device__ __forceinline__ uint32_t sv_get(const ItemCtx& c, uint32_t vloc) {
    if (!c.hn) return c.st[vloc];
    return __hip_atomic_load(slot(c, vloc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t at_min(const ItemCtx& c, uint32_t* p, uint32_t x) {
    if (!c.hn) return atomicMin(p, x);
    return __hip_atomic_fetch_min(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ float at_addf(const ItemCtx& c, uint32_t* p, float x) {
    if (!c.hn) return atomicAdd((float*)p, x);
    return __hip_atomic_fetch_add((float*)p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ float sv_addf(const ItemCtx& c, uint32_t vloc, float x) {
    return at_addf(c, slot(c, vloc), x);
}
__device__ __forceinline__ float sv_takef(const ItemCtx& c, uint32_t vloc) {
    uint32_t* p = slot(c, vloc);
    if (!c.hn) { uint32_t m = *p; *p = 0u; return __uint_as_float(m); }
    return __uint_as_float(__hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}
__device__ __forceinline__ void sv_putf(const ItemCtx& c, uint32_t vloc, float x) {
    // give back residual that was taken but did not qualify for a push
    if (x != 0.f) sv_addf(c, vloc, x);
}

__device__ __forceinline__ float thr_of(const ItemCtx& c, uint32_t gv) {
    if (!c.mode) return c.eps;
    return c.eps * (float)(c.g.rowptr[gv + 1] - c.g.rowptr[gv]);
}

// ------------------------------------------------------------ sort
// Sort the SCAP staged keys of S.sk ascending.  Each wave sorts its 128 keys
// in registers (two per lane) with a bitonic network whose exchanges are lane
// shuffles, so it needs no barrier; two merge rounds then combine the four
// sorted runs, each key moving to (its index in its run) + (the number of
// keys of the other run that precede it).
static_assert(SCAP == 2 * NT && NT == 4 * WAVE, "sort layout: four waves, two keys per lane");

__device__ __forceinline__ unsigned long long keep(unsigned long long x, unsigned long long y, bool want_min) {
    const bool lt = x < y;
    return want_min == lt ? x : y;
}

__device__ __forceinline__ uint32_t merged_pos(const PassShared& S, uint32_t i, unsigned long long x, uint32_t run) {
    const uint32_t base = i & ~(2 * run - 1);
    const bool left = i - base < run;
    const uint32_t own = i - base - (left ? 0u : run);
    const uint32_t other = left ? base + run : base;
    // ties: keys of the left run go first
    uint32_t lo = 0, hi = run;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const unsigned long long y = S.sk[other + mid];
        if (left ? y < x : y <= x) lo = mid + 1;
        else hi = mid;
    }
    return base + own + lo;
}

__device__ __forceinline__ void sort_staged(PassShared& S) {
    const uint32_t t = threadIdx.x, l = t & (WAVE - 1), w = t / WAVE;
    unsigned long long a = S.sk[2 * WAVE * w + l], b = S.sk[2 * WAVE * w + WAVE + l];
    // a holds element l of the wave's run, b element l + 64
    for (uint32_t k = 2; k <= 2 * WAVE; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j == WAVE) {  // k = 128: a and b are partners, ascending
                const unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
                a = lo;
                b = hi;
            } else {
                const unsigned long long pa = __shfl_xor(a, (int)j), pb = __shfl_xor(b, (int)j);
                const uint32_t ia = l, ib = WAVE + l;
                a = keep(a, pa, ((ia & j) == 0) == ((ia & k) == 0));
                b = keep(b, pb, ((ib & j) == 0) == ((ib & k) == 0));
            }
        }
    }
    S.sk[2 * WAVE * w + l] = a;
    S.sk[2 * WAVE * w + WAVE + l] = b;
    __syncthreads();
    for (uint32_t run = 2 * WAVE; run < (uint32_t)SCAP; run <<= 1) {
        const unsigned long long x0 = S.sk[t], x1 = S.sk[t + NT];
        const uint32_t p0 = merged_pos(S, t, x0, run), p1 = merged_pos(S, t + NT, x1, run);
        __syncthreads();
        S.sk[p0] = x0;
        S.sk[p1] = x1;
        __syncthreads();
    }
}

// ------------------------------------------------------------ flush
// Send the staged operations (block-collective; call with uniform control flow).
__device__ __forceinline__ void flush(ItemCtx& c, PassShared& S) {
    __syncthreads();
    const uint32_t ns = S.ns;
    if (ns == 0) return;
    const uint32_t t = threadIdx.x;
    for (uint32_t i = ns + t; i < (uint32_t)SCAP; i += NT) S.sk[i] = ~0ull;  // padding sorts last
    __syncthreads();
    sort_staged(S);
    const bool is_ppr = c.qt == Q_PPR;
    // consolidate equal target vertices; thread owns elements [t*SE, t*SE+SE)
    unsigned long long key[SE];
    bool kept[SE];
    uint32_t nk_l = 0;
#pragma unroll
    for (int k = 0; k < SE; ++k) {
        uint32_t i = t * SE + k;
        kept[k] = false;
        key[k] = 0;
        if (i < ns) {
            unsigned long long s = S.sk[i];
            uint32_t u = (uint32_t)(s >> 32);
            if (i == 0 || (uint32_t)(S.sk[i - 1] >> 32) != u) {
                if (is_ppr) {
                    float acc = __uint_as_float((uint32_t)s);
                    for (uint32_t j = i + 1; j < ns && (uint32_t)(S.sk[j] >> 32) == u; ++j)
                        acc += __uint_as_float((uint32_t)S.sk[j]);
                    s = ((unsigned long long)u << 32) | __float_as_uint(acc);
                }
                kept[k] = true;
                key[k] = s;
                ++nk_l;
            }
        }
    }
    uint32_t nk = 0;
    uint32_t pos = block_excl(S, nk_l, &nk);  // has barriers: all reads above are done
#pragma unroll
    for (int k = 0; k < SE; ++k) {
        if (kept[k]) {
            uint32_t u = (uint32_t)(key[k] >> 32);
            S.sk[pos] = key[k];
            S.tp[pos] = c.g.vpart[u >> c.g.pshift];
            ++pos;
        }
    }
    __syncthreads();
    // runs of equal target partition; the thread holding a run's last element owns it
    const uint32_t lo = t * SE, hi = (lo + SE < nk) ? lo + SE : nk;
    uint32_t rsmax = 0;
    for (uint32_t i = lo; i < hi; ++i)
        if (i == 0 || S.tp[i] != S.tp[i - 1]) rsmax = i;
    // start of the run still open where my block begins
    const uint32_t rstart_prev = block_max_excl(S, rsmax);
    // owners: one 64-bit add on the buffer's tail word reserves slots in the
    // tail chunk; what does not fit goes to fresh chunks.  The one owner whose
    // reservation covers slot CH of the tail (f <= CH < f + len) installs the
    // next tail; owners that arrive while it does (f > CH) use the overflow list.
    uint32_t need_l = 0;
    {
        uint32_t rsv = rstart_prev;
        for (uint32_t i = lo; i < hi; ++i) {
            uint32_t T = S.tp[i];
            if (i == 0 || T != S.tp[i - 1]) rsv = i;
            bool end = (i + 1 == nk) || (S.tp[i + 1] != T);
            if (!end) continue;
            uint32_t len = i - rsv + 1;
            unsigned long long b = (unsigned long long)T * c.Q.qc + c.q;
            const unsigned long long w = dev_add(&c.B.btw[b], (unsigned long long)len);
            uint32_t tl = (uint32_t)(w >> 32), f = (uint32_t)w;
            if (tl != 0xffffffffu && tl >= c.B.nch) {
                // a damaged tail word: flag it (the run ends) and keep every write in range
                dev_or(&c.B.ctl->err, (uint32_t)ERR_CORRUPT);
                tl = 0xffffffffu;
                f = CH + 1;
            }
            uint32_t kk = 0;
            if (tl != 0xffffffffu && f < (uint32_t)CH) kk = ((uint32_t)CH - f) < len ? ((uint32_t)CH - f) : len;
            S.rt[rsv] = (int32_t)tl;
            S.rp[rsv] = (f < 511u ? f : 511u) | (kk << 9) | (need_l << 18);
            S.rbest[rsv] = 0xffffffffu;
            need_l += (len - kk + CH - 1) / CH;
        }
    }
    uint32_t nnew = 0;
    uint32_t my_base = block_excl(S, need_l, &nnew);
    if (need_l) {
        uint32_t rsv = rstart_prev;
        for (uint32_t i = lo; i < hi; ++i) {
            uint32_t T = S.tp[i];
            if (i == 0 || T != S.tp[i - 1]) rsv = i;
            bool end = (i + 1 == nk) || (S.tp[i + 1] != T);
            if (end) S.rp[rsv] += my_base << 18;
        }
    }
    const unsigned long long nch = c.B.nch;
    if (t == 0) {
        // fresh chunks come from the stash; refill it from the pool's ring if short
        unsigned long long base = 0;
        uint32_t k = 0;
        const uint32_t have = S.nstash;
        if (nnew > have) {
            const unsigned long long head = __hip_atomic_load(&c.B.ctl->ring_head, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long avail = c.B.ctl->avail_end > head ? c.B.ctl->avail_end - head : 0ull;
            k = nnew - have;
            if (k < (uint32_t)REFILL && avail > 64ull * REFILL) k = REFILL;  // batch while the pool is not low
            if (k > (uint32_t)STASH - have) k = (uint32_t)STASH - have;
            base = dev_add(&c.B.ctl->ring_head, (unsigned long long)k);
            if (base + k > c.B.ctl->avail_end) {
                dev_or(&c.B.ctl->err, (uint32_t)ERR_CAPACITY);
                base = ~0ull;
            }
        }
        S.base = base;
        S.nrefill = k;
    }
    __syncthreads();
    if (S.base == ~0ull) {
        __syncthreads();
        if (t == 0) S.ns = 0;
        __syncthreads();
        return;
    }
    {
        const uint32_t k = S.nrefill, have = S.nstash;
        for (uint32_t i = t; i < k; i += NT) {
            uint32_t id = c.B.ring[(S.base + i) % nch];
            if (id >= nch) {  // a damaged free ring: flag it (the run ends), keep writes in range
                dev_or(&c.B.ctl->err, (uint32_t)ERR_CORRUPT);
                id = 0;
            }
            S.stash[have + i] = id;
        }
    }
    __syncthreads();
    // this flush takes the top nnew entries of the stash
    const uint32_t sb = S.nstash + S.nrefill - nnew;
    // every element writes its operation
    {
        uint32_t rsv = rstart_prev;
        for (uint32_t i = lo; i < hi; ++i) {
            if (i == 0 || S.tp[i] != S.tp[i - 1]) rsv = i;
            uint32_t off = i - rsv;
            uint32_t info = S.rp[rsv];
            uint32_t s = info & 0x1ffu, kk = (info >> 9) & 0x1ffu, cb = info >> 18;  // s: slot in the tail
            unsigned long long sv = S.sk[i];
            uint2 op = make_uint2((uint32_t)(sv >> 32), (uint32_t)sv);
            atomicMin(&S.rbest[rsv], is_ppr ? ~op.y : (op.y & ~RETAIN));  // the run's best value
            if (off < kk) {
                c.B.chunks[(unsigned long long)(uint32_t)S.rt[rsv] * CH + s + off] = op;
            } else {
                uint32_t j = (off - kk) / CH;
                uint32_t ch = S.stash[sb + cb + j];
                c.B.chunks[(unsigned long long)ch * CH + (off - kk) % CH] = op;
            }
        }
    }
    __syncthreads();
    // owners link their fresh chunks.  Every plain store below has a single
    // writer per pass: a chunk's link and count are written by the workgroup
    // that filled it, except a tail's, which only the owner that replaces the
    // tail writes (the detach of the next pass closes the last tail).
    {
        uint32_t rsv = rstart_prev;
        for (uint32_t i = lo; i < hi; ++i) {
            uint32_t T = S.tp[i];
            if (i == 0 || T != S.tp[i - 1]) rsv = i;
            bool end = (i + 1 == nk) || (S.tp[i + 1] != T);
            if (!end) continue;
            uint32_t len = i - rsv + 1;
            uint32_t info = S.rp[rsv];
            uint32_t f = info & 0x1ffu, kk = (info >> 9) & 0x1ffu, cb = info >> 18;
            uint32_t need = (len - kk + CH - 1) / CH;
            unsigned long long b = (unsigned long long)T * c.Q.qc + c.q;
            if (need) {
                const uint32_t first = S.stash[sb + cb];
                uint32_t last = first;
                for (uint32_t j = 1; j < need; ++j) {
                    uint32_t ch = S.stash[sb + cb + j];
                    c.B.cnext[last] = (int32_t)ch;
                    c.B.ccount[last] = CH;
                    last = ch;
                }
                const uint32_t fill = (len - kk) - (need - 1) * CH;
                const int32_t tl = S.rt[rsv];
                if (f <= (uint32_t)CH && f + len > (uint32_t)CH) {
                    // installer: link after the old tail (now full) and make `last` the tail
                    if (tl != -1) {
                        c.B.cnext[tl] = (int32_t)first;
                        c.B.ccount[tl] = CH;
                    } else {
                        c.B.bhead[b] = (int32_t)first;
                        c.B.bfirst[b] = c.pass;  // the buffer became non-empty
                    }
                    dev_xchg(&c.B.btw[b], ((unsigned long long)last << 32) | fill);
                } else {
                    c.B.ccount[last] = fill;
                    c.B.cnext[last] = dev_xchg(&c.B.bover[b], (int32_t)first);
                }
            }
            // bucket summary for the scheduler.  The count is kept in whole
            // chunks (nonzero exactly when the buffer holds operations), so it
            // changes only when a chunk is added; the best value is updated
            // only when this run improves it (a stale read can only be high,
            // since values only decrease between detaches).  Both feed the
            // schedule only, never the results.
            if (need) dev_add(&c.B.bcnt[b], need * (uint32_t)CH);
            const uint32_t best = S.rbest[rsv];
            if (best < __hip_atomic_load(&c.B.bval[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                dev_min(&c.B.bval[b], best);
            c.c_emitted += len;
        }
    }
    __syncthreads();
    if (t == 0) {
        c.c_chunks += nnew;
        S.ns = 0;
        S.nstash = sb;
    }
    __syncthreads();
}

// Make room for one staged op per thread (block-collective).
__device__ __forceinline__ void stage_room(ItemCtx& c, PassShared& S) {
    __syncthreads();
    if (S.ns + NT > SCAP) flush(c, S);
}

__device__ __forceinline__ void stage(PassShared& S, bool want, uint32_t u, uint32_t val) {
    uint32_t p = block_append(want, &S.ns);
    if (want) S.sk[p] = ((unsigned long long)u << 32) | val;
}

// Add activated vertices to the frontier buffer `cur`; beyond its capacity
// they are retained as operations (requires stage room for them).
__device__ __forceinline__ void push_frontier(ItemCtx& c, PassShared& S, uint32_t cur, bool want, uint32_t vloc,
                                              uint32_t retain_val) {
    uint32_t p = block_append(want, &S.nf);
    bool fits = want && p < (uint32_t)FCAP;
    if (fits) S.fq[cur][p] = vloc;
    c.c_spill += (want && !fits) ? 1u : 0u;
    const unsigned long long sm = wballot(want && !fits);
    if (sm && (threadIdx.x & 63) == 0) atomicAdd(&S.nspill, (uint32_t)__popcll(sm));
    stage(S, want && !fits, c.v0 + vloc, retain_val);
}

// ------------------------------------------------------------ consume
// Apply the work item's buffered operations to the LDS slice (consolidation
// of the buffer into the query's state) and free the chunks.
__device__ __forceinline__ void consume(ItemCtx& c, PassShared& S) {
    const uint32_t t = threadIdx.x;
    // first round: the chunks the detach listed in the item.  A chunk id out
    // of range means a damaged buffer: it is flagged (the run ends with the
    // consistency error) and read as an empty chunk, so no access leaves the pool.
    const uint32_t nch0 = S.it.nch < (uint32_t)ICH ? S.it.nch : (uint32_t)ICH;
    if (t < nch0) {
        uint32_t id = S.it.ch[t].x, cnt = S.it.ch[t].y;
        if (id >= c.B.nch) {
            dev_or(&c.B.ctl->err, (uint32_t)ERR_CORRUPT);
            id = 0;
            cnt = 0;
        }
        S.clist[t] = (int32_t)id;
        S.ccnt[t] = cnt;
    }
    if (t == 0) { S.ncl = nch0; S.chnext = S.it.rest; }
    __syncthreads();
    for (bool first = true;; first = false) {
        if (!first) {
            // longer lists: follow the chain
            if (t == 0) {
                int32_t ch = S.chnext;
                uint32_t n = 0;
                while (ch >= 0 && n < (uint32_t)CCAP) {
                    if ((unsigned long long)ch >= c.B.nch) {  // a damaged link: flag it, end the list
                        dev_or(&c.B.ctl->err, (uint32_t)ERR_CORRUPT);
                        ch = -1;
                        break;
                    }
                    S.clist[n++] = ch;
                    ch = c.B.cnext[ch];
                }
                S.ncl = n;
                S.chnext = ch;
            }
            __syncthreads();
            for (uint32_t i = t; i < S.ncl; i += NT) S.ccnt[i] = c.B.ccount[S.clist[i]];
            __syncthreads();
        }
        const uint32_t ncl = S.ncl;
        if (ncl == 0) break;
        // operations of the round, numbered densely: chunk i holds [cpre[i], cpre[i] + ccnt[i])
        uint32_t total = 0;
        {
            uint32_t cnt = t < ncl ? S.ccnt[t] : 0u;
            cnt = cnt < (uint32_t)CH ? cnt : (uint32_t)CH;
            uint32_t pre = block_excl(S, cnt, &total);
            if (t < ncl) S.cpre[t] = pre;
            __syncthreads();
        }
        // operation s: chunk = last with cpre <= s.  Each step loads the
        // next step's operation ahead, so its latency overlaps this step.
        auto load_op = [&](uint32_t s) -> uint2 {
            uint32_t lo = 0, hi = ncl;
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (S.cpre[mid] <= s) lo = mid; else hi = mid;
            }
            return c.B.chunks[(unsigned long long)(uint32_t)S.clist[lo] * CH + (s - S.cpre[lo])];
        };
        uint2 ahead = t < total ? load_op(t) : make_uint2(0, 0);
        for (uint32_t s0 = 0; s0 < total; s0 += NT) {
            stage_room(c, S);
            const uint32_t cur = S.cur;
            const uint32_t s = s0 + t;
            const bool valid0 = s < total;
            const uint2 op0 = ahead;
            if (s + NT < total) ahead = load_op(s + NT);
            bool valid = valid0;
            uint2 op = valid0 ? op0 : make_uint2(0, 0);
            uint32_t vloc = op.x - c.v0;
            if (valid && vloc >= c.nvp) {
                dev_or(&c.B.ctl->err, (uint32_t)ERR_CORRUPT);
                valid = false;
            }
            bool act = false;
            uint32_t rv = 0;
            int32_t idx = -1;
            if (valid) {
                ++c.c_consumed;
                idx = slot_index(c, vloc);
                uint32_t* sp = slot_at(c, idx, vloc);
                if (c.qt == Q_PPR) {
                    float mass = __uint_as_float(op.y);
                    float nr = at_addf(c, sp, mass) + mass;
                    act = ppr_active(nr, thr_of(c, op.x));
                } else {
                    uint32_t val = op.y & ~RETAIN;
                    uint32_t old = at_min(c, sp, val);
                    bool imp = val < old;
                    c.c_improved += imp;
                    act = imp || (op.y & RETAIN);
                    rv = (imp ? val : old) | RETAIN;
                }
            }
            bool win = act && front_set(c, idx, vloc);
            push_frontier(c, S, cur, win, vloc, rv);
        }
        __syncthreads();
        // free this round's chunks into the stash; what does not fit goes back to the ring
        const uint32_t ns0 = S.nstash;
        const uint32_t keep = ncl < (uint32_t)STASH - ns0 ? ncl : (uint32_t)STASH - ns0;
        for (uint32_t i = t; i < keep; i += NT) S.stash[ns0 + i] = (uint32_t)S.clist[i];
        if (ncl > keep) {
            __syncthreads();
            if (t == 0) S.base = dev_add(&c.B.ctl->ring_tail, (unsigned long long)(ncl - keep));
            __syncthreads();
            for (uint32_t i = keep + t; i < ncl; i += NT) c.B.ring[(S.base + i - keep) % c.B.nch] = (uint32_t)S.clist[i];
        }
        __syncthreads();
        if (t == 0) S.nstash = ns0 + keep;
        __syncthreads();
    }
    if (t == 0 && S.nf > (uint32_t)FCAP) S.nf = FCAP;
    __syncthreads();
}

// Refinement item of a certified PPR query (the threshold was lowered after
// the query terminated): re-activate every vertex of the partition whose
// residual reaches the new threshold, exactly as a zero-mass operation to it
// would, so the visit that follows pushes them (Section 4.1's push).
__device__ __forceinline__ void rescan(ItemCtx& c, PassShared& S) {
    const uint32_t t = threadIdx.x;
    for (uint32_t i0 = 0; i0 < c.nvp; i0 += NT) {
        stage_room(c, S);
        const uint32_t cur = S.cur;
        const uint32_t vloc = i0 + t;
        bool act = false;
        int32_t idx = -1;
        if (vloc < c.nvp && ppr_active(__uint_as_float(c.gstate[c.v0 + vloc]), thr_of(c, c.v0 + vloc))) {
            idx = slot_index(c, vloc);
            slot_at(c, idx, vloc);  // stage the residual into the slice
            act = true;
        }
        bool win = act && front_set(c, idx, vloc);
        push_frontier(c, S, cur, win, vloc, 0u);
    }
    __syncthreads();
    if (t == 0 && S.nf > (uint32_t)FCAP) S.nf = FCAP;
    __syncthreads();
}

// Split the frontier: vertices with value < hi (all for PPR) go to the
// batch (up to BCAP), the rest stay in the other frontier buffer.
__device__ __forceinline__ uint32_t extract(ItemCtx& c, PassShared& S, uint32_t hi, bool by_value) {
    const uint32_t t = threadIdx.x;
    const uint32_t cur = S.cur, nf = S.nf;
    __syncthreads();
    if (t == 0) { S.nb = 0; S.nk = 0; }
    __syncthreads();
    for (uint32_t i0 = 0; i0 < nf; i0 += NT) {
        uint32_t i = i0 + t;
        bool valid = i < nf;
        uint32_t v = valid ? S.fq[cur][i] : 0u;
        bool take = valid && (!by_value || sv_get(c, v) < hi);
        uint32_t p = block_append(take, &S.nb);
        bool tk = take && p < (uint32_t)BCAP;
        if (tk) S.bv[p] = v;
        bool keep = valid && !tk;
        uint32_t kp = block_append(keep, &S.nk);
        if (keep) S.fq[cur ^ 1][kp] = v;
    }
    __syncthreads();
    uint32_t nb = S.nb < (uint32_t)BCAP ? S.nb : (uint32_t)BCAP;
    __syncthreads();
    if (t == 0) { S.nf = S.nk; S.cur = cur ^ 1; S.nb = nb; }
    __syncthreads();
    return nb;
}

// Exclusive prefix of the batch degrees (in bpre) -> returns total edges.
__device__ __forceinline__ uint32_t batch_scan(PassShared& S, uint32_t nb) {
    constexpr uint32_t PE = BCAP / NT;
    const uint32_t t = threadIdx.x;
    uint32_t d[PE];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < PE; ++k) {
        uint32_t j = t * PE + k;
        d[k] = j < nb ? S.bpre[j] : 0u;
        s += d[k];
    }
    uint32_t total = 0;
    uint32_t run = block_excl(S, s, &total);
#pragma unroll
    for (uint32_t k = 0; k < PE; ++k) {
        uint32_t j = t * PE + k;
        if (j < nb) S.bpre[j] = run;
        run += d[k];
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ uint32_t find_b(const PassShared& S, uint32_t nb, uint32_t j) {
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (S.bpre[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------ SSSP / BFS
template <int WB>
__device__ __forceinline__ void sp_visit(ItemCtx& c, PassShared& S, uint32_t win, uint32_t yld, uint32_t budget) {
    const uint32_t t = threadIdx.x;
    uint32_t first_lo = INF;
    unsigned long long edges = 0;
    while (true) {
        __syncthreads();
        const uint32_t nf = S.nf;
        if (nf == 0) break;
        uint32_t lo = INF;
        for (uint32_t i = t; i < nf; i += NT) { uint32_t d = sv_get(c, S.fq[S.cur][i]); lo = d < lo ? d : lo; }
        lo = block_min(S, lo);
        if (first_lo == INF) first_lo = c.qlo != INF ? c.qlo : lo;
        if ((yld && (unsigned long long)lo >= (unsigned long long)first_lo + yld) || (budget && edges >= budget)) break;
        uint32_t hi = lo + win;
        if (hi < lo || hi > INF) hi = INF;
        const uint32_t nb = extract(c, S, hi, true);
        for (uint32_t j = t; j < nb; j += NT) {
            uint32_t v = S.bv[j];
            front_clear(c, v);
            uint32_t gv = c.v0 + v;
            uint32_t r0 = c.g.rowptr[gv], r1 = c.g.rowptr[gv + 1];
            uint32_t dv = sv_get(c, v);
            S.bval[j] = dv;
            S.brow[j] = r0;
            S.bpre[j] = r1 - r0;
            if (c.gfinal) {  // trace run: an expansion is useful when its distance is final
                c.it_work += 1.f;
                c.it_useful += (dv == c.gfinal[gv]) ? 1.f : 0.f;
            }
        }
        __syncthreads();
        if (t == 0) c.c_vpush += nb;
        const uint32_t total = batch_scan(S, nb);
        edges += total;
        // edge j's target, tentative distance and, for a target outside the
        // partition, its stored distance (for pruning).  Each step loads the
        // next step's edge ahead, so its latency overlaps this step.
        auto load_edge = [&](uint32_t j, uint32_t& u, uint32_t& nd, uint32_t& du) {
            uint32_t b = find_b(S, nb, j);
            uint32_t e = S.brow[b] + (j - S.bpre[b]);
            u = c.g.col[e];
            unsigned long long sum = (unsigned long long)S.bval[b] + edge_w<WB>(c.g.w, e);
            nd = sum >= INF ? INF - 1 : (uint32_t)sum;
            du = u - c.v0 >= c.nvp ? c.gstate[u] : 0xffffffffu;
        };
        uint32_t u_ahead = 0, nd_ahead = 0, du_ahead = 0xffffffffu;
        if (t < total) load_edge(t, u_ahead, nd_ahead, du_ahead);
        for (uint32_t k0 = 0; k0 < total; k0 += NT) {
            stage_room(c, S);
            const uint32_t cur = S.cur;
            uint32_t j = k0 + t;
            bool valid = j < total;
            uint32_t u = valid ? u_ahead : 0u, nd = valid ? nd_ahead : 0u;
            const uint32_t du = du_ahead;
            if (j + NT < total) load_edge(j + NT, u_ahead, nd_ahead, du_ahead);
            uint32_t ul = u - c.v0;
            bool intra = valid && ul < c.nvp;
            bool win_ = false;
            if (intra) {
                ++c.c_intra;
                const int32_t idx = slot_index(c, ul);
                uint32_t old = at_min(c, slot_at(c, idx, ul), nd);
                if (nd < old) { ++c.c_improved; win_ = front_set(c, idx, ul); }
            }
            push_frontier(c, S, cur, win_, ul, nd | RETAIN);
            // sender-side pruning (the paper's walk-through of Appendix B.3):
            // no operation is sent when the target already has a path at
            // least as short.  The stored distance, read one step early, can
            // only be stale-high (distances only decrease), so pruning never
            // drops useful work.
            bool send = valid && !intra;
            if (send && nd >= du) { send = false; ++c.c_pruned; }
            stage(S, send, u, nd);
        }
        __syncthreads();
        if (t == 0 && S.nf > (uint32_t)FCAP) S.nf = FCAP;
    }
    // retain the unprocessed frontier in the partition's own buffer
    __syncthreads();
    const uint32_t nf = S.nf;
    if (nf) {
        const uint32_t cur = S.cur;
        for (uint32_t i0 = 0; i0 < nf; i0 += NT) {
            stage_room(c, S);
            uint32_t i = i0 + t;
            bool valid = i < nf;
            uint32_t v = valid ? S.fq[cur][i] : 0u;
            stage(S, valid, c.v0 + v, valid ? (sv_get(c, v) | RETAIN) : 0u);
        }
        __syncthreads();
        if (t == 0) { S.nf = 0; dev_add(&c.B.ctl->c_yields, 1ull); }
    }
    if (t == 0) c.c_edges += edges;
}

// ------------------------------------------------------------ PPR
__device__ __forceinline__ void ppr_visit(ItemCtx& c, PassShared& S, uint32_t budget) {
    const uint32_t t = threadIdx.x;
    unsigned long long edges = 0;
    const float a = c.alpha;
    while (true) {
        __syncthreads();
        if (S.nf == 0) break;
        if (budget && edges >= budget) break;
        const uint32_t nb = extract(c, S, ~0u, false);
        uint32_t pushed = 0;
        for (uint32_t j = t; j < nb; j += NT) {
            uint32_t v = S.bv[j];
            front_clear(c, v);
            uint32_t gv = c.v0 + v;
            uint32_t r0 = c.g.rowptr[gv], r1 = c.g.rowptr[gv + 1];
            uint32_t deg = r1 - r0;
            float thr = c.mode ? c.eps * (float)deg : c.eps;
            float mass = sv_takef(c, v);
            uint32_t push_deg = 0;
            float share = 0.f;
            if (!ppr_active(mass, thr)) {
                sv_putf(c, v, mass);
            } else {
                atomicAdd(&c.gp[gv], a * mass);
                ++pushed;
                if (c.gfinal) { c.it_work += 1.f; c.it_useful += 1.f; }  // a push always moves mass to p
                if (deg) { share = (1.f - a) * mass / (float)deg; push_deg = deg; }
            }
            S.bval[j] = __float_as_uint(share);
            S.brow[j] = r0;
            S.bpre[j] = push_deg;
        }
        c.c_vpush += pushed;
        c.c_vpush_ppr += pushed;
        __syncthreads();
        const uint32_t total = batch_scan(S, nb);
        edges += total;
        // edge j's target and pushed share, loaded one step ahead
        auto load_edge = [&](uint32_t j, uint32_t& u, float& share) {
            uint32_t b = find_b(S, nb, j);
            uint32_t e = S.brow[b] + (j - S.bpre[b]);
            u = c.g.col[e];
            share = __uint_as_float(S.bval[b]);
        };
        uint32_t u_ahead = 0;
        float share_ahead = 0.f;
        if (t < total) load_edge(t, u_ahead, share_ahead);
        for (uint32_t k0 = 0; k0 < total; k0 += NT) {
            stage_room(c, S);
            const uint32_t cur = S.cur;
            uint32_t j = k0 + t;
            bool valid = j < total;
            uint32_t u = valid ? u_ahead : 0u;
            float share = valid ? share_ahead : 0.f;
            if (j + NT < total) load_edge(j + NT, u_ahead, share_ahead);
            uint32_t ul = u - c.v0;
            bool intra = valid && ul < c.nvp;
            bool win_ = false;
            if (intra) {
                ++c.c_intra;
                const int32_t idx = slot_index(c, ul);
                float old = at_addf(c, slot_at(c, idx, ul), share);
                float nr = old + share;
                float thr = thr_of(c, u);
                if (ppr_active(nr, thr) && !ppr_active(old, thr)) win_ = front_set(c, idx, ul);
            }
            push_frontier(c, S, cur, win_, ul, 0u);
            stage(S, valid && !intra, u, __float_as_uint(share));
        }
        __syncthreads();
        if (t == 0 && S.nf > (uint32_t)FCAP) S.nf = FCAP;
    }
    __syncthreads();
    const uint32_t nf = S.nf;
    if (nf) {
        const uint32_t cur = S.cur;
        for (uint32_t i0 = 0; i0 < nf; i0 += NT) {
            stage_room(c, S);
            uint32_t i = i0 + t;
            bool valid = i < nf;
            stage(S, valid, valid ? c.v0 + S.fq[cur][i] : 0u, 0u);
        }
        __syncthreads();
        if (t == 0) { S.nf = 0; dev_add(&c.B.ctl->c_yields, 1ull); }
    }
    if (t == 0) { c.c_edges += edges; c.c_edges_ppr += edges; }
}

// ------------------------------------------------------------ kernels
// Pop work items of the current pass (own XCD's list first) and process
// them until every list is exhausted.
template <int WB>
__device__ __forceinline__ void process_items(ItemCtx& c, PassShared& S, const PassCfg& cfg, unsigned long long& items) {
    const uint32_t t = threadIdx.x;
    const GraphDev& g = c.g;
    const QueryDev& Q = c.Q;
    const BufDev& B = c.B;
    const uint32_t xcd = blockIdx.x % NXCD;
    c.pass = B.ctl->pass;
    for (;;) {
        if (t == 0) {
            unsigned long long pos = ~0ull;
            if (!__hip_atomic_load(&B.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                for (uint32_t k = 0; k < NXCD; ++k) {
                    uint32_t x = (xcd + k) % NXCD;
                    uint32_t n = B.ctl->nitems[x];
                    n = n < B.item_cap ? n : B.item_cap;
                    if (__hip_atomic_load(&B.ctl->next[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
                    uint32_t idx = dev_add(&B.ctl->next[x], 1u);
                    if (idx < n) { pos = (unsigned long long)x * B.item_cap + idx; break; }
                }
            }
            S.itpos = pos;
        }
        __syncthreads();
        {
            const unsigned long long pos = S.itpos;
            if (pos == ~0ull) break;
            constexpr uint32_t W16 = sizeof(Item) / 16;
            if (t < W16) ((uint4*)&S.it)[t] = ((const uint4*)&B.items[pos])[t];
        }
        __syncthreads();
        ++items;
        c.P = S.it.part;
        c.q = S.it.q;
        c.v0 = g.pstart[c.P];
        c.nvp = g.pstart[c.P + 1] - c.v0;
        c.qt = Q.qtype[c.q];
        const unsigned long long off = Q.qoff[c.q];
        c.alpha = Q.qalpha[c.q];
        c.eps = Q.qeps[c.q];
        c.mode = Q.qmode[c.q];
        const bool ppr = c.qt == Q_PPR;
        c.gp = (float*)(Q.state + off);
        c.gstate = ppr ? Q.state + off + g.nv : Q.state + off;
        c.gfinal = (cfg.trace && Q.final_state) ? Q.final_state + off : nullptr;
        c.qlo = (cfg.gate && !ppr) ? B.qmin[c.q] : INF;
        c.it_useful = 0.f;
        c.it_work = 0.f;
        // the slice is staged into LDS on first touch
        if (c.hn) {
            for (uint32_t i = t; i < c.hn; i += NT) { c.st[i] = UNLOADED; c.hkeys[i] = EMPTY_KEY; }
        } else {
            for (uint32_t i = t; i < c.nvp; i += NT) c.st[i] = UNLOADED;
        }
        if (!c.hn)
            for (uint32_t i = t; i < (c.nvp + 31) / 32; i += NT) c.bits[i] = 0u;
        if (t == 0) { S.nf = 0; S.ns = 0; S.cur = 0; S.nspill = 0; }
        __syncthreads();
        uint32_t budget = 0;
        if (cfg.mu > 0.f) {
            uint32_t np_items = B.pn[c.P];
            float e_p = (float)(g.rowptr[c.v0 + c.nvp] - g.rowptr[c.v0]);
            float bgt = cfg.mu * e_p / (float)(np_items ? np_items : 1u);
            budget = bgt < 256.f ? 256u : (bgt > 4.0e9f ? 4000000000u : (uint32_t)bgt);
        }
        if (S.it.rest != RESCAN) consume(c, S);
        else if (ppr) rescan(c, S);
        if (ppr) ppr_visit(c, S, budget);
        else if (c.qt == Q_BFS) sp_visit<0>(c, S, cfg.win_lv, cfg.yld_lv, budget);
        else sp_visit<WB>(c, S, cfg.win_sp, cfg.yld_sp, budget);
        flush(c, S);
        if (t == 0 && S.nspill) {
            dev_max(&B.ctl->c_spill_max, S.nspill);
            if (S.nspill > SPILL_MAX) dev_or(&B.ctl->err, (uint32_t)ERR_SPILL);
        }
        // write the touched part of the slice back
        if (c.hn) {
            for (uint32_t i = t; i < c.hn; i += NT) {
                uint32_t k = c.hkeys[i], x = c.st[i];
                if (k != EMPTY_KEY && x != UNLOADED) c.gstate[c.v0 + (k & ~FRONT)] = x;
            }
        } else {
            for (uint32_t i = t; i < c.nvp; i += NT) {
                uint32_t x = c.st[i];
                if (x != UNLOADED) c.gstate[c.v0 + i] = x;
            }
        }
        if (c.gfinal) {
            float u = c.it_useful, w = c.it_work;
#pragma unroll
            for (int o = 32; o; o >>= 1) { u += __shfl_xor(u, o); w += __shfl_xor(w, o); }
            if ((t & 63) == 0 && w > 0.f) {
                atomicAdd(&B.tr_useful[c.P], u);
                atomicAdd(&B.tr_work[c.P], w);
            }
        }
        __syncthreads();
    }
}

// Give the workgroup's stash back to the pool's ring (block-collective).
__device__ __forceinline__ void return_stash(const BufDev& B, PassShared& S) {
    const uint32_t t = threadIdx.x;
    __syncthreads();
    const uint32_t n = S.nstash;
    if (n == 0) return;
    if (t == 0) S.base = dev_add(&B.ctl->ring_tail, (unsigned long long)n);
    __syncthreads();
    for (uint32_t i = t; i < n; i += NT) B.ring[(S.base + i) % B.nch] = S.stash[i];
    __syncthreads();
    if (t == 0) S.nstash = 0;
    __syncthreads();
}

// Dynamic LDS: dense slice st[vpmax] | frontier bits, or hashed slice st[slots] | keys[slots]
// (the frontier flags live in the keys).
__device__ __forceinline__ void init_ctx(ItemCtx& c, const GraphDev& g, const QueryDev& Q, const BufDev& B,
                                         uint32_t* dyn, uint32_t slice_words, uint32_t hash_slots) {
    c.g = g;
    c.Q = Q;
    c.B = B;
    c.st = dyn;
    c.hn = hash_slots;
    c.hkeys = dyn + hash_slots;
    c.bits = hash_slots ? nullptr : dyn + slice_words;
    c.c_edges = c.c_intra = c.c_improved = c.c_emitted = c.c_consumed = c.c_vpush = c.c_chunks = c.c_pruned = 0;
    c.c_edges_ppr = c.c_vpush_ppr = c.c_spill = 0;
}

__device__ __forceinline__ void publish_counters(const ItemCtx& c, unsigned long long items) {
    const uint32_t t = threadIdx.x;
    const BufDev& B = c.B;
    constexpr int NC = 11;
    unsigned long long v[NC] = {c.c_edges, c.c_intra, c.c_improved, c.c_emitted, c.c_consumed, c.c_vpush, c.c_chunks,
                                c.c_pruned, c.c_edges_ppr, c.c_vpush_ppr, c.c_spill};
    unsigned long long* dst[NC] = {&B.ctl->c_edges, &B.ctl->c_intra, &B.ctl->c_improved, &B.ctl->c_emitted,
                                   &B.ctl->c_consumed, &B.ctl->c_vpush, &B.ctl->c_chunks, &B.ctl->c_pruned,
                                   &B.ctl->c_edges_ppr, &B.ctl->c_vpush_ppr, &B.ctl->c_spill};
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        unsigned long long x = v[k];
#pragma unroll
        for (int o = 32; o; o >>= 1) x += __shfl_xor(x, o);
        if ((t & 63) == 0 && x) dev_add(dst[k], x);
    }
    if (t == 0 && items) dev_add(&B.ctl->c_items, items);
}

// One pass (Algorithm 2's IntraPartProcess over the selected partitions).
// Three workgroups per CU is what the LDS of a typical slice allows; keep the
// register budget within it (168 VGPRs) so registers never lower occupancy.
template <int WB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_process(GraphDev g, QueryDev Q, BufDev B, PassCfg cfg, uint32_t slice_words,
                                                uint32_t hash_slots) {
    __shared__ PassShared S;
    extern __shared__ uint32_t dyn[];
    ItemCtx c;
    init_ctx(c, g, Q, B, dyn, slice_words, hash_slots);
    unsigned long long items = 0;
    if (threadIdx.x == 0) S.nstash = 0;
    __syncthreads();
    process_items<WB>(c, S, cfg, items);
    return_stash(B, S);
    publish_counters(c, items);
}

// Persistent form: one cooperative launch runs up to max_passes passes of
// Algorithm 2 -- buffer summaries (all blocks), [learned scoring], selection
// (block 0), detachment into the
// per-XCD work queues (all blocks), processing (all blocks) -- separated by
// grid-wide barriers, and stops by itself when no buffer holds work.
template <int WB>
__global__ __launch_bounds__(NT) void k_persistent(GraphDev g, QueryDev Q, BufDev B, PassCfg cfg, uint32_t slice_words,
                                                   uint32_t hash_slots, uint32_t max_passes, const float* theta,
                                                   float* score, GStat* gs) {
    __shared__ PassShared S;
    extern __shared__ uint32_t dyn[];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    ItemCtx c;
    init_ctx(c, g, Q, B, dyn, slice_words, hash_slots);
    unsigned long long items = 0;
    const uint32_t t = threadIdx.x;
    if (t == 0) S.nstash = 0;
    __syncthreads();
    const uint32_t dyn_words = hash_slots ? 2 * hash_slots : slice_words + (slice_words + 31) / 32;
    for (uint32_t pass = 0; pass < max_passes; ++pass) {
        // partition summaries from the buffers: per-query windows, then per partition
        for (uint32_t q = blockIdx.x * NT + t; q < Q.nq; q += gridDim.x * NT) qmin_one(B, Q, g.np, q);
        grid.sync();
        for (uint32_t P = blockIdx.x; P < g.np; P += gridDim.x) psum_one(B, Q, cfg, P);
        grid.sync();
        if (cfg.sched == S_LEARNED) {
            if (blockIdx.x == 0) gstat_body(g, B, gs);
            grid.sync();
            // stage the weights in LDS when they fit, score partitions grid-wide
            const bool lds_w = dyn_words >= (uint32_t)MLP_NPARAM;
            if (lds_w)
                for (uint32_t i = t; i < (uint32_t)MLP_NPARAM; i += NT) ((float*)dyn)[i] = theta[i];
            __syncthreads();
            const float* w = lds_w ? (const float*)dyn : theta;
            const GStat s = *gs;
            const uint32_t pnext = B.ctl->pass + 1;
            for (uint32_t P = blockIdx.x * NT + t; P < g.np; P += gridDim.x * NT) {
                float x[MLP_IN];
                partition_features(g, B, s, pnext, P, x);
                float y = mlp_forward(w, x);
                score[P] = B.pcount[P] ? y : -3.0e38f;
            }
            grid.sync();
        }
        if (blockIdx.x == 0) {
            const uint32_t cap = (dyn_words * 4u) / 12u;
            select_body<NT>(g, B, cfg, (unsigned long long*)dyn, (unsigned int*)((unsigned long long*)dyn + cap), cap);
        }
        grid.sync();
        // Every block takes the same exit decision: `stop` is written only by
        // the select step above, while the other blocks wait at the barrier,
        // and nothing writes it again before the next select.  (ctl->err can
        // be raised by a fast block's detach below while a slow block is
        // still reading it, so it must not decide the exit.)
        if (__hip_atomic_load(&B.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        const uint32_t nsel = B.ctl->nsel;
        const uint32_t nqp = (Q.nq + WAVE - 1) / WAVE * WAVE;
        const unsigned long long total = (unsigned long long)nsel * nqp;
        for (unsigned long long i = (unsigned long long)blockIdx.x * NT + t; i < total; i += (unsigned long long)gridDim.x * NT)
            worklist_one(B, Q, cfg, (uint32_t)(i / nqp), (uint32_t)(i % nqp));
        grid.sync();
        process_items<WB>(c, S, cfg, items);
        grid.sync();
    }
    return_stash(B, S);
    publish_counters(c, items);
}

size_t process_dyn_lds(uint32_t vpmax, uint32_t hash_slots) {
    return (hash_slots ? 2 * (size_t)hash_slots : (size_t)vpmax + (vpmax + 31) / 32) * 4;
}

hipError_t launch_process(const GraphDev& g, const QueryDev& Q, const BufDev& B, const PassCfg& cfg,
                          uint32_t blocks, uint32_t vpmax, uint32_t hs, hipStream_t s) {
    size_t dyn = process_dyn_lds(vpmax, hs);
    switch (g.wbytes) {
    case 0: hipLaunchKernelGGL((k_process<0>), dim3(blocks), dim3(NT), dyn, s, g, Q, B, cfg, vpmax, hs); break;
    case 1: hipLaunchKernelGGL((k_process<1>), dim3(blocks), dim3(NT), dyn, s, g, Q, B, cfg, vpmax, hs); break;
    case 2: hipLaunchKernelGGL((k_process<2>), dim3(blocks), dim3(NT), dyn, s, g, Q, B, cfg, vpmax, hs); break;
    default: hipLaunchKernelGGL((k_process<4>), dim3(blocks), dim3(NT), dyn, s, g, Q, B, cfg, vpmax, hs); break;
    }
    return hipGetLastError();
}

const void* process_kernel_ptr(int wbytes) {
    switch (wbytes) {
    case 0: return (const void*)k_process<0>;
    case 1: return (const void*)k_process<1>;
    case 2: return (const void*)k_process<2>;
    default: return (const void*)k_process<4>;
    }
}
const void* persistent_kernel_ptr(int wbytes) {
    switch (wbytes) {
    case 0: return (const void*)k_persistent<0>;
    case 1: return (const void*)k_persistent<1>;
    case 2: return (const void*)k_persistent<2>;
    default: return (const void*)k_persistent<4>;
    }
}

template <int WB>
static hipError_t launch_persistent_wb(const GraphDev& g, const QueryDev& Q, const BufDev& B, const PassCfg& cfg,
                                       uint32_t blocks, uint32_t sw, uint32_t hs, uint32_t max_passes,
                                       const float* theta, float* score, GStat* gs, size_t dyn, hipStream_t s) {
    void* args[] = {(void*)&g, (void*)&Q, (void*)&B, (void*)&cfg, (void*)&sw, (void*)&hs, (void*)&max_passes,
                    (void*)&theta, (void*)&score, (void*)&gs};
    return hipLaunchCooperativeKernel(k_persistent<WB>, dim3(blocks), dim3(NT), args, dyn, s);
}

hipError_t launch_persistent(const GraphDev& g, const QueryDev& Q, const BufDev& B, const PassCfg& cfg,
                             uint32_t blocks, uint32_t vpmax, uint32_t hs, uint32_t max_passes, const float* theta,
                             float* score, void* gstat, hipStream_t s) {
    const size_t dyn = process_dyn_lds(vpmax, hs);
    GStat* gs = (GStat*)gstat;
    switch (g.wbytes) {
    case 0: return launch_persistent_wb<0>(g, Q, B, cfg, blocks, vpmax, hs, max_passes, theta, score, gs, dyn, s);
    case 1: return launch_persistent_wb<1>(g, Q, B, cfg, blocks, vpmax, hs, max_passes, theta, score, gs, dyn, s);
    case 2: return launch_persistent_wb<2>(g, Q, B, cfg, blocks, vpmax, hs, max_passes, theta, score, gs, dyn, s);
    default: return launch_persistent_wb<4>(g, Q, B, cfg, blocks, vpmax, hs, max_passes, theta, score, gs, dyn, s);
    }
}
int process_threads() { return NT; }
size_t process_static_lds() { return sizeof(PassShared); }

}  // namespace fk
