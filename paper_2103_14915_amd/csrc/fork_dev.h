// Device-side data structures shared by the kernels and the host runtime of
// the fork-processing library (gfx950).  Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

constexpr int WAVE = 64;
constexpr int CH = 256;                   // operations per pool chunk
constexpr uint32_t INF = 0x7fffffffu;     // unreachable distance / level
constexpr uint32_t RETAIN = 0x80000000u;  // op flag: retained (yielded) work
constexpr int NXCD = 8;                   // MI355X: 8 XCDs of 32 CUs
constexpr uint32_t VPMAX = 16384;         // default vertices per partition (the dense LDS slice fits)
constexpr uint32_t PVMAX = 65536;         // max vertices per partition (hashed LDS slice)
constexpr uint32_t HS_AUTO = 4096;        // hash slots when the dense slice does not fit
// Largest partition (vertices) for L1-certified PPR queries: at most the
// visit's frontier capacity, so a refinement's re-activations always fit the
// frontier and are never spilled back into the buffers.  (The host build of
// the kernels used by the tests raises it to drive refinements that spill.)
#ifndef FORK_CERT_MAX_PART
#define FORK_CERT_MAX_PART 1024u
#endif
constexpr uint32_t CERT_MAX_PART = FORK_CERT_MAX_PART;
constexpr int MLP_IN = 16, MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 5313

enum QType : uint32_t { Q_SSSP = 1, Q_BFS = 2, Q_PPR = 3 };
enum Sched : uint32_t { S_FIFO = 0, S_PRIORITY = 1, S_LEARNED = 2, S_RANDOM = 3, S_MAXOPS = 4 };

// error flags in Ctl::err
constexpr unsigned long long BTW_EMPTY = 0xffffffff00000000ull | (unsigned long long)CH;
enum : uint32_t { ERR_CAPACITY = 1u, ERR_ITEMS = 2u, ERR_CORRUPT = 4u, ERR_SPILL = 8u };
// Most activated vertices one visit of the buffered engine may retain as
// operations in its own buffer when its frontier is full.  Beyond it the run
// stops with FORK_E_CAPACITY: that regime (a visit re-activating most of a
// large partition, its overflow re-emitted pass after pass) is the one in
// which a GPU run once failed its consistency check for a reason not found,
// so it is refused rather than run.  (Vertices kept outside a hashed slice
// re-enter the frontier once per operation, so a visit of a 4,096-vertex
// partition with a 256-slot table can retain about 18,000; the refinement
// that failed retained about 60,000.)
constexpr uint32_t SPILL_MAX = 32768;

// One device control block per context.  Counters are 64-bit.
struct Ctl {
    unsigned long long ring_head;   // next free-ring slot to pop
    unsigned long long ring_tail;   // next free-ring slot to push
    unsigned long long avail_end;   // pops in this pass must stay below this
    unsigned int err;
    unsigned int pass;              // pass counter (advanced by the select kernel)
    unsigned int nsel;              // partitions selected for this pass
    unsigned int pending_parts;     // partitions holding operations at select time
    unsigned int nitems[NXCD];      // per-XCD work list lengths
    unsigned int next[NXCD];        // per-XCD work list cursors
    unsigned long long c_edges, c_improved, c_emitted, c_consumed, c_vpush, c_yields, c_chunks,
        c_items, c_passes_nonempty, c_intra, c_pruned;
    unsigned long long pending_ops; // operations buffered at select time
    unsigned int stop;              // set by the select step only: no work left, or a device error
                                    // (the persistent kernel's exit test, the same for every block)
    unsigned long long c_sel_edges; // out-edges of the partitions selected, summed over passes
    unsigned long long c_edges_ppr, c_vpush_ppr;  // the PPR share of c_edges / c_vpush
    unsigned long long c_spill;     // activated vertices retained as operations (frontier full)
    unsigned long long c_act;       // grouped engine: (vertex, group) activations in other partitions
    unsigned int c_spill_max;       // most vertices one visit retained because its frontier was full
    unsigned long long c_vtask;     // grouped engine: vertex expansions (each for one or more lanes)
    unsigned long long c_rounds;    // grouped engine: rounds of the visits
    unsigned long long c_tasks;     // grouped engine: 64-edge tasks of the rounds
    unsigned long long c_tphase[5]; // grouped engine: workgroup time (10 ns ticks) in the visit phases:
                                    // bitmap gather, round take, filter, edge tasks, yield
};

// A (partition, query) work item of one pass.
// A detached (partition, query) buffer.  The detach walks the head of the
// chunk list (in parallel over buffers) so that the visit starts without a
// serial chain of dependent loads; longer lists continue at `rest`.
constexpr int ICH = 14;
struct alignas(16) Item {
    uint32_t part;
    uint32_t q;
    int32_t rest;    // next chunk after the inline ones (-1: none)
    uint32_t nch;    // inline chunks
    uint2 ch[ICH];   // (chunk id, valid ops)
};
static_assert(sizeof(Item) == 128, "work item layout");
// Item::rest of a refinement item (certified PPR): no buffered operations;
// the visit starts from every vertex of the partition whose residual
// reaches the query's current threshold.
constexpr int32_t RESCAN = -2;

struct GraphDev {
    uint32_t nv, np, pshift, wbytes;
    const uint32_t* rowptr;   // [nv+1]
    const uint32_t* col;      // [ne]
    const void* w;            // [ne] of wbytes (NULL if unweighted)
    const uint32_t* pstart;   // [np+1]
    const uint16_t* vpart;    // [(nv >> pshift) + 1] partition of each vertex block
};

struct QueryDev {
    uint32_t nq, qc;          // queries in this wave, bucket stride (capacity)
    const uint32_t* qtype;    // [qc]
    const unsigned long long* qoff;  // [qc] word offset of the query's state
    const float* qalpha;      // [qc]
    const float* qeps;        // [qc]
    const uint32_t* qmode;    // [qc]
    uint32_t* state;          // state words; SSSP/BFS: int32[V]; PPR: p f32[V] then r f32[V]
    const uint32_t* final_state;  // trace runs: final state of the same wave (same layout), else NULL
};

struct BufDev {
    // A (partition, query) buffer is a list of chunks bhead -> ... -> tail whose
    // tail still takes appends, plus an overflow list of chunks added while
    // the tail was being replaced.  btw packs (tail chunk << 32 | slots
    // reserved in it); one 64-bit atomic add reserves slots.  An empty buffer
    // has BTW_EMPTY, i.e. no tail and a full reservation count.
    int32_t* bhead;           // [np*qc] first chunk of the main list (-1: empty)
    unsigned long long* btw;  // [np*qc] tail word
    int32_t* bover;           // [np*qc] overflow list (-1: none)
    uint32_t* bval;           // [np*qc] best buffered value: SSSP/BFS min value, PPR ~(max mass bits);
                              //         0xffffffff when empty (min works for both encodings)
    uint32_t* bcnt;           // [np*qc] buffered operations, counted in whole chunks (0 = empty)
    uint32_t* bfirst;         // [np*qc] pass in which the buffer became non-empty
    uint32_t* qmin;           // [qc] SSSP/BFS: best buffered value of the query over all partitions
    uint32_t* pready;         // [np] buffers ready to run (within the query's window)
    uint2* chunks;            // [nch*CH] (vertex, value) operations
    int32_t* cnext;           // [nch]
    uint32_t* ccount;         // [nch] valid ops in the chunk (set when it stops being a tail)
    uint32_t* ring;           // [nch] free chunk ids
    unsigned long long nch;
    // partition summaries (maintained at emission, reset when a partition is scheduled)
    uint32_t* pcount;         // [np] buffered ops
    uint32_t* pbest_sp;       // [np] min buffered SSSP distance
    uint32_t* pbest_lv;       // [np] min buffered BFS level
    uint32_t* pbest_pr;       // [np] max buffered PPR residual mass (float bits)
    uint32_t* pfirst;         // [np] pass of the oldest buffered op
    uint32_t* plast;          // [np] pass of the last visit
    uint32_t* pvisits;        // [np] visits
    uint32_t* pn;             // [np] items of the partition in the current pass
    uint32_t* pqn;            // [np] (partition, query) buffers holding operations
    uint32_t* pqmin;          // [np] SSSP/BFS buffers holding their query's best buffered value (dist_min)
    uint32_t* sel;            // [max parts per pass] selected partitions
    float* score;             // [np] learned score (LEARNED policy)
    float* tr_useful;         // trace runs: [np] useful work of the pass's visits
    float* tr_work;           // trace runs: [np] vertex expansions / pushes of the visits
    Item* items;              // [NXCD * item_cap]
    uint32_t item_cap;
    Ctl* ctl;
};

// Queries of the grouped engine: groups of up to 64 queries of one type,
// lane l of group g being one query; state rows are vertex-major per group.
struct GroupDev {
    uint32_t ng;                      // groups in the wave
    const uint32_t* gtype;            // [ng] query type
    const unsigned long long* goff;   // [ng] word offset of the group's state
    const float* lalpha;              // [ng*64] per lane (PPR)
    const float* leps;                // [ng*64]
    const uint32_t* lmode;            // [ng*64]
    uint32_t* state;                  // SSSP/BFS: dist[V][64]; PPR: r[V][64] then p[V][64]
    unsigned long long* pend;         // [ng][V] pending lanes
    uint32_t* bits;                   // [ng][bw] vertices with pending lanes (may hold stale ones)
    uint32_t bw;                      // bitmap words per group
    uint32_t* icnt;                   // [np*ng] activations since the pair was last detached
    uint32_t* ibest;                  // [np*ng] best pending value (SSSP/BFS min; PPR ~residual bits)
    uint32_t* ifirst;                 // [np*ng] pass of the first activation since the detach
    uint32_t* gmin;                   // [ng] SSSP/BFS: the group's best pending value (heuristic 2)
};

struct PassCfg {
    uint32_t sched;
    uint32_t kmax;            // max partitions per pass
    uint32_t target_items;    // pick partitions until this many work items (0: exactly kmax)
    uint32_t win_sp, win_lv;  // batch window (SSSP, BFS)
    uint32_t yld_sp, yld_lv;  // yield range H2 (0 = off)
    float mu;                 // yield budget H1: mu * |E_P| / items_P (0 = off)
    uint32_t seed;
    uint32_t mixed;           // more than one query type in the wave
    uint32_t trace;           // record per-partition usefulness of each visit
    uint32_t gate;            // process a query's buffer only within its global window (heuristic 2)
};

// Is the buffered work of bucket b (query type qt) within its query's window?
__host__ __device__ inline bool bucket_ready(uint32_t bv, uint32_t qt, uint32_t qmin, const PassCfg& cfg) {
    if (!cfg.gate || qt == Q_PPR) return true;
    const unsigned long long d = qt == Q_BFS ? cfg.yld_lv : cfg.yld_sp;
    return d == 0 || (unsigned long long)bv <= (unsigned long long)qmin + d;
}

__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace fk
