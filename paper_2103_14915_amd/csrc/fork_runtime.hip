// Host runtime of the fork-processing library: graph ingest and partition
// plan, query waves, the pass loop of Algorithm 2, results and digests.
// Everything behind the C ABI of include/fork.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "fork.h"
#include "fork_dev.h"

namespace fk {
hipError_t launch_select(const GraphDev&, const BufDev&, const PassCfg&, hipStream_t);
hipError_t launch_worklist(const BufDev&, const QueryDev&, const PassCfg&, hipStream_t);
hipError_t launch_summaries(const GraphDev&, const BufDev&, const QueryDev&, const PassCfg&, hipStream_t);
hipError_t launch_process(const GraphDev&, const QueryDev&, const BufDev&, const PassCfg&, uint32_t, uint32_t, uint32_t,
                          hipStream_t);
size_t process_dyn_lds(uint32_t vpmax, uint32_t hash_slots);
int process_threads();
hipError_t launch_ring_init(uint32_t*, unsigned long long, hipStream_t);
hipError_t launch_fill64(unsigned long long*, unsigned long long, unsigned long long, hipStream_t);
hipError_t launch_seed(const GraphDev&, const QueryDev&, const BufDev&, const uint32_t*, hipStream_t);
hipError_t launch_digest(const QueryDev&, uint32_t, unsigned long long*, const uint32_t*, hipStream_t);
hipError_t launch_gather(const uint32_t*, const uint32_t*, uint32_t*, uint32_t, hipStream_t);
hipError_t launch_indeg(const uint32_t*, unsigned long long, uint32_t*, hipStream_t);
hipError_t launch_rfill(const uint32_t*, const uint32_t*, uint32_t, const uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                        hipStream_t);
hipError_t launch_sdeg(const uint32_t*, const uint32_t*, uint32_t, uint32_t*, hipStream_t);
hipError_t launch_sweep(const uint32_t*, const unsigned long long*, uint32_t, uint32_t, const uint32_t*, const uint32_t*,
                        const uint32_t*, const uint32_t*, const uint32_t*, unsigned long long, uint32_t, void*,
                        hipStream_t);
size_t sweep_out_bytes();
hipError_t launch_bc(const uint32_t*, const unsigned long long*, const uint32_t*, const uint32_t*, uint32_t, uint32_t,
                     const uint32_t*, const uint32_t*, const void*, uint32_t, const uint32_t*, const uint32_t*,
                     const uint32_t*, uint32_t*, uint32_t*, double*, double*, double*, uint32_t*, hipStream_t);
uint32_t bc_level_cap();
hipError_t launch_rnorm(const QueryDev&, uint32_t, const uint32_t*, uint32_t, double*, hipStream_t);
hipError_t launch_rescan_items(const BufDev&, uint32_t, const uint32_t*, unsigned long long, uint32_t, hipStream_t);
hipError_t launch_mlp_score(const GraphDev&, const BufDev&, const float*, float*, float*, void*, uint32_t, hipStream_t);
size_t gstat_bytes();
hipError_t launch_mlp_grad(const float*, const float*, const float*, const uint32_t*, uint32_t, float*, float*,
                           hipStream_t);
hipError_t launch_adam(float*, const float*, float*, float*, uint32_t, float, hipStream_t);
hipError_t launch_mlp_forward(const float*, const float*, uint32_t, float*, hipStream_t);
const void* process_kernel_ptr(int wbytes);
const void* persistent_kernel_ptr(int wbytes);
hipError_t launch_persistent(const GraphDev&, const QueryDev&, const BufDev&, const PassCfg&, uint32_t, uint32_t,
                             uint32_t, uint32_t, const float*, float*, void*, hipStream_t);
hipError_t launch_gprocess(const GraphDev&, const GroupDev&, const BufDev&, const PassCfg&, uint32_t, uint32_t,
                           hipStream_t);
const void* gprocess_kernel_ptr(int wbytes);
int gprocess_threads();
hipError_t launch_gsummaries(const GraphDev&, const GroupDev&, const BufDev&, const PassCfg&, hipStream_t);
hipError_t launch_gworklist(const BufDev&, const GroupDev&, const PassCfg&, hipStream_t);
hipError_t launch_gseed(const GraphDev&, const GroupDev&, const uint32_t*, hipStream_t);
hipError_t launch_gout(const GroupDev&, uint32_t, uint32_t*, const unsigned long long*, const uint32_t*, hipStream_t);
hipError_t launch_gdigest(const GroupDev&, uint32_t, const uint32_t*, unsigned long long*, const uint32_t*, hipStream_t);
uint32_t train_nmax();
hipError_t train_prepare();
hipError_t train_scratch_address(void**);
hipError_t launch_train_noalloc(uint32_t*, float*, const float*, const float*, uint32_t, uint32_t, uint32_t, float,
                                unsigned long long, float*, hipStream_t);
}  // namespace fk

// Message of the last failing call on this thread (a fixed buffer: reporting
// an error allocates nothing).
static thread_local char g_err[512];

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(FORK_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                \
    } while (0)

struct QueryRec {
    uint32_t type, src, mode;
    float alpha, eps;
    float l1 = 0.f;  // PPR: certified L1 target (0 = off)
};

struct fork_ctx {
    int device = 0;
    uint32_t nv = 0;
    uint64_t ne = 0;
    int wbytes = 0;
    uint32_t np = 0, pshift = 0;
    std::vector<uint32_t> h_pstart;
    std::vector<uint32_t> h_rowptr;  // host copy (partition planning, statistics)
    // caller's vertex order (empty: identity): internal position of each vertex
    std::vector<uint32_t> h_pos;
    uint32_t* d_pos = nullptr;     // [nv] internal position of caller vertex v
    uint32_t* d_orig = nullptr;    // [nv] caller id of internal vertex u
    uint32_t* d_gather = nullptr;  // [nv] staging for fetches to host memory
    // reverse adjacency and undirected degrees (sweep cuts; built on first use)
    uint32_t *d_rrow = nullptr, *d_rcol = nullptr, *d_sdeg = nullptr, *d_reid = nullptr;
    // graph
    uint32_t* d_rowptr = nullptr;
    uint32_t* d_col = nullptr;
    void* d_w = nullptr;
    uint32_t* d_pstart = nullptr;
    uint16_t* d_vpart = nullptr;
    // operation pool
    unsigned long long nch = 0;
    uint2* d_chunks = nullptr;
    int32_t* d_cnext = nullptr;
    uint32_t* d_ccount = nullptr;
    uint32_t* d_ring = nullptr;
    // partition summaries
    uint32_t *d_pcount = nullptr, *d_pbest_sp = nullptr, *d_pbest_lv = nullptr, *d_pbest_pr = nullptr,
             *d_pfirst = nullptr, *d_plast = nullptr, *d_pvisits = nullptr, *d_pn = nullptr,
             *d_sel = nullptr, *d_pqn = nullptr, *d_pready = nullptr, *d_pqmin = nullptr;
    float* d_score = nullptr;
    float* d_mlp = nullptr;
    float* d_feat = nullptr;       // [np*16] features (trace runs)
    float* d_tr = nullptr;         // [2*np] useful / work per partition (trace runs)
    uint32_t* d_final = nullptr;   // final state of the traced wave
    size_t final_words = 0;
    std::vector<float> trace;      // records of FORK_TRACE_WIDTH floats
    unsigned char* d_gstat = nullptr;
    fk::Ctl* d_ctl = nullptr;
    fk::Ctl* h_ctl = nullptr;  // pinned
    // queries
    std::vector<QueryRec> queries;
    uint32_t max_queries = 0;
    // wave buffers (sized for the largest wave)
    uint32_t qcap = 0;           // bucket stride
    size_t state_words_cap = 0;
    uint32_t* d_state = nullptr;
    int32_t* d_bhead = nullptr;
    unsigned long long* d_btw = nullptr;
    int32_t* d_bover = nullptr;
    uint32_t *d_bval = nullptr, *d_bcnt = nullptr, *d_bfirst = nullptr, *d_qmin = nullptr;
    fk::Item* d_items = nullptr;
    uint32_t item_cap = 0, kmax_cap = 0;
    uint32_t *d_qtype = nullptr, *d_qsrc = nullptr, *d_qmode = nullptr;
    unsigned long long* d_qoff = nullptr;
    float *d_qalpha = nullptr, *d_qeps = nullptr;
    unsigned long long* d_digest = nullptr;
    uint32_t* d_certq = nullptr;   // [qcap] certified PPR queries still above their target
    double* d_rnorm = nullptr;     // [qcap] their residual mass
    // results
    std::vector<fork_digest> digests;
    bool ran = false;
    uint32_t res_first = 0, res_n = 0;
    fk::QueryDev resQ{};        // queries of the resident (last) wave
    bool res_grouped = false;   // its results are still in the grouped engine's rows (no vectors)
    fk::GroupDev resG{};        // those rows
    bool dig_pending = false;   // their digests are computed on first request
    std::vector<unsigned long long> res_off;
    fork_stats_t stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> pev;  // pass-kernel timing events (profile mode)
    int blocks_per_cu = 1, num_cu = 1, pers_blocks_per_cu = 0, group_blocks_per_cu = 0;
    // grouped engine (grow-only buffers)
    uint32_t* d_gstate = nullptr;
    size_t gstate_cap = 0;
    unsigned long long* d_gpend = nullptr;
    uint32_t* d_gbits = nullptr;
    size_t gpend_cap = 0, gbits_cap = 0;
    uint32_t *d_icnt = nullptr, *d_ibest = nullptr, *d_ifirst = nullptr, *d_gmin = nullptr;
    size_t pair_cap = 0, grp_cap = 0;
    uint32_t *d_gtype = nullptr, *d_lmode = nullptr, *d_lq = nullptr, *d_lsrc = nullptr;
    unsigned long long* d_goff = nullptr;
    float *d_lalpha = nullptr, *d_leps = nullptr;
    uint32_t hslots = 0;  // hashed LDS slice slots of the current run (0 = dense slice)
    bool dense_ok = true; // the dense slice of the largest partition fits in LDS
    bool spill_refused = false;  // the last run stopped at the frontier-spill bound
    // device memory budget of the batch's wave plan, fixed by its first fork_prepare or
    // fork_run (0: none yet), so that later runs of the batch make the same waves and
    // find their buffers allocated; reset by fork_submit
    size_t plan_budget = 0;
    uint32_t vpmax = 1;  // largest partition (vertices)
    double wmean = 1.0;  // mean edge weight
};

extern "C" const char* fork_last_error(void) { return g_err; }

template <class T> static int dalloc(T** p, size_t n) {
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(FORK_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", n * sizeof(T), hipGetErrorString(e));
    }
    return FORK_OK;
}
#define ALLOC(p, n)                       \
    do {                                  \
        int rc_ = dalloc(&(p), (n));      \
        if (rc_) return rc_;              \
    } while (0)

static void free_wave(fork_ctx* c) {
    hipFree(c->d_state); c->d_state = nullptr;
    hipFree(c->d_bhead); c->d_bhead = nullptr;
    hipFree(c->d_btw); c->d_btw = nullptr;
    hipFree(c->d_bover); c->d_bover = nullptr;
    hipFree(c->d_bval); c->d_bval = nullptr;
    hipFree(c->d_bcnt); c->d_bcnt = nullptr;
    hipFree(c->d_bfirst); c->d_bfirst = nullptr;
    hipFree(c->d_qmin); c->d_qmin = nullptr;
    hipFree(c->d_items); c->d_items = nullptr;
    hipFree(c->d_qtype); c->d_qtype = nullptr;
    hipFree(c->d_qsrc); c->d_qsrc = nullptr;
    hipFree(c->d_qmode); c->d_qmode = nullptr;
    hipFree(c->d_qoff); c->d_qoff = nullptr;
    hipFree(c->d_qalpha); c->d_qalpha = nullptr;
    hipFree(c->d_qeps); c->d_qeps = nullptr;
    hipFree(c->d_digest); c->d_digest = nullptr;
    hipFree(c->d_certq); c->d_certq = nullptr;
    hipFree(c->d_rnorm); c->d_rnorm = nullptr;
    c->qcap = 0;
    c->state_words_cap = 0;
    c->kmax_cap = 0;
}

extern "C" void fork_destroy(fork_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    free_wave(c);
    void* ptrs[] = {c->d_rowptr, c->d_col, c->d_w, c->d_pstart, c->d_vpart, c->d_chunks, c->d_cnext,
                    c->d_ccount, c->d_ring, c->d_pcount, c->d_pbest_sp, c->d_pbest_lv, c->d_pbest_pr,
                    c->d_pfirst, c->d_plast, c->d_pvisits, c->d_pn, c->d_sel, c->d_pqn, c->d_pready, c->d_pqmin,
                    c->d_score, c->d_mlp,
                    c->d_ctl, c->d_gstat, c->d_feat, c->d_tr, c->d_final, c->d_pos, c->d_orig, c->d_gather, c->d_rrow, c->d_rcol, c->d_sdeg, c->d_reid};
    for (void* p : ptrs) if (p) hipFree(p);
    void* gptrs[] = {c->d_gstate, c->d_gpend, c->d_gbits, c->d_icnt, c->d_ibest, c->d_ifirst, c->d_gmin, c->d_gtype,
                     c->d_lmode, c->d_lq, c->d_lsrc, c->d_goff, c->d_lalpha, c->d_leps};
    for (void* p : gptrs) if (p) hipFree(p);
    if (c->h_ctl) hipHostFree(c->h_ctl);
    for (auto& e : c->ev) if (e) hipEventDestroy(e);
    for (auto& e : c->pev) if (e) hipEventDestroy(e);
    delete c;
}

// Partition plan (Definition 2.1): contiguous vertex ranges, boundaries on
// multiples of 2^pshift vertices, at most pv vertices and (unless a single
// block exceeds it) at most pe out-edges each.
static void plan_partitions(const std::vector<uint32_t>& rp, uint32_t nv, uint32_t pv, uint32_t pe,
                            uint32_t pshift, std::vector<uint32_t>& starts) {
    starts.clear();
    const uint32_t g = 1u << pshift;
    uint32_t s = 0;
    while (s < nv) {
        uint32_t e = std::min<uint64_t>((uint64_t)s + g, nv);
        while (e < nv) {
            uint32_t e2 = std::min<uint64_t>((uint64_t)e + g, nv);
            if (e2 - s > pv) break;
            if (rp[e2] - rp[s] > pe) break;
            e = e2;
        }
        starts.push_back(s);
        s = e;
    }
    starts.push_back(nv);
}

// Size the process kernels' dynamic LDS for a dense slice (hs = 0) or a
// hashed slice of hs slots, and record how many workgroups fit per CU.
static int set_slice(fork_ctx* c, uint32_t hs) {
    size_t dyn = fk::process_dyn_lds(c->vpmax, hs);
    const void* kp = fk::process_kernel_ptr(c->wbytes);
    if (hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess)
        return fail(FORK_E_DEVICE, "partition slice of %u vertices (%u hash slots) does not fit in LDS", c->vpmax, hs);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kp, fk::process_threads(), dyn) != hipSuccess || occ <= 0)
        return fail(FORK_E_DEVICE, "process kernel does not fit on a CU with %zu bytes of LDS", dyn);
    c->blocks_per_cu = occ;
    const void* pk = fk::persistent_kernel_ptr(c->wbytes);
    occ = 0;
    if (hipFuncSetAttribute(pk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pk, fk::process_threads(), dyn) == hipSuccess)
        c->pers_blocks_per_cu = occ;
    else
        c->pers_blocks_per_cu = 0;
    c->hslots = hs;
    return FORK_OK;
}

extern "C" int fork_graph_load(fork_ctx** out, uint32_t nv, uint64_t ne, const uint64_t* row_ptr,
                               const uint32_t* col, const uint32_t* weight, const fork_config* cfg_in) {
    g_err[0] = 0;
    if (!out) return fail(FORK_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nv == 0) return fail(FORK_E_INVALID, "num_vertices must be >= 1");
    if (ne >= 0xffffffffull) return fail(FORK_E_INVALID, "num_edges must be < 2^32");
    if (!row_ptr || (ne && !col)) return fail(FORK_E_INVALID, "row_ptr/col is NULL");
    fork_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(FORK_E_DEVICE, "no HIP device");
    if (cfg.device < 0 || cfg.device >= ndev) return fail(FORK_E_INVALID, "bad device ordinal %d", cfg.device);
    // host copies of the inputs (validated)
    std::vector<uint64_t> rp64(nv + 1);
    std::vector<uint32_t> hcol, hw;
    const uint64_t* rps = row_ptr;
    const uint32_t* cols = col;
    const uint32_t* ws = weight;
    if (cfg.inputs_on_device) {
        if (hipSetDevice(cfg.device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
        HIPCHK(hipMemcpy(rp64.data(), row_ptr, (nv + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
        hcol.resize(ne);
        if (ne) HIPCHK(hipMemcpy(hcol.data(), col, ne * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (weight) {
            hw.resize(ne);
            if (ne) HIPCHK(hipMemcpy(hw.data(), weight, ne * sizeof(uint32_t), hipMemcpyDeviceToHost));
            ws = hw.data();
        }
        rps = rp64.data();
        cols = hcol.data();
    }
    if (rps[0] != 0 || rps[nv] != ne) return fail(FORK_E_INVALID, "row_ptr must run from 0 to num_edges");
    for (uint32_t v = 0; v < nv; ++v)
        if (rps[v + 1] < rps[v]) return fail(FORK_E_INVALID, "row_ptr decreases at %u", v);
    uint32_t wmax = 0;
    for (uint64_t e = 0; e < ne; ++e) {
        if (cols[e] >= nv) return fail(FORK_E_INVALID, "col[%llu] = %u out of range", (unsigned long long)e, cols[e]);
        if (ws) {
            if (ws[e] == 0) return fail(FORK_E_INVALID, "weight[%llu] is 0 (weights must be >= 1)", (unsigned long long)e);
            wmax = std::max(wmax, ws[e]);
        }
    }
    if (ws && wmax > 0x7fffffffu) return fail(FORK_E_INVALID, "weights must be < 2^31");
    double wsum = 0;
    if (ws) for (uint64_t e = 0; e < ne; ++e) wsum += ws[e];
    // the caller's vertex order: relabel to internal positions (vertex v ->
    // pos[v]), keeping each adjacency list's order
    std::vector<uint32_t> pos, orig, pcol, pw;
    std::vector<uint64_t> prp;
    if (cfg.vertex_order) {
        pos.resize(nv);
        if (cfg.inputs_on_device)
            HIPCHK(hipMemcpy(pos.data(), cfg.vertex_order, nv * sizeof(uint32_t), hipMemcpyDeviceToHost));
        else
            memcpy(pos.data(), cfg.vertex_order, nv * sizeof(uint32_t));
        orig.assign(nv, 0xffffffffu);
        for (uint32_t v = 0; v < nv; ++v) {
            if (pos[v] >= nv || orig[pos[v]] != 0xffffffffu)
                return fail(FORK_E_INVALID, "vertex_order is not a permutation (entry %u = %u)", v, pos[v]);
            orig[pos[v]] = v;
        }
        prp.assign(nv + 1, 0);
        for (uint32_t u = 0; u < nv; ++u) prp[u + 1] = prp[u] + (rps[orig[u] + 1] - rps[orig[u]]);
        pcol.resize(ne);
        if (ws) pw.resize(ne);
        for (uint32_t u = 0; u < nv; ++u) {
            const uint64_t b = rps[orig[u]], d = rps[orig[u] + 1] - b;
            for (uint64_t k = 0; k < d; ++k) {
                pcol[prp[u] + k] = pos[cols[b + k]];
                if (ws) pw[prp[u] + k] = ws[b + k];
            }
        }
        rps = prp.data();
        cols = pcol.data();
        if (ws) ws = pw.data();
    }

    fork_ctx* c = new fork_ctx();
    c->device = cfg.device;
    if (hipSetDevice(c->device) != hipSuccess) { delete c; return fail(FORK_E_DEVICE, "hipSetDevice failed"); }
    c->nv = nv;
    c->ne = ne;
    c->wbytes = !ws ? 0 : (wmax <= 0xff ? 1 : (wmax <= 0xffff ? 2 : 4));
    c->wmean = (ws && ne) ? wsum / (double)ne : 1.0;
    c->h_rowptr.resize(nv + 1);
    for (uint32_t v = 0; v <= nv; ++v) c->h_rowptr[v] = (uint32_t)rps[v];
    int rc = FORK_OK;
    auto cleanup = [&](int r) { fork_destroy(c); return r; };
    if (!pos.empty()) {
        if ((rc = dalloc(&c->d_pos, nv))) return cleanup(rc);
        if ((rc = dalloc(&c->d_orig, nv))) return cleanup(rc);
        if (hipMemcpy(c->d_pos, pos.data(), nv * 4ull, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_orig, orig.data(), nv * 4ull, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(FORK_E_DEVICE, "hipMemcpy of the vertex order failed"));
        c->h_pos.swap(pos);
    }
    // partition plan
    uint32_t pv = cfg.partition_vertices ? cfg.partition_vertices : fk::VPMAX;
    if (pv > fk::PVMAX) return cleanup(fail(FORK_E_INVALID, "partition_vertices must be <= %u", fk::PVMAX));
    uint32_t pe = cfg.partition_edges ? cfg.partition_edges : (uint32_t)std::min<uint64_t>(0xffffffffu, std::max<uint64_t>(4096, (uint64_t)pv * 64));
    uint32_t pshift = 0;
    while (pshift < 8 && (2u << pshift) <= pv / 4) ++pshift;
    plan_partitions(c->h_rowptr, nv, pv, pe, pshift, c->h_pstart);
    c->np = (uint32_t)c->h_pstart.size() - 1;
    c->pshift = pshift;
    if (c->np > 65535) return cleanup(fail(FORK_E_INVALID, "too many partitions (%u); raise partition_vertices", c->np));
    std::vector<uint16_t> vpart(((size_t)nv >> pshift) + 1);
    for (uint32_t P = 0; P < c->np; ++P)
        for (uint32_t b = c->h_pstart[P] >> pshift; b < ((c->h_pstart[P + 1] + (1u << pshift) - 1) >> pshift); ++b)
            vpart[b] = (uint16_t)P;
    // device graph
    if ((rc = dalloc(&c->d_rowptr, nv + 1))) return cleanup(rc);
    if ((rc = dalloc(&c->d_col, ne))) return cleanup(rc);
    if ((rc = dalloc(&c->d_pstart, c->np + 1))) return cleanup(rc);
    if ((rc = dalloc(&c->d_vpart, vpart.size()))) return cleanup(rc);
    auto cp = [&](void* d, const void* h, size_t bytes) -> int {
        hipError_t e = hipMemcpy(d, h, bytes, hipMemcpyHostToDevice);
        return e == hipSuccess ? FORK_OK : fail(FORK_E_DEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    };
    if ((rc = cp(c->d_rowptr, c->h_rowptr.data(), (nv + 1) * 4ull))) return cleanup(rc);
    if (ne && (rc = cp(c->d_col, cols, ne * 4ull))) return cleanup(rc);
    if ((rc = cp(c->d_pstart, c->h_pstart.data(), (c->np + 1) * 4ull))) return cleanup(rc);
    if ((rc = cp(c->d_vpart, vpart.data(), vpart.size() * 2ull))) return cleanup(rc);
    if (ws) {
        std::vector<uint8_t> packed(ne * (size_t)c->wbytes);
        for (uint64_t e = 0; e < ne; ++e) {
            if (c->wbytes == 1) packed[e] = (uint8_t)ws[e];
            else if (c->wbytes == 2) ((uint16_t*)packed.data())[e] = (uint16_t)ws[e];
            else ((uint32_t*)packed.data())[e] = ws[e];
        }
        uint8_t* dw = nullptr;
        if ((rc = dalloc(&dw, packed.size()))) return cleanup(rc);
        c->d_w = dw;
        if ((rc = cp(c->d_w, packed.data(), packed.size()))) return cleanup(rc);
    }
    // operation pool
    uint64_t pool = cfg.pool_bytes;
    if (!pool) {
        size_t fr = 0, tot = 0;
        hipMemGetInfo(&fr, &tot);
        pool = std::min<uint64_t>((uint64_t)64 << 30, std::max<uint64_t>((uint64_t)64 << 20, fr / 4));
    }
    const uint64_t per_chunk = sizeof(uint2) * fk::CH + 4 + 4 + 4;
    c->nch = std::max<uint64_t>(1024, pool / per_chunk);
    if (c->nch > 0x7fffffffull) c->nch = 0x7fffffffull;  // chunk links are int32
    if ((rc = dalloc(&c->d_chunks, c->nch * fk::CH))) return cleanup(rc);
    if ((rc = dalloc(&c->d_cnext, c->nch))) return cleanup(rc);
    if ((rc = dalloc(&c->d_ccount, c->nch))) return cleanup(rc);
    if ((rc = dalloc(&c->d_ring, c->nch))) return cleanup(rc);
    // partition summaries
    uint32_t** parr[] = {&c->d_pcount, &c->d_pbest_sp, &c->d_pbest_lv, &c->d_pbest_pr, &c->d_pfirst,
                         &c->d_plast, &c->d_pvisits, &c->d_pn, &c->d_sel, &c->d_pqn, &c->d_pready, &c->d_pqmin};
    for (auto pp : parr) if ((rc = dalloc(pp, c->np + 1))) return cleanup(rc);
    if ((rc = dalloc(&c->d_score, c->np + 1))) return cleanup(rc);
    if ((rc = dalloc(&c->d_mlp, fk::MLP_NPARAM))) return cleanup(rc);
    if ((rc = dalloc(&c->d_gstat, fk::gstat_bytes()))) return cleanup(rc);
    if ((rc = dalloc(&c->d_feat, (size_t)(c->np + 1) * fk::MLP_IN))) return cleanup(rc);
    if ((rc = dalloc(&c->d_tr, (size_t)(c->np + 1) * 2))) return cleanup(rc);
    if ((rc = dalloc(&c->d_ctl, 1))) return cleanup(rc);
    if (hipHostMalloc((void**)&c->h_ctl, sizeof(fk::Ctl), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(FORK_E_NOMEM, "hipHostMalloc failed"));
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return cleanup(fail(FORK_E_DEVICE, "hipEventCreate failed"));
    c->max_queries = cfg.max_queries;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    for (uint32_t P = 0; P < c->np; ++P) c->vpmax = std::max(c->vpmax, c->h_pstart[P + 1] - c->h_pstart[P]);
    // the dense slice (one LDS word per partition vertex) when it fits, else a hashed one
    if (set_slice(c, 0) != FORK_OK) {
        (void)hipGetLastError();
        g_err[0] = 0;
        c->dense_ok = false;
        if ((rc = set_slice(c, fk::HS_AUTO))) return cleanup(rc);
    }
    *out = c;
    return FORK_OK;
}

extern "C" int fork_partitions(fork_ctx* c, uint32_t* starts, uint32_t cap, uint32_t* num_parts) {
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (num_parts) *num_parts = c->np;
    if (starts) {
        uint32_t n = std::min<uint32_t>(cap + 1, c->np + 1);
        memcpy(starts, c->h_pstart.data(), n * sizeof(uint32_t));
    }
    return FORK_OK;
}

extern "C" int fork_submit(fork_ctx* c, int type, const uint32_t* sources, uint32_t n, const void* params,
                           uint32_t* first_id) {
    g_err[0] = 0;
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (type != FORK_SSSP && type != FORK_BFS && type != FORK_PPR) return fail(FORK_E_INVALID, "bad query type %d", type);
    if (n && !sources) return fail(FORK_E_INVALID, "sources is NULL");
    QueryRec base{(uint32_t)type, 0, 0, 0.f, 0.f};
    if (type == FORK_PPR) {
        if (!params) return fail(FORK_E_INVALID, "PPR needs fork_ppr_params");
        const fork_ppr_params* pp = (const fork_ppr_params*)params;
        if (!(pp->alpha > 0.f && pp->alpha < 1.f)) return fail(FORK_E_INVALID, "alpha must be in (0,1)");
        if (!(pp->epsilon > 0.f)) return fail(FORK_E_INVALID, "epsilon must be > 0");
        if (pp->eps_mode != 0 && pp->eps_mode != 1) return fail(FORK_E_INVALID, "eps_mode must be 0 or 1");
        if (!(pp->l1_target >= 0.f && pp->l1_target <= 1e30f))
            return fail(FORK_E_INVALID, "l1_target must be finite and >= 0");
        base.alpha = pp->alpha;
        base.eps = pp->epsilon;
        base.mode = (uint32_t)pp->eps_mode;
        base.l1 = pp->l1_target;
    }
    for (uint32_t i = 0; i < n; ++i)
        if (sources[i] >= c->nv) return fail(FORK_E_INVALID, "source %u out of range (V=%u)", sources[i], c->nv);
    c->plan_budget = 0;  // the batch changes: plan its waves again
    if (c->ran) {  // a new batch
        c->queries.clear();
        c->digests.clear();
        c->ran = false;
        c->res_n = 0;
        c->dig_pending = false;
    }
    if (first_id) *first_id = (uint32_t)c->queries.size();
    for (uint32_t i = 0; i < n; ++i) {
        QueryRec r = base;
        r.src = c->h_pos.empty() ? sources[i] : c->h_pos[sources[i]];
        c->queries.push_back(r);
    }
    return FORK_OK;
}

static uint64_t qwords(const fork_ctx* c, uint32_t type) { return (type == FORK_PPR ? 2ull : 1ull) * c->nv; }

// Allocate per-wave buffers for `nq` queries needing `words` state words.
static int ensure_wave(fork_ctx* c, uint32_t nq, size_t words, uint32_t kmax) {
    int rc;
    if (nq > c->qcap || kmax > c->kmax_cap) {
        hipFree(c->d_bhead); hipFree(c->d_btw); hipFree(c->d_bover); hipFree(c->d_items);
        hipFree(c->d_bval); hipFree(c->d_bcnt); hipFree(c->d_bfirst); hipFree(c->d_qmin);
        c->d_bval = c->d_bcnt = c->d_bfirst = c->d_qmin = nullptr;
        hipFree(c->d_qtype); hipFree(c->d_qsrc); hipFree(c->d_qmode); hipFree(c->d_qoff);
        hipFree(c->d_qalpha); hipFree(c->d_qeps); hipFree(c->d_digest);
        hipFree(c->d_certq); hipFree(c->d_rnorm);
        c->d_certq = nullptr; c->d_rnorm = nullptr;
        c->d_bhead = nullptr; c->d_btw = nullptr; c->d_bover = nullptr; c->d_items = nullptr;
        uint32_t qc = std::max(nq, c->qcap);
        uint32_t kc = std::max(kmax, c->kmax_cap);
        size_t nb = (size_t)c->np * qc;
        if ((rc = dalloc(&c->d_bhead, nb))) return rc;
        if ((rc = dalloc(&c->d_btw, nb))) return rc;
        if ((rc = dalloc(&c->d_bover, nb))) return rc;
        if ((rc = dalloc(&c->d_bval, nb))) return rc;
        if ((rc = dalloc(&c->d_bcnt, nb))) return rc;
        if ((rc = dalloc(&c->d_bfirst, nb))) return rc;
        if ((rc = dalloc(&c->d_qmin, qc))) return rc;
        c->item_cap = ((kc + fk::NXCD - 1) / fk::NXCD) * qc;
        if ((rc = dalloc(&c->d_items, (size_t)fk::NXCD * c->item_cap))) return rc;
        if ((rc = dalloc(&c->d_qtype, qc))) return rc;
        if ((rc = dalloc(&c->d_qsrc, qc))) return rc;
        if ((rc = dalloc(&c->d_qmode, qc))) return rc;
        if ((rc = dalloc(&c->d_qoff, qc))) return rc;
        if ((rc = dalloc(&c->d_qalpha, qc))) return rc;
        if ((rc = dalloc(&c->d_qeps, qc))) return rc;
        if ((rc = dalloc(&c->d_digest, (size_t)qc * 6))) return rc;
        if ((rc = dalloc(&c->d_certq, qc))) return rc;
        if ((rc = dalloc(&c->d_rnorm, qc))) return rc;
        c->qcap = qc;
        c->kmax_cap = kc;
    }
    if (words > c->state_words_cap) {
        hipFree(c->d_state);
        c->d_state = nullptr;
        if ((rc = dalloc(&c->d_state, words))) return rc;
        c->state_words_cap = words;
    }
    return FORK_OK;
}

static fk::GraphDev graph_dev(const fork_ctx* c) {
    fk::GraphDev g;
    g.nv = c->nv; g.np = c->np; g.pshift = c->pshift; g.wbytes = c->wbytes;
    g.rowptr = c->d_rowptr; g.col = c->d_col; g.w = c->d_w; g.pstart = c->d_pstart; g.vpart = c->d_vpart;
    return g;
}

static fk::BufDev buf_dev(const fork_ctx* c) {
    fk::BufDev B;
    B.bhead = c->d_bhead; B.btw = c->d_btw; B.bover = c->d_bover; B.bval = c->d_bval; B.bcnt = c->d_bcnt; B.bfirst = c->d_bfirst;
    B.qmin = c->d_qmin; B.pready = c->d_pready; B.chunks = c->d_chunks; B.cnext = c->d_cnext;
    B.ccount = c->d_ccount; B.ring = c->d_ring; B.nch = c->nch; B.pcount = c->d_pcount;
    B.pbest_sp = c->d_pbest_sp; B.pbest_lv = c->d_pbest_lv; B.pbest_pr = c->d_pbest_pr;
    B.pfirst = c->d_pfirst; B.plast = c->d_plast; B.pvisits = c->d_pvisits; B.pn = c->d_pn;
    B.sel = c->d_sel; B.pqn = c->d_pqn; B.pqmin = c->d_pqmin; B.score = c->d_score;
    B.tr_useful = c->d_tr; B.tr_work = c->d_tr + c->np; B.items = c->d_items; B.item_cap = c->item_cap; B.ctl = c->d_ctl;
    return B;
}

// Digests of the resident wave's queries (count, sum and hash of the reached
// values; PPR sums and max), copied to the host.
static int wave_digest(fork_ctx* c, hipStream_t s) {
    if (!c->dig_pending) return FORK_OK;
    const uint32_t q0 = c->res_first, nq = c->res_n;
    HIPCHK(hipEventRecord(c->ev[2], s));
    if (c->res_grouped) {
        HIPCHK(hipMemsetAsync(c->d_digest, 0, (size_t)nq * 6 * 8, s));
        HIPCHK(fk::launch_gdigest(c->resG, c->nv, c->d_lq, c->d_digest, c->d_orig, s));
    } else {
        HIPCHK(fk::launch_digest(c->resQ, c->nv, c->d_digest, c->d_orig, s));
    }
    HIPCHK(hipEventRecord(c->ev[3], s));
    std::vector<unsigned long long> dg((size_t)nq * 6);
    HIPCHK(hipMemcpyAsync(dg.data(), c->d_digest, dg.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < nq; ++i) {
        fork_digest& d = c->digests[q0 + i];
        d.count = dg[i * 6 + 0];
        d.sum = dg[i * 6 + 1];
        d.hash = dg[i * 6 + 2];
        memcpy(&d.fsum, &dg[i * 6 + 3], 8);
        memcpy(&d.fres, &dg[i * 6 + 4], 8);
        memcpy(&d.fmax, &dg[i * 6 + 5], 8);
    }
    float t_dig = 0;
    hipEventElapsedTime(&t_dig, c->ev[2], c->ev[3]);
    c->stats.digest_ms += t_dig;
    c->dig_pending = false;
    return FORK_OK;
}

static int run_wave(fork_ctx* c, uint32_t q0, uint32_t nq, const fork_run_opts& o, hipStream_t s,
                    const fk::PassCfg& cfg, uint64_t& passes_left, bool trace) {
    // layout of the wave's state
    std::vector<uint32_t> qt(nq), qs(nq), qm(nq);
    std::vector<unsigned long long> qo(nq);
    std::vector<float> qa(nq), qe(nq);
    size_t words = 0;
    bool mixed = false;
    for (uint32_t i = 0; i < nq; ++i) {
        const QueryRec& r = c->queries[q0 + i];
        qt[i] = r.type; qs[i] = r.src; qm[i] = r.mode; qa[i] = r.alpha; qe[i] = r.eps;
        qo[i] = words;
        words += qwords(c, r.type);
        if (r.type != c->queries[q0].type) mixed = true;
    }
    int rc = ensure_wave(c, nq, words, cfg.kmax);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(c->d_qtype, qt.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qsrc, qs.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qmode, qm.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qoff, qo.data(), nq * 8ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qalpha, qa.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qeps, qe.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    fk::PassCfg pc = cfg;
    pc.mixed = mixed ? 1u : 0u;
    fk::QueryDev Q;
    Q.nq = nq; Q.qc = c->qcap; Q.qtype = c->d_qtype; Q.qoff = c->d_qoff; Q.qalpha = c->d_qalpha;
    Q.qeps = c->d_qeps; Q.qmode = c->d_qmode; Q.state = c->d_state;
    Q.final_state = trace ? c->d_final : nullptr;
    pc.trace = trace ? 1u : 0u;
    fk::GraphDev g = graph_dev(c);
    fk::BufDev B = buf_dev(c);
    HIPCHK(hipEventRecord(c->ev[0], s));
    // state init: distances/levels = INF, p = r = 0
    for (uint32_t i = 0; i < nq;) {
        uint32_t j = i;
        while (j < nq && (qt[j] == FORK_PPR) == (qt[i] == FORK_PPR)) ++j;
        size_t w0 = qo[i], w1 = (j < nq) ? qo[j] : words;
        if (qt[i] == FORK_PPR) HIPCHK(hipMemsetAsync(c->d_state + w0, 0, (w1 - w0) * 4, s));
        else HIPCHK(hipMemsetD32Async((hipDeviceptr_t)(c->d_state + w0), (int)fk::INF, w1 - w0, s));
        i = j;
    }
    HIPCHK(hipMemsetAsync(c->d_bhead, 0xff, (size_t)c->np * c->qcap * 4, s));
    HIPCHK(hipMemsetAsync(c->d_bover, 0xff, (size_t)c->np * c->qcap * 4, s));
    HIPCHK(fk::launch_fill64(c->d_btw, (unsigned long long)c->np * c->qcap, fk::BTW_EMPTY, s));
    HIPCHK(hipMemsetAsync(c->d_bval, 0xff, (size_t)c->np * c->qcap * 4, s));
    HIPCHK(hipMemsetAsync(c->d_bcnt, 0, (size_t)c->np * c->qcap * 4, s));
    HIPCHK(hipMemsetAsync(c->d_bfirst, 0xff, (size_t)c->np * c->qcap * 4, s));
    HIPCHK(hipMemsetAsync(c->d_ccount, 0, (size_t)c->nch * 4, s));
    HIPCHK(hipMemsetAsync(c->d_pcount, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pbest_sp, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pbest_lv, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetAsync(c->d_pbest_pr, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pfirst, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetAsync(c->d_plast, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pvisits, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pn, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pqn, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pqmin, 0, (c->np + 1) * 4ull, s));
    if (c->nch < nq + 64ull) return fail(FORK_E_CAPACITY, "operation pool too small for %u queries", nq);
    fk::Ctl ctl0{};
    ctl0.ring_head = nq;
    ctl0.ring_tail = c->nch;
    ctl0.avail_end = c->nch;
    *c->h_ctl = ctl0;
    HIPCHK(hipMemcpyAsync(c->d_ctl, c->h_ctl, sizeof(fk::Ctl), hipMemcpyHostToDevice, s));
    HIPCHK(fk::launch_ring_init(c->d_ring, c->nch, s));
    HIPCHK(hipMemcpyAsync(c->d_qsrc, qs.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(fk::launch_seed(g, Q, B, c->d_qsrc, s));
    HIPCHK(hipEventRecord(c->ev[1], s));
    // pass loop (Algorithm 2): select -> detach -> process, until no buffer holds work
    const uint32_t blocks = (uint32_t)std::max(1, c->num_cu * c->blocks_per_cu);
    uint32_t batch = 1;
    bool done = false;
    uint32_t pass_mark = 0;
    const char* prog = getenv("FORK_PROGRESS");
    const double prog_every = prog ? atof(prog) : 0.0;  // seconds between progress lines (0 = off)
    auto t_start = std::chrono::steady_clock::now();
    auto t_last = t_start;
    // L1-certified PPR queries (wave-local ids).  Once the wave has drained,
    // a query whose residual mass ||r||_1 is above 0.9 of its target gets a
    // lower threshold and is pushed again from every vertex that now
    // qualifies.  By the push invariant ||pi_s - p||_1 = ||PPR(r)||_1 <=
    // ||r||_1, so the target holds with a tenth of it left for fp32 rounding.
    std::vector<uint32_t> cert;
    for (uint32_t i = 0; i < nq; ++i)
        if (qt[i] == FORK_PPR && c->queries[q0 + i].l1 > 0.f) cert.push_back(i);
    constexpr uint32_t MAX_REFINE = 32;
    uint32_t refine_rounds = 0;
    // returns < 0 on error, 0 when every certified query meets its target,
    // 1 after launching the refinement passes
    auto refine = [&]() -> int {
        if (cert.empty()) return 0;
        HIPCHK(hipMemcpyAsync(c->d_certq, cert.data(), cert.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(fk::launch_rnorm(Q, c->nv, c->d_certq, (uint32_t)cert.size(), c->d_rnorm, s));
        std::vector<double> rn(cert.size());
        HIPCHK(hipMemcpyAsync(rn.data(), c->d_rnorm, rn.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<uint32_t> above;
        for (size_t k = 0; k < cert.size(); ++k) {
            const uint32_t i = cert[k];
            const double tgt = 0.9 * (double)c->queries[q0 + i].l1;
            if (rn[k] <= tgt) continue;
            // ||r||_1 shrinks roughly in proportion to the threshold
            const double f = std::min(0.5, std::max(1e-3, 0.5 * tgt / rn[k]));
            qe[i] = (float)((double)qe[i] * f);
            if (!(qe[i] > 0.f))
                return fail(FORK_E_NOT_CONVERGED, "query %u: threshold underflow with ||r||_1 = %g", q0 + i, rn[k]);
            above.push_back(i);
        }
        cert.swap(above);
        if (cert.empty()) return 0;
        if (++refine_rounds > MAX_REFINE)
            return fail(FORK_E_NOT_CONVERGED, "L1 target not met after %u threshold reductions", MAX_REFINE);
        const unsigned long long pairs = (unsigned long long)c->np * cert.size();
        const unsigned long long per = (unsigned long long)fk::NXCD * c->item_cap;
        const uint64_t npass = (pairs + per - 1) / per;
        if (passes_left != ~0ull) {
            if (npass > passes_left) return fail(FORK_E_NOT_CONVERGED, "max_passes reached with work pending");
            passes_left -= npass;
        }
        HIPCHK(hipMemcpyAsync(c->d_qeps, qe.data(), nq * 4ull, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->d_certq, cert.data(), cert.size() * 4, hipMemcpyHostToDevice, s));
        if (o.profile && c->pev.size() < 2) {
            c->pev.resize(2, nullptr);
            for (auto& e : c->pev) if (!e) HIPCHK(hipEventCreate(&e));
        }
        for (unsigned long long lo = 0; lo < pairs; lo += per) {
            const uint32_t n = (uint32_t)std::min(per, pairs - lo);
            HIPCHK(fk::launch_rescan_items(B, c->np, c->d_certq, lo, n, s));
            if (o.profile) HIPCHK(hipEventRecord(c->pev[0], s));
            HIPCHK(fk::launch_process(g, Q, B, pc, blocks, c->vpmax, c->hslots, s));
            if (o.profile) {
                HIPCHK(hipEventRecord(c->pev[1], s));
                HIPCHK(hipEventSynchronize(c->pev[1]));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, c->pev[0], c->pev[1]));
                c->stats.process_ms += ms;
                c->stats.process_launches += 1;
            }
        }
        HIPCHK(hipStreamSynchronize(s));  // the host lists stay alive until the copies ran
        c->stats.refine_rounds += 1;
        return 1;
    };
    while (true) {
        if (done) {
            const int r = refine();
            if (r < 0) return r;
            if (r == 0) break;
            done = false;
        }
        uint32_t nb = trace ? 1u : batch;
        if (passes_left != ~0ull) nb = (uint32_t)std::min<uint64_t>(nb, passes_left);
        if (nb == 0) return fail(FORK_E_NOT_CONVERGED, "max_passes reached with work pending");
        if (o.profile && c->pev.size() < 2 * nb) {
            size_t old = c->pev.size();
            c->pev.resize(2 * nb, nullptr);
            for (size_t k = old; k < c->pev.size(); ++k) HIPCHK(hipEventCreate(&c->pev[k]));
        }
        if (trace) {
            // one pass with the features of every partition and the usefulness of the visits
            HIPCHK(hipMemsetAsync(c->d_tr, 0, (size_t)c->np * 2 * sizeof(float), s));
            HIPCHK(fk::launch_summaries(g, B, Q, pc, s));
            HIPCHK(fk::launch_mlp_score(g, B, c->d_mlp, c->d_score, c->d_feat, c->d_gstat, 0, s));
            HIPCHK(fk::launch_select(g, B, pc, s));
            HIPCHK(fk::launch_worklist(B, Q, pc, s));
            HIPCHK(fk::launch_process(g, Q, B, pc, blocks, c->vpmax, c->hslots, s));
            std::vector<uint32_t> sel(c->np);
            std::vector<float> feat((size_t)c->np * fk::MLP_IN), tr((size_t)c->np * 2);
            HIPCHK(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(fk::Ctl), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(sel.data(), c->d_sel, c->np * 4ull, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(feat.data(), c->d_feat, feat.size() * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(tr.data(), c->d_tr, tr.size() * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            const uint32_t nsel = std::min<uint32_t>(c->h_ctl->nsel, c->np);
            for (uint32_t j = 0; j < nsel; ++j) {
                uint32_t P = sel[j];
                if (tr[c->np + P] <= 0.f) continue;
                c->trace.insert(c->trace.end(), feat.begin() + (size_t)P * fk::MLP_IN,
                                feat.begin() + (size_t)(P + 1) * fk::MLP_IN);
                c->trace.push_back(tr[P]);
                c->trace.push_back(tr[c->np + P]);
                c->trace.push_back((float)c->h_ctl->pass);
                c->trace.push_back((float)P);
            }
        } else if (o.persistent) {
            // one cooperative launch runs up to 64 passes per batch slot on the device
            if (c->pers_blocks_per_cu <= 0) return fail(FORK_E_DEVICE, "persistent kernel does not fit on a CU");
            const uint32_t pblocks = (uint32_t)(c->num_cu * c->pers_blocks_per_cu);
            if (o.profile) HIPCHK(hipEventRecord(c->pev[0], s));
            uint64_t lp = 64ull * batch;
            if (passes_left != ~0ull) lp = std::min<uint64_t>(lp, passes_left);
            HIPCHK(fk::launch_persistent(g, Q, B, pc, pblocks, c->vpmax, c->hslots, (uint32_t)lp, c->d_mlp, c->d_score,
                                         c->d_gstat, s));
            if (o.profile) HIPCHK(hipEventRecord(c->pev[1], s));
            nb = 1;
        } else {
            for (uint32_t k = 0; k < nb; ++k) {
                HIPCHK(fk::launch_summaries(g, B, Q, pc, s));
                if (pc.sched == fk::S_LEARNED)
                    HIPCHK(fk::launch_mlp_score(g, B, c->d_mlp, c->d_score, nullptr, c->d_gstat, 0, s));
                HIPCHK(fk::launch_select(g, B, pc, s));
                HIPCHK(fk::launch_worklist(B, Q, pc, s));
                if (o.profile) HIPCHK(hipEventRecord(c->pev[2 * k], s));
                HIPCHK(fk::launch_process(g, Q, B, pc, blocks, c->vpmax, c->hslots, s));
                if (o.profile) HIPCHK(hipEventRecord(c->pev[2 * k + 1], s));
            }
        }
        if (passes_left != ~0ull && !o.persistent) passes_left -= nb;
        HIPCHK(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(fk::Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (o.profile) {
            for (uint32_t k = 0; k < nb; ++k) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, c->pev[2 * k], c->pev[2 * k + 1]));
                c->stats.process_ms += ms;
            }
            c->stats.process_launches += nb;
        }
        const fk::Ctl& h = *c->h_ctl;
        if (h.err & fk::ERR_CORRUPT) return fail(FORK_E_DEVICE, "device consistency check failed (flags 0x%x)", h.err);
        if (h.err & fk::ERR_SPILL) {
            c->spill_refused = true;
            return fail(FORK_E_CAPACITY, "a visit retained %u activated vertices as buffered operations (frontier "
                        "full), more than the bound of %u: this frontier-spill regime is refused; load the graph "
                        "with smaller partitions", h.c_spill_max, fk::SPILL_MAX);
        }
        if (h.err & fk::ERR_CAPACITY)
            return fail(FORK_E_CAPACITY, "operation pool exhausted (%llu chunks) with %u queries in flight",
                        c->nch, nq);
        if (h.err) return fail(FORK_E_DEVICE, "device error flags 0x%x", h.err);
        if (h.pending_parts == 0) done = true;
        if (o.persistent && passes_left != ~0ull) {
            uint64_t used = h.pass - pass_mark;
            pass_mark = h.pass;
            passes_left = used >= passes_left ? 0 : passes_left - used;
        }
        batch = std::min<uint32_t>(batch * 2, 64);
        if (prog_every > 0) {
            auto now = std::chrono::steady_clock::now();
            if (std::chrono::duration<double>(now - t_last).count() >= prog_every) {
                t_last = now;
                fprintf(stderr, "[fork] wave q%u+%u pass %u pending_parts %u pending_ops %llu edges %llu emitted %llu t=%.1fs\n",
                        q0, nq, h.pass, h.pending_parts, h.pending_ops, h.c_edges, h.c_emitted,
                        std::chrono::duration<double>(now - t_start).count());
                fflush(stderr);
            }
        }
    }
    HIPCHK(hipEventRecord(c->ev[2], s));
    HIPCHK(hipStreamSynchronize(s));
    float t_init = 0, t_run = 0, t_dig = 0;
    hipEventElapsedTime(&t_init, c->ev[0], c->ev[1]);
    hipEventElapsedTime(&t_run, c->ev[1], c->ev[2]);
    // digests: computed by fork_run before the next wave reuses the state,
    // or on the first request for the wave that stays resident
    c->resQ = Q;
    c->resQ.final_state = nullptr;
    c->res_grouped = false;
    c->dig_pending = true;
    const fk::Ctl& h = *c->h_ctl;
    fork_stats_t& st = c->stats;
    st.init_ms += t_init;
    st.run_ms += t_run;
    st.passes += h.pass;
    st.work_items += h.c_items;
    st.edges += h.c_edges;
    st.improved += h.c_improved;
    st.ops_emitted += h.c_emitted;
    st.ops_consumed += h.c_consumed;
    st.vertex_pushes += h.c_vpush;
    st.yields += h.c_yields;
    st.chunks += h.c_chunks;
    st.intra_edges += h.c_intra;
    st.pruned += h.c_pruned;
    st.selected_edges += h.c_sel_edges;
    st.ppr_edges += h.c_edges_ppr;
    st.ppr_vertex_pushes += h.c_vpush_ppr;
    st.spilled += h.c_spill;
    st.spill_max = std::max<uint64_t>(st.spill_max, h.c_spill_max);
    st.waves += 1;
    c->res_first = q0;
    c->res_n = nq;
    c->res_off.assign(qo.begin(), qo.end());
    return FORK_OK;
}

// Grow-only device buffer of n elements.
template <class T> static int grow(T** p, size_t& cap, size_t n) {
    if (n <= cap && *p) return FORK_OK;
    hipFree(*p);
    *p = nullptr;
    cap = 0;
    int rc = dalloc(p, n);
    if (rc) return rc;
    cap = n;
    return FORK_OK;
}

// Pair summaries (np x ng) and per-group arrays (ng groups of 64 lanes) of the
// grouped engine, grown to hold ng groups.
static int grow_groups(fork_ctx* c, size_t ng) {
    constexpr size_t GW = 64;
    const size_t npairs = (size_t)c->np * ng;
    int rc;
    size_t cap = c->pair_cap;
    if ((rc = grow(&c->d_icnt, cap, npairs))) return rc;
    cap = c->pair_cap;
    if ((rc = grow(&c->d_ibest, cap, npairs))) return rc;
    cap = c->pair_cap;
    if ((rc = grow(&c->d_ifirst, cap, npairs))) return rc;
    c->pair_cap = std::max(c->pair_cap, npairs);
    if (c->grp_cap < ng) {
        void* gp[] = {c->d_gmin, c->d_gtype, c->d_goff, c->d_lq, c->d_lsrc, c->d_lmode, c->d_lalpha, c->d_leps};
        for (void* q : gp) hipFree(q);
        c->d_gmin = c->d_gtype = c->d_lq = c->d_lsrc = c->d_lmode = nullptr;
        c->d_goff = nullptr;
        c->d_lalpha = c->d_leps = nullptr;
        c->grp_cap = 0;
        if ((rc = dalloc(&c->d_gmin, ng)) || (rc = dalloc(&c->d_gtype, ng)) || (rc = dalloc(&c->d_goff, ng)) ||
            (rc = dalloc(&c->d_lq, ng * GW)) || (rc = dalloc(&c->d_lsrc, ng * GW)) ||
            (rc = dalloc(&c->d_lmode, ng * GW)) || (rc = dalloc(&c->d_lalpha, ng * GW)) ||
            (rc = dalloc(&c->d_leps, ng * GW)))
            return rc;
        c->grp_cap = (uint32_t)ng;
    }
    return FORK_OK;
}

// Size the grouped engine's buffers once for the largest wave of a run.  The
// waves differ in their mix of query types; growing a buffer between waves
// would free it and allocate it again, and an allocation of this size (up to
// the device memory budget) takes seconds.
static int reserve_groups(fork_ctx* c, const std::vector<std::pair<uint32_t, uint32_t>>& waves, uint32_t kmax) {
    constexpr size_t GW = 64;
    size_t words = 0, gwords = 0, ng = 0;
    uint32_t nq = 0;
    for (const auto& w : waves) {
        size_t ww = 0, cnt[3] = {0, 0, 0};
        for (uint32_t i = 0; i < w.second; ++i) {
            const uint32_t t = c->queries[w.first + i].type;
            ww += qwords(c, t);
            ++cnt[t == FORK_SSSP ? 0 : t == FORK_BFS ? 1 : 2];
        }
        size_t g = 0, gw = 0;
        for (int k = 0; k < 3; ++k) {
            const size_t n = (cnt[k] + GW - 1) / GW;
            g += n;
            gw += n * (k == 2 ? 2ull : 1ull) * c->nv * GW;
        }
        words = std::max(words, ww);
        gwords = std::max(gwords, gw);
        ng = std::max(ng, g);
        nq = std::max(nq, w.second);
    }
    int rc = ensure_wave(c, nq, words, kmax);
    if (rc) return rc;
    if ((rc = grow(&c->d_gstate, c->gstate_cap, gwords))) return rc;
    if ((rc = grow(&c->d_gpend, c->gpend_cap, ng * c->nv))) return rc;
    if ((rc = grow(&c->d_gbits, c->gbits_cap, ng * (c->nv / 32 + 2)))) return rc;
    return grow_groups(c, ng);
}

// One wave on the grouped engine: the wave's queries of each type are taken
// 64 at a time as lane groups with vertex-major state rows.  The result vectors
// are written in the per-query layout of run_wave at the end, so fetch,
// digests, sweeps and BC read them the same way.
static int run_wave_group(fork_ctx* c, uint32_t q0, uint32_t nq, const fork_run_opts& o, hipStream_t s,
                          const fk::PassCfg& cfg, uint64_t& passes_left, bool keep_vectors) {
    constexpr uint32_t GW = 64;
    std::vector<uint32_t> qt(nq), qm(nq);
    std::vector<unsigned long long> qo(nq);
    std::vector<float> qa(nq), qe(nq);
    size_t words = 0;
    bool mixed = false;
    for (uint32_t i = 0; i < nq; ++i) {
        const QueryRec& r = c->queries[q0 + i];
        qt[i] = r.type; qm[i] = r.mode; qa[i] = r.alpha; qe[i] = r.eps;
        qo[i] = words;
        words += qwords(c, r.type);
        if (r.type != c->queries[q0].type) mixed = true;
    }
    // lane groups: queries of one type in submit order, 64 to a group
    std::vector<uint32_t> gtype, lq, lsrc, lmode;
    std::vector<unsigned long long> goff;
    std::vector<float> lalpha, leps;
    size_t gwords = 0;
    for (uint32_t t : {(uint32_t)FORK_SSSP, (uint32_t)FORK_BFS, (uint32_t)FORK_PPR}) {
        std::vector<uint32_t> idx;
        for (uint32_t i = 0; i < nq; ++i) if (qt[i] == t) idx.push_back(i);
        for (size_t k = 0; k < idx.size(); k += GW) {
            gtype.push_back(t);
            goff.push_back(gwords);
            gwords += (t == FORK_PPR ? 2ull : 1ull) * c->nv * GW;
            for (uint32_t l = 0; l < GW; ++l) {
                if (k + l < idx.size()) {
                    const QueryRec& r = c->queries[q0 + idx[k + l]];
                    lq.push_back(idx[k + l]); lsrc.push_back(r.src); lmode.push_back(r.mode);
                    lalpha.push_back(r.alpha); leps.push_back(r.eps);
                } else {
                    lq.push_back(0xffffffffu); lsrc.push_back(0xffffffffu); lmode.push_back(0);
                    lalpha.push_back(0.15f); leps.push_back(1.0f);
                }
            }
        }
    }
    const uint32_t ng = (uint32_t)gtype.size();
    if (c->vpmax > 16384)
        return fail(FORK_E_INVALID, "the grouped engine needs partitions of at most 16384 vertices (this graph's "
                    "largest has %u; load it with partition_vertices <= 16384)", c->vpmax);
    if (c->nv >= (1u << 24))  // its kernels address a group's state rows with 32-bit byte offsets
        return fail(FORK_E_INVALID, "the grouped engine takes graphs of fewer than 16,777,216 vertices (this one "
                    "has %u)", c->nv);
    int rc = ensure_wave(c, nq, words, cfg.kmax);
    if (rc) return rc;
    if ((uint64_t)ng * ((cfg.kmax + fk::NXCD - 1) / fk::NXCD) > (uint64_t)c->item_cap)
        return fail(FORK_E_DEVICE, "grouped engine: item list too small");
    const uint32_t bw = c->nv / 32 + 2;
    const size_t npairs = (size_t)c->np * ng;
    if ((rc = grow(&c->d_gstate, c->gstate_cap, gwords))) return rc;
    if ((rc = grow(&c->d_gpend, c->gpend_cap, (size_t)ng * c->nv))) return rc;
    if ((rc = grow(&c->d_gbits, c->gbits_cap, (size_t)ng * bw))) return rc;
    if ((rc = grow_groups(c, ng))) return rc;
    // workgroup size of the grouped pass (waves that share one pair's visit)
    const uint32_t gnt = o.group_threads ? o.group_threads : 256u;
    if (gnt != 256 && gnt != 512 && gnt != 1024)
        return fail(FORK_E_INVALID, "group_threads must be 0, 256, 512 or 1024, got %u", gnt);
    {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fk::gprocess_kernel_ptr(c->wbytes), (int)gnt, 0) !=
                hipSuccess || occ <= 0)
            return fail(FORK_E_DEVICE, "grouped pass kernel does not fit on a CU");
        c->group_blocks_per_cu = occ;
    }
    HIPCHK(hipMemcpyAsync(c->d_qtype, qt.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qmode, qm.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qoff, qo.data(), nq * 8ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qalpha, qa.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_qeps, qe.data(), nq * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_gtype, gtype.data(), ng * 4ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_goff, goff.data(), ng * 8ull, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_lq, lq.data(), lq.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_lsrc, lsrc.data(), lsrc.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_lmode, lmode.data(), lmode.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_lalpha, lalpha.data(), lalpha.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c->d_leps, leps.data(), leps.size() * 4, hipMemcpyHostToDevice, s));
    fk::PassCfg pc = cfg;
    pc.mixed = mixed ? 1u : 0u;
    pc.trace = 0;
    fk::QueryDev Q;
    Q.nq = nq; Q.qc = c->qcap; Q.qtype = c->d_qtype; Q.qoff = c->d_qoff; Q.qalpha = c->d_qalpha;
    Q.qeps = c->d_qeps; Q.qmode = c->d_qmode; Q.state = c->d_state; Q.final_state = nullptr;
    fk::GroupDev G;
    G.ng = ng; G.gtype = c->d_gtype; G.goff = c->d_goff; G.lalpha = c->d_lalpha; G.leps = c->d_leps;
    G.lmode = c->d_lmode; G.state = c->d_gstate; G.pend = c->d_gpend; G.bits = c->d_gbits; G.bw = bw;
    G.icnt = c->d_icnt; G.ibest = c->d_ibest; G.ifirst = c->d_ifirst; G.gmin = c->d_gmin;
    fk::GraphDev g = graph_dev(c);
    fk::BufDev B = buf_dev(c);
    HIPCHK(hipEventRecord(c->ev[0], s));
    for (uint32_t k = 0; k < ng; ++k) {
        const size_t n = (size_t)c->nv * GW;
        if (gtype[k] == FORK_PPR) HIPCHK(hipMemsetAsync(c->d_gstate + goff[k], 0, 2 * n * 4, s));
        else HIPCHK(hipMemsetD32Async((hipDeviceptr_t)(c->d_gstate + goff[k]), (int)fk::INF, n, s));
    }
    HIPCHK(hipMemsetAsync(c->d_gpend, 0, (size_t)ng * c->nv * 8, s));
    HIPCHK(hipMemsetAsync(c->d_gbits, 0, (size_t)ng * bw * 4, s));
    HIPCHK(hipMemsetAsync(c->d_icnt, 0, npairs * 4, s));
    HIPCHK(hipMemsetAsync(c->d_ibest, 0xff, npairs * 4, s));
    HIPCHK(hipMemsetAsync(c->d_ifirst, 0xff, npairs * 4, s));
    HIPCHK(hipMemsetAsync(c->d_pcount, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pbest_sp, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pbest_lv, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetAsync(c->d_pbest_pr, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetD32Async((hipDeviceptr_t)c->d_pfirst, (int)fk::INF, c->np + 1, s));
    HIPCHK(hipMemsetAsync(c->d_plast, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pvisits, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pn, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pqn, 0, (c->np + 1) * 4ull, s));
    HIPCHK(hipMemsetAsync(c->d_pqmin, 0, (c->np + 1) * 4ull, s));
    fk::Ctl ctl0{};
    *c->h_ctl = ctl0;
    HIPCHK(hipMemcpyAsync(c->d_ctl, c->h_ctl, sizeof(fk::Ctl), hipMemcpyHostToDevice, s));
    HIPCHK(fk::launch_gseed(g, G, c->d_lsrc, s));
    HIPCHK(hipEventRecord(c->ev[1], s));
    // twice what fits at once: a workgroup that runs out of items exits, and
    // the next one takes its place on the CU
    const uint32_t blocks = (uint32_t)std::max(1, 2 * c->num_cu * c->group_blocks_per_cu);
    uint32_t batch = 1;
    while (true) {
        uint32_t nb = batch;
        if (passes_left != ~0ull) nb = (uint32_t)std::min<uint64_t>(nb, passes_left);
        if (nb == 0) return fail(FORK_E_NOT_CONVERGED, "max_passes reached with work pending");
        if (o.profile && c->pev.size() < 2 * nb) {
            size_t old = c->pev.size();
            c->pev.resize(2 * nb, nullptr);
            for (size_t k = old; k < c->pev.size(); ++k) HIPCHK(hipEventCreate(&c->pev[k]));
        }
        for (uint32_t k = 0; k < nb; ++k) {
            HIPCHK(fk::launch_gsummaries(g, G, B, pc, s));
            if (pc.sched == fk::S_LEARNED)
                HIPCHK(fk::launch_mlp_score(g, B, c->d_mlp, c->d_score, nullptr, c->d_gstat, 0, s));
            HIPCHK(fk::launch_select(g, B, pc, s));
            HIPCHK(fk::launch_gworklist(B, G, pc, s));
            if (o.profile) HIPCHK(hipEventRecord(c->pev[2 * k], s));
            HIPCHK(fk::launch_gprocess(g, G, B, pc, blocks, gnt, s));
            if (o.profile) HIPCHK(hipEventRecord(c->pev[2 * k + 1], s));
        }
        if (passes_left != ~0ull) passes_left -= nb;
        HIPCHK(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(fk::Ctl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (o.profile) {
            for (uint32_t k = 0; k < nb; ++k) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, c->pev[2 * k], c->pev[2 * k + 1]));
                c->stats.process_ms += ms;
            }
            c->stats.process_launches += nb;
        }
        const fk::Ctl& h = *c->h_ctl;
        if (h.err) return fail(FORK_E_DEVICE, "device error flags 0x%x", h.err);
        if (h.pending_parts == 0) break;
        batch = std::min<uint32_t>(batch * 2, 64);
    }
    // the last wave's vectors stay for fetch, sweeps and BC: transpose them to
    // the per-query layout; earlier waves leave only digests, taken from the rows
    if (keep_vectors) HIPCHK(fk::launch_gout(G, c->nv, c->d_state, c->d_qoff, c->d_lq, s));
    HIPCHK(hipEventRecord(c->ev[2], s));
    HIPCHK(hipStreamSynchronize(s));
    float t_init = 0, t_run = 0;
    hipEventElapsedTime(&t_init, c->ev[0], c->ev[1]);
    hipEventElapsedTime(&t_run, c->ev[1], c->ev[2]);
    c->resQ = Q;
    c->res_grouped = !keep_vectors;
    c->resG = G;
    c->dig_pending = true;
    const fk::Ctl& h = *c->h_ctl;
    fork_stats_t& st = c->stats;
    st.init_ms += t_init;
    st.run_ms += t_run;
    st.passes += h.pass;
    st.work_items += h.c_items;
    st.edges += h.c_edges;
    st.improved += h.c_improved;
    st.vertex_pushes += h.c_vpush;
    st.intra_edges += h.c_intra;
    st.selected_edges += h.c_sel_edges;
    st.ppr_edges += h.c_edges_ppr;
    st.ppr_vertex_pushes += h.c_vpush_ppr;
    st.activations += h.c_act;
    st.expansions += h.c_vtask;
    st.rounds += h.c_rounds;
    st.edge_tasks += h.c_tasks;
    for (int k = 0; k < 5; ++k) st.visit_ns[k] += 10ull * h.c_tphase[k];
    st.waves += 1;
    c->res_first = q0;
    c->res_n = nq;
    c->res_off.assign(qo.begin(), qo.end());
    return FORK_OK;
}

// fork_run, or with prepare = true fork_prepare: plan the waves and allocate
// their device buffers, then return without running.
static int run_impl(fork_ctx* c, const fork_run_opts* opts, bool prepare) {
    const auto t_entry = std::chrono::steady_clock::now();
    g_err[0] = 0;
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (c->queries.empty()) return fail(FORK_E_STATE, "no queries submitted");
    fork_run_opts o{};
    o.scheduler = FORK_SCHED_PRIORITY;
    if (opts) o = *opts;
    if (o.scheduler < 0 || o.scheduler > FORK_SCHED_MAXOPS) return fail(FORK_E_INVALID, "bad scheduler %d", o.scheduler);
    if (o.scheduler == FORK_SCHED_LEARNED && !o.mlp_weights) return fail(FORK_E_INVALID, "LEARNED needs mlp_weights");
    if (o.engine != FORK_ENGINE_BUFFERED && o.engine != FORK_ENGINE_GROUPED)
        return fail(FORK_E_INVALID, "bad engine %d", o.engine);
    const bool grouped = o.engine == FORK_ENGINE_GROUPED;
    if (grouped && (o.persistent || o.trace))
        return fail(FORK_E_INVALID, "the grouped engine runs per-pass kernels without traces (persistent = trace = 0)");
    if (grouped)
        for (const QueryRec& r : c->queries)
            if (r.l1 > 0.f) return fail(FORK_E_INVALID, "certified PPR (l1_target > 0) runs on the buffered engine");
    if (o.slice_slots && (o.slice_slots < 256 || o.slice_slots > 16384 || (o.slice_slots % 256)))
        return fail(FORK_E_INVALID, "slice_slots must be 0 or a multiple of 256 in [256, 16384], got %u", o.slice_slots);
    if (hipSetDevice(c->device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
    {
        // a table with at least half as many slots as the largest partition has
        // vertices saves no LDS: use the dense slice then
        uint32_t hs = (c->dense_ok && 2ull * o.slice_slots >= c->vpmax) ? 0u : o.slice_slots;
        if (!hs && !c->dense_ok) hs = fk::HS_AUTO;
        int rc = hs == c->hslots ? FORK_OK : set_slice(c, hs);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)o.stream;
    const uint32_t nq_total = (uint32_t)c->queries.size();
    for (const QueryRec& r : c->queries)
        if (r.l1 > 0.f && c->vpmax > fk::CERT_MAX_PART)
            return fail(FORK_E_INVALID, "certified PPR (l1_target > 0) needs partitions of at most %u vertices "
                        "(this graph's largest has %u; load it with partition_vertices <= %u)",
                        fk::CERT_MAX_PART, c->vpmax, fk::CERT_MAX_PART);
    // wave capacity from free device memory
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    // memory we already hold for state (and, for the grouped engine, its rows and pending sets)
    size_t reserve = (size_t)c->state_words_cap * 4 +
                     (grouped ? c->gstate_cap * 4 + c->gpend_cap * 8 + c->gbits_cap * 4 : 0);
    size_t budget = (fr + reserve) > ((size_t)2 << 30) ? (fr + reserve) - ((size_t)2 << 30) : 0;
    budget = (size_t)(budget * 0.9);
    // the batch's wave plan is fixed, while it still fits (the per-wave
    // buffers allocated since are small; memory taken by others is not)
    if (c->plan_budget && c->plan_budget <= budget + ((size_t)1 << 30)) budget = c->plan_budget;
    else c->plan_budget = budget;
    uint32_t cap_q = c->max_queries ? c->max_queries : nq_total;
    // per-query bytes beyond state: buckets (28 B per partition) + items; the
    // grouped engine holds its own copy of the state rows plus 8 B of pending
    // lanes and 4 B of pair summaries per vertex and group
    const size_t per_q_extra = (size_t)c->np * 28 + 64 + (grouped ? (size_t)c->nv * 8 / 64 + (size_t)c->np * 12 / 64 + 64 : 0);
    fk::PassCfg cfg{};
    cfg.sched = (uint32_t)o.scheduler;
    cfg.seed = (uint32_t)o.seed;
    cfg.mu = o.edge_budget_mu;
    // value windows / yield ranges (heuristic 2): SSSP in weight units, BFS in levels
    // Heuristic 2 (Section 5.1) with the paper's Delta-stepping guidance:
    // process in windows of about two mean edge weights, yield once a visit
    // has advanced `delta` past its first value (default: 64 mean weights).
    const double wm = c->wbytes ? c->wmean : 1.0;
    uint32_t delta = o.delta ? o.delta : (uint32_t)std::min(1.0e9, 64.0 * wm);
    cfg.win_sp = o.window ? o.window : std::max<uint32_t>(1u, (uint32_t)(2.0 * wm));
    cfg.yld_sp = delta;
    cfg.win_lv = 1;
    cfg.gate = o.window_mode == 0 ? 1u : 0u;
    cfg.yld_lv = o.delta ? std::max<uint32_t>(1u, (uint32_t)(o.delta / wm)) : 64u;
    if (o.scheduler == FORK_SCHED_LEARNED) {
        HIPCHK(hipMemcpyAsync(c->d_mlp, o.mlp_weights, fk::MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    }
    // waves: greedy in submit order under the memory budget
    std::vector<std::pair<uint32_t, uint32_t>> waves;
    for (uint32_t q0 = 0; q0 < nq_total;) {
        size_t bytes = 0;
        uint32_t n = 0;
        while (q0 + n < nq_total && n < cap_q) {
            size_t b = qwords(c, c->queries[q0 + n].type) * 4 * (grouped ? 2 : 1) + per_q_extra;
            if (n > 0 && bytes + b > budget) break;
            bytes += b;
            ++n;
        }
        if (bytes > budget) return fail(FORK_E_NOMEM, "one query's state does not fit in device memory");
        waves.push_back({q0, n});
        q0 += n;
    }
    // partitions per pass: a fixed count if asked for, else as many as it
    // takes to queue items_per_pass work items (default: 16 per workgroup slot)
    const uint32_t slots = (uint32_t)std::max(1, c->num_cu * c->blocks_per_cu);
    cfg.kmax = o.parts_per_pass ? std::min<uint32_t>(o.parts_per_pass, c->np) : c->np;
    cfg.target_items = o.parts_per_pass ? 0u : (o.items_per_pass ? o.items_per_pass : 16u * slots);
    if (grouped) {
        int rc = reserve_groups(c, waves, cfg.kmax);
        if (rc) return rc;
    } else if (prepare) {
        size_t words = 0;
        uint32_t nmax = 0;
        for (const auto& w : waves) {
            size_t ww = 0;
            for (uint32_t i = 0; i < w.second; ++i) ww += qwords(c, c->queries[w.first + i].type);
            words = std::max(words, ww);
            nmax = std::max(nmax, w.second);
        }
        int rc = ensure_wave(c, nmax, words, cfg.kmax);
        if (rc) return rc;
    }
    if (prepare) {
        HIPCHK(hipDeviceSynchronize());
        return FORK_OK;
    }
    c->stats = fork_stats_t{};
    c->stats.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_entry).count();
    c->spill_refused = false;
    c->trace.clear();
    if (o.trace && o.persistent) return fail(FORK_E_INVALID, "trace runs use the per-pass kernels (persistent = 0)");
    c->stats.num_partitions = c->np;
    c->stats.weight_bytes = (uint32_t)c->wbytes;
    c->digests.assign(nq_total, fork_digest{});
    c->res_n = 0;
    c->dig_pending = false;
    uint64_t passes_left = o.max_passes ? o.max_passes : ~0ull;
    // A wave whose pending operations overflow the pool is split in two and
    // re-run (state is re-initialised per wave, so a retry is exact).
    uint32_t wave_cap = 0;
    for (size_t wi = 0; wi < waves.size(); ++wi) {
        uint32_t q0 = waves[wi].first, n = waves[wi].second;
        if (wave_cap && n > wave_cap) {
            waves.insert(waves.begin() + wi + 1, {q0 + wave_cap, n - wave_cap});
            n = waves[wi].second = wave_cap;
        }
        uint64_t saved = passes_left;
        fork_stats_t saved_st = c->stats;
        int rc = grouped ? run_wave_group(c, q0, n, o, s, cfg, passes_left, wi + 1 == waves.size())
                         : run_wave(c, q0, n, o, s, cfg, passes_left, false);
        if (rc == FORK_OK && o.trace) {
            // traced re-run: the final state of the first run marks useful work
            size_t words = c->state_words_cap;
            if (words > c->final_words) {
                hipFree(c->d_final);
                c->d_final = nullptr;
                c->final_words = 0;
                if ((rc = dalloc(&c->d_final, words))) return rc;
                c->final_words = words;
            }
            HIPCHK(hipMemcpyAsync(c->d_final, c->d_state, words * 4, hipMemcpyDeviceToDevice, s));
            c->stats = saved_st;
            uint64_t pl = ~0ull;
            rc = run_wave(c, q0, n, o, s, cfg, pl, true);
        }
        if (rc == FORK_E_CAPACITY && n > 1 && !c->spill_refused) {
            passes_left = saved;
            c->stats = saved_st;
            wave_cap = n / 2;
            waves[wi].second = wave_cap;
            waves.insert(waves.begin() + wi + 1, {q0 + wave_cap, n - wave_cap});
            --wi;
            continue;
        }
        if (rc) return rc;
        if (wi + 1 < waves.size() && (rc = wave_digest(c, s))) return rc;  // the next wave reuses the state
    }
    c->ran = true;
    return FORK_OK;
}

extern "C" int fork_run(fork_ctx* c, const fork_run_opts* opts) {
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = run_impl(c, opts, false);
    if (c && rc == FORK_OK)
        c->stats.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

extern "C" int fork_prepare(fork_ctx* c, const fork_run_opts* opts) { return run_impl(c, opts, true); }

extern "C" int fork_fetch(fork_ctx* c, uint32_t qid, int field, void* dst, uint64_t dst_bytes, int dst_on_device) {
    g_err[0] = 0;
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (!dst) return fail(FORK_E_INVALID, "dst is NULL");
    if (qid >= c->queries.size()) return fail(FORK_E_INVALID, "query id %u out of range", qid);
    if (!c->ran) return fail(FORK_E_STATE, "query %u has not run", qid);
    const uint32_t type = c->queries[qid].type;
    if (field == FORK_FIELD_DIGEST) {
        if (dst_bytes < sizeof(fork_digest)) return fail(FORK_E_INVALID, "dst too small");
        if (c->dig_pending && qid >= c->res_first && qid < c->res_first + c->res_n) {
            if (hipSetDevice(c->device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
            HIPCHK(hipDeviceSynchronize());
            int rc = wave_digest(c, nullptr);
            if (rc) return rc;
        }
        if (dst_on_device) HIPCHK(hipMemcpy(dst, &c->digests[qid], sizeof(fork_digest), hipMemcpyHostToDevice));
        else memcpy(dst, &c->digests[qid], sizeof(fork_digest));
        return FORK_OK;
    }
    if (field == FORK_FIELD_VALUE && type == FORK_PPR) return fail(FORK_E_INVALID, "VALUE field needs SSSP/BFS");
    if ((field == FORK_FIELD_P || field == FORK_FIELD_R) && type != FORK_PPR)
        return fail(FORK_E_INVALID, "P/R fields need PPR");
    if (field < 0 || field > FORK_FIELD_DIGEST) return fail(FORK_E_INVALID, "bad field %d", field);
    if (qid < c->res_first || qid >= c->res_first + c->res_n)
        return fail(FORK_E_STATE, "query %u is not resident (only the last wave keeps vectors)", qid);
    if (dst_bytes < (uint64_t)c->nv * 4) return fail(FORK_E_INVALID, "dst too small");
    if (hipSetDevice(c->device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
    const uint32_t* src = c->d_state + c->res_off[qid - c->res_first] + (field == FORK_FIELD_R ? c->nv : 0);
    if (c->d_pos) {
        // back to the caller's numbering
        uint32_t* g = (uint32_t*)dst;
        if (!dst_on_device) {
            if (!c->d_gather) {
                int rc = dalloc(&c->d_gather, c->nv);
                if (rc) return rc;
            }
            g = c->d_gather;
        }
        HIPCHK(fk::launch_gather(src, c->d_pos, g, c->nv, nullptr));
        if (dst_on_device) HIPCHK(hipDeviceSynchronize());
        else HIPCHK(hipMemcpy(dst, g, (size_t)c->nv * 4, hipMemcpyDeviceToHost));
        return FORK_OK;
    }
    HIPCHK(hipMemcpy(dst, src, (size_t)c->nv * 4, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return FORK_OK;
}

// Reverse adjacency (in-edges) and d(v) = out + in degree, on the device.
static int build_reverse(fork_ctx* c) {
    if (c->d_sdeg) return FORK_OK;
    int rc;
    uint32_t* indeg = nullptr;
    if ((rc = dalloc(&indeg, c->nv))) return rc;
    std::vector<uint32_t> h(c->nv);
    hipError_t e = hipMemset(indeg, 0, (size_t)c->nv * 4);
    if (e == hipSuccess) e = fk::launch_indeg(c->d_col, c->ne, indeg, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h.data(), indeg, (size_t)c->nv * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { hipFree(indeg); return fail(FORK_E_DEVICE, "in-degrees: %s", hipGetErrorString(e)); }
    std::vector<uint32_t> rrow(c->nv + 1, 0);
    for (uint32_t v = 0; v < c->nv; ++v) rrow[v + 1] = rrow[v] + h[v];
    if ((rc = dalloc(&c->d_rrow, c->nv + 1)) || (rc = dalloc(&c->d_rcol, c->ne)) || (rc = dalloc(&c->d_sdeg, c->nv)) ||
        (rc = dalloc(&c->d_reid, c->ne))) {
        hipFree(indeg);
        hipFree(c->d_rrow); hipFree(c->d_rcol); hipFree(c->d_sdeg); hipFree(c->d_reid);
        c->d_rrow = c->d_rcol = c->d_sdeg = c->d_reid = nullptr;
        return rc;
    }
    e = hipMemcpy(c->d_rrow, rrow.data(), (c->nv + 1ull) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(indeg, 0, (size_t)c->nv * 4);  // reused as the fill cursor
    if (e == hipSuccess)
        e = fk::launch_rfill(c->d_rowptr, c->d_col, c->nv, c->d_rrow, indeg, c->d_rcol, c->d_reid, nullptr);
    if (e == hipSuccess) e = fk::launch_sdeg(c->d_rowptr, c->d_rrow, c->nv, c->d_sdeg, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    hipFree(indeg);
    if (e != hipSuccess) {
        hipFree(c->d_rrow); hipFree(c->d_rcol); hipFree(c->d_sdeg); hipFree(c->d_reid);
        c->d_rrow = c->d_rcol = c->d_sdeg = c->d_reid = nullptr;
        return fail(FORK_E_DEVICE, "reverse adjacency: %s", hipGetErrorString(e));
    }
    return FORK_OK;
}

extern "C" int fork_sweep(fork_ctx* c, uint32_t first, uint32_t n, uint32_t max_size, fork_sweep_t* out) {
    g_err[0] = 0;
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (!out && n) return fail(FORK_E_INVALID, "out is NULL");
    if (max_size < 1 || max_size > FORK_SWEEP_MAX) return fail(FORK_E_INVALID, "max_size must be in [1, %d]", FORK_SWEEP_MAX);
    if ((uint64_t)first + n > c->queries.size()) return fail(FORK_E_INVALID, "query range out of bounds");
    if (sizeof(fork_sweep_t) != fk::sweep_out_bytes()) return fail(FORK_E_DEVICE, "sweep record layout mismatch");
    if (n == 0) return FORK_OK;
    if (!c->ran) return fail(FORK_E_STATE, "queries have not run");
    for (uint32_t i = first; i < first + n; ++i) {
        if (c->queries[i].type != FORK_PPR) return fail(FORK_E_INVALID, "query %u is not PPR", i);
        if (i < c->res_first || i >= c->res_first + c->res_n)
            return fail(FORK_E_STATE, "query %u is not resident (only the last wave keeps vectors)", i);
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
    int rc = build_reverse(c);
    if (rc) return rc;
    std::vector<unsigned long long> off(n);
    for (uint32_t i = 0; i < n; ++i) off[i] = c->res_off[first + i - c->res_first];
    unsigned long long* d_off = nullptr;
    void* d_out = nullptr;
    if ((rc = dalloc(&d_off, n))) return rc;
    if (hipMalloc(&d_out, (size_t)n * sizeof(fork_sweep_t)) != hipSuccess) {
        hipFree(d_off);
        return fail(FORK_E_NOMEM, "hipMalloc for sweep results failed");
    }
    hipError_t e = hipMemcpy(d_off, off.data(), (size_t)n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = fk::launch_sweep(c->d_state, d_off, n, c->nv, c->d_rowptr, c->d_col, c->d_rrow, c->d_rcol, c->d_sdeg,
                             2ull * c->ne, max_size, d_out, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d_out, (size_t)n * sizeof(fork_sweep_t), hipMemcpyDeviceToHost);
    hipFree(d_off);
    hipFree(d_out);
    if (e != hipSuccess) return fail(FORK_E_DEVICE, "sweep: %s", hipGetErrorString(e));
    return FORK_OK;
}

extern "C" int fork_bc(fork_ctx* c, uint32_t first, uint32_t n, double* out) {
    g_err[0] = 0;
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    if (!out) return fail(FORK_E_INVALID, "out is NULL");
    if ((uint64_t)first + n > c->queries.size()) return fail(FORK_E_INVALID, "query range out of bounds");
    if (n && !c->ran) return fail(FORK_E_STATE, "queries have not run");
    for (uint32_t i = first; i < first + n; ++i) {
        if (c->queries[i].type == FORK_PPR) return fail(FORK_E_INVALID, "query %u is PPR (BC takes BFS or SSSP)", i);
        if (i < c->res_first || i >= c->res_first + c->res_n)
            return fail(FORK_E_STATE, "query %u is not resident (only the last wave keeps vectors)", i);
    }
    if (n == 0) {
        memset(out, 0, (size_t)c->nv * sizeof(double));
        return FORK_OK;
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(FORK_E_DEVICE, "hipSetDevice failed");
    int rc = build_reverse(c);
    if (rc) return rc;
    std::vector<unsigned long long> off(n);
    std::vector<uint32_t> src(n), qw(n);
    for (uint32_t i = 0; i < n; ++i) {
        off[i] = c->res_off[first + i - c->res_first];
        src[i] = c->queries[first + i].src;  // internal id
        qw[i] = c->queries[first + i].type == FORK_SSSP && c->wbytes ? 1u : 0u;  // SSSP on the graph's weights
    }
    const size_t nv = c->nv, lcap = fk::bc_level_cap() + 2ull;
    unsigned long long* d_off = nullptr;
    uint32_t *d_src = nullptr, *d_qw = nullptr, *d_order = nullptr, *d_ls = nullptr, *d_err = nullptr;
    double *d_lsig = nullptr, *d_delta = nullptr, *d_bc = nullptr;
    auto release = [&]() {
        hipFree(d_off); hipFree(d_src); hipFree(d_qw); hipFree(d_order); hipFree(d_ls); hipFree(d_err);
        hipFree(d_lsig); hipFree(d_delta); hipFree(d_bc);
    };
    if ((rc = dalloc(&d_off, n)) || (rc = dalloc(&d_src, n)) || (rc = dalloc(&d_qw, n)) ||
        (rc = dalloc(&d_order, (size_t)n * nv)) || (rc = dalloc(&d_ls, (size_t)n * lcap)) || (rc = dalloc(&d_err, 1)) ||
        (rc = dalloc(&d_lsig, (size_t)n * nv)) || (rc = dalloc(&d_delta, (size_t)n * nv)) || (rc = dalloc(&d_bc, nv))) {
        release();
        return rc;
    }
    std::vector<double> h(nv);
    uint32_t herr = 0;
    hipError_t e = hipMemcpy(d_off, off.data(), n * 8ull, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_src, src.data(), n * 4ull, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_qw, qw.data(), n * 4ull, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_bc, 0, nv * sizeof(double));
    if (e == hipSuccess) e = hipMemset(d_err, 0, 4);
    if (e == hipSuccess)
        e = fk::launch_bc(c->d_state, d_off, d_src, d_qw, n, c->nv, c->d_rowptr, c->d_col, c->d_w, (uint32_t)c->wbytes,
                          c->d_rrow, c->d_rcol, c->d_reid, d_order, d_ls, d_lsig, d_delta, d_bc, d_err, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h.data(), d_bc, nv * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&herr, d_err, 4, hipMemcpyDeviceToHost);
    release();
    if (e != hipSuccess) return fail(FORK_E_DEVICE, "bc: %s", hipGetErrorString(e));
    if (herr)
        return fail(FORK_E_CAPACITY, "a query's BFS levels or SSSP distances reach %u or more (the value range "
                    "fork_bc sorts by)", fk::bc_level_cap());
    for (size_t v = 0; v < nv; ++v)
        if (!std::isfinite(h[v])) return fail(FORK_E_DEVICE, "bc: non-finite dependency at vertex %zu", v);
    if (c->h_pos.empty()) memcpy(out, h.data(), nv * sizeof(double));
    else for (size_t v = 0; v < nv; ++v) out[v] = h[c->h_pos[v]];
    return FORK_OK;
}

extern "C" int fork_trace(fork_ctx* c, float* dst, uint64_t cap, uint64_t* n) {
    if (!c) return fail(FORK_E_INVALID, "ctx is NULL");
    const uint64_t avail = c->trace.size() / FORK_TRACE_WIDTH;
    if (n) *n = avail;
    if (dst && cap) memcpy(dst, c->trace.data(), std::min(cap, avail) * FORK_TRACE_WIDTH * sizeof(float));
    return FORK_OK;
}

extern "C" int fork_stats(fork_ctx* c, void* dst, uint64_t dst_bytes) {
    if (!c || !dst) return fail(FORK_E_INVALID, "NULL argument");
    if (dst_bytes < sizeof(fork_stats_t)) return fail(FORK_E_INVALID, "dst too small");
    memcpy(dst, &c->stats, sizeof(fork_stats_t));
    return FORK_OK;
}

// ------------------------------------------------------------ learned scheduler: MLP entry points
namespace {
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) hipFree(p); }
};
int dev_upload(DevBuf& b, const void* h, size_t bytes) {
    if (hipMalloc(&b.p, bytes ? bytes : 4) != hipSuccess) return fail(FORK_E_NOMEM, "hipMalloc(%zu) failed", bytes);
    if (h && bytes && hipMemcpy(b.p, h, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FORK_E_DEVICE, "hipMemcpy to device failed");
    return FORK_OK;
}
int mlp_check(const float* theta, const float* x, uint64_t n) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(FORK_E_DEVICE, "no HIP device");
    if (!theta || (n && !x)) return fail(FORK_E_INVALID, "NULL argument");
    if (n > 0xffffffffull) return fail(FORK_E_INVALID, "too many samples");
    return FORK_OK;
}
}  // namespace

extern "C" int fork_mlp_forward(const float* theta, const float* x, uint64_t n, float* y) {
    g_err[0] = 0;
    int rc = mlp_check(theta, x, n);
    if (rc) return rc;
    if (!y) return fail(FORK_E_INVALID, "y is NULL");
    DevBuf dt, dx, dy;
    if ((rc = dev_upload(dt, theta, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dx, x, n * fk::MLP_IN * 4))) return rc;
    if ((rc = dev_upload(dy, nullptr, n * 4))) return rc;
    if (n) HIPCHK(fk::launch_mlp_forward((float*)dt.p, (float*)dx.p, (uint32_t)n, (float*)dy.p, 0));
    HIPCHK(hipMemcpy(y, dy.p, n * 4, hipMemcpyDeviceToHost));
    return FORK_OK;
}

extern "C" int fork_mlp_grad(const float* theta, const float* x, const float* t, uint64_t n, float* grad,
                             float* loss) {
    g_err[0] = 0;
    int rc = mlp_check(theta, x, n);
    if (rc) return rc;
    if (!t || !grad || !loss || n == 0) return fail(FORK_E_INVALID, "NULL argument or no samples");
    DevBuf dt, dx, dtg, dg, dl;
    if ((rc = dev_upload(dt, theta, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dx, x, n * fk::MLP_IN * 4))) return rc;
    if ((rc = dev_upload(dtg, t, n * 4))) return rc;
    if ((rc = dev_upload(dg, nullptr, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dl, nullptr, 4))) return rc;
    HIPCHK(hipMemset(dg.p, 0, fk::MLP_NPARAM * 4));
    HIPCHK(hipMemset(dl.p, 0, 4));
    HIPCHK(fk::launch_mlp_grad((float*)dt.p, (float*)dx.p, (float*)dtg.p, nullptr, (uint32_t)n, (float*)dg.p,
                               (float*)dl.p, 0));
    HIPCHK(hipMemcpy(grad, dg.p, fk::MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(loss, dl.p, 4, hipMemcpyDeviceToHost));
    return FORK_OK;
}

extern "C" int fork_mlp_train(float* theta, const float* x, const float* t, uint64_t n, uint32_t steps,
                              uint32_t batch, float lr, uint64_t seed, float* losses) {
    g_err[0] = 0;
    int rc = mlp_check(theta, x, n);
    if (rc) return rc;
    if (!t || n == 0 || batch == 0 || !(lr > 0.f)) return fail(FORK_E_INVALID, "bad training arguments");
    batch = (uint32_t)std::min<uint64_t>(batch, n);
    DevBuf dt, dx, dtg, dg, dl, dm, dv, di;
    if ((rc = dev_upload(dt, theta, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dx, x, n * fk::MLP_IN * 4))) return rc;
    if ((rc = dev_upload(dtg, t, n * 4))) return rc;
    if ((rc = dev_upload(dg, nullptr, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dl, nullptr, (size_t)std::max(1u, steps) * 4))) return rc;
    if ((rc = dev_upload(dm, nullptr, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(dv, nullptr, fk::MLP_NPARAM * 4))) return rc;
    if ((rc = dev_upload(di, nullptr, n * 4))) return rc;
    HIPCHK(hipMemset(dm.p, 0, fk::MLP_NPARAM * 4));
    HIPCHK(hipMemset(dv.p, 0, fk::MLP_NPARAM * 4));
    HIPCHK(hipMemset(dl.p, 0, (size_t)std::max(1u, steps) * 4));
    // epochs of a seeded permutation (Fisher-Yates with a SplitMix64 stream)
    std::vector<uint32_t> perm(n);
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    unsigned long long st = seed;
    uint64_t pos = n;
    for (uint32_t k = 1; k <= steps; ++k) {
        if (pos + batch > n) {
            for (uint64_t i = n - 1; i > 0; --i) {
                st += 0x9E3779B97F4A7C15ull;
                uint64_t j = fk::mix64(st) % (i + 1);
                std::swap(perm[i], perm[j]);
            }
            HIPCHK(hipMemcpy(di.p, perm.data(), n * 4, hipMemcpyHostToDevice));
            pos = 0;
        }
        HIPCHK(hipMemsetAsync(dg.p, 0, fk::MLP_NPARAM * 4, 0));
        HIPCHK(fk::launch_mlp_grad((float*)dt.p, (float*)dx.p, (float*)dtg.p, (uint32_t*)di.p + pos, batch,
                                   (float*)dg.p, (float*)dl.p + (k - 1), 0));
        HIPCHK(fk::launch_adam((float*)dt.p, (float*)dg.p, (float*)dm.p, (float*)dv.p, k, lr, 0));
        pos += batch;
    }
    HIPCHK(hipMemcpy(theta, dt.p, fk::MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    if (losses && steps) HIPCHK(hipMemcpy(losses, dl.p, steps * 4ull, hipMemcpyDeviceToHost));
    return FORK_OK;
}

// ------------------------------------------------------------ training without allocation
// The scratch array's address, looked up once per device with that device
// current (each GPU holds its own copy of the array).
static std::mutex g_scr_m;
static void* g_scr[64];

extern "C" int fork_mlp_train_noalloc(float* theta, const float* x, const float* t, uint64_t n, uint32_t steps,
                                      uint32_t batch, float lr, uint64_t seed, float* losses, void* stream) {
    g_err[0] = 0;
    if (!theta || !x || !t) return fail(FORK_E_INVALID, "theta, x and t must be device pointers");
    if (n == 0 || n > fk::train_nmax())
        return fail(FORK_E_INVALID, "n = %llu samples; the allocation-free trainer takes 1..%u",
                    (unsigned long long)n, fk::train_nmax());
    if (batch == 0 || !(lr > 0.f)) return fail(FORK_E_INVALID, "bad training arguments");
    if (batch > n) batch = (uint32_t)n;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FORK_E_DEVICE, "device ordinal %d out of range", dev);
    void* scr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scr_m);
        if (!g_scr[dev]) {
            void* p = nullptr;
            HIPCHK(fk::train_scratch_address(&p));
            if (!p) return fail(FORK_E_DEVICE, "no device address for the training scratch");
            HIPCHK(fk::train_prepare());
            g_scr[dev] = p;
        }
        scr = g_scr[dev];
    }
    HIPCHK(fk::launch_train_noalloc((uint32_t*)scr, theta, x, t, (uint32_t)n, steps, batch, lr, seed, losses,
                                    (hipStream_t)stream));
    return FORK_OK;
}
