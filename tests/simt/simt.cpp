// Host execution engine behind the CPU stand-in for the HIP runtime (see
// hip/hip_runtime.h).  Test infrastructure.
#include "hip/hip_runtime.h"

#include <dlfcn.h>
#include <execinfo.h>
#include <signal.h>
#include <sys/mman.h>
#include <ucontext.h>
#include <unistd.h>
#include <sched.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#ifdef __SANITIZE_ADDRESS__
extern "C" void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
extern "C" void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old);
#endif

// Dynamic LDS of the kernels (extern __shared__ arrays in namespace fk).
namespace fk {
thread_local uint32_t dyn[160 * 1024 / 4];
}

// x86-64 context switch: save the callee-saved registers and the stack
// pointer of the current context in *from, resume the context at `to`.
extern "C" void simt_switch(void** from, void* to);
extern "C" void simt_trampoline();
asm(R"(
.text
.globl simt_switch
.type simt_switch,@function
simt_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size simt_switch, .-simt_switch
.globl simt_trampoline
.type simt_trampoline,@function
simt_trampoline:
    movq %r13, %rdi
    callq *%r12
    ud2
.size simt_trampoline, .-simt_trampoline
.section .note.GNU-stack,"",@progbits
.text
)");

namespace simt {
thread_local uint3 tl_thread, tl_block;
thread_local dim3 tl_bdim, tl_gdim;
thread_local uint32_t tl_lane_flat;

namespace {
enum St { RUN, WAVE, BAR, GRID, DONE };
struct Lane {
    void* sp = nullptr;
    char* stack = nullptr;
    int st = RUN;
    int op = 0, param = 0;
    uint64_t val = 0, res = 0;
};
constexpr size_t STACK = 256 * 1024;

struct Block {
    std::vector<Lane> lanes;
    void* sched_sp = nullptr;
    const void* sched_bottom = nullptr;
    size_t sched_size = 0;
    const std::function<void()>* body = nullptr;
    uint32_t cur = 0;
    std::mt19937_64 rng;
};
thread_local Block* tl_blk = nullptr;
struct Stacks {  // lane stacks, reused between the blocks of one thread
    std::vector<char*> v;
    ~Stacks() {
        for (char* p : v) munmap(p, STACK + 4096);
    }
};
thread_local Stacks tl_stacks;
thread_local std::mt19937_64 tl_rng(1);

int env_int(const char* k, int d) {
    const char* v = getenv(k);
    return v ? atoi(v) : d;
}
int g_yield_1_in = -1;
std::atomic<uint64_t> g_launch{0};

[[noreturn]] void die(const std::string& m) {
    fprintf(stderr, "[simt] fatal: %s\n", m.c_str());
    fflush(stderr);
    abort();
}

void to_sched(Block* b, bool finished) {
    Lane& L = b->lanes[b->cur];
#ifdef __SANITIZE_ADDRESS__
    void* fs = nullptr;
    __sanitizer_start_switch_fiber(finished ? nullptr : &fs, b->sched_bottom, b->sched_size);
#endif
    simt_switch(&L.sp, b->sched_sp);
#ifdef __SANITIZE_ADDRESS__
    __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
#endif
    (void)finished;
}

void lane_main(void*) {
    Block* b = tl_blk;
#ifdef __SANITIZE_ADDRESS__
    __sanitizer_finish_switch_fiber(nullptr, &b->sched_bottom, &b->sched_size);
#endif
    (*b->body)();
    b = tl_blk;
    b->lanes[b->cur].st = DONE;
    to_sched(b, true);
    die("finished lane resumed");
}

void resume(Block* b, uint32_t i) {
    b->cur = i;
    tl_lane_flat = i;
    tl_thread = uint3{i % tl_bdim.x, (i / tl_bdim.x) % tl_bdim.y, i / (tl_bdim.x * tl_bdim.y)};
    Lane& L = b->lanes[i];
#ifdef __SANITIZE_ADDRESS__
    void* fs = nullptr;
    __sanitizer_start_switch_fiber(&fs, L.stack, STACK);
#endif
    simt_switch(&b->sched_sp, L.sp);
#ifdef __SANITIZE_ADDRESS__
    __sanitizer_finish_switch_fiber(fs, &b->sched_bottom, &b->sched_size);
#endif
}

// ---- grid barrier across the workgroup threads of a cooperative launch
struct GridBar {
    std::mutex m;
    std::condition_variable cv;
    uint32_t n = 0, arrived = 0, exited = 0;
    uint64_t gen = 0;
    bool broken = false;
};
GridBar* g_bar = nullptr;

void grid_barrier_wait() {
    GridBar& G = *g_bar;
    std::unique_lock<std::mutex> lk(G.m);
    if (G.exited) G.broken = true;
    const uint64_t gen = G.gen;
    if (++G.arrived == G.n - G.exited) {
        G.arrived = 0;
        ++G.gen;
        G.cv.notify_all();
        return;
    }
    while (G.gen == gen && !G.broken) {
        G.cv.wait_for(lk, std::chrono::milliseconds(200));
        if (G.exited && G.arrived == G.n - G.exited) G.broken = true;
    }
    if (G.broken) {
        G.cv.notify_all();
        lk.unlock();
        die("grid barrier reached after a workgroup exited: on the GPU the grid would hang");
    }
}

void grid_block_exit() {
    if (!g_bar) return;
    std::lock_guard<std::mutex> lk(g_bar->m);
    ++g_bar->exited;
    g_bar->cv.notify_all();
}

void run_block(const std::function<void()>& body, uint32_t nthreads) {
    Block b;
    b.body = &body;
    b.lanes.resize(nthreads);
    while (tl_stacks.v.size() < nthreads) {
        // one guard page below each stack: an overflow faults instead of
        // overwriting the neighbouring lane
        char* s = (char*)mmap(nullptr, STACK + 4096, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                              -1, 0);
        if (s == (char*)MAP_FAILED) die("mmap of a lane stack failed");
        mprotect(s, 4096, PROT_NONE);
        tl_stacks.v.push_back(s);
    }
    for (uint32_t i = 0; i < nthreads; ++i) {
        Lane& L = b.lanes[i];
        L.stack = tl_stacks.v[i] + 4096;
        uint64_t* s = (uint64_t*)(L.stack + STACK - 16);
        *(--s) = (uint64_t)&simt_trampoline;  // return address of the first switch
        *(--s) = 0;                            // rbp
        *(--s) = 0;                            // rbx
        *(--s) = (uint64_t)&lane_main;         // r12: entry
        *(--s) = 0;                            // r13: argument
        *(--s) = 0;                            // r14
        *(--s) = 0;                            // r15
        L.sp = s;
        L.st = RUN;
    }
    tl_blk = &b;
    const uint32_t nw = (nthreads + 63) / 64;
    for (;;) {
        // run every runnable lane until it reaches a synchronisation point;
        // waves in a random order each round
        const uint32_t w0 = (uint32_t)(tl_rng() % nw);
        for (uint32_t k = 0; k < nw; ++k) {
            const uint32_t w = (w0 + k) % nw;
            for (uint32_t i = w * 64; i < std::min(nthreads, w * 64 + 64); ++i)
                if (b.lanes[i].st == RUN) resume(&b, i);
        }
        bool resolved = false;
        for (uint32_t w = 0; w < nw; ++w) {
            const uint32_t i0 = w * 64, i1 = std::min(nthreads, i0 + 64);
            uint32_t nwv = 0, nd = 0, op = 0;
            bool same = true;
            for (uint32_t i = i0; i < i1; ++i) {
                const Lane& L = b.lanes[i];
                if (L.st == WAVE) {
                    if (nwv && (uint32_t)L.op != op) same = false;
                    op = (uint32_t)L.op;
                    ++nwv;
                } else if (L.st == DONE) {
                    ++nd;
                }
            }
            if (!nwv || nwv + nd != i1 - i0) continue;
            if (!same) die("lanes of one wave wait at different cross-lane operations");
            uint64_t ballot = 0, first = 0;
            bool have_first = false;
            for (uint32_t i = i0; i < i1; ++i) {
                const Lane& L = b.lanes[i];
                if (L.st != WAVE) continue;
                if (!have_first) { first = L.val; have_first = true; }
                if (L.val) ballot |= 1ull << (i - i0);
            }
            for (uint32_t i = i0; i < i1; ++i) {
                Lane& L = b.lanes[i];
                if (L.st != WAVE) continue;
                const uint32_t l = i - i0;
                auto val_at = [&](uint32_t src) -> uint64_t {
                    if (src >= i1 - i0 || b.lanes[i0 + src].st != WAVE) return 0;
                    return b.lanes[i0 + src].val;
                };
                switch (L.op) {
                case 0: L.res = val_at((uint32_t)L.param & 63u); break;
                case 1: L.res = val_at(l ^ (uint32_t)L.param); break;
                case 2: L.res = l >= (uint32_t)L.param ? val_at(l - (uint32_t)L.param) : L.val; break;
                case 3: L.res = ballot; break;
                case 4: L.res = first; break;
                default: L.res = 0; break;
                }
            }
            for (uint32_t i = i0; i < i1; ++i)
                if (b.lanes[i].st == WAVE) b.lanes[i].st = RUN;
            resolved = true;
        }
        if (resolved) continue;
        uint32_t nbar = 0, ngrid = 0, nd = 0, nrun = 0;
        for (const Lane& L : b.lanes) {
            nbar += L.st == BAR;
            ngrid += L.st == GRID;
            nd += L.st == DONE;
            nrun += L.st == RUN;
        }
        if (nd == nthreads) break;
        if (nrun) continue;
        if (nbar && nbar + nd == nthreads) {
            for (Lane& L : b.lanes) if (L.st == BAR) L.st = RUN;
            continue;
        }
        if (ngrid && ngrid + nd == nthreads) {
            if (nd) die("grid barrier with exited lanes");
            if (!g_bar) die("grid barrier outside a cooperative launch");
            grid_barrier_wait();
            for (Lane& L : b.lanes) if (L.st == GRID) L.st = RUN;
            continue;
        }
        std::string m = "deadlock in a workgroup: lane states";
        for (uint32_t i = 0; i < nthreads; i += 16) m += " " + std::to_string(b.lanes[i].st);
        die(m);
    }
    tl_blk = nullptr;
}
}  // namespace

void maybe_yield() {
    if (g_yield_1_in < 0) g_yield_1_in = env_int("SIMT_YIELD", 16);
    if (g_yield_1_in > 0 && tl_rng() % (uint64_t)g_yield_1_in == 0) sched_yield();
}

static void block_sync_point(int st) {
    Block* b = tl_blk;
    if (!b) die("synchronisation outside a kernel");
    b->lanes[b->cur].st = st;
    to_sched(b, false);
}
void syncthreads() { block_sync_point(BAR); }
void grid_sync() {
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
    block_sync_point(GRID);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);
}
uint64_t wave_op(int op, uint64_t v, int param) {
    Block* b = tl_blk;
    if (!b) die("cross-lane operation outside a kernel");
    const uint32_t me = b->cur;
    Lane& L = b->lanes[me];
    L.op = op;
    L.val = v;
    L.param = param;
    L.st = WAVE;
    to_sched(b, false);
    return tl_blk->lanes[me].res;
}
void wave_barrier() { (void)wave_op(5, 0, 0); }

thread_local const char* tl_kernel = "";

void on_fault(int sig, siginfo_t* si, void* ucv) {
    char buf[320];
    ucontext_t* uc = (ucontext_t*)ucv;
    const uint64_t rip = (uint64_t)uc->uc_mcontext.gregs[REG_RIP], rsp = (uint64_t)uc->uc_mcontext.gregs[REG_RSP];
    int n = snprintf(buf, sizeof buf, "[simt] signal %d at address %p in kernel %s block %u lane %u rip %p [rsp] %p\n",
                     sig, si->si_addr, tl_kernel, tl_block.x, tl_lane_flat, (void*)rip, *(void**)rsp);
    (void)!write(2, buf, n);
    Dl_info di;
    if (dladdr(*(void**)rsp, &di) && di.dli_fname) {
        n = snprintf(buf, sizeof buf, "[simt]   caller %s+0x%lx\n", di.dli_fname,
                     (unsigned long)((char*)*(void**)rsp - (char*)di.dli_fbase));
        (void)!write(2, buf, n);
    }
    void* bt[64];
    int k = backtrace(bt, 64);
    backtrace_symbols_fd(bt, k, 2);
    _exit(128 + sig);
}

hipError_t run_grid(const char* name, dim3 grid, dim3 block, size_t dyn, bool coop, const std::function<void()>& body) {
    static bool handler = false;
    if (!handler && getenv("SIMT_SEGV")) {
        handler = true;
        static char altstack[65536];
        stack_t ss{};
        ss.ss_sp = altstack;
        ss.ss_size = sizeof altstack;
        sigaltstack(&ss, nullptr);
        struct sigaction sa{};
        sa.sa_sigaction = on_fault;
        sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
        sigaction(SIGSEGV, &sa, nullptr);
        sigaction(SIGBUS, &sa, nullptr);
    }
    if (dyn > sizeof(fk::dyn)) die("dynamic LDS request above 160 KB");
    const uint32_t nb = grid.x * grid.y * grid.z, nt = block.x * block.y * block.z;
    if (nb == 0) return hipSuccess;
    if (nt == 0 || nt > 1024) die("bad workgroup size");
    const uint64_t launch = g_launch.fetch_add(1);
    const uint64_t seed = (uint64_t)env_int("SIMT_SEED", 1);
    uint32_t nthr = coop ? nb : std::min<uint32_t>(nb, (uint32_t)std::max(1, env_int("SIMT_THREADS", 8)));
    GridBar bar;
    bar.n = nb;
    if (coop) g_bar = &bar;
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < nthr; ++t) {
        th.emplace_back([&, t]() {
            tl_rng.seed(seed * 0x9E3779B97F4A7C15ull + launch * 1000003ull + t);
            tl_gdim = grid;
            tl_bdim = block;
            tl_kernel = name;
            if (getenv("SIMT_SEGV")) {
                static thread_local char alt[65536];
                stack_t ss{};
                ss.ss_sp = alt;
                ss.ss_size = sizeof alt;
                sigaltstack(&ss, nullptr);
            }
            for (uint32_t bi = t; bi < nb; bi += nthr) {
                tl_block = uint3{bi % grid.x, (bi / grid.x) % grid.y, bi / (grid.x * grid.y)};
                run_block(body, nt);
                if (coop) grid_block_exit();
            }
        });
    }
    for (auto& x : th) x.join();
    g_bar = nullptr;
    return hipSuccess;
}
}  // namespace simt

// ------------------------------------------------------------ host API
namespace {
std::mutex g_mem_m;
size_t g_mem_used = 0;
std::vector<std::pair<void*, size_t>> g_allocs;
int g_last = hipSuccess;
}  // namespace
struct simt_event {
    std::chrono::steady_clock::time_point t;
};

namespace { unsigned long long g_alloc_calls = 0; }
// allocation counters for tests: calls so far and bytes held
extern "C" unsigned long long simt_alloc_calls() { return g_alloc_calls; }
extern "C" unsigned long long simt_mem_used() { return g_mem_used; }

hipError_t hipMalloc(void** p, size_t n) {
    size_t cap = (size_t)simt::env_int("SIMT_MEM_MB", 4096) << 20;
    std::lock_guard<std::mutex> lk(g_mem_m);
    ++g_alloc_calls;
    if (n == 0) n = 1;
    if (g_mem_used + n > cap) { *p = nullptr; return g_last = hipErrorOutOfMemory; }
    size_t sz = (n + 255) & ~(size_t)255;
    void* q = aligned_alloc(256, sz);
    if (!q) { *p = nullptr; return g_last = hipErrorOutOfMemory; }
    // device memory starts with arbitrary contents
    memset(q, 0xcd, std::min<size_t>(sz, (size_t)64 << 20));
    g_mem_used += sz;
    g_allocs.push_back({q, sz});
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_mem_m);
    for (size_t i = 0; i < g_allocs.size(); ++i)
        if (g_allocs[i].first == p) {
            g_mem_used -= g_allocs[i].second;
            g_allocs.erase(g_allocs.begin() + i);
            free(p);
            return hipSuccess;
        }
    return g_last = hipErrorInvalidValue;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
    *p = aligned_alloc(256, (n + 255) & ~(size_t)255);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemset(void* d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetD32Async(hipDeviceptr_t d, int v, size_t n, hipStream_t) {
    uint32_t* p = (uint32_t*)d;
    for (size_t i = 0; i < n; ++i) p[i] = (uint32_t)v;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { int e = g_last; g_last = hipSuccess; return e; }
const char* hipGetErrorString(hipError_t e) {
    switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorInvalidValue: return "hipErrorInvalidValue";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    default: return "hipError(simt)";
    }
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    memset(p, 0, sizeof(*p));
    snprintf(p->name, sizeof p->name, "simt-cpu");
    snprintf(p->gcnArchName, sizeof p->gcnArchName, "gfx950-simt");
    p->totalGlobalMem = (size_t)simt::env_int("SIMT_MEM_MB", 4096) << 20;
    p->sharedMemPerBlock = 160 * 1024;
    p->multiProcessorCount = simt::env_int("SIMT_NUM_CU", 4);
    p->maxThreadsPerBlock = 1024;
    p->warpSize = 64;
    return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* fr, size_t* tot) {
    std::lock_guard<std::mutex> lk(g_mem_m);
    *tot = (size_t)simt::env_int("SIMT_MEM_MB", 4096) << 20;
    *fr = *tot > g_mem_used ? *tot - g_mem_used : 0;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { *e = new simt_event(); (*e)->t = std::chrono::steady_clock::now(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = std::chrono::steady_clock::now(); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int v) {
    return v <= 160 * 1024 ? hipSuccess : (g_last = hipErrorInvalidValue);
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t dyn) {
    *n = dyn <= 160 * 1024 ? std::max(1, simt::env_int("SIMT_BLOCKS_PER_CU", 2)) : 0;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; return hipSuccess; }
