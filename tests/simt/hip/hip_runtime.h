// CPU stand-in for <hip/hip_runtime.h>: lets the library's HIP sources be
// compiled by g++ and run on the host, for tests that need to watch the
// kernels' shared data structures (test infrastructure, never the product).
//
// Execution model (simt.cpp): every workgroup of a launch runs on its own OS
// thread, so workgroups really run concurrently and their device-scope
// atomics really race; inside a workgroup every lane is a coroutine, and the
// lanes switch only at the points where a GPU wave or workgroup synchronises
// (lane shuffles, ballots, __syncthreads, grid barriers).  A wave's lanes
// therefore act together on every cross-lane operation, as on the GPU.
// Global memory is host memory from malloc (AddressSanitizer sees every
// buffer's bounds); __shared__ variables are thread_local, one copy per
// workgroup thread.  Not modelled: the GPU's weak ordering of plain stores
// between workgroups (x86 keeps them in program order).
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdio.h>
#include <time.h>
#include <math.h>
#include <cmath>
#include <algorithm>
#include <functional>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ thread_local
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct uint3 { uint32_t x, y, z; };
struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return uint4{x, y, z, w}; }
inline float2 make_float2(float x, float y) { return float2{x, y}; }

namespace simt {
extern thread_local uint3 tl_thread, tl_block;
extern thread_local dim3 tl_bdim, tl_gdim;
extern thread_local uint32_t tl_lane_flat;

// cross-lane and barrier primitives (simt.cpp)
void syncthreads();
void grid_sync();
void wave_barrier();
uint64_t wave_op(int op, uint64_t v, int param);  // op: 0 shfl idx, 1 xor, 2 up, 3 ballot, 4 first lane
void maybe_yield();                                // random interleaving point at device atomics

template <class T> inline uint64_t to_u64(T v) { uint64_t u = 0; memcpy(&u, &v, sizeof(T)); return u; }
template <class T> inline T from_u64(uint64_t u) { T v; memcpy(&v, &u, sizeof(T)); return v; }
inline uint32_t lane() { return tl_lane_flat & 63u; }

template <class T> inline T atomic_add(T* p, T v) {
    maybe_yield();
    if constexpr (std::is_floating_point<T>::value) {
        using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
        U* q = (U*)p;
        U old = __atomic_load_n(q, __ATOMIC_SEQ_CST);
        for (;;) {
            T o; memcpy(&o, &old, sizeof(T));
            T n = o + v;
            U nu; memcpy(&nu, &n, sizeof(T));
            if (__atomic_compare_exchange_n(q, &old, nu, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) return o;
        }
    } else {
        return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
    }
}
template <class T> inline T atomic_min(T* p, T v) {
    maybe_yield();
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return old;
}
template <class T> inline T atomic_max(T* p, T v) {
    maybe_yield();
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v > old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return old;
}
template <class T> inline T atomic_or(T* p, T v) { maybe_yield(); return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomic_and(T* p, T v) { maybe_yield(); return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomic_xchg(T* p, T v) {
    maybe_yield();
    if constexpr (std::is_floating_point<T>::value) {
        using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
        U r = __atomic_exchange_n((U*)p, to_u64(v), __ATOMIC_SEQ_CST);
        return from_u64<T>(r);
    } else {
        return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST);
    }
}
template <class T> inline T atomic_cas(T* p, T cmp, T v) {
    maybe_yield();
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return cmp;
}
template <class T> inline T atomic_load(T* p) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }

inline uint32_t mbcnt_lo(uint32_t m, uint32_t acc) {
    uint32_t l = lane();
    return acc + (uint32_t)__builtin_popcount(l < 32 ? (m & ((1u << l) - 1u)) : m);
}
inline uint32_t mbcnt_hi(uint32_t m, uint32_t acc) {
    uint32_t l = lane();
    return acc + (l < 32 ? 0u : (uint32_t)__builtin_popcount(m & ((1u << (l - 32)) - 1u)));
}
}  // namespace simt

#define threadIdx (simt::tl_thread)
#define blockIdx (simt::tl_block)
#define blockDim (simt::tl_bdim)
#define gridDim (simt::tl_gdim)

#define __HIP_MEMORY_SCOPE_SINGLETHREAD 1
#define __HIP_MEMORY_SCOPE_WAVEFRONT 2
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5
#define __hip_atomic_fetch_add(p, v, o, s) simt::atomic_add((p), (v))
#define __hip_atomic_fetch_min(p, v, o, s) simt::atomic_min((p), (v))
#define __hip_atomic_fetch_max(p, v, o, s) simt::atomic_max((p), (v))
#define __hip_atomic_fetch_or(p, v, o, s) simt::atomic_or((p), (v))
#define __hip_atomic_exchange(p, v, o, s) simt::atomic_xchg((p), (v))
#define __hip_atomic_load(p, o, s) simt::atomic_load((p))
#define __builtin_amdgcn_mbcnt_lo(m, a) simt::mbcnt_lo((m), (a))
#define __builtin_amdgcn_mbcnt_hi(m, a) simt::mbcnt_hi((m), (a))
#define __builtin_amdgcn_readfirstlane(v) ((uint32_t)simt::wave_op(4, (uint64_t)(uint32_t)(v), 0))
#define __builtin_amdgcn_readlane(v, l) ((int)(uint32_t)simt::wave_op(0, (uint64_t)(uint32_t)(v), (int)(l)))
#define __builtin_amdgcn_fence(o, s) __atomic_thread_fence(__ATOMIC_SEQ_CST)
#define __builtin_amdgcn_wave_barrier() simt::wave_barrier()
inline unsigned long long wall_clock64() {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ((unsigned long long)ts.tv_sec * 1000000000ull + (unsigned long long)ts.tv_nsec) / 10ull;
}
// raw buffer (no stride): a dword at a byte offset past num_records reads 0
struct simt_buffer_rsrc { char* base; uint32_t num; };
typedef simt_buffer_rsrc __amdgpu_buffer_rsrc_t;
inline simt_buffer_rsrc __builtin_amdgcn_make_buffer_rsrc(void* p, short, int num, int) {
    return simt_buffer_rsrc{(char*)p, (uint32_t)num};
}
inline uint32_t __builtin_amdgcn_raw_buffer_load_b32(simt_buffer_rsrc r, uint32_t off, uint32_t soff, int) {
    const uint64_t o = (uint64_t)off + soff;
    if (o + 4 > r.num) return 0u;
    return __atomic_load_n((uint32_t*)(r.base + o), __ATOMIC_RELAXED);
}

inline void __syncthreads() { simt::syncthreads(); }
inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
template <class T> inline T __shfl(T v, int src, int = 64) { return simt::from_u64<T>(simt::wave_op(0, simt::to_u64(v), src)); }
template <class T> inline T __shfl_xor(T v, int m, int = 64) { return simt::from_u64<T>(simt::wave_op(1, simt::to_u64(v), m)); }
template <class T> inline T __shfl_up(T v, unsigned d, int = 64) { return simt::from_u64<T>(simt::wave_op(2, simt::to_u64(v), (int)d)); }
inline unsigned long long __ballot(int p) { return simt::wave_op(3, p ? 1u : 0u, 0); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __popc(unsigned int x) { return __builtin_popcount(x); }
inline int __clz(int x) { return x == 0 ? 32 : __builtin_clz((unsigned)x); }
inline int __clzll(long long x) { return x == 0 ? 64 : __builtin_clzll((unsigned long long)x); }
inline int __ffs(unsigned x) { return __builtin_ffs((int)x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline unsigned __float_as_uint(float f) { unsigned u; memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(unsigned u) { float f; memcpy(&f, &u, 4); return f; }
inline int __float_as_int(float f) { int u; memcpy(&u, &f, 4); return u; }
inline float __int_as_float(int u) { float f; memcpy(&f, &u, 4); return f; }
inline long long __double_as_longlong(double d) { long long u; memcpy(&u, &d, 8); return u; }
inline double __longlong_as_double(long long u) { double d; memcpy(&d, &u, 8); return d; }

#define SIMT_ATOMIC2(name, fn) \
    inline unsigned name(unsigned* p, unsigned v) { return fn(p, v); } \
    inline int name(int* p, int v) { return fn(p, v); } \
    inline unsigned long long name(unsigned long long* p, unsigned long long v) { return fn(p, v); }
SIMT_ATOMIC2(atomicAdd, simt::atomic_add)
SIMT_ATOMIC2(atomicMin, simt::atomic_min)
SIMT_ATOMIC2(atomicMax, simt::atomic_max)
SIMT_ATOMIC2(atomicOr, simt::atomic_or)
SIMT_ATOMIC2(atomicAnd, simt::atomic_and)
SIMT_ATOMIC2(atomicExch, simt::atomic_xchg)
inline float atomicAdd(float* p, float v) { return simt::atomic_add(p, v); }
inline double atomicAdd(double* p, double v) { return simt::atomic_add(p, v); }
inline unsigned atomicCAS(unsigned* p, unsigned c, unsigned v) { return simt::atomic_cas(p, c, v); }
inline int atomicCAS(int* p, int c, int v) { return simt::atomic_cas(p, c, v); }
inline unsigned long long atomicCAS(unsigned long long* p, unsigned long long c, unsigned long long v) {
    return simt::atomic_cas(p, c, v);
}

// ------------------------------------------------------------ host API
typedef int hipError_t;
enum : int { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorLaunchFailure = 719 };
typedef struct simt_stream* hipStream_t;
typedef struct simt_event* hipEvent_t;
typedef void* hipDeviceptr_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
#define hipHostMallocDefault 0u
struct hipDeviceProp_t {
    char name[256];
    size_t totalGlobalMem;
    size_t sharedMemPerBlock;
    int multiProcessorCount;
    int maxThreadsPerBlock;
    int warpSize;
    char gcnArchName[256];
};

hipError_t hipMalloc(void** p, size_t n);
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
template <class T> inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags = 0) { return hipHostMalloc((void**)p, n, flags); }
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipMemsetD32Async(hipDeviceptr_t d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t);
hipError_t hipSetDevice(int);
hipError_t hipGetDevice(int*);
hipError_t hipGetDeviceCount(int*);
hipError_t hipGetDeviceProperties(hipDeviceProp_t*, int);
hipError_t hipMemGetInfo(size_t* fr, size_t* tot);
hipError_t hipEventCreate(hipEvent_t*);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int threads, size_t dyn);
hipError_t hipGetSymbolAddress(void** p, const void* sym);

namespace fk {
struct GraphDev;
struct QueryDev;
struct BufDev;
}  // namespace fk
namespace simt {
// Runs grid x block lanes of `body`; cooperative launches get one thread per
// workgroup at once so that grid barriers can complete.
hipError_t run_grid(const char* name, dim3 grid, dim3 block, size_t dyn, bool cooperative,
                    const std::function<void()>& body);
// Hook called after every launch with the kernel's name and its arguments
// (the buffer checker uses the library's device descriptors).
template <class T> inline void note_arg(const T&) {}
void note_arg(const fk::GraphDev&);
void note_arg(const fk::QueryDev&);
void note_arg(const fk::BufDev&);
void after_launch(const char* name);
}  // namespace simt

template <class... K, class... A>
inline hipError_t simt_launch(const char* name, void (*k)(K...), dim3 grid, dim3 block, size_t dyn, hipStream_t,
                              A&&... a) {
    std::function<void()> body = [&]() { k(a...); };
    hipError_t e = simt::run_grid(name, grid, block, dyn, false, body);
    (simt::note_arg(a), ...);
    simt::after_launch(name);
    return e;
}
#define hipLaunchKernelGGL(k, grid, block, dyn, st, ...) \
    simt_launch(#k, (k), dim3(grid), dim3(block), (size_t)(dyn), (st), ##__VA_ARGS__)

template <class... K, size_t... I>
inline void simt_call_packed(void (*k)(K...), void** args, std::index_sequence<I...>) {
    k(*(typename std::remove_reference<K>::type*)args[I]...);
}
template <class... K, size_t... I>
inline void simt_note_packed(void** args, std::index_sequence<I...>) {
    (simt::note_arg(*(typename std::remove_reference<K>::type*)args[I]), ...);
}
template <class... K>
inline hipError_t hipLaunchCooperativeKernel(void (*k)(K...), dim3 grid, dim3 block, void** args, size_t dyn,
                                             hipStream_t) {
    std::function<void()> body = [&]() { simt_call_packed(k, args, std::index_sequence_for<K...>{}); };
    hipError_t e = simt::run_grid("cooperative", grid, block, dyn, true, body);
    simt_note_packed<K...>(args, std::index_sequence_for<K...>{});
    simt::after_launch("cooperative");
    return e;
}
