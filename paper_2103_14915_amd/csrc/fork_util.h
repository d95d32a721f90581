// Device helpers shared by the fork-processing kernels (gfx950, wave64).
#pragma once
#include "fork_dev.h"

namespace fk {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t rank_in(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ unsigned long long wballot(bool p) { return __ballot(p); }
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
template <class T> __device__ __forceinline__ T wmin(T v) {
#pragma unroll
    for (int o = 32; o; o >>= 1) { T t = __shfl_xor(v, o); v = t < v ? t : v; }
    return v;
}
__device__ __forceinline__ uint32_t wsum(uint32_t v) {
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint32_t wscan_incl(uint32_t v, uint32_t lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) { uint32_t t = __shfl_up(v, o); if (lane >= (uint32_t)o) v += t; }
    return v;
}
__device__ __forceinline__ uint32_t wscan_max_incl(uint32_t v, uint32_t lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) { uint32_t t = __shfl_up(v, o); if (lane >= (uint32_t)o) v = t > v ? t : v; }
    return v;
}
__device__ __forceinline__ uint32_t bcast0(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Query-state atomics: the state slice of a (partition, query) work item is
// owned by one wavefront during a pass, so workgroup scope is sufficient.
__device__ __forceinline__ uint32_t st_min(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t st_read(uint32_t* p) {
    return __hip_atomic_fetch_or(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ float st_addf(float* p, float v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ float st_xchgf(float* p, float v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Buffer bookkeeping shared by all waves of the device.
template <class T> __device__ __forceinline__ T dev_add(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T dev_min(T* p, T v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T dev_max(T* p, T v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T dev_or(T* p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T dev_xchg(T* p, T v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int WB> __device__ __forceinline__ uint32_t edge_w(const void* w, uint32_t e) {
    if constexpr (WB == 0) return 1u;
    else if constexpr (WB == 1) return ((const uint8_t*)w)[e];
    else if constexpr (WB == 2) return ((const uint16_t*)w)[e];
    else return ((const uint32_t*)w)[e];
}

// A PPR vertex is active (must be pushed) while r > 0 and r >= thr.
__device__ __forceinline__ bool ppr_active(float r, float thr) { return r > 0.f && r >= thr; }

}  // namespace fk
