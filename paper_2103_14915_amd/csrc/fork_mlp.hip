// Learned partition scheduler: host launchers of the scoring kernels (the
// device code is in fork_mlp.h).
#include "fork_mlp.h"

namespace fk {

__global__ __launch_bounds__(1024) void k_gstat(GraphDev g, BufDev B, GStat* out) { gstat_body(g, B, out); }

// Scores for all partitions; one thread per partition, weights in LDS.
// Also writes the features when feat != NULL (trace capture for training).
__global__ __launch_bounds__(256) void k_mlp_score(GraphDev g, BufDev B, const GStat* gs, const float* theta,
                                                   float* score, float* feat, uint32_t pass_override) {
    __shared__ float w[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) w[i] = theta[i];
    __syncthreads();
    const uint32_t P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= g.np) return;
    const GStat s = *gs;
    const uint32_t pass = pass_override ? pass_override : B.ctl->pass + 1;
    float x[MLP_IN];
    partition_features(g, B, s, pass, P, x);
    if (feat) {
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) feat[(size_t)P * MLP_IN + i] = x[i];
    }
    float y = mlp_forward(w, x);
    score[P] = B.pcount[P] ? y : -3.0e38f;
}

size_t gstat_bytes() { return sizeof(GStat); }

hipError_t launch_mlp_score(const GraphDev& g, const BufDev& B, const float* theta, float* score, float* feat,
                            void* gstat, uint32_t pass_override, hipStream_t s) {
    hipLaunchKernelGGL(k_gstat, dim3(1), dim3(1024), 0, s, g, B, (GStat*)gstat);
    hipLaunchKernelGGL(k_mlp_score, dim3((g.np + 255) / 256), dim3(256), 0, s, g, B, (const GStat*)gstat, theta,
                       score, feat, pass_override);
    return hipGetLastError();
}

}  // namespace fk

// ---------------------------------------------------------------- training
// Gradient of the mean squared error over a batch, forward and backward in
// fp32 (the fp64 reference is the oracle's MLP).  One block of 256 threads
// takes up to GB samples: phase 1, one thread per sample, runs the forward
// pass and back-propagates to the pre-activations; phase 2, all threads,
// forms each parameter's gradient as a dot product over the block's samples
// and adds it to the global gradient.
namespace fk {

constexpr int GB = 64;  // samples per block

__global__ __launch_bounds__(256) void k_mlp_grad(const float* theta, const float* X, const float* T,
                                                 const uint32_t* idx, uint32_t n, float inv_n, float* grad,
                                                 float* loss) {
    __shared__ float w[MLP_NPARAM];
    __shared__ float sx[GB][MLP_IN];
    __shared__ float a1[GB][MLP_H];
    __shared__ float a2[GB][MLP_H];
    __shared__ float dz1[GB][MLP_H];
    __shared__ float dz2[GB][MLP_H];
    __shared__ float dy[GB];
    __shared__ float sloss;
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < (uint32_t)MLP_NPARAM; i += blockDim.x) w[i] = theta[i];
    if (t == 0) sloss = 0.f;
    const uint32_t s0 = blockIdx.x * GB;
    const uint32_t nb = (n - s0) < (uint32_t)GB ? (n - s0) : (uint32_t)GB;
    for (uint32_t i = t; i < nb * MLP_IN; i += blockDim.x) {
        uint32_t s = i / MLP_IN, k = i % MLP_IN;
        uint32_t src = idx ? idx[s0 + s] : s0 + s;
        sx[s][k] = X[(size_t)src * MLP_IN + k];
    }
    __syncthreads();
    const float* W1 = w;
    const float* b1 = W1 + MLP_H * MLP_IN;
    const float* W2 = b1 + MLP_H;
    const float* b2 = W2 + MLP_H * MLP_H;
    const float* W3 = b2 + MLP_H;
    const float* b3 = W3 + MLP_H;
    if (t < nb) {
        const uint32_t s = t;
        for (int o = 0; o < MLP_H; ++o) {
            float a = b1[o];
            for (int k = 0; k < MLP_IN; ++k) a = fmaf(W1[o * MLP_IN + k], sx[s][k], a);
            a1[s][o] = a > 0.f ? a : 0.f;
        }
        float y = b3[0];
        for (int o = 0; o < MLP_H; ++o) {
            float a = b2[o];
            for (int i = 0; i < MLP_H; ++i) a = fmaf(W2[o * MLP_H + i], a1[s][i], a);
            dz2[s][o] = a;                 // pre-activation for now
            a2[s][o] = a > 0.f ? a : 0.f;
            y = fmaf(W3[o], a2[s][o], y);
        }
        uint32_t src = idx ? idx[s0 + s] : s0 + s;
        float diff = y - T[src];
        atomicAdd(&sloss, diff * diff * inv_n);
        float d = 2.f * diff * inv_n;
        dy[s] = d;
        for (int o = 0; o < MLP_H; ++o) dz2[s][o] = dz2[s][o] > 0.f ? d * W3[o] : 0.f;
        for (int i = 0; i < MLP_H; ++i) {
            float g = 0.f;
            for (int o = 0; o < MLP_H; ++o) g = fmaf(W2[o * MLP_H + i], dz2[s][o], g);
            dz1[s][i] = a1[s][i] > 0.f ? g : 0.f;
        }
    }
    __syncthreads();
    for (uint32_t p = t; p < (uint32_t)MLP_NPARAM; p += blockDim.x) {
        float g = 0.f;
        if (p < (uint32_t)(MLP_H * MLP_IN)) {                       // W1[o][k]
            uint32_t o = p / MLP_IN, k = p % MLP_IN;
            for (uint32_t s = 0; s < nb; ++s) g = fmaf(dz1[s][o], sx[s][k], g);
        } else if (p < (uint32_t)(MLP_H * MLP_IN + MLP_H)) {        // b1[o]
            uint32_t o = p - MLP_H * MLP_IN;
            for (uint32_t s = 0; s < nb; ++s) g += dz1[s][o];
        } else if (p < (uint32_t)(MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H)) {  // W2[o][i]
            uint32_t q = p - (MLP_H * MLP_IN + MLP_H), o = q / MLP_H, i = q % MLP_H;
            for (uint32_t s = 0; s < nb; ++s) g = fmaf(dz2[s][o], a1[s][i], g);
        } else if (p < (uint32_t)(MLP_H * MLP_IN + 2 * MLP_H + MLP_H * MLP_H)) {  // b2[o]
            uint32_t o = p - (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H);
            for (uint32_t s = 0; s < nb; ++s) g += dz2[s][o];
        } else if (p < (uint32_t)(MLP_NPARAM - 1)) {                 // W3[o]
            uint32_t o = p - (MLP_H * MLP_IN + 2 * MLP_H + MLP_H * MLP_H);
            for (uint32_t s = 0; s < nb; ++s) g = fmaf(dy[s], a2[s][o], g);
        } else {                                                     // b3
            for (uint32_t s = 0; s < nb; ++s) g += dy[s];
        }
        atomicAdd(&grad[p], g);
    }
    if (t == 0) atomicAdd(loss, sloss);
}

// Adam (Kingma and Ba 2015) on the flat parameter vector; step counts from 1.
__global__ void k_adam(float* theta, const float* grad, float* m, float* v, uint32_t step, float lr, float b1,
                       float b2, float eps) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)MLP_NPARAM) return;
    float g = grad[i];
    float mi = b1 * m[i] + (1.f - b1) * g;
    float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / (1.f - powf(b1, (float)step));
    float vh = vi / (1.f - powf(b2, (float)step));
    theta[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* theta, const float* X, uint32_t n, float* y) {
    __shared__ float w[MLP_NPARAM];
    for (uint32_t i = threadIdx.x; i < (uint32_t)MLP_NPARAM; i += blockDim.x) w[i] = theta[i];
    __syncthreads();
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[MLP_IN];
    for (int k = 0; k < MLP_IN; ++k) x[k] = X[(size_t)s * MLP_IN + k];
    y[s] = mlp_forward(w, x);
}

}  // namespace fk

namespace fk {
hipError_t launch_mlp_grad(const float*, const float*, const float*, const uint32_t*, uint32_t, float*, float*,
                           hipStream_t);
hipError_t launch_adam(float*, const float*, float*, float*, uint32_t, float, hipStream_t);
// ------------------------------------------------------------ training without allocation
// Scratch of fork_mlp_train_noalloc, one copy per GPU for the life of the
// process: the gradient, Adam's two moments, a loss sink, the generator
// state of the epoch shuffles and the sample permutation.
constexpr uint32_t TRAIN_NMAX = 32768;  // samples (the shuffle runs in one workgroup's LDS)
constexpr size_t SCR_GRAD = 0, SCR_M = MLP_NPARAM, SCR_V = 2 * MLP_NPARAM, SCR_SINK = 3 * MLP_NPARAM;
constexpr size_t SCR_RNG = (3 * MLP_NPARAM + 2) & ~(size_t)1;  // 8-byte aligned word index
constexpr size_t SCR_PERM = SCR_RNG + 2;
constexpr size_t SCRATCH_WORDS = SCR_PERM + TRAIN_NMAX;
static __device__ __align__(256) uint32_t scratch[SCRATCH_WORDS];

__global__ void k_fill32(uint32_t* p, uint32_t n, uint32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// perm = identity, generator state = seed.
__global__ void k_perm_init(uint32_t* perm, uint32_t n, unsigned long long* st, unsigned long long seed) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) perm[i] = i;
    if (blockIdx.x == 0 && threadIdx.x == 0) *st = seed;
}

// One epoch's shuffle of perm: the Fisher-Yates pass of fork_mlp_train with
// the same SplitMix64 stream, done by one thread on an LDS copy.
__global__ __launch_bounds__(256) void k_perm_shuffle(uint32_t* perm, uint32_t n, unsigned long long* st) {
    extern __shared__ uint32_t dyn[];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dyn[i] = perm[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = *st;
        for (uint32_t i = n - 1; i > 0; --i) {
            s += 0x9E3779B97F4A7C15ull;
            const uint32_t j = (uint32_t)(mix64(s) % (unsigned long long)(i + 1));
            const uint32_t x = dyn[i];
            dyn[i] = dyn[j];
            dyn[j] = x;
        }
        *st = s;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) perm[i] = dyn[i];
}

uint32_t train_nmax() { return TRAIN_NMAX; }
// Once per device: the shuffle's LDS copy of the permutation exceeds the default 64 KB.
hipError_t train_prepare() {
    return hipFuncSetAttribute((const void*)k_perm_shuffle, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(TRAIN_NMAX * sizeof(uint32_t)));
}
size_t train_scratch_bytes() { return sizeof(scratch); }
// The scratch array's device address on the current device.
hipError_t train_scratch_address(void** p) { return hipGetSymbolAddress(p, HIP_SYMBOL(scratch)); }

hipError_t launch_train_noalloc(uint32_t* scr, float* theta, const float* X, const float* T, uint32_t n,
                                uint32_t steps, uint32_t batch, float lr, unsigned long long seed, float* losses,
                                hipStream_t s) {
    float* grad = (float*)scr + SCR_GRAD;
    float* m = (float*)scr + SCR_M;
    float* v = (float*)scr + SCR_V;
    float* sink = (float*)scr + SCR_SINK;
    unsigned long long* st = (unsigned long long*)(scr + SCR_RNG);
    uint32_t* perm = scr + SCR_PERM;
    // everything that must start at zero is cleared by a kernel (the array keeps the last call's contents)
    hipLaunchKernelGGL(k_fill32, dim3(64), dim3(256), 0, s, scr, (uint32_t)(3 * MLP_NPARAM + 1), 0u);
    if (losses && steps) hipLaunchKernelGGL(k_fill32, dim3(64), dim3(256), 0, s, (uint32_t*)losses, steps, 0u);
    hipLaunchKernelGGL(k_perm_init, dim3(64), dim3(256), 0, s, perm, n, st, seed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t pos = n;
    for (uint32_t k = 1; k <= steps; ++k) {
        if (pos + batch > n) {
            hipLaunchKernelGGL(k_perm_shuffle, dim3(1), dim3(256), n * sizeof(uint32_t), s, perm, n, st);
            pos = 0;
        }
        hipLaunchKernelGGL(k_fill32, dim3(8), dim3(256), 0, s, (uint32_t*)grad, (uint32_t)MLP_NPARAM, 0u);
        e = launch_mlp_grad(theta, X, T, perm + pos, batch, grad, losses ? losses + (k - 1) : sink, s);
        if (e != hipSuccess) return e;
        e = launch_adam(theta, grad, m, v, k, lr, s);
        if (e != hipSuccess) return e;
        pos += batch;
    }
    return hipGetLastError();
}
}  // namespace fk

namespace fk {
hipError_t launch_mlp_grad(const float* theta, const float* X, const float* T, const uint32_t* idx, uint32_t n,
                           float* grad, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3((n + GB - 1) / GB), dim3(256), 0, s, theta, X, T, idx, n, 1.f / (float)n,
                       grad, loss);
    return hipGetLastError();
}
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, uint32_t step, float lr, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, theta, grad, m, v, step, lr, 0.9f,
                       0.999f, 1e-8f);
    return hipGetLastError();
}
hipError_t launch_mlp_forward(const float* theta, const float* X, uint32_t n, float* y, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, theta, X, n, y);
    return hipGetLastError();
}
}  // namespace fk
