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
