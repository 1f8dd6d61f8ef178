// adam.hip -- one Adam step with projection over all factor matrices at once
// (Kolda & Hong, Alg. 4 inner loop; Kingma & Ba's moment estimates).
//
// The step counter lives on the device: every block reads t = state[0] + 1
// before it updates anything, and the last block to finish (counted with a
// device-scope atomic in state[1]) stores state[0] = t and clears state[1].
// Repeated steps therefore need no host round trip and can be captured in a
// HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "device.hpp"

namespace gcp {

struct AdamArgs {
    int64_t P;
    void* A;
    float* A_master;
    const void* G;
    void* B;
    void* C;
    int64_t* state;
    double alpha, beta1, beta2, eps, lower;
    int eps_mode;
};

// T: arithmetic and moment type; SHADOW: A is a bf16 copy of the float master.
template <typename T, bool SHADOW>
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    __shared__ int64_t t_shared;
    if (threadIdx.x == 0) t_shared = a.state[0] + 1;
    __syncthreads();
    const int64_t t = t_shared;
    const T bc1 = (T)(1.0 - pow(a.beta1, (double)t));
    const T bc2 = (T)(1.0 - pow(a.beta2, (double)t));
    // 1 - beta is formed in double and rounded once: in float, 1 - 0.999f is
    // off by 1.3e-5 relative because 0.999 is not representable.
    const T b1 = (T)a.beta1, b2 = (T)a.beta2, alpha = (T)a.alpha, eps = (T)a.eps, lower = (T)a.lower;
    const T omb1 = (T)(1.0 - a.beta1), omb2 = (T)(1.0 - a.beta2);
    const T* __restrict__ G = static_cast<const T*>(a.G);
    T* __restrict__ B = static_cast<T*>(a.B);
    T* __restrict__ C = static_cast<T*>(a.C);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < a.P;
         e += (int64_t)gridDim.x * blockDim.x) {
        const T g = G[e];
        const T bm = b1 * B[e] + omb1 * g;
        const T cm = b2 * C[e] + omb2 * g * g;
        B[e] = bm;
        C[e] = cm;
        const T bhat = bm / bc1;
        const T chat = cm / bc2;
        const T den = a.eps_mode == GCP_EPS_INSIDE_SQRT ? sqrt(chat + eps) : sqrt(chat) + eps;
        if constexpr (SHADOW) {
            float v = a.A_master[e] - (float)(alpha * bhat / den);
            v = v < (float)lower ? (float)lower : v;
            a.A_master[e] = v;
            static_cast<bf16_t*>(a.A)[e] = to_bf16(v);
        } else {
            T* __restrict__ A = static_cast<T*>(a.A);
            T v = A[e] - alpha * bhat / den;
            A[e] = v < lower ? lower : v;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long done =
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.state[1]), 1ull);
        if (done == (unsigned long long)gridDim.x - 1ull) {
            a.state[0] = t;
            a.state[1] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void bf16_round_kernel(int64_t P, const float* __restrict__ src,
                                                           bf16_t* __restrict__ dst) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < P; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = to_bf16(src[e]);
}

gcp_status launch_bf16_round(int64_t P, const float* src, void* dst, hipStream_t s) {
    if (P <= 0) return GCP_OK;
    const int64_t blocks = std::min<int64_t>((P + 255) / 256, 8192);
    hipLaunchKernelGGL(bf16_round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, src, static_cast<bf16_t*>(dst));
    return check_launch("gcp_bf16_round");
}

gcp_status launch_adam(int64_t P, gcp_dtype dtype, void* A, float* A_master, const void* G, void* B, void* C,
                       int64_t* state, double alpha, double beta1, double beta2, double eps, double lower,
                       gcp_eps_mode eps_mode, hipStream_t s) {
    AdamArgs a{P, A, A_master, G, B, C, state, alpha, beta1, beta2, eps, lower, (int)eps_mode};
    int64_t blocks = (P + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    const dim3 g((unsigned)blocks), b(256);
    if (dtype == GCP_F64) hipLaunchKernelGGL((adam_kernel<double, false>), g, b, 0, s, a);
    else if (dtype == GCP_F32) hipLaunchKernelGGL((adam_kernel<float, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((adam_kernel<float, true>), g, b, 0, s, a);
    return check_launch("gcp_adam_step");
}

}  // namespace gcp
