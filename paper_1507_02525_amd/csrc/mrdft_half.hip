// Gradient of the packed half-spectrum output of a real plan.
//
// A real window's spectrum is Hermitian, Y[L-k] = conj(Y[k]), so the packed
// output keeps L/2 slots per window: slot 0 = (Y[0], Y[L/2]), slot k = Y[k].
// With g the packed gradient unpacked with zeros (slot 0 -> bins 0 and L/2 as
// real numbers, slot k -> bin k, bins above L/2 zero), the gradient of a real
// loss with respect to x is Re(A^H g) = A^H h / 2 with the Hermitian
// extension h[k] = g[k] + conj(g[(L - k) mod L]).  This kernel writes h / 2:
//   bin 0: Re slot 0;  bin L/2: Im slot 0;  0 < k < L/2: slot k / 2;
//   L/2 < k < L: conj(slot L - k) / 2,
// after which the full-spectrum adjoint (whose real part is taken) gives the
// gradient.
#include "mrdft_internal.h"

namespace mrdft {

namespace {

constexpr int kExpandThreads = 256;

__global__ __launch_bounds__(kExpandThreads) void expand_half_kernel(const float2* __restrict__ gh,
                                                                     float2* __restrict__ g,
                                                                     const HalfJob* __restrict__ jobs) {
    const HalfJob jb = jobs[blockIdx.x];
    const int64_t L = int64_t(1) << jb.lg, M = L / 2;
    for (int e = threadIdx.x; e < jb.len; e += kExpandThreads) {
        const int64_t idx = jb.c0 + e;                   // bin position inside the level
        const int64_t k = idx & (L - 1);
        const float2* hw = gh + jb.hlev + (idx >> jb.lg) * M;
        float2 v;
        if (k == 0) v = make_float2(hw[0].x, 0.0f);
        else if (k == M) v = make_float2(hw[0].y, 0.0f);
        else if (k < M) v = make_float2(0.5f * hw[k].x, 0.5f * hw[k].y);
        else v = make_float2(0.5f * hw[L - k].x, -0.5f * hw[L - k].y);
        g[jb.flev + idx] = v;
    }
}

}  // namespace

hipError_t launch_expand_half(const float2* gh, float2* g, const HalfJob* jobs, int64_t njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(expand_half_kernel, dim3((unsigned)njobs), dim3(kExpandThreads), 0, s, gh, g, jobs);
    return hipGetLastError();
}

}  // namespace mrdft
