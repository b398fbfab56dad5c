// Batched Stockham FFT steps on data held in LDS (shared by the tile kernels
// and the global pass kernels).
//
// nfft independent FFTs of size M = 2^lgM; element q of FFT f sits at
// buf[f * fst + q * est].  One radix-R step with span Ns = 2^lgNs takes, for
// job j in [0, M/R), the R inputs q = j + s*M/R, multiplies input s by
// w_{Ns*R}^{(j mod Ns)*s}, runs an R-point DFT and writes output s to
// position (j / Ns)*Ns*R + (j mod Ns) + s*Ns.  After all steps the FFT output
// is in natural order (Stockham auto-sort), so no bit reversal is needed.
#pragma once
#include "mrdft_device.h"

namespace mrdft {

template <int R>
struct Log2 {
    static constexpr int v = (R == 1) ? 0 : (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
};

// Load the inputs of this thread's jobs, apply the step twiddles and the
// R-point DFT.  Results stay in v[c*R + s].
template <int R, int JPT, bool INV>
__device__ __forceinline__ void step_load(const float2* buf, int lgM, int lgNs, int fst, int est, int nfft,
                                          const float2* __restrict__ tab, float2* v, int tid, int nthr) {
    constexpr int lgR = Log2<R>::v;
    const int lgper = lgM - lgR;
    const int per = 1 << lgper;
    const int jobs = nfft << lgper;
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * nthr;
        if (J < jobs) {
            const int f = J >> lgper;
            const int j = J & (per - 1);
#pragma unroll
            for (int s = 0; s < R; ++s) v[c * R + s] = buf[f * fst + (j + s * per) * est];
            if (lgNs > 0) {
                const int jm = j & ((1 << lgNs) - 1);
#pragma unroll
                for (int s = 1; s < R; ++s) {
                    const float2 w = tw_tile(tab, lgNs + lgR, jm * s);
                    v[c * R + s] = INV ? cmulc(v[c * R + s], w) : cmul(v[c * R + s], w);
                }
            }
            dft_reg<R, INV>(&v[c * R]);
        }
    }
}

// Write the results of step_load to their Stockham output positions.
template <int R, int JPT>
__device__ __forceinline__ void step_store(float2* buf, int lgM, int lgNs, int fst, int est, int nfft,
                                           const float2* v, int tid, int nthr) {
    constexpr int lgR = Log2<R>::v;
    const int lgper = lgM - lgR;
    const int per = 1 << lgper;
    const int jobs = nfft << lgper;
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * nthr;
        if (J < jobs) {
            const int f = J >> lgper;
            const int j = J & (per - 1);
            const int jm = j & ((1 << lgNs) - 1);
            const int base = ((j >> lgNs) << (lgNs + lgR)) + jm;
#pragma unroll
            for (int s = 0; s < R; ++s) buf[f * fst + (base + (s << lgNs)) * est] = v[c * R + s];
        }
    }
}

// A full in-place Stockham step: load, barrier, store, barrier.
template <int R, int JPT, bool INV>
__device__ __forceinline__ void lds_step(float2* buf, int lgM, int lgNs, int fst, int est, int nfft,
                                         const float2* __restrict__ tab, int tid, int nthr) {
    float2 v[JPT * R];
    step_load<R, JPT, INV>(buf, lgM, lgNs, fst, est, nfft, tab, v, tid, nthr);
    __syncthreads();
    step_store<R, JPT>(buf, lgM, lgNs, fst, est, nfft, v, tid, nthr);
    __syncthreads();
}

}  // namespace mrdft
