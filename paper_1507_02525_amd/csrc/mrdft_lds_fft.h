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

// LDS padding: one spare element after every 32, so that power-of-two strides
// of 32 or more elements do not fall on the same bank.
constexpr int kPadShift = 5;
__device__ __forceinline__ int pad(int i) { return i + (i >> kPadShift); }
constexpr int padded_size(int n) { return n + (n >> kPadShift); }
// Padding inside each FFT instead (PADC): element q of FFT f at
// f * fst + q + (q >> 5); with a suitable fst the Stockham steps' strided
// accesses and the column-wise accesses of the global passes both spread
// over the banks.
__device__ __forceinline__ int padc(int q) { return q + (q >> kPadShift); }

// Twiddles w_{2^lg}^e (lg <= kTileMaxLog) read from a global FP32 table.
struct TwGlobal {
    const float2* tab;
    __device__ __forceinline__ float2 operator()(int lg, int e) const { return tw_tile(tab, lg, e); }
};

// Same twiddles from a quarter-period table in LDS: q[r] = w_{4096}^r, r < 1024;
// w^{r + 1024 c} = (-j)^c w^r.
constexpr int kQuarter = kTileMax / 4;
struct TwQuarter {
    const float2* q;
    __device__ __forceinline__ float2 operator()(int lg, int e) const {
        const int E = (e << (kTileMaxLog - lg)) & (kTileMax - 1);
        const float2 a = q[E & (kQuarter - 1)];
        const int c = E >> (kTileMaxLog - 2);
        float re = (c & 1) ? a.y : a.x;
        float im = (c & 1) ? -a.x : a.y;
        if (c & 2) {
            re = -re;
            im = -im;
        }
        return make_float2(re, im);
    }
};

// Fill a quarter table in LDS from the global FP32 table (first quarter).
__device__ __forceinline__ void load_quarter(float2* q, const float2* __restrict__ tab, int tid, int nthr) {
    for (int r = tid; r < kQuarter; r += nthr) q[r] = tab[r];
}

// Load the inputs of this thread's jobs, apply the step twiddles and the
// R-point DFT.  Results stay in v[c*R + s].
template <int R, int JPT, bool INV, bool PAD = false, bool PADC = false, class TW = TwGlobal>
__device__ __forceinline__ void step_load(const float2* buf, int lgM, int lgNs, int fst, int est, int nfft,
                                          const TW& tw, float2* v, int tid, int nthr) {
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
            for (int s = 0; s < R; ++s) {
                const int li = PADC ? f * fst + padc(j + s * per) : f * fst + (j + s * per) * est;
                v[c * R + s] = buf[PAD ? pad(li) : li];
            }
            if (lgNs > 0) {
                const int jm = j & ((1 << lgNs) - 1);
#pragma unroll
                for (int s = 1; s < R; ++s) {
                    const float2 w = tw(lgNs + lgR, jm * s);
                    v[c * R + s] = INV ? cmulc(v[c * R + s], w) : cmul(v[c * R + s], w);
                }
            }
            dft_reg<R, INV>(&v[c * R]);
        }
    }
}

// Write the results of step_load to their Stockham output positions.
template <int R, int JPT, bool PAD = false, bool PADC = false>
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
            for (int s = 0; s < R; ++s) {
                const int li = PADC ? f * fst + padc(base + (s << lgNs)) : f * fst + (base + (s << lgNs)) * est;
                buf[PAD ? pad(li) : li] = v[c * R + s];
            }
        }
    }
}

// A full in-place Stockham step: load, barrier, store, barrier.
template <int R, int JPT, bool INV, bool PAD = false, bool PADC = false, class TW = TwGlobal>
__device__ __forceinline__ void lds_step(float2* buf, int lgM, int lgNs, int fst, int est, int nfft,
                                         const TW& tw, int tid, int nthr) {
    float2 v[JPT * R];
    step_load<R, JPT, INV, PAD, PADC>(buf, lgM, lgNs, fst, est, nfft, tw, v, tid, nthr);
    __syncthreads();
    step_store<R, JPT, PAD, PADC>(buf, lgM, lgNs, fst, est, nfft, v, tid, nthr);
    __syncthreads();
}

}  // namespace mrdft
