// Device-side helpers for the MrDFT kernels (gfx950, wave64).
//
// Complex numbers are float2 (re, im), the interleaved complex64 layout.
// All small DFTs use the forward sign exp(-j*2*pi*n*k/R) of eq. (1) unless
// INV is set, in which case they use the conjugate kernel (adjoint).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrdft {

constexpr int kTileMaxLog = 12;                 // largest on-chip tile, 2^12 samples
constexpr int kTileMax = 1 << kTileMaxLog;
constexpr int kTileThreads = 256;
constexpr int kPassSmallLog = 12;               // global Stockham pass: 4096-point workgroups ...
constexpr int kPassSmallMaxLog = 8;             // ... for radices up to 2^8
constexpr int kPassBigLog = 13;                 // 8192-point workgroups for radix 2^9
constexpr int kPassMaxLog = 9;                  // radix of one global pass <= 2^9
constexpr int kTwFineLog = 14;                  // FP64 twiddle split: 2^28 = 2^14 * 2^14
constexpr int kMaxOrder = 28;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// acc + a * b as four fused multiply-adds (cadd(acc, cmul(a, b)) compiles to
// six instructions: the product is rounded before the sum)
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, acc.x)),
                       __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, acc.y)));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float norm2(float2 a) { return a.x * a.x + a.y * a.y; }
// a * (-j) and a * (+j)
__device__ __forceinline__ float2 mul_mj(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_pj(float2 a) { return make_float2(-a.y, a.x); }

// Twiddle w_n^q for n <= 16, compile-time after unrolling; trivial factors
// (w^0 = 1, w^{n/4} = -j, Section 5) become sign/swap operations.
template <bool INV>
__device__ __forceinline__ float2 twiddle_small(float2 a, int q, int n) {
    if (q == 0) return a;
    if (4 * q == n) return INV ? mul_pj(a) : mul_mj(a);
    // cos/sin of 2*pi*q/n for n in {8, 16}: index e = q * 16 / n in [1, 8)
    const int e = q * (16 / n);
    const float c16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f,
                          0.0f, -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f};
    const float s16[8] = {0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f,
                          1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f};
    const float c = c16[e], s = INV ? s16[e] : -s16[e];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// Output store with the non-temporal hint: the level spectra are written once
// and not read again by the launch, so they should not displace the input
// samples that other workgroups of the launch re-read from L2.
typedef float ntf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_out(float2* p, float4 v) {
    const ntf4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (ntf4*)p);
}

__host__ __device__ constexpr int bitrev_ct(int v, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register R-point DFT (R = 1, 2, 4, 8, 16), natural order in and out.
// Radix-2 decimation in frequency followed by a compile-time bit-reversal
// (pure register renaming after unrolling).
template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* v) {
    if constexpr (R > 1) {
#pragma unroll
        for (int half = R / 2; half >= 1; half >>= 1) {
#pragma unroll
            for (int b = 0; b < R; b += 2 * half) {
#pragma unroll
                for (int q = 0; q < half; ++q) {
                    float2 a = v[b + q], c = v[b + q + half];
                    v[b + q] = cadd(a, c);
                    v[b + q + half] = twiddle_small<INV>(csub(a, c), q, 2 * half);
                }
            }
        }
        constexpr int bits = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = bitrev_ct(k, bits);
            if (r > k) {
                float2 t = v[k];
                v[k] = v[r];
                v[r] = t;
            }
        }
    }
}

// FP32 twiddle w_{2^lg}^e from the on-device table of w_{kTileMax}^e
// (FP64-generated, rounded once), valid for lg <= kTileMaxLog.
__device__ __forceinline__ float2 tw_tile(const float2* __restrict__ tab, int lg, int e) {
    return tab[(e << (kTileMaxLog - lg)) & (kTileMax - 1)];
}

// Twiddle w_{2^lg}^e for lg <= kMaxOrder: split the exponent of w_{2^28} into
// coarse and fine parts, multiply the two FP64 table entries in FP64 and round
// once to FP32 (one rounding, like the FP32 tile table).
__device__ __forceinline__ float2 tw_big(const double2* __restrict__ hi, const double2* __restrict__ lo,
                                         int lg, int64_t e) {
    const int64_t mask = ((int64_t)1 << kMaxOrder) - 1;
    const int64_t E = (e << (kMaxOrder - lg)) & mask;
    const double2 a = hi[E >> kTwFineLog];
    const double2 b = lo[E & ((1 << kTwFineLog) - 1)];
    return make_float2((float)(a.x * b.x - a.y * b.y), (float)(a.x * b.y + a.y * b.x));
}

// Bin k (0 <= k < Lw) of one window held as packed half spectra (Lw/2 slots:
// slot 0 = (bin 0, bin Lw/2), slot k = bin k), read as a Hermitian spectrum:
// bins 0 and Lw/2 the real numbers of slot 0, bin k < Lw/2 hs * slot k, bin
// k > Lw/2 hs * conj(slot Lw - k).  hs = 1/2 reads a half plan's packed
// gradient as the Hermitian extension halved, whose real adjoint is the
// packed adjoint; hs = 1 reads packed spectra of real signals back whole.
// One load per bin and no branches (selects), so that a thread's loads can
// all be in flight together.
__device__ __forceinline__ float2 half_bin(const float2* __restrict__ hw, int64_t k, int64_t Lw, float hs) {
    const int64_t M = Lw >> 1;
    const bool up = k > M;
    const int64_t slot = up ? Lw - k : (k == M ? 0 : k);
    const float2 v = hw[slot];
    const float re = (k == 0) ? v.x : (k == M) ? v.y : hs * v.x;
    const float im = (k == 0 || k == M) ? 0.0f : (up ? -hs * v.y : hs * v.y);
    return make_float2(re, im);
}

// Same twiddle in FP64 (not rounded).
__device__ __forceinline__ double2 tw_big64(const double2* __restrict__ hi, const double2* __restrict__ lo, int lg,
                                            int64_t e) {
    const int64_t mask = ((int64_t)1 << kMaxOrder) - 1;
    const int64_t E = (e << (kMaxOrder - lg)) & mask;
    const double2 a = hi[E >> kTwFineLog];
    const double2 b = lo[E & ((1 << kTwFineLog) - 1)];
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace mrdft
