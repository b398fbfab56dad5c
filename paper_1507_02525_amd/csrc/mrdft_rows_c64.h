// Levels above the complex tile, one workgroup-sized piece at a time.
//
// Level lg is the L-point DFT (L = 2^lg) of every window (Section 2, eq. (1)).
// With L = R * 256, n = n1 + 256 n2 and k = k2 + R k1 (n1, k1 < 256;
// n2, k2 < R):
//
//     Y[k2 + R k1] = sum_{n1} w_256^{n1 k1} ( w_L^{n1 k2} C[n1][k2] ),
//     C[n1][k2]    = sum_{n2} x[n1 + 256 n2] w_R^{n2 k2}          (column DFTs).
//
// Piece g transforms the 16 rows k2 = 16g .. 16g+15 and writes, for every k1,
// their 16 consecutive outputs (128 bytes).  With n2 = r + P b (P = R/16,
// b < 16), C[16g + q] = sum_r w_R^{r (16g + q)} DFT16(x[n1 + 256 (r + P b)])[q]:
// P sub-DFTs of 16 points per column, combined with FP64-exact factors.
// 256 threads, 37 KB of LDS; levels 12..16 (R = 16..256).
#pragma once
#include "mrdft_device.h"
#include "mrdft_rows_real.h"

namespace mrdft {

constexpr int kCRowsMinLevel = 12;
constexpr int kCRows = 16;                  // rows per piece

struct CRowsLds {
    float2 C[kCRows * kRowsStride];
    float2 T[kRowsN];                       // w_256^e
};

// Combine factors w_R^{r (16 g + q)} of one level, index ((g * P + r) * 16 + q).
__host__ __device__ constexpr int64_t crows_combine_offset(int lg) {
    return lg <= kCRowsMinLevel ? 0
                                : crows_combine_offset(lg - 1) +
                                      (int64_t)(1 << (lg - 1 - kCRowsMinLevel)) * (1 << (lg - 1 - kCRowsMinLevel)) * 16;
}
constexpr int64_t crows_combine_entries() { return crows_combine_offset(kRowsMaxLevel + 1); }

// One radix-16 Stockham step over the 16 rows (one job per thread).
template <int LNS>
__device__ __forceinline__ void crows_step(CRowsLds& S, int tid) {
    constexpr int NS = 1 << LNS;
    const int r = tid >> 4, j = tid & 15;
    float2 v[16];
    const float2* src = S.C + r * kRowsStride;
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = src[rpad(j + 16 * s)];
    if constexpr (LNS > 0) {
        const int jm = j & (NS - 1);
#pragma unroll
        for (int s = 1; s < 16; ++s) v[s] = cmul(v[s], S.T[(jm * s) << (kRowsLog - LNS - 4)]);
    }
    dft_reg<16, false>(v);
    __syncthreads();
    float2* dst = S.C + r * kRowsStride;
    const int base = ((j >> LNS) << (LNS + 4)) + (j & (NS - 1));
#pragma unroll
    for (int s = 0; s < 16; ++s) dst[rpad(base + s * NS)] = v[s];
    __syncthreads();
}

// Piece g of one window of level lg = RL + 8 (4 <= RL <= 8).
//   xw    : the window's first sample      yw: the window's first output
//   rowtw : this level's row twiddles, rowtw[k2 * 256 + n1] = w_L^{n1 k2}
//   comb  : this level's combine factors (crows_combine_offset)
template <int RL>
__device__ __forceinline__ void rows_c64_body(CRowsLds& S, const float2* __restrict__ xw, float2* __restrict__ yw,
                                              int g, const float2* __restrict__ t4096,
                                              const float2* __restrict__ rowtw, const float2* __restrict__ comb,
                                              int tid) {
    constexpr int R = 1 << RL, P = R / 16;
    static_assert(P >= 1 && P <= 16, "rows of 256 cover windows of 2^12 .. 2^16");
    const int k0 = 16 * g;
    const int n1 = tid;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void*)xw, (short)0, R * kRowsN * (int)sizeof(float2), kBufferWord3);
    const int vo = n1 * (int)sizeof(float2);
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    auto xload = [&](int n2) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(xr, vo, n2 * kRowsN * (int)sizeof(float2), 0);
        return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    };
    const float2* cb = comb + (int64_t)g * P * 16;
    float2 acc[16];
    float2 zn[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) zn[b] = xload(P * b);
    auto sub = [&](int r, bool first) {
        float2 z[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) z[b] = zn[b];
        if (r + 1 < P) {
#pragma unroll
            for (int b = 0; b < 16; ++b) zn[b] = xload(r + 1 + P * b);
        }
        dft_reg<16, false>(z);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (first) {
                acc[q] = z[q];                                      // r = 0: factor 1
            } else {
                const float2 w = cb[r * 16 + q];                    // wave-uniform: scalar loads
                acc[q] = cmac(acc[q], z[q], w);
            }
        }
    };
    sub(0, true);
#pragma unroll 1
    for (int r = 1; r < P; ++r) sub(r, false);
#pragma unroll
    for (int q = 0; q < 16; ++q) S.C[q * kRowsStride + rpad(n1)] = cmul(acc[q], rowtw[(k0 + q) * kRowsN + n1]);
    __syncthreads();
    crows_step<0>(S, tid);
    crows_step<4>(S, tid);
    // outputs: 16 consecutive bins k0 .. k0+15 at every k1
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * kRowsThreads;
        const int k1 = e >> 3, kp = (e & 7) * 2;
        const float2 a = S.C[kp * kRowsStride + rpad(k1)];
        const float2 c = S.C[(kp + 1) * kRowsStride + rpad(k1)];
        store_out(yw + k0 + kp + (int64_t)R * k1, make_float4(a.x, a.y, c.x, c.y));
    }
}

// Piece g of one window of level lg = RL + 8 (13 <= lg <= 16) with the 32
// rows k2 = 32g .. 32g+31 (groups 2g and 2g+1): the sub-DFTs of the columns
// are computed once for both groups (half of them per window against two
// 16-row pieces), the two groups' sums stay in registers, and the row FFTs
// run one group after the other in the same LDS.  No loads are issued ahead:
// the registers hold the second group's sums instead.
template <int RL>
__device__ __forceinline__ void rows_c64_body2(CRowsLds& S, const float2* __restrict__ xw, float2* __restrict__ yw,
                                               int g, const float2* __restrict__ t4096,
                                               const float2* __restrict__ rowtw, const float2* __restrict__ comb,
                                               int tid) {
    constexpr int R = 1 << RL, P = R / 16;
    static_assert(P >= 2 && P <= 16, "two groups of 16 rows: windows of 2^13 .. 2^16");
    const int k0 = 32 * g;
    const int n1 = tid;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void*)xw, (short)0, R * kRowsN * (int)sizeof(float2), kBufferWord3);
    const int vo = n1 * (int)sizeof(float2);
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    auto xload = [&](int n2) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(xr, vo, n2 * kRowsN * (int)sizeof(float2), 0);
        return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    };
    const float2* cb0 = comb + (int64_t)(2 * g) * P * 16;        // group 2g
    const float2* cb1 = comb + (int64_t)(2 * g + 1) * P * 16;    // group 2g + 1
    float2 acc[32];
#pragma unroll 1
    for (int r = 0; r < P; ++r) {
        float2 z[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) z[b] = xload(r + P * b);
        dft_reg<16, false>(z);
        if (r == 0) {
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = acc[16 + q] = z[q];     // factor 1
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                acc[q] = cmac(acc[q], z[q], cb0[r * 16 + q]);    // wave-uniform: scalar loads
                acc[16 + q] = cmac(acc[16 + q], z[q], cb1[r * 16 + q]);
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int kh = k0 + 16 * h;
        if (h) __syncthreads();                                    // the first group's outputs are read
#pragma unroll
        for (int q = 0; q < 16; ++q)
            S.C[q * kRowsStride + rpad(n1)] = cmul(acc[16 * h + q], rowtw[(kh + q) * kRowsN + n1]);
        __syncthreads();
        crows_step<0>(S, tid);
        crows_step<4>(S, tid);
        // outputs: 16 consecutive bins kh .. kh+15 at every k1
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int k1 = e >> 3, kp = (e & 7) * 2;
            const float2 a = S.C[kp * kRowsStride + rpad(k1)];
            const float2 c = S.C[(kp + 1) * kRowsStride + rpad(k1)];
            store_out(yw + kh + kp + (int64_t)R * k1, make_float4(a.x, a.y, c.x, c.y));
        }
    }
}

}  // namespace mrdft
