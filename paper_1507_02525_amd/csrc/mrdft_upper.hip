// Levels whose window L = 2^i exceeds the tile, computed in one pass from x.
//
// Level i is the L-point DFT of every length-L window (Section 2, eq. (1)).
// With L = R * 1024, n = n1 + 1024*n2 and k = k2 + R*k1 (n1, k1 < 1024;
// n2, k2 < R) the window DFT factors as
//
//     Y[k2 + R*k1] = sum_{n1} w_1024^{n1*k1} * ( w_L^{n1*k2} * C[n1][k2] ),
//     C[n1][k2]    = sum_{n2} x[n1 + 1024*n2] * w_R^{n2*k2}          (column DFTs)
//
// A workgroup owns G = min(R, 16) consecutive k2 of one window: it forms the
// G column values of every n1 straight from x (the input is small and stays
// in cache, so re-reading it costs no HBM traffic), applies the twiddles,
// runs G row FFTs of 1024 points in LDS, and writes 16 consecutive outputs
// (128 bytes) per k1.  No intermediate array goes through HBM.
#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"

namespace mrdft {

constexpr int kRowLog = 10;
constexpr int kRow = 1 << kRowLog;          // row FFT length
constexpr int kUpThreads = 512;
constexpr int kUpMaxG = 16;
constexpr int kRowStride = kRow + 1;        // odd row stride: rows start on different LDS banks

template <bool REAL>
__device__ __forceinline__ float2 ld_x(const void* __restrict__ x, int64_t idx) {
    if constexpr (REAL) return make_float2(((const float*)x)[idx], 0.0f);
    else return ((const float2*)x)[idx];
}

// Split Z = DFT(a + j b) of two real sequences a, b (length N) into
// A[k] = (Z[k] + conj(Z[-k])) / 2 and B[k] = -j (Z[k] - conj(Z[-k])) / 2.
template <int N>
__device__ __forceinline__ void split_real_pair(const float2* Z, float2* A, float2* B) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float2 z = Z[k], zc = cconj(Z[(N - k) & (N - 1)]);
        A[k] = make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y + zc.y));
        const float2 d = make_float2(0.5f * (z.x - zc.x), 0.5f * (z.y - zc.y));
        B[k] = mul_mj(d);
    }
}

// Column DFT values C[n1][16g + kap] (R > 16) or C[n1][kap] (R <= 16) for the
// input columns in v[] (v[n2] = x[n1 + 1024*n2]); R = 16 * P splits into the
// sub-sequences n2 = r + P*b:  C[16g + kap] = sum_r w_R^{r(16g + kap)} DFT16(v[r + P b])[kap].
template <int RL>
__device__ __forceinline__ void column_from_complex(const float2* v, int g, const float2* __restrict__ tab, float2* out) {
    constexpr int R = 1 << RL;
    if constexpr (R <= 16) {
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) out[n2] = v[n2];
        dft_reg<R, false>(out);
    } else {
        constexpr int P = R / 16;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            float2 f[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) f[b] = v[r + P * b];
            dft_reg<16, false>(f);
#pragma unroll
            for (int kap = 0; kap < 16; ++kap) {
                if (r == 0) out[kap] = f[kap];
                else out[kap] = cmac(out[kap], f[kap], tw_tile(tab, RL, (r * (16 * g + kap)) & (R - 1)));
            }
        }
    }
}

// Same for two real columns a, b at once (one complex DFT per sub-sequence).
template <int RL>
__device__ __forceinline__ void column_from_real_pair(const float* va, const float* vb, int g,
                                                      const float2* __restrict__ tab, float2* oa, float2* ob) {
    constexpr int R = 1 << RL;
    if constexpr (R <= 16) {
        float2 z[R];
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) z[n2] = make_float2(va[n2], vb[n2]);
        dft_reg<R, false>(z);
        split_real_pair<R>(z, oa, ob);
    } else {
        constexpr int P = R / 16;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            float2 z[16], fa[16], fb[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) z[b] = make_float2(va[r + P * b], vb[r + P * b]);
            dft_reg<16, false>(z);
            split_real_pair<16>(z, fa, fb);
#pragma unroll
            for (int kap = 0; kap < 16; ++kap) {
                if (r == 0) {
                    oa[kap] = fa[kap];
                    ob[kap] = fb[kap];
                } else {
                    const float2 w = tw_tile(tab, RL, (r * (16 * g + kap)) & (R - 1));
                    oa[kap] = cmac(oa[kap], fa[kap], w);
                    ob[kap] = cmac(ob[kap], fb[kap], w);
                }
            }
        }
    }
}

template <int RL, bool REAL>
__global__ __launch_bounds__(kUpThreads) void upper_fwd_kernel(const void* __restrict__ x, float2* __restrict__ Y,
                                                               PassGeom geo, const float2* __restrict__ tab,
                                                               const float2* __restrict__ rowtw) {
    constexpr int R = 1 << RL;
    constexpr int G = R < kUpMaxG ? R : kUpMaxG;
    constexpr int NG = R / G;                     // workgroups per window
    extern __shared__ float2 lds[];
    float2* C = lds;                                 // G rows of kRow, padded
    float2* Q = lds + padded_size(G * kRowStride);   // twiddle quarter table

    const int lg = geo.lg;                        // = RL + kRowLog
    const int64_t L = (int64_t)1 << lg;
    const int64_t blk = blockIdx.x;
    const int64_t gwin = blk / NG;
    const int g = (int)(blk - gwin * NG);
    const int64_t b = gwin / geo.wps, W = gwin - b * geo.wps;
    const int64_t ib = (geo.in_sig ? geo.in_sig[b] : b * geo.in_stride) + W * L;
    const int64_t ob = (geo.out_sig ? geo.out_sig[b] : b * geo.out_stride) + W * L;
    const int tid = threadIdx.x;
    const int k0 = g * G;
    // rowtw[k2 * kRow + n1] = w_L^{n1 * k2}
    const float2* __restrict__ rt = rowtw + (int64_t)k0 * kRow;

    load_quarter(Q, tab, tid, kUpThreads);
    // Column DFTs and twiddles w_L^{n1 (k0 + kap)} into LDS rows.  Each thread
    // owns n1 = tid and tid + 512; all of its x loads are issued before any use.
    static_assert(kRow == 2 * kUpThreads, "two columns per thread");
    const int na = tid, nb = tid + kUpThreads;
    if constexpr (REAL) {
        const float* xr = (const float*)x + ib;
        float va[R], vb[R];
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) {
            va[n2] = xr[na + n2 * kRow];
            vb[n2] = xr[nb + n2 * kRow];
        }
        float2 ca[G], cb[G];
        column_from_real_pair<RL>(va, vb, g, tab, ca, cb);
#pragma unroll
        for (int kap = 0; kap < G; ++kap) {
            C[pad(kap * kRowStride + na)] = cmul(ca[kap], rt[kap * kRow + na]);
            C[pad(kap * kRowStride + nb)] = cmul(cb[kap], rt[kap * kRow + nb]);
        }
    } else {
        const float2* xc = (const float2*)x + ib;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int n1 = h ? nb : na;
            float2 v[R];
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) v[n2] = xc[n1 + n2 * kRow];
            float2 col[G];
            column_from_complex<RL>(v, g, tab, col);
#pragma unroll
            for (int kap = 0; kap < G; ++kap) C[pad(kap * kRowStride + n1)] = cmul(col[kap], rt[kap * kRow + n1]);
        }
    }
    __syncthreads();
    // Row FFTs (1024 points, natural order output): radix 4, 16, 16.
    const TwQuarter tw{Q};
    lds_step<4, (G * kRow / 4 + kUpThreads - 1) / kUpThreads, false, true>(C, kRowLog, 0, kRowStride, 1, G, tw, tid,
                                                                           kUpThreads);
    lds_step<16, (G * kRow / 16 + kUpThreads - 1) / kUpThreads, false, true>(C, kRowLog, 2, kRowStride, 1, G, tw, tid,
                                                                             kUpThreads);
    lds_step<16, (G * kRow / 16 + kUpThreads - 1) / kUpThreads, false, true>(C, kRowLog, 6, kRowStride, 1, G, tw, tid,
                                                                             kUpThreads);
    // Y[k0 + kap + R*k1]: G consecutive complex values per k1.
    constexpr int HP = G / 2 > 0 ? G / 2 : 1;
    for (int e = tid; e < kRow * HP; e += kUpThreads) {
        const int k1 = e / HP;
        const int kp = (e - k1 * HP) * 2;
        float4* dst = (float4*)(Y + ob + k0 + kp + (int64_t)R * k1);
        const float2 a = C[pad(kp * kRowStride + k1)];
        const float2 c = C[pad((kp + 1) * kRowStride + k1)];
        *dst = make_float4(a.x, a.y, c.x, c.y);
    }
}

// Offset of level lg's row-twiddle block (rows for k2 < 2^(lg-10), 1024 each)
// in the concatenated table for levels 11..16.
int64_t row_twiddle_offset(int lg) {
    int64_t off = 0;
    for (int l = kRowLog + 1; l < lg; ++l) off += (int64_t)kRow << (l - kRowLog);
    return off;
}

int64_t row_twiddle_entries() { return row_twiddle_offset(kUpperMaxLevel + 1); }

size_t upper_lds_bytes(int rl) {
    const int R = 1 << rl;
    const int G = R < kUpMaxG ? R : kUpMaxG;
    return sizeof(float2) * (size_t)(padded_size(G * kRowStride) + kQuarter);
}

hipError_t launch_upper_fwd(bool real_in, const void* x, float2* Y, const PassGeom& g, const Twiddles& tw,
                            hipStream_t s) {
    const float2* tab = tw.tile;
    const float2* tab16 = tw.rowtw + row_twiddle_offset(g.lg);
    const int rl = g.lg - kRowLog;
    const int R = 1 << rl;
    const int G = R < kUpMaxG ? R : kUpMaxG;
    const int64_t nblk = g.nwin * (R / G);
    if (nblk <= 0) return hipSuccess;
    const size_t lds = upper_lds_bytes(rl);
    dim3 grid((unsigned)nblk), block(kUpThreads);
#define MRDFT_UP(RL_)                                                                                       \
    do {                                                                                                  \
        if (real_in) {                                                                                    \
            (void)hipFuncSetAttribute((const void*)upper_fwd_kernel<RL_, true>,                           \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);              \
            hipLaunchKernelGGL((upper_fwd_kernel<RL_, true>), grid, block, lds, s, x, Y, g, tab, tab16);  \
        } else {                                                                                          \
            (void)hipFuncSetAttribute((const void*)upper_fwd_kernel<RL_, false>,                          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);              \
            hipLaunchKernelGGL((upper_fwd_kernel<RL_, false>), grid, block, lds, s, x, Y, g, tab, tab16); \
        }                                                                                                 \
    } while (0)
    switch (rl) {
        case 1: MRDFT_UP(1); break;
        case 2: MRDFT_UP(2); break;
        case 3: MRDFT_UP(3); break;
        case 4: MRDFT_UP(4); break;
        case 5: MRDFT_UP(5); break;
        case 6: MRDFT_UP(6); break;
        default: return hipErrorInvalidValue;
    }
#undef MRDFT_UP
    return hipGetLastError();
}

}  // namespace mrdft
