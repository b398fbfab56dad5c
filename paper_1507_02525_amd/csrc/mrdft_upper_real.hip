// Single-pass levels above the tile for real input (window L = R * 1024,
// 8 <= R <= 64).  Same column-first factorisation as mrdft_upper.hip:
//
//     Y[k2 + R*k1] = sum_{n1} w_1024^{n1*k1} ( w_L^{n1*k2} C[n1][k2] ),
//     C[n1][k2]    = sum_{n2} x[n1 + 1024*n2] w_R^{n2*k2},
//
// using the Hermitian symmetry of real windows, Y[L-k] = conj(Y[k]), i.e.
// row R-k2 at k1 equals conj(row k2 at 1023-k1): only rows k2 <= R/2 are
// transformed.
//
// * R <= 16: one workgroup per window transforms rows 0..R/2 and writes the
//   whole window.
// * R >= 32 (16-row groups g = 0..R/16-1): workgroup g < R/32 transforms the
//   17 rows 16g..16g+16 and writes group g directly and group R/16-1-g (rows
//   16g+16..16g+1) as conjugates.  Every store is 16 consecutive complex
//   values (128 bytes).
//
// Column DFTs are taken straight from x (two real columns per complex DFT);
// the row FFTs (radix 4, 16, 16) run in LDS with a 1024-entry twiddle table.
#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"

namespace mrdft {

namespace {
constexpr int kRowLog = 10;
constexpr int kRow = 1 << kRowLog;
constexpr int kRowStride = kRow + 1;
constexpr int kThr = 512;

template <int RL>
struct RealUpperShape {
    static constexpr int R = 1 << RL;
    static constexpr bool WHOLE = R <= 16;                 // one workgroup per window
    static constexpr int NR = WHOLE ? R / 2 + 1 : 17;      // rows transformed
    static constexpr int NG = WHOLE ? 1 : R / 16;           // 16-row output groups per window
    static constexpr int WPW = WHOLE ? 1 : NG / 2;          // workgroups per window
};

__device__ __forceinline__ float2 half_sum(float2 a, float2 b) { return make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y)); }

// Z = DFT(a + j b) of two real length-N sequences -> A[k], B[k] for k in [0, K).
template <int N, int K>
__device__ __forceinline__ void split_pair(const float2* Z, float2* A, float2* B) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float2 z = Z[k % N], zc = cconj(Z[(N - k % N) % N]);
        A[k] = half_sum(z, zc);
        B[k] = mul_mj(half_sum(z, make_float2(-zc.x, -zc.y)));
    }
}

// One in-place radix-RR Stockham step over NR rows of 1024 points (row stride
// kRowStride), span 2^LNS, jobs spread over kThr threads.
template <int RR, int NR, int LNS>
__device__ __forceinline__ void row_step(float2* C, const float2* W, int tid) {
    constexpr int LR = (RR == 4) ? 2 : 4;
    constexpr int PER = kRow / RR;
    constexpr int JOBS = NR * PER;
    constexpr int RND = (JOBS + kThr - 1) / kThr;
    constexpr int NS = 1 << LNS;
    float2 v[RND][RR];
#pragma unroll
    for (int c = 0; c < RND; ++c) {
        const int J = tid + c * kThr;
        if (J < JOBS) {
            const int r = J / PER, j = J % PER;
            const float2* src = C + r * kRowStride + j;
#pragma unroll
            for (int s = 0; s < RR; ++s) v[c][s] = src[s * PER];
            if constexpr (LNS > 0) {
                const int jm = j & (NS - 1);
#pragma unroll
                for (int s = 1; s < RR; ++s) v[c][s] = cmul(v[c][s], W[(jm * s) << (kRowLog - LNS - LR)]);
            }
            dft_reg<RR, false>(v[c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < RND; ++c) {
        const int J = tid + c * kThr;
        if (J < JOBS) {
            const int r = J / PER, j = J % PER;
            float2* dst = C + r * kRowStride + ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
#pragma unroll
            for (int s = 0; s < RR; ++s) dst[s * NS] = v[c][s];
        }
    }
    __syncthreads();
}

template <int RL>
__global__ __launch_bounds__(kThr) void upper_real_kernel(const float* __restrict__ x, float2* __restrict__ Y,
                                                          PassGeom geo, const float2* __restrict__ tab,
                                                          const float2* __restrict__ rowtw) {
    using S = RealUpperShape<RL>;
    constexpr int R = S::R, NR = S::NR;
    extern __shared__ float2 lds[];
    float2* C = lds;                              // NR rows
    float2* W = lds + NR * kRowStride;            // w_1024^e
    const int64_t L = (int64_t)R * kRow;
    const int64_t blk = blockIdx.x;
    const int64_t gwin = blk / S::WPW;
    const int g = (int)(blk - gwin * S::WPW);
    const int64_t b = gwin / geo.wps, Wi = gwin - b * geo.wps;
    const int64_t ib = (geo.in_sig ? geo.in_sig[b] : b * geo.in_stride) + Wi * L;
    const int64_t ob = (geo.out_sig ? geo.out_sig[b] : b * geo.out_stride) + Wi * L;
    const int tid = threadIdx.x;
    const int k0 = S::WHOLE ? 0 : 16 * g;        // first row's k2

    for (int e = tid; e < kRow; e += kThr) W[e] = tab[e << 2];
    // ---- column DFTs of columns na, nb (paired as one complex DFT), row twiddles ----
    {
        const int na = tid, nb = tid + kThr;
        const float* xa = x + ib + na;
        const float* xb = x + ib + nb;
        float2 ca[NR], cb[NR];
        if constexpr (S::WHOLE) {
            float2 z[R];
#pragma unroll
            for (int n2 = 0; n2 < R; ++n2) z[n2] = make_float2(xa[n2 * kRow], xb[n2 * kRow]);
            dft_reg<R, false>(z);
            split_pair<R, NR>(z, ca, cb);
        } else {
            constexpr int P = R / 16;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                float2 z[16], fa[16], fb[16];
#pragma unroll
                for (int bb = 0; bb < 16; ++bb) z[bb] = make_float2(xa[(r + P * bb) * kRow], xb[(r + P * bb) * kRow]);
                dft_reg<16, false>(z);
                split_pair<16, 16>(z, fa, fb);
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const float2 a = fa[q & 15], bq = fb[q & 15];
                    if (r == 0) {
                        ca[q] = a;
                        cb[q] = bq;
                    } else {
                        const float2 w = tab[((r * (k0 + q)) & (R - 1)) << (12 - RL)];     // w_R^{r(k0+q)}
                        ca[q] = cadd(ca[q], cmul(a, w));
                        cb[q] = cadd(cb[q], cmul(bq, w));
                    }
                }
            }
        }
        const float2* rt = rowtw + (int64_t)k0 * kRow;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            C[q * kRowStride + na] = cmul(ca[q], rt[q * kRow + na]);
            C[q * kRowStride + nb] = cmul(cb[q], rt[q * kRow + nb]);
        }
    }
    __syncthreads();
    row_step<4, NR, 0>(C, W, tid);
    row_step<16, NR, 2>(C, W, tid);
    row_step<16, NR, 6>(C, W, tid);
    // ---- outputs ----
    float2* yw = Y + ob;
    if constexpr (S::WHOLE) {
        // position k = k2 + R*k1; rows k2 <= R/2 direct, others mirrored
        for (int e = tid; e < (int)(L / 2); e += kThr) {
            const int k = 2 * e;
            const int k1 = k >> RL, k2 = k & (R - 1);
            float2 v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int q = k2 + u;
                v[u] = (q <= R / 2) ? C[q * kRowStride + k1] : cconj(C[(R - q) * kRowStride + (kRow - 1 - k1)]);
            }
            *(float4*)(yw + k) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        }
    } else {
        const int gm = S::NG - 1 - g;            // mirrored group
        for (int e = tid; e < kRow * 8; e += kThr) {
            const int k1 = e >> 3, kp = (e & 7) * 2;
            const float2 a = C[kp * kRowStride + k1], c = C[(kp + 1) * kRowStride + k1];
            *(float4*)(yw + k0 + kp + (int64_t)R * k1) = make_float4(a.x, a.y, c.x, c.y);
            // group gm, bin 16*gm + kp (+1) <- conj(row 16 - kp (-1) at 1023 - k1)
            const float2 ma = cconj(C[(16 - kp) * kRowStride + (kRow - 1 - k1)]);
            const float2 mc = cconj(C[(15 - kp) * kRowStride + (kRow - 1 - k1)]);
            *(float4*)(yw + 16 * gm + kp + (int64_t)R * k1) = make_float4(ma.x, ma.y, mc.x, mc.y);
        }
    }
}

template <int RL>
size_t real_upper_lds() {
    return sizeof(float2) * (size_t)(RealUpperShape<RL>::NR * kRowStride + kRow);
}
}  // namespace

bool upper_real_supported(int lg) { return lg >= 13 && lg <= 16; }

hipError_t launch_upper_real(const float* x, float2* Y, const PassGeom& g, const Twiddles& tw, hipStream_t s) {
    const int rl = g.lg - kRowLog;
    const float2* rowtw = tw.rowtw + row_twiddle_offset(g.lg);
#define MRDFT_UPR(RL_)                                                                                      \
    do {                                                                                                  \
        const size_t lds = real_upper_lds<RL_>();                                                          \
        const int64_t nblk = g.nwin * RealUpperShape<RL_>::WPW;                                            \
        if (nblk <= 0) return hipSuccess;                                                                  \
        (void)hipFuncSetAttribute((const void*)upper_real_kernel<RL_>,                                     \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                   \
        hipLaunchKernelGGL((upper_real_kernel<RL_>), dim3((unsigned)nblk), dim3(kThr), lds, s, x, Y, g,   \
                           tw.tile, rowtw);                                                                \
    } while (0)
    switch (rl) {
        case 3: MRDFT_UPR(3); break;
        case 4: MRDFT_UPR(4); break;
        case 5: MRDFT_UPR(5); break;
        case 6: MRDFT_UPR(6); break;
        default: return hipErrorInvalidValue;
    }
#undef MRDFT_UPR
    return hipGetLastError();
}

}  // namespace mrdft
