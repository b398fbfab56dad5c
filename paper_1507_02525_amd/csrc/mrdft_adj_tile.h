// Adjoint tile: levels 11..1 of a 2048-sample tile, real or complex gx.
//
// The adjoint of eq. (1) is gx = sum_i A_i^H gY^(i).  It is computed with
// the transpose of the recurrence of Section 3 (eq. (4)), top level down:
// with G_i the gradient reaching level i (G_11 = gY^(11)),
// * odd bins (transpose of V^(i), D^(i), F^(i), eq. (3)): the conjugate
//   L/2-point DFT of G_i[w][2k+1] gives d[q]; d[q] w_L^{-q} is added to
//   gx[wL + q] and subtracted from gx[wL + q + L/2];
// * even bins (transpose of U^(i), eq. (2)): G_i[w][2k] is added to bin k of
//   both child windows, G_{i-1} = gY^(i-1) + U^T G_i;
// * level 1: gx[2w] += g0 + g1, gx[2w+1] += g0 - g1.
// Levels 4..9 (windows inside one wave's 512 samples) run wave by wave: the
// conjugate DFT of the odd bins goes through the cross-lane FFT of
// mrdft_xlane.h (conjugated in and out) and one LDS pass back to natural
// order, with no workgroup barrier; the other levels run as Stockham steps
// on the natural-order bins.  Only Re(gx) is accumulated for a real signal
// (the real part is linear).  256 threads; 28 KB of LDS (real gx) or 36 KB
// (complex gx).
#pragma once
#include "mrdft_device.h"
#include "mrdft_internal.h"
#include "mrdft_tile_c64.h"
#include "mrdft_xlane.h"

namespace mrdft {

template <bool REAL>
struct AdjTileLds {
    float2 P[kCT];                                   // G_i; the FFT work space overlays it
    typename std::conditional<REAL, float, float2>::type A[kCT];   // gx accumulator
    float2 Q[kCT / 4];                               // w_2048^e, e < 512 (swizzled)
    float2 H[REAL ? kCT / 2 : 1];                    // packed input: one level's slots of the tile
};

// conj(w_{2^lg}^e)
__device__ __forceinline__ float2 adj_tw(const float2* Q, int lg, int e) { return cconj(TwQ2048{Q}(lg, e)); }

// One radix-R conjugate Stockham step over the 1024 points of F.
template <int R, int M, int LNS>
__device__ __forceinline__ void adj_step(float2* F, const float2* Q, int tid) {
    constexpr int LR = (R == 2) ? 1 : 2;
    constexpr int PER = M / R;
    constexpr int JPT = kCT / 2 / R / kCThreads;
    constexpr int NS = 1 << LNS;
    float2 v[JPT][R];
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kCThreads;
        const int w = J / PER, j = J % PER;
#pragma unroll
        for (int s = 0; s < R; ++s) v[c][s] = F[cfpad(w * M + j + s * PER)];
        if constexpr (LNS > 0) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int s = 1; s < R; ++s) v[c][s] = cmul(v[c][s], adj_tw(Q, LNS + LR, jm * s));
        }
        dft_reg<R, true>(v[c]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kCThreads;
        const int w = J / PER, j = J % PER;
        const int base = w * M + ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
#pragma unroll
        for (int s = 0; s < R; ++s) F[cfpad(base + s * NS)] = v[c][s];
    }
    __syncthreads();
}

template <int M, int LNS, int LM>
struct AdjSteps {
    static __device__ __forceinline__ void run(float2* F, const float2* Q, int tid) {
        if constexpr (LNS < LM) {
            adj_step<((LM - LNS) & 1) ? 2 : 4, M, LNS>(F, Q, tid);
            AdjSteps<M, LNS + (((LM - LNS) & 1) ? 1 : 2), LM>::run(F, Q, tid);
        }
    }
};

// Orders one wave's LDS accesses (the compiler may not move them across).
__device__ __forceinline__ void wave_sync_c() { ct_wave_sync(); }

template <bool REAL>
__device__ __forceinline__ void adj_acc(AdjTileLds<REAL>& S, int i, float2 v, bool add) {
    if constexpr (REAL) {
        if (add) S.A[i] += v.x;
        else S.A[i] = v.x;
    } else {
        S.A[i] = add ? cadd(S.A[i], v) : v;
    }
}

// Level I (2 <= I <= 11): P holds G_I on entry and G_{I-1} on exit.
//   gyl : gY of level I-1 at this tile (level-major, complex64; HALF: the
//         packed half spectra, 2^(I-2) slots per window, read by half_bin)
template <int I, bool REAL, bool HALF = false>
__device__ __forceinline__ void adj_level(AdjTileLds<REAL>& S, const float2* __restrict__ gyl, int tid, bool have,
                                          float hsc) {
    constexpr int L = 1 << I, M = L / 2, LM = I - 1;
    constexpr int PPT = kCT / 2 / kCThreads;            // (w, k) jobs per thread
    constexpr bool FIRST = (I == kCTLog);               // A not yet written
    float2* F = S.P;
    float2 e[PPT], nxt0[PPT], nxt1[PPT];
    if constexpr (HALF) {
        // the level's packed slots of this tile (contiguous) into H, coalesced;
        // read back through half_bin after the next barrier
#pragma unroll
        for (int r = 0; r < kCT / 4 / kCThreads; ++r) {
            const int p = tid + r * kCThreads;
            *(float4*)(S.H + 2 * p) = have ? ((const float4*)gyl)[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kCThreads;               // = w * M + k
        const int w = J / M, k = J % M;
        // level I-1 gradient inputs of the two children (loaded early; zero
        // for a level outside the plan's range)
        if constexpr (!HALF) {
            nxt0[c] = have ? gyl[2 * w * M + k] : make_float2(0.0f, 0.0f);
            nxt1[c] = have ? gyl[(2 * w + 1) * M + k] : make_float2(0.0f, 0.0f);
        }
        e[c] = S.P[2 * J];
    }
    float2 d[PPT];
#pragma unroll
    for (int c = 0; c < PPT; ++c) d[c] = S.P[2 * (tid + c * kCThreads) + 1];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PPT; ++c) F[cfpad(tid + c * kCThreads)] = d[c];
    __syncthreads();
    AdjSteps<M, 0, LM>::run(F, S.Q, tid);
    // untwiddle and scatter: +d w_L^{-q} at wL + q, - at wL + q + M
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kCThreads;
        const int w = J / M, q = J % M;
        const float2 t = cmul(F[cfpad(J)], adj_tw(S.Q, I, q));
        adj_acc<REAL>(S, w * L + q, t, !FIRST);
        adj_acc<REAL>(S, w * L + q + M, make_float2(-t.x, -t.y), !FIRST);
    }
    __syncthreads();
    // G_{I-1} = gY^(I-1) + even bins of G_I on both children
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kCThreads;
        const int w = J / M, k = J % M;
        if constexpr (HALF) {
            nxt0[c] = half_bin(S.H + 2 * w * (M / 2), k, M, hsc);
            nxt1[c] = half_bin(S.H + (2 * w + 1) * (M / 2), k, M, hsc);
        }
        S.P[2 * w * M + k] = cadd(nxt0[c], e[c]);
        S.P[(2 * w + 1) * M + k] = cadd(nxt1[c], e[c]);
    }
    __syncthreads();
}

// Level I (4 <= I <= 9), wave by wave: wave v owns samples and A entries
// [512 v, 512 v + 512), pairs [256 v, 256 v + 256) of P (P[512 v, 512 v +
// 512)), bins [512 v, 512 v + 512) of gY at every level and (HALF) packed
// slots [256 v, 256 v + 256) of H.  P holds G_I on entry and G_{I-1} on exit.
template <int I, bool REAL, bool HALF>
__device__ __forceinline__ void adj_level_wave(AdjTileLds<REAL>& S, const float2* __restrict__ gyl, int tid,
                                               bool have, float hsc, const XLane& ln) {
    constexpr int L = 1 << I, M = L / 2, n = I - 1;
    constexpr int NQ = n - 2;                        // FFT-index bits held by the lane
    const int v = tid >> 6, lane = tid & 63;
    float2* Pb = S.P + 512 * v;
    if constexpr (HALF) {
        // the wave's packed slots of level I-1 into H (coalesced), read back
        // through half_bin below
        float2* Hb = S.H + 256 * v;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int p = 64 * c + lane;
            *(float4*)(Hb + 2 * p) = have ? ((const float4*)(gyl + 256 * v))[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
    }
    // even bins of the wave's pairs J = 64 c + lane (window J / M, bin 2k) and
    // the children's gradient inputs of level I-1
    float2 e[4], nxt0[4], nxt1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = 64 * c + lane;
        const int w = J / M, k = J % M;
        if constexpr (!HALF) {
            nxt0[c] = have ? gyl[512 * v + 2 * w * M + k] : make_float2(0.0f, 0.0f);
            nxt1[c] = have ? gyl[512 * v + (2 * w + 1) * M + k] : make_float2(0.0f, 0.0f);
        }
        e[c] = Pb[2 * J];
    }
    // odd bins in the cross-lane input layout (bin plow + 2^NQ r of window wl),
    // conjugated: conj(DFT(conj(d))) is the conjugate DFT of d
    const int plow = ln.c & ((1 << (NQ < 6 ? NQ : 6)) - 1);
    const int wl = NQ < 6 ? ln.c >> NQ : 0;
    float2 a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = cconj(Pb[2 * (wl * M + plow + (r << NQ)) + 1]);
    xl_fft<n>(a, ln, TwQ2048{S.Q});
    wave_sync_c();                                   // P reads before the overlaying writes
#pragma unroll
    for (int r = 0; r < 4; ++r) Pb[xl_fsw(xl_pos<n>(ln.c, r))] = cconj(a[r]);
    wave_sync_c();
    float2 t[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] = Pb[xl_fsw(64 * c + lane)];
    // untwiddle and scatter: +d w_L^{-q} at wL + q, - at wL + q + M
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int pq = 64 * c + lane;
        const int w = pq / M, q = pq % M;
        const float2 tt = cmul(t[c], adj_tw(S.Q, I, q));
        adj_acc<REAL>(S, 512 * v + w * L + q, tt, true);
        adj_acc<REAL>(S, 512 * v + w * L + q + M, make_float2(-tt.x, -tt.y), true);
    }
    wave_sync_c();                                   // scratch reads before the new G
    // G_{I-1} = gY^(I-1) + even bins of G_I on both children
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = 64 * c + lane;
        const int w = J / M, k = J % M;
        if constexpr (HALF) {
            nxt0[c] = half_bin(S.H + 256 * v + 2 * w * (M / 2), k, M, hsc);
            nxt1[c] = half_bin(S.H + 256 * v + (2 * w + 1) * (M / 2), k, M, hsc);
        }
        Pb[2 * w * M + k] = cadd(nxt0[c], e[c]);
        Pb[(2 * w + 1) * M + k] = cadd(nxt1[c], e[c]);
    }
    // the next level reads its own quarter (wave levels), or all of P
    if constexpr (I == 4) __syncthreads();
    else wave_sync_c();
}

template <int I, bool REAL, bool HALF>
struct AdjLevels {
    static __device__ __forceinline__ void run(AdjTileLds<REAL>& S, const float2* __restrict__ gy, int64_t ls,
                                               int tid, LevelRange lv, float hsc, const XLane& ln) {
        if constexpr (I >= 2) {
            if constexpr (I >= 4 && I <= kCtWaveMaxLog)
                adj_level_wave<I, REAL, HALF>(S, gy + (int64_t)(I - 2) * ls, tid, lv.in(I - 1), hsc, ln);
            else
                adj_level<I, REAL, HALF>(S, gy + (int64_t)(I - 2) * ls, tid, lv.in(I - 1), hsc);
            AdjLevels<I - 1, REAL, HALF>::run(S, gy, ls, tid, lv, hsc, ln);
        }
    }
};

// One tile: gy at the tile's level-1 gradient (level i at gy + (i-1) ls),
// gx at the tile's first sample (float for REAL, float2 otherwise); gx is
// overwritten.  HALF (real output): gy holds packed half spectra, the tile's
// 1024 slots per level, read by half_bin with scale hsc.
template <bool REAL, bool HALF = false>
__device__ __forceinline__ void adj_tile_body(AdjTileLds<REAL>& S, const float2* __restrict__ gy, void* __restrict__ gx,
                                              int64_t ls, const float2* __restrict__ t4096, int tid, LevelRange lv,
                                              float hsc = 0.5f) {
    for (int e = tid; e < kCT / 4; e += kCThreads) S.Q[cqswz(e)] = t4096[2 * e];
    {
        const float2* g11 = gy + (int64_t)(kCTLog - 1) * ls;
        const bool have = lv.in(kCTLog);
        if constexpr (HALF) {
            // the top level's 1024 packed slots into H, then unpacked into P
#pragma unroll
            for (int r = 0; r < kCT / 4 / kCThreads; ++r) {
                const int p = tid + r * kCThreads;
                *(float4*)(S.H + 2 * p) = have ? ((const float4*)g11)[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kCT / 2 / kCThreads; ++r) {
                const int p = tid + r * kCThreads;
                const float2 a = half_bin(S.H, 2 * p, kCT, hsc), b = half_bin(S.H, 2 * p + 1, kCT, hsc);
                *(float4*)(S.P + 2 * p) = make_float4(a.x, a.y, b.x, b.y);
            }
        } else {
#pragma unroll
            for (int r = 0; r < kCT / 2 / kCThreads; ++r) {
                const int p = tid + r * kCThreads;
                *(float4*)(S.P + 2 * p) = have ? ((const float4*)g11)[p] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
    }
    __syncthreads();
    const XLane ln = xl_lane(tid & 63, TwQ2048{S.Q});
    AdjLevels<kCTLog, REAL, HALF>::run(S, gy, ls, tid, lv, hsc, ln);
    // level 1: windows of two
#pragma unroll
    for (int r = 0; r < kCT / 2 / kCThreads; ++r) {
        const int w = tid + r * kCThreads;
        const float2 g0 = S.P[2 * w], g1 = S.P[2 * w + 1];
        adj_acc<REAL>(S, 2 * w, cadd(g0, g1), true);
        adj_acc<REAL>(S, 2 * w + 1, csub(g0, g1), true);
    }
    __syncthreads();
    if constexpr (REAL) {
        float2* o = (float2*)gx;                      // real signals start at even samples (8-byte aligned)
#pragma unroll
        for (int r = 0; r < kCT / 2 / kCThreads; ++r) {
            const int p = tid + r * kCThreads;
            o[p] = make_float2(S.A[2 * p], S.A[2 * p + 1]);
        }
    } else {
        float4* o = (float4*)gx;
#pragma unroll
        for (int r = 0; r < kCT / 2 / kCThreads; ++r) {
            const int p = tid + r * kCThreads;
            o[p] = make_float4(S.A[2 * p].x, S.A[2 * p].y, S.A[2 * p + 1].x, S.A[2 * p + 1].y);
        }
    }
}

}  // namespace mrdft
