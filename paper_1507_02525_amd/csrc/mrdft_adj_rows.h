// Adjoint of the levels above the tile (12..16), in two phases.
//
// For a window of L = R * 256 points, the level's adjoint (conjugate
// transpose of the window DFT of eq. (1)) factors as
//
//     g[n1 + 256 n2] = sum_{k2} w_R^{-n2 k2} B[k2][n1],
//     B[k2][n1]      = w_L^{-n1 k2} sum_{k1} gY[k2 + R k1] w_256^{-n1 k1}.
//
// * Rows phase: piece g takes the rows k2 = 16g .. 16g+15 (16 consecutive
//   gradient values, 128 bytes, per k1), runs their conjugate 256-point DFTs
//   in LDS and writes B rows to a scratch block laid out like the level.
// * Columns phase: for 16 consecutive columns n1 of a region of up to 2^16
//   samples, the conjugate R-point DFTs over k2 of every level 12..16 that
//   covers the region run in LDS, their sum stays in registers, and gx is
//   updated once (the tiles wrote the levels below before).
#pragma once
#include <type_traits>

#include "mrdft_device.h"
#include "mrdft_rows_c64.h"

namespace mrdft {

constexpr int kAdjRegionLog = 16;                    // columns phase region: up to 2^16 samples
constexpr int kAdjColsPoints = 4096;                 // 16 columns x 2^16 / 256 rows

// One radix-16 conjugate Stockham step over the 16 rows of a rows piece.
template <int LNS>
__device__ __forceinline__ void adj_rows_step(CRowsLds& S, int tid) {
    constexpr int NS = 1 << LNS;
    const int r = tid >> 4, j = tid & 15;
    float2 v[16];
    const float2* src = S.C + r * kRowsStride;
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = src[rpad(j + 16 * s)];
    if constexpr (LNS > 0) {
        const int jm = j & (NS - 1);
#pragma unroll
        for (int s = 1; s < 16; ++s) v[s] = cmulc(v[s], S.T[(jm * s) << (kRowsLog - LNS - 4)]);
    }
    dft_reg<16, true>(v);
    __syncthreads();
    float2* dst = S.C + r * kRowsStride;
    const int base = ((j >> LNS) << (LNS + 4)) + (j & (NS - 1));
#pragma unroll
    for (int s = 0; s < 16; ++s) dst[rpad(base + s * NS)] = v[s];
    __syncthreads();
}

// Rows piece g of one window of level lg = RL + 8.
//   gyw   : the window's gradient at its level       scw: the window's scratch block (L values)
//   rowtw : this level's row twiddles rowtw[k2 * 256 + n1] = w_L^{n1 k2}
// HALF: gyw holds the window's packed half spectrum (L/2 slots, half_bin with scale hsc).
template <int RL, bool HALF = false>
__device__ __forceinline__ void adj_rows_body(CRowsLds& S, const float2* __restrict__ gyw, float2* __restrict__ scw,
                                              int g, const float2* __restrict__ t4096,
                                              const float2* __restrict__ rowtw, int tid, float hsc = 0.5f) {
    constexpr int R = 1 << RL;
    constexpr int64_t L = (int64_t)R * kRowsN;
    const int k0 = 16 * g;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * kRowsThreads;
        const int k1 = e >> 3, kp = (e & 7) * 2;
        float4 v;
        if constexpr (HALF) {
            const float2 a = half_bin(gyw, k0 + kp + (int64_t)R * k1, L, hsc);
            const float2 b = half_bin(gyw, k0 + kp + 1 + (int64_t)R * k1, L, hsc);
            v = make_float4(a.x, a.y, b.x, b.y);
        } else {
            v = *(const float4*)(gyw + k0 + kp + (int64_t)R * k1);
        }
        S.C[kp * kRowsStride + rpad(k1)] = make_float2(v.x, v.y);
        S.C[(kp + 1) * kRowsStride + rpad(k1)] = make_float2(v.z, v.w);
    }
    __syncthreads();
    adj_rows_step<0>(S, tid);
    adj_rows_step<4>(S, tid);
    const int n1 = tid;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k2 = k0 + q;
        scw[k2 * kRowsN + n1] = cmulc(S.C[q * kRowsStride + rpad(n1)], rowtw[k2 * kRowsN + n1]);
    }
}

// Rows piece g (g < R/32) of one window of level lg = RL + 8 (13 <= lg <= 16)
// for real output.  Only Re(A^H gY) is wanted, which is A^H h for the
// Hermitian part h[k] = (gY[k] + conj(gY[L - k])) / 2, so B is Hermitian in
// k2 as well (B[R - k2][n1] = conj(B[k2][n1])) and only its rows
// k2 = 0 .. R/2 are formed: piece g takes the rows 16g .. 16g+16.  The
// partners of rows 16g+1 .. 16g+16 are the 16 rows of group R/16 - 1 - g at
// k1' = 255 - k1 (the mirror of the forward's Hermitian store); the partner of
// row 16g is row R - 16g at 255 - k1, or row 0 at -k1 mod 256 when g = 0.
// Rows 16g .. 16g+15 are written, and row R/2 by the last piece.
// HALF: gyw holds the window's packed half spectrum, whose half_bin reading
// (scale hsc) is Hermitian already: h is read directly.
template <int RL, bool HALF = false>
__device__ __forceinline__ void adj_rows_real_body(RowsLds& S, const float2* __restrict__ gyw,
                                                   float2* __restrict__ scw, int g, const float2* __restrict__ t4096,
                                                   const float2* __restrict__ rowtw, int tid, float hsc = 0.5f) {
    constexpr int R = 1 << RL, NG = R / 16;
    static_assert(NG >= 2, "levels 13..16");
    const int k0 = 16 * g;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
    if constexpr (HALF) {
        constexpr int64_t L = (int64_t)R * kRowsN;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int c = e >> 3, kp = (e & 7) * 2;
            S.C[kp * kRowsStride + rpad(c)] = half_bin(gyw, k0 + kp + (int64_t)R * c, L, hsc);
            S.C[(kp + 1) * kRowsStride + rpad(c)] = half_bin(gyw, k0 + kp + 1 + (int64_t)R * c, L, hsc);
        }
        S.C[16 * kRowsStride + rpad(tid)] =
            g == NG / 2 - 1 ? half_bin(gyw, k0 + 16 + (int64_t)R * tid, L, hsc) : make_float2(0.0f, 0.0f);
        __syncthreads();
    } else {
        const int gm = NG - 1 - g;
        float4 dv[8], pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int k1 = e >> 3, kp = (e & 7) * 2;
            dv[u] = *(const float4*)(gyw + k0 + kp + (int64_t)R * k1);          // rows k0 + kp, +1 at k1
            pv[u] = *(const float4*)(gyw + 16 * gm + kp + (int64_t)R * k1);     // rows 16 gm + kp, +1 at k1
        }
        const int k1 = tid;
        // row k0 + 16 (stored by the last piece only: the others skip its
        // 256 scattered loads and transform zeros there)
        const float2 d16 = g == NG / 2 - 1 ? gyw[k0 + 16 + (int64_t)R * k1] : make_float2(0.0f, 0.0f);
        const float2 p0 = gyw[((R - k0) & (R - 1)) + (int64_t)R * k1];              // partner of row k0
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int c = e >> 3, kp = (e & 7) * 2;
            S.C[kp * kRowsStride + rpad(c)] = make_float2(dv[u].x, dv[u].y);
            S.C[(kp + 1) * kRowsStride + rpad(c)] = make_float2(dv[u].z, dv[u].w);
        }
        S.C[16 * kRowsStride + rpad(k1)] = d16;
        __syncthreads();
        // h = (direct + conj(partner)) / 2; every slot is updated by one thread
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int c = 255 - (e >> 3), kp = (e & 7) * 2;
            float2* a = &S.C[(16 - kp) * kRowsStride + rpad(c)];                   // partner row 16 gm + kp
            float2* b = &S.C[(15 - kp) * kRowsStride + rpad(c)];                   // partner row 16 gm + kp + 1
            *a = make_float2(0.5f * (a->x + pv[u].x), 0.5f * (a->y - pv[u].y));
            *b = make_float2(0.5f * (b->x + pv[u].z), 0.5f * (b->y - pv[u].w));
        }
        {
            const int c = g == 0 ? ((kRowsN - k1) & (kRowsN - 1)) : kRowsN - 1 - k1;
            float2* a = &S.C[rpad(c)];
            *a = make_float2(0.5f * (a->x + p0.x), 0.5f * (a->y - p0.y));
        }
        __syncthreads();
    }
    rows_step<0, true>(S, tid);
    rows_step<4, true>(S, tid);
    __syncthreads();                                  // row 16 (wave 0) before the outputs
    const int n1 = tid;
    const int nq = (g == NG / 2 - 1) ? 17 : 16;       // row R/2 by the last piece
#pragma unroll
    for (int q = 0; q < 17; ++q) {
        if (q < nq) {
            const int k2 = k0 + q;
            scw[k2 * kRowsN + n1] = cmulc(S.C[q * kRowsStride + rpad(n1)], rowtw[k2 * kRowsN + n1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Columns phase.

struct AdjColsLds {
    float2 V[kAdjColsPoints + kAdjColsPoints / 16];   // FFTs of one level, padded
    float2 T[kRowsN];                                 // w_256^e
};

__device__ __forceinline__ int cpad(int i) { return i + (i >> 4); }

// One conjugate Stockham step of radix RR over the first NP points of V (NP / R
// FFTs of R points, FFT f at f * R), span 2^LNS; NP / RR jobs over 256 threads.
template <int RR, int R, int LNS, int NP = kAdjColsPoints>
__device__ __forceinline__ void adj_cols_step(AdjColsLds& S, int tid) {
    constexpr int LR = (RR == 2) ? 1 : (RR == 4) ? 2 : (RR == 8) ? 3 : 4;
    constexpr int PER = R / RR;
    constexpr int JOBS = NP / RR;
    constexpr int JPT = (JOBS + kRowsThreads - 1) / kRowsThreads;
    constexpr int NS = 1 << LNS;
    float2 v[JPT][RR];
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kRowsThreads;
        if (JOBS % kRowsThreads && J >= JOBS) break;
        const int f = J / PER, j = J % PER;
#pragma unroll
        for (int s = 0; s < RR; ++s) v[c][s] = S.V[cpad(f * R + j + s * PER)];
        if constexpr (LNS > 0) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int s = 1; s < RR; ++s) v[c][s] = cmulc(v[c][s], S.T[(jm * s) << (kRowsLog - LNS - LR)]);
        }
        dft_reg<RR, true>(v[c]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kRowsThreads;
        if (JOBS % kRowsThreads && J >= JOBS) break;
        const int f = J / PER, j = J % PER;
        const int base = f * R + ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
#pragma unroll
        for (int s = 0; s < RR; ++s) S.V[cpad(base + s * NS)] = v[c][s];
    }
    __syncthreads();
}

// R-point conjugate DFTs (R = 16 .. 256): a first step of radix R/16 (if R > 16),
// then radix 16.
template <int R, int NP = kAdjColsPoints>
__device__ __forceinline__ void adj_cols_fft(AdjColsLds& S, int tid) {
    if constexpr (R == 16) {
        adj_cols_step<16, R, 0, NP>(S, tid);
    } else {
        constexpr int R0 = R / 16;
        constexpr int L0 = (R0 == 2) ? 1 : (R0 == 4) ? 2 : (R0 == 8) ? 3 : 4;
        adj_cols_step<R0, R, 0, NP>(S, tid);
        adj_cols_step<16, R, L0, NP>(S, tid);
    }
}

// One level lg = RL + 8 of a columns job: region of `region` samples (a
// multiple of L), columns c0 .. c0+15; acc[s] is the contribution to the
// thread's gx values at region row rho = (tid >> 4) + 16 s, column tid & 15.
//   scr : the scratch block of this level at the region's first sample
// HERM (real output, levels 13..16): only the rows k2 <= R/2 are in the
// scratch; the others are their conjugates (B[R - k2] = conj(B[k2])).  The
// conjugate DFT of such a column is real, so columns c and c + 8 share one
// complex FFT of Z = B_c + i B_{c+8}: its real part is the first column's
// result, its imaginary part the second's (half the FFTs).
template <int RL, bool REAL, class ACC>
__device__ __forceinline__ void adj_cols_level(AdjColsLds& S, const float2* __restrict__ scr, int region_log, int c0,
                                               ACC* acc, int tid) {
    constexpr int R = 1 << RL, L = R * kRowsN;
    constexpr bool HERM = REAL && RL >= 5;
    const int nwin = 1 << (region_log - RL - kRowsLog);          // windows of this level in the region
    const int rows = nwin * R;                                    // = region / 256
    if constexpr (HERM) {
        // FFT f = w * 8 + pc holds Z[k2] = B[w][k2][c0 + pc] + i B[w][k2][c0 + pc + 8]
        typedef float nt2 __attribute__((ext_vector_type(2)));
        constexpr int kPer = kAdjColsPoints / 2 / kRowsThreads;  // (pair, row) items per thread
        float2 va[kPer], vb[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * kRowsThreads;
            const int pc = e & 7, rr = e >> 3;                    // rr = w * R + k2
            const int w = rr / R, k2 = rr % R;
            if (e < rows * 8 && k2 <= R / 2) {
                const float2* q = scr + (int64_t)w * L + k2 * kRowsN + c0 + pc;
                const nt2 a = __builtin_nontemporal_load((const nt2*)q);
                const nt2 b = __builtin_nontemporal_load((const nt2*)(q + 8));
                va[u] = make_float2(a.x, a.y);
                vb[u] = make_float2(b.x, b.y);
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + u * kRowsThreads;
            const int pc = e & 7, rr = e >> 3;
            const int w = rr / R, k2 = rr % R;
            if (e < rows * 8 && k2 <= R / 2) {
                const float2 a = va[u], b = vb[u];
                const int f0 = (w * 8 + pc) * R;
                if (k2 == 0 || k2 == R / 2) {
                    S.V[cpad(f0 + k2)] = make_float2(a.x, b.x);   // real rows: their real parts
                } else {
                    S.V[cpad(f0 + k2)] = make_float2(a.x - b.y, a.y + b.x);
                    S.V[cpad(f0 + R - k2)] = make_float2(a.x + b.y, b.x - a.y);   // conj(B_c) + i conj(B_c+8)
                }
            }
        }
        __syncthreads();
        adj_cols_fft<R, kAdjColsPoints / 2>(S, tid);
        const int col = tid & 15;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int rho = (tid >> 4) + 16 * s;
            if (rho < rows) {
                const int w = rho / R, n2 = rho % R;
                const float2 o = S.V[cpad((w * 8 + (col & 7)) * R + n2)];
                acc[s] += col < 8 ? o.x : o.y;
            }
        }
        __syncthreads();
        return;
    }
    // load B[w][k2][c0 + col] (128-byte chunks) into FFT f = w * 16 + col, point
    // k2; all of a thread's loads are issued before the first LDS store.  The
    // scratch is read once: non-temporal loads (complex gradients of
    // 64 x 2^16: this launch 77 -> 67 us)
    typedef float nt2 __attribute__((ext_vector_type(2)));
    constexpr int kPer = kAdjColsPoints / kRowsThreads;
    float2 v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kRowsThreads;
        const int col = e & 15, rr = e >> 4;                      // rr = w * R + k2
        const int w = rr / R, k2 = rr % R;
        if (e < rows * 16 && (!HERM || k2 <= R / 2)) {
            const nt2 t = __builtin_nontemporal_load((const nt2*)(scr + (int64_t)w * L + k2 * kRowsN + c0 + col));
            v[u] = make_float2(t.x, t.y);
        }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + u * kRowsThreads;
        const int col = e & 15, rr = e >> 4;
        const int w = rr / R, k2 = rr % R;
        if (e < rows * 16 && (!HERM || k2 <= R / 2)) {
            S.V[cpad((w * 16 + col) * R + k2)] = v[u];
            if (HERM && k2 > 0 && k2 < R / 2) S.V[cpad((w * 16 + col) * R + R - k2)] = cconj(v[u]);
        }
    }
    __syncthreads();
    // all 4096 points go through the steps; with a region below 2^16 the FFTs
    // past rows * 16 points hold stale values and are never read
    adj_cols_fft<R>(S, tid);
    const int col = tid & 15;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int rho = (tid >> 4) + 16 * s;
        if (rho < rows) {
            const int w = rho / R, n2 = rho % R;
            const float2 v = S.V[cpad((w * 16 + col) * R + n2)];
            if constexpr (REAL) acc[s] += v.x;
            else acc[s] = cadd(acc[s], v);
        }
    }
    __syncthreads();
}

}  // namespace mrdft
