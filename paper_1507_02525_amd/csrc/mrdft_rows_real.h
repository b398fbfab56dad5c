// Levels above the tile for real input, one workgroup-sized piece at a time.
//
// Level lg is the L-point DFT (L = 2^lg) of every window (Section 2, eq. (1)).
// With L = R * 256, n = n1 + 256 n2 and k = k2 + R k1 (n1, k1 < 256;
// n2, k2 < R) a window's DFT factors as
//
//     Y[k2 + R k1] = sum_{n1} w_256^{n1 k1} ( w_L^{n1 k2} C[n1][k2] ),
//     C[n1][k2]    = sum_{n2} x[n1 + 256 n2] w_R^{n2 k2}          (column DFTs).
//
// The window is real, so Y[L - k] = conj(Y[k]): row R - k2 at k1 equals
// conj(row k2 at 255 - k1), and only rows k2 <= R/2 are transformed.  Rows
// come in groups of 16 (NG = R/16 groups); piece g < NG/2 transforms the 17
// rows 16g .. 16g + 16 and writes group g directly and group NG-1-g (the
// mirrors of rows 16g+16 .. 16g+1).  Every output chunk is 16 consecutive
// complex values (128 bytes).
//
// Column DFTs are formed straight from x (R/16 sub-DFTs of 16 points, two real
// sub-sequences per complex DFT); the 256-point row FFTs run in LDS (radix
// 16, two Stockham steps).  256 threads, 39 KB of LDS.
#pragma once
#include "mrdft_device.h"

namespace mrdft {

constexpr int kRowsLog = 8;
constexpr int kRowsN = 1 << kRowsLog;       // row FFT length
constexpr int kRowsMax = 17;                // rows held by one piece
constexpr int kRowsStride = 273;            // padded row stride (float2)
constexpr int kRowsThreads = 256;
constexpr int kRowsMinLevel = 13;
constexpr int kRowsMaxLevel = 16;
// Word 3 of a raw buffer descriptor: 32-bit data format (raw loads need a
// non-zero data format).
constexpr int kBufferWord3 = 0x00020000;

struct RowsLds {
    float2 C[kRowsMax * kRowsStride];       // 17 rows of 256 points, padded
    float2 T[kRowsN];                       // w_256^e
};

// One spare element after every 16: the radix-16 Stockham accesses at stride
// 16 then fall on distinct banks.
__device__ __forceinline__ int rpad(int i) { return i + (i >> 4); }

// One radix-16 job of a Stockham step with span 2^LNS (LNS = 0 or 4) on row
// r: 16 points j + 16 s in, positions (j / NS) * 16 NS + (j mod NS) + s NS out.
// INV: the conjugate transform (the adjoint's rows).
template <int LNS, bool INV = false>
__device__ __forceinline__ void rows_job_load(const RowsLds& S, int r, int j, float2* v) {
    constexpr int NS = 1 << LNS;
    const float2* src = S.C + r * kRowsStride;
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = src[rpad(j + 16 * s)];
    if constexpr (LNS > 0) {
        const int jm = j & (NS - 1);
#pragma unroll
        for (int s = 1; s < 16; ++s) {
            const float2 w = S.T[(jm * s) << (kRowsLog - LNS - 4)];
            v[s] = INV ? cmulc(v[s], w) : cmul(v[s], w);
        }
    }
    dft_reg<16, INV>(v);
}
template <int LNS>
__device__ __forceinline__ void rows_job_store(RowsLds& S, int r, int j, const float2* v) {
    constexpr int NS = 1 << LNS;
    float2* dst = S.C + r * kRowsStride;
    const int base = ((j >> LNS) << (LNS + 4)) + (j & (NS - 1));
#pragma unroll
    for (int s = 0; s < 16; ++s) dst[rpad(base + s * NS)] = v[s];
}

// Orders LDS accesses of the lanes of one wave (LDS executes a wave's
// instructions in issue order; this only keeps the compiler from moving them).
__device__ __forceinline__ void rows_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One radix-16 Stockham step: rows 0..15 with one job per thread, then row 16
// by lanes 0..15 of wave 0 alone (no other wave touches that row, so a wave
// sync separates its reads from its writes).
template <int LNS, bool INV = false>
__device__ __forceinline__ void rows_step(RowsLds& S, int tid) {
    {
        float2 v[16];
        rows_job_load<LNS, INV>(S, tid >> 4, tid & 15, v);
        __syncthreads();
        rows_job_store<LNS>(S, tid >> 4, tid & 15, v);
        __syncthreads();
    }
    if (tid < 16) {
        float2 v[16];
        rows_job_load<LNS, INV>(S, 16, tid, v);
        rows_wave_sync();
        rows_job_store<LNS>(S, 16, tid, v);
        rows_wave_sync();
    }
}

// Column-combine factors of one level, per (piece g, pair s, row q):
//   u = (w_R^{2s k} - j w_R^{(2s+1) k}) / 2,  v = (w_R^{2s k} + j w_R^{(2s+1) k}) / 2,  k = 16 g + q,
// packed as float4 (u.x, u.y, v.x, v.y), index ((g * P/2 + s) * 17 + q).
__host__ __device__ constexpr int64_t rows_combine_offset(int lg) {
    return lg <= kRowsMinLevel ? 0
                               : rows_combine_offset(lg - 1) +
                                     (int64_t)(1 << (lg - 1 - kRowsMinLevel)) * (1 << (lg - 1 - 8 - 5)) * kRowsMax;
}
constexpr int64_t rows_combine_entries() { return rows_combine_offset(kRowsMaxLevel + 1); }

// Piece g of one window of level lg = RL + 8 (5 <= RL <= 8).
//   xw    : the window's first sample
//   yw    : the window's first output (level lg)
//   t4096 : w_4096^e, e < 4096 (FP32, rounded once from FP64)
//   rowtw : this level's row twiddles, rowtw[k2 * 256 + n1] = w_L^{n1 k2}
//   comb  : this level's column-combine factors (see rows_combine_offset)
// HALF: only bins k < L/2 (k1 < 128) are stored, with slot 0 = (Y[0], Y[L/2])
// (Y[L/2] is row 0 at k1 = 128).
template <int RL, bool RED = false, bool HALF = false>
__device__ __forceinline__ void rows_real_body(RowsLds& S, const float* __restrict__ xw, float2* __restrict__ yw,
                                               int g, const float2* __restrict__ t4096,
                                               const float2* __restrict__ rowtw, const float4* __restrict__ comb,
                                               int tid, const float* __restrict__ xsub = nullptr,
                                               double* norm = nullptr, float scale = 1.0f) {
    constexpr int R = 1 << RL, P = R / 16, NG = R / 16;
    static_assert(P >= 2 && P <= 16, "rows of 256 cover windows of 2^13 .. 2^16");
    const int k0 = 16 * g;
    const int n1 = tid;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
    // ---- column DFTs: C[k0 + q] = sum_r w_R^{r (k0 + q)} DFT16(x[n1 + 256 (r + P b)])[q mod 16] ----
    // Sub-sequences a = 2s and b = 2s+1 form one complex DFT Z; with
    // Zc = conj(Z[-q]) their transforms are (Z + Zc)/2 and -j (Z - Zc)/2, so the
    // pair contributes Z u + Zc v.
    // x is read through a buffer descriptor: every load shares one lane
    // offset and takes its column offset from a scalar register, so the
    // addresses cost no vector registers.  The next pair's samples load one
    // pair ahead.
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void*)xw, (short)0, R * kRowsN * (int)sizeof(float), kBufferWord3);
    const int vo = n1 * (int)sizeof(float);
    const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(xsub ? xsub : xw), (short)0, R * kRowsN * (int)sizeof(float), kBufferWord3);
    auto xload = [&](int n2) {
        const int so = n2 * kRowsN * (int)sizeof(float);
        float a = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, vo, so, 0));
        if (xsub) a -= __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(zr, vo, so, 0));   // x - xsub
        return a;
    };
    const float4* cb = comb + (int64_t)g * (P / 2) * kRowsMax;
    float2 acc[kRowsMax];
    float2 zn[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) zn[b] = make_float2(xload(P * b), xload(1 + P * b));
    auto pair = [&](int s, bool first) {
        float2 z[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) z[b] = zn[b];
        if (s + 1 < P / 2) {
#pragma unroll
            for (int b = 0; b < 16; ++b) zn[b] = make_float2(xload(2 * s + 2 + P * b), xload(2 * s + 3 + P * b));
        }
        dft_reg<16, false>(z);
#pragma unroll
        for (int q = 0; q < kRowsMax; ++q) {
            const int kk = q & 15, kc = (16 - kk) & 15;
            const float2 Z = z[kk], Zm = z[kc];                     // Zc = conj(Zm)
            const float4 uv = cb[s * kRowsMax + q];                 // wave-uniform: scalar loads
            // acc += Z u + conj(Zm) v as a chain of fused multiply-adds
            const float2 a0 = first ? make_float2(0.0f, 0.0f) : acc[q];
            acc[q] = make_float2(
                __builtin_fmaf(Z.x, uv.x, __builtin_fmaf(-Z.y, uv.y, __builtin_fmaf(Zm.x, uv.z, __builtin_fmaf(Zm.y, uv.w, a0.x)))),
                __builtin_fmaf(Z.x, uv.y, __builtin_fmaf(Z.y, uv.x, __builtin_fmaf(Zm.x, uv.w, __builtin_fmaf(-Zm.y, uv.z, a0.y)))));
        }
    };
    pair(0, true);
#pragma unroll 1
    for (int s = 1; s < P / 2; ++s) pair(s, false);
    // row twiddles of this thread's column (no store precedes these loads)
#pragma unroll
    for (int q = 0; q < kRowsMax; ++q) S.C[q * kRowsStride + rpad(n1)] = cmul(acc[q], rowtw[(k0 + q) * kRowsN + n1]);
    __syncthreads();
    // ---- row FFTs (256 points, natural order out) ----
    rows_step<0>(S, tid);
    rows_step<4>(S, tid);
    __syncthreads();                              // row 16 (wave 0) before the outputs
    // ---- outputs: group g rows 0..15 direct, group NG-1-g from rows 16..1 conjugated ----
    const int gm = NG - 1 - g;
    if constexpr (RED) {
        // spectral loss: only the squared magnitudes of both groups, per thread
        float t = 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * kRowsThreads;
            const int k1 = e >> 3, kp = (e & 7) * 2;
            t += norm2(S.C[kp * kRowsStride + rpad(k1)]) + norm2(S.C[(kp + 1) * kRowsStride + rpad(k1)]) +
                 norm2(S.C[(16 - kp) * kRowsStride + rpad(kRowsN - 1 - k1)]) +
                 norm2(S.C[(15 - kp) * kRowsStride + rpad(kRowsN - 1 - k1)]);
        }
        *norm += (double)t;
        return;
    }
    constexpr int U = HALF ? 4 : 8;                // k1 < 128 for the half spectrum
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * kRowsThreads;
        const int k1 = e >> 3, kp = (e & 7) * 2;
        float2 a = S.C[kp * kRowsStride + rpad(k1)];
        const float2 c = S.C[(kp + 1) * kRowsStride + rpad(k1)];
        if (HALF && u == 0 && tid == 0 && g == 0) a.y = S.C[rpad(kRowsN / 2)].x;   // (DC, Nyquist)
        store_out(yw + k0 + kp + (int64_t)R * k1, make_float4(scale * a.x, scale * a.y, scale * c.x, scale * c.y));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = tid + u * kRowsThreads;
        const int k1 = e >> 3, kp = (e & 7) * 2;
        // bin 16 gm + kp (+1) at k1 = conj(row 16 - kp (15 - kp) at 255 - k1)
        const float2 a = S.C[(16 - kp) * kRowsStride + rpad(kRowsN - 1 - k1)];
        const float2 c = S.C[(15 - kp) * kRowsStride + rpad(kRowsN - 1 - k1)];
        store_out(yw + 16 * gm + kp + (int64_t)R * k1, make_float4(scale * a.x, -scale * a.y, scale * c.x,
                                                                       -scale * c.y));
    }
}

}  // namespace mrdft
