// Forward tile for complex input: levels 1..11 of a 2048-sample tile, 256
// threads, 40 KB of LDS.
//
// The recurrence of Section 3 (eq. (4)), level by level, on chip:
// * even bins: U^(i) (eq. (2)), Y^(i)[w][2k] = Y^(i-1)[2w][k] + Y^(i-1)[2w+1][k];
// * odd bins: V^(i), D^(i), F^(i) (eq. (3)): the L/2-point DFT of the window
//   difference d[q] = x[wL + q] - x[wL + q + L/2] twiddled by w_L^q,
//   Y^(i)[w][2k+1] = DFT(d)[k].  The bins are put in natural order in LDS
//   (the bit reversal of Section 3 is never executed).
// Levels 1..3 run in registers (one 8-sample window per thread) and are
// written through wave-private LDS staging, so that every store instruction
// covers 1 KB of consecutive output.  Levels 4..9 (windows inside one wave's
// 512 samples) run wave by wave: each wave's 256 odd-bin points sit in
// registers (4 per lane), the first radix-4 stage runs in registers and the
// others as cross-lane butterflies (DPP within rows of 16 lanes, permlane
// swaps across them), with one pass through LDS to put the bins in natural
// order.  Levels 10 and 11 take one radix-4 stage in registers and one
// exchange between waves through LDS, after which the same cross-lane FFT
// finishes each wave's sub-FFTs.  U^(i) is formed first and kept in
// registers, which lets the FFT work space overlay the level spectra.
#pragma once
#include "mrdft_device.h"
#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"
#include "mrdft_xlane.h"

namespace mrdft {

constexpr int kCTLog = 11;
constexpr int kCT = 1 << kCTLog;        // tile length (complex samples)
constexpr int kCThreads = 256;

struct CTileLds {
    float2 X[kCT];                      // samples
    float2 P[kCT];                      // level spectra; the FFT work space overlays them
    float2 Q[kCT / 4];                  // w_2048^e, e < 512
};                                      // 36 KB
static_assert(sizeof(CTileLds) <= 40 * 1024 - 256, "four workgroups per CU");

// w_{2^lg}^e (lg <= 11) from the quarter table q[r] = w_2048^r, r < 512:
// w^{r + 512 c} = (-j)^c w^r.  Entry r sits at r ^ ((r >> 5) & 15): twiddles
// at a power-of-two stride (one FFT stage) spread over the banks.
__device__ __forceinline__ int cqswz(int r) { return r ^ ((r >> 5) & 15); }
struct TwQ2048 {
    const float2* q;
    __device__ __forceinline__ float2 operator()(int lg, int e) const {
        const int E = (e << (kCTLog - lg)) & (kCT - 1);
        const float2 a = q[cqswz(E & (kCT / 4 - 1))];
        const int c = E >> (kCTLog - 2);
        float re = (c & 1) ? a.y : a.x;
        float im = (c & 1) ? -a.x : a.y;
        if (c & 2) {
            re = -re;
            im = -im;
        }
        return make_float2(re, im);
    }
};

// FFT work space index of the adjoint tile's Stockham steps: one spare
// element after every 32 (bank spread of the strided accesses); 1024 points
// need 1056 slots of P.
__device__ __forceinline__ int cfpad(int i) { return i + (i >> 5); }

// Sample index in X: bits 4..6 folded into bits 1..3 (bit 0 kept, so sample
// pairs stay adjacent).  The strided reads of the wave levels (lanes over
// windows of 16..64 samples) then fall on distinct banks, as do the 16-byte
// accesses of the load and of the register levels.
__device__ __forceinline__ int cx(int e) { return e ^ (((e >> 4) & 7) << 1); }

// Where position t of a tile level goes, relative to the level's base: the
// tile lies inside one signal (MULTI false: t itself), or it holds several
// consecutive signals of 2^m samples (signal t >> m at output stride S,
// position t mod 2^m) of which the first vlen samples are valid.
struct SubMap {
    int m;
    int vlen;
    int64_t S;
    template <bool MULTI>
    __device__ __forceinline__ int64_t off(int t) const {
        if constexpr (MULTI) return (int64_t)(t >> m) * S + (t & ((1 << m) - 1));
        else return t;
    }
};

__device__ __forceinline__ void ct_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- levels 4..9: one wave per 512 samples, butterflies across lanes ----
//
// Wave v owns X[512 v, 512 v + 512) and P[512 v, 512 v + 512) (its pairs
// 256 v .. 256 v + 255 of every level), so these levels need no workgroup
// barrier.  The wave's 256 odd-bin points of level I (FFTs of 2^(I-1)
// points) are transformed by xl_fft (mrdft_xlane.h).
constexpr int kCtWaveMaxLog = 9;

template <int I, bool MULTI>
__device__ __forceinline__ void ct_level_wave(CTileLds& S, float2* __restrict__ y, int tid, bool store,
                                              const SubMap& sm, const XLane& ln) {
    constexpr int L = 1 << I, M = L / 2, n = I - 1;
    constexpr int NQ = n - 2;                            // FFT-index bits held by the lane
    const int v = tid >> 6, lane = tid & 63;
    float2* Pb = S.P + 512 * v;
    // ---- U^(i): even bins of the wave's pairs J = 64 c + lane ----
    float2 u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = 64 * c + lane;
        const int w = J / M, k = J % M;
        u[c] = cadd(Pb[2 * w * M + k], Pb[(2 * w + 1) * M + k]);
    }
    // ---- the twiddled differences d[q] w_L^q, q = qlow + 2^NQ r ----
    const int qlow = ln.c & ((1 << (NQ < 6 ? NQ : 6)) - 1);
    const int wl = NQ < 6 ? ln.c >> NQ : 0;
    float2 a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = qlow + (r << NQ);
        const int e = 512 * v + wl * L + q;
        a[r] = cmul(csub(S.X[cx(e)], S.X[cx(e + M)]), TwQ2048{S.Q}(I, q));
    }
    xl_fft<n>(a, ln, TwQ2048{S.Q});
    ct_wave_sync();                                      // U reads before the overlaying writes
#pragma unroll
    for (int r = 0; r < 4; ++r) Pb[xl_fsw(xl_pos<n>(ln.c, r))] = a[r];
    ct_wave_sync();
    float2 d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) d[c] = Pb[xl_fsw(64 * c + lane)];
    ct_wave_sync();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = 64 * c + lane;                // the wave's pair: window J / M, bins 2k, 2k+1
        const int JG = 256 * v + J;                 // the pair's index in the tile
        const float4 pr = make_float4(u[c].x, u[c].y, d[c].x, d[c].y);
        *(float4*)(Pb + 2 * J) = pr;
        if (store && (!MULTI || 2 * JG < sm.vlen)) store_out(y + sm.off<MULTI>(2 * JG), pr);
    }
    // the next level reads P: its own quarter (wave levels), or all of it
    if constexpr (I == kCtWaveMaxLog) __syncthreads();
    else ct_wave_sync();
}

// Level I = 10 or 11 (windows spanning two or four waves).  The odd-bin FFT
// of M = 2^n points (n = I - 1) per window: a radix-4 stage over the two top
// index bits (lane l, register r holding point qlow + (M/4) r, qlow from the
// lane's content bits and the wave), one exchange through LDS after which
// each wave holds whole sub-FFTs of M/4 points (one of 256 at level 11, two of
// 128 at level 10: sub-FFT s = window * 4 + first-stage digit), xl_fft on
// them, and one pass through LDS back to natural order (index p ^ ((p >>
// (n-4)) & 15): the bins a 16-lane row scatters then differ in their low bits).
template <int I, bool MULTI>
__device__ __forceinline__ void ct_level_x(CTileLds& S, float2* __restrict__ y, int tid, bool store,
                                           const SubMap& sm, const XLane& ln) {
    constexpr int L = 1 << I, M = L / 2, n = I - 1;
    constexpr int Q4 = M / 4;                           // sub-FFT size
    constexpr int NS = n - 2;                           // its index bits: 8 or 7
    constexpr int SH = n - 4;                           // natural-order swizzle shift
    static_assert(I == 10 || I == 11, "levels whose windows span several waves");
    const int v = tid >> 6;
    float2* F = S.P;
    // ---- U^(i): even bins from the two child windows (pairs J = tid + 256 c) ----
    float2 u[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = tid + c * kCThreads;
        const int w = J / M, k = J % M;
        u[c] = cadd(S.P[2 * w * M + k], S.P[(2 * w + 1) * M + k]);
    }
    __syncthreads();
    // ---- radix 4 over the top two index bits of the twiddled differences ----
    const int qb = I == 11 ? v : (v & 1);               // index bits above the lane's six
    const int wb = I == 11 ? 0 : (v >> 1);              // window (level 10)
    const int qlow = ln.c + 64 * qb;                    // < M/4
    float2 a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int q = qlow + Q4 * r;
        const int e = wb * L + q;
        a[r] = cmul(csub(S.X[cx(e)], S.X[cx(e + M)]), TwQ2048{S.Q}(I, q));
    }
    dft_reg<4, false>(a);
#pragma unroll
    for (int f = 1; f < 4; ++f) a[f] = cmul(a[f], TwQ2048{S.Q}(n, qlow * f));
    // ---- exchange: sub-FFT s = window * 4 + digit, point qlow ----
#pragma unroll
    for (int r = 0; r < 4; ++r) F[(wb * 4 + r) * Q4 + qlow] = a[r];
    __syncthreads();
    // the wave's sub-FFT(s) in the xl_fft<NS> layout: point plow + 2^(NS-2) r'
    // of sub-FFT s (level 11: s = v; level 10: s = 2 v + content bit 5)
    const int plow = ln.c & ((1 << (NS - 2)) - 1);
    const int s0 = I == 11 ? v : 2 * v + (ln.c >> 5);
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = F[s0 * Q4 + plow + (r << (NS - 2))];
    xl_fft<NS>(a, ln, TwQ2048{S.Q});
    __syncthreads();                                    // every wave's exchange reads before the writes
    // ---- bins to natural order: window s >> 2, bin (s & 3) + 4 k' ----
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pos = xl_pos<NS>(ln.c, r);
        const int s = I == 11 ? v : 2 * v + (pos >> 7);
        const int kp = I == 11 ? pos : (pos & 127);
        const int P = (s >> 2) * M + (s & 3) + 4 * kp;
        F[P ^ ((P >> SH) & 15)] = a[r];
    }
    __syncthreads();
    float2 d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = tid + c * kCThreads;
        d[c] = F[J ^ ((J >> SH) & 15)];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int J = tid + c * kCThreads;          // = w * M + k: the pair (2k, 2k+1) of window w
        const float4 pr = make_float4(u[c].x, u[c].y, d[c].x, d[c].y);
        *(float4*)(S.P + 2 * J) = pr;
        if (store && (!MULTI || 2 * J < sm.vlen)) store_out(y + sm.off<MULTI>(2 * J), pr);
    }
    __syncthreads();
}

template <int I, bool MULTI>
struct CtLevels {
    static __device__ __forceinline__ void run(CTileLds& S, float2* __restrict__ y, int64_t ls, int tid,
                                               LevelRange lv, const SubMap& sm, const XLane& ln) {
        if constexpr (I <= kCTLog) {
            if (I > lv.hi) return;                    // levels above the range are not computed
            if constexpr (I <= kCtWaveMaxLog)
                ct_level_wave<I, MULTI>(S, y + (int64_t)(I - 1) * ls, tid, lv.in(I), sm, ln);
            else
                ct_level_x<I, MULTI>(S, y + (int64_t)(I - 1) * ls, tid, lv.in(I), sm, ln);
            CtLevels<I + 1, MULTI>::run(S, y, ls, tid, lv, sm, ln);
        }
    }
};

// Writes one register level (8 values per thread, one window each) through
// the wave's 4 KB of staging (pair e of lane l at 4l + (e ^ (l & 3))).
//   yl: the level's base; t0: the wave's first tile position (512 v)
template <bool MULTI>
__device__ __forceinline__ void ct_stage(const float2* pv, float4* st, float2* __restrict__ yl, int t0, int lane,
                                         bool store, const SubMap& sm) {
    if (!store) return;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        st[4 * lane + (e ^ (lane & 3))] = make_float4(pv[2 * e].x, pv[2 * e].y, pv[2 * e + 1].x, pv[2 * e + 1].y);
    ct_wave_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = 64 * r + lane, wl = p >> 2, e = p & 3;
        const int t = t0 + 2 * p;
        if (!MULTI || t < sm.vlen) store_out(yl + sm.off<MULTI>(t), st[4 * wl + (e ^ (wl & 3))]);
    }
    ct_wave_sync();
}

// Register levels I..3 of an 8-sample window (full spectra, natural order).
template <int I, bool MULTI>
struct CtLocal {
    static __device__ __forceinline__ void run(const float2* xv, float2* pv, float4* st, float2* y, int t0, int64_t ls,
                                               int lane, LevelRange lv, const SubMap& sm) {
        if constexpr (I <= 3) {
            constexpr int C = 8, L = 1 << I, M = L / 2;
            float2 nv[C];
#pragma unroll
            for (int w = 0; w < C / L; ++w) {
                float2 d[M];
#pragma unroll
                for (int q = 0; q < M; ++q) d[q] = twiddle_small<false>(csub(xv[w * L + q], xv[w * L + q + M]), q, L);
                dft_reg<M, false>(d);
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    nv[w * L + 2 * k] = cadd(pv[w * L + k], pv[w * L + M + k]);
                    nv[w * L + 2 * k + 1] = d[k];
                }
            }
#pragma unroll
            for (int e = 0; e < C; ++e) pv[e] = nv[e];
            ct_stage<MULTI>(pv, st, y + (int64_t)(I - 1) * ls, t0, lane, lv.in(I), sm);
            CtLocal<I + 1, MULTI>::run(xv, pv, st, y, t0, ls, lane, lv, sm);
        }
    }
};

// One tile: x at its first sample, y at its level-1 output (level i at
// y + (i-1) ls).  Wave v owns samples [512 v, 512 v + 512).  MULTI: the tile
// holds consecutive signals of 2^sm.m samples (ls = 2^sm.m, lv.hi <= sm.m),
// samples past sm.vlen are not read and their outputs not written.  REALIN:
// x is float32 (real samples, imaginary parts zero).
template <bool MULTI = false, bool REALIN = false>
__device__ __forceinline__ void c64_tile_body(CTileLds& S, const void* __restrict__ x, float2* __restrict__ y,
                                              int64_t ls, const float2* __restrict__ t4096, int tid, LevelRange lv,
                                              const SubMap& sm = SubMap{31, kCT, 0}) {
    constexpr int C = 8;
    const int v = tid >> 6, lane = tid & 63;
    for (int e = tid; e < kCT / 4; e += kCThreads) S.Q[cqswz(e)] = t4096[2 * e];   // before any store
    // coalesced load of the wave's samples into X (their final place)
    {
        float4 a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!MULTI || 512 * v + 2 * (64 * r + lane) < sm.vlen) {
                if constexpr (REALIN) {
                    const float2 f = ((const float2*)((const float*)x + 512 * v))[64 * r + lane];
                    a[r] = make_float4(f.x, 0.0f, f.y, 0.0f);
                } else {
                    a[r] = ((const float4*)((const float2*)x + 512 * v))[64 * r + lane];
                }
            } else {
                a[r] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) *(float4*)(S.X + cx(512 * v + 2 * (64 * r + lane))) = a[r];
    }
    ct_wave_sync();
    float2 xv[C], pv[C];
#pragma unroll
    for (int e = 0; e < C / 2; ++e) {
        const float4 a = *(const float4*)(S.X + cx(C * tid + 2 * e));
        xv[2 * e] = make_float2(a.x, a.y);
        xv[2 * e + 1] = make_float2(a.z, a.w);
    }
#pragma unroll
    for (int b = 0; b < C / 2; ++b) {
        pv[2 * b] = cadd(xv[2 * b], xv[2 * b + 1]);
        pv[2 * b + 1] = csub(xv[2 * b], xv[2 * b + 1]);
    }
    float4* st = (float4*)S.P + 256 * v;            // the wave's 4 KB of P
    ct_stage<MULTI>(pv, st, y, 512 * v, lane, lv.in(1), sm);
    CtLocal<2, MULTI>::run(xv, pv, st, y, 512 * v, ls, lane, lv, sm);
    // level-3 spectra into P (this wave's own region, after its staging reads)
#pragma unroll
    for (int e = 0; e < C / 2; ++e)
        *(float4*)(S.P + C * tid + 2 * e) = make_float4(pv[2 * e].x, pv[2 * e].y, pv[2 * e + 1].x, pv[2 * e + 1].y);
    __syncthreads();
    const XLane ln = xl_lane(lane, TwQ2048{S.Q});
    CtLevels<4, MULTI>::run(S, y, ls, tid, lv, sm, ln);
}

}  // namespace mrdft
