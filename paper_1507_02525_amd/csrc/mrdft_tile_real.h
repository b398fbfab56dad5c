// Forward tile for real input: levels 1..12 of a 4096-sample tile.
//
// Same recurrence as the complex tile kernel (Section 3, eq. (4): even bins
// of level i are sums of the two child windows of level i-1, U^(i), eq. (2);
// odd bins are a transform of the twiddled window difference, V^(i), eq. (3),
// D^(i), F^(i)), specialised to real x, whose window spectra are Hermitian:
// Y[L-k] = conj(Y[k]).
//
// * State: each window of length L keeps L/2 complex slots, slot k = Y[k] for
//   0 < k < L/2 and slot 0 = (Y[0], Y[L/2]) (DC and Nyquist are real).  With
//   this packing the U step keeps its form: new slot 2k = child0[k] + child1[k]
//   for every k < L/4, including the packed slot 0.
// * Odd bins O[k] = sum_q d[q] w_L^{q(2k+1)} (d = x_lo - x_hi, real, M = L/2
//   points) are needed for k < M/2 only; they come from one complex FFT of
//   M/2 points: z[p] = (d[2p] + j d[2p+1]) w_M^p, Z = DFT(z), and with
//   A = (Z[k] + conj(Z[M/2-1-k]))/2, B = -j (Z[k] - conj(Z[M/2-1-k]))/2,
//   T = w_L^{2k+1} B:  O[k] = A + T,  O[M/2-1-k] = conj(A - T).
// * Every level is written out as the full spectrum (the upper half as
//   conjugates), straight from registers, or (half-spectrum output) as the
//   packed slots themselves.
//
// Everything level-dependent is a compile-time constant (one instantiation per
// level), so LDS addressing folds into immediate offsets.
#pragma once
#include <stddef.h>

#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"
#include "mrdft_xlane.h"

namespace mrdft {

constexpr int kRTLog = 12;
constexpr int kRT = 1 << kRTLog;         // tile length
constexpr int kRThreads = 256;

struct RealTileLds {
    float X[kRT];                        // input tile
    float2 P[kRT / 2];                   // half spectra; also the FFT work space
    float2 Q[kRT / 4];                   // twiddle quarter table w_4096^e, e < 1024
};                                       // 40 KB: four workgroups per CU
// The register phase stages 4 waves x 512 float4 in X and P.
static_assert(offsetof(RealTileLds, P) == sizeof(float) * kRT, "X and P adjacent");
static_assert(sizeof(float) * kRT + sizeof(float2) * kRT / 2 == (kRThreads / 64) * 512 * sizeof(float4), "staging size");

// No global load may follow a global store inside this kernel: the vector
// memory counter retires loads and stores in issue order, so such a load would
// wait for every earlier store.  All twiddles therefore come from LDS.

__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Orders LDS accesses of lanes of one wave (LDS executes a wave's
// instructions in issue order; this only stops the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Where the level spectra go: stored to Y, or (spectral loss) only their
// squared magnitudes summed per level in FP64, Y never written.
// HALF: each window of L bins is stored as its L/2 packed half-spectrum
// slots (slot 0 = (Y[0], Y[L/2]), slot k = Y[k]), levels N/2 apart.
template <bool HALF>
struct StoreOutT {
    static constexpr bool kReduce = false;
    static constexpr bool kHalf = HALF;
    LevelRange lv;                                 // levels stored
    __device__ __forceinline__ float2 sc(int, float2 v) const { return v; }
    __device__ __forceinline__ bool keep(int level) const { return lv.in(level); }
};
using StoreOut = StoreOutT<false>;
// Stored times a per-level factor (spectral-loss gradient).
template <bool HALF>
struct ScaledOutT {
    static constexpr bool kReduce = false;
    static constexpr bool kHalf = HALF;
    const float* alpha;
    __device__ __forceinline__ float2 sc(int level, float2 v) const {
        const float a = alpha[level - 1];
        return make_float2(a * v.x, a * v.y);
    }
    __device__ __forceinline__ bool keep(int) const { return true; }
};
using ScaledOut = ScaledOutT<false>;
struct NormOut {
    static constexpr bool kReduce = true;
    static constexpr bool kHalf = false;
    double* sums;                                   // this signal's per-level sums
    __device__ __forceinline__ float2 sc(int, float2 v) const { return v; }
    __device__ __forceinline__ bool keep(int) const { return true; }
    // Adds the wave's partial sums of one level (every lane must call it).
    __device__ __forceinline__ void add(int level, float t) {
        const double v = xl_wave_sum((double)t);
        if ((threadIdx.x & 63) == 0) atomicAdd(sums + level - 1, v);
    }
};

// The quarter table w_4096^e (e < 1024) sits at a swizzled index: the low 5
// bits are XORed with bits 5..9, so that entries at a power-of-two stride of
// 32 or more (the twiddles of one Stockham step) fall on different banks.
__device__ __forceinline__ int qswz(int E) { return E ^ ((E >> 5) & 31); }

// w_{2^lg}^e (lg <= 12) from the LDS quarter table: w^{r + 1024 c} = (-j)^c w^r.
struct RtTw {
    const float2* Q;
    __device__ __forceinline__ float2 operator()(int lg, int e) const {
        const int E = (e << (kRTLog - lg)) & (kRT - 1);
        const float2 a = Q[qswz(E & (kRT / 4 - 1))];
        const int c = E >> (kRTLog - 2);
        float re = (c & 1) ? a.y : a.x;
        float im = (c & 1) ? -a.x : a.y;
        if (c & 2) {
            re = -re;
            im = -im;
        }
        return make_float2(re, im);
    }
};
template <int LG>
__device__ __forceinline__ float2 wl(const float2* Q, int e) {
    return RtTw{Q}(LG, e);
}
// Same for exponents known to lie in the first quadrant (e < 2^LG / 4).
template <int LG>
__device__ __forceinline__ float2 wq1(const float2* Q, int e) {
    return Q[qswz(e << (kRTLog - LG))];
}
// First two quadrants (e < 2^LG / 2): w^{e} = -j w^{e - 2^LG/4} beyond the first.
template <int LG>
__device__ __forceinline__ float2 wq2(const float2* Q, int e) {
    const int E = e << (kRTLog - LG);
    const float2 a = Q[qswz(E & (kRT / 4 - 1))];
    return (E >= kRT / 4) ? make_float2(a.y, -a.x) : a;
}

// FFT work space index: one spare element after every 32, so that the
// strided Stockham accesses spread over the banks (1024 points use 1056
// slots of P).
__device__ __forceinline__ int fpad(int i) { return i + (i >> 5); }

// The samples X sit at a swizzled index: within each 64-sample (256-byte)
// row the sixteen 16-byte slots are XORed with (5 row) mod 16.  The first
// step of every level reads the window halves of many small windows at once
// (windows of 64 samples all start on the same banks); the swizzle spreads
// them over the banks and keeps 16-byte groups (float4) and pairs contiguous.
__device__ __forceinline__ int xsw(int i) { return i ^ (((5 * (i >> 6)) & 15) << 2); }

// One in-place radix-R Stockham step over NW FFTs of H points in F (contiguous
// per window), span 2^LNS before the step.  256 threads, R in {2, 4}.
template <int R, int H, int NW, int LNS>
__device__ __forceinline__ void rstep(float2* F, const float2* W, int tid) {
    constexpr int LR = (R == 2) ? 1 : 2;
    constexpr int PER = H / R;
    constexpr int JOBS = NW * PER;
    constexpr int JPT = JOBS / kRThreads;
    static_assert(JOBS % kRThreads == 0, "job count");
    constexpr int NS = 1 << LNS;
    float2 v[JPT][R];
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kRThreads;
        const int w = J / PER, j = J % PER;
#pragma unroll
        for (int s = 0; s < R; ++s) v[c][s] = F[fpad(w * H + j + s * PER)];
        if constexpr (LNS > 0) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int s = 1; s < R; ++s) v[c][s] = cmul(v[c][s], wl<LNS + LR>(W, jm * s));
        }
        dft_reg<R, false>(v[c]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kRThreads;
        const int w = J / PER, j = J % PER;
        const int base = w * H + ((j >> LNS) << (LNS + LR)) + (j & (NS - 1));
#pragma unroll
        for (int s = 0; s < R; ++s) F[fpad(base + s * NS)] = v[c][s];
    }
    __syncthreads();
}

// Remaining radix-4 steps after span 2^LNS, until the FFT of 2^LH points is done.
template <int H, int NW, int LNS, int LH>
struct RSteps {
    static __device__ __forceinline__ void run(float2* F, const float2* W, int tid) {
        if constexpr (LNS < LH) {
            rstep<4, H, NW, LNS>(F, W, tid);
            RSteps<H, NW, LNS + 2, LH>::run(F, W, tid);
        }
    }
};

// A level's outputs of post job (w, k) (j = H - 1 - k): the full spectrum
// (bins 2k, 2k+1, 2j, 2j+1 and their mirrored upper pairs), the packed slots
// (half-spectrum output) or only their squared magnitudes (norm).
template <int I, class O>
__device__ __forceinline__ void real_level_out(float2* __restrict__ y, int w, int k, int j, float2 uk, float2 uj,
                                               float2 uk1, float2 uj1, float2 ok, float2 oj, float& nrm, O& out) {
    constexpr int L = 1 << I, M = L / 2;
    // Full spectrum: bins 2k, 2k+1 (lower half) and the aligned upper pairs
    // (L/2 + 2t, L/2 + 2t + 1) = (conj u[H-t], conj o[H-1-t]), t = j and t = k;
    // bin 0 is real, bin L/2 (Nyquist) is the second half of slot 0.
    float2* yw = y + (int64_t)w * L;
    const float2 u0 = (k == 0) ? make_float2(uk.x, 0.0f) : uk;
    const float2 ua = cconj(uk1);
    const float2 ub = (k == 0) ? make_float2(uj1.y, 0.0f) : cconj(uj1);
    const float2 oka = cconj(ok), oja = cconj(oj);
    if constexpr (O::kReduce) {
        nrm += norm2(u0) + norm2(ok) + norm2(uj) + norm2(oj) + norm2(ua) + norm2(oka) + norm2(ub) + norm2(oja);
    } else if (O::kHalf) {
        if (out.keep(I)) {                          // the packed slots themselves (slot 0 = uk at k = 0)
            float2* yh = y + (int64_t)w * M;
            const float2 s0 = out.sc(I, uk), s1 = out.sc(I, ok), s2 = out.sc(I, uj), s3 = out.sc(I, oj);
            store_out(yh + 2 * k, make_float4(s0.x, s0.y, s1.x, s1.y));
            store_out(yh + 2 * j, make_float4(s2.x, s2.y, s3.x, s3.y));
        }
    } else if (out.keep(I)) {
        const float2 s0 = out.sc(I, u0), s1 = out.sc(I, ok), s2 = out.sc(I, uj), s3 = out.sc(I, oj);
        const float2 s4 = out.sc(I, ua), s5 = out.sc(I, oka), s6 = out.sc(I, ub), s7 = out.sc(I, oja);
        store_out(yw + 2 * k, make_float4(s0.x, s0.y, s1.x, s1.y));
        store_out(yw + 2 * j, make_float4(s2.x, s2.y, s3.x, s3.y));
        store_out(yw + M + 2 * j, make_float4(s4.x, s4.y, s5.x, s5.y));
        store_out(yw + M + 2 * k, make_float4(s6.x, s6.y, s7.x, s7.y));
    }
}

// Level I = 11 or 12 of the tile (windows spanning several waves).
template <int I, class O>
__device__ __forceinline__ void real_level(RealTileLds& S, float2* __restrict__ y, int tid, O& out) {
    constexpr int L = 1 << I, M = L / 2, H = M / 2, LH = I - 2;
    constexpr int NW = kRT / L;
    constexpr int R1 = (LH & 1) ? 2 : 4;        // first step radix
    constexpr int LR1 = (R1 == 2) ? 1 : 2;
    constexpr int PJ = NW * (H / 2);            // post jobs: (w, k), k < H/2
    constexpr int PPT = PJ / kRThreads;
    static_assert(PJ % kRThreads == 0, "post job count");
    float2* F = S.P;                            // FFT work space aliases the half spectra
    // ---- U^(i) first: even bins from the two child windows, kept in registers ----
    // Job (w, k) also takes u[k+1] and u[H-k], the even bins its mirrored
    // (upper-half) output pairs need; u[H] stands for the Nyquist bin.
    float2 uk[PPT], uj[PPT], uk1[PPT], uj1[PPT];
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kRThreads;
        const int w = J / (H / 2), k = J % (H / 2);
        const int j = H - 1 - k;
        const float2* c0 = S.P + (2 * w) * H;
        uk[c] = cadd(c0[k], c0[H + k]);
        uj[c] = cadd(c0[j], c0[H + j]);
        uk1[c] = cadd(c0[k + 1], c0[H + k + 1]);
        const int jn = (k == 0) ? 0 : j + 1;
        uj1[c] = cadd(c0[jn], c0[H + jn]);
    }
    __syncthreads();
    // ---- first step: pack the real window differences, pre-twiddle w_M^p, DFT ----
    {
        constexpr int PER = H / R1;
        constexpr int JOBS = NW * PER;
        constexpr int JPT = JOBS / kRThreads;
        float2 v[JPT][R1];
#pragma unroll
        for (int c = 0; c < JPT; ++c) {
            const int J = tid + c * kRThreads;
            const int w = J / PER, j = J % PER;
#pragma unroll
            for (int s = 0; s < R1; ++s) {
                const int p = j + s * PER;
                const float2 lo = *(const float2*)(S.X + xsw(w * L + 2 * p));
                const float2 hi = *(const float2*)(S.X + xsw(w * L + M + 2 * p));
                const float2 z = make_float2(lo.x - hi.x, lo.y - hi.y);
                v[c][s] = cmul(z, wq2<I - 1>(S.Q, p));                   // w_M^p, p < M/2
            }
            dft_reg<R1, false>(v[c]);
        }
#pragma unroll
        for (int c = 0; c < JPT; ++c) {
            const int J = tid + c * kRThreads;
            const int w = J / PER, j = J % PER;
#pragma unroll
            for (int s = 0; s < R1; ++s) F[fpad(w * H + j * R1 + s)] = v[c][s];
        }
        __syncthreads();
    }
    RSteps<H, NW, LR1, LH>::run(F, S.Q, tid);
    // ---- post-processing, new half spectra and the level's output ----
    float2 ok[PPT], oj[PPT];
    float nrm = 0.0f;
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kRThreads;
        const int w = J / (H / 2), k = J % (H / 2);
        const int j = H - 1 - k;
        const float2 zk = F[fpad(w * H + k)], zj = F[fpad(w * H + j)];
        const float2 zjc = cconj(zj);
        const float2 A = cscale(cadd(zk, zjc), 0.5f);
        const float2 B = mul_mj(cscale(csub(zk, zjc), 0.5f));
        const float2 T = cmul(wq1<I>(S.Q, 2 * k + 1), B);              // w_L^{2k+1}, 2k+1 < L/4
        ok[c] = cadd(A, T);
        oj[c] = cconj(csub(A, T));
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
        const int J = tid + c * kRThreads;
        const int w = J / (H / 2), k = J % (H / 2);
        const int j = H - 1 - k;
        // one 16-byte store per slot pair (lanes 16 bytes apart fill the banks)
        float2* pw = S.P + w * M;
        *(float4*)(pw + 2 * k) = make_float4(uk[c].x, uk[c].y, ok[c].x, ok[c].y);
        *(float4*)(pw + 2 * j) = make_float4(uj[c].x, uj[c].y, oj[c].x, oj[c].y);
        real_level_out<I, O>(y, w, k, j, uk[c], uj[c], uk1[c], uj1[c], ok[c], oj[c], nrm, out);
    }
    if constexpr (O::kReduce) out.add(I, nrm);
    __syncthreads();
}

// ---- levels 5..10: windows inside one wave's 1024 samples ----
//
// Wave v owns samples [1024 v, 1024 v + 1024) and half-spectrum slots
// [512 v, 512 v + 512); its 256 points of the packed odd-bin FFTs (FFTs of
// H = 2^(I-2) points) are transformed across lanes by xl_fft, then put in
// natural order through the wave's slots; no workgroup barrier is needed.
constexpr int kRtWaveMaxLog = 10;

template <int I, class O>
__device__ __forceinline__ void real_level_wave(RealTileLds& S, float2* __restrict__ y, int tid, O& out,
                                                const XLane& ln) {
    constexpr int L = 1 << I, M = L / 2, H = M / 2, n = I - 2;
    constexpr int NQ = n - 2;                   // FFT-index bits held by the lane
    constexpr int HJ = H / 2;                   // post jobs per window
    const int v = tid >> 6, lane = tid & 63;
    float2* Pb = S.P + 512 * v;
    // ---- U^(i) of the wave's post jobs J = 64 c + lane (window J / HJ, k = J mod HJ) ----
    float2 uk[2], uj[2], uk1[2], uj1[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int J = 64 * c + lane;
        const int w = J / HJ, k = J % HJ;
        const int j = H - 1 - k;
        const float2* c0 = Pb + (2 * w) * H;
        uk[c] = cadd(c0[k], c0[H + k]);
        uj[c] = cadd(c0[j], c0[H + j]);
        uk1[c] = cadd(c0[k + 1], c0[H + k + 1]);
        const int jn = (k == 0) ? 0 : j + 1;
        uj1[c] = cadd(c0[jn], c0[H + jn]);
    }
    // ---- packed real window differences, pre-twiddled by w_M^p, p = plow + 2^NQ r ----
    const int plow = ln.c & ((1 << (NQ < 6 ? NQ : 6)) - 1);
    const int wl_ = NQ < 6 ? ln.c >> NQ : 0;
    float2 a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = plow + (r << NQ);
        const int base = 1024 * v + wl_ * L;
        const float2 lo = *(const float2*)(S.X + xsw(base + 2 * p));
        const float2 hi = *(const float2*)(S.X + xsw(base + M + 2 * p));
        a[r] = cmul(make_float2(lo.x - hi.x, lo.y - hi.y), wq2<I - 1>(S.Q, p));
    }
    xl_fft<n>(a, ln, RtTw{S.Q});
    wave_sync();                                // U reads before the overlaying writes
#pragma unroll
    for (int r = 0; r < 4; ++r) Pb[xl_fsw(xl_pos<n>(ln.c, r))] = a[r];
    wave_sync();
    // ---- post-processing, new half spectra and the level's output ----
    float2 ok[2], oj[2];
    float nrm = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int J = 64 * c + lane;
        const int w = J / HJ, k = J % HJ;
        const int j = H - 1 - k;
        const float2 zk = Pb[xl_fsw(w * H + k)], zj = Pb[xl_fsw(w * H + j)];
        const float2 zjc = cconj(zj);
        const float2 A = cscale(cadd(zk, zjc), 0.5f);
        const float2 B = mul_mj(cscale(csub(zk, zjc), 0.5f));
        const float2 T = cmul(wq1<I>(S.Q, 2 * k + 1), B);              // w_L^{2k+1}, 2k+1 < L/4
        ok[c] = cadd(A, T);
        oj[c] = cconj(csub(A, T));
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int J = 64 * c + lane;
        const int w = J / HJ, k = J % HJ;
        const int j = H - 1 - k;
        const int wg = (1024 / L) * v + w;      // the window's index in the tile
        float2* pw = Pb + w * M;
        *(float4*)(pw + 2 * k) = make_float4(uk[c].x, uk[c].y, ok[c].x, ok[c].y);
        *(float4*)(pw + 2 * j) = make_float4(uj[c].x, uj[c].y, oj[c].x, oj[c].y);
        real_level_out<I, O>(y, wg, k, j, uk[c], uj[c], uk1[c], uj1[c], ok[c], oj[c], nrm, out);
    }
    if constexpr (O::kReduce) out.add(I, nrm);
    if constexpr (I == kRtWaveMaxLog) __syncthreads();
    else wave_sync();
}

template <int I, class O>
struct RealLevels {
    static __device__ __forceinline__ void run(RealTileLds& S, float2* __restrict__ y, int64_t ls, int tid, O& out,
                                               const XLane& ln) {
        if constexpr (I <= kRTLog) {
            if constexpr (I <= kRtWaveMaxLog) real_level_wave<I, O>(S, y + (int64_t)(I - 1) * ls, tid, out, ln);
            else real_level<I, O>(S, y + (int64_t)(I - 1) * ls, tid, out);
            RealLevels<I + 1, O>::run(S, y, ls, tid, out, ln);
        }
    }
};


// Writes one register-phase level (16 complex values per thread, one window
// each) through the wave's private LDS region, so that every global store
// instruction covers 1 KB of consecutive output.  Pair e of lane l sits at
// 8l + (e ^ ((l / 2) mod 8)): the 16 lanes served per LDS cycle (16 bytes
// each) then fall on distinct banks, for the writes and for the reads.
// Half-spectrum output: the lane's 8 packed slots (slot 0 of each window =
// (Y[0], Y[L/2])), pair e of lane l at 4l + (e ^ ((l / 4) mod 4)), 512 B per
// store instruction.
template <int I, class O>
__device__ __forceinline__ void stage_level(const float2* pv, float4* st, float2* __restrict__ yl, int lane, O& out) {
    constexpr int level = I;
    if constexpr (O::kReduce) {
        float t = 0.0f;
#pragma unroll
        for (int e = 0; e < 16; ++e) t += norm2(pv[e]);
        out.add(level, t);
        return;
    }
    if (!out.keep(level)) return;
    if constexpr (O::kHalf) {
        constexpr int L = 1 << I, M = L / 2;
        float2 hv[8];
#pragma unroll
        for (int w = 0; w < 16 / L; ++w) {
            hv[w * M] = out.sc(level, make_float2(pv[w * L].x, pv[w * L + M].x));
#pragma unroll
            for (int k = 1; k < M; ++k) hv[w * M + k] = out.sc(level, pv[w * L + k]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            st[4 * lane + (e ^ ((lane >> 2) & 3))] = make_float4(hv[2 * e].x, hv[2 * e].y, hv[2 * e + 1].x, hv[2 * e + 1].y);
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 64 * r + lane, wl = p >> 2, e = p & 3;
            store_out(yl + 2 * p, st[4 * wl + (e ^ ((wl >> 2) & 3))]);
        }
        wave_sync();
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float2 a = out.sc(level, pv[2 * e]), b = out.sc(level, pv[2 * e + 1]);
        st[8 * lane + (e ^ ((lane >> 1) & 7))] = make_float4(a.x, a.y, b.x, b.y);
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int p = 64 * r + lane, wl = p >> 3, e = p & 7;
        store_out(yl + 2 * p, st[8 * wl + (e ^ ((wl >> 1) & 7))]);
    }
    wave_sync();
}

// Register recurrence for levels I..4 of 16 samples (full spectra, natural order).
template <int I, class O>
struct LocalFwdReal {
    static __device__ __forceinline__ void run(const float2* xv, float2* pv, float4* st, float2* y, int64_t ls,
                                               int lane, O& out) {
        if constexpr (I <= 4) {
            constexpr int C = 16, L = 1 << I, M = L / 2;
            float2 nv[C];
#pragma unroll
            for (int w = 0; w < C / L; ++w) {
                float2 d[M];
#pragma unroll
                for (int q = 0; q < M; ++q)
                    d[q] = twiddle_small<false>(csub(xv[w * L + q], xv[w * L + q + M]), q, L);
                dft_reg<M, false>(d);
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    nv[w * L + 2 * k] = cadd(pv[w * L + k], pv[w * L + M + k]);
                    nv[w * L + 2 * k + 1] = d[k];
                }
            }
#pragma unroll
            for (int e = 0; e < C; ++e) pv[e] = nv[e];
            stage_level<I, O>(pv, st, y + (int64_t)(I - 1) * ls, lane, out);
            LocalFwdReal<I + 1, O>::run(xv, pv, st, y, ls, lane, out);
        }
    }
};

// Register phase: each thread takes one 16-sample window through levels 1..4;
// wave v owns samples [1024 v, 1024 v + 1024).  X and P (32 KB, contiguous)
// serve as staging space first; at the end they receive the samples and the
// level-4 half spectra (8 slots per window, slot 0 = (Y[0], Y[8])).
template <class O>
__device__ __forceinline__ void real_local(const float* __restrict__ xin, const float* __restrict__ xsub,
                                           float2* __restrict__ y, int64_t ls, RealTileLds& S, int tid, O& out) {
    constexpr int C = 16;
    const int v = tid >> 6, lane = tid & 63;
    float* xs = S.X + 1024 * v;
    // coalesced load of the wave's samples (8-byte aligned: signal offsets are even)
    {
        const float2* xg = (const float2*)(xin + 1024 * v);
        float2 a[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] = xg[64 * r + lane];
        if (xsub) {                                   // input x - xsub (spectral loss)
            const float2* zg = (const float2*)(xsub + 1024 * v);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const float2 b = zg[64 * r + lane];
                a[r] = make_float2(a[r].x - b.x, a[r].y - b.y);
            }
        }
        // pair q goes to lane q / 8, 16-byte slot ((q / 2) mod 4) XOR ((q / 32) mod 4)
        // of that lane's 64 bytes: the lanes' 16-byte reads below then cover
        // all banks
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int q = 64 * r + lane, ol = q >> 3, e = q & 7;
            *(float2*)(xs + C * ol + 4 * ((e >> 1) ^ ((ol >> 2) & 3)) + 2 * (e & 1)) = a[r];
        }
    }
    wave_sync();
    float2 xv[C], pv[C];
#pragma unroll
    for (int e = 0; e < C / 4; ++e) {
        const float4 a = *(const float4*)(xs + C * lane + 4 * (e ^ ((lane >> 2) & 3)));
        xv[4 * e] = make_float2(a.x, 0.0f);
        xv[4 * e + 1] = make_float2(a.y, 0.0f);
        xv[4 * e + 2] = make_float2(a.z, 0.0f);
        xv[4 * e + 3] = make_float2(a.w, 0.0f);
    }
    __syncthreads();                             // the staging space overlaps other waves' samples
    float4* st = (float4*)S.X + 512 * v;
#pragma unroll
    for (int b = 0; b < C / 2; ++b) {
        pv[2 * b] = cadd(xv[2 * b], xv[2 * b + 1]);
        pv[2 * b + 1] = csub(xv[2 * b], xv[2 * b + 1]);
    }
    float2* yv = y + (O::kHalf ? 512 : 1024) * v;
    stage_level<1, O>(pv, st, yv, lane, out);
    LocalFwdReal<2, O>::run(xv, pv, st, yv, ls, lane, out);
    __syncthreads();                             // staging done in every wave
#pragma unroll
    for (int e = 0; e < C / 4; ++e)
        *(float4*)(S.X + xsw(C * tid + 4 * e)) =
            make_float4(xv[4 * e].x, xv[4 * e + 1].x, xv[4 * e + 2].x, xv[4 * e + 3].x);
    // the 8 slots as four 16-byte pairs, pair c written at step c XOR ((tid / 4)
    // mod 4), so that the 16 lanes of one step cover all banks
    pv[0].y = pv[8].x;
    float4* pd = (float4*)(S.P + tid * 8);
    const int rot = (tid >> 2) & 3;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int cc = c ^ rot;
        const float2 a = cc == 0 ? pv[0] : cc == 1 ? pv[2] : cc == 2 ? pv[4] : pv[6];
        const float2 b = cc == 0 ? pv[1] : cc == 1 ? pv[3] : cc == 2 ? pv[5] : pv[7];
        pd[cc] = make_float4(a.x, a.y, b.x, b.y);
    }
}

// One full tile: x points at the tile's first sample (minus xsub's, if given),
// y at its level-1 output (level i at y + (i-1)*ls).
template <class O>
__device__ __forceinline__ void real_tile_body(RealTileLds& S, const float* __restrict__ x,
                                               const float* __restrict__ xsub, float2* __restrict__ y, int64_t ls,
                                               const float2* __restrict__ t4096, int tid, O& out) {
    for (int e = tid; e < kRT / 4; e += kRThreads) S.Q[qswz(e)] = t4096[e];   // before any store
    real_local<O>(x, xsub, y, ls, S, tid, out);
    __syncthreads();
    const XLane ln = xl_lane(tid & 63, RtTw{S.Q});
    RealLevels<5, O>::run(S, y, ls, tid, out, ln);
}

}  // namespace mrdft
