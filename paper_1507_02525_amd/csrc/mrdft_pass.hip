// Global Stockham passes for the levels whose windows exceed the on-chip tile.
//
// Level i (window L = 2^i) is the L-point DFT of every window (Section 2,
// eq. (1)).  A window larger than the tile is transformed by a few passes over
// HBM; pass p has radix r = 2^r_log and span Ns (product of earlier radices):
// column j in [0, L/r) gathers the r inputs j + s*L/r, multiplies input s by
// w_{Ns*r}^{(j mod Ns)*s}, runs an r-point DFT in LDS and writes output s to
// (j / Ns)*Ns*r + (j mod Ns) + s*Ns.  The last pass leaves every window in
// natural bin order, i.e. already permuted as Gamma asks.
//
// A workgroup handles 2^LP points with 2^LP / 16 threads: 2^LP / r consecutive
// columns (at least 16, so every global load and store touches at least 128
// consecutive bytes; a small radix gets more columns, i.e. longer runs,
// instead of more workgroups); the first pass radix is at least 16.  Radices
// up to 2^8 use 4096-point workgroups (four per CU), radix 2^9 8192-point
// workgroups (two per CU, 74 KB of LDS), so that levels 17 and 18 take two
// passes instead of three.  (16384-point workgroups for radix 2^10, one per
// CU, moved 2.5 TB/s against 3.4 TB/s here and 3.9 TB/s for the 4096-point
// form: two of them cost more than three small passes.)  Twiddles of large windows
// come from two FP64 tables (coarse and fine exponent), multiplied in FP64 and
// rounded once: a thread looks up w^{j s0} and w^{16 j} for its column j and
// first row s0 and forms its further rows s0 + 16 i by FP64 multiplication
// (no scattered table reads per element).  With INV the conjugate kernel is used (adjoint), and the last
// pass can accumulate into the gradient instead of storing.
//
// Recurrence chains (levels 18 and up, when the level below is kept): level
// lg is built from level lg - 1 as Section 3 does on chip.  The odd bins are
// the L/2-point DFT of the twiddled difference of the window's halves
// (eq. (3)): the first pass forms it while loading x (IN_DIFF), so the chain
// moves half the points.  The even bins are the sums of the child windows'
// bins at level lg - 1 (eq. (2)): the last pass (OUT_REC) loads those with
// its data and stores both bins of each k side by side.  Level 18 and level
// 17 share their first pass (pass_head2_kernel: both halves and their
// twiddled difference from one read of x) and their last pass
// (pass_tail2_kernel: level 17's two windows give level 18's even bins in
// registers); those two launches also carry level 17 of the signals of
// order 17, whose workgroups follow the pairs'.
#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"

namespace mrdft {

// LDS column of r points: element s at column * kColStride(r) + padc(s).  The
// stride (one spare element per 32 inside a column, plus 1 or 2) keeps the
// column-wise accesses of the loads and stores and the strided accesses of
// the Stockham steps spread over the banks (a model of the 64 banks for the
// radices used: 40-65 % fewer conflict cycles than a stride of r + 1); it
// stays within r + r/16 per column.
constexpr int kColStride(int r) { return r + (r >> 5) + (r >= 256 ? 2 : r == 32 ? 0 : 1); }

// Points, threads and LDS of a pass workgroup of 2^LP points.
template <int LP>
struct PassShape {
    static constexpr int kPoints = 1 << LP;
    static constexpr int kThreads = kPoints / 16;     // 16 points per thread
    static constexpr int kTwLog = LP - 4;             // largest radix (16 columns); w_{2^kTwLog} in LDS
    static constexpr int kLdsFloat2 = kPoints + kPoints / 16 + (1 << kTwLog);
    static constexpr size_t kLdsBytes = sizeof(float2) * kLdsFloat2;
};

// w_{2^lg}^e (lg <= TL) from a table of w_{2^TL} in LDS.
template <int TL>
struct TwLds {
    const float2* t;
    __device__ __forceinline__ float2 operator()(int lg, int e) const {
        return t[(e << (TL - lg)) & ((1 << TL) - 1)];
    }
};

// The r-point FFTs (r = 2^rl) of the workgroup's 2^LP / r columns: a first
// step of radix 2, 4 or 8 if rl is not a multiple of 4, then radix 16; every
// step has 2^LP / radix jobs over the threads.
template <int LP, bool INV>
__device__ __forceinline__ void column_fft(float2* B, int rl, const float2* T, int tid) {
    using Sh = PassShape<LP>;
    const int fst = kColStride(1 << rl);
    const int nc = Sh::kPoints >> rl;
    int lgNs = 0;
    const int rem = rl & 3;
    const TwLds<Sh::kTwLog> tw{T};
    constexpr int J = Sh::kPoints / Sh::kThreads;     // jobs per thread of a radix-1 step
    constexpr int NT = Sh::kThreads;
    if (rem == 1) { lds_step<2, J / 2, INV, false, true>(B, rl, 0, fst, 1, nc, tw, tid, NT); lgNs = 1; }
    else if (rem == 2) { lds_step<4, J / 4, INV, false, true>(B, rl, 0, fst, 1, nc, tw, tid, NT); lgNs = 2; }
    else if (rem == 3) { lds_step<8, J / 8, INV, false, true>(B, rl, 0, fst, 1, nc, tw, tid, NT); lgNs = 3; }
    while (lgNs < rl) {
        lds_step<16, J / 16, INV, false, true>(B, rl, lgNs, fst, 1, nc, tw, tid, NT);
        lgNs += 4;
    }
}

extern __shared__ float2 g_pass_lds[];

template <int LP, bool INV, int IN_KIND, int OUT_KIND>
__global__ __launch_bounds__(PassShape<LP>::kThreads) void pass_kernel(const void* __restrict__ in,
                                                                       void* __restrict__ out, PassGeom g,
                                                                       const float2* __restrict__ tab,
                                                                       const double2* __restrict__ hi,
                                                                       const double2* __restrict__ lo) {
    using Sh = PassShape<LP>;
    constexpr int kPassPoints = Sh::kPoints, kPassThreads = Sh::kThreads;
    float2* const B = g_pass_lds;                      // nc columns of r + 1
    float2* const T = g_pass_lds + kPassPoints + (kPassPoints >> 4);   // w_{2^(LP-4)}^e for the column FFT steps
    const int rl = g.r_log;
    const int r = 1 << rl;
    const int fst = kColStride(r);
    const int lnc = LP - rl;                           // log2 of the columns per workgroup
    const int nc = 1 << lnc;
    const int64_t L = (int64_t)1 << g.lg;
    const int64_t cols = L >> rl;                      // columns j per window
    const int64_t jblocks = cols >> lnc;
    const int64_t blk = blockIdx.x;
    const int64_t gwin = blk / jblocks;
    const int64_t j0 = (blk - gwin * jblocks) << lnc;
    const int64_t b = gwin / g.wps, W = gwin - b * g.wps;
    constexpr bool kDiff = IN_KIND == IN_DIFF || IN_KIND == IN_DIFF_R32;
    constexpr bool kPairIn = IN_KIND == IN_HALF_PAIR || IN_KIND == IN_R32_PAIR, kPairOut = OUT_KIND == OUT_ADD_R32_PAIR;
    // paired chains: block window gwin is the pair of windows 2 gwin, 2 gwin + 1
    // of the (wps, signal tables, strides) geometry; the second may be absent
    const bool has2 = (kPairIn || kPairOut) && 2 * gwin + 1 < g.pair_nwin;
    auto in_base = [&](int64_t w) {
        const int64_t bw = w / g.wps;
        return (g.in_sig ? g.in_sig[bw] : bw * g.in_stride) + (w - bw * g.wps) * (IN_KIND == IN_HALF_PAIR ? L / 2 : L);
    };
    auto out_base = [&](int64_t w) {
        const int64_t bw = w / g.wps;
        return (g.out_sig ? g.out_sig[bw] : bw * g.out_stride) + (w - bw * g.wps) * L;
    };
    const int64_t ib = kPairIn ? in_base(2 * gwin)
                               : (g.in_sig ? g.in_sig[b] : b * g.in_stride) +
                                     W * (IN_KIND == IN_HALF ? L / 2 : kDiff ? 2 * L : L);
    const int64_t ib2 = kPairIn && has2 ? in_base(2 * gwin + 1) : ib;
    const int64_t ob = kPairOut ? out_base(2 * gwin)
                                : (g.out_sig ? g.out_sig[b] : b * g.out_stride) +
                                      W * (OUT_KIND == OUT_HALF ? L / 2 : OUT_KIND == OUT_REC ? 2 * L : L);
    const int64_t ob2 = kPairOut && has2 ? out_base(2 * gwin + 1) : ob;
    const int tid = threadIdx.x;
    const int ns_log = g.ns_log;
    const int64_t nsm = ((int64_t)1 << ns_log) - 1;
    constexpr int kRowsPerThread = kPassPoints / kPassThreads;

    {
        // thread: column jj = tid mod nc, rows s = s0 + (256 / nc) i (s0 = tid / nc),
        // 16 rows per thread; all of the thread's loads are issued before the
        // first one is used
        const int jj = tid & (nc - 1), s0 = tid >> lnc;
        const int rstep = kPassThreads >> lnc;
        const int64_t j = j0 + jj;
        const int tlg = ns_log + rl;
        // Inputs are read once per pass, in 128-byte runs scattered over the
        // window: loaded with the non-temporal hint, so that they do not
        // displace the scratch written for the next pass (measured: the two
        // passes of levels 17 and 18 of the ragged batch 598 -> 553 us; the
        // same hint on the stores was slower)
        typedef float f2v __attribute__((ext_vector_type(2)));
        float2 v[kRowsPerThread];
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            const int s = s0 + rstep * i;
            const int64_t idx = ib + j + (int64_t)s * cols;
            if constexpr (IN_KIND == IN_R32) {
                v[i] = make_float2(__builtin_nontemporal_load((const float*)in + idx), 0.0f);
            } else if constexpr (IN_KIND == IN_DIFF_R32) {
                const float* xr = (const float*)in + idx;
                v[i] = make_float2(__builtin_nontemporal_load(xr) - __builtin_nontemporal_load(xr + L), 0.0f);
            } else if constexpr (IN_KIND == IN_DIFF) {
                const f2v a = __builtin_nontemporal_load((const f2v*)((const float2*)in + idx));
                const f2v c = __builtin_nontemporal_load((const f2v*)((const float2*)in + idx + L));
                v[i] = make_float2(a.x - c.x, a.y - c.y);
            } else if constexpr (IN_KIND == IN_HALF) {
                v[i] = half_bin((const float2*)in + ib, idx - ib, L, g.half_scale);   // first pass: bin idx - ib
            } else if constexpr (IN_KIND == IN_R32_PAIR) {
                const int64_t n = idx - ib;             // sample n of both windows
                v[i] = make_float2(__builtin_nontemporal_load((const float*)in + idx),
                                   has2 ? __builtin_nontemporal_load((const float*)in + ib2 + n) : 0.0f);
            } else if constexpr (kPairIn) {
                const int64_t n = idx - ib;             // bin n of both windows
                const float2 h1 = half_bin((const float2*)in + ib, n, L, g.half_scale);
                const float2 h2 = has2 ? half_bin((const float2*)in + ib2, n, L, g.half_scale) : make_float2(0.0f, 0.0f);
                v[i] = make_float2(h1.x - h2.y, h1.y + h2.x);
            } else {
                const f2v t = __builtin_nontemporal_load((const f2v*)((const float2*)in + idx));
                v[i] = make_float2(t.x, t.y);
            }
        }
        T[tid] = tab[tid << (kTileMaxLog - Sh::kTwLog)];   // after the data loads: its wait covers them
        double2 w = make_double2(1.0, 0.0), step = make_double2(1.0, 0.0);
        if (ns_log > 0) {
            w = tw_big64(hi, lo, tlg, (j & nsm) * s0);
            step = tw_big64(hi, lo, tlg, (j & nsm) * rstep);
        } else if constexpr (kDiff) {                   // w_{2L}^n, n = j + s cols
            w = tw_big64(hi, lo, g.lg + 1, j + (int64_t)s0 * cols);
            step = tw_big64(hi, lo, g.lg + 1, (int64_t)rstep * cols);
        }
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            const int s = s0 + rstep * i;
            float2 u = v[i];
            if (ns_log > 0 || kDiff) {
                const float2 wf = make_float2((float)w.x, (float)w.y);
                u = INV ? cmulc(u, wf) : cmul(u, wf);
                w = make_double2(w.x * step.x - w.y * step.y, w.x * step.y + w.y * step.x);
            }
            B[jj * fst + padc(s)] = u;
        }
    }
    __syncthreads();
    column_fft<LP, INV>(B, rl, T, tid);

    typedef float f2v __attribute__((ext_vector_type(2)));
    float2 ev[OUT_KIND == OUT_REC ? kRowsPerThread : 1];
    if constexpr (OUT_KIND == OUT_REC) {
        // even bins 2k of the thread's outputs k (the store loop's mapping:
        // column j0 + tid mod nc, rows tid / nc + i kPassThreads / nc): bin k
        // of the two child windows, all loads in flight before the first sum
        const int64_t jo = j0 + (tid & (nc - 1));
        const float2* pv = (const float2*)out + (ob - g.rec_prev + ((jo >> ns_log) << (ns_log + rl)) + (jo & nsm) +
                                                 ((int64_t)(tid >> lnc) << ns_log));
        const int64_t dk = (int64_t)(kPassThreads >> lnc) << ns_log;
        f2v p0[kRowsPerThread], p1[kRowsPerThread];
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            p0[i] = __builtin_nontemporal_load((const f2v*)(pv + i * dk));
            p1[i] = __builtin_nontemporal_load((const f2v*)(pv + i * dk + L));
        }
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) ev[i] = make_float2(p0[i].x + p1[i].x, p0[i].y + p1[i].y);
    }

    double nacc = 0.0;                                 // OUT_NORM: this thread's squared magnitudes
    const float osc = (OUT_KIND == OUT_HALF && g.out_scale) ? g.out_scale[b * g.out_scale_m + g.lg - 1] : 1.0f;
#pragma unroll
    for (int ie = 0; ie < kRowsPerThread; ++ie) {
        const int e = tid + ie * kPassThreads;
        int jj, s;
        int64_t o;
        if (ns_log == 0) {          // outputs of column j are the r consecutive values j*r + s
            jj = e >> rl;
            s = e & (r - 1);
            o = ob + (j0 + jj) * r + s;
        } else {                    // consecutive columns -> consecutive outputs per s (within a span)
            jj = e & (nc - 1);
            s = e >> lnc;
            const int64_t j = j0 + jj;
            o = ob + ((j >> ns_log) << (ns_log + rl)) + (j & nsm) + ((int64_t)s << ns_log);
        }
        const float2 v = B[jj * fst + padc(s)];
        if constexpr (OUT_KIND == OUT_STORE) {
            ((float2*)out)[o] = v;
        } else if constexpr (OUT_KIND == OUT_NORM) {
            (void)o;
            nacc += (double)v.x * v.x + (double)v.y * v.y;
        } else if constexpr (OUT_KIND == OUT_HALF) {
            // bin k = o - ob of a real window: k < L/2 kept, the DC and
            // Nyquist real parts share slot 0, the upper half is dropped
            const int64_t k = o - ob;
            float* sl = (float*)((float2*)out + ob);
            const float2 w = g.out_scale ? make_float2(v.x * osc, v.y * osc) : v;
            if (k == 0) sl[0] = w.x;
            else if (k == L / 2) sl[1] = w.x;
            else if (k < L / 2) ((float2*)out)[o] = w;
        } else if constexpr (OUT_KIND == OUT_REC) {
            float2* q = (float2*)out + ob + 2 * (o - ob);
            q[0] = ev[ie];
            q[1] = v;
        } else if constexpr (kPairOut) {
            const int64_t k = o - ob;
            float* p1 = (float*)out + o;
            *p1 += v.x;
            if (has2) {
                float* p2 = (float*)out + ob2 + k;
                *p2 += v.y;
            }
        } else if constexpr (OUT_KIND == OUT_ADD_C64) {
            float2* p = (float2*)out + o;
            *p = cadd(*p, v);
        } else {
            float* p = (float*)out + o;
            *p += v.x;
        }
    }
    if constexpr (OUT_KIND == OUT_NORM) {
        // block sum, then one FP64 atomic per workgroup into sums[b * out_stride + lg - 1]
        __syncthreads();                               // B is free again
        double* red = reinterpret_cast<double*>(B);
        red[tid] = nacc;
        __syncthreads();
        for (int h = kPassThreads / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        // a pair chain (windows 2 gwin, 2 gwin + 1 of one signal) adds to that signal's sum
        const int64_t bn = g.pair_nwin > 0 ? (2 * gwin) / g.wps : b;
        if (tid == 0) atomicAdd((double*)out + bn * g.out_stride + g.lg - 1, red[0]);
    }
}

// Heads of two chains from one read of x: the first passes of level lg (its
// two windows inside a window of level lg + 1) and of the recurrence chain
// of level lg + 1 (the twiddled difference of those two windows, eq. (3))
// use the same columns j + s L / r of the same samples (L = 2^lg, radix r).
// A workgroup loads its 16 columns of both halves once and runs three column
// FFTs through LDS: the first half (level lg, window 2 W), the second half
// (window 2 W + 1), both written to out_lo in the lower chain's dense
// layout, and (x0 - x1) w_{2L}^n, written to out_hi in the upper chain's.
// g: lg, r_log (the first radix), nwin / wps / in_sig / in_stride of the
// windows of level lg + 1; outputs dense (window index x L).
// gs (gs.nwin may be 0): windows of level lg whose signals end at that level
// (no level lg + 1): the plain first pass of their chain (one FFT, to out_s),
// run by the workgroups after the pairs' so that the last, partly filled
// round of the pair workgroups is shared with this shorter work.
template <int LP, int IN_KIND>
__global__ __launch_bounds__(PassShape<LP>::kThreads, 4) void pass_head2_kernel(const void* __restrict__ in,
                                                                             float2* __restrict__ out_lo,
                                                                             float2* __restrict__ out_hi, PassGeom g,
                                                                             float2* __restrict__ out_s, PassGeom gs,
                                                                             const float2* __restrict__ tab,
                                                                             const double2* __restrict__ hi,
                                                                             const double2* __restrict__ lo) {
    using Sh = PassShape<LP>;
    constexpr int kPassPoints = Sh::kPoints, kPassThreads = Sh::kThreads;
    constexpr int kRowsPerThread = kPassPoints / kPassThreads;
    typedef float f2v __attribute__((ext_vector_type(2)));
    float2* const B = g_pass_lds;
    float2* const T = g_pass_lds + kPassPoints + (kPassPoints >> 4);
    const int rl = g.r_log;
    const int r = 1 << rl;
    const int fst = kColStride(r);
    const int lnc = LP - rl;
    const int nc = 1 << lnc;
    const int64_t L = (int64_t)1 << g.lg;
    const int64_t cols = L >> rl;
    const int64_t jblocks = cols >> lnc;
    const int64_t npair = g.nwin * jblocks;
    const bool single = (int64_t)blockIdx.x >= npair;              // uniform over the workgroup
    const int64_t blk = single ? (int64_t)blockIdx.x - npair : (int64_t)blockIdx.x;
    const int64_t gwin = blk / jblocks;
    const int64_t j0 = (blk - gwin * jblocks) << lnc;
    const int tid = threadIdx.x;
    const int jj = tid & (nc - 1), s0 = tid >> lnc;
    const int rstep = kPassThreads >> lnc;
    const int64_t j = j0 + jj;
    T[tid] = tab[tid << (kTileMaxLog - Sh::kTwLog)];
    // one column-FFT phase: the data already in LDS, the FFTs, the r
    // consecutive outputs of each column to dst (first pass: span 1).  The
    // thread index goes through an empty asm per phase, so that the LDS
    // addresses derived from it are formed per phase, not kept in registers
    // across the three.
    auto to_lds = [&](const float2* v) __attribute__((always_inline)) {
        int t = tid;
        asm volatile("" : "+v"(t));
        const int tj = t & (nc - 1), ts = t >> lnc;
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) B[tj * fst + padc(ts + rstep * i)] = v[i];
    };
    auto fft_out = [&](float2* __restrict__ dst) __attribute__((always_inline)) {
        int t = tid;
        asm volatile("" : "+v"(t));
        __syncthreads();
        column_fft<LP, false>(B, rl, T, t);
#pragma unroll
        for (int ie = 0; ie < kRowsPerThread; ++ie) {
            const int e = t + ie * kPassThreads;
            const int jo = e >> rl, s = e & (r - 1);
            dst[(j0 + jo) * r + s] = B[jo * fst + padc(s)];
        }
        __syncthreads();                               // B read before the next phase writes it
    };
    auto load = [&](int64_t idx) __attribute__((always_inline)) {
        if constexpr (IN_KIND == IN_R32) {
            return make_float2(__builtin_nontemporal_load((const float*)in + idx), 0.0f);
        } else {
            const f2v a = __builtin_nontemporal_load((const f2v*)((const float2*)in + idx));
            return make_float2(a.x, a.y);
        }
    };
    if (single) {                                      // one window: its first pass only
        const int64_t b = gwin / gs.wps, W = gwin - b * gs.wps;
        const int64_t ib = (gs.in_sig ? gs.in_sig[b] : b * gs.in_stride) + W * L;
        float2 xs[kRowsPerThread];
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) xs[i] = load(ib + j + (int64_t)(s0 + rstep * i) * cols);
        to_lds(xs);
        fft_out(out_s + gwin * L);
        return;
    }
    const int64_t b = gwin / g.wps, W = gwin - b * g.wps;
    const int64_t ib = (g.in_sig ? g.in_sig[b] : b * g.in_stride) + W * 2 * L;
    float2 x0[kRowsPerThread], x1[kRowsPerThread];
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
        const int64_t idx = ib + j + (int64_t)(s0 + rstep * i) * cols;
        x0[i] = load(idx);
        x1[i] = load(idx + L);
    }
    // first half into LDS; its registers then take the twiddled difference
    // (x0 - x1) w_{2L}^n, n = j + s cols (FP64 recurrence), before the FFTs
    to_lds(x0);
    {
        double2 w = tw_big64(hi, lo, g.lg + 1, j + (int64_t)s0 * cols);
        const double2 step = tw_big64(hi, lo, g.lg + 1, (int64_t)rstep * cols);
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            x0[i] = cmul(make_float2(x0[i].x - x1[i].x, x0[i].y - x1[i].y), make_float2((float)w.x, (float)w.y));
            w = make_double2(w.x * step.x - w.y * step.y, w.x * step.y + w.y * step.x);
        }
    }
    fft_out(out_lo + (2 * gwin) * L);
    to_lds(x1);
    fft_out(out_lo + (2 * gwin + 1) * L);
    to_lds(x0);
    fft_out(out_hi + gwin * L);
}

template <int LP>
static hipError_t launch_head2_t(int in_kind, const void* in, float2* out_lo, float2* out_hi, const PassGeom& g,
                                 float2* out_s, const PassGeom& gs, const Twiddles& tw, hipStream_t s) {
    using Sh = PassShape<LP>;
    if (g.lg < LP) return hipErrorInvalidValue;
    const int64_t nblk = (g.nwin + gs.nwin) << (g.lg - LP);
    if (nblk <= 0) return hipSuccess;
    if (nblk > INT32_MAX) return hipErrorInvalidValue;
    static const bool attr = [] {
        (void)hipFuncSetAttribute((const void*)pass_head2_kernel<LP, IN_C64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  Sh::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_head2_kernel<LP, IN_R32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  Sh::kLdsBytes);
        return true;
    }();
    (void)attr;
    dim3 grid((unsigned)nblk), block(Sh::kThreads);
    if (in_kind == IN_R32)
        hipLaunchKernelGGL((pass_head2_kernel<LP, IN_R32>), grid, block, Sh::kLdsBytes, s, in, out_lo, out_hi, g,
                           out_s, gs, tw.tile, tw.hi, tw.lo);
    else
        hipLaunchKernelGGL((pass_head2_kernel<LP, IN_C64>), grid, block, Sh::kLdsBytes, s, in, out_lo, out_hi, g,
                           out_s, gs, tw.tile, tw.hi, tw.lo);
    return hipGetLastError();
}

hipError_t launch_pass_head2(int in_kind, const void* in, float2* out_lo, float2* out_hi, const PassGeom& g,
                             float2* out_s, const PassGeom* gs, const Twiddles& tw, hipStream_t s) {
    if (g.r_log < 4 || g.r_log > kPassMaxLog || g.lg + 1 > kMaxOrder || (in_kind != IN_C64 && in_kind != IN_R32) ||
        g.nwin < 0)
        return hipErrorInvalidValue;
    PassGeom one = g;                                  // no single windows unless given
    one.nwin = 0;
    one.wps = 1;
    one.in_sig = nullptr;
    one.in_stride = 0;
    if (gs) {
        if (gs->lg != g.lg || gs->r_log != g.r_log || gs->nwin < 0 || (gs->nwin > 0 && (!out_s || gs->wps <= 0)))
            return hipErrorInvalidValue;
        one = *gs;
    }
    return g.r_log <= kPassSmallMaxLog
               ? launch_head2_t<kPassSmallLog>(in_kind, in, out_lo, out_hi, g, out_s, one, tw, s)
               : launch_head2_t<kPassBigLog>(in_kind, in, out_lo, out_hi, g, out_s, one, tw, s);
}

// Tails of the same two chains: the last pass of level lg (windows 2 W and
// 2 W + 1 of level lg) and the last pass of level lg + 1's recurrence chain
// (window W) have the same radix and span, so the outputs k = j + s Ns of a
// column block are the same positions in all three.  A workgroup runs the
// three column FFTs one after the other: level lg's two windows are stored
// and their sum kept in registers, which is level lg + 1's even bin 2k
// (eq. (2)) beside the odd bin 2k + 1 of the third FFT: level lg's spectra
// are not read back.
// g: lg, r_log and ns_log of the last pass (ns_log + r_log = lg), nwin / wps
// of the windows of level lg + 1, out_sig / out_stride of both levels;
// s_lo / s_hi: the two chains' scratch (dense, window index x L).
// gs (gs.nwin may be 0): level lg of signals that end at that level, the
// plain last pass of their chain (scratch s_s, output y_s with gs's wps /
// out_sig / out_stride), after the pair workgroups as in the head.
template <int LP>
__global__ __launch_bounds__(PassShape<LP>::kThreads, 4) void pass_tail2_kernel(const float2* __restrict__ s_lo,
                                                                             const float2* __restrict__ s_hi,
                                                                             float2* __restrict__ y_lo,
                                                                             float2* __restrict__ y_hi, PassGeom g,
                                                                             const float2* __restrict__ s_s,
                                                                             float2* __restrict__ y_s, PassGeom gs,
                                                                             const float2* __restrict__ tab,
                                                                             const double2* __restrict__ hi,
                                                                             const double2* __restrict__ lo) {
    using Sh = PassShape<LP>;
    constexpr int kPassPoints = Sh::kPoints, kPassThreads = Sh::kThreads;
    constexpr int kRowsPerThread = kPassPoints / kPassThreads;
    typedef float f2v __attribute__((ext_vector_type(2)));
    float2* const B = g_pass_lds;
    float2* const T = g_pass_lds + kPassPoints + (kPassPoints >> 4);
    const int rl = g.r_log;
    const int fst = kColStride(1 << rl);
    const int lnc = LP - rl;
    const int nc = 1 << lnc;
    const int64_t L = (int64_t)1 << g.lg;
    const int64_t cols = L >> rl;
    const int64_t jblocks = cols >> lnc;
    const int64_t npair = g.nwin * jblocks;
    const bool single = (int64_t)blockIdx.x >= npair;              // uniform over the workgroup
    const int64_t blk = single ? (int64_t)blockIdx.x - npair : (int64_t)blockIdx.x;
    const int64_t gwin = blk / jblocks;
    const int64_t j0 = (blk - gwin * jblocks) << lnc;
    const int ns_log = g.ns_log;
    const int64_t nsm = ((int64_t)1 << ns_log) - 1;
    const int tid = threadIdx.x;
    T[tid] = tab[tid << (kTileMaxLog - Sh::kTwLog)];
    // one FFT phase over the L-point window at src: load, span twiddles,
    // column FFTs; the results stay in LDS for the caller's output loop
    auto phase = [&](const float2* __restrict__ src) __attribute__((always_inline)) {
        int t = tid;
        asm volatile("" : "+v"(t));
        const int tj = t & (nc - 1), ts = t >> lnc;
        const int rstep = kPassThreads >> lnc;
        const int64_t j = j0 + tj;
        float2 v[kRowsPerThread];
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            const f2v a = __builtin_nontemporal_load((const f2v*)(src + j + (int64_t)(ts + rstep * i) * cols));
            v[i] = make_float2(a.x, a.y);
        }
        double2 w = tw_big64(hi, lo, ns_log + rl, (j & nsm) * ts);
        const double2 step = tw_big64(hi, lo, ns_log + rl, (j & nsm) * rstep);
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i) {
            B[tj * fst + padc(ts + rstep * i)] = cmul(v[i], make_float2((float)w.x, (float)w.y));
            w = make_double2(w.x * step.x - w.y * step.y, w.x * step.y + w.y * step.x);
        }
        __syncthreads();
        column_fft<LP, false>(B, rl, T, t);
    };
    // output ie of this thread: column j0 + (e mod nc), row e / nc, at
    // ((j >> ns) << (ns + r)) + (j mod 2^ns) + (row << ns) of the window
    // (offsets inside a window fit 32 bits)
    auto out_pos = [&](int t, int ie, int& lds) __attribute__((always_inline)) {
        const int e = t + ie * kPassThreads;
        const int jj = e & (nc - 1), s = e >> lnc;
        const int j = (int)j0 + jj;
        lds = jj * fst + padc(s);
        return ((j >> ns_log) << (ns_log + rl)) + (j & (int)nsm) + (s << ns_log);
    };
    if (single) {                                      // one window: its last pass only
        const int64_t b = gwin / gs.wps, W = gwin - b * gs.wps;
        const int64_t obase = gs.out_sig ? gs.out_sig[b] : b * gs.out_stride;
        phase(s_s + gwin * L);
        int t = tid;
        asm volatile("" : "+v"(t));
        float2* const yw = y_s + obase + W * L;
#pragma unroll
        for (int ie = 0; ie < kRowsPerThread; ++ie) {
            int li;
            const int o = out_pos(t, ie, li);
            const float2 vo = B[li];
            __builtin_nontemporal_store(f2v{vo.x, vo.y}, (f2v*)(yw + o));
        }
        return;
    }
    const int64_t b = gwin / g.wps, W = gwin - b * g.wps;
    const int64_t obase = g.out_sig ? g.out_sig[b] : b * g.out_stride;
    float2 esum[kRowsPerThread];
    auto lower = [&](int h) __attribute__((always_inline)) {
        phase(s_lo + (2 * gwin + h) * L);
        int t = tid;
        asm volatile("" : "+v"(t));
        float2* const yw = y_lo + obase + (2 * W + h) * L;
#pragma unroll
        for (int ie = 0; ie < kRowsPerThread; ++ie) {
            int li;
            const int o = out_pos(t, ie, li);
            const float2 vo = B[li];
            __builtin_nontemporal_store(f2v{vo.x, vo.y}, (f2v*)(yw + o));
            esum[ie] = h ? cadd(esum[ie], vo) : vo;
        }
        __syncthreads();
    };
    lower(0);
    lower(1);
    phase(s_hi + gwin * L);
    {
        int t = tid;
        asm volatile("" : "+v"(t));
        float2* const yh = y_hi + obase + W * 2 * L;
#pragma unroll
        for (int ie = 0; ie < kRowsPerThread; ++ie) {
            int li;
            const int o = out_pos(t, ie, li);
            const float2 vo = B[li];
            typedef float f4v __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(f4v{esum[ie].x, esum[ie].y, vo.x, vo.y}, (f4v*)(yh + 2 * o));
        }
    }
}

template <int LP>
static hipError_t launch_tail2_t(const float2* s_lo, const float2* s_hi, float2* y_lo, float2* y_hi, const PassGeom& g,
                                 const float2* s_s, float2* y_s, const PassGeom& gs, const Twiddles& tw,
                                 hipStream_t s) {
    using Sh = PassShape<LP>;
    if (g.lg < LP) return hipErrorInvalidValue;
    const int64_t nblk = (g.nwin + gs.nwin) << (g.lg - LP);
    if (nblk <= 0) return hipSuccess;
    if (nblk > INT32_MAX) return hipErrorInvalidValue;
    static const bool attr = [] {
        (void)hipFuncSetAttribute((const void*)pass_tail2_kernel<LP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  Sh::kLdsBytes);
        return true;
    }();
    (void)attr;
    dim3 grid((unsigned)nblk), block(Sh::kThreads);
    hipLaunchKernelGGL((pass_tail2_kernel<LP>), grid, block, Sh::kLdsBytes, s, s_lo, s_hi, y_lo, y_hi, g, s_s, y_s,
                       gs, tw.tile, tw.hi, tw.lo);
    return hipGetLastError();
}

hipError_t launch_pass_tail2(const float2* s_lo, const float2* s_hi, float2* y_lo, float2* y_hi, const PassGeom& g,
                             const float2* s_s, float2* y_s, const PassGeom* gs, const Twiddles& tw, hipStream_t s) {
    if (g.r_log < 4 || g.r_log > kPassMaxLog || g.ns_log <= 0 || g.ns_log + g.r_log != g.lg || g.lg + 1 > kMaxOrder ||
        g.nwin < 0)
        return hipErrorInvalidValue;
    PassGeom one = g;                                  // no single windows unless given
    one.nwin = 0;
    one.wps = 1;
    one.out_sig = nullptr;
    one.out_stride = 0;
    if (gs) {
        if (gs->lg != g.lg || gs->r_log != g.r_log || gs->ns_log != g.ns_log || gs->nwin < 0 ||
            (gs->nwin > 0 && (!s_s || !y_s || gs->wps <= 0)))
            return hipErrorInvalidValue;
        one = *gs;
    }
    return g.r_log <= kPassSmallMaxLog
               ? launch_tail2_t<kPassSmallLog>(s_lo, s_hi, y_lo, y_hi, g, s_s, y_s, one, tw, s)
               : launch_tail2_t<kPassBigLog>(s_lo, s_hi, y_lo, y_hi, g, s_s, y_s, one, tw, s);
}

// Lets every large-workgroup instantiation use its dynamic LDS (above 64 KB).
template <int LP, bool INV, int IK>
static void allow_pass_lds() {
    const size_t b = PassShape<LP>::kLdsBytes;
    (void)hipFuncSetAttribute((const void*)pass_kernel<LP, INV, IK, OUT_STORE>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)pass_kernel<LP, INV, IK, OUT_HALF>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)pass_kernel<LP, INV, IK, OUT_NORM>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)pass_kernel<LP, INV, IK, OUT_ADD_C64>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute((const void*)pass_kernel<LP, INV, IK, OUT_ADD_R32>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
}
struct PassLdsInit {
    PassLdsInit() {
        allow_pass_lds<kPassBigLog, false, IN_R32>();
        allow_pass_lds<kPassBigLog, false, IN_C64>();
        allow_pass_lds<kPassBigLog, true, IN_R32>();
        allow_pass_lds<kPassBigLog, true, IN_C64>();
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, true, IN_HALF, OUT_STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, false, IN_R32_PAIR, OUT_STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, true, IN_HALF_PAIR, OUT_STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, true, IN_C64, OUT_ADD_R32_PAIR>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, false, IN_DIFF, OUT_STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, false, IN_DIFF_R32, OUT_STORE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
        (void)hipFuncSetAttribute((const void*)pass_kernel<kPassBigLog, false, IN_C64, OUT_REC>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, PassShape<kPassBigLog>::kLdsBytes);
    }
};

template <int LP, bool INV>
static hipError_t launch_pass_t(int in_kind, int out_kind, const void* in, void* out, const PassGeom& g,
                                const Twiddles& tw, hipStream_t s) {
    using Sh = PassShape<LP>;
    if (g.lg < LP) return hipErrorInvalidValue;        // a workgroup's points lie in one window
    const int64_t nblk = g.nwin << (g.lg - LP);
    if (nblk <= 0) return hipSuccess;
    dim3 grid((unsigned)nblk), block(Sh::kThreads);
#define MRDFT_PASS(IK, OK)                                                                                      \
    hipLaunchKernelGGL((pass_kernel<LP, INV, IK, OK>), grid, block, Sh::kLdsBytes, s, in, out, g, tw.tile, tw.hi, \
                       tw.lo)
    if (in_kind == IN_R32_PAIR) {
        // the norm chains of the loss: pairs of windows of one signal
        if constexpr (INV) {
            return hipErrorInvalidValue;
        } else {
            if (out_kind != OUT_STORE || g.pair_nwin <= 0 || g.nwin * 2 != g.pair_nwin || g.wps % 2 || g.ns_log != 0)
                return hipErrorInvalidValue;
            MRDFT_PASS(IN_R32_PAIR, OUT_STORE);
        }
    } else if (in_kind == IN_HALF_PAIR || out_kind == OUT_ADD_R32_PAIR) {
        // paired chains of the real adjoint: first passes read two packed
        // windows, last passes add into two real windows
        if constexpr (!INV) {
            return hipErrorInvalidValue;
        } else {
            if (g.pair_nwin <= 0 || g.nwin != (g.pair_nwin + 1) / 2) return hipErrorInvalidValue;
            if (in_kind == IN_HALF_PAIR) {
                if (out_kind != OUT_STORE) return hipErrorInvalidValue;
                MRDFT_PASS(IN_HALF_PAIR, OUT_STORE);
            } else {
                if (in_kind != IN_C64 || g.ns_log == 0) return hipErrorInvalidValue;
                MRDFT_PASS(IN_C64, OUT_ADD_R32_PAIR);
            }
        }
    } else if (in_kind == IN_HALF) {
        if constexpr (INV) {                          // first adjoint passes only
            if (out_kind != OUT_STORE) return hipErrorInvalidValue;
            MRDFT_PASS(IN_HALF, OUT_STORE);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (in_kind == IN_DIFF || in_kind == IN_DIFF_R32 || out_kind == OUT_REC) {
        // the recurrence chains of the forward: IN_DIFF first passes, OUT_REC last passes
        if constexpr (INV) {
            return hipErrorInvalidValue;
        } else {
            if (out_kind == OUT_REC) {
                if (in_kind != IN_C64 || g.ns_log == 0 || g.rec_prev < 2 * ((int64_t)1 << g.lg))
                    return hipErrorInvalidValue;
                MRDFT_PASS(IN_C64, OUT_REC);
            } else {
                if (out_kind != OUT_STORE || g.ns_log != 0 || g.lg + 1 > kMaxOrder) return hipErrorInvalidValue;
                if (in_kind == IN_DIFF) MRDFT_PASS(IN_DIFF, OUT_STORE);
                else MRDFT_PASS(IN_DIFF_R32, OUT_STORE);
            }
        }
    } else if (in_kind == IN_R32) {
        if (out_kind == OUT_STORE) MRDFT_PASS(IN_R32, OUT_STORE);
        else if (out_kind == OUT_HALF) MRDFT_PASS(IN_R32, OUT_HALF);
        else if (out_kind == OUT_NORM) MRDFT_PASS(IN_R32, OUT_NORM);
        else if (out_kind == OUT_ADD_C64) MRDFT_PASS(IN_R32, OUT_ADD_C64);
        else MRDFT_PASS(IN_R32, OUT_ADD_R32);
    } else {
        if (out_kind == OUT_STORE) MRDFT_PASS(IN_C64, OUT_STORE);
        else if (out_kind == OUT_HALF) MRDFT_PASS(IN_C64, OUT_HALF);
        else if (out_kind == OUT_NORM) MRDFT_PASS(IN_C64, OUT_NORM);
        else if (out_kind == OUT_ADD_C64) MRDFT_PASS(IN_C64, OUT_ADD_C64);
        else MRDFT_PASS(IN_C64, OUT_ADD_R32);
    }
#undef MRDFT_PASS
    return hipGetLastError();
}

hipError_t launch_pass(bool inv, int in_kind, int out_kind, const void* in, void* out, const PassGeom& g,
                       const Twiddles& tw, hipStream_t s) {
    if (g.r_log < 4 || g.r_log > kPassMaxLog) return hipErrorInvalidValue;
    if (g.r_log <= kPassSmallMaxLog)
        return inv ? launch_pass_t<kPassSmallLog, true>(in_kind, out_kind, in, out, g, tw, s)
                   : launch_pass_t<kPassSmallLog, false>(in_kind, out_kind, in, out, g, tw, s);
    static PassLdsInit once;
    return inv ? launch_pass_t<kPassBigLog, true>(in_kind, out_kind, in, out, g, tw, s)
               : launch_pass_t<kPassBigLog, false>(in_kind, out_kind, in, out, g, tw, s);
}

}  // namespace mrdft
