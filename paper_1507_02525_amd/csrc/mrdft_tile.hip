// On-chip tile kernels: levels 1..t of a 2^t-sample tile (t <= 12).
//
// Forward (Section 3, eq. (4)).  With every level kept in natural bin order,
// the factors of eq. (4) reduce to, for level i (window L = 2^i, M = L/2):
//   even bins  Y^(i)[w][2k]   = Y^(i-1)[2w][k] + Y^(i-1)[2w+1][k]          (U^(i), eq. (2))
//   odd bins   Y^(i)[w][2k+1] = DFT_M( (x[wL+q] - x[wL+q+M]) * w_L^q )[k]   (V^(i), eq. (3),
//                                                                            then D^(i), F^(i))
// so each level reuses the level below for half of its bins and runs one
// half-length FFT of the twiddled window difference for the other half.  The
// permutation Gamma is absorbed by the natural-order (Stockham) FFT.
//
// Levels 1..min(t,4) run in registers on 16-sample chunks; higher levels keep
// x and the previous level in LDS and run the odd-bin FFT as radix-2/4/8
// Stockham steps.  Every level is streamed to HBM with 16-byte stores.
//
// Adjoint: the transpose of the same recurrence, top level first.  The odd-bin
// gradient goes through the conjugate FFT and the conjugate twiddles into x
// (added at q, subtracted at q + M); the even-bin gradient is added to both
// child windows of the level below.
#include "mrdft_internal.h"
#include "mrdft_lds_fft.h"

namespace mrdft {

template <bool REAL>
struct XType {
    using T = float2;
};
template <>
struct XType<true> {
    using T = float;
};

// LDS of one launch, sized for its largest tile 2^tmax (dynamic shared
// memory): small tiles leave room for more workgroups per CU.
extern __shared__ __align__(16) unsigned char g_tile_lds[];
template <typename XT>
struct TileLds {
    XT* X;
    float2* P;
    float2* F;
    float2* Q;
};
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }
template <typename XT>
__host__ __device__ constexpr size_t tile_lds_bytes(int tmax) {
    return align16(sizeof(XT) * padded_size(1 << tmax)) + sizeof(float2) * padded_size(1 << tmax) +
           sizeof(float2) * padded_size((1 << tmax) / 2) + sizeof(float2) * kQuarter;
}
template <typename XT>
__device__ __forceinline__ TileLds<XT> tile_lds(int tmax) {
    TileLds<XT> L;
    L.X = (XT*)g_tile_lds;
    L.P = (float2*)(g_tile_lds + align16(sizeof(XT) * padded_size(1 << tmax)));
    L.F = L.P + padded_size(1 << tmax);
    L.Q = L.F + padded_size((1 << tmax) / 2);
    return L;
}

__device__ __forceinline__ float2 to_c(float v) { return make_float2(v, 0.0f); }
__device__ __forceinline__ float2 to_c(float2 v) { return v; }

// ---------------------------------------------------------------------------
// Register phase, forward: levels 2..LC of a chunk of C = 2^LC samples.
// ---------------------------------------------------------------------------
// One level of a register chunk (C values, windows of L natural-order bins)
// to y: full spectra, or (HALF) the C/2 packed half-spectrum slots, slot 0 of
// a window = (Y[0], Y[L/2]).  16-byte stores.
template <int C, int L, bool HALF>
__device__ __forceinline__ void store_chunk(const float2* pv, float2* y) {
    float4* yo = (float4*)y;
    if constexpr (HALF) {
        constexpr int M = L / 2;
        float2 hv[C / 2];
#pragma unroll
        for (int w = 0; w < C / L; ++w) {
            hv[w * M] = make_float2(pv[w * L].x, pv[w * L + M].x);
#pragma unroll
            for (int k = 1; k < M; ++k) hv[w * M + k] = pv[w * L + k];
        }
#pragma unroll
        for (int e = 0; e < C / 4; ++e) yo[e] = make_float4(hv[2 * e].x, hv[2 * e].y, hv[2 * e + 1].x, hv[2 * e + 1].y);
    } else {
#pragma unroll
        for (int e = 0; e < C / 2; ++e) yo[e] = make_float4(pv[2 * e].x, pv[2 * e].y, pv[2 * e + 1].x, pv[2 * e + 1].y);
    }
}

template <int I, int LC, bool HALF>
struct LocalFwd {
    static __device__ __forceinline__ void run(const float2* xv, float2* pv, float2* y, int64_t ls, LevelRange lv) {
        if constexpr (I <= LC) {
            constexpr int C = 1 << LC, L = 1 << I, M = L / 2;
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
            if (lv.in(I)) store_chunk<C, L, HALF>(pv, y + (int64_t)(I - 1) * ls);
            LocalFwd<I + 1, LC, HALF>::run(xv, pv, y, ls, lv);
        }
    }
};

template <int LC, bool REAL, bool HALF>
__device__ __forceinline__ void fwd_local(const typename XType<REAL>::T* __restrict__ xin, float2* y, int64_t ls,
                                          typename XType<REAL>::T* Xs, float2* Ps, int c0, bool keep, LevelRange lv) {
    constexpr int C = 1 << LC;
    float2 xv[C], pv[C];
    if constexpr (REAL) {
        // 8-byte loads: ragged real signals are only guaranteed 8-byte aligned.
#pragma unroll
        for (int e = 0; e < C / 2; ++e) {
            float2 a = ((const float2*)xin)[e];
            xv[2 * e] = to_c(a.x);
            xv[2 * e + 1] = to_c(a.y);
        }
    } else {
#pragma unroll
        for (int e = 0; e < C / 2; ++e) {
            float4 a = ((const float4*)xin)[e];
            xv[2 * e] = make_float2(a.x, a.y);
            xv[2 * e + 1] = make_float2(a.z, a.w);
        }
    }
    // Level 1: A^(1) = I (x) H_2 (D^(1) multiplies by w_2^0 = 1).
#pragma unroll
    for (int b = 0; b < C / 2; ++b) {
        pv[2 * b] = cadd(xv[2 * b], xv[2 * b + 1]);
        pv[2 * b + 1] = csub(xv[2 * b], xv[2 * b + 1]);
    }
    if (lv.in(1)) store_chunk<C, 2, HALF>(pv, y);
    LocalFwd<2, LC, HALF>::run(xv, pv, y, ls, lv);
    if (keep) {
#pragma unroll
        for (int e = 0; e < C; ++e) {
            if constexpr (REAL) Xs[pad(c0 + e)] = xv[e].x; else Xs[pad(c0 + e)] = xv[e];
            Ps[pad(c0 + e)] = pv[e];
        }
    }
}

// First Stockham step of the odd-bin FFT at level i: its inputs are the
// twiddled window differences (x[wL+q] - x[wL+q+M]) * w_L^q read from LDS.
template <int R, int JPT, typename XT>
__device__ __forceinline__ void first_load_fwd(const XT* Xs, int i, int nw, const TwQuarter& tw, float2* v,
                                               int tid) {
    constexpr int lgR = Log2<R>::v;
    const int lgM = i - 1, M = 1 << lgM, L = 2 * M;
    const int lgper = lgM - lgR, per = 1 << lgper;
    const int jobs = nw << lgper;
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kTileThreads;
        if (J < jobs) {
            const int w = J >> lgper, j = J & (per - 1);
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int q = j + s * per;
                float2 d = csub(to_c(Xs[pad(w * L + q)]), to_c(Xs[pad(w * L + q + M)]));
                v[c * R + s] = cmul(d, tw(i, q));
            }
            dft_reg<R, false>(&v[c * R]);
        }
    }
}

// HALF (real input, tiles of at least 4 samples): packed half-spectrum
// output, job offsets and level stride in those units.
template <bool REAL, bool HALF>
__global__ __launch_bounds__(kTileThreads) void tile_fwd_kernel(const void* __restrict__ x, float2* __restrict__ Y,
                                                                const TileJob* __restrict__ jobs,
                                                                const float2* __restrict__ tab, int tmax) {
    using XT = typename XType<REAL>::T;
    const TileLds<XT> L = tile_lds<XT>(tmax);
    XT* Xs = L.X;                                     // x tile
    float2* Ps = L.P;                                 // previous level, natural bin order
    float2* Fs = L.F;                                 // odd-bin FFT work space
    float2* Qs = L.Q;                                 // twiddle quarter table

    const TileJob jb = jobs[blockIdx.x];
    const int t = jb.t;
    const int T = 1 << t;
    const int tid = threadIdx.x;
    const XT* xin = (const XT*)x + jb.in_off;
    float2* y = Y + jb.out_off;
    const int64_t ls = jb.level_stride;
    const LevelRange lv = LevelRange::unpack(jb.pad);
    const int top = t < lv.hi ? t : lv.hi;            // levels above the range are not computed

    const int lc = t < 4 ? t : 4;
    const bool keep = top > 4;
    if (keep) load_quarter(Qs, tab, tid, kTileThreads);
    if (tid < (T >> lc)) {
        const int c0 = tid << lc;
        float2* yc = y + (c0 >> (HALF ? 1 : 0));
        switch (lc) {
            case 1:
                if constexpr (!HALF) fwd_local<1, REAL, false>(xin + c0, yc, ls, Xs, Ps, c0, keep, lv);
                break;
            case 2: fwd_local<2, REAL, HALF>(xin + c0, yc, ls, Xs, Ps, c0, keep, lv); break;
            case 3: fwd_local<3, REAL, HALF>(xin + c0, yc, ls, Xs, Ps, c0, keep, lv); break;
            default: fwd_local<4, REAL, HALF>(xin + c0, yc, ls, Xs, Ps, c0, keep, lv); break;
        }
    }
    if (!keep) return;
    const TwQuarter tw{Qs};
    __syncthreads();

    for (int i = 5; i <= top; ++i) {
        const int lgM = i - 1, M = 1 << lgM, L = 2 * M;
        const int nw = T >> i;
        const int rem = lgM % 3;
        int lgNs;
        // First step: V^(i) and D^(i) folded into the loads.
        if (rem == 1) {
            float2 v[8];
            first_load_fwd<2, 4>(Xs, i, nw, tw, v, tid);
            step_store<2, 4, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
            lgNs = 1;
        } else if (rem == 2) {
            float2 v[8];
            first_load_fwd<4, 2>(Xs, i, nw, tw, v, tid);
            step_store<4, 2, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
            lgNs = 2;
        } else {
            float2 v[8];
            first_load_fwd<8, 1>(Xs, i, nw, tw, v, tid);
            step_store<8, 1, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
            lgNs = 3;
        }
        __syncthreads();
        // Middle radix-8 steps of R^(i).
        while (lgNs + 3 < lgM) {
            lds_step<8, 1, false, true>(Fs, lgM, lgNs, M, 1, nw, tw, tid, kTileThreads);
            lgNs += 3;
        }
        // Last radix-8 step: outputs stay in registers, k = j + s*Ns.
        float2 o[8];
        step_load<8, 1, false, true>(Fs, lgM, lgNs, M, 1, nw, tw, o, tid, kTileThreads);
        const int lgper = lgM - 3;
        const int jobs_last = nw << lgper;
        float2 sv[8];
        int w = 0, j = 0;
        if (tid < jobs_last) {
            w = tid >> lgper;
            j = tid & ((1 << lgper) - 1);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k = j + (s << lgper);
                sv[s] = cadd(Ps[pad(w * L + k)], Ps[pad(w * L + M + k)]);     // U^(i): even bins
            }
        }
        __syncthreads();
        if (tid < jobs_last) {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k = j + (s << lgper);
                Ps[pad(w * L + 2 * k)] = sv[s];
                Ps[pad(w * L + 2 * k + 1)] = o[s];
            }
        }
        __syncthreads();
        if (lv.in(i)) {
            float4* yo = (float4*)(y + (int64_t)(i - 1) * ls);
            if constexpr (HALF) {
                // slots 2e, 2e + 1 of window w (M >= 16: one window per pair)
                for (int e = tid; e < T / 4; e += kTileThreads) {
                    const int w = (2 * e) >> lgM, k = (2 * e) & (M - 1);
                    float2 a = Ps[pad(w * L + k)];
                    if (k == 0) a.y = Ps[pad(w * L + M)].x;
                    const float2 b = Ps[pad(w * L + k + 1)];
                    yo[e] = make_float4(a.x, a.y, b.x, b.y);
                }
            } else {
                for (int e = tid; e < T / 2; e += kTileThreads) {
                    const float2 a = Ps[pad(2 * e)], b = Ps[pad(2 * e + 1)];
                    yo[e] = make_float4(a.x, a.y, b.x, b.y);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------
template <int I>
struct LocalAdj {
    // G: level-I gradient (natural order) for a chunk of C values; gx accumulates.
    template <int C>
    static __device__ __forceinline__ void run(float2* G, float2* gx, const float2* __restrict__ gy, int64_t ls,
                                               LevelRange lv) {
        if constexpr (I >= 2) {
            constexpr int L = 1 << I, M = L / 2;
            float2 gn[C];
            const float4* gl = (const float4*)(gy + (int64_t)(I - 2) * ls);   // gY^(I-1) chunk
            const bool have = lv.in(I - 1);                                   // levels outside the range: zero
#pragma unroll
            for (int e = 0; e < C / 2; ++e) {
                const float4 a = have ? gl[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                gn[2 * e] = make_float2(a.x, a.y);
                gn[2 * e + 1] = make_float2(a.z, a.w);
            }
#pragma unroll
            for (int w = 0; w < C / L; ++w) {
                float2 z[M];
#pragma unroll
                for (int k = 0; k < M; ++k) z[k] = G[w * L + 2 * k + 1];
                dft_reg<M, true>(z);
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const float2 zz = twiddle_small<true>(z[q], q, L);
                    gx[w * L + q] = cadd(gx[w * L + q], zz);
                    gx[w * L + q + M] = csub(gx[w * L + q + M], zz);
                }
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const float2 ge = G[w * L + 2 * k];
                    gn[w * L + k] = cadd(gn[w * L + k], ge);
                    gn[w * L + M + k] = cadd(gn[w * L + M + k], ge);
                }
            }
#pragma unroll
            for (int e = 0; e < C; ++e) G[e] = gn[e];
            LocalAdj<I - 1>::template run<C>(G, gx, gy, ls, lv);
        } else {
            // Level 1: transpose of I (x) H_2.
#pragma unroll
            for (int b = 0; b < C / 2; ++b) {
                const float2 g0 = G[2 * b], g1 = G[2 * b + 1];
                gx[2 * b] = cadd(gx[2 * b], cadd(g0, g1));
                gx[2 * b + 1] = cadd(gx[2 * b + 1], csub(g0, g1));
            }
        }
    }
};

template <int LC, bool REAL>
__device__ __forceinline__ void adj_local(const float2* __restrict__ gy, int64_t ls, typename XType<REAL>::T* gout,
                                          const float2* Gs /* LDS level-LC gradient or null */,
                                          const typename XType<REAL>::T* Xs /* LDS partial gx or null */, int c0,
                                          LevelRange lv) {
    constexpr int C = 1 << LC;
    float2 G[C], gx[C];
    if (Gs) {
#pragma unroll
        for (int e = 0; e < C; ++e) G[e] = Gs[pad(c0 + e)];
    } else {
        const float4* gl = (const float4*)(gy + (int64_t)(LC - 1) * ls);
        const bool have = lv.in(LC);
#pragma unroll
        for (int e = 0; e < C / 2; ++e) {
            const float4 a = have ? gl[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            G[2 * e] = make_float2(a.x, a.y);
            G[2 * e + 1] = make_float2(a.z, a.w);
        }
    }
#pragma unroll
    for (int e = 0; e < C; ++e) {
        if (Xs) gx[e] = to_c(Xs[pad(c0 + e)]);
        else gx[e] = make_float2(0.0f, 0.0f);
    }
    LocalAdj<LC>::template run<C>(G, gx, gy, ls, lv);
    if constexpr (REAL) {
#pragma unroll
        for (int e = 0; e < C / 2; ++e) ((float2*)gout)[e] = make_float2(gx[2 * e].x, gx[2 * e + 1].x);
    } else {
#pragma unroll
        for (int e = 0; e < C / 2; ++e)
            ((float4*)gout)[e] = make_float4(gx[2 * e].x, gx[2 * e].y, gx[2 * e + 1].x, gx[2 * e + 1].y);
    }
}

// First step of the conjugate odd-bin FFT: inputs are the odd bins of G.
template <int R, int JPT>
__device__ __forceinline__ void first_load_adj(const float2* Ps, int i, int nw, float2* v, int tid) {
    constexpr int lgR = Log2<R>::v;
    const int lgM = i - 1, L = 2 << lgM;
    const int lgper = lgM - lgR, per = 1 << lgper;
    const int jobs = nw << lgper;
#pragma unroll
    for (int c = 0; c < JPT; ++c) {
        const int J = tid + c * kTileThreads;
        if (J < jobs) {
            const int w = J >> lgper, j = J & (per - 1);
#pragma unroll
            for (int s = 0; s < R; ++s) v[c * R + s] = Ps[pad(w * L + 2 * (j + s * per) + 1)];
            dft_reg<R, true>(&v[c * R]);
        }
    }
}

template <bool REAL>
__global__ __launch_bounds__(kTileThreads) void tile_adj_kernel(const float2* __restrict__ gY, void* __restrict__ gx,
                                                                const TileJob* __restrict__ jobs,
                                                                const float2* __restrict__ tab, int tmax) {
    using XT = typename XType<REAL>::T;
    const TileLds<XT> L = tile_lds<XT>(tmax);
    XT* Xs = L.X;                                     // gx accumulator (real part only for real x)
    float2* Ps = L.P;                                 // current level gradient G
    float2* Fs = L.F;
    float2* Qs = L.Q;

    const TileJob jb = jobs[blockIdx.x];
    const int t = jb.t;
    const int T = 1 << t;
    const int tid = threadIdx.x;
    const float2* gy = gY + jb.out_off;
    XT* gout = (XT*)gx + jb.in_off;
    const int64_t ls = jb.level_stride;
    const LevelRange lv = LevelRange::unpack(jb.pad);

    if (t > 4) {
        const TwQuarter tw{Qs};
        load_quarter(Qs, tab, tid, kTileThreads);
        const float4* g4 = (const float4*)(gy + (int64_t)(t - 1) * ls);
        const bool have_t = lv.in(t);
        for (int e = tid; e < T / 2; e += kTileThreads) {
            const float4 a = have_t ? g4[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            Ps[pad(2 * e)] = make_float2(a.x, a.y);
            Ps[pad(2 * e + 1)] = make_float2(a.z, a.w);
        }
        for (int e = tid; e < T; e += kTileThreads) {
            if constexpr (REAL) Xs[pad(e)] = 0.0f; else Xs[pad(e)] = make_float2(0.0f, 0.0f);
        }
        __syncthreads();
        for (int i = t; i >= 5; --i) {
            const int lgM = i - 1, M = 1 << lgM, L = 2 * M;
            const int nw = T >> i;
            const int rem = lgM % 3;
            int lgNs;
            // Even-bin gradient of level i, read before G is overwritten.
            float2 ge[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int e = tid + c * kTileThreads;          // e = w*M + k
                if (e < T / 2) {
                    const int w = e >> lgM, k = e & (M - 1);
                    ge[c] = Ps[pad(w * L + 2 * k)];
                }
            }
            if (rem == 1) {
                float2 v[8];
                first_load_adj<2, 4>(Ps, i, nw, v, tid);
                step_store<2, 4, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
                lgNs = 1;
            } else if (rem == 2) {
                float2 v[8];
                first_load_adj<4, 2>(Ps, i, nw, v, tid);
                step_store<4, 2, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
                lgNs = 2;
            } else {
                float2 v[8];
                first_load_adj<8, 1>(Ps, i, nw, v, tid);
                step_store<8, 1, true>(Fs, lgM, 0, M, 1, nw, v, tid, kTileThreads);
                lgNs = 3;
            }
            __syncthreads();
            while (lgNs + 3 < lgM) {
                lds_step<8, 1, true, true>(Fs, lgM, lgNs, M, 1, nw, tw, tid, kTileThreads);
                lgNs += 3;
            }
            float2 z[8];
            step_load<8, 1, true, true>(Fs, lgM, lgNs, M, 1, nw, tw, z, tid, kTileThreads);
            const int lgper = lgM - 3;
            if (tid < (nw << lgper)) {
                const int w = tid >> lgper, j = tid & ((1 << lgper) - 1);
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int q = j + (s << lgper);
                    const float2 zz = cmulc(z[s], tw(i, q));   // conj(D^(i))
                    const int p0 = pad(w * L + q), p1 = pad(w * L + q + M);
                    if constexpr (REAL) {
                        Xs[p0] += zz.x;
                        Xs[p1] -= zz.x;
                    } else {
                        Xs[p0] = cadd(Xs[p0], zz);
                        Xs[p1] = csub(Xs[p1], zz);
                    }
                }
            }
            // Push the even-bin gradient to both children (transpose of U^(i)),
            // adding the level i-1 input gradient.
            const float2* gl = gy + (int64_t)(i - 2) * ls;
            const bool have = lv.in(i - 1);
            const float2 zero = make_float2(0.0f, 0.0f);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int e = tid + c * kTileThreads;
                if (e < T / 2) {
                    const int w = e >> lgM, k = e & (M - 1);
                    const int p0 = w * L + k, p1 = p0 + M;
                    Ps[pad(p0)] = cadd(ge[c], have ? gl[p0] : zero);
                    Ps[pad(p1)] = cadd(ge[c], have ? gl[p1] : zero);
                }
            }
            __syncthreads();
        }
    }
    const int lc = t < 4 ? t : 4;
    if (tid < (T >> lc)) {
        const int c0 = tid << lc;
        const float2* Gs = (t > 4) ? Ps : nullptr;
        const XT* Xp = (t > 4) ? Xs : nullptr;
        switch (lc) {
            case 1: adj_local<1, REAL>(gy + c0, ls, gout + c0, Gs, Xp, c0, lv); break;
            case 2: adj_local<2, REAL>(gy + c0, ls, gout + c0, Gs, Xp, c0, lv); break;
            case 3: adj_local<3, REAL>(gy + c0, ls, gout + c0, Gs, Xp, c0, lv); break;
            default: adj_local<4, REAL>(gy + c0, ls, gout + c0, Gs, Xp, c0, lv); break;
        }
    }
}

// Allow the largest tile's dynamic LDS (above the 64 KB default) once per kernel.
template <typename XT, typename K>
void allow_tile_lds(K kernel) {
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)tile_lds_bytes<XT>(kTileMaxLog));
}
struct TileLdsInit {
    TileLdsInit() {
        allow_tile_lds<float>(tile_fwd_kernel<true, true>);
        allow_tile_lds<float>(tile_fwd_kernel<true, false>);
        allow_tile_lds<float2>(tile_fwd_kernel<false, false>);
        allow_tile_lds<float>(tile_adj_kernel<true>);
        allow_tile_lds<float2>(tile_adj_kernel<false>);
    }
};

hipError_t launch_tile_fwd(bool real_in, const void* x, float2* Y, const TileJob* jobs, int64_t njobs, int tmax,
                           const Twiddles& tw, hipStream_t s, bool half) {
    if (njobs <= 0) return hipSuccess;
    if ((half && !real_in) || tmax < 1 || tmax > kTileMaxLog) return hipErrorInvalidValue;
    static TileLdsInit once;
    dim3 grid((unsigned)njobs), block(kTileThreads);
    const size_t lds = real_in ? tile_lds_bytes<float>(tmax) : tile_lds_bytes<float2>(tmax);
    if (half) hipLaunchKernelGGL((tile_fwd_kernel<true, true>), grid, block, lds, s, x, Y, jobs, tw.tile, tmax);
    else if (real_in) hipLaunchKernelGGL((tile_fwd_kernel<true, false>), grid, block, lds, s, x, Y, jobs, tw.tile, tmax);
    else hipLaunchKernelGGL((tile_fwd_kernel<false, false>), grid, block, lds, s, x, Y, jobs, tw.tile, tmax);
    return hipGetLastError();
}

hipError_t launch_tile_adj(bool real_out, const float2* gY, void* gx, const TileJob* jobs, int64_t njobs, int tmax,
                           const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (tmax < 1 || tmax > kTileMaxLog) return hipErrorInvalidValue;
    static TileLdsInit once;
    dim3 grid((unsigned)njobs), block(kTileThreads);
    const size_t lds = real_out ? tile_lds_bytes<float>(tmax) : tile_lds_bytes<float2>(tmax);
    if (real_out) hipLaunchKernelGGL(tile_adj_kernel<true>, grid, block, lds, s, gY, gx, jobs, tw.tile, tmax);
    else hipLaunchKernelGGL(tile_adj_kernel<false>, grid, block, lds, s, gY, gx, jobs, tw.tile, tmax);
    return hipGetLastError();
}

}  // namespace mrdft
