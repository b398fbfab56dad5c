// In-wave FFTs of 256 points (4 per lane) with butterflies across lanes.
//
// Shared by the forward tiles and the adjoint tile: at each level of the
// recurrence (Section 3, eq. (4)) the odd bins of every window are the DFT of
// a twiddled window difference (eq. (3), D^(i), F^(i)); the adjoint takes the
// conjugate DFT of the odd-bin gradient (conjugating input and output).  For
// windows that fit in one wave the
// wave's 256 FFT points (256 / 2^n windows of 2^n points, 3 <= n <= 8) are
// transformed in registers:
//
// * lane l, register r holds the point whose 8-bit wave index has the two
//   top FFT-index bits in r and the other six bits ("content" bits c0..c5:
//   low FFT-index bits first, then window bits) in the lane, with
//   c0 = l0^l2, c1 = l1^l2, c2 = l2^l3, c3 = l3, c4 = l4, c5 = l5;
// * a radix-4 decimation-in-frequency stage runs over the registers;
// * the DPP lane permutations inside a row of 16 lanes (swap neighbours,
//   swap pairs, mirror 8, mirror 16) each flip exactly one content bit
//   (c0, c1, c2, c3), so each gives one radix-2 stage across lanes;
// * content bits 4 and 5 are exchanged with the register bits by permlane
//   swaps (lane halves, rows of 16) and transformed in registers.
//
// The bins come out in a known scattered order (xl_pos); one pass through
// LDS (xl_fsw layout) puts them in natural order.
#pragma once
#include "mrdft_device.h"

namespace mrdft {

struct XLane {
    int c;                 // content bits of this lane
    float s[4];            // +1 / -1: content bit b clear / set
    float2 tw[4];          // stage b >= 1: 1, or -w_{2^(b+1)}^{c mod 2^b} where bit b is set
};

__device__ __forceinline__ int xl_content(int lane) {
    const int l2 = (lane >> 2) & 1, l3 = (lane >> 3) & 1;
    return (lane & 0x30) | (l3 << 3) | ((l2 ^ l3) << 2) | ((((lane >> 1) & 1) ^ l2) << 1) | ((lane & 1) ^ l2);
}

// TW(lg, e) = w_{2^lg}^e (lg <= 4 here).
template <class TW>
__device__ __forceinline__ XLane xl_lane(int lane, const TW& tw) {
    XLane ln;
    ln.c = xl_content(lane);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const bool hi = (ln.c >> b) & 1;
        ln.s[b] = hi ? -1.0f : 1.0f;
        if (b > 0) {
            const float2 t = tw(b + 1, ln.c & ((1 << b) - 1));
            ln.tw[b] = hi ? make_float2(-t.x, -t.y) : make_float2(1.0f, 0.0f);
        }
    }
    return ln;
}

// Value of lane l ^ 1, l ^ 2, l ^ 7 (within 8) or l ^ 15 (within 16): the
// lane whose content differs in bit B only.
template <int B>
__device__ __forceinline__ float xl_dpp(float x) {
    constexpr int ctrl = B == 0 ? 0xB1 : B == 1 ? 0x4E : B == 2 ? 0x141 : 0x140;
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), ctrl, 0xF, 0xF, false));
}

// Radix-2 decimation-in-frequency stage over content bit B: the lane with
// the bit clear ends with a + b, the other with (a - b) w (B > 0) or a - b
// (B = 0), computed as (partner * s + self) * tw with s = -1 and the sign of
// tw flipped on the second lane.
template <int B>
__device__ __forceinline__ float2 xl_bfly(float2 v, const XLane& ln) {
    const float px = xl_dpp<B>(v.x), py = xl_dpp<B>(v.y);
    const float2 t = make_float2(__builtin_fmaf(px, ln.s[B], v.x), __builtin_fmaf(py, ln.s[B], v.y));
    if constexpr (B == 0) return make_float2(t.x * ln.s[0], t.y * ln.s[0]);
    else return cmul(t, ln.tw[B]);
}

template <int B>
struct XStages {
    static __device__ __forceinline__ void run(float2* a, const XLane& ln) {
        if constexpr (B >= 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = xl_bfly<B>(a[r], ln);
            XStages<B - 1>::run(a, ln);
        }
    }
};

// Sum of v over the 64 lanes of a wave, every lane receiving it, in FP64:
// the four DPP permutations pair lanes that differ in one of bits 0..3 of
// the lane index (within a row of 16 any pairing across the bit will do,
// all lanes of a group hold the same partial sum by then), the permlane
// swaps pair rows and wave halves.  Each 64-bit value moves as two 32-bit
// halves; nothing goes through LDS.
template <int B>
__device__ __forceinline__ double xl_dpp64(double v) {
    constexpr int ctrl = B == 0 ? 0xB1 : B == 1 ? 0x4E : B == 2 ? 0x141 : 0x140;
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, ctrl, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), ctrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double xl_wave_sum(double v) {
    v += xl_dpp64<0>(v);
    v += xl_dpp64<1>(v);
    v += xl_dpp64<2>(v);
    v += xl_dpp64<3>(v);
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
    // rows of 16: a = [r0, r0, r2, r2], b = [r1, r1, r3, r3] per 32-bit half
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    v = __builtin_bit_cast(double, ((unsigned long long)(unsigned)rh[0] << 32) | (unsigned)rl[0]) +
        __builtin_bit_cast(double, ((unsigned long long)(unsigned)rh[1] << 32) | (unsigned)rl[1]);
    // wave halves
    const unsigned long long w = __builtin_bit_cast(unsigned long long, v);
    const unsigned wl = (unsigned)w, wh = (unsigned)(w >> 32);
    const auto hl = __builtin_amdgcn_permlane32_swap(wl, wl, false, false);
    const auto hh = __builtin_amdgcn_permlane32_swap(wh, wh, false, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hh[0] << 32) | (unsigned)hl[0]) +
           __builtin_bit_cast(double, ((unsigned long long)(unsigned)hh[1] << 32) | (unsigned)hl[1]);
}

// Exchange register bit 1 with lane bit 5 and register bit 0 with lane bit 4.
__device__ __forceinline__ void xl_swap(float& a, float& b, bool rows) {
    const unsigned ua = __builtin_bit_cast(unsigned, a), ub = __builtin_bit_cast(unsigned, b);
    if (rows) {
        const auto r = __builtin_amdgcn_permlane16_swap(ua, ub, false, false);   // odd rows of a <-> even rows of b
        a = __builtin_bit_cast(float, (unsigned)r[0]);
        b = __builtin_bit_cast(float, (unsigned)r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(ua, ub, false, false);   // upper half of a <-> lower half of b
        a = __builtin_bit_cast(float, (unsigned)r[0]);
        b = __builtin_bit_cast(float, (unsigned)r[1]);
    }
}
__device__ __forceinline__ void xl_transpose45(float2* a) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {             // register pairs (0, 2), (1, 3): bit 1 <-> lane bit 5
        xl_swap(a[r].x, a[r + 2].x, false);
        xl_swap(a[r].y, a[r + 2].y, false);
    }
#pragma unroll
    for (int r = 0; r < 4; r += 2) {          // register pairs (0, 1), (2, 3): bit 0 <-> lane bit 4
        xl_swap(a[r].x, a[r + 1].x, true);
        xl_swap(a[r].y, a[r + 1].y, true);
    }
}

// The wave's FFTs of 2^N points: a[r] holds the point of FFT index
// plow + 2^(N-2) r of window wl (plow and wl from the lane's content bits).
// TW(lg, e) = w_{2^lg}^e for lg <= N.  On return a[r] holds the bin given by
// xl_pos<N>(ln.c, r).
template <int N, class TW>
__device__ __forceinline__ void xl_fft(float2* a, const XLane& ln, const TW& tw) {
    constexpr int NQ = N - 2;                           // FFT-index bits held by the lane
    constexpr int NB = NQ < 4 ? NQ : 4;                 // DPP stages (content bits 0..NB-1)
    const int plow = ln.c & ((1 << (NQ < 6 ? NQ : 6)) - 1);
    // radix 4 over the top two index bits, twiddles w_{2^N}^(plow f)
    dft_reg<4, false>(a);
#pragma unroll
    for (int f = 1; f < 4; ++f) a[f] = cmul(a[f], tw(N, plow * f));
    if constexpr (N == 8) {
        // index bits 5, 4 into the registers, radix 4 over them (64-point sub-FFTs)
        xl_transpose45(a);
        dft_reg<4, false>(a);
#pragma unroll
        for (int f = 1; f < 4; ++f) a[f] = cmul(a[f], tw(6, (ln.c & 15) * f));
    } else if constexpr (N == 7) {
        // register bit 1 <- window bit, register bit 0 <- index bit 4: radix 2
        xl_transpose45(a);
        const float2 t = tw(5, ln.c & 15);
#pragma unroll
        for (int h = 0; h < 4; h += 2) {
            const float2 p0 = a[h], p1 = a[h + 1];
            a[h] = cadd(p0, p1);
            a[h + 1] = cmul(csub(p0, p1), t);
        }
    }
    // radix-2 stages across lanes: content bit b gives bin bit N-1-b
    XStages<NB - 1>::run(a, ln);
}

// Wave-local position window * 2^N + bin of a[r] after xl_fft<N>.
template <int N>
__device__ __forceinline__ int xl_pos(int c, int r) {
    constexpr int NQ = N - 2;
    constexpr int NB = NQ < 4 ? NQ : 4;
    int p = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) p |= ((c >> b) & 1) << (N - 1 - b);
    if constexpr (N == 8) p |= ((c >> 4) & 3) | (r & 1) << 2 | (r >> 1) << 3;    // first digit went to lanes 4, 5
    else if constexpr (N == 7) p |= ((c >> 4) & 3) | (r & 1) << 2 | (r >> 1) << 7;
    else p |= r | (c >> NQ) << N;                                                   // window bits above
    return p;
}

// Index of wave-local point p in the natural-order scratch: bits 4..7
// folded into bits 0..3, so that the lane-scattered writes and the
// natural-order reads both fall on distinct banks.
__device__ __forceinline__ int xl_fsw(int p) { return p ^ ((p >> 4) & 15); }

}  // namespace mrdft
