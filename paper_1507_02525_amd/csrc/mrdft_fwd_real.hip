// Forward MrDFT of real signals in one launch: every workgroup takes one job
// from a table, either a 4096-sample tile (levels 1..12 on chip, see
// mrdft_tile_real.h) or one piece of a window of a level 13..16 (column-first
// 256-point rows, see mrdft_rows_real.h).  Both kinds use 256 threads and at
// most 40 KB of LDS, so four workgroups of either kind share a CU and the
// store streams of the levels overlap instead of running one after another.
// The level spectra are stored with the non-temporal hint, so that the
// pieces' re-reads of their windows' samples stay in L2 (64 x 2^16 samples:
// 118 -> 115 us; the loss's scaled launch reads x and z and gains more).
#include "mrdft_internal.h"
#include "mrdft_rows_real.h"
#include "mrdft_tile_real.h"

namespace mrdft {

namespace {

union FwdRealLds {
    RealTileLds tile;
    RowsLds rows;
};
static_assert(sizeof(FwdRealLds) <= 40 * 1024, "four workgroups per CU");
static_assert(kRThreads == kRowsThreads, "one block size for both job kinds");

constexpr int kModeStore = 0, kModeNorms = 1, kModeScaled = 2, kModeHalf = 3, kModeScaledHalf = 4;

// MODE kModeStore: the level spectra are stored to Y (kModeHalf: as packed
// half spectra, the job offsets and level stride in half-spectrum units).  kModeScaled
// (spectral-loss gradient): the input is x - xsub and level i of signal b is
// stored times alpha[b * m + i - 1].  kModeNorms (spectral loss): the input is
// x - xsub (xsub may be null) and only the squared magnitudes of every level
// are summed, into sums[b * m + level - 1]; Y is not touched.  The last two
// need a uniform batch (signal b = in_off / N).
// At least 4 waves per SIMD: 4 workgroups per CU (128 VGPRs).
template <int MODE>
__global__ __launch_bounds__(kRThreads, 4) void fwd_real_kernel(const float* __restrict__ x, float2* __restrict__ Y,
                                                                const RealJob* __restrict__ jobs,
                                                                const float2* __restrict__ t4096,
                                                                const float2* __restrict__ rowtw,
                                                                const float4* __restrict__ comb,
                                                                const float* __restrict__ xsub,
                                                                double* __restrict__ sums,
                                                                const float* __restrict__ alpha, int m) {
    constexpr bool RED = MODE == kModeNorms;
    __shared__ FwdRealLds S;
    const RealJob jb = jobs[blockIdx.x];
    // Tile waves issue ahead of piece waves on a SIMD: the tiles carry most of
    // the launch's stores, and keeping that stream steady while the pieces'
    // arithmetic takes the remaining issue slots shortens the mixed launch.
    // The norm mode stores nothing and keeps one priority.
    if (MODE != kModeNorms && jb.lg == 0) __builtin_amdgcn_s_setprio(1);
    const int tid = threadIdx.x;
    const float* xj = x + jb.in_off;
    const float* zj = (MODE != kModeStore && xsub) ? xsub + jb.in_off : nullptr;
    float2* yj = RED ? nullptr : Y + jb.out_off;
    if constexpr (MODE == kModeStore || MODE == kModeHalf) {
        constexpr bool H = MODE == kModeHalf;
        StoreOutT<H> out{LevelRange::unpack(jb.g)};   // tile jobs carry the plan's level range
        switch (jb.lg) {
            case 0: real_tile_body(S.tile, xj, nullptr, yj, jb.level_stride, t4096, tid, out); break;
            case 13: rows_real_body<5, false, H>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                                 comb + rows_combine_offset(13), tid); break;
            case 14: rows_real_body<6, false, H>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                                 comb + rows_combine_offset(14), tid); break;
            case 15: rows_real_body<7, false, H>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                                 comb + rows_combine_offset(15), tid); break;
            case 16: rows_real_body<8, false, H>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                                 comb + rows_combine_offset(16), tid); break;
            default: break;
        }
    } else if constexpr (MODE == kModeScaled || MODE == kModeScaledHalf) {
        // kModeScaledHalf: packed half spectra from a full-spectrum job table
        // (every output offset and the tiles' level stride halved)
        constexpr bool H = MODE == kModeScaledHalf;
        const ScaledOutT<H> out{alpha + (jb.in_off / jb.level_stride) * m};
        const float sc = jb.lg > 0 ? out.alpha[jb.lg - 1] : 1.0f;
        float2* const yo = H ? Y + (jb.out_off >> 1) : yj;
        switch (jb.lg) {
            case 0: real_tile_body(S.tile, xj, zj, yo, jb.level_stride >> (H ? 1 : 0), t4096, tid, out); break;
            case 13: rows_real_body<5, false, H>(S.rows, xj, yo, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                                 comb + rows_combine_offset(13), tid, zj, nullptr, sc); break;
            case 14: rows_real_body<6, false, H>(S.rows, xj, yo, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                                 comb + rows_combine_offset(14), tid, zj, nullptr, sc); break;
            case 15: rows_real_body<7, false, H>(S.rows, xj, yo, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                                 comb + rows_combine_offset(15), tid, zj, nullptr, sc); break;
            case 16: rows_real_body<8, false, H>(S.rows, xj, yo, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                                 comb + rows_combine_offset(16), tid, zj, nullptr, sc); break;
            default: break;
        }
    } else {
        const int64_t b = jb.in_off / jb.level_stride;
        double* sb = sums + b * m;
        const int lane = tid & 63;
        if (jb.lg == 0) {
            NormOut out{sb};                          // flushes each level's sums as it completes
            real_tile_body(S.tile, xj, zj, nullptr, jb.level_stride, t4096, tid, out);
        } else {
            double acc = 0.0;
            switch (jb.lg) {
                case 13: rows_real_body<5, true>(S.rows, xj, nullptr, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                                 comb + rows_combine_offset(13), tid, zj, &acc); break;
                case 14: rows_real_body<6, true>(S.rows, xj, nullptr, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                                 comb + rows_combine_offset(14), tid, zj, &acc); break;
                case 15: rows_real_body<7, true>(S.rows, xj, nullptr, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                                 comb + rows_combine_offset(15), tid, zj, &acc); break;
                case 16: rows_real_body<8, true>(S.rows, xj, nullptr, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                                 comb + rows_combine_offset(16), tid, zj, &acc); break;
                default: break;
            }
            const double t = xl_wave_sum(acc);
            if (lane == 0) atomicAdd(sb + jb.lg - 1, t);
        }
    }
}

}  // namespace

hipError_t launch_fwd_real(const float* x, float2* Y, const RealJob* jobs, int64_t njobs, const Twiddles& tw,
                           hipStream_t s, bool half) {
    if (njobs <= 0) return hipSuccess;
    if (half)
        hipLaunchKernelGGL(fwd_real_kernel<kModeHalf>, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, Y, jobs,
                           tw.tile, tw.rows, tw.rows_comb, nullptr, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL(fwd_real_kernel<kModeStore>, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, Y, jobs,
                           tw.tile, tw.rows, tw.rows_comb, nullptr, nullptr, nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_fwd_real_scaled(const float* x, const float* xsub, const float* alpha, int m, float2* Y,
                                  const RealJob* jobs, int64_t njobs, const Twiddles& tw, hipStream_t s, bool half) {
    if (njobs <= 0) return hipSuccess;
    if (half)
        hipLaunchKernelGGL(fwd_real_kernel<kModeScaledHalf>, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, Y, jobs,
                           tw.tile, tw.rows, tw.rows_comb, xsub, nullptr, alpha, m);
    else
        hipLaunchKernelGGL(fwd_real_kernel<kModeScaled>, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, Y, jobs,
                           tw.tile, tw.rows, tw.rows_comb, xsub, nullptr, alpha, m);
    return hipGetLastError();
}

hipError_t launch_fwd_real_norms(const float* x, const float* xsub, double* sums, int m, const RealJob* jobs,
                                 int64_t njobs, const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(fwd_real_kernel<kModeNorms>, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, nullptr, jobs,
                       tw.tile, tw.rows, tw.rows_comb, xsub, sums, nullptr, m);
    return hipGetLastError();
}

}  // namespace mrdft
