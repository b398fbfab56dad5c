// Forward MrDFT of real signals in one launch: every workgroup takes one job
// from a table, either a 4096-sample tile (levels 1..12 on chip, see
// mrdft_tile_real.h) or one piece of a window of a level 13..16 (column-first
// 256-point rows, see mrdft_rows_real.h).  Both kinds use 256 threads and at
// most 40 KB of LDS, so four workgroups of either kind share a CU and the
// store streams of the levels overlap instead of running one after another.
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

// at least 4 waves per SIMD: 4 workgroups per CU (128 VGPRs)
__global__ __launch_bounds__(kRThreads, 4) void fwd_real_kernel(const float* __restrict__ x, float2* __restrict__ Y,
                                                             const RealJob* __restrict__ jobs,
                                                             const float2* __restrict__ t4096,
                                                             const float2* __restrict__ rowtw,
                                                             const float4* __restrict__ comb) {
    __shared__ FwdRealLds S;
    const RealJob jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const float* xj = x + jb.in_off;
    float2* yj = Y + jb.out_off;
    switch (jb.lg) {
        case 0: real_tile_body(S.tile, xj, yj, jb.level_stride, t4096, tid); break;
        case 13: rows_real_body<5>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                         comb + rows_combine_offset(13), tid); break;
        case 14: rows_real_body<6>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                         comb + rows_combine_offset(14), tid); break;
        case 15: rows_real_body<7>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                         comb + rows_combine_offset(15), tid); break;
        case 16: rows_real_body<8>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                         comb + rows_combine_offset(16), tid); break;
        default: break;
    }
}

}  // namespace

hipError_t launch_fwd_real(const float* x, float2* Y, const RealJob* jobs, int64_t njobs, const Twiddles& tw,
                           hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(fwd_real_kernel, dim3((unsigned)njobs), dim3(kRThreads), 0, s, x, Y, jobs, tw.tile, tw.rows,
                       tw.rows_comb);
    return hipGetLastError();
}

}  // namespace mrdft
