// Forward MrDFT of complex signals in one persistent launch: each workgroup
// repeatedly takes the next job of a table, either a 2048-sample tile (levels
// 1..11 on chip, mrdft_tile_c64.h) or one 16-row piece of a window of a level
// 12..16 (mrdft_rows_c64.h).  Signals of any order share the launch; their
// offsets are int64.
#include "mrdft_internal.h"
#include "mrdft_rows_c64.h"
#include "mrdft_tile_c64.h"

namespace mrdft {

namespace {

union FwdC64Lds {
    CTileLds tile;
    CRowsLds rows;
};
static_assert(sizeof(FwdC64Lds) <= 40 * 1024, "four workgroups per CU");
static_assert(kCThreads == kRowsThreads, "one block size for both job kinds");

__global__ __launch_bounds__(kCThreads, 4) void fwd_c64_kernel(const float2* __restrict__ x, float2* __restrict__ Y,
                                                               const RealJob* __restrict__ jobs, int64_t njobs,
                                                               unsigned* queue, const float2* __restrict__ t4096,
                                                               const float2* __restrict__ rowtw,
                                                               const float2* __restrict__ comb) {
    __shared__ FwdC64Lds S;
    __shared__ unsigned s_job;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_job = atomicAdd(&queue[0], 1u);
        __syncthreads();
        const int64_t j = s_job;
        if (j >= njobs) break;                        // every workgroup reaches this exit
        const RealJob jb = jobs[j];
        const float2* xj = x + jb.in_off;
        float2* yj = Y + jb.out_off;
        // A fresh copy of the thread index each iteration: nothing derived from
        // it is hoisted out of the loop (six inlined job bodies would otherwise
        // keep their lane addresses live across it and spill).
        int t;
        asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(tid));
        switch (jb.lg) {
            case 0: c64_tile_body(S.tile, xj, yj, jb.level_stride, t4096, t); break;
            case 12: rows_c64_body<4>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(12),
                                      comb + crows_combine_offset(12), t); break;
            case 13: rows_c64_body<5>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                      comb + crows_combine_offset(13), t); break;
            case 14: rows_c64_body<6>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                      comb + crows_combine_offset(14), t); break;
            case 15: rows_c64_body<7>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                      comb + crows_combine_offset(15), t); break;
            case 16: rows_c64_body<8>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                      comb + crows_combine_offset(16), t); break;
            default: break;
        }
        __syncthreads();                              // LDS and s_job reuse
    }
    // The last workgroup to leave clears the queue for the next launch: all
    // others have made their final fetch before they counted themselves out.
    if (tid == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

}  // namespace

hipError_t launch_fwd_c64(const float2* x, float2* Y, const RealJob* jobs, int64_t njobs, unsigned* queue, int grid,
                          const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fwd_c64_kernel, dim3((unsigned)grid), dim3(kCThreads), 0, s, x, Y, jobs, njobs, queue, tw.tile,
                       tw.rows, tw.crows_comb);
    return hipGetLastError();
}

}  // namespace mrdft
