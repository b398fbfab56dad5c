// Adjoint MrDFT (gx = sum_i A_i^H gY^(i)) in two launches.
//   (a) one workgroup per job: 2048-sample tiles (levels 11..1 by the
//       transposed recurrence, mrdft_adj_tile.h; gx of the tile is written)
//       and rows pieces of the levels 12..16 (scratch B, mrdft_adj_rows.h;
//       for real output the levels 13..16 form only the Hermitian half of B);
//   (b) one workgroup per (region, 16 columns): the column DFTs of the levels
//       12..16, summed and added to gx.
// Real plans accumulate Re(gx) only.
#include "mrdft_adj_rows.h"
#include "mrdft_adj_tile.h"
#include "mrdft_internal.h"

namespace mrdft {

namespace {

template <bool REAL>
union AdjALds {
    AdjTileLds<REAL> tile;
    CRowsLds rows;
    RowsLds hrows;                                    // Hermitian rows pieces (real output)
};
static_assert(sizeof(AdjALds<true>) <= 40 * 1024 && sizeof(AdjALds<false>) <= 40 * 1024, "four workgroups per CU");

// HALF (real output): gY holds the packed half spectra of a half-spectrum plan.
template <bool REAL, bool HALF>
__global__ __launch_bounds__(kCThreads, 4) void adj_a_kernel(const float2* __restrict__ gY, void* __restrict__ gx,
                                                             float2* __restrict__ scratch,
                                                             const RealJob* __restrict__ jobs,
                                                             const float2* __restrict__ t4096,
                                                             const float2* __restrict__ rowtw, int gshift,
                                                             float hsc) {
    __shared__ AdjALds<REAL> S;
    const RealJob jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const float2* gyj = gY + (jb.in_off >> gshift);
    switch (jb.lg) {
        case 0: {
            void* gxj = REAL ? (void*)((float*)gx + jb.out_off) : (void*)((float2*)gx + jb.out_off);
            adj_tile_body<REAL, HALF>(S.tile, gyj, gxj, jb.level_stride >> gshift, t4096, tid, LevelRange::unpack(jb.g),
                                      hsc);
            break;
        }
        case 12:
            adj_rows_body<4, HALF>(S.rows, gyj, scratch + jb.out_off, jb.g, t4096, rowtw + rows_twiddle_offset(12), tid,
                                   hsc);
            break;
        // real output: Hermitian pieces of 17 rows (half the rows of B)
#define MRDFT_ADJ_ROWS(LG, RL)                                                                                   \
    case LG:                                                                                                    \
        if constexpr (REAL)                                                                                     \
            adj_rows_real_body<RL, HALF>(S.hrows, gyj, scratch + jb.out_off, jb.g, t4096,                      \
                                         rowtw + rows_twiddle_offset(LG), tid, hsc);                            \
        else                                                                                                    \
            adj_rows_body<RL>(S.rows, gyj, scratch + jb.out_off, jb.g, t4096, rowtw + rows_twiddle_offset(LG), tid); \
        break;
        MRDFT_ADJ_ROWS(13, 5)
        MRDFT_ADJ_ROWS(14, 6)
        MRDFT_ADJ_ROWS(15, 7)
        MRDFT_ADJ_ROWS(16, 8)
#undef MRDFT_ADJ_ROWS
        default: break;
    }
}

template <bool REAL>
__global__ __launch_bounds__(kRowsThreads, 4) void adj_b_kernel(void* __restrict__ gx, const float2* __restrict__ scratch,
                                                               const AdjColJob* __restrict__ jobs,
                                                               const float2* __restrict__ t4096) {
    __shared__ AdjColsLds S;
    const AdjColJob jb = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    S.T[tid] = t4096[tid << (kTileMaxLog - kRowsLog)];
    typedef typename std::conditional<REAL, float, float2>::type Acc;
    Acc acc[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        if constexpr (REAL) acc[s] = 0.0f;
        else acc[s] = make_float2(0.0f, 0.0f);
    }
    const int c0 = 16 * (jb.c & 15);
    const LevelRange lv = LevelRange::unpack(jb.c >> 8);
    int top = jb.region_log < kRowsMaxLevel ? jb.region_log : kRowsMaxLevel;
    if (top > lv.hi) top = lv.hi;
    const int first = lv.lo > kCRowsMinLevel ? lv.lo : kCRowsMinLevel;
    for (int lg = first; lg <= top; ++lg) {
        const float2* scr = scratch + jb.scr_off + (int64_t)(lg - kCRowsMinLevel) * jb.level_stride;
        // a fresh copy of the thread index per level: nothing derived from it is
        // hoisted out of this loop (five inlined bodies would spill)
        int t;
        asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(tid));
        switch (lg) {
            case 12: adj_cols_level<4, REAL>(S, scr, jb.region_log, c0, acc, t); break;
            case 13: adj_cols_level<5, REAL>(S, scr, jb.region_log, c0, acc, t); break;
            case 14: adj_cols_level<6, REAL>(S, scr, jb.region_log, c0, acc, t); break;
            case 15: adj_cols_level<7, REAL>(S, scr, jb.region_log, c0, acc, t); break;
            default: adj_cols_level<8, REAL>(S, scr, jb.region_log, c0, acc, t); break;
        }
    }
    // gx[region + c0 + col + 256 rho] += acc
    const int col = tid & 15;
    const int rows = 1 << (jb.region_log - kRowsLog);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int rho = (tid >> 4) + 16 * s;
        if (rho < rows) {
            const int64_t i = jb.gx_off + c0 + col + (int64_t)kRowsN * rho;
            if constexpr (REAL) ((float*)gx)[i] += acc[s];
            else ((float2*)gx)[i] = cadd(((float2*)gx)[i], acc[s]);
        }
    }
}

__global__ __launch_bounds__(256) void zero_kernel(float* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0f;
}

}  // namespace

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / (int64_t)sizeof(float);
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (float*)p, n);
    return hipGetLastError();
}

hipError_t launch_adj_a(bool real_out, bool half, int gshift, float hsc, const float2* gY, void* gx, float2* scratch,
                        const RealJob* jobs, int64_t njobs, const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if ((half && !real_out) || gshift < 0 || gshift > 1) return hipErrorInvalidValue;
    if (half)
        hipLaunchKernelGGL((adj_a_kernel<true, true>), dim3((unsigned)njobs), dim3(kCThreads), 0, s, gY, gx, scratch,
                           jobs, tw.tile, tw.rows, gshift, hsc);
    else if (real_out)
        hipLaunchKernelGGL((adj_a_kernel<true, false>), dim3((unsigned)njobs), dim3(kCThreads), 0, s, gY, gx, scratch,
                           jobs, tw.tile, tw.rows, gshift, hsc);
    else
        hipLaunchKernelGGL((adj_a_kernel<false, false>), dim3((unsigned)njobs), dim3(kCThreads), 0, s, gY, gx, scratch,
                           jobs, tw.tile, tw.rows, gshift, hsc);
    return hipGetLastError();
}

hipError_t launch_adj_b(bool real_out, void* gx, const float2* scratch, const AdjColJob* jobs, int64_t njobs,
                        const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (real_out)
        hipLaunchKernelGGL(adj_b_kernel<true>, dim3((unsigned)njobs), dim3(kRowsThreads), 0, s, gx, scratch, jobs, tw.tile);
    else
        hipLaunchKernelGGL(adj_b_kernel<false>, dim3((unsigned)njobs), dim3(kRowsThreads), 0, s, gx, scratch, jobs,
                           tw.tile);
    return hipGetLastError();
}

}  // namespace mrdft
