// Forward MrDFT of complex signals in one launch, each job either a
// 2048-sample tile (levels 1..11 on chip, mrdft_tile_c64.h) or one 16-row
// piece of a window of a level 12..16 (mrdft_rows_c64.h).  Signals of any
// order share the launch; their offsets are int64.
//
// Persistent form: each workgroup repeatedly takes the next job of a table
// that holds one segment per XCD, with all pieces of a window in one
// segment.  A workgroup takes jobs from the segment of the XCD it runs on
// (read from the hardware register), so the pieces of a window share their x
// columns through that XCD's L2; when its segment is empty it takes jobs from
// the other segments.  Direct form: one workgroup per job.
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

constexpr int kXcds = 8;

// A tile of several consecutive signals of 2^m samples (m < 11): job lg =
// kMultiTileLg + m, level_stride = 2^m | (valid samples << 32).
template <bool REALIN = false>
__device__ __forceinline__ void multi_tile(CTileLds& S, const void* x, float2* y, const RealJob& jb,
                                           const float2* t4096, int tid) {
    const int m = jb.lg - kMultiTileLg;
    const int64_t N = jb.level_stride & 0xffffffffLL;
    const LevelRange lv = LevelRange::unpack(jb.g);
    const SubMap sm{m, (int)(jb.level_stride >> 32), (int64_t)(lv.hi - lv.lo + 1) * N};
    c64_tile_body<true, REALIN>(S, x, y, N, t4096, tid, lv, sm);
}

__device__ __forceinline__ unsigned xcc_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & (kXcds - 1);
}

// queue[q] (q < 8): next job of segment q; queue[8]: workgroups done.
__global__ __launch_bounds__(kCThreads, 4) void fwd_c64_kernel(const float2* __restrict__ x, float2* __restrict__ Y,
                                                               const RealJob* __restrict__ jobs,
                                                               const unsigned* __restrict__ seg, unsigned* queue,
                                                               const float2* __restrict__ t4096,
                                                               const float2* __restrict__ rowtw,
                                                               const float2* __restrict__ comb) {
    __shared__ FwdC64Lds S;
    __shared__ int s_job;
    const int tid = threadIdx.x;
    const unsigned home = xcc_id();
    for (;;) {
        if (tid == 0) {
            int found = -1;
            for (int k = 0; k < kXcds && found < 0; ++k) {
                const unsigned q = (home + k) & (kXcds - 1);
                const unsigned len = seg[q + 1] - seg[q];
                if (__hip_atomic_load(&queue[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) continue;
                const unsigned i = atomicAdd(&queue[q], 1u);
                if (i < len) found = (int)(seg[q] + i);
            }
            s_job = found;
        }
        __syncthreads();
        const int j = s_job;
        if (j < 0) break;                             // every segment is exhausted: every workgroup exits
        const RealJob jb = jobs[j];
        const float2* xj = x + jb.in_off;
        float2* yj = Y + jb.out_off;
        // A fresh copy of the thread index each iteration: nothing derived from
        // it is hoisted out of the loop (six inlined job bodies would otherwise
        // keep their lane addresses live across it and spill).
        int t;
        asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(tid));
        switch (jb.lg) {
            case 0: c64_tile_body(S.tile, xj, yj, jb.level_stride, t4096, t, LevelRange::unpack(jb.g)); break;
            case 12: rows_c64_body<4>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(12),
                                      comb + crows_combine_offset(12), t); break;
            case 13: rows_c64_body2<5>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                       comb + crows_combine_offset(13), t); break;
            case 14: rows_c64_body2<6>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                       comb + crows_combine_offset(14), t); break;
            case 15: rows_c64_body2<7>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                       comb + crows_combine_offset(15), t); break;
            case 16: rows_c64_body2<8>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                       comb + crows_combine_offset(16), t); break;
            default:
                if (jb.lg >= kMultiTileLg) multi_tile(S.tile, xj, yj, jb, t4096, t);
                break;
        }
        __syncthreads();                              // LDS and s_job reuse
    }
    // The last workgroup to leave clears the queue for the next launch: all
    // others have made their final fetch before they counted themselves out.
    if (tid == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&queue[kXcds], 1u);
        if (done == gridDim.x - 1) {
            for (int q = 0; q <= kXcds; ++q) atomicExch(&queue[q], 0u);
        }
    }
}

// One workgroup per job (the table dealt so that block b, which runs on XCD
// b mod 8, holds a job of that XCD's bucket).  In the persistent form the
// loads of a workgroup's next job queue behind the stores of its previous one
// (one in-order vector memory counter); here every job starts fresh.
// REALIN: real float32 signals below 4096 samples of a real plan (tiles and
// multi-signal tiles only; the full complex spectra are written).
template <bool REALIN>
__global__ __launch_bounds__(kCThreads, 4) void fwd_c64_direct(const void* __restrict__ x, float2* __restrict__ Y,
                                                               const RealJob* __restrict__ jobs,
                                                               const float2* __restrict__ t4096,
                                                               const float2* __restrict__ rowtw,
                                                               const float2* __restrict__ comb) {
    __shared__ FwdC64Lds S;
    const int tid = threadIdx.x;
    const RealJob jb = jobs[blockIdx.x];
    // tile waves (single- and multi-signal) issue ahead of piece waves: they
    // carry most of the stores (as in the real one-launch forward)
    if (jb.lg == 0 || jb.lg >= kMultiTileLg) __builtin_amdgcn_s_setprio(1);
    float2* yj = Y + jb.out_off;
    if constexpr (REALIN) {
        const float* xj = (const float*)x + jb.in_off;
        if (jb.lg == 0) c64_tile_body<false, true>(S.tile, xj, yj, jb.level_stride, t4096, tid, LevelRange::unpack(jb.g));
        else if (jb.lg >= kMultiTileLg) multi_tile<true>(S.tile, xj, yj, jb, t4096, tid);
        return;
    }
    const float2* xj = (const float2*)x + jb.in_off;
    switch (jb.lg) {
        case 0: c64_tile_body(S.tile, xj, yj, jb.level_stride, t4096, tid, LevelRange::unpack(jb.g)); break;
        case 12: rows_c64_body<4>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(12),
                                  comb + crows_combine_offset(12), tid); break;
        case 13: rows_c64_body2<5>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(13),
                                   comb + crows_combine_offset(13), tid); break;
        case 14: rows_c64_body2<6>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(14),
                                   comb + crows_combine_offset(14), tid); break;
        case 15: rows_c64_body2<7>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(15),
                                   comb + crows_combine_offset(15), tid); break;
        case 16: rows_c64_body2<8>(S.rows, xj, yj, jb.g, t4096, rowtw + rows_twiddle_offset(16),
                                   comb + crows_combine_offset(16), tid); break;
        default:
            if (jb.lg >= kMultiTileLg) multi_tile(S.tile, xj, yj, jb, t4096, tid);
            break;
    }
}

}  // namespace

hipError_t launch_fwd_c64_direct(const void* x, float2* Y, const RealJob* jobs, int64_t njobs, const Twiddles& tw,
                                 hipStream_t s, bool real_in) {
    if (njobs <= 0) return hipSuccess;
    if (real_in)
        hipLaunchKernelGGL(fwd_c64_direct<true>, dim3((unsigned)njobs), dim3(kCThreads), 0, s, x, Y, jobs, tw.tile,
                           tw.rows, tw.crows_comb);
    else
        hipLaunchKernelGGL(fwd_c64_direct<false>, dim3((unsigned)njobs), dim3(kCThreads), 0, s, x, Y, jobs, tw.tile,
                           tw.rows, tw.crows_comb);
    return hipGetLastError();
}

hipError_t launch_fwd_c64(const float2* x, float2* Y, const RealJob* jobs, int64_t njobs, const unsigned* seg,
                          unsigned* queue, int grid, const Twiddles& tw, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fwd_c64_kernel, dim3((unsigned)grid), dim3(kCThreads), 0, s, x, Y, jobs, seg, queue, tw.tile,
                       tw.rows, tw.crows_comb);
    return hipGetLastError();
}

}  // namespace mrdft
