// Internal declarations shared by the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrdft {

// Every device allocation and free of the library goes through these two.
// They count the library's live allocations (mrdft_live_device_allocations)
// and implement failure injection: with MRDFT_FAIL_ALLOC_AT=k in the
// environment, the k-th allocation inside the outermost AllocScope of the
// calling thread fails as if the device were out of memory (tests of the
// error paths).
hipError_t dev_malloc_raw(void** p, size_t bytes);
void dev_free(void* p);
template <class T>
hipError_t dev_malloc(T** p, size_t bytes) {
    return dev_malloc_raw(reinterpret_cast<void**>(p), bytes);
}
// Outermost allocating entry point of a call: restarts the allocation count
// (nested calls, e.g. a 2-D plan creating its 1-D plans, share the count).
struct AllocScope {
    AllocScope();
    ~AllocScope();
};

// Levels kept by a plan: [lo, hi] (1-based).  Outputs of other levels are not
// stored and their gradients read as zero; packed into one job field.
struct LevelRange {
    int lo, hi;
    __host__ __device__ bool in(int i) const { return i >= lo && i <= hi; }
    __host__ __device__ static constexpr int32_t pack(int lo, int hi) { return lo | (hi << 8); }
    __host__ __device__ static LevelRange unpack(int32_t v) { return LevelRange{v & 255, (v >> 8) & 255}; }
};

// One on-chip tile of 2^t consecutive samples of one signal.
struct TileJob {
    int64_t in_off;        // element offset of the tile's first sample in x
    int64_t out_off;       // element offset in Y of level 1 at that sample
    int64_t level_stride;  // distance in Y between two levels of this signal (= N)
    int32_t t;             // levels 1..t are computed on chip
    int32_t pad;           // LevelRange::pack(lo, hi) of the levels stored
};

// Geometry of one global Stockham pass over all windows of one level.
struct PassGeom {
    int lg;              // window order: windows hold L = 2^lg points
    int r_log;           // radix of this pass, 2^r_log points per column FFT
    int ns_log;          // span before this pass (log2)
    int64_t nwin;        // number of windows processed
    int64_t wps;         // windows per signal
    // input element offset of window g = (b, W):  in_sig ? in_sig[b] : b*in_stride, + W*L
    const int64_t* in_sig;
    int64_t in_stride;
    const int64_t* out_sig;
    int64_t out_stride;
    float half_scale = 0.5f;   // IN_HALF: scale of half_bin
    // OUT_HALF, if set: the outputs of signal b (of a uniform batch) are
    // multiplied by out_scale[b * out_scale_m + lg - 1] (the loss gradient's
    // per-level factors)
    const float* out_scale = nullptr;
    int out_scale_m = 0;
    // OUT_REC: elements from a window of level lg + 1 back to the same
    // position of level lg in the output (the signal length N)
    int64_t rec_prev = 0;
    // IN_HALF_PAIR / OUT_ADD_R32_PAIR: the chain runs over pairs of windows;
    // window w (< pair_nwin) of the (wps, in_sig/out_sig, strides) geometry
    // is half of pair w / 2
    int64_t pair_nwin = 0;
};

// IN_HALF: a real plan's packed half-spectrum gradient (window W at W * L/2),
// read through half_bin; first passes of the adjoint only (OUT_STORE).
// IN_DIFF, IN_DIFF_R32: odd bins of level lg + 1 (Section 3, eq. (3)): the
// L-point sequence of window W (L = 2^lg) is (x[n] - x[n + L]) w_{2L}^n, with
// x[n] the n-th sample of window W of level lg + 1 (at W * 2L); first passes
// only (OUT_STORE).
// IN_HALF_PAIR: two windows' packed gradients h1, h2 (read as IN_HALF reads
// one) enter as h1 + i h2; since both are Hermitian, the conjugate DFT of the
// sum is G1 + i G2 with G1, G2 real (adjoint with real output).
// IN_R32_PAIR: two real windows x1, x2 of one signal enter as x1 + i x2; the
// spectrum Z = X1 + i X2 has sum_k |Z[k]|^2 = sum_k |X1[k]|^2 + |X2[k]|^2
// (X1, X2 are Hermitian), so an OUT_NORM chain over such pairs adds the two
// windows' squared magnitudes (first passes only).
enum InKind { IN_C64 = 0, IN_R32 = 1, IN_HALF = 2, IN_DIFF = 3, IN_DIFF_R32 = 4, IN_HALF_PAIR = 5, IN_R32_PAIR = 6 };
// OUT_HALF: store packed half spectra (window W at W * L/2, slot 0 = (Y[0], Y[L/2])).
// OUT_NORM: nothing stored; the squared magnitudes of signal b's level lg are
// added (FP64) to ((double*)out)[b * out_stride + lg - 1].
// OUT_REC: the last pass of an IN_DIFF chain stores window W of level lg + 1
// (at W * 2L): bin 2k + 1 is the pass output k, bin 2k the sum of bin k of
// the two child windows of level lg, read rec_prev elements back (eq. (2)).
// OUT_ADD_R32_PAIR: the last pass of an IN_HALF_PAIR chain adds the real
// part of its output to the first window's samples and the imaginary part
// to the second's.
enum OutKind { OUT_STORE = 0, OUT_ADD_C64 = 1, OUT_ADD_R32 = 2, OUT_HALF = 3, OUT_NORM = 4, OUT_REC = 5,
               OUT_ADD_R32_PAIR = 6 };

struct Twiddles {
    const float2* tile;   // w_{4096}^e, e < 4096 (FP32, rounded once from FP64)
    const float2* rowtw;  // row twiddles w_{2^l}^{n1*k2} of the single-pass levels (FP32, rounded once)
    const float2* rows;   // row twiddles of the real 256-point-row levels 13..16 (FP32, rounded once)
    const float4* rows_comb;  // column-combine factors of the real levels (FP32, rounded once)
    const float2* crows_comb; // column-combine factors of the complex levels 12..16 (FP32, rounded once)
    const double2* hi;    // w_{2^28}^{a*2^14}, a < 2^14 (FP64)
    const double2* lo;    // w_{2^28}^{b}, b < 2^14 (FP64)
};

// One job of the real forward launch (mrdft_fwd_real.hip).
struct RealJob {
    int64_t in_off;        // x offset of the tile, or of the window
    int64_t out_off;       // Y offset of the tile's level-1 output, or of the window's output at its level
    int64_t level_stride;  // tile: distance in Y between two levels (= N); rows piece: unused
    int32_t lg;            // 0: tile of 4096 samples (levels 1..12); 13..16: rows piece of level lg
    int32_t g;             // rows piece index, 0 <= g < 2^(lg-13); tile: LevelRange::pack of the levels kept
};
// Row twiddles w_L^{n1 k2} (n1 < 256, k2 < L/256) of levels 12..16, [k2][n1] per level.
__host__ __device__ constexpr int64_t rows_twiddle_offset(int lg) {
    return lg <= 12 ? 0 : rows_twiddle_offset(lg - 1) + ((int64_t)1 << (lg - 1));
}
constexpr int64_t rows_twiddle_entries() { return rows_twiddle_offset(17); }
// half: packed half-spectrum output (job offsets and level strides in those units).
hipError_t launch_fwd_real(const float* x, float2* Y, const RealJob* jobs, int64_t njobs, const Twiddles& tw,
                           hipStream_t s, bool half = false);
// Same jobs, spectral loss: the input is x - xsub (xsub may be null) and the
// squared magnitudes of every level are added to sums[b * m + level - 1]
// (uniform batch; the rows jobs carry level_stride = N).  Y is not written.
// Same jobs, spectral-loss gradient: input x - xsub, level i of signal b
// stored times alpha[b * m + i - 1] (uniform batch); half: as packed half
// spectra (offsets of the full-spectrum job table halved).
hipError_t launch_fwd_real_scaled(const float* x, const float* xsub, const float* alpha, int m, float2* Y,
                                  const RealJob* jobs, int64_t njobs, const Twiddles& tw, hipStream_t s,
                                  bool half = false);
hipError_t launch_fwd_real_norms(const float* x, const float* xsub, double* sums, int m, const RealJob* jobs,
                                 int64_t njobs, const Twiddles& tw, hipStream_t s);
// Complex input: 2048-sample tiles (lg = 0, levels 1..11) and pieces of levels
// 12..16 (mrdft_fwd_c64.hip).  Persistent: `grid` workgroups take jobs from
// the table's 8 per-XCD segments [seg[q], seg[q+1]) through the counters
// queue[0..7] until every segment is exhausted; the last workgroup out
// (counted in queue[8]) clears queue[0..8] for the next launch (the plan
// zeroes them once at creation).
constexpr int kC64TileLog = 11;
// Job kind of a 2048-sample tile holding several consecutive signals of
// 2^m samples, m < 11: lg = kMultiTileLg + m, level_stride = 2^m | (valid
// samples << 32), g = LevelRange::pack(lo, min(hi, m)).
constexpr int kMultiTileLg = 32;
constexpr int kC64Queues = 9;
// Adjoint (mrdft_adj.hip).  Launch (a): RealJob with in_off = gY offset (the
// tile's level-1 gradient, or the window's gradient at its level), out_off =
// gx offset of the tile or scratch offset of the window's block, lg = 0 for a
// 2048-sample tile, 12..16 for a rows piece g.  Launch (b): one columns job.
struct AdjColJob {
    int64_t gx_off;        // gx offset of the region's first sample
    int64_t scr_off;       // scratch offset of the region in the level-12 block
    int64_t level_stride;  // distance between two levels' scratch blocks (= N)
    int32_t region_log;    // region of 2^region_log samples (12 .. 16)
    int32_t c;             // columns 16 (c & 15) .. +15; c >> 8 = LevelRange::pack of the levels kept
};
// Half-spectrum plans: one job unpacks `len` consecutive bins (from bin c0)
// of one level of one signal from the packed gradient (level at hlev) into the
// full-spectrum gradient (level at flev), windows of 2^lg bins.
struct HalfJob {
    int64_t hlev;
    int64_t flev;
    int64_t c0;
    int32_t lg;
    int32_t len;
};
constexpr int kHalfChunk = 4096;
hipError_t launch_expand_half(const float2* gh, float2* g, const HalfJob* jobs, int64_t njobs, hipStream_t s);
// half: gY holds packed half spectra (real output only), read by half_bin
// with scale hsc; the jobs' gradient offsets and tile level strides are
// shifted right by gshift (1: a full-spectrum job table over a packed gradient).
hipError_t launch_adj_a(bool real_out, bool half, int gshift, float hsc, const float2* gY, void* gx, float2* scratch,
                        const RealJob* jobs, int64_t njobs, const Twiddles& tw, hipStream_t s);
// Clears `bytes` (a multiple of 4) at p (4-byte aligned) with vector stores.
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);
hipError_t launch_adj_b(bool real_out, void* gx, const float2* scratch, const AdjColJob* jobs, int64_t njobs,
                        const Twiddles& tw, hipStream_t s);
hipError_t launch_fwd_c64(const float2* x, float2* Y, const RealJob* jobs, int64_t njobs, const unsigned* seg,
                          unsigned* queue, int grid, const Twiddles& tw, hipStream_t s);
// Same jobs, one workgroup per job (table dealt round-robin over the XCDs).
// real_in: float32 signals below 4096 samples of a real plan (tile and
// multi-signal tile jobs only), written as full complex spectra.
hipError_t launch_fwd_c64_direct(const void* x, float2* Y, const RealJob* jobs, int64_t njobs, const Twiddles& tw,
                                 hipStream_t s, bool real_in = false);
// half (real input only): packed half-spectrum output, job offsets and level
// strides in those units.
// tmax: the largest tile order t among the jobs (sizes the launch's LDS).
hipError_t launch_tile_fwd(bool real_in, const void* x, float2* Y, const TileJob* jobs, int64_t njobs, int tmax,
                           const Twiddles& tw, hipStream_t s, bool half = false);
// Real input, 4096-sample tiles (levels 1..12): see mrdft_tile_real.h.
constexpr int kRealTileLog = 12;
hipError_t launch_tile_adj(bool real_out, const float2* gY, void* gx, const TileJob* jobs, int64_t njobs, int tmax,
                           const Twiddles& tw, hipStream_t s);
// Single-pass levels with window 2^(10 + rl), 1 <= rl <= 6 (see mrdft_upper.hip).
constexpr int kUpperMaxLevel = 16;
int64_t row_twiddle_offset(int lg);
int64_t row_twiddle_entries();
hipError_t launch_upper_fwd(bool real_in, const void* x, float2* Y, const PassGeom& g, const Twiddles& tw,
                            hipStream_t s);
// The first passes of level lg (two windows) and of the recurrence chain of
// level lg + 1 from one read of x (radix up to 2^kPassMaxLog): see mrdft_pass.hip.
// gs (or null): windows of level lg of signals that end there, their plain
// first pass (to out_s) in the same launch.
hipError_t launch_pass_head2(int in_kind, const void* in, float2* out_lo, float2* out_hi, const PassGeom& g,
                             float2* out_s, const PassGeom* gs, const Twiddles& tw, hipStream_t s);
// The last passes of level lg (two windows) and of level lg + 1's recurrence
// chain in one launch; level lg's spectra give level lg + 1's even bins
// without being read back (see mrdft_pass.hip).  gs (or null): the plain
// last pass of the windows given to the head's gs, from s_s to y_s.
hipError_t launch_pass_tail2(const float2* s_lo, const float2* s_hi, float2* y_lo, float2* y_hi, const PassGeom& g,
                             const float2* s_s, float2* y_s, const PassGeom* gs, const Twiddles& tw, hipStream_t s);
hipError_t launch_pass(bool inv, int in_kind, int out_kind, const void* in, void* out, const PassGeom& g,
                       const Twiddles& tw, hipStream_t s);

}  // namespace mrdft
