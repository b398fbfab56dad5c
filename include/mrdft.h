/*
 * mrdft.h — multiresolution discrete Fourier transform (MrDFT) on AMD Instinct
 * MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The transform (Section 2, eq. (1), with the level block read as
 * I_{2^{m-i}} (x) E_{2^i} so that every level is N x N): for a signal
 * x[0..N-1], N = 2^m, and every level i = 1..m,
 *
 *     Y^(i)[w*2^i + k] = sum_{n < 2^i} x[w*2^i + n] * exp(-j*2*pi*n*k / 2^i),
 *
 * windows w = 0..N/2^i-1 in time order, bins k = 0..2^i-1 in natural order,
 * no normalisation.  The output of one signal is the m*N values
 * [Y^(1); Y^(2); ...; Y^(m)] (level 1 first), complex64.
 *
 * It is computed with the rationalised recurrence of Section 3, eq. (4): the
 * even bins of level i are sums of adjacent level-(i-1) windows (U^(i), eq. (2))
 * and the odd bins are a half-length FFT of the twiddled window difference
 * (V^(i), eq. (3), D^(i), F^(i)).
 *
 * Conventions common to every entry point
 *   - Memory: every x / Y / gY / gx / z / num_den / L / gL pointer is DEVICE
 *     memory owned by the caller; the plan owns its twiddle tables, tile
 *     tables and workspace.  `offsets` in mrdft_plan_create is HOST memory,
 *     copied during the call.
 *   - Layout: complex64 = interleaved (re, im) float32; real input = float32.
 *     Uniform batches are contiguous: x[b][N], Y[b][m][N].  Ragged batches:
 *     signal j occupies samples [off[j], off[j+1]) of x and the m_j*N_j
 *     outputs starting at O_j = sum_{j'<j} m_j' * N_j' of Y (level-major).
 *   - Pointers must be non-NULL and 16-byte aligned (8 for float32 inputs).
 *   - Asynchrony: every call enqueues work on `stream` (0 = the null stream)
 *     and returns without synchronising.  A plan is immutable after creation;
 *     concurrent calls on the same plan from different streams are NOT
 *     supported (they share one workspace).
 *   - Errors: a non-zero mrdft_status is returned and mrdft_last_error()
 *     gives a thread-local message.  No call aborts or throws.
 */
#ifndef MRDFT_H
#define MRDFT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrdft_plan* mrdft_plan_t;

typedef enum {
    MRDFT_OK = 0,
    MRDFT_E_INVALID_ARG = 1, /* bad order, length, offsets, pointer, alignment or dtype */
    MRDFT_E_UNSUPPORTED = 2, /* valid request the library does not handle */
    MRDFT_E_ALLOC = 3,       /* device or host allocation failed */
    MRDFT_E_HIP = 4          /* a HIP runtime call failed (message has the HIP error) */
} mrdft_status;

typedef enum {
    MRDFT_C64 = 0, /* complex64 input */
    MRDFT_R32 = 1  /* real float32 input (treated as complex with zero imaginary part) */
} mrdft_dtype;

/* Largest supported order m (N = 2^m samples per signal). */
#define MRDFT_MAX_ORDER 28

/* Plan flags */
#define MRDFT_FLAG_NONE 0u
/* Time the candidate schedules (tile depth, job order, persistent grid, and
 * for the winner whether the levels above the tile run on side streams) on
 * scratch buffers at plan creation and keep the fastest; without it the
 * defaults are used.  Costs a few forward calls at creation.
 *
 * Environment, read at plan creation:
 *   MRDFT_TUNE=0|1        overrides MRDFT_FLAG_TUNE (off / on).
 *   MRDFT_TUNE_CACHE=path a tuning cache file (include/mrdft_tune.h): a
 *                         tuned plan whose key is in the file takes the stored
 *                         schedule without timing; otherwise the result of
 *                         timing is stored.  A corrupt file is ignored.
 *   MRDFT_TILE_T=11|12    pins the tile depth after tuning (12 only for
 *                         real plans).
 *   MRDFT_GRAPH=0|1       overrides MRDFT_FLAG_GRAPH.
 *   MRDFT_SERIAL=1        no side streams at all.
 * A malformed value makes plan creation fail with MRDFT_E_INVALID_ARG. */
#define MRDFT_FLAG_TUNE 1u
/* Capture mrdft_forward into a HIP graph on first use for a given (x, Y) pair
 * and replay it afterwards (one graph launch per call); a call with other
 * pointers captures again.  Not combinable with kernel timing. */
#define MRDFT_FLAG_GRAPH 2u
/* Half-spectrum output, real (MRDFT_R32) plans only.  A real window's
 * spectrum is Hermitian (Y[L-k] = conj(Y[k])), so each window of L = 2^i
 * points is stored as L/2 complex values: value 0 = (Y[0], Y[L/2]) (both are
 * real: DC in the real part, Nyquist in the imaginary part), value k = Y[k]
 * for 0 < k < L/2.  Every level then holds N/2 complex values per signal and
 * every length in the layout rules below (N_j per level, m_j * N_j per
 * signal) is halved; output bytes halve.  Level 1 (L = 2) becomes the single
 * value (x0 + x1, x0 - x1).  The adjoint takes gY in the same packed layout:
 * it returns the gradient of a real loss of the packed values, i.e.
 * Re(sum_i A_i^H g^(i)) with g^(i) the packed gradient unpacked with zeros
 * (value 0 -> bins 0 and L/2 as real numbers, value k -> bin k, bins above
 * L/2 zero).  Needs signals of at least 4 samples (m_j >= 2, so that every
 * signal's output stays 16-byte aligned); the spectral-loss calls return
 * MRDFT_E_UNSUPPORTED on such a plan. */
#define MRDFT_FLAG_HALF 4u

/*
 * Create a plan.  Section 2 (problem statement of eq. (1)).
 *   plan    : out, receives the handle.
 *   m       : order of every signal of a uniform batch, 1 <= m <= MRDFT_MAX_ORDER.
 *             Must be 0 when `offsets` is given.
 *   batch   : number of signals, >= 1.
 *   offsets : NULL for a uniform batch; otherwise host int64[batch+1] sample
 *             offsets, offsets[0] = 0, each length offsets[j+1]-offsets[j] a
 *             power of two 2^m_j with 1 <= m_j <= MRDFT_MAX_ORDER.
 *   dtype   : element type of x (MRDFT_C64 or MRDFT_R32).
 *   flags   : MRDFT_FLAG_NONE or an OR of MRDFT_FLAG_TUNE, MRDFT_FLAG_GRAPH,
 *             MRDFT_FLAG_HALF.
 *   stream  : stream used for the plan's one-time uploads (synchronised
 *             before return).
 * Errors: MRDFT_E_INVALID_ARG for any violated rule (MRDFT_FLAG_HALF with
 * complex input or a signal shorter than 4 samples included), MRDFT_E_ALLOC,
 * MRDFT_E_HIP.
 */
mrdft_status mrdft_plan_create(mrdft_plan_t* plan, int m, int64_t batch, const int64_t* offsets,
                               mrdft_dtype dtype, unsigned flags, hipStream_t stream);

/*
 * Same, keeping only the levels lo..hi (1 <= lo <= hi <= MRDFT_MAX_ORDER):
 * signal j stores its levels lo..min(hi, m_j), level i at O_j + (i - lo) N_j
 * with O_j = sum_{j' < j} max(0, min(hi, m_j') - lo + 1) N_j' (a signal with
 * m_j < lo stores nothing).  Output bytes shrink in proportion; the levels
 * above hi inside a tile are not computed, the ones below lo only as far as
 * the recurrence needs them.  The adjoint takes gY in the same layout (the
 * missing levels' gradients are zero).  Uniform batches need lo <= m.  The
 * spectral loss needs the full range.
 * Errors: as mrdft_plan_create, and MRDFT_E_INVALID_ARG for a bad range.
 */
mrdft_status mrdft_plan_create_levels(mrdft_plan_t* plan, int m, int64_t batch, const int64_t* offsets,
                                      mrdft_dtype dtype, unsigned flags, int lo, int hi, hipStream_t stream);

/*
 * Output offsets of a plan, in complex elements: host int64[batch+1],
 * out[j] = O_j (start of signal j's levels in Y), out[batch] = total outputs.
 * Section 2 stacks the m levels of one signal into one mN-vector (eq. (1));
 * these offsets place the stacked vector of every signal of a batch.
 *   out : host memory of batch+1 int64, written.
 * Errors: MRDFT_E_INVALID_ARG for a handle that is not live or out = NULL.
 */
mrdft_status mrdft_plan_output_offsets(mrdft_plan_t plan, int64_t* out);

/* Total number of input samples (the N of Section 2 summed over the batch)
 * and of complex outputs (the mN of eq. (1), summed; shrunk by level ranges
 * and half-spectrum output) of the plan, written to host int64s.
 * Errors: MRDFT_E_INVALID_ARG for a handle that is not live or a NULL pointer. */
mrdft_status mrdft_plan_sizes(mrdft_plan_t plan, int64_t* n_in, int64_t* n_out);

/*
 * Schedule of the forward transform chosen at creation (by the tuner when
 * MRDFT_FLAG_TUNE was given, else the defaults):
 *   tile_log : levels computed per on-chip tile (11 or 12 for complex plans,
 *              12 for real plans); the levels above come from the upper-level
 *              jobs and passes.
 *   grid     : workgroups of the persistent complex launch (0: one
 *              workgroup per job, or not used).
 *   order    : job order, MRDFT_ORDER_*.
 * Any output pointer may be NULL.
 */
#define MRDFT_ORDER_TILES_FIRST 0 /* tiles, then upper-level pieces from the highest level down */
#define MRDFT_ORDER_ROWS_FIRST 1  /* upper-level pieces (highest level first), then tiles */
#define MRDFT_ORDER_INTERLEAVED 2 /* tiles and pieces alternate in proportion */
#define MRDFT_ORDER_BLOCKS 3      /* per block of 2^16 samples: its tiles and the pieces inside it, together */
/* OR-ed into `order`: every forward launch on the caller's stream (the levels
 * above the tile do not run on the plan's side streams). */
#define MRDFT_SCHED_SERIAL 0x100
/* OR-ed into `order`: the levels above the one-launch kernel's levels start
 * when that kernel has finished, on the plan's side streams (concurrently
 * with each other).  Excludes MRDFT_SCHED_SERIAL. */
#define MRDFT_SCHED_AFTER 0x200
mrdft_status mrdft_plan_schedule(mrdft_plan_t plan, int* tile_log, int* grid, int* order);

/*
 * Pin the forward schedule (e.g. one saved from an earlier tuning run) instead
 * of tuning again.  tile_log: 11 or 12 for complex plans, 12 for real plans;
 * grid: workgroups of the persistent complex launch (>= 1; 0: one workgroup
 * per job; ignored for real plans and tile_log 12);
 * order: MRDFT_ORDER_*, optionally OR MRDFT_SCHED_SERIAL or MRDFT_SCHED_AFTER.  Drops a captured
 * forward graph.  Synchronises
 * `stream` (the job table is re-uploaded).
 * Errors: MRDFT_E_INVALID_ARG for values outside these sets.
 */
mrdft_status mrdft_plan_set_schedule(mrdft_plan_t plan, int tile_log, int grid, int order, hipStream_t stream);

/*
 * Forward MrDFT, eq. (1) computed by eq. (4).
 *   x : device, plan dtype, n_in elements.
 *   Y : device, complex64, n_out elements (see layout above); fully overwritten.
 */
mrdft_status mrdft_forward(mrdft_plan_t plan, const void* x, void* Y, hipStream_t stream);

/*
 * Adjoint (conjugate transpose of eq. (1)): gx = sum_i (I (x) E_{2^i})^H gY^(i),
 * i.e. gx[w*2^i + n] += sum_k gY^(i)[w*2^i + k] * exp(+j*2*pi*n*k/2^i), summed
 * over levels.  For real plans gx receives the real part (the gradient of a
 * real loss with respect to a real input).
 *   gY : device, complex64, n_out elements.
 *   gx : device, plan dtype, n_in elements; fully overwritten.
 */
mrdft_status mrdft_adjoint(mrdft_plan_t plan, const void* gY, void* gx, hipStream_t stream);

/*
 * Multi-resolution spectral loss.  NOT part of the paper: a training loss
 * built on the level spectra of eq. (1) (Section 2); the paper defines the
 * transform only.  Readings this library takes: the batch loss is the SUM of
 * the per-signal losses (so a signal's gradient does not depend on the batch
 * size), and z is a constant (not differentiated).
 * Uniform real (MRDFT_R32) plans only:
 *   num_i = || Y^(i)(x) - Y^(i)(z) ||^2,  den_i = || Y^(i)(z) ||^2,
 *   L_b = (1/m) sum_i num_i / den_i,  L = sum_b L_b.
 *   x, z    : device float32 [batch][N].
 *   num_den : device double [batch][m][2] receives (num_i, den_i).
 *   L       : device float, receives L.
 * den_i = 0 (z = 0 on a whole signal) gives an infinite or NaN loss.
 * The first call of either loss entry point on a plan allocates the plan's
 * loss workspace (device memory: x - z and, for N >= 2^12, the packed half
 * spectra of x - z, about 4 m N bytes per signal, and the loss launches' job
 * table; for smaller N both full spectra); make that first call outside any
 * stream capture.
 */
mrdft_status mrdft_spectral_loss_fwd(mrdft_plan_t plan, const float* x, const float* z, double* num_den,
                                     float* L, hipStream_t stream);

/*
 * mrdft_spectral_loss_fwd without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * mrdft_spectral_loss_fwd, for uniform real full-spectrum plans of order
 * 12 <= m <= 16 and batch * m <= 32768; other plans give MRDFT_E_UNSUPPORTED
 * with a message (nothing is enqueued).  The per-level sums live in a
 * workspace inside the library (512 KiB per device, held until the process
 * ends; found once per device at the first call on it), not in the plan:
 * every call on one device shares it, so calls that overlap in time on one
 * device (on different streams, or from different threads) race and must
 * be serialised by the caller.  The call clears the workspace itself, in a
 * kernel, before using it.
 */
mrdft_status mrdft_spectral_loss_fwd_noalloc(mrdft_plan_t plan, const float* x, const float* z, double* num_den,
                                             float* L, hipStream_t stream);

/*
 * Gradient of the spectral loss with respect to x (NOT part of the paper: the
 * adjoint of eq. (1) applied to the loss's level gradients), scaled by *gL:
 *   gx = Re( sum_i A_i^H [ gL * 2 (Y^(i)(x) - Y^(i)(z)) / (m * den_i) ] ),
 * with A_i^H the level-i adjoint above.  The level spectra are recomputed from
 * x and z (nothing of the forward is stored).
 *   num_den : device double [batch][m][2] from mrdft_spectral_loss_fwd.
 *   gL      : device float, upstream gradient of L.
 *   gx      : device float32 [batch][N], overwritten.
 */
mrdft_status mrdft_spectral_loss_bwd(mrdft_plan_t plan, const float* x, const float* z, const double* num_den,
                                     const float* gL, float* gx, hipStream_t stream);

/*
 * Opt-in kernel timing (instrumentation, not part of the transform).  When
 * enabled, every kernel launch of the plan is bracketed by two HIP events
 * recorded on the launch stream.  mrdft_plan_read_profile waits for the
 * recorded events, writes per kind the summed duration in milliseconds and
 * the number of launches (arrays of nkinds entries), and clears the record.
 * Kinds: */
#define MRDFT_KERNEL_TILE_FWD 0 /* on-chip tile levels, forward */
#define MRDFT_KERNEL_PASS_FWD 1 /* global pass of a level above the tile, forward */
#define MRDFT_KERNEL_TILE_ADJ 2 /* on-chip tile levels, adjoint */
#define MRDFT_KERNEL_PASS_ADJ 3 /* global pass, adjoint */
#define MRDFT_KERNEL_FUSED_FWD 4 /* real input: tiles and levels 13..16 in one launch, forward */
#define MRDFT_KERNEL_LOSS 5      /* spectral loss: level norms of the one-launch forward, Y not written */
#define MRDFT_KERNEL_KINDS 6
mrdft_status mrdft_plan_set_profiling(mrdft_plan_t plan, int enable);
mrdft_status mrdft_plan_read_profile(mrdft_plan_t plan, int nkinds, double* total_ms, int64_t* launches);

/* Destroy a plan (NULL is accepted): releases what mrdft_plan_create
 * allocated for the transform of Section 2 (twiddle tables, job tables,
 * workspace, captured graph).  The handle must not be used afterwards.
 * Freeing the plan's device memory waits for the device, so work of the plan
 * still queued on any stream completes first.
 * Errors: MRDFT_E_INVALID_ARG for a handle that is not live (destroyed twice). */
mrdft_status mrdft_plan_destroy(mrdft_plan_t plan);

/*
 * Two-dimensional separable MrDFT.  Section 6 names two-dimensional signals
 * as an application of the multiresolution representation; the transform is
 * the 1-D one of eq. (1) applied along both axes.  For an image x of
 * N1 x N2 = 2^m1 x 2^m2 samples (row-major: N2 consecutive samples per row)
 * and every pair of levels (i1, i2), the 2-D DFT of every non-overlapping
 * 2^i1 x 2^i2 block, L1 = 2^i1, L2 = 2^i2:
 *
 *   Y^(i1,i2)[b1 L1 + k1][b2 L2 + k2] =
 *       sum_{n1 < L1, n2 < L2} x[b1 L1 + n1][b2 L2 + n2] w_L1^{n1 k1} w_L2^{n2 k2},
 *
 * w_L = exp(-j 2 pi / L), no normalisation; m1 * m2 * N1 * N2 complex outputs
 * per image.  Layout of Y (complex64): Y[b][i1-1][n1][i2-1][n2], so the plane
 * of the level pair (i1, i2) of image b starts at ((b m1 + i1 - 1) N1 m2 +
 * i2 - 1) N2 with row stride m2 N2.  Computed as a column transform of the
 * transposed images, a transpose, and a row transform; the plan owns that
 * workspace (about (2 m1 + 1) N1 N2 complex values per image).
 *
 *   mrdft_plan2d_create : 1 <= m1, m2; batch >= 1 images; dtype of x
 *                         (MRDFT_R32 or MRDFT_C64); uploads on `stream`
 *                         (synchronised).  Errors: MRDFT_E_INVALID_ARG,
 *                         MRDFT_E_ALLOC, MRDFT_E_HIP.
 *   mrdft_plan2d_sizes  : samples in (batch N1 N2) and complex outputs
 *                         (batch m1 m2 N1 N2).
 *   mrdft_forward2d     : x device [batch][N1][N2] of the plan dtype ->
 *                         Y device complex64 (layout above), overwritten.
 *   mrdft_adjoint2d     : conjugate transpose, gY in Y's layout -> gx of the
 *                         plan dtype (real plans: the real part), overwritten.
 * Asynchronous on `stream`; one call at a time per plan (shared workspace).
 * A handle that is not live gives MRDFT_E_INVALID_ARG.
 */
typedef struct mrdft_plan2d* mrdft_plan2d_t;
mrdft_status mrdft_plan2d_create(mrdft_plan2d_t* plan, int m1, int m2, int64_t batch, mrdft_dtype dtype,
                                 hipStream_t stream);
mrdft_status mrdft_plan2d_sizes(mrdft_plan2d_t plan, int64_t* n_in, int64_t* n_out);
mrdft_status mrdft_forward2d(mrdft_plan2d_t plan, const void* x, void* Y, hipStream_t stream);
mrdft_status mrdft_adjoint2d(mrdft_plan2d_t plan, const void* gY, void* gx, hipStream_t stream);
mrdft_status mrdft_plan2d_destroy(mrdft_plan2d_t plan);    /* NULL is accepted */

/* Number of device allocations the library currently holds, over all plans
 * of the process (diagnostics: a plan whose creation fails holds none, and
 * destroying every plan brings the count back).  The library's error paths
 * can be exercised by setting MRDFT_FAIL_ALLOC_AT=k in the environment: the
 * k-th device allocation of each subsequent plan creation (or first loss
 * call) then fails with MRDFT_E_ALLOC. */
int64_t mrdft_live_device_allocations(void);

/* Thread-local message of the last failing call on this thread ("" if none).
 * Error reporting of the library itself (the paper defines no interface);
 * the string is owned by the library and valid until the thread's next
 * failing call. */
const char* mrdft_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MRDFT_H */
