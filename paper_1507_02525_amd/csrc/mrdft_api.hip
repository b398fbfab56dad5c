// Host side of the C ABI declared in include/mrdft.h: plan creation and
// validation, FP64 twiddle generation, tile tables, launch sequencing.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/mrdft.h"
#include "../../include/mrdft_tune.h"
#include "mrdft_device.h"
#include "mrdft_internal.h"
#include "mrdft_loss.h"
#include "mrdft_rows_c64.h"
#include "mrdft_rows_real.h"

using namespace mrdft;

namespace {

thread_local std::string g_last_error;

// Live plans, so that a destroyed or foreign handle is rejected instead of
// being dereferenced.
std::mutex g_plans_mu;
std::set<const void*> g_plans;

mrdft_status fail(mrdft_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(MRDFT_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int ilog2_exact(int64_t v) {
    if (v <= 0 || (v & (v - 1))) return -1;
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// Signals of one order share the global passes of their upper levels.
struct Group {
    int order = 0;
    int64_t count = 0;
    int64_t* d_in_sig = nullptr;    // x offset of each signal (ragged only)
    int64_t* d_out_sig = nullptr;   // Y offset of each signal (ragged only)
};

// Bit split of the passes for a window of 2^lg points (each pass radix <= 2^8,
// first pass radix >= 2^4).
std::vector<int> pass_bits(int lg) {
    const int np = (lg + kPassMaxLog - 1) / kPassMaxLog;
    std::vector<int> b(np, lg / np);
    for (int p = 0; p < lg % np; ++p) b[p] += 1;
    return b;
}

// Lowest level of a forward recurrence chain: from level 18 up a level is
// built from the level below (even bins, eq. (2)) and the half-length DFT of
// the twiddled difference (odd bins, eq. (3)).  Level 18's chain shares its
// head with level 17's (one read of x, launch_pass_head2) and its tail (level
// 17's spectra give the even bins without a read back, launch_pass_tail2):
// the two levels move 6 units of 8N bytes instead of 8; each level whose
// direct chain needs three passes moves 4 (level 19) or 5 instead of 6.
constexpr int kRecMinLevel = 2 * kPassMaxLog;

}  // namespace

struct mrdft_plan {
    int m = 0;
    int64_t batch = 0;
    mrdft_dtype dtype = MRDFT_C64;
    bool ragged = false;
    std::vector<int64_t> in_off, out_off;   // [batch+1]
    // levels kept: [lo, hi]; signal j stores levels lo..min(hi, m_j) at
    // out_off[j] + (i - lo) N_j, i.e. at base(j) + (i - 1) N_j (N_j / 2 for
    // half-spectrum plans, hs = 1)
    int lo = 1, hi = MRDFT_MAX_ORDER;
    int hs = 0;
    int kept(int order) const { return std::max(0, std::min(hi, order) - lo + 1); }
    int64_t base(int64_t j) const { return out_off[j] - (int64_t)(lo - 1) * ((in_off[j + 1] - in_off[j]) >> hs); }
    // full-spectrum layout of the same levels (the half plans' adjoint works in it)
    std::vector<int64_t> fout_off;
    int64_t n_fout = 0;
    int64_t basef(int64_t j) const { return fout_off[j] - (int64_t)(lo - 1) * (in_off[j + 1] - in_off[j]); }
    HalfJob* d_hjobs = nullptr;             // half plans: unpacking jobs of the adjoint
    int64_t nhjobs = 0;
    float2* d_gfull = nullptr;              // half plans: unpacked gradient, full layout
    int32_t range() const { return LevelRange::pack(lo, std::min(hi, 255)); }
    bool full_range(int order) const { return lo == 1 && hi >= order; }
    std::vector<int> orders;
    int64_t n_in = 0, n_out = 0;
    int max_order = 0;
    TileJob* d_jobs = nullptr;
    int64_t njobs = 0;
    int64_t njobs_full = 0;                 // leading jobs with t = 12 (full 4096-sample tiles)
    int jobs_tmax = 1, tail_tmax = 1;       // largest t of all tile jobs / of those after njobs_full
    int asmall_tmax = 1;                    // largest t of d_asmall
    std::vector<Group> groups;
    float2* d_tw_tile = nullptr;
    double2* d_tw_hi = nullptr;
    double2* d_tw_lo = nullptr;
    float2* d_tw16 = nullptr;
    float2* d_tw_rows = nullptr;
    float4* d_tw_comb = nullptr;
    float2* d_tw_ccomb = nullptr;
    // real input: tiles of 4096 samples and rows pieces of levels 13..16, one launch
    RealJob* d_rjobs = nullptr;
    int64_t nrjobs = 0;
    RealJob* d_ljobs = nullptr;             // the fused loss's own table of the same jobs
    int64_t nljobs = 0;
    RealJob* d_sjobs = nullptr;             // real full-spectrum plans: signals below 4096 samples
    int64_t nsjobs = 0;                     // (complex-launch tiles reading real input)
    // complex input: tiles of 2048 samples (several signals of order < 11 per
    // tile) and rows pieces of levels 12..16 in one launch (tile_log 11: one
    // workgroup per job, or persistent), or the tile kernel with 4096-sample
    // tiles and one launch per upper level (tile_log 12)
    RealJob* d_cjobs = nullptr;
    int64_t ncjobs = 0;
    bool cjobs_direct = false;              // d_cjobs dealt for one workgroup per job (grid 0)
    unsigned* d_queue = nullptr;            // persistent launch: next job per XCD segment, workgroups done
    unsigned* d_cseg = nullptr;             // starts of the 8 segments of the complex job table
    // adjoint: launch (a) tiles + rows pieces, launch (b) columns jobs, scratch B
    RealJob* d_ajobs = nullptr;
    int64_t najobs = 0;
    AdjColJob* d_acols = nullptr;
    int64_t nacols = 0;
    TileJob* d_asmall = nullptr;            // signals of order < 11: tile adjoint kernel
    int64_t nasmall = 0;
    bool adj_zero = false;                  // no tile level kept: gx is cleared instead of running the tiles
    float2* d_ascratch = nullptr;
    // schedule (tuned or default)
    unsigned flags = 0;
    int tile_log = kTileMaxLog;
    int grid = 0;
    int order = MRDFT_ORDER_BLOCKS;
    int num_cu = 0;
    // graph replay of the forward
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gkey_x = nullptr;
    void* gkey_y = nullptr;
    float2* d_s[2] = {nullptr, nullptr};    // pass ping-pong scratch of the caller's stream / side stream 0
    float2* d_ss[3][2] = {};                // ping-pong scratch of side streams 1..3
    int64_t scratch_pts = 0;                // complex points of each of those arrays
    // spectral loss workspace
    float* d_v = nullptr;
    float2* d_Yv = nullptr;
    float2* d_Yz = nullptr;
    double* d_part = nullptr;
    double* d_sums = nullptr;               // fused loss: [2][batch * m] (num, den) sums
    float* d_alpha = nullptr;               // loss gradient: per-level factors [batch * m]
    // side stream for the levels above the tile (they write other parts of Y,
    // so they run concurrently with the tile kernel); fork/join via events
    static constexpr int kSides = 4;
    hipStream_t side[kSides] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSides] = {nullptr, nullptr, nullptr, nullptr};
    int nsides = 0;
    bool serial = false;                    // forward: every launch on the caller's stream (tuned choice)
    bool after = false;                     // forward: side-stream levels start after the main launch (tuned choice)
    // opt-in kernel timing: events recorded around every launch on its stream
    bool profiling = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> event_pool;

    Twiddles tw() const { return Twiddles{d_tw_tile, d_tw16, d_tw_rows, d_tw_comb, d_tw_ccomb, d_tw_hi, d_tw_lo}; }
};

namespace {

void dfree(void* ptr) { dev_free(ptr); }

void free_plan(mrdft_plan* p) {
    if (!p) return;
    for (auto& r : p->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : p->event_pool) (void)hipEventDestroy(e);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (int k = 0; k < p->nsides; ++k) {
        if (p->join_ev[k]) (void)hipEventDestroy(p->join_ev[k]);
        if (p->side[k]) (void)hipStreamDestroy(p->side[k]);
    }
    dfree(p->d_jobs);
    for (auto& g : p->groups) {
        dfree(g.d_in_sig);
        dfree(g.d_out_sig);
    }
    dfree(p->d_tw_tile);
    dfree(p->d_tw_hi);
    dfree(p->d_tw_lo);
    dfree(p->d_tw16);
    dfree(p->d_tw_rows);
    dfree(p->d_tw_comb);
    dfree(p->d_tw_ccomb);
    dfree(p->d_rjobs);
    dfree(p->d_ljobs);
    dfree(p->d_sjobs);
    dfree(p->d_cjobs);
    dfree(p->d_queue);
    dfree(p->d_cseg);
    dfree(p->d_ajobs);
    dfree(p->d_acols);
    dfree(p->d_asmall);
    dfree(p->d_ascratch);
    dfree(p->d_hjobs);
    dfree(p->d_gfull);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    dfree(p->d_s[0]);
    dfree(p->d_s[1]);
    for (auto& pr : p->d_ss) {
        dfree(pr[0]);
        dfree(pr[1]);
    }
    dfree(p->d_v);
    dfree(p->d_Yv);
    dfree(p->d_Yz);
    dfree(p->d_part);
    dfree(p->d_sums);
    dfree(p->d_alpha);
    delete p;
}

mrdft_status upload_twiddles(mrdft_plan* p, hipStream_t s) {
    std::vector<float2> tile(kTileMax);
    for (int e = 0; e < kTileMax; ++e) {
        const double a = 2.0 * M_PI * (double)e / (double)kTileMax;
        tile[e] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
    }
    const int nf = 1 << kTwFineLog;
    std::vector<double2> hi(nf), lo(nf);
    for (int e = 0; e < nf; ++e) {
        const double ah = 2.0 * M_PI * (double)e / (double)nf;                       // a * 2^14 / 2^28
        const double al = 2.0 * M_PI * (double)e / (double)(int64_t(1) << kMaxOrder);
        hi[e] = make_double2(std::cos(ah), -std::sin(ah));
        lo[e] = make_double2(std::cos(al), -std::sin(al));
    }
    // Row twiddles w_{2^l}^{n1*k2} (n1 < 1024, k2 < 2^(l-10)) of the single-pass
    // levels l = 11..16, each block laid out [k2][n1].
    const int64_t nrow = row_twiddle_entries();
    std::vector<float2> rt(nrow);
    for (int l = 11; l <= kUpperMaxLevel; ++l) {
        const int64_t off = row_twiddle_offset(l);
        const int64_t Ll = int64_t(1) << l;
        for (int64_t k2 = 0; k2 < (Ll >> 10); ++k2)
            for (int64_t n1 = 0; n1 < 1024; ++n1) {
                const double a = 2.0 * M_PI * (double)((n1 * k2) % Ll) / (double)Ll;
                rt[off + k2 * 1024 + n1] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
            }
    }
    if (dev_malloc(&p->d_tw16, sizeof(float2) * nrow) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "twiddle table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_tw16, rt.data(), sizeof(float2) * nrow, hipMemcpyHostToDevice, s));
    // Row twiddles w_L^{n1*k2} (n1 < 256, k2 < L/256) of the real levels 13..16, [k2][n1].
    const int64_t nrows = rows_twiddle_entries();
    std::vector<float2> rr(nrows);
    for (int l = kCRowsMinLevel; l <= kRowsMaxLevel; ++l) {
        const int64_t off = rows_twiddle_offset(l);
        const int64_t Ll = int64_t(1) << l;
        for (int64_t k2 = 0; k2 < (Ll >> kRowsLog); ++k2)
            for (int64_t n1 = 0; n1 < kRowsN; ++n1) {
                const double a = 2.0 * M_PI * (double)((n1 * k2) % Ll) / (double)Ll;
                rr[off + k2 * kRowsN + n1] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
            }
    }
    if (dev_malloc(&p->d_tw_rows, sizeof(float2) * nrows) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "twiddle table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_tw_rows, rr.data(), sizeof(float2) * nrows, hipMemcpyHostToDevice, s));
    // Column-combine factors of those levels: for piece g, pair s, row q (k = 16 g + q),
    // wa = w_R^{2s k}, wb = w_R^{(2s+1) k}, u = (wa - j wb)/2, v = (wa + j wb)/2.
    const int64_t ncomb = rows_combine_entries();
    std::vector<float4> cv(ncomb);
    for (int l = kRowsMinLevel; l <= kRowsMaxLevel; ++l) {
        const int64_t R = int64_t(1) << (l - kRowsLog);
        const int64_t half = R / 32;                      // pieces per window = pairs per column
        for (int64_t g = 0; g < half; ++g)
            for (int64_t sp = 0; sp < half; ++sp)
                for (int q = 0; q < kRowsMax; ++q) {
                    const int64_t k = 16 * g + q;
                    const double aa = 2.0 * M_PI * (double)((2 * sp * k) % R) / (double)R;
                    const double ab = 2.0 * M_PI * (double)(((2 * sp + 1) * k) % R) / (double)R;
                    const double wax = std::cos(aa), way = -std::sin(aa), wbx = std::cos(ab), wby = -std::sin(ab);
                    cv[rows_combine_offset(l) + (g * half + sp) * kRowsMax + q] =
                        make_float4((float)(0.5 * (wax + wby)), (float)(0.5 * (way - wbx)),
                                    (float)(0.5 * (wax - wby)), (float)(0.5 * (way + wbx)));
                }
    }
    if (dev_malloc(&p->d_tw_comb, sizeof(float4) * ncomb) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "twiddle table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_tw_comb, cv.data(), sizeof(float4) * ncomb, hipMemcpyHostToDevice, s));
    // Combine factors of the complex levels 12..16: w_R^{r (16 g + q)}, index ((g * P + r) * 16 + q).
    const int64_t nccomb = crows_combine_entries();
    std::vector<float2> cc(nccomb);
    for (int l = kCRowsMinLevel; l <= kRowsMaxLevel; ++l) {
        const int64_t R = int64_t(1) << (l - kRowsLog), P = R / 16;
        for (int64_t g = 0; g < R / 16; ++g)
            for (int64_t r = 0; r < P; ++r)
                for (int q = 0; q < 16; ++q) {
                    const double a = 2.0 * M_PI * (double)((r * (16 * g + q)) % R) / (double)R;
                    cc[crows_combine_offset(l) + (g * P + r) * 16 + q] =
                        make_float2((float)std::cos(a), (float)(-std::sin(a)));
                }
    }
    if (dev_malloc(&p->d_tw_ccomb, sizeof(float2) * nccomb) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "twiddle table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_tw_ccomb, cc.data(), sizeof(float2) * nccomb, hipMemcpyHostToDevice, s));
    if (dev_malloc(&p->d_tw_tile, sizeof(float2) * kTileMax) != hipSuccess ||
        dev_malloc(&p->d_tw_hi, sizeof(double2) * nf) != hipSuccess ||
        dev_malloc(&p->d_tw_lo, sizeof(double2) * nf) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "twiddle table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_tw_tile, tile.data(), sizeof(float2) * kTileMax, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_tw_hi, hi.data(), sizeof(double2) * nf, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_tw_lo, lo.data(), sizeof(double2) * nf, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MRDFT_OK;
}

// Order of a block's jobs in the block-major order: tiles and pieces
// alternating in proportion, all pieces first, or all tiles first.
enum class InBlock { kAlternate, kPiecesFirst, kTilesFirst };
std::vector<RealJob> real_jobs(const mrdft_plan* p, int order, InBlock in = InBlock::kPiecesFirst);
struct JobBlock {
    std::vector<RealJob> tiles, pieces;
    int64_t cost;
};
std::vector<RealJob> deal_blocks(const std::vector<JobBlock>& blocks);
std::vector<RealJob> complex_jobs(const mrdft_plan* p, int order, std::vector<unsigned>* seg);
std::vector<RealJob> small_real_jobs(const mrdft_plan* p);
mrdft_status upload_cjobs(mrdft_plan* p, int order, hipStream_t s, bool direct);
mrdft_status upload_jobs(const std::vector<RealJob>& v, RealJob** dst, int64_t* n, hipStream_t s);

mrdft_status build_tables(mrdft_plan* p, hipStream_t s) {
    std::vector<TileJob> jobs;
    std::vector<std::vector<int64_t>> gin(kMaxOrder + 1), gout(kMaxOrder + 1);
    for (int64_t j = 0; j < p->batch; ++j) {
        const int mj = p->orders[j];
        const int64_t N = int64_t(1) << mj;
        const int t = mj < kTileMaxLog ? mj : kTileMaxLog;
        const int64_t T = int64_t(1) << t;
        for (int64_t tau = 0; p->lo <= t && tau < N / T; ++tau) {     // a tile below the range stores nothing
            TileJob jb;
            jb.in_off = p->in_off[j] + tau * T;
            jb.out_off = p->base(j) + ((tau * T) >> p->hs);
            jb.level_stride = N >> p->hs;
            jb.t = t;
            jb.pad = p->range();
            jobs.push_back(jb);
        }
        if (mj > kTileMaxLog) {
            gin[mj].push_back(p->in_off[j]);
            gout[mj].push_back(p->base(j));
        }
    }
    // full tiles first: the real-input kernel handles exactly those
    std::stable_partition(jobs.begin(), jobs.end(), [](const TileJob& a) { return a.t == kRealTileLog; });
    p->njobs = (int64_t)jobs.size();
    p->njobs_full = 0;
    while (p->njobs_full < p->njobs && jobs[p->njobs_full].t == kRealTileLog) ++p->njobs_full;
    for (int64_t q = 0; q < p->njobs; ++q) {
        p->jobs_tmax = std::max(p->jobs_tmax, (int)jobs[q].t);
        if (q >= p->njobs_full) p->tail_tmax = std::max(p->tail_tmax, (int)jobs[q].t);
    }
    if (!jobs.empty()) {
        if (dev_malloc(&p->d_jobs, sizeof(TileJob) * jobs.size()) != hipSuccess)
            return fail(MRDFT_E_ALLOC, "tile table allocation failed (%zu bytes)", sizeof(TileJob) * jobs.size());
        HIP_TRY(hipMemcpyAsync(p->d_jobs, jobs.data(), sizeof(TileJob) * jobs.size(), hipMemcpyHostToDevice, s));
    }
    if (p->dtype == MRDFT_R32) {
        mrdft_status st = upload_jobs(real_jobs(p, p->order), &p->d_rjobs, &p->nrjobs, s);
        if (st) return st;
        if (!p->hs) {
            st = upload_jobs(small_real_jobs(p), &p->d_sjobs, &p->nsjobs, s);
            if (st) return st;
        }
    } else {
        mrdft_status st = upload_cjobs(p, p->order, s, true);   // default: one workgroup per job
        if (st) return st;
        if (p->ncjobs > 0) {
            if (!p->d_queue && dev_malloc(&p->d_queue, kC64Queues * sizeof(unsigned)) != hipSuccess)
                return fail(MRDFT_E_ALLOC, "queue allocation failed");
            HIP_TRY(hipMemsetAsync(p->d_queue, 0, kC64Queues * sizeof(unsigned), s));   // once; kernels restore it
            p->tile_log = kC64TileLog;
            p->grid = 0;      // one workgroup per job (the tuner also tries persistent grids)
        }
    }
    {
        // adjoint tables: 2048-sample tiles and rows pieces of levels 12..16 (launch a),
        // columns jobs per region of up to 2^16 samples (launch b), scratch B per signal
        std::vector<JobBlock> ablocks;
        std::vector<AdjColJob> cj;
        std::vector<TileJob> sm;
        int64_t scr = 0;
        static const int kColOrder[16] = {0, 2, 4, 6, 8, 10, 12, 14, 1, 3, 5, 7, 9, 11, 13, 15};
        // with no tile level kept the tiles would only write zeros: gx is
        // cleared by one fill before the columns phase adds to it
        p->adj_zero = p->lo > kC64TileLog;
        for (int64_t j = 0; j < p->batch; ++j) {
            const int mj = p->orders[j];
            const int64_t N = int64_t(1) << mj;
            if (mj < kC64TileLog) {
                if (!p->adj_zero) sm.push_back(TileJob{p->in_off[j], p->basef(j), N, mj, p->range()});
                continue;
            }
            // gradient offsets: packed half spectra for half plans (read through
            // half_bin), the full layout otherwise
            const int64_t gb = p->hs ? p->base(j) : p->basef(j);
            const int hs = p->hs;
            const int top = std::min(mj, kRowsMaxLevel);
            bool any_upper = false;
            // one block per region of 2^top samples: its tiles and the rows
            // pieces of its windows (a real piece reads rows that its
            // neighbours read too, so a region's jobs share one XCD's L2)
            const int64_t region = int64_t(1) << top;
            for (int64_t u0 = 0; u0 < N; u0 += region) {
                JobBlock blk;
                for (int64_t tau = u0 >> kC64TileLog; !p->adj_zero && tau < (u0 + region) >> kC64TileLog; ++tau)
                    blk.tiles.push_back(RealJob{gb + ((tau << kC64TileLog) >> hs), p->in_off[j] + (tau << kC64TileLog),
                                                N >> hs, 0, p->range()});
                for (int lg = kCRowsMinLevel; lg <= top; ++lg) {
                    if (lg < p->lo || lg > p->hi) continue;
                    any_upper = true;
                    const int64_t L = int64_t(1) << lg;
                    // real plans: 17-row Hermitian pieces above level 12 (half as many)
                    const int pieces = (p->dtype == MRDFT_R32 && lg > kCRowsMinLevel) ? 1 << (lg - kCRowsMinLevel - 1)
                                                                                       : 1 << (lg - kCRowsMinLevel);
                    for (int64_t w = u0 / L; w < (u0 + region) / L; ++w)
                        for (int g = 0; g < pieces; ++g)
                            blk.pieces.push_back(RealJob{gb + (((int64_t)(lg - 1) * N + w * L) >> hs),
                                                         scr + (int64_t)(lg - kCRowsMinLevel) * N + w * L, 0, lg, g});
                }
                // cost ~ gradient bytes read: 11 levels of a tile, ~2 x 17 rows of a piece
                blk.cost = 11 * (int64_t)blk.tiles.size() + 6 * (int64_t)blk.pieces.size();
                if (blk.cost) ablocks.push_back(std::move(blk));
            }
            if (top >= kCRowsMinLevel) {
                if (any_upper)
                    for (int64_t r = 0; r < N / region; ++r)
                        for (int c = 0; c < 16; ++c)
                            cj.push_back(AdjColJob{p->in_off[j] + r * region, scr + r * region, N, top,
                                                   kColOrder[c] | (p->range() << 8)});
                scr += (int64_t)(top - kCRowsMinLevel + 1) * N;
            }
        }
        const std::vector<RealJob> aj = deal_blocks(ablocks);
        p->najobs = (int64_t)aj.size();
        p->nacols = (int64_t)cj.size();
        p->nasmall = (int64_t)sm.size();
        for (const TileJob& t : sm) p->asmall_tmax = std::max(p->asmall_tmax, (int)t.t);
        if ((!aj.empty() && dev_malloc(&p->d_ajobs, sizeof(RealJob) * aj.size()) != hipSuccess) ||
            (!cj.empty() && dev_malloc(&p->d_acols, sizeof(AdjColJob) * cj.size()) != hipSuccess) ||
            (!sm.empty() && dev_malloc(&p->d_asmall, sizeof(TileJob) * sm.size()) != hipSuccess) ||
            (scr > 0 && dev_malloc(&p->d_ascratch, sizeof(float2) * scr) != hipSuccess))
            return fail(MRDFT_E_ALLOC, "adjoint tables or scratch allocation failed (%lld complex)", (long long)scr);
        if (!aj.empty()) HIP_TRY(hipMemcpyAsync(p->d_ajobs, aj.data(), sizeof(RealJob) * aj.size(), hipMemcpyHostToDevice, s));
        if (!cj.empty())
            HIP_TRY(hipMemcpyAsync(p->d_acols, cj.data(), sizeof(AdjColJob) * cj.size(), hipMemcpyHostToDevice, s));
        if (!sm.empty()) HIP_TRY(hipMemcpyAsync(p->d_asmall, sm.data(), sizeof(TileJob) * sm.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (p->hs) {
        // adjoint of the packed output: the tiles, pieces and passes read the
        // packed gradient directly; signals below the 2048-sample tile (tile
        // adjoint kernel) are unpacked into the full layout first
        std::vector<HalfJob> hj;
        for (int64_t j = 0; j < p->batch; ++j) {
            const int mj = p->orders[j];
            if (mj >= kC64TileLog) continue;
            const int64_t N = int64_t(1) << mj;
            for (int i = p->lo; i <= std::min(p->hi, mj); ++i)
                for (int64_t c0 = 0; c0 < N; c0 += kHalfChunk)
                    hj.push_back(HalfJob{p->base(j) + (int64_t)(i - 1) * (N / 2), p->basef(j) + (int64_t)(i - 1) * N,
                                         c0, i, (int32_t)std::min<int64_t>(N, kHalfChunk)});
        }
        p->nhjobs = (int64_t)hj.size();
        if (!hj.empty()) {
            if (dev_malloc(&p->d_hjobs, sizeof(HalfJob) * hj.size()) != hipSuccess ||
                dev_malloc(&p->d_gfull, sizeof(float2) * p->n_fout) != hipSuccess)
                return fail(MRDFT_E_ALLOC, "half-spectrum gradient workspace allocation failed (%lld complex)",
                            (long long)p->n_fout);
            HIP_TRY(hipMemcpyAsync(p->d_hjobs, hj.data(), sizeof(HalfJob) * hj.size(), hipMemcpyHostToDevice, s));
        }
    }
    int64_t scratch = 0;
    for (int o = kTileMaxLog + 1; o <= kMaxOrder; ++o) {
        if (gin[o].empty()) continue;
        Group g;
        g.order = o;
        g.count = (int64_t)gin[o].size();
        if (p->ragged) {
            if (dev_malloc(&g.d_in_sig, sizeof(int64_t) * g.count) != hipSuccess ||
                dev_malloc(&g.d_out_sig, sizeof(int64_t) * g.count) != hipSuccess) {
                p->groups.push_back(g);
                return fail(MRDFT_E_ALLOC, "signal table allocation failed");
            }
            p->groups.push_back(g);
            HIP_TRY(hipMemcpyAsync(g.d_in_sig, gin[o].data(), sizeof(int64_t) * g.count, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(g.d_out_sig, gout[o].data(), sizeof(int64_t) * g.count, hipMemcpyHostToDevice, s));
        } else {
            p->groups.push_back(g);
        }
        const int64_t need = g.count << o;
        if (need > scratch) scratch = need;
    }
    const char* serial = std::getenv("MRDFT_SERIAL");        // 1: keep all levels on the caller's stream
    bool need_side = false;
    for (const Group& g : p->groups) need_side |= p->dtype != MRDFT_R32 || g.order > kRowsMaxLevel;
    if (need_side && !(serial && serial[0] == '1')) {
        // one side stream per level above the tile (up to kSides), default priority;
        // the real launch covers the levels up to 16
        int levels = 0;
        for (const Group& g : p->groups)
            levels = std::max(levels, g.order - (p->dtype == MRDFT_R32 ? kRowsMaxLevel : kTileMaxLog));
        HIP_TRY(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
        for (int k = 0; k < std::min(levels, (int)mrdft_plan::kSides); ++k) {
            HIP_TRY(hipStreamCreateWithFlags(&p->side[k], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&p->join_ev[k], hipEventDisableTiming));
            p->nsides = k + 1;
        }

    }
    if (scratch > 0) {
        // one ping-pong pair per side stream: chains of passes of different
        // levels run concurrently
        if (dev_malloc(&p->d_s[0], sizeof(float2) * scratch) != hipSuccess ||
            dev_malloc(&p->d_s[1], sizeof(float2) * scratch) != hipSuccess)
            return fail(MRDFT_E_ALLOC, "pass workspace allocation failed (2 x %lld complex)", (long long)scratch);
        for (int k = 1; k < p->nsides; ++k)
            if (dev_malloc(&p->d_ss[k - 1][0], sizeof(float2) * scratch) != hipSuccess ||
                dev_malloc(&p->d_ss[k - 1][1], sizeof(float2) * scratch) != hipSuccess)
                return fail(MRDFT_E_ALLOC, "pass workspace allocation failed (%d x 2 x %lld complex)", p->nsides,
                            (long long)scratch);
        p->scratch_pts = scratch;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return MRDFT_OK;
}

// Job tables of the one-launch forwards.  Workgroups of a launch are dealt
// to the 8 XCDs in block order (block b runs on XCD b mod 8), so all pieces of
// one window go to one bucket: launched one workgroup per job, they share the
// window's x columns through that XCD's L2.  Inside a bucket the order is
//   tiles first : tiles (store-bound, they keep HBM busy from the start), then
//                 the pieces from the highest level down (longest first, the
//                 short ones fill the tail);
//   rows first  : the pieces (highest level first), then the tiles;
//   interleaved : tiles and pieces alternate in proportion;
//   blocks      : every block of 2^16 samples (or the whole signal if shorter)
//                 goes whole to one bucket: the block's samples are read from
//                 HBM about once and then served by the XCD's L2.  Inside a
//                 block the pieces of its windows come before its tiles in
//                 the real forward and after them in the complex forward; the
//                 fused loss's norm and scaled launches alternate the two
//                 (for each the fastest of the three, with tile waves at
//                 raised priority).
struct JobBuckets {
    static constexpr int kX = 8;
    std::vector<std::vector<RealJob>> tiles = std::vector<std::vector<RealJob>>(kX);
    std::vector<std::vector<RealJob>> rows = std::vector<std::vector<RealJob>>(kX);
    std::vector<int64_t> load = std::vector<int64_t>(kX, 0);
    int lightest() const { return (int)(std::min_element(load.begin(), load.end()) - load.begin()); }
    void add_tile(const RealJob& jb, int64_t cost) {
        const int b = lightest();
        tiles[b].push_back(jb);
        load[b] += cost;
    }
    // all pieces of one window, into one bucket
    void add_window(const RealJob& first, int pieces) {
        const int b = lightest();
        for (int g = 0; g < pieces; ++g) {
            RealJob jb = first;
            jb.g = g;
            rows[b].push_back(jb);
        }
        load[b] += pieces;
    }
    // t and r alternate in proportion (r first on a tie)
    static void alternate(std::vector<RealJob>& out, const std::vector<RealJob>& t, const std::vector<RealJob>& r) {
        const size_t nt = t.size(), nr = r.size();
        size_t it = 0, ir = 0;
        while (it < nt || ir < nr) {
            if (ir < nr && (it >= nt || ir * nt <= it * nr)) out.push_back(r[ir++]);
            else out.push_back(t[it++]);
        }
    }
    std::vector<std::vector<RealJob>> blocks = std::vector<std::vector<RealJob>>(kX);
    // a block's tiles t and pieces r to the lightest bucket, in the order `in`
    void add_block(const std::vector<RealJob>& t, const std::vector<RealJob>& r, int64_t cost,
                   InBlock in = InBlock::kTilesFirst) {
        const int b = lightest();
        if (in == InBlock::kAlternate) {
            alternate(blocks[b], t, r);
        } else {
            const std::vector<RealJob>& a = in == InBlock::kPiecesFirst ? r : t;
            const std::vector<RealJob>& c = in == InBlock::kPiecesFirst ? t : r;
            blocks[b].insert(blocks[b].end(), a.begin(), a.end());
            blocks[b].insert(blocks[b].end(), c.begin(), c.end());
        }
        load[b] += cost;
    }
    // contiguous: the buckets one after the other, their starts in seg[0..8]
    // (persistent launch); otherwise interleaved so that block b falls in
    // bucket b mod 8 (one workgroup per job).
    std::vector<RealJob> deal(int order, std::vector<unsigned>* seg = nullptr) {
        std::vector<std::vector<RealJob>> bucket(kX);
        for (int b = 0; b < kX; ++b) {
            std::stable_sort(rows[b].begin(), rows[b].end(),
                             [](const RealJob& a, const RealJob& c) { return a.lg > c.lg; });
            if (order == MRDFT_ORDER_BLOCKS) {
                bucket[b] = blocks[b];
            } else if (order == MRDFT_ORDER_ROWS_FIRST) {
                bucket[b] = rows[b];
                bucket[b].insert(bucket[b].end(), tiles[b].begin(), tiles[b].end());
            } else if (order == MRDFT_ORDER_INTERLEAVED) {
                alternate(bucket[b], tiles[b], rows[b]);
            } else {
                bucket[b] = tiles[b];
                bucket[b].insert(bucket[b].end(), rows[b].begin(), rows[b].end());
            }
        }
        std::vector<RealJob> out;
        if (seg) {
            seg->assign(kX + 1, 0);
            for (int b = 0; b < kX; ++b) {
                (*seg)[b] = (unsigned)out.size();
                out.insert(out.end(), bucket[b].begin(), bucket[b].end());
            }
            (*seg)[kX] = (unsigned)out.size();
            return out;
        }
        for (size_t i = 0;; ++i) {
            bool any = false;
            for (int b = 0; b < kX; ++b)
                if (i < bucket[b].size()) {
                    out.push_back(bucket[b][i]);
                    any = true;
                }
            if (!any) break;
        }
        return out;
    }
};

// Blocks of jobs (tiles first), each whole to the least loaded of the 8
// buckets, interleaved so that bucket b runs on XCD b.
std::vector<RealJob> deal_blocks(const std::vector<JobBlock>& blocks) {
    JobBuckets jb;
    for (const JobBlock& b : blocks) jb.add_block(b.tiles, b.pieces, b.cost, InBlock::kTilesFirst);
    return jb.deal(MRDFT_ORDER_BLOCKS);
}

// Real signals of order >= 12: 4096-sample tiles and pieces of levels 13..16
// (2^(lg-13) pieces per window).
std::vector<RealJob> real_jobs(const mrdft_plan* p, int order, InBlock in) {
    JobBuckets jb;
    constexpr int64_t kTileCost = 6;                           // 12 x 32 KB against 64 KB per piece
    for (int64_t j = 0; j < p->batch; ++j) {
        const int mj = p->orders[j];
        if (mj < kRealTileLog) continue;
        const int64_t N = int64_t(1) << mj;
        const bool tiles = p->lo <= kRealTileLog;              // tiles keep a level
        const int plo = std::max(kRowsMinLevel, p->lo), phi = std::min({mj, kRowsMaxLevel, p->hi});
        auto tile = [&](int64_t tau) {
            return RealJob{p->in_off[j] + (tau << kRealTileLog), p->base(j) + ((tau << kRealTileLog) >> p->hs),
                           N >> p->hs, 0, p->range()};
        };
        auto window = [&](int lg, int64_t w) {                 // piece 0 of window w of level lg
            const int64_t L = int64_t(1) << lg;
            return RealJob{p->in_off[j] + w * L, p->base(j) + (((int64_t)(lg - 1) * N + w * L) >> p->hs), N, lg, 0};
        };
        if (order == MRDFT_ORDER_BLOCKS) {
            const int64_t U = int64_t(1) << std::min(mj, kRowsMaxLevel);   // holds whole windows of every piece level
            for (int64_t u0 = 0; u0 < N; u0 += U) {
                std::vector<RealJob> t, r;
                for (int64_t tau = u0 >> kRealTileLog; tiles && tau < (u0 + U) >> kRealTileLog; ++tau) t.push_back(tile(tau));
                // pieces from the highest level down (full spectra) or from
                // the lowest up (half spectra): the faster order for each
                for (int q = 0; q <= phi - plo; ++q) {
                    const int lg = p->hs ? plo + q : phi - q;
                    for (int64_t w = u0 >> lg; w < (u0 + U) >> lg; ++w)
                        for (int g = 0; g < (1 << (lg - kRowsMinLevel)); ++g) {
                            RealJob jb1 = window(lg, w);
                            jb1.g = g;
                            r.push_back(jb1);
                        }
                }
                jb.add_block(t, r, kTileCost * (int64_t)t.size() + (int64_t)r.size(), in);
            }
            continue;
        }
        for (int64_t tau = 0; tiles && tau < (N >> kRealTileLog); ++tau) jb.add_tile(tile(tau), kTileCost);
        for (int lg = plo; lg <= phi; ++lg)
            for (int64_t w = 0; w < (N >> lg); ++w) jb.add_window(window(lg, w), 1 << (lg - kRowsMinLevel));
    }
    return jb.deal(order);
}

// Real signals below 4096 samples (full-spectrum plans): the complex launch's
// 2048-sample tiles (order 11) and multi-signal tiles (orders below 11),
// reading real input; several short signals share one workgroup.
std::vector<RealJob> small_real_jobs(const mrdft_plan* p) {
    JobBuckets jb;
    for (int64_t j = 0; j < p->batch; ++j) {
        const int mj = p->orders[j];
        if (mj >= kRealTileLog || mj < p->lo) continue;    // the real launch / no level kept
        const int64_t N = int64_t(1) << mj;
        if (mj < kC64TileLog) {
            const int64_t per = int64_t(1) << (kC64TileLog - mj);
            int64_t n = 1;
            while (j + n < p->batch && p->orders[j + n] == mj && n < per) ++n;
            const int64_t vlen = n * N;
            jb.add_block({RealJob{p->in_off[j], p->base(j), N | (vlen << 32), kMultiTileLg + mj,
                                  LevelRange::pack(p->lo, std::min(p->hi, mj))}},
                         {}, 1);
            j += n - 1;
            continue;
        }
        jb.add_block({RealJob{p->in_off[j], p->base(j), N, 0, p->range()}}, {}, 1);
    }
    return jb.deal(MRDFT_ORDER_BLOCKS);
}

// Pieces per window of a complex level 12..16: one of 16 rows at level 12,
// 2^(lg-13) of 32 rows above.
int cpieces(int lg) { return lg == kCRowsMinLevel ? 1 : 1 << (lg - kCRowsMinLevel - 1); }

// Complex signals of order >= 11: 2048-sample tiles and pieces of levels
// 12..16 (cpieces per window).
std::vector<RealJob> complex_jobs(const mrdft_plan* p, int order, std::vector<unsigned>* seg) {
    JobBuckets jb;
    constexpr int64_t kTileCost = 5;                           // 11 x 16 KB against 32 KB per piece
    for (int64_t j = 0; j < p->batch; ++j) {
        const int mj = p->orders[j];
        if (mj < kC64TileLog) {
            // a run of consecutive signals of this order (x and outputs are
            // contiguous), 2^(11 - m) of them per tile; signals that keep no
            // level are skipped
            if (mj < p->lo) continue;
            const int64_t N = int64_t(1) << mj, per = int64_t(1) << (kC64TileLog - mj);
            int64_t n = 1;
            while (j + n < p->batch && p->orders[j + n] == mj && n < per) ++n;
            const int64_t vlen = n * N;
            const RealJob mt{p->in_off[j], p->base(j), N | (vlen << 32), kMultiTileLg + mj,
                             LevelRange::pack(p->lo, std::min(p->hi, mj))};
            if (order == MRDFT_ORDER_BLOCKS) jb.add_block({mt}, {}, kTileCost);
            else jb.add_tile(mt, kTileCost);
            j += n - 1;
            continue;
        }
        const int64_t N = int64_t(1) << mj;
        const bool tiles = p->lo <= kC64TileLog;               // tiles keep a level
        const int plo = std::max(kCRowsMinLevel, p->lo), phi = std::min({mj, kRowsMaxLevel, p->hi});
        auto tile = [&](int64_t tau) {
            return RealJob{p->in_off[j] + (tau << kC64TileLog), p->base(j) + (tau << kC64TileLog), N, 0, p->range()};
        };
        auto window = [&](int lg, int64_t w) {                 // piece 0 of window w of level lg
            const int64_t L = int64_t(1) << lg;
            return RealJob{p->in_off[j] + w * L, p->base(j) + (int64_t)(lg - 1) * N + w * L, 0, lg, 0};
        };
        if (order == MRDFT_ORDER_BLOCKS) {
            const int64_t U = int64_t(1) << std::min(mj, kRowsMaxLevel);
            for (int64_t u0 = 0; u0 < N; u0 += U) {
                std::vector<RealJob> t, r;
                for (int64_t tau = u0 >> kC64TileLog; tiles && tau < (u0 + U) >> kC64TileLog; ++tau) t.push_back(tile(tau));
                for (int lg = phi; lg >= plo; --lg)
                    for (int64_t w = u0 >> lg; w < (u0 + U) >> lg; ++w)
                        for (int g = 0; g < cpieces(lg); ++g) {
                            RealJob jb1 = window(lg, w);
                            jb1.g = g;
                            r.push_back(jb1);
                        }
                jb.add_block(t, r, kTileCost * (int64_t)t.size() + (int64_t)r.size());
            }
            continue;
        }
        for (int64_t tau = 0; tiles && tau < (N >> kC64TileLog); ++tau) jb.add_tile(tile(tau), kTileCost);
        for (int lg = plo; lg <= phi; ++lg)
            for (int64_t w = 0; w < (N >> lg); ++w) jb.add_window(window(lg, w), cpieces(lg));
    }
    return jb.deal(order, seg);
}

// Complex job table in per-XCD segments, with its segment starts.
mrdft_status upload_cjobs(mrdft_plan* p, int order, hipStream_t s, bool direct) {
    std::vector<unsigned> seg;
    mrdft_status st = upload_jobs(complex_jobs(p, order, direct ? nullptr : &seg), &p->d_cjobs, &p->ncjobs, s);
    if (st) return st;
    p->cjobs_direct = direct;
    if (direct) return MRDFT_OK;
    if (!p->d_cseg && dev_malloc(&p->d_cseg, sizeof(unsigned) * seg.size()) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "segment table allocation failed");
    HIP_TRY(hipMemcpyAsync(p->d_cseg, seg.data(), sizeof(unsigned) * seg.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MRDFT_OK;
}

// Upload a job table (replacing a previous one of the same slot).
mrdft_status upload_jobs(const std::vector<RealJob>& v, RealJob** dst, int64_t* n, hipStream_t s) {
    dfree(*dst);
    *dst = nullptr;
    *n = (int64_t)v.size();
    if (v.empty()) return MRDFT_OK;
    if (dev_malloc(dst, sizeof(RealJob) * v.size()) != hipSuccess)
        return fail(MRDFT_E_ALLOC, "job table allocation failed (%zu bytes)", sizeof(RealJob) * v.size());
    HIP_TRY(hipMemcpyAsync(*dst, v.data(), sizeof(RealJob) * v.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MRDFT_OK;
}

hipEvent_t take_event(mrdft_plan* p) {
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Scoped timing of one launch (no-op unless profiling is enabled).
struct ProfScope {
    mrdft_plan* p;
    hipStream_t s;
    int kind;
    hipEvent_t a = nullptr;
    ProfScope(mrdft_plan* p_, int kind_, hipStream_t s_) : p(p_), s(s_), kind(kind_) {
        if (p->profiling) {
            a = take_event(p);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = take_event(p);
            if (b) {
                (void)hipEventRecord(b, s);
                p->recs.push_back({kind, a, b});
            } else {
                p->event_pool.push_back(a);
            }
        }
    }
};

// Level i of a group launch: ragged signals address it through their base
// offsets (already shifted by -(lo-1) N), uniform ones as b * kept * N + (i - lo) N.
float2* level_ptr(const mrdft_plan* p, float2* Y, int i, int64_t N) {
    return Y + (int64_t)(p->ragged ? i - 1 : i - p->lo) * N;
}

// Forward transform of all levels of every signal (x of the plan dtype, or an
// explicit override of kind `in_kind`).
mrdft_status run_forward(mrdft_plan* p, const void* x, int in_kind, float2* Y, hipStream_t s0) {
    const Twiddles tw = p->tw();
    // Levels above the tile go to the side streams, which first wait for
    // everything already queued on the caller's stream: with the default
    // schedule they run beside the tile / one-launch kernel, with
    // MRDFT_SCHED_AFTER they start when it has finished (still concurrently
    // with each other), with MRDFT_SCHED_SERIAL everything runs in order on the
    // caller's stream.
    const int nsides = p->serial ? 0 : p->nsides;
    const bool real_jobs_cover = in_kind == IN_R32 && p->d_rjobs;
    const bool cjobs_cover = in_kind == IN_C64 && p->d_cjobs && p->tile_log == kC64TileLog;
    auto fork = [&]() -> mrdft_status {
        if (nsides) {
            HIP_TRY(hipEventRecord(p->fork_ev, s0));
            for (int k = 0; k < nsides; ++k) HIP_TRY(hipStreamWaitEvent(p->side[k], p->fork_ev, 0));
        }
        return MRDFT_OK;
    };
    // Signals of order kRecMinLevel - 1 (that level by a direct chain of two
    // passes) run it inside the shared head and tail launches of the first
    // longer group: their workgroups, shorter than the pairs', follow them and
    // fill the pair launches' last, partly filled round of workgroups.  Their
    // scratch follows the longer group's upper chain in ds[1].
    const Group* g_one = nullptr;                     // the order kRecMinLevel - 1 group
    const Group* g_two = nullptr;                     // the group whose head and tail take it along
    {
        const int l1 = kRecMinLevel - 1;
        if (!p->hs && l1 >= p->lo && l1 + 1 <= p->hi && pass_bits(l1).size() == 2)
            for (const Group& g : p->groups) {
                if (g.order == l1) g_one = &g;
                else if (g.order > l1 && !g_two) g_two = &g;
            }
        if (!g_one || !g_two ||
            (g_two->count << (g_two->order - 1)) + (g_one->count << l1) > p->scratch_pts)
            g_one = g_two = nullptr;
    }
    auto upper = [&]() -> mrdft_status {
    int chain = 0;                                    // multi-pass levels, dealt over the side streams
    for (const Group& g : p->groups) {
        const int64_t N = int64_t(1) << g.order;
        int kprev = 0;                                // stream of level i - 1
        bool head_done = false;                       // level kRecMinLevel's first pass ran with level i - 1's
        for (int i = kTileMaxLog + 1; i <= g.order; ++i) {
            if ((real_jobs_cover || cjobs_cover) && i <= kRowsMaxLevel) continue;     // in the one launch
            if (i < p->lo || i > p->hi) continue;                                      // level not kept
            if (&g == g_one && i == kRecMinLevel - 1) continue;                        // with g_two's head and tail
            // recurrence chain: level i - 1 is stored by this plan, by the
            // chain just before on the same stream
            const bool rec = i >= kRecMinLevel && i - 1 >= p->lo && !p->hs;
            // levels spread over the side streams; the passes of one level run
            // in order on one stream with that stream's scratch pair, and a
            // recurrence chain follows the level below on its stream
            const int si = (i <= kUpperMaxLevel) ? (i - kTileMaxLog - 1) : chain++;
            const int k = !nsides ? 0 : rec ? kprev : si % nsides;
            kprev = k;
            const hipStream_t s = nsides ? p->side[k] : s0;
            float2* const* ds = k == 0 ? p->d_s : p->d_ss[k - 1];
            if (i <= kUpperMaxLevel) {
                if (p->hs) return fail(MRDFT_E_UNSUPPORTED, "half-spectrum output of level %d without the real launch", i);
                PassGeom geo;
                geo.lg = i;
                geo.r_log = 0;
                geo.ns_log = 0;
                geo.nwin = g.count * (N >> i);
                geo.wps = N >> i;
                geo.in_sig = g.d_in_sig;
                geo.in_stride = N;
                geo.out_sig = g.d_out_sig;
                geo.out_stride = (int64_t)p->kept(g.order) * N;
                ProfScope ps(p, MRDFT_KERNEL_PASS_FWD, s);
                HIP_TRY(launch_upper_fwd(in_kind == IN_R32, x, level_ptr(p, Y, i, N), geo, tw, s));
                continue;
            }
            const int dl = rec ? i - 1 : i;            // order of the DFTs of the chain
            std::vector<int> bits = pass_bits(dl);
            const int64_t wlen = rec ? N / 2 : N;      // scratch points per signal
            // the chains of levels 17 and 18 (2^17-point DFTs) start with the
            // smaller radix: the shared head, three FFTs per workgroup, then runs
            // four 4096-point workgroups per CU, the shared tail two 8192-point
            // ones (the 1000-signal batch ~1.773 -> ~1.755 ms)
            if ((i == kRecMinLevel - 1 || i == kRecMinLevel) && bits.size() == 2) std::swap(bits[0], bits[1]);
            // level kRecMinLevel - 1 with the next level built from it: one
            // head for both chains (this level's scratch ds[0], the next's ds[1])
            const bool head2 = !rec && i + 1 == kRecMinLevel && i + 1 <= g.order && i + 1 <= p->hi && !p->hs &&
                               bits.size() == 2;
            const bool skip_head = rec && i == kRecMinLevel && head_done;
            // g_one's windows of level kRecMinLevel - 1 beside this group's pairs
            const bool with_one = &g == g_two && (head2 || skip_head);
            const int64_t N1 = g_one ? int64_t(1) << g_one->order : 0;
            float2* const s_one = with_one ? ds[1] + (g.count << (g.order - 1)) : nullptr;
            auto one_geo = [&](int r_log, int ns_log) {
                PassGeom o;
                o.lg = kRecMinLevel - 1;
                o.r_log = r_log;
                o.ns_log = ns_log;
                o.nwin = g_one->count * (N1 >> o.lg);
                o.wps = N1 >> o.lg;
                o.in_sig = g_one->d_in_sig;
                o.in_stride = N1;
                o.out_sig = g_one->d_out_sig;
                o.out_stride = (int64_t)p->kept(g_one->order) * N1;
                return o;
            };
            int ns = 0;
            for (size_t q = 0; q < bits.size(); ++q) {
                const bool first = q == 0, last = q + 1 == bits.size();
                if (first && head2) {
                    PassGeom geo;
                    geo.lg = i;
                    geo.r_log = bits[0];
                    geo.ns_log = 0;
                    geo.nwin = g.count * (N >> (i + 1));
                    geo.wps = N >> (i + 1);
                    geo.in_sig = g.d_in_sig;
                    geo.in_stride = N;
                    const PassGeom g1 = with_one ? one_geo(bits[0], 0) : geo;
                    ProfScope ps(p, MRDFT_KERNEL_PASS_FWD, s);
                    HIP_TRY(launch_pass_head2(in_kind, x, ds[0], ds[1], geo, s_one, with_one ? &g1 : nullptr, tw, s));
                    head_done = true;
                    ns += bits[q];
                    continue;
                }
                if (first && skip_head) {              // ran with the level below
                    ns += bits[q];
                    continue;
                }
                if (last && head2) continue;           // stored by the next level's tail
                if (last && skip_head && bits.size() == 2) {
                    // both levels' last passes: level i - 1's windows from
                    // ds[0], this level's odd bins from ds[1]
                    PassGeom geo;
                    geo.lg = dl;
                    geo.r_log = bits[q];
                    geo.ns_log = ns;
                    geo.nwin = g.count * (N >> i);
                    geo.wps = N >> i;
                    geo.out_sig = g.d_out_sig;
                    geo.out_stride = (int64_t)p->kept(g.order) * N;
                    const PassGeom g1 = with_one ? one_geo(bits[q], ns) : geo;
                    float2* const y_one = with_one ? level_ptr(p, Y, kRecMinLevel - 1, N1) : nullptr;
                    ProfScope ps(p, MRDFT_KERNEL_PASS_FWD, s);
                    HIP_TRY(launch_pass_tail2(ds[0], ds[1], level_ptr(p, Y, i - 1, N), level_ptr(p, Y, i, N), geo, s_one,
                                              y_one, with_one ? &g1 : nullptr, tw, s));
                    ns += bits[q];
                    continue;
                }
                PassGeom geo;
                geo.lg = dl;
                geo.r_log = bits[q];
                geo.ns_log = ns;
                geo.nwin = g.count * (N >> i);
                geo.wps = N >> i;
                geo.in_sig = first ? g.d_in_sig : nullptr;
                geo.in_stride = first ? N : wlen;
                geo.out_sig = last ? g.d_out_sig : nullptr;
                geo.out_stride = last ? (int64_t)p->kept(g.order) * (N >> p->hs) : wlen;
                geo.rec_prev = (rec && last) ? N : 0;
                const void* in = first ? x : (const void*)ds[((q - 1) & 1) ^ (skip_head ? 1 : 0)];
                void* out = last ? (void*)level_ptr(p, Y, i, N >> p->hs) : (void*)ds[q & 1];
                const int ik = !first ? IN_C64 : !rec ? in_kind : in_kind == IN_R32 ? IN_DIFF_R32 : IN_DIFF;
                const int ok = (last && p->hs) ? OUT_HALF : (last && rec) ? OUT_REC : OUT_STORE;
                ProfScope ps(p, MRDFT_KERNEL_PASS_FWD, s);
                HIP_TRY(launch_pass(false, ik, ok, in, out, geo, tw, s));
                ns += bits[q];
            }
        }
    }
    return MRDFT_OK;
    };
    auto main_launch = [&]() -> mrdft_status {
        if (real_jobs_cover) {
            {
                ProfScope ps(p, MRDFT_KERNEL_FUSED_FWD, s0);
                HIP_TRY(launch_fwd_real((const float*)x, Y, p->d_rjobs, p->nrjobs, tw, s0, p->hs != 0));
            }
            if (p->nsjobs) {                          // signals below 4096 samples
                ProfScope ps(p, MRDFT_KERNEL_TILE_FWD, s0);
                HIP_TRY(launch_fwd_c64_direct(x, Y, p->d_sjobs, p->nsjobs, tw, s0, true));
            } else if (p->njobs > p->njobs_full) {
                ProfScope ps(p, MRDFT_KERNEL_TILE_FWD, s0);
                HIP_TRY(launch_tile_fwd(true, x, Y, p->d_jobs + p->njobs_full, p->njobs - p->njobs_full, p->tail_tmax, tw, s0,
                                        p->hs != 0));
            }
        } else if (in_kind == IN_R32) {
            ProfScope ps(p, MRDFT_KERNEL_TILE_FWD, s0);
            if (p->nsjobs) HIP_TRY(launch_fwd_c64_direct(x, Y, p->d_sjobs, p->nsjobs, tw, s0, true));
            else HIP_TRY(launch_tile_fwd(true, x, Y, p->d_jobs, p->njobs, p->jobs_tmax, tw, s0, p->hs != 0));
        } else if (cjobs_cover) {
            {
                ProfScope ps(p, MRDFT_KERNEL_FUSED_FWD, s0);
                if (p->grid == 0)
                    HIP_TRY(launch_fwd_c64_direct((const float2*)x, Y, p->d_cjobs, p->ncjobs, tw, s0));
                else
                    HIP_TRY(launch_fwd_c64((const float2*)x, Y, p->d_cjobs, p->ncjobs, p->d_cseg, p->d_queue, p->grid,
                                           tw, s0));
            }
        } else {
            ProfScope ps(p, MRDFT_KERNEL_TILE_FWD, s0);
            HIP_TRY(launch_tile_fwd(false, x, Y, p->d_jobs, p->njobs, p->jobs_tmax, tw, s0));
        }
        return MRDFT_OK;
    };
    mrdft_status st = MRDFT_OK;
    if (p->after) {
        st = main_launch();
        if (!st) st = fork();
        if (!st) st = upper();
    } else {
        st = fork();
        if (!st) st = upper();
        if (!st) st = main_launch();
    }
    if (st) return st;
    for (int k = 0; k < nsides; ++k) {
        HIP_TRY(hipEventRecord(p->join_ev[k], p->side[k]));
        HIP_TRY(hipStreamWaitEvent(s0, p->join_ev[k], 0));
    }
    return MRDFT_OK;
}

// packed_from_full: gY holds packed half spectra of a full-spectrum (real,
// uniform) plan's levels, read with the plan's full-layout tables halved
// (the spectral-loss gradient).
// Passes q0 .. q1-1 of the adjoint chain of level i of group g on stream s
// with the ping-pong scratch ds: the first pass reads the level's gradient
// (packed for half plans), the last adds its result into gx.
mrdft_status adj_chain(mrdft_plan* p, const Group& g, int i, const float2* gY, void* gx, bool real_out, int half,
                       bool packed_from_full, size_t q0, size_t q1, float2* const* ds, hipStream_t s) {
    const Twiddles tw = p->tw();
    const int64_t N = int64_t(1) << g.order;
    const std::vector<int> bits = pass_bits(i);
    // real output from packed (Hermitian) gradients: the windows go through
    // the chain in pairs, h1 + i h2, so half the transforms run
    const bool pair = real_out && half;
    const int64_t nwin = g.count * (N >> i);
    int ns = 0;
    for (size_t q = 0; q < q0; ++q) ns += bits[q];
    for (size_t q = q0; q < q1; ++q) {
        const bool first = q == 0, last = q + 1 == bits.size();
        PassGeom geo;
        geo.lg = i;
        geo.r_log = bits[q];
        geo.ns_log = ns;
        geo.nwin = pair ? (nwin + 1) / 2 : nwin;
        geo.pair_nwin = pair && (first || last) ? nwin : 0;
        geo.wps = N >> i;
        geo.in_sig = first ? g.d_out_sig : nullptr;
        geo.in_stride = first ? (int64_t)p->kept(g.order) * (N >> half) : N;
        geo.out_sig = last ? g.d_in_sig : nullptr;
        geo.out_stride = N;
        geo.half_scale = packed_from_full ? 1.0f : 0.5f;
        const void* in = first ? (const void*)level_ptr(p, (float2*)gY, i, N >> half) : (const void*)ds[(q - 1) & 1];
        void* out = last ? gx : (void*)ds[q & 1];
        const int ok = !last ? OUT_STORE : pair ? OUT_ADD_R32_PAIR : real_out ? OUT_ADD_R32 : OUT_ADD_C64;
        const int ik = !(first && half) ? IN_C64 : pair ? IN_HALF_PAIR : IN_HALF;
        ProfScope ps(p, MRDFT_KERNEL_PASS_ADJ, s);
        HIP_TRY(launch_pass(true, ik, ok, in, out, geo, tw, s));
        ns += bits[q];
    }
    return MRDFT_OK;
}

mrdft_status run_adjoint(mrdft_plan* p, const float2* gY, void* gx, bool real_out, hipStream_t s,
                         bool packed_from_full = false) {
    const Twiddles tw = p->tw();
    const int half = (p->hs || packed_from_full) ? 1 : 0;
    if (packed_from_full && (p->hs || p->ragged || !real_out || p->nasmall))
        return fail(MRDFT_E_UNSUPPORTED, "packed gradient of a full-spectrum plan: uniform real plans of order >= 11 only");
    // the job tables of a real plan hold Hermitian pieces: real output only
    if (real_out != (p->dtype == MRDFT_R32)) return fail(MRDFT_E_UNSUPPORTED, "adjoint output type differs from the plan's");
    // Levels above 16 run as chains of global passes whose last pass adds into
    // gx.  With a side stream per chain, every pass but the last runs on the
    // chain's side stream (with its own scratch) beside the tile and column
    // launches below; the last passes follow those launches on s, one chain
    // after another, so the additions into gx never overlap.
    std::vector<std::pair<const Group*, int>> chains;
    for (const Group& g : p->groups)
        for (int i = kRowsMaxLevel + 1; i <= g.order; ++i)
            if (i >= p->lo && i <= p->hi) chains.push_back({&g, i});
    const bool par = !chains.empty() && (int)chains.size() <= p->nsides;
    auto scratch_of = [&](size_t c) -> float2* const* { return !par || c == 0 ? p->d_s : p->d_ss[c - 1]; };
    if (par) {
        HIP_TRY(hipEventRecord(p->fork_ev, s));
        for (size_t c = 0; c < chains.size(); ++c) {
            const hipStream_t sk = p->side[c];
            HIP_TRY(hipStreamWaitEvent(sk, p->fork_ev, 0));
            const size_t nb = pass_bits(chains[c].second).size();
            mrdft_status st = adj_chain(p, *chains[c].first, chains[c].second, gY, gx, real_out, half, packed_from_full,
                                        0, nb - 1, scratch_of(c), sk);
            if (st) return st;
            HIP_TRY(hipEventRecord(p->join_ev[c], sk));
        }
    }
    if (p->hs && p->nhjobs) {
        // signals below the tile: packed gradient -> full-spectrum layout
        ProfScope ps(p, MRDFT_KERNEL_TILE_ADJ, s);
        HIP_TRY(launch_expand_half(gY, p->d_gfull, p->d_hjobs, p->nhjobs, s));
    }
    if (p->adj_zero) {
        ProfScope ps(p, MRDFT_KERNEL_TILE_ADJ, s);
        HIP_TRY(launch_zero(gx, p->n_in * (int64_t)(real_out ? sizeof(float) : sizeof(float2)), s));
    }
    if (p->najobs) {
        ProfScope ps(p, MRDFT_KERNEL_TILE_ADJ, s);
        // a half plan's packed gradient is read as its Hermitian extension
        // halved, packed spectra of real signals (the loss) whole
        HIP_TRY(launch_adj_a(real_out, half != 0, packed_from_full ? 1 : 0, packed_from_full ? 1.0f : 0.5f, gY, gx,
                             p->d_ascratch, p->d_ajobs, p->najobs, tw, s));
    }
    if (p->nasmall) {
        ProfScope ps(p, MRDFT_KERNEL_TILE_ADJ, s);
        HIP_TRY(launch_tile_adj(real_out, p->hs ? p->d_gfull : gY, gx, p->d_asmall, p->nasmall, p->asmall_tmax, tw, s));
    }
    if (p->nacols) {
        ProfScope ps(p, MRDFT_KERNEL_PASS_ADJ, s);
        HIP_TRY(launch_adj_b(real_out, gx, p->d_ascratch, p->d_acols, p->nacols, tw, s));
    }
    for (size_t c = 0; c < chains.size(); ++c) {
        const size_t nb = pass_bits(chains[c].second).size();
        if (par) HIP_TRY(hipStreamWaitEvent(s, p->join_ev[c], 0));
        mrdft_status st = adj_chain(p, *chains[c].first, chains[c].second, gY, gx, real_out, half, packed_from_full,
                                    par ? nb - 1 : 0, nb, scratch_of(c), s);
        if (st) return st;
    }
    return MRDFT_OK;
}

// Levels above 16 of a uniform plan through the global passes, written to
// W[b][i - 17][n] (compact) or to the plan's output layout W[b][i - 1][n]
// (half: as packed half spectra, N/2 values per level); with `norms`, nothing
// is written and the squared magnitudes of signal b's level i are added to
// norms[b * m + i - 1].  scr: the ping-pong scratch of the stream s (default:
// the plan's own); only: that one level (0: every level).
mrdft_status upper_passes(mrdft_plan* p, const float* x, float2* W, hipStream_t s, bool full_layout = false,
                          double* norms = nullptr, bool half = false, float2* const* scr = nullptr,
                          int only = 0, const float* out_scale = nullptr) {
    float2* const* ds = scr ? scr : p->d_s;           // ping-pong scratch of the stream s
    const Twiddles tw = p->tw();
    const int64_t N = int64_t(1) << p->m;
    const int top = p->m - kRowsMaxLevel;
    for (const Group& g : p->groups) {
        for (int i = kRowsMaxLevel + 1; i <= g.order; ++i) {
            if (i < p->lo || i > p->hi) continue;                                      // level not kept
            if (only && i != only) continue;                                           // one level asked for
            const std::vector<int> bits = pass_bits(i);
            // norms of a level with an even number of windows per signal: the
            // windows go through the chain in pairs, x1 + i x2
            const bool pair = norms && ((N >> i) & 1) == 0;
            const int64_t nwin = g.count * (N >> i);
            int ns = 0;
            for (size_t q = 0; q < bits.size(); ++q) {
                const bool first = q == 0, last = q + 1 == bits.size();
                PassGeom geo;
                geo.lg = i;
                geo.r_log = bits[q];
                geo.ns_log = ns;
                geo.nwin = pair ? nwin / 2 : nwin;
                geo.pair_nwin = pair && (first || last) ? nwin : 0;
                geo.wps = N >> i;
                geo.in_sig = nullptr;
                geo.in_stride = N;
                geo.out_sig = nullptr;
                geo.out_stride = last ? (int64_t)(full_layout ? p->m : top) * (N >> (half ? 1 : 0)) : N;
                const int slot = full_layout ? i - 1 : i - kRowsMaxLevel - 1;
                const void* in = first ? (const void*)x : (const void*)ds[(q - 1) & 1];
                void* out = (void*)ds[q & 1];
                int ok = OUT_STORE;
                if (last && norms) {
                    out = norms;
                    geo.out_stride = p->m;
                    ok = OUT_NORM;
                } else if (last) {
                    out = (void*)(W + (int64_t)slot * (N >> (half ? 1 : 0)));
                    if (half) {
                        ok = OUT_HALF;
                        geo.out_scale = out_scale;              // uniform batches only (one group)
                        geo.out_scale_m = p->m;
                    }
                }
                ProfScope ps(p, MRDFT_KERNEL_PASS_FWD, s);
                HIP_TRY(launch_pass(false, !first ? IN_C64 : pair ? IN_R32_PAIR : IN_R32, ok, in, out, geo, tw, s));
                ns += bits[q];
            }
        }
    }
    return MRDFT_OK;
}

// Time one candidate schedule: forward on scratch buffers, median of 3.
mrdft_status time_forward(mrdft_plan* p, const void* x, float2* Y, hipStream_t s, float* ms_out) {
    const int in_kind = p->dtype == MRDFT_R32 ? IN_R32 : IN_C64;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best[3];
    mrdft_status st = run_forward(p, x, in_kind, Y, s);          // warm-up
    for (int r = 0; r < 3 && st == MRDFT_OK; ++r) {
        HIP_TRY(hipEventRecord(a, s));
        st = run_forward(p, x, in_kind, Y, s);
        HIP_TRY(hipEventRecord(b, s));
        HIP_TRY(hipEventSynchronize(b));
        HIP_TRY(hipEventElapsedTime(&best[r], a, b));
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st) return st;
    std::sort(best, best + 3);
    *ms_out = best[1];
    return MRDFT_OK;
}

// Autotuner: time the candidate schedules on zero-filled scratch buffers and
// keep the fastest.  Complex plans: tile depth 12 (tile kernel, one launch per
// upper level) or 11 (one launch: one workgroup per job, or persistent with 1,
// 2 or 4 workgroups per CU) with each job order; real plans: the job order.
mrdft_status tune(mrdft_plan* p, hipStream_t s) {
    const bool real = p->dtype == MRDFT_R32;
    if (real ? p->nrjobs == 0 : p->ncjobs == 0) return MRDFT_OK;
    void* x = nullptr;
    float2* Y = nullptr;
    const size_t xbytes = (size_t)p->n_in * (real ? sizeof(float) : sizeof(float2));
    if (dev_malloc(&x, xbytes) != hipSuccess || dev_malloc(&Y, sizeof(float2) * (size_t)p->n_out) != hipSuccess) {
        dfree(x);
        return fail(MRDFT_E_ALLOC, "tuning buffers allocation failed");
    }
    mrdft_status st = MRDFT_OK;
    if (hipMemsetAsync(x, 0, xbytes, s) != hipSuccess) st = fail(MRDFT_E_HIP, "tuning buffer clear failed");
    struct Cand {
        int tile_log, order, grid;
    };
    std::vector<Cand> cands;
    for (int order = 0; order <= MRDFT_ORDER_BLOCKS; ++order) {
        if (real) {
            cands.push_back({kRealTileLog, order, 0});
        } else {
            cands.push_back({kC64TileLog, order, 0});
            for (int per = 1; per <= 4; per *= 2)
                cands.push_back({kC64TileLog, order, (int)std::min<int64_t>(p->ncjobs, (int64_t)per * p->num_cu)});
        }
    }
    if (!real) cands.push_back({kTileMaxLog, MRDFT_ORDER_TILES_FIRST, 0});
    float best_ms = 1e30f;
    Cand best = {p->tile_log, p->order, p->grid};
    int cur_order = p->order;
    for (const Cand& c : cands) {
        if (st) break;
        if (c.tile_log != kTileMaxLog && (c.order != cur_order || (!real && (c.grid == 0) != p->cjobs_direct))) {
            st = real ? upload_jobs(real_jobs(p, c.order), &p->d_rjobs, &p->nrjobs, s)
                      : upload_cjobs(p, c.order, s, c.grid == 0);
            cur_order = c.order;
            if (st) break;
        }
        p->tile_log = c.tile_log;
        p->grid = c.grid;
        float ms = 0.0f;
        st = time_forward(p, x, Y, s, &ms);
        if (!st && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    if (!st && best.tile_log != kTileMaxLog &&
        (best.order != cur_order || (!real && (best.grid == 0) != p->cjobs_direct)))
        st = real ? upload_jobs(real_jobs(p, best.order), &p->d_rjobs, &p->nrjobs, s)
                  : upload_cjobs(p, best.order, s, best.grid == 0);
    p->tile_log = best.tile_log;
    p->order = best.tile_log == kTileMaxLog && !real ? cur_order : best.order;
    p->grid = best.grid;
    // the winner once more with every launch on the caller's stream: pass
    // chains beside the one-launch kernel share the GPU with it, which can
    // cost more than it overlaps
    if (!st && p->nsides > 0) {
        p->after = true;
        float ms = 0.0f;
        st = time_forward(p, x, Y, s, &ms);
        if (!st && ms < best_ms) best_ms = ms;
        else p->after = false;
        const bool keep_after = p->after;
        p->after = false;
        p->serial = true;
        if (!st) st = time_forward(p, x, Y, s, &ms);
        if (st || !(ms < best_ms)) {
            p->serial = false;
            p->after = keep_after;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess && !st) st = fail(MRDFT_E_HIP, "tuning failed");
    dfree(x);
    dfree(Y);
    return st;
}

// Pin a forward schedule (validated; job tables re-uploaded when needed; a
// captured graph is dropped).
mrdft_status apply_schedule(mrdft_plan* plan, int tile_log, int grid, int order, bool serial, bool after,
                            hipStream_t stream) {
    const bool real = plan->dtype == MRDFT_R32;
    if (order < MRDFT_ORDER_TILES_FIRST || order > MRDFT_ORDER_BLOCKS)
        return fail(MRDFT_E_INVALID_ARG, "unknown job order %d", order);
    if (real ? tile_log != kRealTileLog : (tile_log != kC64TileLog && tile_log != kTileMaxLog))
        return fail(MRDFT_E_INVALID_ARG, "tile_log %d is not available for this plan", tile_log);
    if (!real && tile_log == kC64TileLog && grid < 0) return fail(MRDFT_E_INVALID_ARG, "grid must be >= 0");
    const bool direct = !real && tile_log == kC64TileLog && grid == 0;
    if (order != plan->order || (!real && plan->ncjobs > 0 && direct != plan->cjobs_direct)) {
        mrdft_status st = real ? upload_jobs(real_jobs(plan, order), &plan->d_rjobs, &plan->nrjobs, stream)
                               : upload_cjobs(plan, order, stream, direct);
        if (st) return st;
        plan->order = order;
    }
    if (!real) {
        plan->tile_log = plan->ncjobs > 0 ? tile_log : kTileMaxLog;
        plan->grid = grid;
    }
    plan->serial = serial;
    plan->after = after && !serial;
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->gexec = nullptr;
    plan->graph = nullptr;
    return MRDFT_OK;
}

// Key of a plan in the tuning cache: device architecture, input type, output
// form, level range and the exact batch shape (orders and their counts).
std::string tune_key(const mrdft_plan* p) {
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char& c : arch)
            if (c == '"' || c == '\\' || (unsigned char)c < 0x20) c = '_';
    }
    std::string k = arch + (p->dtype == MRDFT_R32 ? "|r32" : "|c64") + (p->hs ? "|half" : "|full") + "|levels" +
                    std::to_string(p->lo) + "-" + std::to_string(std::min(p->hi, p->max_order)) +
                    (p->ragged ? "|ragged" : "|uniform");
    int64_t count[kMaxOrder + 1] = {};
    for (int o : p->orders) ++count[o];
    for (int o = 1; o <= kMaxOrder; ++o)
        if (count[o]) k += "|" + std::to_string(count[o]) + "x2^" + std::to_string(o);
    return k;
}

// Integer value of an environment variable (def if unset; -1 if not a number).
int env_int(const char* name, int def) {
    const char* v = std::getenv(name);
    if (!v || !*v) return def;
    char* end = nullptr;
    const long r = std::strtol(v, &end, 10);
    if (*end || r < 0 || r > 1000000) return -1;
    return (int)r;
}

// Tuning at plan creation: MRDFT_TUNE (0/1) overrides the flag; with
// MRDFT_TUNE_CACHE set, a cached schedule is applied without timing and a
// fresh result is stored.  MRDFT_TILE_T then pins the tile depth.
mrdft_status tune_with_cache(mrdft_plan* p, hipStream_t s) {
    const int env_tune = env_int("MRDFT_TUNE", -2);
    if (env_tune == -1 || env_tune > 1) return fail(MRDFT_E_INVALID_ARG, "MRDFT_TUNE must be 0 or 1");
    const bool want = env_tune == -2 ? (p->flags & MRDFT_FLAG_TUNE) != 0 : env_tune == 1;
    mrdft_status st = MRDFT_OK;
    if (want) {
        const char* path = std::getenv("MRDFT_TUNE_CACHE");
        const std::string key = tune_key(p);
        int t = 0, g = 0, o = 0, se = 0;
        bool hit = false;
        if (path && *path && mrdft_tune_cache_lookup(path, key.c_str(), &t, &g, &o, &se) == 1) {
            const bool sides = p->nsides > 0;
            hit = apply_schedule(p, t, g, o, se == 1 && sides, se == 2 && sides, s) == MRDFT_OK;   // an unusable entry is re-tuned
        }
        if (!hit) {
            st = tune(p, s);
            if (!st && path && *path) {
                // a cache that cannot be written does not fail the plan
                (void)mrdft_tune_cache_store(path, key.c_str(), p->tile_log, p->grid, p->order,
                                             p->serial ? 1 : (p->after ? 2 : 0));
            }
        }
    }
    if (st) return st;
    const int tt = env_int("MRDFT_TILE_T", 0);
    if (tt != 0) {
        if (tt < 0) return fail(MRDFT_E_INVALID_ARG, "MRDFT_TILE_T must be a tile depth (11 or 12)");
        st = apply_schedule(p, tt, p->dtype == MRDFT_R32 ? 0 : p->grid, p->order, p->serial, p->after, s);
        if (st) return fail(st, "MRDFT_TILE_T=%d: %s", tt, g_last_error.c_str());
    }
    return MRDFT_OK;
}

// Graph replay of the forward: capture once per (x, Y) pair on the plan's own
// stream, then launch the instantiated graph on the caller's stream.
mrdft_status graph_forward(mrdft_plan* p, const void* x, float2* Y, hipStream_t stream) {
    const int in_kind = p->dtype == MRDFT_R32 ? IN_R32 : IN_C64;
    if (!p->gexec || p->gkey_x != x || p->gkey_y != (void*)Y) {
        if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
        // capturing records work without running it; the replay on the
        // caller's stream is ordered after what the caller queued before
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
        mrdft_status st = run_forward(p, x, in_kind, Y, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(MRDFT_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        p->graph = g;
        HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
        p->gkey_x = x;
        p->gkey_y = Y;
    }
    HIP_TRY(hipGraphLaunch(p->gexec, stream));
    return MRDFT_OK;
}

bool misaligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) & (a - 1)) != 0; }

mrdft_status check_plan(mrdft_plan_t plan) {
    if (!plan) return fail(MRDFT_E_INVALID_ARG, "plan is NULL");
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!g_plans.count(plan)) return fail(MRDFT_E_INVALID_ARG, "plan handle is not live (destroyed or invalid)");
    return MRDFT_OK;
}

mrdft_status ensure_loss_workspace(mrdft_plan* p, hipStream_t s) {
    // The fused path (one-launch real forward) keeps its own job table (the
    // forward's jobs, block-major with tiles and pieces alternating inside a
    // block: the faster order for its norm and scaled launches), the level
    // sums, the gradient factors, x - z and the packed half spectra of x - z;
    // the generic path the full spectra of x - z and of z and per-chunk sums.
    const bool fused = p->d_rjobs != nullptr;
    if (fused && !p->d_ljobs) {
        mrdft_status st = upload_jobs(real_jobs(p, MRDFT_ORDER_BLOCKS, InBlock::kAlternate), &p->d_ljobs, &p->nljobs, s);
        if (st) return st;
    }
    if (p->d_Yv) return MRDFT_OK;
    const int64_t rows = p->batch * p->m;
    const int64_t N = int64_t(1) << p->m;
    const int nch = loss_chunks(N);
    bool ok = dev_malloc(&p->d_sums, sizeof(double) * 2 * rows) == hipSuccess &&
              dev_malloc(&p->d_alpha, sizeof(float) * rows) == hipSuccess &&
              dev_malloc(&p->d_v, sizeof(float) * p->n_in) == hipSuccess &&
              dev_malloc(&p->d_Yv, sizeof(float2) * (fused ? p->n_out / 2 : p->n_out)) == hipSuccess;
    if (ok && !fused)
        ok = dev_malloc(&p->d_Yz, sizeof(float2) * p->n_out) == hipSuccess &&
             dev_malloc(&p->d_part, sizeof(double) * 2 * rows * nch) == hipSuccess;
    if (!ok) {
        // all or nothing: a failed first call leaves the plan as it was
        dfree(p->d_ljobs);
        p->d_ljobs = nullptr;
        p->nljobs = 0;
        dfree(p->d_sums);
        dfree(p->d_alpha);
        dfree(p->d_v);
        dfree(p->d_Yv);
        dfree(p->d_Yz);
        dfree(p->d_part);
        p->d_sums = nullptr;
        p->d_alpha = nullptr;
        p->d_v = nullptr;
        p->d_Yv = p->d_Yz = nullptr;
        p->d_part = nullptr;
        return fail(MRDFT_E_ALLOC, "spectral-loss workspace allocation failed");
    }
    return MRDFT_OK;
}

}  // namespace

namespace mrdft {
// Error reporting for the other host files of the library (thread-local
// message returned by mrdft_last_error).
mrdft_status report_error(mrdft_status st, const char* msg) { return fail(st, "%s", msg); }

namespace {
std::atomic<int64_t> g_live_allocs{0};
thread_local int g_scope_depth = 0;
thread_local int64_t g_scope_allocs = 0;
thread_local int64_t g_fail_at = 0;         // 0: no injected failure
}  // namespace

AllocScope::AllocScope() {
    if (g_scope_depth++ == 0) {
        g_scope_allocs = 0;
        const char* v = std::getenv("MRDFT_FAIL_ALLOC_AT");
        g_fail_at = (v && *v) ? std::strtoll(v, nullptr, 10) : 0;
    }
}

AllocScope::~AllocScope() {
    if (--g_scope_depth == 0) g_fail_at = 0;
}

hipError_t dev_malloc_raw(void** ptr, size_t bytes) {
    *ptr = nullptr;
    ++g_scope_allocs;
    if (g_scope_depth > 0 && g_fail_at > 0 && g_scope_allocs == g_fail_at) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e == hipSuccess) g_live_allocs.fetch_add(1);
    else *ptr = nullptr;
    return e;
}

void dev_free(void* ptr) {
    if (!ptr) return;
    (void)hipFree(ptr);
    g_live_allocs.fetch_sub(1);
}
}  // namespace mrdft

namespace {

// Workspace of mrdft_spectral_loss_fwd_noalloc: the per-level (num, den)
// sums, FP64.  One copy per device, held until the process ends.
constexpr int64_t kNoallocMaxSums = int64_t(1) << 16;             // 512 KiB of doubles
static __device__ __align__(256) double scratch[kNoallocMaxSums];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;                                // device address per device (null: not yet)

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address).
mrdft_status scratch_address(double** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MRDFT_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MRDFT_OK;
}

}  // namespace

extern "C" {

const char* mrdft_last_error(void) { return g_last_error.c_str(); }

int64_t mrdft_live_device_allocations(void) { return g_live_allocs.load(); }

mrdft_status mrdft_plan_create(mrdft_plan_t* plan, int m, int64_t batch, const int64_t* offsets, mrdft_dtype dtype,
                               unsigned flags, hipStream_t stream) {
    return mrdft_plan_create_levels(plan, m, batch, offsets, dtype, flags, 1, MRDFT_MAX_ORDER, stream);
}

mrdft_status mrdft_plan_create_levels(mrdft_plan_t* plan, int m, int64_t batch, const int64_t* offsets,
                                      mrdft_dtype dtype, unsigned flags, int lo, int hi, hipStream_t stream) {
    if (!plan) return fail(MRDFT_E_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    AllocScope alloc_scope;
    if (lo < 1 || hi < lo || hi > MRDFT_MAX_ORDER)
        return fail(MRDFT_E_INVALID_ARG, "level range [%d, %d] must satisfy 1 <= lo <= hi <= %d", lo, hi,
                    MRDFT_MAX_ORDER);
    if (!offsets && m >= 1 && lo > m)
        return fail(MRDFT_E_INVALID_ARG, "level range starts at %d above the order %d", lo, m);
    if (batch < 1) return fail(MRDFT_E_INVALID_ARG, "batch must be >= 1 (got %lld)", (long long)batch);
    if (dtype != MRDFT_C64 && dtype != MRDFT_R32) return fail(MRDFT_E_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (flags & ~(MRDFT_FLAG_TUNE | MRDFT_FLAG_GRAPH | MRDFT_FLAG_HALF))
        return fail(MRDFT_E_INVALID_ARG, "unknown flags 0x%x", flags);
    if ((flags & MRDFT_FLAG_HALF) && dtype != MRDFT_R32)
        return fail(MRDFT_E_INVALID_ARG, "half-spectrum output (MRDFT_FLAG_HALF) needs real (MRDFT_R32) input");
    mrdft_plan* p = new (std::nothrow) mrdft_plan();
    if (!p) return fail(MRDFT_E_ALLOC, "host allocation failed");
    p->batch = batch;
    p->dtype = dtype;
    p->flags = flags;
    p->lo = lo;
    p->hi = hi;
    p->hs = (flags & MRDFT_FLAG_HALF) ? 1 : 0;
    p->in_off.resize(batch + 1);
    p->out_off.resize(batch + 1);
    p->fout_off.resize(batch + 1);
    p->orders.resize(batch);
    if (offsets) {
        if (m != 0) {
            delete p;
            return fail(MRDFT_E_INVALID_ARG, "m must be 0 for a ragged plan (got %d)", m);
        }
        if (offsets[0] != 0) {
            delete p;
            return fail(MRDFT_E_INVALID_ARG, "offsets[0] must be 0 (got %lld)", (long long)offsets[0]);
        }
        p->ragged = true;
        for (int64_t j = 0; j < batch; ++j) {
            const int64_t len = offsets[j + 1] - offsets[j];
            const int o = ilog2_exact(len);
            if (o < 1 || o > MRDFT_MAX_ORDER) {
                delete p;
                return fail(MRDFT_E_INVALID_ARG,
                            "signal %lld has length %lld: lengths must be 2^m with 1 <= m <= %d",
                            (long long)j, (long long)len, MRDFT_MAX_ORDER);
            }
            p->orders[j] = o;
        }
    } else {
        if (m < 1 || m > MRDFT_MAX_ORDER) {
            delete p;
            return fail(MRDFT_E_INVALID_ARG, "m must be in [1, %d] (got %d)", MRDFT_MAX_ORDER, m);
        }
        for (int64_t j = 0; j < batch; ++j) p->orders[j] = m;
    }
    for (int64_t j = 0; j < batch && p->hs; ++j) {
        if (p->orders[j] < 2) {
            delete p;
            return fail(MRDFT_E_INVALID_ARG, "half-spectrum output needs signals of at least 4 samples (signal %lld)",
                        (long long)j);
        }
    }
    p->in_off[0] = p->out_off[0] = p->fout_off[0] = 0;
    for (int64_t j = 0; j < batch; ++j) {
        const int64_t N = int64_t(1) << p->orders[j];
        p->in_off[j + 1] = p->in_off[j] + N;
        p->out_off[j + 1] = p->out_off[j] + (int64_t)p->kept(p->orders[j]) * (N >> p->hs);
        p->fout_off[j + 1] = p->fout_off[j] + (int64_t)p->kept(p->orders[j]) * N;
        if (p->orders[j] > p->max_order) p->max_order = p->orders[j];
    }
    p->n_fout = p->fout_off[batch];
    p->m = offsets ? 0 : m;
    p->n_in = p->in_off[batch];
    p->n_out = p->out_off[batch];
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&p->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            p->num_cu < 1) {
            delete p;
            return fail(MRDFT_E_HIP, "no usable HIP device");
        }
    }
    {
        const int g = env_int("MRDFT_GRAPH", -2);          // 0/1 overrides MRDFT_FLAG_GRAPH
        if (g == -1 || g > 1) {
            delete p;
            return fail(MRDFT_E_INVALID_ARG, "MRDFT_GRAPH must be 0 or 1");
        }
        if (g == 0) p->flags &= ~MRDFT_FLAG_GRAPH;
        if (g == 1) p->flags |= MRDFT_FLAG_GRAPH;
    }
    mrdft_status st = upload_twiddles(p, stream);
    if (st == MRDFT_OK) st = build_tables(p, stream);
    if (st == MRDFT_OK) st = tune_with_cache(p, stream);
    if (st != MRDFT_OK) {
        free_plan(p);
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        g_plans.insert(p);
    }
    *plan = p;
    return MRDFT_OK;
}

mrdft_status mrdft_plan_output_offsets(mrdft_plan_t plan, int64_t* out) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (!out) return fail(MRDFT_E_INVALID_ARG, "out is NULL");
    std::memcpy(out, plan->out_off.data(), sizeof(int64_t) * (plan->batch + 1));
    return MRDFT_OK;
}

mrdft_status mrdft_plan_sizes(mrdft_plan_t plan, int64_t* n_in, int64_t* n_out) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (!n_in || !n_out) return fail(MRDFT_E_INVALID_ARG, "size output pointer is NULL");
    *n_in = plan->n_in;
    *n_out = plan->n_out;
    return MRDFT_OK;
}

mrdft_status mrdft_forward(mrdft_plan_t plan, const void* x, void* Y, hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (!x || !Y) return fail(MRDFT_E_INVALID_ARG, "x and Y must be non-NULL");
    if (misaligned(Y, 16) || misaligned(x, plan->dtype == MRDFT_C64 ? 16 : 8))
        return fail(MRDFT_E_INVALID_ARG, "x or Y is not sufficiently aligned");
    if ((plan->flags & MRDFT_FLAG_GRAPH) && !plan->profiling) return graph_forward(plan, x, (float2*)Y, stream);
    return run_forward(plan, x, plan->dtype == MRDFT_R32 ? IN_R32 : IN_C64, (float2*)Y, stream);
}

mrdft_status mrdft_plan_set_schedule(mrdft_plan_t plan, int tile_log, int grid, int order, hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (order & ~(MRDFT_SCHED_SERIAL | MRDFT_SCHED_AFTER | 0xff))
        return fail(MRDFT_E_INVALID_ARG, "unknown schedule bits in order 0x%x", order);
    if ((order & MRDFT_SCHED_SERIAL) && (order & MRDFT_SCHED_AFTER))
        return fail(MRDFT_E_INVALID_ARG, "MRDFT_SCHED_SERIAL and MRDFT_SCHED_AFTER exclude each other");
    return apply_schedule(plan, tile_log, grid, order & 0xff, (order & MRDFT_SCHED_SERIAL) != 0,
                          (order & MRDFT_SCHED_AFTER) != 0, stream);
}

mrdft_status mrdft_plan_schedule(mrdft_plan_t plan, int* tile_log, int* grid, int* order) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (tile_log) *tile_log = plan->dtype == MRDFT_R32 ? kRealTileLog : plan->tile_log;
    if (grid) *grid = (plan->dtype == MRDFT_C64 && plan->tile_log == kC64TileLog) ? plan->grid : 0;
    if (order) *order = plan->order | (plan->serial ? MRDFT_SCHED_SERIAL : 0) | (plan->after ? MRDFT_SCHED_AFTER : 0);
    return MRDFT_OK;
}

mrdft_status mrdft_adjoint(mrdft_plan_t plan, const void* gY, void* gx, hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (!gY || !gx) return fail(MRDFT_E_INVALID_ARG, "gY and gx must be non-NULL");
    if (misaligned(gY, 16) || misaligned(gx, plan->dtype == MRDFT_C64 ? 16 : 8))
        return fail(MRDFT_E_INVALID_ARG, "gY or gx is not sufficiently aligned");
    return run_adjoint(plan, (const float2*)gY, gx, plan->dtype == MRDFT_R32, stream);
}

mrdft_status mrdft_spectral_loss_fwd(mrdft_plan_t plan, const float* x, const float* z, double* num_den, float* L,
                                     hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (plan->ragged || plan->dtype != MRDFT_R32)
        return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs a uniform real (MRDFT_R32) plan");
    if (!plan->full_range(plan->m))
        return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs every level (plan created with a level range)");
    if (plan->hs) return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs a full-spectrum plan");
    if (!x || !z || !num_den || !L) return fail(MRDFT_E_INVALID_ARG, "x, z, num_den and L must be non-NULL");
    if (misaligned(x, 16) || misaligned(z, 16) || misaligned(num_den, 8) || misaligned(L, 4))
        return fail(MRDFT_E_INVALID_ARG, "x or z is not 16-byte aligned");
    {
        AllocScope alloc_scope;
        st = ensure_loss_workspace(plan, stream);
    }
    if (st) return st;
    const int64_t N = int64_t(1) << plan->m;
    const int64_t rows = plan->batch * plan->m;
    const int nch = loss_chunks(N);
    if (plan->d_rjobs) {
        // Fused: levels 1..16 of x - z and of z reduced on chip (Y never
        // written), levels above 16 through the passes into the workspace.
        const Twiddles tw = plan->tw();
        double* snum = plan->d_sums;
        double* sden = plan->d_sums + rows;
        // a fill kernel, not a memset node: the call may be captured into a graph
        HIP_TRY(launch_zero(plan->d_sums, (int64_t)sizeof(double) * 2 * rows, stream));
        // Levels above 16: the last pass of each level adds the squared
        // magnitudes straight into the level sums.  With two side streams the
        // sums of z run on the second one (with its own pass scratch): its
        // one-launch norms beside those of x - z, then its passes beside the
        // passes of x - z.  (Passes started beside a one-launch norm launch
        // were starved: a first pass of ~55 us took ~330 us and slowed the
        // norm launch from ~190 to ~340 us; this order saved ~50 us per
        // forward + backward on 32 x 2^18.)
        const bool upper = plan->m > kRowsMaxLevel;
        const bool par = upper && plan->nsides >= 2;
        const hipStream_t s2 = par ? plan->side[1] : stream;
        if (par) {
            HIP_TRY(hipEventRecord(plan->fork_ev, stream));
            HIP_TRY(hipStreamWaitEvent(s2, plan->fork_ev, 0));
        }
        {
            ProfScope ps(plan, MRDFT_KERNEL_LOSS, stream);
            HIP_TRY(launch_fwd_real_norms(x, z, snum, plan->m, plan->d_ljobs, plan->nljobs, tw, stream));
        }
        {
            ProfScope ps(plan, MRDFT_KERNEL_LOSS, s2);
            HIP_TRY(launch_fwd_real_norms(z, nullptr, sden, plan->m, plan->d_ljobs, plan->nljobs, tw, s2));
        }
        if (par) {
            st = upper_passes(plan, z, nullptr, s2, false, sden, false, plan->d_ss[0]);
            if (st) return st;
        }
        if (upper) {
            HIP_TRY(launch_sub_real(x, z, plan->d_v, plan->n_in, stream));
            st = upper_passes(plan, plan->d_v, nullptr, stream, false, snum);
            if (st) return st;
            if (!par) {
                st = upper_passes(plan, z, nullptr, stream, false, sden);
                if (st) return st;
            }
        }
        if (par) {
            HIP_TRY(hipEventRecord(plan->join_ev[1], s2));
            HIP_TRY(hipStreamWaitEvent(stream, plan->join_ev[1], 0));
        }
        HIP_TRY(launch_finalize(snum, sden, num_den, L, plan->batch, plan->m, 1, stream));
        return MRDFT_OK;
    }
    HIP_TRY(launch_sub_real(x, z, plan->d_v, plan->n_in, stream));
    st = run_forward(plan, plan->d_v, IN_R32, plan->d_Yv, stream);
    if (st) return st;
    st = run_forward(plan, z, IN_R32, plan->d_Yz, stream);
    if (st) return st;
    HIP_TRY(launch_sumsq(plan->d_Yv, plan->d_part, rows, N, stream));
    HIP_TRY(launch_sumsq(plan->d_Yz, plan->d_part + rows * nch, rows, N, stream));
    HIP_TRY(launch_finalize(plan->d_part, plan->d_part + rows * nch, num_den, L, plan->batch, plan->m, nch, stream));
    return MRDFT_OK;
}

mrdft_status mrdft_spectral_loss_fwd_noalloc(mrdft_plan_t plan, const float* x, const float* z, double* num_den,
                                             float* L, hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (plan->ragged || plan->dtype != MRDFT_R32 || plan->hs || !plan->full_range(plan->m))
        return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs a uniform real full-spectrum plan of every level");
    if (plan->m < kRealTileLog || plan->m > kRowsMaxLevel || !plan->d_rjobs)
        return fail(MRDFT_E_UNSUPPORTED,
                    "mrdft_spectral_loss_fwd_noalloc handles orders %d..%d (one launch per input, no passes); "
                    "the plan has order %d", kRealTileLog, kRowsMaxLevel, plan->m);
    const int64_t rows = plan->batch * plan->m;
    if (2 * rows > kNoallocMaxSums)
        return fail(MRDFT_E_UNSUPPORTED,
                    "mrdft_spectral_loss_fwd_noalloc: batch * m = %lld exceeds its workspace of %lld levels",
                    (long long)rows, (long long)(kNoallocMaxSums / 2));
    if (!x || !z || !num_den || !L) return fail(MRDFT_E_INVALID_ARG, "x, z, num_den and L must be non-NULL");
    if (misaligned(x, 16) || misaligned(z, 16) || misaligned(num_den, 8) || misaligned(L, 4))
        return fail(MRDFT_E_INVALID_ARG, "x or z is not 16-byte aligned");
    double* sums = nullptr;
    st = scratch_address(&sums);
    if (st) return st;
    const Twiddles tw = plan->tw();
    // the sums start at zero (a fill kernel: the call may be captured)
    HIP_TRY(launch_zero(sums, (int64_t)sizeof(double) * 2 * rows, stream));
    HIP_TRY(launch_fwd_real_norms(x, z, sums, plan->m, plan->d_rjobs, plan->nrjobs, tw, stream));
    HIP_TRY(launch_fwd_real_norms(z, nullptr, sums + rows, plan->m, plan->d_rjobs, plan->nrjobs, tw, stream));
    HIP_TRY(launch_finalize(sums, sums + rows, num_den, L, plan->batch, plan->m, 1, stream));
    return MRDFT_OK;
}

mrdft_status mrdft_spectral_loss_bwd(mrdft_plan_t plan, const float* x, const float* z, const double* num_den,
                                     const float* gL, float* gx, hipStream_t stream) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (plan->ragged || plan->dtype != MRDFT_R32)
        return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs a uniform real (MRDFT_R32) plan");
    if (!plan->full_range(plan->m))
        return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs every level (plan created with a level range)");
    if (plan->hs) return fail(MRDFT_E_UNSUPPORTED, "the spectral loss needs a full-spectrum plan");
    if (!x || !z || !num_den || !gL || !gx) return fail(MRDFT_E_INVALID_ARG, "null pointer argument");
    if (misaligned(x, 16) || misaligned(z, 16) || misaligned(gx, 16))
        return fail(MRDFT_E_INVALID_ARG, "x, z or gx is not 16-byte aligned");
    {
        AllocScope alloc_scope;
        st = ensure_loss_workspace(plan, stream);
    }
    if (st) return st;
    const int64_t N = int64_t(1) << plan->m;
    const int64_t rows = plan->batch * plan->m;
    if (plan->d_rjobs) {
        // Recompute the spectra of x - z with each level already scaled by its
        // gradient factor (levels 1..16 in the one-launch forward), as packed
        // half spectra (x - z is real: its level spectra are Hermitian, and
        // the real adjoint of the packed values is the gradient), then the adjoint.
        // Levels above 16 run on side streams when the plan has one per
        // level, after the one-launch forward was issued (passes started
        // beside it were starved; this order saved ~20 us per forward +
        // backward on 32 x 2^18): x - z and its passes, the last pass of each
        // level storing its packed spectra already scaled.  The adjoint's
        // chain of each level follows on the same side stream, so the
        // caller's stream does not wait for these passes.
        const bool upper = plan->m > kRowsMaxLevel;
        const int nup = plan->m - kRowsMaxLevel;
        const bool par = upper && plan->nsides >= nup;
        HIP_TRY(launch_loss_alpha(num_den, gL, plan->d_alpha, rows, plan->m, stream));
        {
            ProfScope ps(plan, MRDFT_KERNEL_LOSS, stream);
            HIP_TRY(launch_fwd_real_scaled(x, z, plan->d_alpha, plan->m, plan->d_Yv, plan->d_ljobs, plan->nljobs,
                                           plan->tw(), stream, true));
        }
        if (par) {
            HIP_TRY(hipEventRecord(plan->fork_ev, stream));
            HIP_TRY(hipStreamWaitEvent(plan->side[0], plan->fork_ev, 0));
            HIP_TRY(launch_sub_real(x, z, plan->d_v, plan->n_in, plan->side[0]));
            HIP_TRY(hipEventRecord(plan->join_ev[0], plan->side[0]));      // x - z ready
            for (int k = 0; k < nup; ++k) {
                const hipStream_t sk = plan->side[k];
                if (k) HIP_TRY(hipStreamWaitEvent(sk, plan->join_ev[0], 0));
                st = upper_passes(plan, plan->d_v, plan->d_Yv, sk, true, nullptr, true,
                                  k ? plan->d_ss[k - 1] : plan->d_s, kRowsMaxLevel + 1 + k, plan->d_alpha);
                if (st) return st;
            }
            for (int k = 0; k < nup; ++k) HIP_TRY(hipEventRecord(plan->join_ev[k], plan->side[k]));
        }
        if (upper) {
            if (par) {
                // read only by the adjoint's chains on the same side streams
            } else {
                HIP_TRY(launch_sub_real(x, z, plan->d_v, plan->n_in, stream));
                st = upper_passes(plan, plan->d_v, plan->d_Yv, stream, true, nullptr, true, nullptr, 0, plan->d_alpha);
                if (st) return st;
            }
        }
        return run_adjoint(plan, plan->d_Yv, gx, true, stream, true);
    }
    HIP_TRY(launch_sub_real(x, z, plan->d_v, plan->n_in, stream));
    st = run_forward(plan, plan->d_v, IN_R32, plan->d_Yv, stream);
    if (st) return st;
    HIP_TRY(launch_scale_levels(plan->d_Yv, num_den, gL, plan->m, N, rows, stream));
    return run_adjoint(plan, plan->d_Yv, gx, true, stream);
}

mrdft_status mrdft_plan_set_profiling(mrdft_plan_t plan, int enable) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    plan->profiling = enable != 0;
    return MRDFT_OK;
}

mrdft_status mrdft_plan_read_profile(mrdft_plan_t plan, int nkinds, double* total_ms, int64_t* launches) {
    mrdft_status st = check_plan(plan);
    if (st) return st;
    if (nkinds < 0 || (nkinds > 0 && (!total_ms || !launches)))
        return fail(MRDFT_E_INVALID_ARG, "bad profile output arrays");
    for (int k = 0; k < nkinds; ++k) {
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& r : plan->recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.kind < nkinds) {
            total_ms[r.kind] += ms;
            launches[r.kind] += 1;
        }
        plan->event_pool.push_back(r.a);
        plan->event_pool.push_back(r.b);
    }
    plan->recs.clear();
    return MRDFT_OK;
}

mrdft_status mrdft_plan_destroy(mrdft_plan_t plan) {
    if (!plan) return MRDFT_OK;
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        if (!g_plans.erase(plan)) return fail(MRDFT_E_INVALID_ARG, "plan handle is not live (destroyed twice?)");
    }
    free_plan(plan);
    return MRDFT_OK;
}

}  // extern "C"
