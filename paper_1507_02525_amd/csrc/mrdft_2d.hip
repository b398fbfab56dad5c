// Two-dimensional separable MrDFT: the 1-D transform of eq. (1) along the
// columns and along the rows of every image, for every pair of levels (the
// paper names two-dimensional signals as an application in Section 6).
//
//   x[b][n1][n2] --transpose--> xt[b][n2][n1]
//     --1-D MrDFT of the N2 columns (order m1, plan dtype)--> c[b][n2][i1][n1]
//     --transpose of each (b, i1) plane--> d[b][i1][n1][n2]
//     --1-D MrDFT of the rows (order m2, complex)--> Y[b][i1][n1][i2][n2]
//
// The adjoint runs the same steps backwards with the 1-D adjoints.  The
// transposes move 32 x 32 tiles through LDS (coalesced 128- or 256-byte rows
// on both sides).
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <new>
#include <set>

#include "../../include/mrdft.h"
#include "mrdft_internal.h"

namespace mrdft {
mrdft_status report_error(mrdft_status st, const char* msg);
}  // namespace mrdft

using namespace mrdft;

namespace {

constexpr int kTT = 32;          // transpose tile edge
constexpr int kTRows = 8;        // thread rows: 32 x 8 threads, 4 elements each

// Batched strided transpose: for every (u, v) with u < nb0, v < nb1, the
// R x C matrix at src + u sb0 + v sb1 (row stride srs) is written transposed
// (C x R, row stride drs) at dst + u db0 + v db1.  One workgroup per tile.
struct TGeom {
    int64_t R, C, srs, drs, sb0, sb1, db0, db1, nb1, tiles_c, tiles_r;
};

template <typename T>
__global__ __launch_bounds__(kTT * kTRows) void transpose_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                                 TGeom g) {
    __shared__ T tile[kTT][kTT + 1];
    int64_t blk = blockIdx.x;
    const int64_t tc = blk % g.tiles_c;
    blk /= g.tiles_c;
    const int64_t tr = blk % g.tiles_r;
    blk /= g.tiles_r;
    const int64_t v = blk % g.nb1, u = blk / g.nb1;
    const T* s = src + u * g.sb0 + v * g.sb1;
    T* d = dst + u * g.db0 + v * g.db1;
    const int tx = threadIdx.x % kTT, ty = threadIdx.x / kTT;
    const int64_t r0 = tr * kTT, c0 = tc * kTT;
#pragma unroll
    for (int k = 0; k < kTT; k += kTRows) {
        const int64_t r = r0 + ty + k, c = c0 + tx;
        if (r < g.R && c < g.C) tile[ty + k][tx] = s[r * g.srs + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTT; k += kTRows) {
        const int64_t c = c0 + ty + k, r = r0 + tx;     // output row c, column r
        if (r < g.R && c < g.C) d[c * g.drs + r] = tile[tx][ty + k];
    }
}

template <typename T>
hipError_t transpose(const T* src, T* dst, TGeom g, int64_t nb0, hipStream_t s) {
    g.tiles_r = (g.R + kTT - 1) / kTT;
    g.tiles_c = (g.C + kTT - 1) / kTT;
    const int64_t blocks = g.tiles_r * g.tiles_c * g.nb1 * nb0;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)blocks), dim3(kTT * kTRows), 0, s, src, dst, g);
    return hipGetLastError();
}

}  // namespace

struct mrdft_plan2d {
    int m1 = 0, m2 = 0;
    int64_t batch = 0, N1 = 0, N2 = 0;
    mrdft_dtype dtype = MRDFT_C64;
    mrdft_plan_t cols = nullptr;     // N2 * batch column signals of order m1, plan dtype
    mrdft_plan_t rows = nullptr;     // m1 * N1 * batch row signals of order m2, complex
    void* xt = nullptr;              // transposed images (plan dtype)
    float2* c = nullptr;             // column transforms [b][n2][i1][n1]
    float2* d = nullptr;             // transposed planes [b][i1][n1][n2]
    int64_t n_in = 0, n_out = 0;
};

namespace {

mrdft_status fail2(mrdft_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mrdft_status fail2(mrdft_status st, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return report_error(st, buf);
}

void free2d(mrdft_plan2d* p) {
    if (!p) return;
    if (p->cols) mrdft_plan_destroy(p->cols);
    if (p->rows) mrdft_plan_destroy(p->rows);
    dev_free(p->xt);
    dev_free(p->c);
    dev_free(p->d);
    delete p;
}

// Live 2-D plans: a destroyed or foreign handle is rejected, not dereferenced.
std::mutex g_plans2d_mu;
std::set<const void*> g_plans2d;

mrdft_status check2d(mrdft_plan2d_t p) {
    if (!p) return fail2(MRDFT_E_INVALID_ARG, "plan is NULL");
    std::lock_guard<std::mutex> lk(g_plans2d_mu);
    if (!g_plans2d.count(p)) return fail2(MRDFT_E_INVALID_ARG, "2-D plan handle is not live (destroyed or invalid)");
    return MRDFT_OK;
}

bool misaligned2(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) & (a - 1)) != 0; }

// T1 / its inverse: image b, R x C = N1 x N2 (forward) or N2 x N1 (adjoint).
TGeom image_geom(int64_t R, int64_t C) {
    TGeom g{};
    g.R = R;
    g.C = C;
    g.srs = C;
    g.drs = R;
    g.sb0 = g.db0 = R * C;
    g.sb1 = g.db1 = 0;
    g.nb1 = 1;
    return g;
}

}  // namespace

extern "C" {

mrdft_status mrdft_plan2d_create(mrdft_plan2d_t* plan, int m1, int m2, int64_t batch, mrdft_dtype dtype,
                                 hipStream_t stream) {
    if (!plan) return fail2(MRDFT_E_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (m1 < 1 || m2 < 1 || m1 > MRDFT_MAX_ORDER || m2 > MRDFT_MAX_ORDER || m1 + m2 > 40)
        return fail2(MRDFT_E_INVALID_ARG, "orders m1 = %d, m2 = %d must be >= 1 with m1 + m2 <= 40", m1, m2);
    if (batch < 1) return fail2(MRDFT_E_INVALID_ARG, "batch must be >= 1 (got %lld)", (long long)batch);
    if (dtype != MRDFT_C64 && dtype != MRDFT_R32) return fail2(MRDFT_E_INVALID_ARG, "unknown dtype %d", (int)dtype);
    const int64_t N1 = int64_t(1) << m1, N2 = int64_t(1) << m2;
    if (batch > (int64_t(1) << 46) / (N1 * N2 * m1 * m2))
        return fail2(MRDFT_E_INVALID_ARG, "2-D transform of %lld images of 2^%d x 2^%d is too large",
                     (long long)batch, m1, m2);
    AllocScope alloc_scope;
    mrdft_plan2d* p = new (std::nothrow) mrdft_plan2d();
    if (!p) return fail2(MRDFT_E_ALLOC, "host allocation failed");
    p->m1 = m1;
    p->m2 = m2;
    p->batch = batch;
    p->N1 = N1;
    p->N2 = N2;
    p->dtype = dtype;
    p->n_in = batch * N1 * N2;
    p->n_out = p->n_in * m1 * m2;
    mrdft_status st = mrdft_plan_create(&p->cols, m1, batch * N2, nullptr, dtype, MRDFT_FLAG_NONE, stream);
    if (st == MRDFT_OK) st = mrdft_plan_create(&p->rows, m2, batch * m1 * N1, nullptr, MRDFT_C64, MRDFT_FLAG_NONE, stream);
    if (st != MRDFT_OK) {
        free2d(p);
        return st;                       // message already set by the 1-D plan
    }
    const size_t esz = dtype == MRDFT_R32 ? sizeof(float) : sizeof(float2);
    const size_t cbytes = sizeof(float2) * (size_t)(p->n_in * m1);
    if (dev_malloc(&p->xt, esz * (size_t)p->n_in) != hipSuccess || dev_malloc(&p->c, cbytes) != hipSuccess ||
        dev_malloc(&p->d, cbytes) != hipSuccess) {
        free2d(p);
        return fail2(MRDFT_E_ALLOC, "2-D workspace allocation failed (%zu bytes)", esz * (size_t)p->n_in + 2 * cbytes);
    }
    {
        std::lock_guard<std::mutex> lk(g_plans2d_mu);
        g_plans2d.insert(p);
    }
    *plan = p;
    return MRDFT_OK;
}

mrdft_status mrdft_plan2d_sizes(mrdft_plan2d_t plan, int64_t* n_in, int64_t* n_out) {
    mrdft_status st = check2d(plan);
    if (st) return st;
    if (!n_in || !n_out) return fail2(MRDFT_E_INVALID_ARG, "size output pointer is NULL");
    *n_in = plan->n_in;
    *n_out = plan->n_out;
    return MRDFT_OK;
}

mrdft_status mrdft_forward2d(mrdft_plan2d_t p, const void* x, void* Y, hipStream_t s) {
    if (mrdft_status c = check2d(p)) return c;
    if (!x || !Y) return fail2(MRDFT_E_INVALID_ARG, "x and Y must be non-NULL");
    if (misaligned2(x, p->dtype == MRDFT_R32 ? 8 : 16) || misaligned2(Y, 16))
        return fail2(MRDFT_E_INVALID_ARG, "x or Y is not sufficiently aligned");
    const int64_t N1 = p->N1, N2 = p->N2, m1 = p->m1;
    hipError_t e = p->dtype == MRDFT_R32
                       ? transpose((const float*)x, (float*)p->xt, image_geom(N1, N2), p->batch, s)
                       : transpose((const float2*)x, (float2*)p->xt, image_geom(N1, N2), p->batch, s);
    if (e != hipSuccess) return fail2(MRDFT_E_HIP, "transpose launch failed: %s", hipGetErrorString(e));
    mrdft_status st = mrdft_forward(p->cols, p->xt, p->c, s);
    if (st) return st;
    TGeom g{};                           // plane (b, i1): N2 x N1 at row stride m1 N1 -> N1 x N2
    g.R = N2;
    g.C = N1;
    g.srs = m1 * N1;
    g.sb0 = N2 * m1 * N1;
    g.sb1 = N1;
    g.drs = N2;
    g.db0 = m1 * N1 * N2;
    g.db1 = N1 * N2;
    g.nb1 = m1;
    e = transpose((const float2*)p->c, p->d, g, p->batch, s);
    if (e != hipSuccess) return fail2(MRDFT_E_HIP, "transpose launch failed: %s", hipGetErrorString(e));
    return mrdft_forward(p->rows, p->d, Y, s);
}

mrdft_status mrdft_adjoint2d(mrdft_plan2d_t p, const void* gY, void* gx, hipStream_t s) {
    if (mrdft_status c = check2d(p)) return c;
    if (!gY || !gx) return fail2(MRDFT_E_INVALID_ARG, "gY and gx must be non-NULL");
    if (misaligned2(gY, 16) || misaligned2(gx, p->dtype == MRDFT_R32 ? 8 : 16))
        return fail2(MRDFT_E_INVALID_ARG, "gY or gx is not sufficiently aligned");
    const int64_t N1 = p->N1, N2 = p->N2, m1 = p->m1;
    mrdft_status st = mrdft_adjoint(p->rows, gY, p->d, s);
    if (st) return st;
    TGeom g{};                           // plane (b, i1): N1 x N2 -> N2 x N1 at row stride m1 N1
    g.R = N1;
    g.C = N2;
    g.srs = N2;
    g.sb0 = m1 * N1 * N2;
    g.sb1 = N1 * N2;
    g.drs = m1 * N1;
    g.db0 = N2 * m1 * N1;
    g.db1 = N1;
    g.nb1 = m1;
    hipError_t e = transpose((const float2*)p->d, p->c, g, p->batch, s);
    if (e != hipSuccess) return fail2(MRDFT_E_HIP, "transpose launch failed: %s", hipGetErrorString(e));
    st = mrdft_adjoint(p->cols, p->c, p->xt, s);
    if (st) return st;
    e = p->dtype == MRDFT_R32 ? transpose((const float*)p->xt, (float*)gx, image_geom(N2, N1), p->batch, s)
                              : transpose((const float2*)p->xt, (float2*)gx, image_geom(N2, N1), p->batch, s);
    if (e != hipSuccess) return fail2(MRDFT_E_HIP, "transpose launch failed: %s", hipGetErrorString(e));
    return MRDFT_OK;
}

mrdft_status mrdft_plan2d_destroy(mrdft_plan2d_t plan) {
    if (!plan) return MRDFT_OK;
    {
        std::lock_guard<std::mutex> lk(g_plans2d_mu);
        if (!g_plans2d.erase(plan)) return fail2(MRDFT_E_INVALID_ARG, "2-D plan handle is not live (destroyed or invalid)");
    }
    free2d(plan);
    return MRDFT_OK;
}

}  // extern "C"
