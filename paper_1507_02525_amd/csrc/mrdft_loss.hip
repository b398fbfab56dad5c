// Multi-resolution spectral loss helpers: the per-level energies
// num_i = ||Y^(i)(x) - Y^(i)(z)||^2 and den_i = ||Y^(i)(z)||^2, the loss
// L = sum_b (1/m) sum_i num_i / den_i, and the per-level scaling of the
// recomputed spectra by dL/dY = gL * 2 (Y(x) - Y(z)) / (m * den_i) that feeds
// the adjoint.  Reductions accumulate in FP64.  The partial sums of the
// generic path (sumsq_kernel, then finalize_kernel) use fixed chunks and a
// fixed tree order, so they are bit-for-bit repeatable; the fused path adds
// its per-level sums with FP64 atomics from workgroups that finish in no fixed
// order, so its num_den and L can differ in the last bits between calls.
#include "mrdft_internal.h"
#include "mrdft_loss.h"

namespace mrdft {

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(256) void sub_real_kernel(const float* __restrict__ x, const float* __restrict__ z,
                                                       float* __restrict__ v, int64_t n) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 + 3 < n) {
        float4 a = *(const float4*)(x + i0), b = *(const float4*)(z + i0);
        *(float4*)(v + i0) = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
    } else {
        for (int64_t i = i0; i < n; ++i) v[i] = x[i] - z[i];
    }
}

// One block per (row, chunk): row = b*m + (i-1) of a [rows][N] complex array.
__global__ __launch_bounds__(kRedThreads) void sumsq_kernel(const float2* __restrict__ Y, double* __restrict__ part,
                                                            int64_t N, int64_t chunk, int nchunks) {
    const int64_t row = blockIdx.x / nchunks;
    const int c = blockIdx.x - (int)(row * nchunks);
    const float2* p = Y + row * N + (int64_t)c * chunk;
    const int64_t n = (N - (int64_t)c * chunk) < chunk ? (N - (int64_t)c * chunk) : chunk;
    // pairs of values (16-byte loads), four loads in flight per thread
    double acc = 0.0;
    const int64_t npair = n >> 1;
    const float4* p4 = (const float4*)p;          // rows and chunks start at even elements
    int64_t e = threadIdx.x;
    for (; e + 3 * kRedThreads < npair; e += 4 * kRedThreads) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = p4[e + u * kRedThreads];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc += ((double)v[u].x * v[u].x + (double)v[u].y * v[u].y) + ((double)v[u].z * v[u].z + (double)v[u].w * v[u].w);
    }
    for (; e < npair; e += kRedThreads) {
        const float4 v = p4[e];
        acc += ((double)v.x * v.x + (double)v.y * v.y) + ((double)v.z * v.z + (double)v.w * v.w);
    }
    if ((n & 1) && threadIdx.x == 0) {
        const float2 v = p[n - 1];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// num_den[row] = (sum of num partials, sum of den partials); then
// L = (1/m) sum over rows of num / den.  One block; thread t takes rows
// t, t + 256, ... and the block sums in a fixed tree (deterministic).
__global__ __launch_bounds__(kRedThreads) void finalize_kernel(const double* __restrict__ pnum,
                                                               const double* __restrict__ pden,
                                                               double* __restrict__ num_den, float* __restrict__ L,
                                                               int64_t batch, int m, int nchunks) {
    const int64_t rows = batch * m;
    double acc = 0.0;
    for (int64_t row = threadIdx.x; row < rows; row += kRedThreads) {
        double num = 0.0, den = 0.0;
        for (int c = 0; c < nchunks; ++c) {
            num += pnum[row * nchunks + c];
            den += pden[row * nchunks + c];
        }
        num_den[2 * row] = num;
        num_den[2 * row + 1] = den;
        acc += num / den;
    }
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *L = (float)(red[0] / (double)m);
}

// Y[b][i][:] *= gL * 2 / (m * den_{b,i})
// Levels first+1 .. m of every signal (rows = batch * (m - first)).
__global__ __launch_bounds__(256) void scale_levels_kernel(float2* __restrict__ Y, const double* __restrict__ num_den,
                                                           const float* __restrict__ gL, int m, int64_t N,
                                                           int64_t rows, int first) {
    const int64_t r = blockIdx.y;
    if (r >= rows) return;
    const int per = m - first;
    const int64_t row = (r / per) * m + first + (r % per);
    const double s = (double)(*gL) * 2.0 / ((double)m * num_den[2 * row + 1]);
    const float sf = (float)s;
    float2* p = Y + row * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
        float2 v = p[e];
        p[e] = make_float2(v.x * sf, v.y * sf);
    }
}

hipError_t launch_sub_real(const float* x, const float* z, float* v, int64_t n, hipStream_t s) {
    const int64_t nb = (n + 4 * 256 - 1) / (4 * 256);
    hipLaunchKernelGGL(sub_real_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, z, v, n);
    return hipGetLastError();
}

int loss_chunks(int64_t N) { return (int)((N + kLossChunk - 1) / kLossChunk); }

hipError_t launch_sumsq(const float2* Y, double* part, int64_t rows, int64_t N, hipStream_t s) {
    const int nch = loss_chunks(N);
    hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)(rows * nch)), dim3(kRedThreads), 0, s, Y, part, N,
                       (int64_t)kLossChunk, nch);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* pnum, const double* pden, double* num_den, float* L, int64_t batch, int m,
                           int nchunks, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kRedThreads), 0, s, pnum, pden, num_den, L, batch, m,
                       nchunks);
    return hipGetLastError();
}

hipError_t launch_scale_levels(float2* Y, const double* num_den, const float* gL, int m, int64_t N, int64_t rows,
                               hipStream_t s, int first) {
    int64_t bx = (N + 255) / 256;
    if (bx > 256) bx = 256;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_levels_kernel, dim3((unsigned)bx, (unsigned)rows), dim3(256), 0, s, Y, num_den, gL, m,
                       N, rows, first);
    return hipGetLastError();
}

// alpha[row] = gL * 2 / (m * den_row), the per-level factor of the loss gradient.
__global__ void loss_alpha_kernel(const double* __restrict__ num_den, const float* __restrict__ gL, float* alpha,
                                  int64_t rows, int m) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows) alpha[r] = (float)((double)(*gL) * 2.0 / ((double)m * num_den[2 * r + 1]));
}

hipError_t launch_loss_alpha(const double* num_den, const float* gL, float* alpha, int64_t rows, int m, hipStream_t s) {
    hipLaunchKernelGGL(loss_alpha_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, num_den, gL, alpha,
                       rows, m);
    return hipGetLastError();
}

}  // namespace mrdft
