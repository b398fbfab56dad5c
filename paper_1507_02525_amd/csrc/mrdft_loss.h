#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrdft {

constexpr int64_t kLossChunk = 8192;    // elements reduced by one block

int loss_chunks(int64_t N);
hipError_t launch_sub_real(const float* x, const float* z, float* v, int64_t n, hipStream_t s);
hipError_t launch_sumsq(const float2* Y, double* part, int64_t rows, int64_t N, hipStream_t s);
// num_den[row] = sums of the row's nchunks partials (pnum/pden laid out
// [batch * m][nchunks]), L = (1/m) sum_row num / den.
hipError_t launch_finalize(const double* pnum, const double* pden, double* num_den, float* L, int64_t batch, int m,
                           int nchunks, hipStream_t s);
// Y[b][i][:] *= gL * 2 / (m * den_{b,i}) for levels i > first (rows = batch * (m - first)).
hipError_t launch_scale_levels(float2* Y, const double* num_den, const float* gL, int m, int64_t N, int64_t rows,
                               hipStream_t s, int first = 0);
// alpha[b * m + i] = gL * 2 / (m * den_{b,i})
hipError_t launch_loss_alpha(const double* num_den, const float* gL, float* alpha, int64_t rows, int m, hipStream_t s);

}  // namespace mrdft
