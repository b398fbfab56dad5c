#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrdft {

constexpr int64_t kLossChunk = 65536;   // elements reduced by one block

int loss_chunks(int64_t N);
hipError_t launch_sub_real(const float* x, const float* z, float* v, int64_t n, hipStream_t s);
hipError_t launch_sumsq(const float2* Y, double* part, int64_t rows, int64_t N, hipStream_t s);
hipError_t launch_finalize(const double* pnum, const double* pden, double* num_den, float* L, int64_t batch, int m,
                           int64_t N, hipStream_t s);
hipError_t launch_scale_levels(float2* Y, const double* num_den, const float* gL, int m, int64_t N, int64_t rows,
                               hipStream_t s);

}  // namespace mrdft
