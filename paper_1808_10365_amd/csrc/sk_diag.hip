// Per-channel mean, variance and effective receiver count of the estimator
// (App. A: N_eff = 4 / (n var)). One workgroup per channel, two passes
// (mean, then squared deviations) in FP64 with fixed-order reductions.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sk_diag.h"
#include "sk_internal.h"

namespace sk {

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void channel_stats_kernel(const float* v, int64_t B, int32_t M, double* mean,
                                                            double* var, double* n_eff, int64_t* count) {
  __shared__ double sh[256];
  const int f = blockIdx.x;
  const float* row = v + (int64_t)f * B;
  double s = 0.0, c = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    const float x = row[b];
    if (!isnan(x)) { s += (double)x; c += 1.0; }
  }
  const double S = block_sum(s, sh);
  const double C = block_sum(c, sh);
  const double m = C > 0.0 ? S / C : __builtin_nan("");
  double q = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    const float x = row[b];
    if (!isnan(x)) { const double d = (double)x - m; q += d * d; }
  }
  const double Q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    const double vv = C > 1.0 ? Q / (C - 1.0) : __builtin_nan("");
    mean[f] = m;
    var[f] = vv;
    n_eff[f] = (C > 1.0 && vv > 0.0) ? 4.0 / ((double)M * vv) : __builtin_nan("");
    count[f] = (int64_t)C;
  }
}

}  // namespace sk

extern "C" int sk_channel_stats(const float* d_v, int32_t n_channels, int64_t n_blocks, int32_t block_len,
                                double* d_mean, double* d_var, double* d_n_eff, int64_t* d_count, void* stream) {
  sk::clear_error();
  if (n_channels < 0 || n_blocks < 0 || block_len < 2 ||
      (n_channels > 0 && (!d_mean || !d_var || !d_n_eff || !d_count || (n_blocks > 0 && !d_v)))) {
    sk::set_error("bad arguments");
    return SK_ERR_INVALID_ARG;
  }
  if (n_channels == 0) return SK_OK;
  sk::channel_stats_kernel<<<dim3(n_channels), dim3(256), 0, (hipStream_t)stream>>>(d_v, n_blocks, block_len, d_mean,
                                                                                    d_var, d_n_eff, d_count);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}
