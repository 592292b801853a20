// Monte-Carlo calibration of thresholds under digitisation (App. B): the GPU
// simulates 4+4-bit Gaussian data with a counter-based generator and
// evaluates the multi-receiver estimator on every simulated block.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <vector>

#include "sk_calib.h"
#include "sk_internal.h"

namespace sk {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct McArgs {
  uint64_t key;
  int32_t n_inputs, block_len, estimator, n_thr;
  int64_t n_sim;
  uint32_t thr[16];
  double* values;   // [n_sim]
};

// One workgroup per simulated estimate; lanes walk the inputs.
__global__ __launch_bounds__(256) void mc_kernel(McArgs a) {
#pragma clang fp contract(off)
  __shared__ double sh_q[256];
  __shared__ int32_t sh_n[256];
  const int64_t s = blockIdx.x;
  const int tid = threadIdx.x;
  const int C = a.n_thr / 2;
  double q = 0.0;
  int32_t n = 0;
  for (int i = tid; i < a.n_inputs; i += 256) {
    int64_t s1 = 0, s2 = 0;
    const uint64_t base = ((uint64_t)s * a.n_inputs + i) * (uint64_t)a.block_len;
    for (int j = 0; j < a.block_len; ++j) {
      const uint64_t r = mix64(a.key + (base + j + 1) * 0x9E3779B97F4A7C15ULL);
      const uint32_t ure = (uint32_t)(r >> 32), uim = (uint32_t)r;
      int re = -C, im = -C;
      for (int k = 0; k < a.n_thr; ++k) {
        re += a.thr[k] <= ure;
        im += a.thr[k] <= uim;
      }
      const int64_t p = re * re + im * im;
      s1 += p;
      s2 += p * p;
    }
    if (s1 > 0) {
      const double x = (double)s1;
      q += (double)s2 / (x * x);
      n += 1;
    }
  }
  sh_q[tid] = q;
  sh_n[tid] = n;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      sh_q[tid] += sh_q[tid + st];
      sh_n[tid] += sh_n[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double Bq = sh_q[0];
    const int32_t N = sh_n[0];
    const double Md = (double)a.block_len, Kd = (double)N * Md;
    double V = __builtin_nan("");
    if ((int64_t)N * a.block_len >= 2 && N > 0) {
      // L = 1: A = N exactly (each S1_i / S1_i is 1).
      const double A = (double)N;
      if (a.estimator == SK_EST_TILDE)
        V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)N - 1.0);
      else
        V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);
    }
    a.values[s] = V;
  }
}

static double mc_phi(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

}  // namespace sk

extern "C" int sk_calibrate_mc(const sk_mc_desc* d, double* moments, double* d_values, void* stream) {
  using namespace sk;
  clear_error();
  if (!d || !moments || d->n_inputs < 1 || d->block_len < 2 || d->block_len > 131071 || d->clip < 1 ||
      d->clip > 7 || !(d->sigma > 0.0) || d->n_sim < 1 || d->n_sim > (1LL << 31) ||
      (d->estimator != SK_EST_HAT && d->estimator != SK_EST_TILDE)) {
    set_error("bad Monte-Carlo description");
    return SK_ERR_INVALID_ARG;
  }
  McArgs a;
  a.key = 0;
  {
    // Key = SplitMix64 output of the seed (host side, same mixing function).
    uint64_t z = d->seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    a.key = z ^ (z >> 31);
  }
  a.n_inputs = d->n_inputs;
  a.block_len = d->block_len;
  a.estimator = d->estimator;
  a.n_thr = 2 * d->clip;
  a.n_sim = d->n_sim;
  for (int k = 0; k < a.n_thr; ++k) {
    double s = floor(mc_phi(((double)(k - d->clip) + 0.5) / d->sigma) * 4294967296.0);
    if (s < 0) s = 0;
    if (s > 4294967295.0) s = 4294967295.0;
    a.thr[k] = (uint32_t)s;
  }
  hipStream_t st = (hipStream_t)stream;
  double* vals = d_values;
  if (!vals) SK_HIP_TRY(hipMalloc((void**)&vals, sizeof(double) * d->n_sim));
  a.values = vals;
  mc_kernel<<<dim3((unsigned)d->n_sim), dim3(256), 0, st>>>(a);
  hipError_t le = hipGetLastError();
  std::vector<double> h(d->n_sim);
  hipError_t ce = le == hipSuccess ? hipMemcpyAsync(h.data(), vals, sizeof(double) * d->n_sim, hipMemcpyDeviceToHost, st) : le;
  hipError_t se = hipStreamSynchronize(st);
  if (!d_values) (void)hipFree(vals);
  if (le != hipSuccess || ce != hipSuccess || se != hipSuccess) {
    set_error("Monte-Carlo launch failed: %s", hipGetErrorString(le != hipSuccess ? le : (ce != hipSuccess ? ce : se)));
    return SK_ERR_DEVICE;
  }
  // Moments of the valid estimates (host, FP64, two passes).
  double s = 0.0;
  int64_t n = 0;
  for (double v : h) if (!std::isnan(v)) { s += v; ++n; }
  const double m = n ? s / (double)n : NAN;
  double m2 = 0.0, m3 = 0.0, m4 = 0.0;
  for (double v : h) {
    if (std::isnan(v)) continue;
    const double e = v - m;
    m2 += e * e;
    m3 += e * e * e;
    m4 += e * e * e * e;
  }
  const double pv = n ? m2 / (double)n : NAN;
  moments[0] = m;
  moments[1] = n > 1 ? m2 / (double)(n - 1) : NAN;
  moments[2] = (n && pv > 0) ? (m3 / (double)n) / pow(pv, 1.5) : NAN;
  moments[3] = (n && pv > 0) ? (m4 / (double)n) / (pv * pv) - 3.0 : NAN;
  return SK_OK;
}
