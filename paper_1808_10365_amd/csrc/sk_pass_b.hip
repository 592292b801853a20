// Pass B: normaliser window, array combine, estimator and flags.
//
// Per (channel f, input i) the blocks form one sequence e: the H history
// blocks kept from earlier calls (oldest first), then this call's B blocks.
// The normaliser of block e is the window sum P = sum of S1 over e-L+1 .. e
// (Eq. discreteMean is L = 1: the block's own power). Its common factor
// (M times the number of blocks in the window) is the same for every input
// of a (channel, block) and cancels in the estimator, so the weights are
// 1/P_i (Eq. normedSum1, normedSum2).
//
// Kernels, in launch order for L >= 2:
//   chunk_sum_kernel     sum of S1 over each chunk of R consecutive e
//   chunk_scan_kernel    exclusive prefix over chunks (int64)
//   combine_kernel       one workgroup per (chunk, channel): window sums by
//                        sliding P += S1[e] - S1[e-L] from a start value made
//                        of two prefix lookups; per block, FP64 A and Bq and
//                        int64 R1, R2 summed over inputs in a fixed order
//                        (lane-sequential, then a fixed tree), then V and flags
//   hist_update_kernel   keep the last min(L-1, H+B) blocks for the next call
// For L <= 1 only combine_kernel runs (P is the block's own S1).
#include <hip/hip_runtime.h>
#include <math.h>

#include "sk_internal.h"

namespace sk {

__device__ __forceinline__ int32_t seq_s1(const PassBArgs& a, int f, int64_t e, int i) {
  if (e < a.hist_len) return a.hist[((int64_t)f * a.hist_cap + e) * a.n_inputs + i];
  return a.s1[((int64_t)f * a.n_blocks + (e - a.hist_len)) * a.n_inputs + i];
}

__global__ __launch_bounds__(256) void chunk_sum_kernel(PassBArgs a) {
  const int c = blockIdx.x, f = blockIdx.y;
  const int i = blockIdx.z * 256 + threadIdx.x;
  if (i >= a.n_inputs) return;
  const int64_t total = (int64_t)a.hist_len + a.n_blocks;
  const int64_t e0 = (int64_t)c * a.chunk;
  const int64_t e1 = e0 + a.chunk < total ? e0 + a.chunk : total;
  int64_t s = 0;
  for (int64_t e = e0; e < e1; ++e) s += seq_s1(a, f, e, i);
  a.chunk_sum[((int64_t)f * a.n_chunks + c) * a.n_inputs + i] = s;
}

__global__ __launch_bounds__(256) void chunk_scan_kernel(PassBArgs a) {
  const int f = blockIdx.x;
  const int i = blockIdx.y * 256 + threadIdx.x;
  if (i >= a.n_inputs) return;
  const int64_t N = a.n_inputs;
  int64_t run = 0;
  int64_t* out = a.chunk_prefix + (int64_t)f * (a.n_chunks + 1) * N + i;
  const int64_t* in = a.chunk_sum + (int64_t)f * a.n_chunks * N + i;
  out[0] = 0;
  for (int c = 0; c < a.n_chunks; ++c) {
    run += in[(int64_t)c * N];
    out[(int64_t)(c + 1) * N] = run;
  }
}

// Exclusive prefix of S1 over the sequence up to (not including) x.
__device__ int64_t seq_prefix(const PassBArgs& a, int f, int64_t x, int i) {
  const int64_t q = x / a.chunk;
  int64_t s = a.chunk_prefix[((int64_t)f * (a.n_chunks + 1) + q) * a.n_inputs + i];
  for (int64_t e = q * a.chunk; e < x; ++e) s += seq_s1(a, f, e, i);
  return s;
}

struct Partial {
  double a, q;
  int64_t r1, r2;
  int32_t n;
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Estimator and flags from the combined sums (Eq. avgSK, final; Sec. 3.2).
// Written with contraction off so the rounding steps are the plain ones.
__device__ void finish(const PassBArgs& a, int f, int b, const Partial& p) {
#pragma clang fp contract(off)
  const int64_t K = (int64_t)p.n * a.block_len;
  const double Kd = (double)K, Md = (double)a.block_len;
  bool invalid = K < 2;
  double V = 0.0;
  double A = p.a, Bq = p.q;
  if (a.window == 0) {
    invalid = invalid || p.r1 == 0;
    if (!invalid) {
      // Eq. (2) over all K samples, numerator K R2 - R1^2 formed exactly.
      const __int128 num = (__int128)K * (__int128)p.r2 - (__int128)p.r1 * (__int128)p.r1;
      const __int128 den = (__int128)p.r1 * (__int128)p.r1;
      const double nd = (double)(int64_t)(num >> 64) * 18446744073709551616.0 + (double)(uint64_t)num;
      const double dd = (double)(int64_t)(den >> 64) * 18446744073709551616.0 + (double)(uint64_t)den;
      V = (Kd + 1.0) / (Kd - 1.0) * (nd / dd);
    }
  } else {
    invalid = invalid || A == 0.0;
    if (!invalid) {
      if (a.estimator == SK_EST_TILDE)
        V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)p.n - 1.0);
      else
        V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);
    }
  }
  uint8_t fl;
  if (invalid) {
    V = __builtin_nan("");
    fl = SK_FLAG_INVALID;
  } else {
    double e0 = 1.0;
    if (a.estimator == SK_EST_HAT && a.window == 1) e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));
    const double E = e0 + a.expect_offset;
    const double s = a.sigma_override > 0.0 ? a.sigma_override : sqrt(4.0 / Kd);
    const double lo = E - a.k_sigma * s, hi = E + a.k_sigma * s;
    fl = (V < lo ? SK_FLAG_LOW : 0) | (V > hi ? SK_FLAG_HIGH : 0);
  }
  const int64_t o = (int64_t)f * a.n_blocks + b;
  if (a.r1) a.r1[o] = p.r1;
  if (a.r2) a.r2[o] = p.r2;
  if (a.v) a.v[o] = (float)V;
  if (a.flags) a.flags[o] = fl;
  if (a.n_eff) a.n_eff[o] = p.n;
}

__global__ __launch_bounds__(256) void combine_kernel(PassBArgs a) {
  extern __shared__ int32_t pwin[];          // [N] running window sums (L >= 2)
  __shared__ Partial wpart[4];

  const int c = blockIdx.x, f = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int N = a.n_inputs, L = a.window, H = a.hist_len;
  const int64_t total = (int64_t)H + a.n_blocks;
  int64_t e0 = (int64_t)c * a.chunk;
  if (e0 < H) e0 = H;
  int64_t e1 = (int64_t)(c + 1) * a.chunk;
  if (e1 > total) e1 = total;
  if (e0 >= e1) return;

  if (L >= 2) {
    for (int i = tid; i < N; i += 256) {
      const int64_t lo = e0 - L > 0 ? e0 - L : 0;
      pwin[i] = (int32_t)(seq_prefix(a, f, e0, i) - seq_prefix(a, f, lo, i));
    }
  }

  for (int64_t e = e0; e < e1; ++e) {
    const int b = (int)(e - H);
    Partial p = {0.0, 0.0, 0, 0, 0};
    const int32_t* r1p = a.s1 + ((int64_t)f * a.n_blocks + b) * N;
    const int32_t* r2p = a.s2 + ((int64_t)f * a.n_blocks + b) * N;
    for (int i = tid; i < N; i += 256) {
      const int32_t x1 = r1p[i], x2 = r2p[i];
      int32_t P = x1;
      if (L >= 2) {
        const int32_t old = e - L >= 0 ? seq_s1(a, f, e - L, i) : 0;
        P = pwin[i] + x1 - old;
        pwin[i] = P;
      }
      const bool use = (a.mask == nullptr || a.mask[(int64_t)f * N + i] != 0) && P > 0;
      if (use) {
        p.n += 1;
        p.r1 += x1;
        p.r2 += x2;
        if (L >= 1) {
          const double pd = (double)P;
          p.a += (double)x1 / pd;
          p.q += (double)x2 / (pd * pd);
        }
      }
    }
    p.a = wave_sum(p.a);
    p.q = wave_sum(p.q);
    p.r1 = wave_sum(p.r1);
    p.r2 = wave_sum(p.r2);
    p.n = wave_sum(p.n);
    if (lane == 0) wpart[wid] = p;
    __syncthreads();
    if (tid == 0) {
      Partial s = wpart[0];
      for (int w = 1; w < 4; ++w) {
        s.a += wpart[w].a;
        s.q += wpart[w].q;
        s.r1 += wpart[w].r1;
        s.r2 += wpart[w].r2;
        s.n += wpart[w].n;
      }
      finish(a, f, b, s);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void hist_update_kernel(PassBArgs a, int new_len) {
  const int j = blockIdx.x, f = blockIdx.y;
  const int i = blockIdx.z * 256 + threadIdx.x;
  if (i >= a.n_inputs) return;
  const int64_t e = (int64_t)a.hist_len + a.n_blocks - new_len + j;
  a.hist_next[((int64_t)f * a.hist_cap + j) * a.n_inputs + i] = seq_s1(a, f, e, i);
}

int launch_pass_b(const PassBArgs& a, hipStream_t s) {
  const int N = a.n_inputs, F = a.n_channels;
  const int ig = (N + 255) / 256;
  if (a.n_blocks <= 0) return SK_OK;
  if (a.window >= 2) {
    chunk_sum_kernel<<<dim3(a.n_chunks, F, ig), dim3(256), 0, s>>>(a);
    SK_HIP_TRY(hipGetLastError());
    chunk_scan_kernel<<<dim3(F, ig), dim3(256), 0, s>>>(a);
    SK_HIP_TRY(hipGetLastError());
  }
  const size_t lds = a.window >= 2 ? sizeof(int32_t) * (size_t)N : 0;
  if (lds > 48 * 1024) {
    static bool raised = false;
    if (!raised) {
      SK_HIP_TRY(hipFuncSetAttribute((const void*)combine_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
      raised = true;
    }
  }
  combine_kernel<<<dim3(a.n_chunks, F), dim3(256), lds, s>>>(a);
  SK_HIP_TRY(hipGetLastError());
  if (a.window >= 2) {
    const int64_t total = (int64_t)a.hist_len + a.n_blocks;
    const int new_len = (int)(total < a.hist_cap ? total : a.hist_cap);
    if (new_len > 0) {
      hist_update_kernel<<<dim3(new_len, F, ig), dim3(256), 0, s>>>(a, new_len);
      SK_HIP_TRY(hipGetLastError());
    }
  }
  return SK_OK;
}

__global__ __launch_bounds__(256) void flags_kernel(FlagArgs a) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const double V = (double)a.v[j];
  const int64_t K = (int64_t)a.n_eff[j] * a.block_len;
  uint8_t fl;
  if (K < 2 || isnan(V)) {
    fl = SK_FLAG_INVALID;
  } else {
    const double Kd = (double)K, Md = (double)a.block_len;
    double e0 = 1.0;
    if (a.estimator == SK_EST_HAT && a.window == 1) e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));
    const double E = e0 + a.expect_offset;
    const double s = a.sigma_override > 0.0 ? a.sigma_override : sqrt(4.0 / Kd);
    const double lo = E - a.k_sigma * s, hi = E + a.k_sigma * s;
    fl = (V < lo ? SK_FLAG_LOW : 0) | (V > hi ? SK_FLAG_HIGH : 0);
  }
  a.flags[j] = fl;
}

int launch_flags(const FlagArgs& a, hipStream_t s) {
  if (a.n <= 0) return SK_OK;
  const int64_t grid = (a.n + 255) / 256;
  flags_kernel<<<dim3((unsigned)grid), dim3(256), 0, s>>>(a);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

}  // namespace sk
