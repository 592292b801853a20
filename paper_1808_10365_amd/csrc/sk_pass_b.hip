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
// Kernels:
//   chunk_sum_kernel   (L > 16) sum of S1 over each chunk of R consecutive e;
//                      shorter windows are summed from their rows.
//   partial_kernel     one wavefront per (chunk, channel, 64*V inputs): the
//                      window start of the chunk from chunk sums plus fewer
//                      than R edge reads, then per block the sliding update
//                      P += S1[e] - S1[e-L] and the lane's FP64 A, Bq and
//                      int64 R1, R2 over its V inputs, a butterfly reduction
//                      across the wavefront, one partial per (block, group).
//                      It also writes the blocks that form the next history.
//   finalize_kernel    one thread per (channel, block): sums the partials in
//                      group order, then the estimator and the flags.
//   hist_copy_kernel   only when a call has fewer than L-1 blocks: carries the
//                      still-needed old history entries forward.
// Every sum runs in a fixed order (lane-sequential, butterfly, group order),
// so results are identical from call to call.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sk_internal.h"
#include "sk_pass_b_dev.h"

namespace sk {

__global__ __launch_bounds__(256) void chunk_sum_kernel_1(PassBArgs a) { chunk_sum_body<1>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z); }
__global__ __launch_bounds__(256) void chunk_sum_kernel_4(PassBArgs a) { chunk_sum_body<4>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z); }
__global__ __launch_bounds__(256) void partial_kernel_1(PassBArgs a) { partial_body<1>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z); }
template <int D>
__global__ __launch_bounds__(256) void partial_kernel_4(PassBArgs a) {
  partial_body<4, D>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z);
}
__global__ __launch_bounds__(256) void chunk_sum_kernel_8(PassBArgs a) { chunk_sum_body<8>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z); }
__global__ __launch_bounds__(256) void partial_kernel_8(PassBArgs a) { partial_body<8>(a, a.chunk0 + blockIdx.x, blockIdx.y, blockIdx.z); }
__global__ __launch_bounds__(256) void finalize_kernel(PassBArgs a) { finalize_body(a, blockIdx.x); }
// Partial sums and estimator together: one workgroup per (chunk, channel),
// one wavefront per input group.
template <int V, int D>
__global__ __launch_bounds__(64 * MAX_FIN_GROUPS) void partial_finish_kernel(PassBArgs a) {
  partial_body<V, D, true>(a, a.chunk0 + blockIdx.x, blockIdx.y, 0);
}
__global__ __launch_bounds__(256) void hist_copy_kernel(PassBArgs a) { hist_copy_body(a, blockIdx.x, blockIdx.y, blockIdx.z); }

template <int V>
static int launch_v(const PassBArgs& a0, int32_t c_begin, int32_t c_end, int32_t b_begin, int32_t b_end,
                    bool with_hist_copy, hipStream_t s) {
  PassBArgs a = a0;
  const int F = a.n_channels;
  const int nc = c_end - c_begin;
  a.chunk0 = c_begin;
  a.fin_b0 = b_begin;
  a.fin_nb = b_end - b_begin;
  const int zc = (a.n_inputs + 256 * V - 1) / (256 * V);
  if (a.window >= 2) {
    if (nc > 0 && a.window > SHORT_WINDOW) {
      if (V == 8) chunk_sum_kernel_8<<<dim3(nc, F, zc), dim3(256), 0, s>>>(a);
      else if (V == 4) chunk_sum_kernel_4<<<dim3(nc, F, zc), dim3(256), 0, s>>>(a);
      else chunk_sum_kernel_1<<<dim3(nc, F, zc), dim3(256), 0, s>>>(a);
      SK_HIP_TRY(hipGetLastError());
    }
    const int n_old = a.hist_next_len - a.n_blocks;
    if (with_hist_copy && n_old > 0) {
      hist_copy_kernel<<<dim3(n_old, F, (a.n_inputs + 255) / 256), dim3(256), 0, s>>>(a);
      SK_HIP_TRY(hipGetLastError());
    }
  }
  // A whole call whose channels fit one workgroup of at most 4 wavefronts:
  // partial sums and estimator in one launch, no per-group partials in
  // memory. Wider channels keep the separate finalize launch: their 8-wave
  // workgroups, tied by the barriers, retire later than independent 4-wave
  // ones, which costs what the launch saves (CHIME M = 256: 40.6 us against
  // 34.8 + 4.6).
  const bool whole = c_begin == 0 && c_end == a.n_chunks && b_begin == 0 && b_end == a.n_blocks;
  if (whole && nc > 0 && a.n_groups <= MAX_FIN_GROUPS) {
    const dim3 grid(nc, F), wg(64 * a.n_groups);
    if (V == 8) partial_finish_kernel<8, 4><<<grid, wg, 0, s>>>(a);
    else if (V == 4 && a.depth == 8) partial_finish_kernel<4, 8><<<grid, wg, 0, s>>>(a);
    else if (V == 4 && a.depth == 2) partial_finish_kernel<4, 2><<<grid, wg, 0, s>>>(a);
    else if (V == 4) partial_finish_kernel<4, 4><<<grid, wg, 0, s>>>(a);
    else partial_finish_kernel<1, 4><<<grid, wg, 0, s>>>(a);
    SK_HIP_TRY(hipGetLastError());
    return SK_OK;
  }
  if (nc > 0) {
    if (V == 8) partial_kernel_8<<<dim3(nc, F, (a.n_groups + 3) / 4), dim3(256), 0, s>>>(a);
    else if (V == 4 && a.depth == 8) partial_kernel_4<8><<<dim3(nc, F, (a.n_groups + 3) / 4), dim3(256), 0, s>>>(a);
    else if (V == 4 && a.depth == 2) partial_kernel_4<2><<<dim3(nc, F, (a.n_groups + 3) / 4), dim3(256), 0, s>>>(a);
    else if (V == 4) partial_kernel_4<4><<<dim3(nc, F, (a.n_groups + 3) / 4), dim3(256), 0, s>>>(a);
    else partial_kernel_1<<<dim3(nc, F, (a.n_groups + 3) / 4), dim3(256), 0, s>>>(a);
    SK_HIP_TRY(hipGetLastError());
  }
  const int64_t fb = (int64_t)F * a.fin_nb;
  if (fb > 0) {
    finalize_kernel<<<dim3((unsigned)((fb + 255) / 256)), dim3(256), 0, s>>>(a);
    SK_HIP_TRY(hipGetLastError());
  }
  return SK_OK;
}

int pass_b_vec(int32_t n_inputs) { return n_inputs % 4 == 0 ? 4 : 1; }

int launch_pass_b_range(PassBArgs a, int32_t c_begin, int32_t c_end, int32_t b_begin, int32_t b_end,
                        bool with_hist_copy, hipStream_t s) {
  if (a.n_blocks <= 0) return SK_OK;
  if (a.vec == 8) return launch_v<8>(a, c_begin, c_end, b_begin, b_end, with_hist_copy, s);
  if (a.vec == 4) return launch_v<4>(a, c_begin, c_end, b_begin, b_end, with_hist_copy, s);
  return launch_v<1>(a, c_begin, c_end, b_begin, b_end, with_hist_copy, s);
}

int launch_pass_b(const PassBArgs& a, hipStream_t s) {
  return launch_pass_b_range(a, 0, a.n_chunks, 0, a.n_blocks, true, s);
}

__global__ __launch_bounds__(256) void flags_kernel(FlagArgs a) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.n) return;
  const double V = (double)a.v[j];
  const int64_t K = (int64_t)a.n_eff[j] * a.block_len;
  uint8_t fl;
  if (K < 2 || isnan(V) || (a.thresholds && a.n_eff[j] > a.n_max)) {
    fl = SK_FLAG_INVALID;
  } else {
    const double Kd = (double)K, Md = (double)a.block_len;
    double e0 = 1.0;
    if (a.estimator == SK_EST_HAT && a.window == 1) e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));
    const double E = e0 + a.expect_offset;
    const double s = a.sigma_override > 0.0 ? a.sigma_override : sqrt(4.0 / Kd);
    double lo = E - a.k_sigma * s, hi = E + a.k_sigma * s;
    if (a.thresholds) {
      lo = a.thresholds[2 * a.n_eff[j]];
      hi = a.thresholds[2 * a.n_eff[j] + 1];
    }
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
