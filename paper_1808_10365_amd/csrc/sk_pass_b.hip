// Pass B: normaliser window, array combine, estimator and flags
// (Eq. discreteMean, normedSum1, normedSum2, avgSK, final; Sec. 3.2).
//
// The normaliser of block b is the window sum P = sum of S1 over b - L + 1 .. b
// (Eq. discreteMean is L = 1: the block's own power). Its common factor (M
// times the number of blocks in the window) is the same for every input of a
// (channel, block) and cancels in the estimator, so the weights are 1/P_i
// (Eq. normedSum1, normedSum2). The kernels are described in
// sk_pass_b_dev.h: a prefix scan of S1 over chunk boundaries (L >= 2), then
// one combine workgroup per (channel, chunk) that finishes its blocks.
// Every sum runs in a fixed order (lane-sequential, the fixed wavefront tree,
// wavefronts in order), so results are identical from call to call and do not
// depend on the chunk length.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sk_internal.h"
#include "sk_pass_b_dev.h"

namespace sk {

template <int R>
__global__ __launch_bounds__(64 * SCAN_MAX_WAVES) void scan_kernel(PassBArgs a) {
  __shared__ uint32_t lds[SCAN_MAX_WAVES * 64];
  scan_body<R>(a, blockIdx.y, blockIdx.x, wave_id(), blockDim.x >> 6, lds);
}

template <int V, int R, typename RI, bool OFF32>
__global__ __launch_bounds__(64 * COMBINE_MAX_WAVES) void combine_kernel(PassBArgs a) {
  __shared__ CombineShared sh;
  combine_body<V, R, RI, OFF32>(a, blockIdx.x, blockIdx.y, wave_id(), blockDim.x >> 6, sh);
}

template <int V, int R>
static void launch_combine_r(const PassBArgs& a, bool fit32, dim3 grid, dim3 wg, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
  const bool off32 = combine_offsets_fit_32(a.n_inputs, a.n_blocks, a.n_chunks, a.hist_cap);
  if (fit32 && off32) launch_kernel(combine_kernel<V, R, int32_t, true>, grid, wg, 0, s, e0, e1, a);
  else if (fit32) launch_kernel(combine_kernel<V, R, int32_t, false>, grid, wg, 0, s, e0, e1, a);
  else if (off32) launch_kernel(combine_kernel<V, R, int64_t, true>, grid, wg, 0, s, e0, e1, a);
  else launch_kernel(combine_kernel<V, R, int64_t, false>, grid, wg, 0, s, e0, e1, a);
}

template <int V>
static int launch_combine_v(const PassBArgs& a, bool fit32, dim3 grid, dim3 wg, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
  switch (a.chunk) {
    case 1: launch_combine_r<V, 1>(a, fit32, grid, wg, s, e0, e1); break;
    case 2: launch_combine_r<V, 2>(a, fit32, grid, wg, s, e0, e1); break;
    case 4: launch_combine_r<V, 4>(a, fit32, grid, wg, s, e0, e1); break;
    default:
      set_error("pass B: chunk length %d is not 1, 2 or 4", a.chunk);
      return SK_ERR_INVALID_ARG;
  }
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

int launch_pass_b(const PassBArgs& a, hipStream_t s, PassEvents ev) {
  if (a.n_blocks <= 0) return SK_OK;
  const int F = a.n_channels;
  hipEvent_t start = ev.start;
  if (pass_b_needs_scan(a.window, a.chunk, a.n_blocks)) {
    // Enough wavefronts for the chunks, or for the history rows a call
    // shorter than the window moves.
    const int64_t sg = shift_groups(a.hist_next_len, a.n_blocks);
    const dim3 grid((a.n_inputs + 63) / 64, F), wg(64 * scan_waves(sg > a.n_chunks ? (int)sg : a.n_chunks));
    switch (a.chunk) {
      case 1: launch_kernel(scan_kernel<1>, grid, wg, 0, s, start, nullptr, a); break;
      case 2: launch_kernel(scan_kernel<2>, grid, wg, 0, s, start, nullptr, a); break;
      case 4: launch_kernel(scan_kernel<4>, grid, wg, 0, s, start, nullptr, a); break;
      default:
        set_error("pass B: chunk length %d is not 1, 2 or 4", a.chunk);
        return SK_ERR_INVALID_ARG;
    }
    SK_HIP_TRY(hipGetLastError());
    start = nullptr;
  }
  const dim3 grid(a.n_chunks, F), wg(64 * combine_waves(a.n_inputs, a.vec));
  const bool fit32 = combine_sums_fit_32(a.n_inputs, a.vec, a.block_len);
  if (a.vec == 4) return launch_combine_v<4>(a, fit32, grid, wg, s, start, ev.stop);
  return launch_combine_v<1>(a, fit32, grid, wg, s, start, ev.stop);
}

int pass_b_vec(int32_t n_inputs) { return n_inputs % 4 == 0 ? 4 : 1; }

int pass_b_chunk(int32_t n_inputs, int32_t n_channels, int64_t n_blocks, int32_t window) {
  // Four blocks per combine workgroup, fewer while there are too few
  // wavefronts to fill the device (at least ~4 per SIMD).
  const int64_t waves_per_chunk = combine_waves(n_inputs, pass_b_vec(n_inputs));
  int R = 4;
  while (R > 1 && ((n_blocks + R - 1) / R) * n_channels * waves_per_chunk < 4096) R /= 2;
  (void)window;
  return R;
}

size_t pass_b_prefix_bytes(int32_t n_inputs, int32_t n_channels, int64_t n_blocks, int32_t chunk) {
  return (size_t)n_channels * (size_t)((n_blocks + chunk - 1) / chunk + 1) * (size_t)n_inputs * sizeof(uint32_t);
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
