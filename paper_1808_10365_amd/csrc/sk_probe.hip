// Read-only streaming probe: the practical HBM read ceiling that streaming
// kernels such as pass A are measured against. Each workgroup reads one
// contiguous slab with 16-byte nontemporal loads (8 per lane in flight) and
// folds them with XOR; one word per lane is written so no load is removed.
#include <hip/hip_runtime.h>

#include "sk_internal.h"
#include "sk_profile.h"

namespace sk {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32x4 ld16(const uint8_t* x, int64_t k) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) u32x4*)(x + k * 16));
}

__global__ __launch_bounds__(256) void read_probe_kernel(const uint8_t* x, int64_t n16, int64_t per_wg,
                                                         uint32_t* sink) {
  const int64_t w0 = (int64_t)blockIdx.x * per_wg;
  const int64_t w1 = w0 + per_wg < n16 ? w0 + per_wg : n16;
  u32x4 acc = {0, 0, 0, 0};
  int64_t k = w0 + threadIdx.x;
  for (; k + 7 * 256 < w1; k += 8 * 256) {
    u32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld16(x, k + u * 256);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc ^= v[u];
  }
  for (; k < w1; k += 256) acc ^= ld16(x, k);
  sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

}  // namespace
}  // namespace sk

extern "C" int sk_read_probe(const uint8_t* d_x, int64_t bytes, int32_t workgroups, uint32_t* d_sink,
                             void* stream) {
  using namespace sk;
  clear_error();
  if (!d_x || !d_sink || bytes < 0 || workgroups < 1 || bytes % 16 != 0 ||
      reinterpret_cast<uintptr_t>(d_x) % 16 != 0) {
    set_error("sk_read_probe: need a 16-byte aligned buffer, bytes %% 16 == 0 and workgroups >= 1");
    return SK_ERR_INVALID_ARG;
  }
  if (bytes == 0) return SK_OK;
  const int64_t n16 = bytes / 16;
  const int64_t per_wg = (n16 + workgroups - 1) / workgroups;
  read_probe_kernel<<<dim3(workgroups), dim3(256), 0, (hipStream_t)stream>>>(d_x, n16, per_wg, d_sink);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}
