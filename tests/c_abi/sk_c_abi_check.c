/*
 * A plain C client of the library (no Python, no C++): it uses only the
 * public header and the HIP runtime's C API. Pure-CW input (every sample one
 * of the 12 integer points with Re^2 + Im^2 = 25) makes every input's power
 * constant, so with the block's own mean as normaliser (L = 1, Eq.
 * discreteMean) every S_i / P_i is exact and V = 0 exactly (Eq. avgSK); 0 is
 * far below E - k sigma, so every block is flagged low. Also checks the
 * error path for a block length that does not divide the samples.
 * Exit status 0 and "c abi ok" on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sk.h"

#define CHECK(cond, msg)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      fprintf(stderr, "c abi check failed: %s\n", msg);   \
      return 1;                                           \
    }                                                     \
  } while (0)

int main(void) {
  const int32_t N = 64, F = 2, M = 256;
  const int64_t T = 16 * 256;
  const int64_t B = T / M;
  static const int pts[12][2] = {{5, 0}, {-5, 0}, {0, 5}, {0, -5}, {3, 4}, {3, -4},
                                 {-3, 4}, {-3, -4}, {4, 3}, {4, -3}, {-4, 3}, {-4, -3}};
  const size_t nbytes = (size_t)T * F * N;
  uint8_t* host = (uint8_t*)malloc(nbytes);
  CHECK(host != NULL, "host allocation");
  uint64_t s = 12345;
  for (size_t k = 0; k < nbytes; ++k) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    const int j = (int)((s >> 33) % 12);
    host[k] = (uint8_t)(((pts[j][0] + 8) << 4) | (pts[j][1] + 8));
  }

  /* The error path: T not a multiple of M. */
  sk_plan_desc bad;
  memset(&bad, 0, sizeof bad);
  bad.n_inputs = N;
  bad.n_channels = F;
  bad.n_samples = T + 1;
  bad.block_len = M;
  bad.norm_window_blocks = 1;
  bad.estimator = SK_EST_HAT;
  bad.k_sigma = 5.0;
  sk_plan_t plan = NULL;
  CHECK(sk_plan_create(&bad, &plan) == SK_ERR_SHAPE && plan == NULL, "shape error expected");
  CHECK(strlen(sk_last_error()) > 0, "error message expected");

  sk_plan_desc d = bad;
  d.n_samples = T;
  CHECK(sk_plan_create(&d, &plan) == SK_OK, sk_last_error());

  uint8_t* d_x = NULL;
  float* d_v = NULL;
  uint8_t* d_flags = NULL;
  int32_t* d_neff = NULL;
  CHECK(hipMalloc((void**)&d_x, nbytes) == hipSuccess, "hipMalloc input");
  CHECK(hipMalloc((void**)&d_v, sizeof(float) * F * B) == hipSuccess, "hipMalloc v");
  CHECK(hipMalloc((void**)&d_flags, (size_t)F * B) == hipSuccess, "hipMalloc flags");
  CHECK(hipMalloc((void**)&d_neff, sizeof(int32_t) * F * B) == hipSuccess, "hipMalloc n_eff");
  CHECK(hipMemcpy(d_x, host, nbytes, hipMemcpyHostToDevice) == hipSuccess, "copy input");

  sk_outputs o;
  memset(&o, 0, sizeof o);
  o.v = d_v;
  o.flags = d_flags;
  o.n_eff = d_neff;
  for (int call = 0; call < 2; ++call) CHECK(sk_compute(plan, d_x, NULL, &o, NULL) == SK_OK, sk_last_error());
  CHECK(hipDeviceSynchronize() == hipSuccess, "synchronize");

  float v[2 * 16];
  uint8_t fl[2 * 16];
  int32_t ne[2 * 16];
  CHECK(hipMemcpy(v, d_v, sizeof v, hipMemcpyDeviceToHost) == hipSuccess, "copy v");
  CHECK(hipMemcpy(fl, d_flags, sizeof fl, hipMemcpyDeviceToHost) == hipSuccess, "copy flags");
  CHECK(hipMemcpy(ne, d_neff, sizeof ne, hipMemcpyDeviceToHost) == hipSuccess, "copy n_eff");
  for (int k = 0; k < F * B; ++k) {
    CHECK(v[k] == 0.0f, "V is exactly 0 for constant power");
    CHECK(fl[k] == SK_FLAG_LOW, "every block flagged low");
    CHECK(ne[k] == N, "every input used");
  }
  CHECK(sk_plan_destroy(plan) == SK_OK, "destroy");
  hipFree(d_x);
  hipFree(d_v);
  hipFree(d_flags);
  hipFree(d_neff);
  free(host);
  printf("c abi ok\n");
  return 0;
}
