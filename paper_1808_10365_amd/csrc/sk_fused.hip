// Single-launch path for wide rows that fill one round of CUs: one
// cooperative kernel, one 512-lane workgroup per segment of Q consecutive
// blocks (workgroup w owns blocks w*Q .. w*Q+Q-1 and all column groups of
// the row, at most 512 groups of 16 inputs).
//
//   phase 1  the deferred-store walk of pass A (Eq. singlesums): every
//            block's S1/S2 stay in registers and are stored after the last
//            block; the segment's S1 sum per input is written too.
//   -- grid sync --
//   phase 2  per input, the exclusive prefix of the segment sums over
//            segments, and the suffix sums of the history rows (the S1 of
//            the previous calls' last blocks still inside the window).
//   -- grid sync --
//   phase 3  each workgroup finishes its own blocks: the window
//            P_i[b] = sum of S1_i over blocks b-L+1..b (Eq. discreteMean for
//            L = 1, here L >= 2) from its registers, one prefix vector and at
//            most Q rows of S1 (or one history suffix vector); the combine
//            A = sum S1/P, Bq = sum S2/P^2, R1, R2, N_eff (Eq. normedSum1,
//            normedSum2) within the workgroup, V and flags (Eq. avgSK;
//            Sec. 3.2); the rows of the next history.
//
// Compared with pass A + pass B this removes pass B's second read of S1/S2
// and its three dependent launches. Prefix arithmetic is modulo 2^32: every
// window sum P is below 2^31 (checked at plan creation), so differences of
// wrapped prefixes are exact.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "sk_internal.h"
#include "sk_pass_a_dev.h"
#include "sk_pass_b_dev.h"

namespace sk {

namespace cgrp = cooperative_groups;

constexpr int FUSED_WG = 512;

// Loads 16 consecutive int32 (16-byte aligned).
__device__ __forceinline__ void load16(const int32_t* p, uint32_t* v) {
#pragma unroll
  for (int k = 0; k < 16; k += 4) {
    const u32x4 q = *reinterpret_cast<const u32x4*>(p + k);
    v[k] = q.x; v[k + 1] = q.y; v[k + 2] = q.z; v[k + 3] = q.w;
  }
}

__device__ __forceinline__ void store16(int32_t* p, const uint32_t* v) {
#pragma unroll
  for (int k = 0; k < 16; k += 4)
    *reinterpret_cast<u32x4*>(p + k) = u32x4{v[k], v[k + 1], v[k + 2], v[k + 3]};
}

// In-workgroup exclusive/inclusive scans for phase 2: 16 lanes per input,
// lane `part` holds the total of its part; returns the sum of the parts
// before it (prefix) or after it (suffix). red: LDS scratch [32][17].
__device__ __forceinline__ uint32_t parts_before(uint32_t* red, int ii, int part, uint32_t total) {
  red[ii * 17 + part] = total;
  __syncthreads();
  uint32_t s = 0;
  for (int p = 0; p < part; ++p) s += red[ii * 17 + p];
  __syncthreads();
  return s;
}

__device__ __forceinline__ uint32_t parts_after(uint32_t* red, int ii, int part, uint32_t total) {
  red[ii * 17 + part] = total;
  __syncthreads();
  uint32_t s = 0;
  for (int p = part + 1; p < 16; ++p) s += red[ii * 17 + p];
  __syncthreads();
  return s;
}

template <int Q>
__global__ __launch_bounds__(FUSED_WG) void fused_kernel(FusedArgs fa) {
  constexpr int VEC = 16;
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  __shared__ double red_a[FUSED_WG / 64], red_q[FUSED_WG / 64];
  __shared__ int64_t red_r1[FUSED_WG / 64], red_r2[FUSED_WG / 64];
  __shared__ int32_t red_n[FUSED_WG / 64];
  __shared__ uint32_t red_scan[32 * 17];

  const PassATask& t = fa.a;
  const PassBArgs& a = fa.b;
  const int tid = threadIdx.x;
  const int w = blockIdx.x;
  const int N = a.n_inputs, B = a.n_blocks, M = a.block_len;
  const int H = a.hist_len, L = a.window;
  const int64_t G = t.row_bytes;
  const int64_t Cn = (int64_t)a.n_channels * N;     // inputs per row
  const int g = tid;                                  // column group
  const bool active = g < t.col_groups;
  const int64_t col = (int64_t)g * VEC;
  const int f = active ? (int)(col / N) : 0;
  const int i = active ? (int)(col % N) : 0;
  const int b0 = w * Q;
  cgrp::grid_group grid = cgrp::this_grid();

  // ---- phase 1: stream the segment's blocks.
  fill_lane_packed_lut<FUSED_WG>(lut32, tid);
  __syncthreads();
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  uint32_t a1[Q][VEC], a2[Q][VEC];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) a1[q][k] = a2[q][k] = 0;
    if (active && b0 + q < B)
      sum_rows_packed<VEC, 1, 16>(t.x + (int64_t)(b0 + q) * M * G + col, G, M, 0, lut, a1[q], a2[q]);
  }
  if (active) {
    uint32_t seg[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) seg[k] = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (b0 + q >= B) continue;
      const int64_t o = ((int64_t)f * B + b0 + q) * N + i;
      store16(t.s1 + o, a1[q]);
      if (t.s2) store16(t.s2 + o, a2[q]);
#pragma unroll
      for (int k = 0; k < VEC; ++k) seg[k] += a1[q][k];
    }
    store16(fa.segsum + (int64_t)w * Cn + col, seg);
  }
  __threadfence();
  grid.sync();

  // ---- phase 2: scans. Workgroup w handles inputs [w*S, w*S + S), 32 at a
  // time, 16 lanes per input, each lane one part of the segments / history
  // rows.
  {
    const int S = (int)((Cn + gridDim.x - 1) / gridDim.x);
    for (int base = 0; base < S; base += 32) {
      // Consecutive lanes take consecutive inputs (coalesced rows of the
      // segment sums and of the history); the 16 parts are 32 lanes apart.
      const int ii = tid % 32, part = tid / 32;
      const int64_t in = (int64_t)w * S + base + ii;
      const bool ok = base + ii < S && in < Cn;
      // exclusive prefix of segment sums
      const int nseg = gridDim.x;
      const int per = (nseg + 15) / 16;
      const int s0 = part * per, s1e = s0 + per < nseg ? s0 + per : nseg;
      uint32_t tot = 0;
      if (ok)
        for (int s = s0; s < s1e; ++s) tot += (uint32_t)fa.segsum[(int64_t)s * Cn + in];
      uint32_t run = parts_before(red_scan, ii, part, tot);
      if (ok)
        for (int s = s0; s < s1e; ++s) {
          fa.segpre[(int64_t)s * Cn + in] = (int32_t)run;
          run += (uint32_t)fa.segsum[(int64_t)s * Cn + in];
        }
      // suffix sums of the history rows: hsuf[j] = sum of hist rows j..H-1
      if (H > 0) {
        const int fi = ok ? (int)(in / N) : 0, ni = ok ? (int)(in % N) : 0;
        const int hper = (H + 15) / 16;
        const int h0 = part * hper, h1 = h0 + hper < H ? h0 + hper : H;
        uint32_t htot = 0;
        if (ok)
          for (int j = h0; j < h1; ++j) htot += (uint32_t)a.hist[((int64_t)fi * a.hist_cap + j) * N + ni];
        uint32_t suf = parts_after(red_scan, ii, part, htot);
        if (ok)
          for (int j = h1 - 1; j >= h0; --j) {
            suf += (uint32_t)a.hist[((int64_t)fi * a.hist_cap + j) * N + ni];
            fa.hsuf[(int64_t)j * Cn + in] = (int32_t)suf;
          }
      }
    }
  }
  __threadfence();
  grid.sync();

  // ---- phase 3: windows, combine, estimator and flags for own blocks.
  const int total = H + B;
  const int hist_from = total - a.hist_next_len;           // first position of the next history
  uint32_t use_mask = 0;
  uint32_t cur[VEC];
  if (active) {
#pragma unroll
    for (int k = 0; k < VEC; ++k)
      if (a.mask == nullptr || a.mask[(int64_t)f * N + i + k] != 0) use_mask |= 1u << k;
    load16(fa.segpre + (int64_t)w * Cn + col, cur);
  }
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = b0 + q;
    if (b >= B) break;                                     // uniform over the workgroup
    double pa = 0.0, pq = 0.0;
    int64_t r1 = 0, r2 = 0;
    int32_t n = 0;
    if (active) {
      // low[k]: prefix of S1 through the position just below the window.
      uint32_t low[VEC];
      const int x = H + b - L;                             // last position outside the window
      if (x >= H) {
        const int bx = x - H, wx = bx / Q, qx = bx % Q;
        load16(fa.segpre + (int64_t)wx * Cn + col, low);
        for (int qq = 0; qq <= qx; ++qq) {
          uint32_t r[VEC];
          load16(t.s1 + ((int64_t)f * B + wx * Q + qq) * N + i, r);
#pragma unroll
          for (int k = 0; k < VEC; ++k) low[k] += r[k];
        }
      } else {
        // The window reaches into the history (or before the stream start):
        // P = (history rows from max(x + 1, 0) on) + (current blocks 0..b).
        const int j = x + 1 > 0 ? x + 1 : 0;
        uint32_t hs[VEC];
        if (j < H) load16(fa.hsuf + (int64_t)j * Cn + col, hs);
        else {
#pragma unroll
          for (int k = 0; k < VEC; ++k) hs[k] = 0;
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) low[k] = 0u - hs[k];
      }
#pragma unroll
      for (int k = 0; k < VEC; ++k) cur[k] += a1[q][k];
      float ski[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const int32_t P = (int32_t)(cur[k] - low[k]);
        const int32_t x1 = (int32_t)a1[q][k], x2 = (int32_t)a2[q][k];
        if (a.sk_i) ski[k] = per_input_sk(x1, x2, M);
        if ((use_mask >> k & 1u) && P > 0) {
          n += 1;
          r1 += x1;
          r2 += x2;
          const double rp = recip_pos((double)P);
          pa += (double)x1 * rp;
          pq += (double)x2 * rp * rp;
        }
      }
      if (a.sk_i) {
        float* dst = a.sk_i + ((int64_t)f * B + b) * N + i;
#pragma unroll
        for (int k = 0; k < VEC; ++k) dst[k] = ski[k];
      }
      const int e = H + b;
      if (e >= hist_from)
        store16(a.hist_next + ((int64_t)f * a.hist_cap + (e - hist_from)) * N + i, a1[q]);
    }
    pa = wave_sum_to_last(pa);
    pq = wave_sum_to_last(pq);
    r1 = wave_sum_to_last(r1);
    r2 = wave_sum_to_last(r2);
    n = wave_sum_to_last(n);
    if (lane == 63) {
      red_a[wave] = pa;
      red_q[wave] = pq;
      red_r1[wave] = r1;
      red_r2[wave] = r2;
      red_n[wave] = n;
    }
    __syncthreads();
    // One thread per channel sums its wavefronts in order (each wavefront's
    // 1024 inputs lie in one channel: N % 1024 == 0).
    const int waves_per_ch = N / 1024;
    if (tid < a.n_channels) {
      double A = 0.0, Bq = 0.0;
      int64_t R1 = 0, R2 = 0;
      int32_t nn = 0;
      for (int v = tid * waves_per_ch; v < (tid + 1) * waves_per_ch; ++v) {
        A += red_a[v];
        Bq += red_q[v];
        R1 += red_r1[v];
        R2 += red_r2[v];
        nn += red_n[v];
      }
      finish(a, tid, b, A, Bq, R1, R2, nn);
    }
    __syncthreads();
  }

  // Old history rows that stay in the window of the next call (a call
  // shorter than the window): positions hist_from .. H-1, spread over the
  // workgroups.
  if (active && hist_from < H) {
    for (int e = hist_from + w; e < H; e += gridDim.x) {
      uint32_t r[VEC];
      load16(a.hist + ((int64_t)f * a.hist_cap + e) * N + i, r);
      store16(a.hist_next + ((int64_t)f * a.hist_cap + (e - hist_from)) * N + i, r);
    }
  }
}

int fused_max_workgroups() {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fused_kernel<4>, FUSED_WG, 0) != hipSuccess) return 0;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return occ * ncu;
}

int launch_fused(const FusedArgs& fa, int q, hipStream_t s) {
  const int grid = (fa.b.n_blocks + q - 1) / q;
  void* args[] = {const_cast<FusedArgs*>(&fa)};
  hipError_t e;
  switch (q) {
    case 1: e = hipLaunchCooperativeKernel((const void*)fused_kernel<1>, dim3(grid), dim3(FUSED_WG), args, 0, s); break;
    case 2: e = hipLaunchCooperativeKernel((const void*)fused_kernel<2>, dim3(grid), dim3(FUSED_WG), args, 0, s); break;
    case 3: e = hipLaunchCooperativeKernel((const void*)fused_kernel<3>, dim3(grid), dim3(FUSED_WG), args, 0, s); break;
    case 4: e = hipLaunchCooperativeKernel((const void*)fused_kernel<4>, dim3(grid), dim3(FUSED_WG), args, 0, s); break;
    default:
      set_error("fused path: 1..4 blocks per workgroup, got %d", q);
      return SK_ERR_INVALID_ARG;
  }
  if (e != hipSuccess) {
    set_error("cooperative launch failed: %s", hipGetErrorString(e));
    return SK_ERR_DEVICE;
  }
  return SK_OK;
}

}  // namespace sk
