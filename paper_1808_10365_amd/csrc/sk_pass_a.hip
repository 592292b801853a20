// Pass A: per-input block sums of power and square power (Eq. singlesums).
//
// The input is one byte per complex sample, [T][F][N] (time-major, inputs
// innermost). Each lane owns VEC consecutive inputs of one channel and walks
// the rows (time samples) of a block with one VEC-byte nontemporal load per
// row, so a wavefront reads 64*VEC contiguous bytes per row. Power comes from
// a 256-entry LDS table indexed by the byte (Re and Im decoded from the
// nibbles, Sec. 2.2.3 "Calculating Power"). Two rows' powers are packed into
// the 16-bit halves of one register; v_dot2_u32_u16 then adds p0^2 + p1^2 to
// the S2 accumulator and p0 + p1 (dot with (1,1)) to S1, so each sample costs
// one byte extract, one LDS read and one dot-lane. Sums are exact in 32 bits:
// p <= 128, so S2 <= M * 2^14 < 2^31 for M <= 131071.
//
// The shared 512-byte table makes the 64 lookups of a wavefront collide in
// LDS banks whenever codes differ in the right bits; the lane-replicated
// table (64 KiB, one 256-byte row per code with a dword slot per lane) is
// conflict-free and its address is one v_perm_b32 of the code byte and the
// lane's slot. Wide rows use it by default with one 256-lane row phase.
#include <hip/hip_runtime.h>

#include "sk_internal.h"
#include "sk_pass_a_dev.h"

namespace sk {

// Workgroup size: 256 lanes, or LPR lanes (512, 1024) when a workgroup spans
// a whole wide row with one row phase (one contiguous slab per block).
template <int LPR>
constexpr int wg_size() { return LPR > 256 ? LPR : 256; }

// Stores one lane's sums of column group g (VEC inputs) for block b.
template <int VEC>
__device__ __forceinline__ void store_group(const PassATask& t, int b, int g, const uint32_t* s1,
                                            const uint32_t* s2) {
  const int N = t.n_inputs;
  const int B = t.n_blocks;
  const int64_t col = (int64_t)g * VEC;
  const int64_t f = col / N, i = col % N;
  int32_t* d1 = t.s1 + (f * B + b) * N + i;
  int32_t* d2 = t.s2 + (f * B + b) * N + i;
  if constexpr (VEC >= 4) {
#pragma unroll
    for (int k = 0; k < VEC; k += 4) {
      u32x4 a = {s1[k], s1[k + 1], s1[k + 2], s1[k + 3]};
      u32x4 c = {s2[k], s2[k + 1], s2[k + 2], s2[k + 3]};
      // Plain stores: nontemporal ones measured far slower here (the sums
      // then reach HBM as scattered partial writes).
      *reinterpret_cast<u32x4*>(d1 + k) = a;
      *reinterpret_cast<u32x4*>(d2 + k) = c;
    }
  } else {
    d1[0] = (int32_t)s1[0];
    d2[0] = (int32_t)s2[0];
  }
}

// One task is (block b, chunk ch) of LPR * GPL column groups. Lane lc of
// row phase ph owns groups ch * LPR * GPL + j * LPR + lc (j < GPL), so for
// every j a wavefront's loads of one row are 64 * VEC contiguous bytes.
//
// REP selects the lane-replicated 64 KiB power table (16-byte lanes only):
// bank-conflict free whatever the codes, at the price of LDS that limits a
// CU to two workgroups. With several row phases the table's LDS is reused
// for their reduction (S1, then S2) and refilled if the workgroup takes
// another task.
// PACKED (with REP, one row phase, one group per lane): the packed lane
// table, one add per sample for both sums.
template <int VEC, int LPR, int U, bool PF, int GPL, bool REP, int WG = wg_size<LPR>(), bool PACKED = false>
__global__ __launch_bounds__(WG) void pass_a_kernel(PassATask t) {
  constexpr int RP = WG / LPR;          // row phases per workgroup
  constexpr int W = 2 * VEC + 1;        // LDS stride of one lane's partials (odd: no bank conflicts)
  static_assert(WG % LPR == 0, "whole row phases");
  static_assert(!REP || (VEC == 16 && (RP == 1 || WG * (VEC + 1) <= LANE_LUT_DWORDS)),
                "lane table: 16-byte lanes; the row-phase reduction must fit in the table's LDS");
  __shared__ uint16_t lut16[REP ? 1 : 256];
  __shared__ __attribute__((aligned(16))) uint32_t lut32[REP ? LANE_LUT_DWORDS : 1];
  extern __shared__ uint32_t red[];     // [RP * LPR][W] when RP > 1

  static_assert(!PACKED || (REP && RP == 1 && GPL == 1), "packed table: one row phase, one group per lane");
  const int tid = threadIdx.x;
  if constexpr (PACKED) {
    fill_lane_packed_lut<WG>(lut32, tid);
  } else if constexpr (REP) {
    fill_lane_lut<WG>(lut32, tid);
  } else {
    for (int k = tid; k < 256; k += WG) lut16[k] = (uint16_t)code_power((uint32_t)k);
  }
  __syncthreads();
  const LaneLut llut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  const LanePackedLut plut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};

  const int lc = tid % LPR;
  const int ph = tid / LPR;
  const int M = t.block_len;
  const int64_t G = t.row_bytes;

  if constexpr (PACKED) {
    // A task walks blocks_per_task consecutive blocks (contiguous rows) of
    // one column chunk, storing each block's sums as it ends.
    const int Q = t.blocks_per_task;
    for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
      const int b_first = t.block0 + (int)(task / t.chunks) * Q;
      const int ch = (int)(task % t.chunks);
      const int g0 = ch * LPR + lc;
      if (g0 >= t.col_groups) continue;
      for (int b = b_first; b < b_first + Q && b < t.block_end; ++b) {
        uint32_t s1[VEC], s2[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) s1[k] = s2[k] = 0;
        sum_rows_packed<VEC, RP, U>(t.x + (int64_t)b * M * G + (int64_t)g0 * VEC, G, M, ph, plut, s1, s2);
        store_group<VEC>(t, b, g0, s1, s2);
      }
    }
    return;
  }

  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
    const int b = t.block0 + (int)(task / t.chunks);
    const int ch = (int)(task % t.chunks);
    const int g0 = ch * LPR * GPL + lc;
    uint32_t s1[GPL][VEC], s2[GPL][VEC];
#pragma unroll
    for (int j = 0; j < GPL; ++j)
#pragma unroll
      for (int k = 0; k < VEC; ++k) s1[j][k] = s2[j][k] = 0;

    if (g0 < t.col_groups) {
      const uint8_t* blk = t.x + (int64_t)b * M * G;
      if constexpr (GPL == 1 && REP) {
        sum_rows<VEC, RP, U, PF>(blk + (int64_t)g0 * VEC, G, M, ph, llut, s1[0], s2[0]);
      } else if constexpr (GPL == 1) {
        sum_rows<VEC, RP, U, PF>(blk + (int64_t)g0 * VEC, G, M, ph, lut16, s1[0], s2[0]);
      } else {
        // A group past the row's end walks group g0 again (in bounds); its
        // sums are discarded below.
        const uint8_t* base[GPL];
#pragma unroll
        for (int j = 0; j < GPL; ++j) {
          const int g = g0 + j * LPR;
          base[j] = blk + (int64_t)(g < t.col_groups ? g : g0) * VEC;
        }
        if constexpr (REP)
          sum_rows_multi<VEC, RP, U, GPL>(base, G, M, ph, llut, s1, s2);
        else
          sum_rows_multi<VEC, RP, U, GPL>(base, G, M, ph, lut16, s1, s2);
      }
    }

    if constexpr (RP == 1) {
#pragma unroll
      for (int j = 0; j < GPL; ++j) {
        const int g = g0 + j * LPR;
        if (g < t.col_groups) store_group<VEC>(t, b, g, s1[j], s2[j]);
      }
    } else if constexpr (REP) {
      // Every lane is done with the table: reuse it for the reduction, one
      // sum (S1, then S2) at a time, VEC + 1 words per lane (odd stride).
      const int N = t.n_inputs;
      const int B = t.n_blocks;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < GPL; ++j) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          uint32_t* mine = lut32 + tid * (VEC + 1);
#pragma unroll
          for (int k = 0; k < VEC; ++k) mine[k] = half ? s2[j][k] : s1[j][k];
          __syncthreads();
          for (int o = tid; o < LPR * VEC; o += WG) {
            const int l = o / VEC, k = o % VEC;
            uint32_t sum = 0;
#pragma unroll
            for (int q = 0; q < RP; ++q) sum += lut32[(q * LPR + l) * (VEC + 1) + k];
            const int gg = ch * LPR * GPL + j * LPR + l;
            if (gg < t.col_groups) {
              const int64_t col = (int64_t)gg * VEC + k;
              const int64_t f = col / N, i = col % N;
              (half ? t.s2 : t.s1)[(f * B + b) * N + i] = (int32_t)sum;
            }
          }
          __syncthreads();
        }
      }
      if (task + gridDim.x < t.n_tasks) {
        fill_lane_lut<WG>(lut32, tid);
        __syncthreads();
      }
    } else {
      const int N = t.n_inputs;
      const int B = t.n_blocks;
#pragma unroll
      for (int j = 0; j < GPL; ++j) {
        uint32_t* mine = red + (ph * LPR + lc) * W;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          mine[k] = s1[j][k];
          mine[VEC + k] = s2[j][k];
        }
        __syncthreads();
        for (int o = tid; o < LPR * 2 * VEC; o += WG) {
          const int l = o / (2 * VEC), k = o % (2 * VEC);
          uint32_t s = 0;
#pragma unroll 8
          for (int q = 0; q < RP; ++q) s += red[(q * LPR + l) * W + k];
          const int gg = ch * LPR * GPL + j * LPR + l;
          if (gg < t.col_groups) {
            const int64_t col = (int64_t)gg * VEC + (k % VEC);
            const int64_t f = col / N, i = col % N;
            int32_t* dst = k < VEC ? t.s1 : t.s2;
            dst[(f * B + b) * N + i] = (int32_t)s;
          }
        }
        __syncthreads();
      }
    }
  }
}

template <int VEC, int LPR, int U, bool PF, int GPL, bool REP = false>
static int launch_one(const PassATask& t, int grid, hipStream_t s) {
  constexpr int WG = wg_size<LPR>();
  constexpr int RP = WG / LPR;
  const size_t lds = RP > 1 ? sizeof(uint32_t) * WG * (2 * VEC + 1) : 0;
  pass_a_kernel<VEC, LPR, U, PF, GPL, REP><<<dim3(grid), dim3(WG), lds, s>>>(t);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

// Lane-table variants: one row phase, so 256, 512 or 1024 lanes per row
// (narrower tiles are widened to 256 by the planner).
template <int U, int GPL, bool PF = false>
static int launch_rep(const PassATask& t, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 256: return launch_one<16, 256, U, PF, GPL, true>(t, grid, s);
    case 512: return launch_one<16, 512, U, PF, GPL, true>(t, grid, s);
    case 1024: return launch_one<16, 1024, U, PF, GPL, true>(t, grid, s);
  }
  set_error("pass A: lane-table variant needs 256..1024 lanes per row, got %d", lpr);
  return SK_ERR_INVALID_ARG;
}

// Packed lane table, one row phase (256, 512 or 1024 lanes per row).
template <int U>
static int launch_packed(const PassATask& t, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 256:
      pass_a_kernel<16, 256, U, false, 1, true, 256, true><<<dim3(grid), dim3(256), 0, s>>>(t);
      break;
    case 512:
      pass_a_kernel<16, 512, U, false, 1, true, 512, true><<<dim3(grid), dim3(512), 0, s>>>(t);
      break;
    case 1024:
      pass_a_kernel<16, 1024, U, false, 1, true, 1024, true><<<dim3(grid), dim3(1024), 0, s>>>(t);
      break;
    default:
      set_error("pass A: packed lane-table variant needs 256..1024 lanes per row, got %d", lpr);
      return SK_ERR_INVALID_ARG;
  }
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

// Variant 16: packed lane table, 256-lane tasks with blocks side by side for
// narrow rows (t.blocks_per_task blocks per task) or 256-group chunks of one
// block for wide rows; no row phases, so no reduction across lanes.
template <int U>
__global__ __launch_bounds__(256) void pass_a_side_by_side_kernel(PassATask t, int lpb) {
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  const int tid = threadIdx.x;
  fill_lane_packed_lut<256>(lut32, tid);
  __syncthreads();
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) pass_a_task_side_by_side<U>(t, lpb, task, lut);
}

int pass_a_side_by_side_lanes(int64_t col_groups) {
  int lpb = 1;
  while (lpb < 256 && lpb < col_groups) lpb *= 2;
  return lpb;
}

// Variant 17: packed table, 512-lane workgroups over chunks of 512 column
// groups; a task walks Q consecutive blocks holding every block's sums in
// registers and stores them only after its last block. With about one task
// per CU the call becomes a read phase followed by a write phase: mixing
// the sums' writes into the read stream costs far more than their bytes
// (CHIME M = 256: 335 against 382 us with a store after each block).
template <int Q, int U>
__global__ __launch_bounds__(512) void pass_a_deferred_kernel(PassATask t) {
  constexpr int VEC = 16;
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  const int tid = threadIdx.x;
  fill_lane_packed_lut<512>(lut32, tid);
  __syncthreads();
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  const int M = t.block_len;
  const int64_t G = t.row_bytes;
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
    const int b0 = t.block0 + (int)(task / t.chunks) * Q;
    const int g = (int)(task % t.chunks) * 512 + tid;
    if (g >= t.col_groups) continue;
    uint32_t a1[Q][VEC], a2[Q][VEC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) a1[q][k] = a2[q][k] = 0;
      if (b0 + q < t.block_end)
        sum_rows_packed<VEC, 1, U>(t.x + (int64_t)(b0 + q) * M * G + (int64_t)g * VEC, G, M, 0, lut, a1[q], a2[q]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (b0 + q < t.block_end) store_group<VEC>(t, b0 + q, g, a1[q], a2[q]);
  }
}

// Blocks per task for variant 17: about one task per CU, at most 4 (the
// sums of 4 blocks take 128 registers per lane).
int pass_a_deferred_blocks(int64_t n_blocks, int64_t col_groups, int n_cu) {
  const int64_t chunks = (col_groups + 511) / 512;
  int64_t q = (n_blocks * chunks + n_cu - 1) / (n_cu > 0 ? n_cu : 1);
  return (int)(q < 1 ? 1 : (q > 4 ? 4 : q));
}

// Lane table shared by 512-lane workgroups of 512 / lpr row phases (16
// wavefronts per CU at two workgroups); lanes per row 64..512 (the planner
// clamps others into that range).
template <int LPR, int U, int GPL>
static int launch_rep512_one(const PassATask& t, int grid, hipStream_t s) {
  pass_a_kernel<16, LPR, U, false, GPL, true, 512><<<dim3(grid), dim3(512), 0, s>>>(t);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

template <int U, int GPL>
static int launch_rep512(const PassATask& t, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 64: return launch_rep512_one<64, U, GPL>(t, grid, s);
    case 128: return launch_rep512_one<128, U, GPL>(t, grid, s);
    case 256: return launch_rep512_one<256, U, GPL>(t, grid, s);
    case 512: return launch_rep512_one<512, U, GPL>(t, grid, s);
  }
  set_error("pass A: 512-lane lane-table variant needs 64..512 lanes per row, got %d", lpr);
  return SK_ERR_INVALID_ARG;
}

template <int VEC, int U, bool PF, int GPL = 1>
static int launch_lpr(const PassATask& t, int lpr, int grid, hipStream_t s) {
  switch (lpr) {
    case 1: return launch_one<VEC, 1, U, PF, GPL>(t, grid, s);
    case 2: return launch_one<VEC, 2, U, PF, GPL>(t, grid, s);
    case 4: return launch_one<VEC, 4, U, PF, GPL>(t, grid, s);
    case 8: return launch_one<VEC, 8, U, PF, GPL>(t, grid, s);
    case 16: return launch_one<VEC, 16, U, PF, GPL>(t, grid, s);
    case 32: return launch_one<VEC, 32, U, PF, GPL>(t, grid, s);
    case 64: return launch_one<VEC, 64, U, PF, GPL>(t, grid, s);
    case 128: return launch_one<VEC, 128, U, PF, GPL>(t, grid, s);
    case 256: return launch_one<VEC, 256, U, PF, GPL>(t, grid, s);
    case 512: return launch_one<VEC, 512, U, PF, GPL>(t, grid, s);
    case 1024: return launch_one<VEC, 1024, U, PF, GPL>(t, grid, s);
  }
  set_error("pass A: unsupported lanes-per-row %d", lpr);
  return SK_ERR_INVALID_ARG;
}

// Row batching variants (the 16-byte path only; others use variant 0):
//   0: 8 rows per batch            1: 8 rows, next batch prefetched
//   2: 4 rows, prefetched          3: 16 rows per batch
//   4: 2 column groups per lane, 4 rows per batch
//   5: 2 column groups per lane, 8 rows per batch
//   6: 4 column groups per lane, 2 rows per batch
//   7: lane-replicated power table, 8 rows per batch
//   8: lane-replicated power table, 2 column groups per lane, 4 rows
//   9: lane-replicated power table, 8 rows, next batch prefetched
//  10: lane-replicated power table, 16 rows per batch
//  11: lane-replicated power table, 16 rows, next batch prefetched
//  12: lane-replicated table in 512-lane workgroups (512 / LPR row phases), 8 rows
//  13: as 12 with 2 column groups per lane, 4 rows
//  14: packed lane table (p | p^2 << 12 per entry), 8 rows per load
//  15: packed lane table, 16 rows per load
//  16: packed lane table, 256-lane workgroups, blocks side by side for
//      narrow rows (lanes per row = power of two covering the row, <= 256)
//  17: packed lane table, 512-lane workgroups, Q blocks per task with the
//      stores deferred to the task's end (Q = blocks_per_task, 1..4)
int pass_a_groups_per_lane(int vec, int variant) {
  if (vec != 16) return 1;
  switch (variant) {
    case 4: case 5: case 8: case 13: return 2;
    case 6: return 4;
    default: return 1;
  }
}

bool pass_a_lane_table(int vec, int variant) { return vec == 16 && variant >= 7 && variant <= 17; }

bool pass_a_packed(int vec, int variant) { return vec == 16 && (variant == 14 || variant == 15); }

bool pass_a_side_by_side(int vec, int variant) { return vec == 16 && variant == 16; }

bool pass_a_deferred(int vec, int variant) { return vec == 16 && variant == 17; }

void pass_a_lane_range(int vec, int variant, int* lo, int* hi) {
  *lo = 1;
  *hi = 1024;
  if (!pass_a_lane_table(vec, variant)) return;
  if (variant == 12 || variant == 13) { *lo = 64; *hi = 512; }
  else if (variant == 16) { *lo = 1; *hi = 256; }
  else if (variant == 17) { *lo = 512; *hi = 512; }
  else { *lo = 256; }
}

template <int VEC>
static int launch_vec(const PassATask& t, int lpr, int variant, int grid, hipStream_t s) {
  if constexpr (VEC == 16) {
    switch (variant) {
      case 1: return launch_lpr<VEC, 8, true>(t, lpr, grid, s);
      case 2: return launch_lpr<VEC, 4, true>(t, lpr, grid, s);
      case 3: return launch_lpr<VEC, 16, false>(t, lpr, grid, s);
      case 4: return launch_lpr<VEC, 4, false, 2>(t, lpr, grid, s);
      case 5: return launch_lpr<VEC, 8, false, 2>(t, lpr, grid, s);
      case 6: return launch_lpr<VEC, 2, false, 4>(t, lpr, grid, s);
      case 7: return launch_rep<8, 1>(t, lpr, grid, s);
      case 8: return launch_rep<4, 2>(t, lpr, grid, s);
      case 9: return launch_rep<8, 1, true>(t, lpr, grid, s);
      case 10: return launch_rep<16, 1>(t, lpr, grid, s);
      case 11: return launch_rep<16, 1, true>(t, lpr, grid, s);
      case 12: return launch_rep512<8, 1>(t, lpr, grid, s);
      case 13: return launch_rep512<4, 2>(t, lpr, grid, s);
      case 14: return launch_packed<8>(t, lpr, grid, s);
      case 15: return launch_packed<16>(t, lpr, grid, s);
      case 16:
        pass_a_side_by_side_kernel<16><<<dim3(grid), dim3(256), 0, s>>>(t, lpr);
        SK_HIP_TRY(hipGetLastError());
        return SK_OK;
      case 17:
        switch (t.blocks_per_task) {
          case 1: pass_a_deferred_kernel<1, 16><<<dim3(grid), dim3(512), 0, s>>>(t); break;
          case 2: pass_a_deferred_kernel<2, 16><<<dim3(grid), dim3(512), 0, s>>>(t); break;
          case 3: pass_a_deferred_kernel<3, 16><<<dim3(grid), dim3(512), 0, s>>>(t); break;
          case 4: pass_a_deferred_kernel<4, 16><<<dim3(grid), dim3(512), 0, s>>>(t); break;
          default:
            set_error("pass A: deferred-store variant needs 1..4 blocks per task, got %d", t.blocks_per_task);
            return SK_ERR_INVALID_ARG;
        }
        SK_HIP_TRY(hipGetLastError());
        return SK_OK;
      default: break;
    }
  }
  return launch_lpr<VEC, 8, false>(t, lpr, grid, s);
}

int pick_vec(const uint8_t* x, int32_t n_inputs) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(x);
  if (n_inputs % 16 == 0 && a % 16 == 0) return 16;
  if (n_inputs % 4 == 0 && a % 4 == 0) return 4;
  return 1;
}

PassAConfig default_pass_a_config(int vec, int64_t row_bytes, int64_t n_blocks, int block_len, bool lane_table,
                                  int n_cu) {
  const int64_t cg = row_bytes / vec;
  // Wide rows whose 4-block tasks (512-lane workgroups) fill one round of
  // the CUs: hold every block's sums and store them at the end of the task,
  // so the call reads, then writes (CHIME M = 256: 349 against 359 us).
  // With two or three blocks per task, or several rounds, the stores meet
  // the reads again and the per-block variants below are faster.
  if (lane_table && vec == 16 && cg >= 512 && n_cu > 0) {
    const int64_t units = n_blocks * ((cg + 511) / 512);
    if ((units + 3) / 4 <= n_cu && units > 3 * (int64_t)n_cu) {
      PassAConfig c;
      c.vec = vec;
      c.lpr = 512;
      c.variant = 17;
      c.grid = (int)((units + 3) / 4);
      return c;
    }
  }
  // Wide rows with at least one task per CU take the lane-replicated table
  // (no bank conflicts on the power lookups), measured fastest on MI355X:
  //  * >= 512 groups of 16 inputs: packed entries (one add per sample for
  //    both sums) in 1024-lane workgroups, one per CU, each streaming whole
  //    rows of a block (rows of 8 KiB: 316 us for 2 GiB at M = 1024 against
  //    333 us for the next best; equal at M = 256);
  //  * >= 256 groups: one row phase of 256 lanes, packed entries.
  if (lane_table && vec == 16 && cg >= 512 && n_blocks * ((cg + 1023) / 1024) >= 256) {
    const int64_t tasks = n_blocks * ((cg + 1023) / 1024);
    PassAConfig c;
    c.vec = vec;
    c.lpr = 1024;
    c.variant = 15;
    c.grid = (int)(tasks < (1 << 30) ? tasks : (1 << 30));
    return c;
  }
  if (lane_table && vec == 16 && cg >= 256 && n_blocks * ((cg + 255) / 256) >= 256) {
    const int64_t tasks = n_blocks * ((cg + 255) / 256);
    PassAConfig c;
    c.vec = vec;
    c.lpr = 256;
    c.variant = 14;   // packed entries: 2048-input serving frames 68.6 against 76.2 us unpacked
    c.grid = (int)(tasks < (1 << 30) ? tasks : (1 << 30));
    return c;
  }
  // Narrow rows with at least one task per CU: blocks side by side in
  // 256-lane workgroups with the packed table, every lane summing whole rows
  // (the Pathfinder shape: 53 against 57 us with row phases).
  if (lane_table && vec == 16 && cg < 256) {
    int lpb = 1;
    while (lpb < cg) lpb *= 2;
    const int64_t tasks = (n_blocks + 256 / lpb - 1) / (256 / lpb);
    if (tasks >= 256) {
      PassAConfig c;
      c.vec = vec;
      c.lpr = lpb;
      c.variant = 16;
      c.grid = (int)(tasks < (1 << 30) ? tasks : (1 << 30));
      return c;
    }
  }
  int lpr = 1;
  while (lpr < 256 && lpr < cg) lpr *= 2;
  // Keep at least ~2048 workgroups in flight: trade lanes per row for row
  // phases (reduced in LDS), down to 64 lanes, then on to 16 while a
  // workgroup's row phases do not outnumber the block's rows (the 256-input
  // serving frame, 192 blocks of 1 KiB rows: 17.1 against 28.0 us at 64).
  while (lpr > 64 && n_blocks * ((cg + lpr - 1) / lpr) < 2048) lpr /= 2;
  while (lpr > 16 && 512 / lpr <= block_len && n_blocks * ((cg + lpr - 1) / lpr) < 2048) lpr /= 2;
  const int64_t tasks = n_blocks * ((cg + lpr - 1) / lpr);
  PassAConfig c;
  c.vec = vec;
  c.lpr = lpr;
  c.variant = 0;
  c.grid = (int)(tasks < (1 << 30) ? (tasks > 0 ? tasks : 1) : (1 << 30));
  return c;
}

int launch_pass_a(const PassATask& t, const PassAConfig& c, hipStream_t s) {
  if (t.n_tasks <= 0) return SK_OK;
  const int grid = (int)(c.grid < t.n_tasks ? c.grid : t.n_tasks);
  switch (c.vec) {
    case 16: return launch_vec<16>(t, c.lpr, c.variant, grid, s);
    case 4: return launch_vec<4>(t, c.lpr, c.variant, grid, s);
    case 1: return launch_vec<1>(t, c.lpr, c.variant, grid, s);
  }
  set_error("pass A: unsupported vector width %d", c.vec);
  return SK_ERR_INVALID_ARG;
}

}  // namespace sk
