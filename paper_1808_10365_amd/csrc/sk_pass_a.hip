// Pass A: per-input block sums of power and square power (Eq. singlesums).
//
// The input is one byte per complex sample, [T][F][N] (time-major, inputs
// innermost). Each lane owns VEC consecutive inputs of one channel and walks
// the rows (time samples) of a block with one VEC-byte nontemporal load per
// row, so a wavefront reads 64*VEC contiguous bytes per row. Power comes from
// an LDS table indexed by the byte (Re and Im decoded from the nibbles,
// Sec. 2.2.3 "Calculating Power"). Sums are exact in 32 bits: p <= 128, so
// S2 <= M * 2^14 < 2^31 for M <= 131071.
//
// Variants (sk_profile.h):
//   0 shared 256-entry table of p; two rows' powers packed into the 16-bit
//     halves of a register so v_dot2_u32_u16 adds p0^2 + p1^2 to S2 and
//     p0 + p1 to S1; a workgroup of 256 lanes covers LPR column groups times
//     256 / LPR row phases, reduced in LDS. Any vector width (16, 4, 1).
//   1, 2 packed lane-replicated table (entries p | p^2 << 12, one add per
//     sample for both sums), one row phase of 256..1024 lanes, 8 or 16 rows
//     per load.
//   3 packed table, 256-lane workgroups whose lanes sum whole rows; narrow
//     rows put 256 / L blocks side by side.
//   4 packed table, 512-lane workgroups walking up to 4 consecutive blocks
//     with every block's sums held in registers and stored at the task's end.
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

// Variant 0: shared table. One task is (block b, chunk ch) of LPR column
// groups; lane lc of row phase ph owns group ch * LPR + lc, so a wavefront's
// loads of one row are 64 * VEC contiguous bytes. The row phases' partial
// sums meet in LDS (VEC words of S1 then VEC of S2 per lane, odd stride).
template <int VEC, int LPR>
__global__ __launch_bounds__(wg_size<LPR>()) void pass_a_shared_kernel(PassATask t) {
  constexpr int WG = wg_size<LPR>();
  constexpr int RP = WG / LPR;          // row phases per workgroup
  constexpr int W = 2 * VEC + 1;        // LDS stride of one lane's partials (odd: no bank conflicts)
  constexpr int U = 8;                  // rows per load batch
  __shared__ uint16_t lut16[256];
  extern __shared__ uint32_t red[];     // [RP * LPR][W] when RP > 1
  const int tid = threadIdx.x;
  for (int k = tid; k < 256; k += WG) lut16[k] = (uint16_t)code_power((uint32_t)k);
  __syncthreads();
  const int lc = tid % LPR;
  const int ph = tid / LPR;
  const int M = t.block_len;
  const int64_t G = t.row_bytes;
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
    const int b = t.block0 + (int)(task / t.chunks);
    const int ch = (int)(task % t.chunks);
    const int g0 = ch * LPR + lc;
    uint32_t s1[VEC], s2[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) s1[k] = s2[k] = 0;
    if (g0 < t.col_groups)
      sum_rows<VEC, RP, U>(t.x + (int64_t)b * M * G + (int64_t)g0 * VEC, G, M, ph, lut16, s1, s2);
    if constexpr (RP == 1) {
      if (g0 < t.col_groups) store_group<VEC>(t, b, g0, s1, s2);
    } else {
      const int N = t.n_inputs;
      const int B = t.n_blocks;
      uint32_t* mine = red + (ph * LPR + lc) * W;
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        mine[k] = s1[k];
        mine[VEC + k] = s2[k];
      }
      __syncthreads();
      for (int o = tid; o < LPR * 2 * VEC; o += WG) {
        const int l = o / (2 * VEC), k = o % (2 * VEC);
        uint32_t s = 0;
#pragma unroll 8
        for (int q = 0; q < RP; ++q) s += red[(q * LPR + l) * W + k];
        const int gg = ch * LPR + l;
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

template <int VEC, int LPR>
static int launch_shared_one(const PassATask& t, int grid, hipStream_t s, PassEvents ev) {
  constexpr int WG = wg_size<LPR>();
  constexpr int RP = WG / LPR;
  const size_t lds = RP > 1 ? sizeof(uint32_t) * WG * (2 * VEC + 1) : 0;
  launch_kernel(pass_a_shared_kernel<VEC, LPR>, dim3(grid), dim3(WG), (uint32_t)lds, s, ev.start, ev.stop, t);
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

template <int VEC>
static int launch_shared(const PassATask& t, int lpr, int grid, hipStream_t s, PassEvents ev) {
  switch (lpr) {
    case 1: return launch_shared_one<VEC, 1>(t, grid, s, ev);
    case 2: return launch_shared_one<VEC, 2>(t, grid, s, ev);
    case 4: return launch_shared_one<VEC, 4>(t, grid, s, ev);
    case 8: return launch_shared_one<VEC, 8>(t, grid, s, ev);
    case 16: return launch_shared_one<VEC, 16>(t, grid, s, ev);
    case 32: return launch_shared_one<VEC, 32>(t, grid, s, ev);
    case 64: return launch_shared_one<VEC, 64>(t, grid, s, ev);
    case 128: return launch_shared_one<VEC, 128>(t, grid, s, ev);
    case 256: return launch_shared_one<VEC, 256>(t, grid, s, ev);
    case 512: return launch_shared_one<VEC, 512>(t, grid, s, ev);
    case 1024: return launch_shared_one<VEC, 1024>(t, grid, s, ev);
  }
  set_error("pass A: unsupported lanes-per-row %d", lpr);
  return SK_ERR_INVALID_ARG;
}

// Variants 1 and 2: packed lane table, one row phase of LPR lanes (256, 512
// or 1024). A task walks blocks_per_task consecutive blocks (contiguous
// rows) of one column chunk, storing each block's sums as it ends.
template <int LPR, int U>
__global__ __launch_bounds__(LPR) void pass_a_packed_kernel(PassATask t) {
  constexpr int VEC = 16;
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  const int tid = threadIdx.x;
  fill_lane_packed_lut<LPR>(lut32, tid);
  __syncthreads();
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  const int M = t.block_len;
  const int64_t G = t.row_bytes;
  const int Q = t.blocks_per_task;
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
    const int b_first = t.block0 + (int)(task / t.chunks) * Q;
    const int g0 = (int)(task % t.chunks) * LPR + tid;
    if (g0 >= t.col_groups) continue;
    for (int b = b_first; b < b_first + Q && b < t.block_end; ++b) {
      uint32_t s1[VEC], s2[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) s1[k] = s2[k] = 0;
      sum_rows_packed<VEC, 1, U>(t.x + (int64_t)b * M * G + (int64_t)g0 * VEC, G, M, 0, lut, s1, s2);
      store_group<VEC>(t, b, g0, s1, s2);
    }
  }
}

template <int U>
static int launch_packed(const PassATask& t, int lpr, int grid, hipStream_t s, PassEvents ev) {
  switch (lpr) {
    case 256: launch_kernel(pass_a_packed_kernel<256, U>, dim3(grid), dim3(256), 0, s, ev.start, ev.stop, t); break;
    case 512: launch_kernel(pass_a_packed_kernel<512, U>, dim3(grid), dim3(512), 0, s, ev.start, ev.stop, t); break;
    case 1024: launch_kernel(pass_a_packed_kernel<1024, U>, dim3(grid), dim3(1024), 0, s, ev.start, ev.stop, t); break;
    default:
      set_error("pass A: packed lane-table variant needs 256..1024 lanes per row, got %d", lpr);
      return SK_ERR_INVALID_ARG;
  }
  SK_HIP_TRY(hipGetLastError());
  return SK_OK;
}

// Variant 3: packed lane table, 256-lane tasks with blocks side by side for
// narrow rows (t.blocks_per_task blocks per task) or 256-group chunks of one
// block for wide rows; no row phases, so no reduction across lanes.
template <int U>
__global__ __launch_bounds__(256) void pass_a_side_by_side_kernel(PassATask t, int lpb) {
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  const int tid = threadIdx.x;
  fill_lane_packed_lut<256>(lut32, tid);
  __syncthreads();
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x)
    pass_a_task_side_by_side<U>(t, lpb, task, lut, tid);
}

int pass_a_side_by_side_lanes(int64_t col_groups) {
  int lpb = 1;
  while (lpb < 256 && lpb < col_groups) lpb *= 2;
  return lpb;
}

// Variant 4: packed table, 512-lane workgroups over chunks of 512 column
// groups; a task walks Q consecutive blocks holding every block's sums in
// registers and stores them only after its last block. With about one task
// per CU the call becomes a read phase followed by a write phase: mixing
// the sums' writes into the read stream costs far more than their bytes
// (CHIME M = 256: 335 against 382 us with a store after each block). The
// two wavefronts of each SIMD keep level through SimdBalance.
//
// With t.timeline set (one task per workgroup), lane 0 of every wavefront
// records the real-time clock (100 MHz) at its start, after its reads (the
// stamp depends on the sums, so it follows the last load) and after its
// stores have completed, then its XCD and HW_ID registers, at
// timeline[6 (8 blockIdx.x + wavefront) ...]. BAL = false leaves the
// wavefronts of a SIMD to the arbiter (for timelines that compare).
template <int Q, int U, bool BAL = true>
__global__ __launch_bounds__(512) void pass_a_deferred_kernel(PassATask t) {
  constexpr int VEC = 16;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  __shared__ __attribute__((aligned(16))) uint32_t lut32[LANE_LUT_DWORDS];
  __shared__ uint32_t simd_of[8], progress[8];
  const int tid = threadIdx.x;
  fill_lane_packed_lut<512>(lut32, tid);
  simd_balance_post(simd_of, progress, tid);
  __syncthreads();
  SimdBalance bal = simd_balance_pair(simd_of, progress, 8);
  NoBalance arbiter;
  const LanePackedLut lut{reinterpret_cast<const uint8_t*>(lut32), (uint32_t)(tid & 63) * 4};
  const int M = t.block_len;
  const int64_t G = t.row_bytes;
  uint64_t t_reads = 0;
  for (int64_t task = blockIdx.x; task < t.n_tasks; task += gridDim.x) {
    const int b0 = t.block0 + (int)(task / t.chunks) * Q;
    const int g = (int)(task % t.chunks) * 512 + tid;
    if (g >= t.col_groups) continue;
    uint32_t a1[Q][VEC], a2[Q][VEC];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) a1[q][k] = a2[q][k] = 0;
      if (b0 + q < t.block_end) {
        const uint8_t* base = t.x + (int64_t)(b0 + q) * M * G + (int64_t)g * VEC;
        if constexpr (BAL) sum_rows_packed<VEC, 1, U>(base, G, M, 0, lut, a1[q], a2[q], bal);
        else sum_rows_packed<VEC, 1, U>(base, G, M, 0, lut, a1[q], a2[q], arbiter);
      }
    }
    if (t.timeline) {
      uint32_t dep = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) dep |= a1[q][0] >> 31;
      t_reads = __builtin_amdgcn_s_memrealtime() + __builtin_amdgcn_readfirstlane(dep);
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (b0 + q < t.block_end) store_group<VEC>(t, b0 + q, g, a1[q], a2[q]);
    if (t.cs) {
      // S1 over the task's blocks: the chunk sums pass B's prefix scan reads
      // instead of the rows (blocks past the end hold zero sums).
      uint32_t c[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        c[k] = a1[0][k];
#pragma unroll
        for (int q = 1; q < Q; ++q) c[k] += a1[q][k];
      }
      const int N = t.n_inputs;
      const int64_t col = (int64_t)g * VEC;
      const int64_t f = col / N, i = col % N;
      const int64_t nk = (t.n_blocks + Q - 1) / Q;
      int32_t* d = t.cs + (f * nk + (b0 - t.block0) / Q) * N + i;
#pragma unroll
      for (int k = 0; k < VEC; k += 4) *reinterpret_cast<u32x4*>(d + k) = u32x4{c[k], c[k + 1], c[k + 2], c[k + 3]};
    }
  }
  if (t.timeline) {
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t_end = __builtin_amdgcn_s_memrealtime();
    if ((tid & 63) == 0) {
      uint64_t* o = t.timeline + ((int64_t)blockIdx.x * 8 + (tid >> 6)) * 6;
      o[0] = t_start;
      o[1] = t_reads;
      o[2] = t_end;
      o[3] = (uint32_t)__builtin_amdgcn_s_getreg(20 | (3 << 11));   // XCC_ID bits 3:0
      o[4] = (uint32_t)__builtin_amdgcn_s_getreg(4 | (31 << 11));   // HW_ID
      o[5] = simd_id();
    }
  }
}

// Blocks per task for variant 4: about one task per CU, at most 4 (the
// sums of 4 blocks take 128 registers per lane).
int pass_a_deferred_blocks(int64_t n_blocks, int64_t col_groups, int n_cu) {
  const int64_t chunks = (col_groups + 511) / 512;
  int64_t q = (n_blocks * chunks + n_cu - 1) / (n_cu > 0 ? n_cu : 1);
  return (int)(q < 1 ? 1 : (q > 4 ? 4 : q));
}

bool pass_a_packed(int vec, int variant) { return vec == 16 && (variant == 1 || variant == 2); }

bool pass_a_side_by_side(int vec, int variant) { return vec == 16 && variant == 3; }

bool pass_a_deferred(int vec, int variant) { return vec == 16 && variant == 4; }

void pass_a_lane_range(int vec, int variant, int* lo, int* hi) {
  *lo = 1;
  *hi = 1024;
  if (vec != 16 || variant == 0) return;
  if (variant == 3) { *lo = 1; *hi = 256; }
  else if (variant == 4) { *lo = 512; *hi = 512; }
  else { *lo = 256; }
}

template <int VEC>
static int launch_vec(const PassATask& t, int lpr, int variant, int grid, hipStream_t s, PassEvents ev) {
  if constexpr (VEC == 16) {
    const dim3 g(grid), w512(512);
    switch (variant) {
      case 1: return launch_packed<8>(t, lpr, grid, s, ev);
      case 2: return launch_packed<16>(t, lpr, grid, s, ev);
      case 3:
        launch_kernel(pass_a_side_by_side_kernel<16>, g, dim3(256), 0, s, ev.start, ev.stop, t, lpr);
        SK_HIP_TRY(hipGetLastError());
        return SK_OK;
      case 4:
        switch (t.blocks_per_task) {
          case 1: launch_kernel(pass_a_deferred_kernel<1, 16>, g, w512, 0, s, ev.start, ev.stop, t); break;
          case 2: launch_kernel(pass_a_deferred_kernel<2, 16>, g, w512, 0, s, ev.start, ev.stop, t); break;
          case 3: launch_kernel(pass_a_deferred_kernel<3, 16>, g, w512, 0, s, ev.start, ev.stop, t); break;
          case 4:
            if (t.simd_balance) launch_kernel(pass_a_deferred_kernel<4, 16>, g, w512, 0, s, ev.start, ev.stop, t);
            else launch_kernel(pass_a_deferred_kernel<4, 16, false>, g, w512, 0, s, ev.start, ev.stop, t);
            break;
          default:
            set_error("pass A: deferred-store variant needs 1..4 blocks per task, got %d", t.blocks_per_task);
            return SK_ERR_INVALID_ARG;
        }
        SK_HIP_TRY(hipGetLastError());
        return SK_OK;
      default: break;
    }
  }
  return launch_shared<VEC>(t, lpr, grid, s, ev);
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
      c.variant = 4;
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
    c.variant = 2;
    c.grid = (int)(tasks < (1 << 30) ? tasks : (1 << 30));
    return c;
  }
  if (lane_table && vec == 16 && cg >= 256 && n_blocks * ((cg + 255) / 256) >= 256) {
    const int64_t tasks = n_blocks * ((cg + 255) / 256);
    PassAConfig c;
    c.vec = vec;
    c.lpr = 256;
    c.variant = 1;    // packed entries: 2048-input serving frames 68.6 against 76.2 us unpacked
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
      c.variant = 3;
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

int launch_pass_a(const PassATask& t, const PassAConfig& c, hipStream_t s, PassEvents ev) {
  if (t.n_tasks <= 0) return SK_OK;
  const int grid = (int)(c.grid < t.n_tasks ? c.grid : t.n_tasks);
  switch (c.vec) {
    case 16: return launch_vec<16>(t, c.lpr, c.variant, grid, s, ev);
    case 4: return launch_vec<4>(t, c.lpr, c.variant, grid, s, ev);
    case 1: return launch_vec<1>(t, c.lpr, c.variant, grid, s, ev);
  }
  set_error("pass A: unsupported vector width %d", c.vec);
  return SK_ERR_INVALID_ARG;
}

}  // namespace sk
