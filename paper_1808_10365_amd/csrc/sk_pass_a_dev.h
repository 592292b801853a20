// Pass A device code shared by the single-plan and batched kernels:
// decode, power table, and the per-lane row walk (Eq. singlesums).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sk_internal.h"

namespace sk {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Power of one offset-encoded byte: high nibble = Re + 8, low = Im + 8.
__device__ __forceinline__ uint32_t code_power(uint32_t c) {
  const int re = (int)(c >> 4) - 8;
  const int im = (int)(c & 15u) - 8;
  return (uint32_t)(re * re + im * im);
}

#define SK_GLOBAL __attribute__((address_space(1)))

// Input rows always live in device (global) memory. Loading through a
// global-address-space pointer keeps the loads global_load_* even where the
// compiler cannot infer the address space (flat loads would also count
// against the LDS wait counter and serialise the table reads behind them).
template <int VEC>
struct Row {
  static constexpr int DW = VEC >= 4 ? VEC / 4 : 1;
  uint32_t w[DW];
  __device__ __forceinline__ void load(const uint8_t* p) {
    if constexpr (VEC == 16) {
      const u32x4 v = __builtin_nontemporal_load((const SK_GLOBAL u32x4*)p);
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (VEC == 4) {
      w[0] = __builtin_nontemporal_load((const SK_GLOBAL uint32_t*)p);
    } else {
      w[0] = *(const SK_GLOBAL uint8_t*)p;
    }
  }
  __device__ __forceinline__ uint32_t byte(int k) const {
    return (w[k >> 2] >> (8 * (k & 3))) & 0xFFu;
  }
};

template <int VEC>
__device__ __forceinline__ void accumulate_pair(const Row<VEC>& r0, const Row<VEC>& r1,
                                                const uint16_t* lut, uint32_t* s1, uint32_t* s2) {
  const u16x2 ones = {1, 1};
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const uint32_t pp = (uint32_t)lut[r0.byte(k)] | ((uint32_t)lut[r1.byte(k)] << 16);
    const u16x2 P = __builtin_bit_cast(u16x2, pp);
    s2[k] = __builtin_amdgcn_udot2(P, P, s2[k], false);
    s1[k] = __builtin_amdgcn_udot2(P, ones, s1[k], false);
  }
}

template <int VEC>
__device__ __forceinline__ void accumulate_one(const Row<VEC>& r0, const uint16_t* lut,
                                               uint32_t* s1, uint32_t* s2) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const uint32_t p = lut[r0.byte(k)];
    s1[k] += p;
    s2[k] += p * p;
  }
}

// Packed power table replicated per lane: the entry of code c for lane l is
// the dword at byte (c << 8) | (l % 64) * 4, 64 KiB in all, holding
// p | p^2 << 12 for code c. The 64 lanes of a wavefront always read 64
// distinct consecutive dwords (no bank conflicts whatever the codes), and
// one v_perm_b32 forms the address: byte 1 = the code byte, byte 0 = the
// lane's offset. Over at most 16 rows, sum p <= 2048 stays in
// the low 12 bits and sum p^2 <= 2^18 in the next 19, so one 32-bit add per
// sample (v_add3_u32 folds two rows) accumulates both sums; every 16 rows
// the packed sums are split into S1 and S2.
struct LanePackedLut {
  const uint8_t* base;
  uint32_t laneoff;
  __device__ __forceinline__ uint32_t at(uint32_t w, int k) const {
    const uint32_t sel = 0x0C0C0000u | ((uint32_t)(4 + k) << 8);
    return *reinterpret_cast<const uint32_t*>(base + __builtin_amdgcn_perm(w, laneoff, sel));
  }
};
constexpr int PACK_ROWS = 16;
constexpr int PACK_SHIFT = 12;

constexpr int LANE_LUT_DWORDS = 256 * 64;

template <int WG>
__device__ __forceinline__ void fill_lane_packed_lut(uint32_t* t, int tid) {
  for (int k = tid; k < LANE_LUT_DWORDS / 4; k += WG) {
    const uint32_t p = code_power((uint32_t)(k >> 4));
    const uint32_t e = p | (p * p << PACK_SHIFT);
    reinterpret_cast<u32x4*>(t)[k] = u32x4{e, e, e, e};
  }
}

// Nothing between packed runs.
struct NoBalance {
  __device__ __forceinline__ void operator()() {}
};

// Wavefronts that share a SIMD do not progress alike: the instruction
// arbiter favours the older one, so with equal work the younger one ends
// last and then runs alone, with half the loads in flight, for the end of
// the kernel (CHIME M = 256, variant 4: the first wavefront of each SIMD
// ended its reads about 55 us before the second). After every packed run a
// wavefront posts its progress in LDS and compares it with its partner's
// (another wavefront of the workgroup on the same SIMD): ahead, it drops to
// priority 0; level or behind, it takes priority 2. No wavefront waits.
struct SimdBalance {
  uint32_t* prog;   // LDS, one word per wavefront of the workgroup
  int self, partner;
  uint32_t done;
  __device__ __forceinline__ void operator()() {
    ++done;
    // Every lane stores the same value: no divergent branch.
    __atomic_store_n(&prog[self], done, __ATOMIC_RELAXED);
    const uint32_t other = __builtin_amdgcn_readfirstlane(__atomic_load_n(&prog[partner], __ATOMIC_RELAXED));
    // One asm block for the compare and both priorities, so the compiler's
    // control flow (and its register allocation) is not split.
    asm volatile("s_cmp_gt_u32 %0, %1\n\ts_cbranch_scc0 1f\n\ts_setprio 0\n\ts_branch 2f\n1:\n\ts_setprio 2\n2:"
                 :: "s"(__builtin_amdgcn_readfirstlane(done)), "s"(other) : "scc");
  }
};

// SIMD of the calling wavefront (HW_ID bits 5:4).
__device__ __forceinline__ uint32_t simd_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg(4 | (4 << 6) | (1 << 11));
}

// First half of setting up SimdBalance for a workgroup of `waves`
// wavefronts: each posts its SIMD and zero progress. The caller then
// synchronises the workgroup before simd_balance_pair.
__device__ __forceinline__ void simd_balance_post(uint32_t* sid, uint32_t* prog, int tid) {
  if ((tid & 63) == 0) {
    sid[tid >> 6] = simd_id();
    prog[tid >> 6] = 0;
  }
}

// Second half: the partner is the first other wavefront on the same SIMD
// (none: the wavefront is its own partner and always takes priority 2).
__device__ __forceinline__ SimdBalance simd_balance_pair(const uint32_t* sid, uint32_t* prog, int waves) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int partner = w;
  for (int j = waves - 1; j >= 0; --j)
    if (j != w && sid[j] == sid[w]) partner = j;
  return SimdBalance{prog, w, __builtin_amdgcn_readfirstlane(partner), 0u};
}

// Rows ph, ph + RP, ... (< M) of this lane with the packed table, in loads of
// U rows, unpacking every PACK_ROWS rows; `bal` runs after every packed run.
template <int VEC, int RP, int U, typename Balance = NoBalance>
__device__ __forceinline__ void sum_rows_packed(const uint8_t* base, int64_t G, int M, int ph,
                                                const LanePackedLut& lut, uint32_t* s1, uint32_t* s2,
                                                Balance&& bal = Balance()) {
  static_assert(VEC >= 4 && U % 2 == 0 && PACK_ROWS % U == 0, "whole row pairs per packed run");
  const int nrow = ph < M ? (M - ph + RP - 1) / RP : 0;
  const int64_t step = (int64_t)RP * G;
  const uint8_t* p = base + (int64_t)ph * G;
  for (int done = 0; done < nrow; done += PACK_ROWS) {
    const int n = nrow - done < PACK_ROWS ? nrow - done : PACK_ROWS;
    uint32_t acc[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) acc[k] = 0;
    int r = 0;
    for (; r + U <= n; r += U) {
      Row<VEC> q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) q[u].load(p + u * step);
      p += U * step;
#pragma unroll
      for (int u = 0; u < U; u += 2)
#pragma unroll
        for (int k = 0; k < VEC; ++k)
          acc[k] = acc[k] + lut.at(q[u].w[k >> 2], k & 3) + lut.at(q[u + 1].w[k >> 2], k & 3);
    }
    for (; r < n; ++r) {
      Row<VEC> q;
      q.load(p);
      p += step;
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[k] += lut.at(q.w[k >> 2], k & 3);
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      s1[k] += acc[k] & ((1u << PACK_SHIFT) - 1);
      s2[k] += acc[k] >> PACK_SHIFT;
    }
    bal();
  }
}

// Rows of this lane in batches of U: r = ph, ph + RP, ... (< M), the loads
// of a batch issued together, then reduced in row pairs.
template <int VEC, int RP, int U>
__device__ __forceinline__ void sum_rows(const uint8_t* base, int64_t G, int M, int ph,
                                         const uint16_t* lut, uint32_t* s1, uint32_t* s2) {
  const int nrow = ph < M ? (M - ph + RP - 1) / RP : 0;
  const int nb = nrow / U;
  int r = ph;
  for (int bt = 0; bt < nb; ++bt) {
    Row<VEC> q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u].load(base + (int64_t)(r + u * RP) * G);
#pragma unroll
    for (int u = 0; u < U / 2; ++u) accumulate_pair<VEC>(q[2 * u], q[2 * u + 1], lut, s1, s2);
    r += U * RP;
  }
  for (; r + RP < M; r += 2 * RP) {
    Row<VEC> q0, q1;
    q0.load(base + (int64_t)r * G);
    q1.load(base + (int64_t)(r + RP) * G);
    accumulate_pair<VEC>(q0, q1, lut, s1, s2);
  }
  if (r < M) {
    Row<VEC> q0;
    q0.load(base + (int64_t)r * G);
    accumulate_one<VEC>(q0, lut, s1, s2);
  }
}

// One 256-lane task with the packed lane table (Eq. singlesums), every lane
// (tid, 0..255) summing whole rows of one (block, column group). lpb = lanes per block row:
// 256 for wide rows (task = t.blocks_per_task consecutive blocks, walked one
// after the other, of a chunk of 256 column groups); a power of two >= the
// row's column groups otherwise (task = t.blocks_per_task = 256 / lpb
// consecutive blocks side by side, lane l on block l / lpb, column group
// l % lpb). Needs the PassATask fields chunks, blocks_per_task, block0 and
// block_end set to match. With wide rows and t.cs set, the task also writes
// its blocks' S1 total (the chunk sum of pass B chunks of blocks_per_task
// blocks); narrow rows need t.cs null.
template <int U, typename Balance = NoBalance>
__device__ __forceinline__ void pass_a_task_side_by_side(const PassATask& t, int lpb, int64_t task,
                                                         const LanePackedLut& lut, int tid,
                                                         Balance&& bal = Balance()) {
  constexpr int VEC = 16;
  const int64_t bg = task / t.chunks;
  const int ch = (int)(task % t.chunks);
  int64_t b, b_end;
  int g;
  if (lpb >= 256) {
    b = t.block0 + bg * t.blocks_per_task;
    b_end = b + t.blocks_per_task;
    g = ch * 256 + tid;
  } else {
    b = t.block0 + bg * t.blocks_per_task + tid / lpb;
    b_end = b + 1;
    g = tid % lpb;
  }
  if (b_end > t.block_end) b_end = t.block_end;
  if (g >= t.col_groups) return;
  const int M = t.block_len;
  const int64_t G = t.row_bytes;
  const int N = t.n_inputs, B = t.n_blocks;
  const int64_t col = (int64_t)g * VEC;
  const int64_t f = col / N, i = col % N;
  const int64_t b_first = b;
  uint32_t c[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) c[k] = 0;
  for (; b < b_end; ++b) {
    uint32_t s1[VEC], s2[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) s1[k] = s2[k] = 0;
    sum_rows_packed<VEC, 1, U>(t.x + b * M * G + (int64_t)g * VEC, G, M, 0, lut, s1, s2, bal);
    int32_t* d1 = t.s1 + (f * B + b) * N + i;
    int32_t* d2 = t.s2 + (f * B + b) * N + i;
#pragma unroll
    for (int k = 0; k < VEC; k += 4) {
      *reinterpret_cast<u32x4*>(d1 + k) = u32x4{s1[k], s1[k + 1], s1[k + 2], s1[k + 3]};
      *reinterpret_cast<u32x4*>(d2 + k) = u32x4{s2[k], s2[k + 1], s2[k + 2], s2[k + 3]};
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) c[k] += s1[k];
  }
  if (lpb >= 256 && t.cs) {
    // S1 over the task's blocks (wide rows): the chunk sums the prefix scan
    // reads instead of the rows when the task's blocks are one pass B chunk.
    const int Q = t.blocks_per_task;
    const int64_t nk = (t.n_blocks + Q - 1) / Q;
    int32_t* d = t.cs + (f * nk + (b_first - t.block0) / Q) * N + i;
#pragma unroll
    for (int k = 0; k < VEC; k += 4) *reinterpret_cast<u32x4*>(d + k) = u32x4{c[k], c[k + 1], c[k + 2], c[k + 3]};
  }
}

// One 512-lane task of Q consecutive blocks over 512 column groups (chunk
// task % chunks), every lane summing whole rows of one column group, with
// all Q blocks' sums held in registers and stored after the last block, so
// the stores do not interleave with the task's reads; with t.cs set, the S1
// total of the Q blocks too (the chunk sums of pass B chunks of Q blocks).
// Contains no barrier.
template <int Q, int U, typename Balance>
__device__ __forceinline__ void pass_a_task_deferred(const PassATask& t, int64_t task, const LanePackedLut& lut,
                                                     Balance&& bal) {
  constexpr int VEC = 16;
  const int tid = threadIdx.x;
  const int b0 = t.block0 + (int)(task / t.chunks) * Q;
  const int g = (int)(task % t.chunks) * 512 + tid;
  if (g >= t.col_groups) return;
  const int M = t.block_len, N = t.n_inputs, B = t.n_blocks;
  const int64_t G = t.row_bytes;
  uint32_t a1[Q][VEC], a2[Q][VEC];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) a1[q][k] = a2[q][k] = 0;
    if (b0 + q < t.block_end)
      sum_rows_packed<VEC, 1, U>(t.x + (int64_t)(b0 + q) * M * G + (int64_t)g * VEC, G, M, 0, lut, a1[q], a2[q], bal);
  }
  __builtin_amdgcn_s_setprio(0);
  const int64_t col = (int64_t)g * VEC;
  const int64_t f = col / N, i = col % N;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (b0 + q >= t.block_end) continue;
    int32_t* d1 = t.s1 + (f * B + b0 + q) * N + i;
    int32_t* d2 = t.s2 + (f * B + b0 + q) * N + i;
#pragma unroll
    for (int k = 0; k < VEC; k += 4) {
      *reinterpret_cast<u32x4*>(d1 + k) = u32x4{a1[q][k], a1[q][k + 1], a1[q][k + 2], a1[q][k + 3]};
      *reinterpret_cast<u32x4*>(d2 + k) = u32x4{a2[q][k], a2[q][k + 1], a2[q][k + 2], a2[q][k + 3]};
    }
  }
  if (t.cs) {
    const int64_t nk = (t.n_blocks + Q - 1) / Q;
    int32_t* d = t.cs + (f * nk + (b0 - t.block0) / Q) * N + i;
#pragma unroll
    for (int k = 0; k < VEC; k += 4) {
      u32x4 c = {a1[0][k], a1[0][k + 1], a1[0][k + 2], a1[0][k + 3]};
#pragma unroll
      for (int q = 1; q < Q; ++q) c += u32x4{a1[q][k], a1[q][k + 1], a1[q][k + 2], a1[q][k + 3]};
      *reinterpret_cast<u32x4*>(d + k) = c;
    }
  }
}

}  // namespace sk
