// Pass B device code shared by the single-plan and batched kernels:
// window sums, array combine, estimator and flags (Eq. discreteMean,
// normedSum1/2, avgSK, final; Sec. 3.2).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sk_internal.h"

namespace sk {

template <int V>
struct IVec;
template <>
struct IVec<1> {
  int32_t v[1];
  __device__ __forceinline__ void load(const int32_t* p) { v[0] = *p; }
  __device__ __forceinline__ void store(int32_t* p) const { *p = v[0]; }
};
template <>
struct IVec<4> {
  int32_t v[4];
  __device__ __forceinline__ void load(const int32_t* p) {
    const int4 q = *reinterpret_cast<const int4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ __forceinline__ void store(int32_t* p) const {
    *reinterpret_cast<int4*>(p) = make_int4(v[0], v[1], v[2], v[3]);
  }
};

template <>
struct IVec<8> {
  int32_t v[8];
  __device__ __forceinline__ void load(const int32_t* p) {
    const int4 q = *reinterpret_cast<const int4*>(p);
    const int4 r = *reinterpret_cast<const int4*>(p + 4);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    v[4] = r.x; v[5] = r.y; v[6] = r.z; v[7] = r.w;
  }
  __device__ __forceinline__ void store(int32_t* p) const {
    *reinterpret_cast<int4*>(p) = make_int4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<int4*>(p + 4) = make_int4(v[4], v[5], v[6], v[7]);
  }
};

// Row of S1 for sequence position e (history or this call), channel f.
__device__ __forceinline__ const int32_t* seq_row(const PassBArgs& a, int f, int64_t e) {
  if (e < a.hist_len) return a.hist + ((int64_t)f * a.hist_cap + e) * a.n_inputs;
  return a.s1 + ((int64_t)f * a.n_blocks + (e - a.hist_len)) * a.n_inputs;
}

template <int V>
__device__ __forceinline__ void chunk_sum_body(const PassBArgs& a, int c, int f, int z) {
  const int i0 = (z * 256 + threadIdx.x) * V;
  if (i0 >= a.n_inputs) return;
  const int64_t total = (int64_t)a.hist_len + a.n_blocks;
  const int64_t e0 = (int64_t)c * a.chunk;
  const int64_t e1 = e0 + a.chunk < total ? e0 + a.chunk : total;
  IVec<V> s;
#pragma unroll
  for (int k = 0; k < V; ++k) s.v[k] = 0;
  // Rows in groups of 8 loaded together (independent loads in flight).
  int64_t e = e0;
  for (; e + 8 <= e1; e += 8) {
    IVec<V> x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u].load(seq_row(a, f, e + u) + i0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) s.v[k] += x[u].v[k];
  }
  for (; e < e1; ++e) {
    IVec<V> x;
    x.load(seq_row(a, f, e) + i0);
#pragma unroll
    for (int k = 0; k < V; ++k) s.v[k] += x.v[k];
  }
  s.store(a.chunk_sum + ((int64_t)f * a.n_chunks + c) * a.n_inputs + i0);
}

// Adds S1 of sequence positions [from, to) for V inputs at i0 into out,
// eight rows loaded together (independent loads in flight, the last group
// predicated).
template <int V>
__device__ __forceinline__ void add_rows(const PassBArgs& a, int f, int64_t from, int64_t to, int i0, int32_t* out) {
  for (int64_t e = from; e < to; e += 8) {
    IVec<V> x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < V; ++k) x[u].v[k] = 0;
      if (e + u < to) x[u].load(seq_row(a, f, e + u) + i0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < V; ++k) out[k] += x[u].v[k];
  }
}

// Windows of at most SHORT_WINDOW blocks are summed from their rows (a
// batch or two of loads); the chunk sums, and their launch, serve longer ones.
constexpr int SHORT_WINDOW = 16;

// Sum of S1 over sequence positions [lo, hi) for V inputs at i0: the chunk
// sums of the chunks wholly inside, plus the rows at either edge.
template <int V>
__device__ void window_sum(const PassBArgs& a, int f, int64_t lo, int64_t hi, int i0, int32_t* out) {
#pragma unroll
  for (int k = 0; k < V; ++k) out[k] = 0;
  if (hi <= lo) return;
  const int64_t R = a.chunk;
  const int64_t cs = (lo + R - 1) / R;   // first chunk fully inside
  const int64_t ce = hi / R;             // one past the last chunk fully inside
  if (a.window > SHORT_WINDOW && cs < ce) {
#pragma unroll 8
    for (int64_t c = cs; c < ce; ++c) {
      IVec<V> t;
      t.load(a.chunk_sum + ((int64_t)f * a.n_chunks + c) * a.n_inputs + i0);
#pragma unroll
      for (int k = 0; k < V; ++k) out[k] += t.v[k];
    }
    add_rows<V>(a, f, lo, cs * R, i0, out);
    add_rows<V>(a, f, ce * R, hi, i0, out);
  } else {
    add_rows<V>(a, f, lo, hi, i0, out);
  }
}

// Wavefront sums with DPP lane moves (VALU only, no LDS). Butterflies
// inside each row of 16 lanes (quad_perm xor 1, xor 2, half-row mirror, row
// mirror), then row_bcast:15 and row_bcast:31 fold the four rows; the total
// lands in lane 63. The order of additions is fixed.
// With every row enabled (the butterflies) each lane is written, so a plain
// DPP move suffices; the broadcast steps enable some rows only, and the
// others must read 0, so they keep an explicit zero as the old value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  if constexpr (ROW_MASK == 0xF)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, ROW_MASK, 0xF, false);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// 64-bit values move as their two 32-bit halves; the halves are regrouped
// through a two-lane vector (a register pair, no shifts or adds).
typedef uint32_t dpp_u32x2 __attribute__((ext_vector_type(2)));

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_step(double v) {
  const dpp_u32x2 u = __builtin_bit_cast(dpp_u32x2, v);
  dpp_u32x2 m;
  m.x = dpp_mov<CTRL, ROW_MASK>(u.x);
  m.y = dpp_mov<CTRL, ROW_MASK>(u.y);
  return v + __builtin_bit_cast(double, m);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int64_t dpp_step(int64_t v) {
  const dpp_u32x2 u = __builtin_bit_cast(dpp_u32x2, v);
  dpp_u32x2 m;
  m.x = dpp_mov<CTRL, ROW_MASK>(u.x);
  m.y = dpp_mov<CTRL, ROW_MASK>(u.y);
  return v + __builtin_bit_cast(int64_t, m);
}

// 32-bit sums: the zero-old form folds into one v_add_u32 with a DPP source.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_step(int32_t v) {
  return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

// Sum over the 64 lanes, valid in lane 63.
template <typename T>
__device__ __forceinline__ T wave_sum_to_last(T v) {
  v = dpp_step<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_step<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_step<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_step<0x140, 0xF>(v);   // row_mirror
  v = dpp_step<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_step<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Eq. originalSK: (M+1)/(M-1) (M S2 / S1^2 - 1), NaN where S1 = 0.
__device__ __forceinline__ float per_input_sk(int32_t s1, int32_t s2, int32_t block_len) {
#pragma clang fp contract(off)
  if (s1 == 0) return __builtin_nanf("");
  const double Md = (double)block_len, x = (double)s1;
  return (float)((Md + 1.0) / (Md - 1.0) * (Md * (double)s2 / (x * x) - 1.0));
}

// 1/p for p >= 1: the hardware reciprocal estimate refined by two Newton
// steps (each squares the relative error), within a few ulps of the
// correctly rounded quotient. S1/P and S2/P^2 then cost multiplies.
__device__ __forceinline__ double recip_pos(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = __builtin_fma(-p, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-p, r, 1.0);
  return __builtin_fma(r, e, r);
}

// RI: integer type of the per-wavefront R1/R2 sums: int32_t when a
// wavefront's sums provably fit (64 V M 2^14 < 2^31), else int64_t.
// Estimator and flags from the combined sums (Eq. avgSK, final; Sec. 3.2).
// Contraction is off so the rounding steps are the plain ones.
__device__ __forceinline__ void finish(const PassBArgs& a, int f, int b, double A, double Bq, int64_t R1, int64_t R2,
                       int32_t n) {
#pragma clang fp contract(off)
  const int64_t K = (int64_t)n * a.block_len;
  const double Kd = (double)K, Md = (double)a.block_len;
  bool invalid = K < 2;
  double V = 0.0;
  if (a.window == 0) {
    invalid = invalid || R1 == 0;
    if (!invalid) {
      // Eq. (2) over all K samples, numerator K R2 - R1^2 formed exactly.
      const __int128 num = (__int128)K * (__int128)R2 - (__int128)R1 * (__int128)R1;
      const __int128 den = (__int128)R1 * (__int128)R1;
      const double nd = (double)(int64_t)(num >> 64) * 18446744073709551616.0 + (double)(uint64_t)num;
      const double dd = (double)(int64_t)(den >> 64) * 18446744073709551616.0 + (double)(uint64_t)den;
      V = (Kd + 1.0) / (Kd - 1.0) * (nd / dd);
    }
  } else {
    invalid = invalid || A == 0.0;
    if (!invalid) {
      if (a.estimator == SK_EST_TILDE)
        V = (Md + 1.0) / (Md - 1.0) * (Md * Bq / (double)n - 1.0);
      else
        V = (Kd + 1.0) / (Kd - 1.0) * (Kd * Bq / (A * A) - 1.0);
    }
  }
  uint8_t fl;
  double sig = __builtin_nan("");
  if (invalid) {
    V = __builtin_nan("");
    fl = SK_FLAG_INVALID;
  } else {
    double e0 = 1.0;
    if (a.estimator == SK_EST_HAT && a.window == 1) e0 = ((Kd + 1.0) * (Md - 1.0)) / ((Kd - 1.0) * (Md + 1.0));
    const double E = e0 + a.expect_offset;
    const double s = a.sigma_override > 0.0 ? a.sigma_override : sqrt(4.0 / Kd);
    double lo = E - a.k_sigma * s, hi = E + a.k_sigma * s;
    if (a.thresholds) {
      lo = a.thresholds[2 * n];
      hi = a.thresholds[2 * n + 1];
    }
    fl = (V < lo ? SK_FLAG_LOW : 0) | (V > hi ? SK_FLAG_HIGH : 0);
    sig = (V - E) / s;
  }
  const int64_t o = (int64_t)f * a.n_blocks + b;
  if (a.significance) a.significance[o] = (float)sig;
  if (a.r1) a.r1[o] = R1;
  if (a.r2) a.r2[o] = R2;
  if (a.v) a.v[o] = (float)V;
  if (a.flags) a.flags[o] = fl;
  if (a.n_eff) a.n_eff[o] = n;
}

// FIN: the workgroup holds every input group of the channel (one wavefront
// per group, z = 0, at most MAX_FIN_GROUPS) and finishes its blocks itself.
// The wavefront sums of up to FIN_SLOTS blocks wait in LDS; then, after one
// barrier, they are added in group order (the order finalize_body uses, so
// every output is the same bit for bit) and the blocks are finished.
constexpr int MAX_FIN_GROUPS = 4;
constexpr int FIN_SLOTS = 32;

template <int V, typename RI, int U, bool FIN = false>
__device__ __forceinline__ void partial_body_t(const PassBArgs& a, int c, int f, int z) {
  // U: blocks whose rows are loaded together.
  static_assert(!FIN || U <= FIN_SLOTS, "a batch must fit the slots");
  __shared__ double fin_a[FIN ? FIN_SLOTS : 1][FIN ? MAX_FIN_GROUPS : 1];
  __shared__ double fin_q[FIN ? FIN_SLOTS : 1][FIN ? MAX_FIN_GROUPS : 1];
  __shared__ int64_t fin_r1[FIN ? FIN_SLOTS : 1][FIN ? MAX_FIN_GROUPS : 1];
  __shared__ int64_t fin_r2[FIN ? FIN_SLOTS : 1][FIN ? MAX_FIN_GROUPS : 1];
  __shared__ int32_t fin_n[FIN ? FIN_SLOTS : 1][FIN ? MAX_FIN_GROUPS : 1];
  int pend = 0;                                                // blocks waiting in LDS
  const int lane = threadIdx.x & 63;
  const int g = z * 4 + (threadIdx.x >> 6);                   // input group of 64*V
  const int N = a.n_inputs, L = a.window, H = a.hist_len;
  const int i0 = (g * 64 + lane) * V;
  if (g >= a.n_groups) return;                                 // whole wavefront exits
  const bool active = i0 < N;
  const int64_t total = (int64_t)H + a.n_blocks;
  int64_t e0 = (int64_t)c * a.chunk;
  if (e0 < H) e0 = H;
  int64_t e1 = (int64_t)(c + 1) * a.chunk;
  if (e1 > total) e1 = total;
  if (e0 >= e1) return;
  const int64_t hist_from = total - a.hist_next_len;          // first e of the next history

  int32_t P[V];
#pragma unroll
  for (int k = 0; k < V; ++k) P[k] = 0;
  uint32_t use_mask = 0;
  if (active) {
    if (L >= 2) window_sum<V>(a, f, e0 - L > 0 ? e0 - L : 0, e0, i0, P);
#pragma unroll
    for (int k = 0; k < V; ++k)
      if (a.mask == nullptr || a.mask[(int64_t)f * N + i0 + k] != 0) use_mask |= 1u << k;
  }

  for (int64_t eb = e0; eb < e1; eb += U) {
    IVec<V> x1[U], x2[U], old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = eb + u;
#pragma unroll
      for (int k = 0; k < V; ++k) x1[u].v[k] = x2[u].v[k] = old[u].v[k] = 0;
      if (active && e < e1) {
        const int64_t row = ((int64_t)f * a.n_blocks + (e - H)) * N + i0;
        x1[u].load(a.s1 + row);
        x2[u].load(a.s2 + row);
        if (L >= 2 && e - L >= 0) old[u].load(seq_row(a, f, e - L) + i0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = eb + u;
      if (e >= e1) break;
      double pa = 0.0, pq = 0.0;
      RI r1 = 0, r2 = 0;
      int32_t n = 0;
      if (active) {
        if (L >= 2) {
#pragma unroll
          for (int k = 0; k < V; ++k) P[k] += x1[u].v[k] - old[u].v[k];
          if (e >= hist_from) x1[u].store(a.hist_next + ((int64_t)f * a.hist_cap + (e - hist_from)) * N + i0);
        } else {
#pragma unroll
          for (int k = 0; k < V; ++k) P[k] = x1[u].v[k];
        }
        if (a.sk_i) {
          // Eq. originalSK for every input of this block (masked or not).
          float ski[V];
#pragma unroll
          for (int k = 0; k < V; ++k) ski[k] = per_input_sk(x1[u].v[k], x2[u].v[k], a.block_len);
          float* dst = a.sk_i + ((int64_t)f * a.n_blocks + (e - H)) * N + i0;
#pragma unroll
          for (int k = 0; k < V; ++k) dst[k] = ski[k];
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
          if ((use_mask >> k & 1u) && P[k] > 0) {
            n += 1;
            r1 += x1[u].v[k];
            r2 += x2[u].v[k];
            if (L >= 1) {
              const double rp = recip_pos((double)P[k]);
              pa += (double)x1[u].v[k] * rp;
              pq += (double)x2[u].v[k] * rp * rp;
            }
          }
        }
      }
      pa = wave_sum_to_last(pa);
      pq = wave_sum_to_last(pq);
      r1 = wave_sum_to_last(r1);
      r2 = wave_sum_to_last(r2);
      n = wave_sum_to_last(n);
      if constexpr (FIN) {
        if (lane == 63) {
          fin_a[pend + u][g] = pa;
          fin_q[pend + u][g] = pq;
          fin_r1[pend + u][g] = (int64_t)r1;
          fin_r2[pend + u][g] = (int64_t)r2;
          fin_n[pend + u][g] = n;
        }
      } else if (lane == 63) {
        const int64_t o = ((int64_t)f * a.n_groups + g) * a.n_blocks + (e - H);
        a.part_a[o] = pa;
        a.part_q[o] = pq;
        a.part_r1[o] = (int64_t)r1;
        a.part_r2[o] = (int64_t)r2;
        a.part_n[o] = n;
      }
    }
    if constexpr (FIN) {
      const int nb = e1 - eb < U ? (int)(e1 - eb) : U;
      pend += nb;
      if (eb + U >= e1 || pend + U > FIN_SLOTS) {
        // Slot j holds block e = eb + nb - pend + j. It is finished by lane
        // j / W of wavefront j % W (W wavefronts), spreading the work; the
        // second barrier keeps the slots until every finisher is done.
        __syncthreads();
        const int nw = (int)(blockDim.x >> 6);
        const int j = (threadIdx.x & 63) * nw + (threadIdx.x >> 6);
        if (j < pend) {
          double A = 0.0, Bq = 0.0;
          int64_t R1 = 0, R2 = 0;
          int32_t nn = 0;
          for (int gg = 0; gg < a.n_groups; ++gg) {
            A += fin_a[j][gg];
            Bq += fin_q[j][gg];
            R1 += fin_r1[j][gg];
            R2 += fin_r2[j][gg];
            nn += fin_n[j][gg];
          }
          finish(a, f, (int)(eb + nb - pend + j - H), A, Bq, R1, R2, nn);
        }
        __syncthreads();
        pend = 0;
      }
    }
  }
}

template <int V, int U = 4, bool FIN = false>
__device__ __forceinline__ void partial_body(const PassBArgs& a, int c, int f, int z) {
  // S2 of one input is at most M * 128^2 = M * 2^14 (Eq. singlesums).
  if ((int64_t)64 * V * a.block_len * 16384 < ((int64_t)1 << 31))
    partial_body_t<V, int32_t, U, FIN>(a, c, f, z);
  else
    partial_body_t<V, int64_t, U, FIN>(a, c, f, z);
}


__device__ __forceinline__ void finalize_body(const PassBArgs& a, int64_t blk) {
  const int64_t j = blk * 256 + threadIdx.x;
  if (j >= (int64_t)a.n_channels * a.fin_nb) return;
  const int f = (int)(j / a.fin_nb), b = a.fin_b0 + (int)(j % a.fin_nb);
  double A = 0.0, Bq = 0.0;
  int64_t R1 = 0, R2 = 0;
  int32_t n = 0;
  // Group order is fixed; the loads of 8 groups are issued together.
#pragma unroll 8
  for (int g = 0; g < a.n_groups; ++g) {
    const int64_t o = ((int64_t)f * a.n_groups + g) * a.n_blocks + b;
    A += a.part_a[o];
    Bq += a.part_q[o];
    R1 += a.part_r1[o];
    R2 += a.part_r2[o];
    n += a.part_n[o];
  }
  finish(a, f, b, A, Bq, R1, R2, n);
}

__device__ __forceinline__ void hist_copy_body(const PassBArgs& a, int j, int f, int z) {
  const int i = z * 256 + threadIdx.x;
  if (i >= a.n_inputs || j >= a.hist_next_len - a.n_blocks) return;
  const int64_t src = (int64_t)a.hist_len + a.n_blocks - a.hist_next_len + j;   // < hist_len
  a.hist_next[((int64_t)f * a.hist_cap + j) * a.n_inputs + i] =
      a.hist[((int64_t)f * a.hist_cap + src) * a.n_inputs + i];
}

// The same carry with four inputs per thread (N % 4 == 0, 16-byte rows).
__device__ __forceinline__ void hist_copy_body_v4(const PassBArgs& a, int j, int f, int z) {
  const int i = (z * 256 + threadIdx.x) * 4;
  if (i >= a.n_inputs || j >= a.hist_next_len - a.n_blocks) return;
  const int64_t src = (int64_t)a.hist_len + a.n_blocks - a.hist_next_len + j;   // < hist_len
  *reinterpret_cast<int4*>(a.hist_next + ((int64_t)f * a.hist_cap + j) * a.n_inputs + i) =
      *reinterpret_cast<const int4*>(a.hist + ((int64_t)f * a.hist_cap + src) * a.n_inputs + i);
}

}  // namespace sk
