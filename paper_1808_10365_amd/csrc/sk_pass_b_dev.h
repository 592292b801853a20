// Pass B device code shared by the single-plan and batched kernels: the
// normaliser window (Eq. discreteMean, running form), the array combine
// (Eq. normedSum1, normedSum2), the estimator (Eq. avgSK, final) and the
// flags (Sec. 3.2).
//
// Positions. Per (channel f, input i) the blocks of a call are positions
// b = 0 .. B-1; the history, the last H <= L-1 blocks of earlier calls, sits
// at positions -H .. -1. The window of block b is [max(b - L + 1, -H), b].
//
// State. The history is kept as suffix sums HS(y) = sum of S1 over positions
// [y, 0), y in [-H, 0) (HS(0) = 0, and HS(y) = HS(-H) for y < -H), one int32
// per (f, slot, i) with slot = y + L - 1. A history block is the difference
// of two neighbours, and the window's history part is one value.
//
// Kernels.
//   scan     (L >= 2) exclusive prefix sums of S1 at the chunk boundaries of
//            the call, PC[k] = sum of S1 over [0, k R) (mod 2^32: every
//            difference that is used is a window sum < 2^31, so it is exact),
//            one lane per (f, i), a workgroup's wavefronts over consecutive
//            chunk ranges joined through LDS. It also carries the older
//            history into the next call's suffix sums when a call is shorter
//            than the window.
//   combine  one workgroup per (f, chunk k of R blocks), one wavefront per
//            64 V inputs. The window sum before the chunk is at most two
//            prefix values, R - 1 edge rows and one history value; then the
//            sliding update P += S1[b] - S1[b - L] over the chunk. Per input
//            FP64 S1/P and S2/P^2 and the raw int sums, wavefront sums in a
//            fixed tree, wavefronts joined in LDS in a fixed order, then the
//            estimator and flags of the chunk's blocks. It also writes the
//            next call's history suffix sums for its blocks.
// Every load of a wavefront is issued before any of them is used, so a
// combine wavefront costs one memory round trip.
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

template <int V>
__device__ __forceinline__ void zero(IVec<V>& x) {
#pragma unroll
  for (int k = 0; k < V; ++k) x.v[k] = 0;
}

// ------------------------------------------------------------------ wavefront sums
//
// One fixed tree for every value: lanes l and l + 32 first (v_permlane32_swap),
// then rows 0 + 1 and 2 + 3 of the result (v_permlane16_swap), then within a
// row of 16 lanes l + 8, l + 4, l + 2, l + 1 (DPP row rotations). Two values
// share each swap step (a reduce-scatter), so n values cost about n/4 of n
// separate reductions, and each value is added in the same order whichever
// values it is reduced with: results do not depend on the tile.

template <typename T>
__device__ __forceinline__ void swap_halves(T& x, T& y) {
  // After the swap, x holds x's lanes 0-31 and y's lanes 0-31 (in lanes
  // 32-63); y holds x's lanes 32-63 (in lanes 0-31) and y's lanes 32-63.
  if constexpr (sizeof(T) == 4) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, x), __builtin_bit_cast(uint32_t, y),
                                                    false, false);
    x = __builtin_bit_cast(T, (uint32_t)r[0]);
    y = __builtin_bit_cast(T, (uint32_t)r[1]);
  } else {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    u2 a = __builtin_bit_cast(u2, x), b = __builtin_bit_cast(u2, y);
    const auto r0 = __builtin_amdgcn_permlane32_swap(a.x, b.x, false, false);
    const auto r1 = __builtin_amdgcn_permlane32_swap(a.y, b.y, false, false);
    a.x = r0[0]; b.x = r0[1];
    a.y = r1[0]; b.y = r1[1];
    x = __builtin_bit_cast(T, a);
    y = __builtin_bit_cast(T, b);
  }
}

template <typename T>
__device__ __forceinline__ void swap_rows(T& x, T& y) {
  // Rows of 16 lanes: x becomes (x0, y0, x2, y2), y becomes (x1, y1, x3, y3).
  if constexpr (sizeof(T) == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, x), __builtin_bit_cast(uint32_t, y),
                                                    false, false);
    x = __builtin_bit_cast(T, (uint32_t)r[0]);
    y = __builtin_bit_cast(T, (uint32_t)r[1]);
  } else {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    u2 a = __builtin_bit_cast(u2, x), b = __builtin_bit_cast(u2, y);
    const auto r0 = __builtin_amdgcn_permlane16_swap(a.x, b.x, false, false);
    const auto r1 = __builtin_amdgcn_permlane16_swap(a.y, b.y, false, false);
    a.x = r0[0]; b.x = r0[1];
    a.y = r1[0]; b.y = r1[1];
    x = __builtin_bit_cast(T, a);
    y = __builtin_bit_cast(T, b);
  }
}

// Lane l + r (mod 16, within its row) of v, every row enabled.
template <int R, typename T>
__device__ __forceinline__ T row_rot(T v) {
  constexpr int CTRL = 0x120 + R;   // DPP row_ror:R
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
  } else {
    typedef int i2 __attribute__((ext_vector_type(2)));
    i2 a = __builtin_bit_cast(i2, v);
    a.x = __builtin_amdgcn_mov_dpp(a.x, CTRL, 0xF, 0xF, false);
    a.y = __builtin_amdgcn_mov_dpp(a.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, a);
  }
}

template <typename T>
__device__ __forceinline__ T row_total(T v) {
  v = v + row_rot<8>(v);
  v = v + row_rot<4>(v);
  v = v + row_rot<2>(v);
  v = v + row_rot<1>(v);
  return v;
}

// Sums each of NV values (NV a power of two >= 2) over the wavefront.
// Value j ends in every lane of the row of out[j / 4] that
// wave_value_of_row names.
template <int NV, typename T>
__device__ __forceinline__ void wave_sums(const T (&v)[NV], T (&out)[(NV + 3) / 4]) {
  static_assert(NV >= 2 && (NV & (NV - 1)) == 0, "a power of two, at least 2");
  constexpr int NC = NV / 2;
  T c[NC];
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    T x = v[2 * m], y = v[2 * m + 1];
    swap_halves(x, y);
    c[m] = x + y;
  }
#pragma unroll
  for (int q = 0; q < (NV + 3) / 4; ++q) {
    T x = c[2 * q], y = 2 * q + 1 < NC ? c[2 * q + 1] : c[2 * q];
    swap_rows(x, y);
    out[q] = row_total(x + y);
  }
}

// The value a lane of row r holds in out[q] after wave_sums: 4q + 2 (r & 1) + (r >> 1).
__device__ __forceinline__ int wave_value_of_row(int q, int r) { return 4 * q + 2 * (r & 1) + (r >> 1); }

// ------------------------------------------------------------------ estimator

// Eq. originalSK: (M+1)/(M-1) (M S2 / S1^2 - 1), NaN where S1 = 0.
__device__ __forceinline__ float per_input_sk(int32_t s1, int32_t s2, int32_t block_len) {
#pragma clang fp contract(off)
  if (s1 == 0) return __builtin_nanf("");
  const double Md = (double)block_len, x = (double)s1;
  return (float)((Md + 1.0) / (Md - 1.0) * (Md * (double)s2 / (x * x) - 1.0));
}

// 1/p for p >= 1: the hardware reciprocal estimate (relative error about
// 2^-24 on gfx950) refined by two Newton steps, each squaring the error, to
// within an ulp of the correctly rounded quotient. One step would leave
// about 2^-48, enough for the tolerance on V but not for exact results such
// as V = 0 on constant-modulus input. S1/P and S2/P^2 then cost multiplies.
__device__ __forceinline__ double recip_pos(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = __builtin_fma(-p, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-p, r, 1.0);
  return __builtin_fma(r, e, r);
}

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

// Index of the calling wavefront in its workgroup, in a scalar register (the
// compiler cannot tell on its own that it is the same for every lane, and
// would keep everything derived from it per lane).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// ------------------------------------------------------------------ scan
// ------------------------------------------------------------------ scan

constexpr int SCAN_MAX_WAVES = 16;

// History rows a scan wavefront moves per group (all loads, then all stores).
constexpr int SHIFT_ROWS = 16;

// History blocks that stay in the window of the next call (a call shorter
// than the window): their suffix sums grow by the whole call, `carry`.
// Next-call slot s holds position s - Hc, which is old position s - Hc + B,
// so it reads old slot s + B. Wavefront w of W takes groups of SHIFT_ROWS
// rows; a group's loads all issue before its stores (the two history buffers
// are distinct), so a short call against a long window does not walk its
// rows one load at a time.
__device__ __forceinline__ void shift_history(const PassBArgs& a, int f, int i, bool active, uint32_t carry,
                                              int w, int W) {
  const int Hc = a.hist_cap, B = a.n_blocks;
  const int from = Hc - a.hist_next_len, to = Hc - B;
  if (!active || !a.hs_next || from >= to) return;
  const int64_t rowN = a.n_inputs;
  const int32_t* src = a.hs + ((int64_t)f * Hc + B) * rowN + i;
  int32_t* dst = a.hs_next + (int64_t)f * Hc * rowN + i;
  const bool had = a.hist_len > 0;
  for (int s0 = from + w * SHIFT_ROWS; s0 < to; s0 += W * SHIFT_ROWS) {
    int32_t old[SHIFT_ROWS];
#pragma unroll
    for (int j = 0; j < SHIFT_ROWS; ++j) old[j] = (had && s0 + j < to) ? src[(int64_t)(s0 + j) * rowN] : 0;
#pragma unroll
    for (int j = 0; j < SHIFT_ROWS; ++j)
      if (s0 + j < to) dst[(int64_t)(s0 + j) * rowN] = (int32_t)((uint32_t)old[j] + carry);
  }
}

// Wavefronts the history shift of one 64-input slice can use: its rows in
// SHIFT_ROWS groups (0 when the call is at least as long as the window).
__host__ __device__ __forceinline__ int64_t shift_groups(int64_t hist_next_len, int64_t n_blocks) {
  const int64_t rows = hist_next_len - n_blocks;
  return rows > 0 ? (rows + SHIFT_ROWS - 1) / SHIFT_ROWS : 0;
}

// Chunks a scan lane holds per round: 64 rows of S1 in flight at most.
template <int R>
constexpr int scan_chunks_per_lane() { return 64 / R; }

// One workgroup of W wavefronts: channel f, inputs [64 slice, 64 slice + 64),
// one input per lane. Wavefront w takes chunks [k0, k0 + C) of each round of
// C W chunks (C = 64 / R); the rounds carry the running prefix. S1 of a
// chunk is the pass A chunk sum when the call has them (a.cs), else the sum
// of its R rows. lds: W * 64 words.
template <int R>
__device__ __forceinline__ void scan_body(const PassBArgs& a, int f, int slice, int w, int W, uint32_t* lds) {
  constexpr int C = scan_chunks_per_lane<R>();
  const int lane = threadIdx.x & 63;
  const int i = slice * 64 + lane;
  const bool active = i < a.n_inputs;
  const int nk = a.n_chunks, B = a.n_blocks;
  const int64_t rowN = a.n_inputs;
  uint32_t* pc = a.pc + (int64_t)f * (nk + 1) * rowN + i;
  if (w == 0 && active) pc[0] = 0u;
  uint32_t carry = 0;   // prefix before this round, for this lane's input
  for (int base = 0; base < nk; base += C * W) {
    const int k0 = base + w * C;
    uint32_t cs[C];
    if (a.cs) {
      const int32_t* p = a.cs + ((int64_t)f * nk + k0) * rowN + i;
#pragma unroll
      for (int j = 0; j < C; ++j) cs[j] = (active && k0 + j < nk) ? (uint32_t)p[(int64_t)j * rowN] : 0u;
    } else {
      uint32_t x[C][R];
      const int32_t* p = a.s1 + ((int64_t)f * B + (int64_t)k0 * R) * rowN + i;
#pragma unroll
      for (int j = 0; j < C; ++j)
#pragma unroll
        for (int r = 0; r < R; ++r)
          x[j][r] = (active && (k0 + j) * R + r < B) ? (uint32_t)p[(int64_t)(j * R + r) * rowN] : 0u;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        uint32_t t = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) t += x[j][r];
        cs[j] = t;
      }
    }
#pragma unroll
    for (int j = 1; j < C; ++j) cs[j] += cs[j - 1];
    lds[w * 64 + lane] = cs[C - 1];
    __syncthreads();
    uint32_t off = carry, all = carry;
    for (int q = 0; q < W; ++q) {
      const uint32_t t = lds[q * 64 + lane];
      if (q < w) off += t;
      all += t;
    }
    carry = all;
    if (active) {
#pragma unroll
      for (int j = 0; j < C; ++j)
        if (k0 + j < nk) pc[(int64_t)(k0 + j + 1) * rowN] = off + cs[j];
    }
    __syncthreads();
  }
  shift_history(a, f, i, active, carry, w, W);
}

// The same scan for a chunk length known only at run time (the batched
// kernel's problems differ in it): each lane holds SCAN_ROWS units (rows of
// S1, or pass A's chunk sums) per round and writes its running sum at every
// chunk end, so the registers do not depend on the chunk length. Rounds are
// SCAN_ROWS W units; R (a power of two) divides SCAN_ROWS. The prefix values
// are exact integers mod 2^32, equal to scan_body's.
constexpr int SCAN_ROWS = 32;

__device__ __forceinline__ void scan_body_rows(const PassBArgs& a, int f, int slice, int w, int W, uint32_t* lds) {
  // Units: the chunk sums from pass A when the call has them (every unit
  // ends a chunk), else the rows of S1 (a chunk ends every R rows).
  const int nk = a.n_chunks, B = a.n_blocks;
  const int U = a.cs ? nk : B;
  const int R = a.cs ? 1 : a.chunk, lgR = __builtin_ctz((unsigned)R);
  const int lane = threadIdx.x & 63;
  const int i = slice * 64 + lane;
  const bool active = i < a.n_inputs;
  const int64_t rowN = a.n_inputs;
  uint32_t* pc = a.pc + (int64_t)f * (nk + 1) * rowN + i;
  if (w == 0 && active) pc[0] = 0u;
  const int32_t* src = a.cs ? a.cs + (int64_t)f * nk * rowN + i : a.s1 + (int64_t)f * B * rowN + i;
  uint32_t carry = 0;
  for (int base = 0; base < U; base += SCAN_ROWS * W) {
    const int r0 = base + w * SCAN_ROWS;
    uint32_t x[SCAN_ROWS];
    const int32_t* p = src + (int64_t)r0 * rowN;
#pragma unroll
    for (int r = 0; r < SCAN_ROWS; ++r) x[r] = (active && r0 + r < U) ? (uint32_t)p[(int64_t)r * rowN] : 0u;
    uint32_t tot = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ROWS; ++r) tot += x[r];
    lds[w * 64 + lane] = tot;
    __syncthreads();
    uint32_t off = carry, all = carry;
    for (int q = 0; q < W; ++q) {
      const uint32_t t = lds[q * 64 + lane];
      if (q < w) off += t;
      all += t;
    }
    carry = all;
    if (active) {
#pragma unroll
      for (int r = 0; r < SCAN_ROWS; ++r) {
        off += x[r];
        const int row = r0 + r;
        // Chunk c ends at unit c R + R - 1, or at U - 1 for a short last chunk.
        if (row < U && (((row + 1) & (R - 1)) == 0 || row == U - 1)) pc[(int64_t)((row + R) >> lgR) * rowN] = off;
      }
    }
    __syncthreads();
  }
  shift_history(a, f, i, active, carry, w, W);
}

// Waves per slice of the batched scan: a power of two covering the call's
// rows in SCAN_ROWS-row lanes, at most max_waves (a power of two: the
// workgroup's wavefronts, so slices tile it).
__host__ __device__ __forceinline__ int scan_rows_waves(int64_t n_blocks, int max_waves) {
  int W = 1;
  while (W < max_waves && (int64_t)W * SCAN_ROWS < n_blocks) W *= 2;
  return W;
}

// Whether a call needs the prefix scan. With a window of at most one chunk
// (L <= R) no combine workgroup reads prefix sums: a window start lies in the
// chunk before, as edge rows. When the call also spans the window
// (B >= L - 1) no older history is carried either, and the combine forms the
// next history's suffix sums from the rows it reads.
__host__ __device__ __forceinline__ bool pass_b_needs_scan(int window, int chunk, int64_t n_blocks) {
  return window >= 2 && !(window <= chunk && n_blocks >= window - 1);
}

// ------------------------------------------------------------------ combine

constexpr int COMBINE_MAX_WAVES = 8;
constexpr int COMBINE_MAX_R = 4;

struct CombineShared {
  double A[COMBINE_MAX_R][COMBINE_MAX_WAVES];
  double Q[COMBINE_MAX_R][COMBINE_MAX_WAVES];
  int64_t R1[COMBINE_MAX_R][COMBINE_MAX_WAVES];
  int64_t R2[COMBINE_MAX_R][COMBINE_MAX_WAVES];
  int32_t n[COMBINE_MAX_R][COMBINE_MAX_WAVES];
};

// Element `e` of a per-channel array. OFF32: the offset is a 32-bit byte
// count added to a uniform base, so each load takes one scalar base and a
// vector offset (fewer scalar registers than a 64-bit address per row).
template <bool OFF32>
__device__ __forceinline__ const int32_t* elem_at(const int32_t* base, int64_t e) {
  if constexpr (OFF32)
    return reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(base) + (uint32_t)((uint32_t)e * 4u));
  else
    return base + e;
}

// Chunk k of channel f, wavefront w of W. R blocks per chunk, V inputs per
// lane, RI the integer type of a lane's R1/R2 sums, OFF32 when every
// per-channel array holds fewer than 2^30 elements.
//
// Every lane loads: a lane past the last input reads the last group's
// inputs (in bounds) and contributes nothing. Loads that a chunk does not
// need are replaced by zeros in wavefront-uniform branches.
template <int V, int R, typename RI, bool OFF32>
__device__ __forceinline__ void combine_body(const PassBArgs& a, int k, int f, int w, int W, CombineShared& sh,
                                             bool live = true) {
  static_assert(R >= 1 && R <= COMBINE_MAX_R && (R & (R - 1)) == 0, "R a power of two <= 4");
  if (!live) {
    // A wavefront group with no chunk: meet the workgroup's one barrier.
    __syncthreads();
    return;
  }
  constexpr int RO = R > 1 ? R - 1 : 1;               // old-row slots
  const int lane = threadIdx.x & 63;
  const int N = a.n_inputs, L = a.window, H = a.hist_len, B = a.n_blocks;
  const int b0 = k * R;
  const int nb = B - b0 < R ? B - b0 : R;
  const int wa = b0 - L + 1;                          // first position of block b0's window
  const int n_groups = (N + 64 * V - 1) / (64 * V);
  // Prefix values the window start needs (L >= 2): PC[k] - PC[kc], kc the
  // first chunk boundary at or after max(wa, 0); positions [max(wa, 0), kc R)
  // are edge rows, a subset of the R - 1 old rows [wa, wa + R - 1).
  const int kc = wa <= 0 ? 0 : (wa + R - 1) / R;
  const bool use_pc = L >= 2 && kc < k;
  const bool scan_free = L >= 2 && !pass_b_needs_scan(L, R, B);   // no prefix sums this call
  const int edges = L >= 2 && wa > 0 ? (kc * R < b0 ? kc * R : b0) - wa : 0;
  const int hn = a.hist_next_len;
  const int tail_from = B - hn;                       // first position of the next history
  const bool tail = L >= 2 && a.hs_next && b0 + nb > tail_from;   // this chunk writes next-history sums
  const bool head = L >= 2 && wa < 0 && H > 0;        // the window reaches into the history
  const int64_t rowF = (int64_t)f * B;
  // Channel bases (uniform).
  const int32_t* s1c = a.s1 + rowF * N;
  const int32_t* s2c = a.s2 + rowF * N;
  const int32_t* pcc = reinterpret_cast<const int32_t*>(a.pc) + (int64_t)f * (a.n_chunks + 1) * N;
  const int32_t* hsc = a.hs + (int64_t)f * a.hist_cap * N;

  double accA[R], accQ[R];
  RI acc1[R], acc2[R];
  int cnt[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    accA[j] = accQ[j] = 0.0;
    acc1[j] = acc2[j] = 0;
    cnt[j] = 0;
  }

  for (int g = w; g < n_groups; g += W) {
    const int i0 = (g * 64 + lane) * V;
    const bool active = i0 < N;
    const int il = active ? i0 : N - V;               // the input this lane loads
    IVec<V> x1[R], x2[R], old[RO], hsv[R], pck, pcl, pct;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j < nb) {
        const int64_t e = (int64_t)(b0 + j) * N + il;
        x1[j].load(elem_at<OFF32>(s1c, e));
        x2[j].load(elem_at<OFF32>(s2c, e));
      } else {
        zero(x1[j]);
        zero(x2[j]);
      }
    }
    if (L >= 2) {
#pragma unroll
      for (int j = 0; j < RO; ++j) {
        const int y = wa + j;               // rows past the call's end are never used
        if (R > 1 && y >= 0 && y < B) old[j].load(elem_at<OFF32>(s1c, (int64_t)y * N + il));
        else zero(old[j]);
      }
      if (head) {
        // History suffix sums at positions wa .. wa + R - 1 (clamped to -H;
        // positions >= 0 have none). Old rows in the history are differences.
#pragma unroll
        for (int j = 0; j < R; ++j) {
          int y = wa + j;
          if (y < 0) hsv[j].load(elem_at<OFF32>(hsc, (int64_t)((y < -H ? -H : y) + a.hist_cap) * N + il));
          else zero(hsv[j]);
        }
#pragma unroll
        for (int j = 0; j < RO; ++j) {
          if (R > 1 && wa + j < 0) {
#pragma unroll
            for (int q = 0; q < V; ++q) old[j].v[q] = hsv[j].v[q] - (wa + j + 1 < 0 ? hsv[j + 1].v[q] : 0);
          }
        }
      } else {
        zero(hsv[0]);
      }
      if (!scan_free && (use_pc || tail) && k > 0) pck.load(elem_at<OFF32>(pcc, (int64_t)k * N + il));
      else zero(pck);
      if (use_pc && kc > 0) pcl.load(elem_at<OFF32>(pcc, (int64_t)kc * N + il));
      else zero(pcl);
      if (tail && !scan_free) pct.load(elem_at<OFF32>(pcc, (int64_t)a.n_chunks * N + il));
      if (tail && scan_free) {
        // S1 from the chunk's first block to the end of the call: its own rows
        // plus the at most R - 2 rows after it (pck is zero, so the next
        // history's suffix sums below come out as pct minus the rows before).
        IVec<V> after;
        zero(after);
#pragma unroll
        for (int j = 0; j < RO; ++j) {
          const int y = b0 + nb + j;
          if (R > 1 && y < B) {
            IVec<V> r;
            r.load(elem_at<OFF32>(s1c, (int64_t)y * N + il));
#pragma unroll
            for (int q = 0; q < V; ++q) after.v[q] = (int32_t)((uint32_t)after.v[q] + (uint32_t)r.v[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < V; ++q) {
          uint32_t t = (uint32_t)after.v[q];
#pragma unroll
          for (int j = 0; j < R; ++j)
            if (j < nb) t += (uint32_t)x1[j].v[q];
          pct.v[q] = (int32_t)t;
        }
      }
    }
    uint32_t use = active ? (1u << V) - 1 : 0u;
    if (a.mask) {
#pragma unroll
      for (int q = 0; q < V; ++q)
        if (a.mask[(int64_t)f * N + il + q] == 0) use &= ~(1u << q);
    }

    // Window sums, block by block (uint32 arithmetic, exact below 2^31).
    uint32_t P[V], pre[V];
    if (L >= 2) {
#pragma unroll
      for (int q = 0; q < V; ++q) {
        P[q] = (uint32_t)hsv[0].v[q] + (use_pc ? (uint32_t)pck.v[q] - (uint32_t)pcl.v[q] : 0u);
        pre[q] = (uint32_t)pck.v[q];                  // S1 of this call before the block
      }
#pragma unroll
      for (int j = 0; j < RO; ++j)
        if (j < edges) {
#pragma unroll
          for (int q = 0; q < V; ++q) P[q] += (uint32_t)old[j].v[q];
        }
    }
    uint32_t inc[R];                                  // bit q: input q of block j is included
    bool all_in = true;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      inc[j] = 0;
      if (j >= nb) break;
      if (L >= 2) {
#pragma unroll
        for (int q = 0; q < V; ++q) {
          if (j > 0) P[q] -= (uint32_t)old[j - 1].v[q];
          P[q] += (uint32_t)x1[j].v[q];
        }
        if (tail && b0 + j >= tail_from) {
          if (active) {
            IVec<V> h;
#pragma unroll
            for (int q = 0; q < V; ++q) h.v[q] = (int32_t)((uint32_t)pct.v[q] - pre[q]);
            h.store(a.hs_next + ((int64_t)f * a.hist_cap + (b0 + j - B + a.hist_cap)) * N + i0);
          }
        }
#pragma unroll
        for (int q = 0; q < V; ++q) pre[q] += (uint32_t)x1[j].v[q];
      } else {
#pragma unroll
        for (int q = 0; q < V; ++q) P[q] = (uint32_t)x1[j].v[q];
      }
      if (a.sk_i && active) {
        float ski[V];
#pragma unroll
        for (int q = 0; q < V; ++q) ski[q] = per_input_sk(x1[j].v[q], x2[j].v[q], a.block_len);
        float* dst = a.sk_i + (rowF + b0 + j) * N + i0;
#pragma unroll
        for (int q = 0; q < V; ++q) dst[q] = ski[q];
      }
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const bool in = (use >> q & 1u) && (int32_t)P[q] > 0;
        const uint64_t bal = __ballot(in);
        cnt[j] += __builtin_popcountll(bal);
        all_in = all_in && bal == ~0ull;
        inc[j] |= (uint32_t)in << q;
      }
      if (L >= 1) {
        // Reciprocals now, while P holds this block's window.
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const double rp = recip_pos((double)P[q]);
          if (all_in) {
            accA[j] = __builtin_fma((double)x1[j].v[q], rp, accA[j]);
            accQ[j] = __builtin_fma((double)x2[j].v[q] * rp, rp, accQ[j]);
          } else {
            const double rs = (inc[j] >> q & 1u) ? rp : 0.0;
            accA[j] = __builtin_fma((double)x1[j].v[q], rs, accA[j]);
            accQ[j] = __builtin_fma((double)x2[j].v[q] * rs, rs, accQ[j]);
          }
        }
      }
    }
    // Raw integer sums of the included inputs.
    if (all_in) {
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int q = 0; q < V; ++q) {
          acc1[j] += (RI)x1[j].v[q];
          acc2[j] += (RI)x2[j].v[q];
        }
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j)
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const bool in = inc[j] >> q & 1u;
          acc1[j] += in ? (RI)x1[j].v[q] : (RI)0;
          acc2[j] += in ? (RI)x2[j].v[q] : (RI)0;
        }
    }
  }

  // Wavefront sums: (A, Bq) of each block as 2R doubles, (R1, R2) as 2R ints.
  {
    constexpr int NV = 2 * R;
    double dv[NV];
    RI iv[NV];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      dv[2 * j] = accA[j];
      dv[2 * j + 1] = accQ[j];
      iv[2 * j] = acc1[j];
      iv[2 * j + 1] = acc2[j];
    }
    double dout[(NV + 3) / 4];
    RI iout[(NV + 3) / 4];
    wave_sums<NV>(dv, dout);
    wave_sums<NV>(iv, iout);
    const int r = lane >> 4;
    if ((lane & 15) == 0) {
#pragma unroll
      for (int q = 0; q < (NV + 3) / 4; ++q) {
        const int val = wave_value_of_row(q, r);
        if (val < NV) {
          const int j = val >> 1;
          if (val & 1) {
            sh.Q[j][w] = dout[q];
            sh.R2[j][w] = (int64_t)iout[q];
          } else {
            sh.A[j][w] = dout[q];
            sh.R1[j][w] = (int64_t)iout[q];
          }
        }
      }
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) sh.n[j][w] = cnt[j];
    }
  }
  __syncthreads();
  if (w == 0 && lane < nb) {
    const int j = lane;
    double A = 0.0, Bq = 0.0;
    int64_t R1 = 0, R2 = 0;
    int32_t n = 0;
    for (int q = 0; q < W; ++q) {
      A += sh.A[j][q];
      Bq += sh.Q[j][q];
      R1 += sh.R1[j][q];
      R2 += sh.R2[j][q];
      n += sh.n[j][q];
    }
    finish(a, f, b0 + j, A, Bq, R1, R2, n);
  }
}

// Waves of a combine workgroup for N inputs at V per lane.
__host__ __device__ __forceinline__ int combine_waves(int n_inputs, int vec) {
  const int g = (n_inputs + 64 * vec - 1) / (64 * vec);
  return g < COMBINE_MAX_WAVES ? g : COMBINE_MAX_WAVES;
}

// Waves of a scan workgroup for nk chunks.
__host__ __device__ __forceinline__ int scan_waves(int n_chunks) {
  return n_chunks < SCAN_MAX_WAVES ? (n_chunks > 0 ? n_chunks : 1) : SCAN_MAX_WAVES;
}

// Whether every per-channel array of a call (S1, S2, prefix sums, history)
// holds fewer than 2^30 elements, so 32-bit byte offsets reach all of it.
__host__ __device__ __forceinline__ bool combine_offsets_fit_32(int n_inputs, int64_t n_blocks, int n_chunks,
                                                                int hist_cap) {
  const int64_t lim = (int64_t)1 << 30;
  return n_blocks * n_inputs < lim && ((int64_t)n_chunks + 1) * n_inputs < lim && (int64_t)hist_cap * n_inputs < lim;
}

// Integer type of a lane's R1/R2 sums: 32 bits while a whole wavefront's
// S2 sums fit (64 V M 2^14 < 2^31, S2 of one input <= M 2^14), over all the
// groups a wavefront takes.
__host__ __device__ __forceinline__ bool combine_sums_fit_32(int n_inputs, int vec, int block_len) {
  const int W = combine_waves(n_inputs, vec);
  const int64_t groups = (n_inputs + 64 * vec - 1) / (64 * vec);
  const int64_t per_wave = (groups + W - 1) / W;
  return per_wave * 64 * vec * (int64_t)block_len * 16384 < ((int64_t)1 << 31);
}

}  // namespace sk
