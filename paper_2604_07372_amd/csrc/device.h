// Device-side building blocks shared by the NS-RGS kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsrgs.h"

namespace nsrgs {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxD = 16;          // largest block size d supported
constexpr int kMaxWaves = 8;       // waves per workgroup in the streaming kernels

// --------------------------------------------------------------------------
// Control block at the start of every workspace.  All fields are written by
// kernels only; the host reads them back with a copy.  `arrive*` counters are
// zero between launches (the last arriving workgroup resets them).
// --------------------------------------------------------------------------
struct alignas(256) DevCtl {
  unsigned int arrive;        // step kernel: arrivals of the current launch
  unsigned int arrive2;       // init kernels: arrivals of the current launch
  int done;                   // solve: stop flag (tolerance met or non-finite)
  int iters;                  // solve: iterations completed (t + 1 of the last step)
  int nonfinite;              // last step: non-finite value seen
  int converged;              // solve: tolerance met
  int init_done;              // init: residual tolerance met
  int init_iters;             // init: iterations completed
  int init_bad;               // init: Cholesky breakdown or non-finite
  int polar_steps;            // init: max Newton-Schulz steps used by the polar
  int pad0[6];
  double rel_change;          // last step monitors
  double max_defect;
  double sum_dx2;
  double sum_x2;
  double init_res;            // init: ||A Y - Y T||_F / ||T||_F of the last iteration
  double pad1[3];
  double T[kMaxD * kMaxD];    // init: Rayleigh quotient Y^T A Y (FP64)
  double Rinv[kMaxD * kMaxD]; // init: inverse Cholesky factor of (AY)^T (AY)
  double ritz[kMaxD];         // init: Ritz values, descending
};

static_assert(sizeof(DevCtl) % 256 == 0, "DevCtl must keep 256-byte alignment");

// --------------------------------------------------------------------------
// Packed upper-block-triangle storage of a symmetric A (ld == NSRGS_LD_PACKED).
// With G = 64 and ndp = n d rounded up to G, row r of block i = r / d stores
// the columns [c0(i), ndp), c0(i) = G floor(i d / G): the row's part on and
// above its diagonal block, widened to the left to a multiple of G so that
// every row starts on a 256-byte boundary (FP32; 128 bytes for 2-byte
// formats): a wave's 16-byte loads then cover whole cache lines, as in the
// full layout with ld a multiple of 64.  Rows follow one another; element
// (r, c), c >= c0(i), is at packed_row_offset(r) + c - c0(i).  Columns past
// n d are padding.
// --------------------------------------------------------------------------
constexpr int kPackedG = 64;

__host__ __device__ inline int packed_c0(int64_t i, int d) { return (int)(kPackedG * ((i * d) / kPackedG)); }

// Elements stored before block row i: d * sum_{b < i} (ndp - c0(b)).
__host__ __device__ inline int64_t packed_block_start(int64_t i, int d, int64_t ndp) {
  // sum_{b < i} floor(b d / G) = (d i (i - 1) / 2 - sum_{b < i} (b d mod G)) / G; the residues
  // b d mod G repeat with period P = G / gcd(d, G), taking every multiple of gcd(d, G) below G
  // once, so they sum to G (P - 1) / 2 over a period
  int g = kPackedG, x = d;
  while (x) {
    const int t = g % x;
    g = x;
    x = t;
  }
  const int64_t P = kPackedG / g;
  const int64_t q = i / P, rem = i % P;
  int64_t res = q * (kPackedG / 2) * (P - 1);
  for (int64_t b = 0; b < rem; ++b) res += (b * d) % kPackedG;
  const int64_t floors = (d * i * (i - 1) / 2 - res) / kPackedG;
  return (int64_t)d * (i * ndp - kPackedG * floors);
}

__host__ __device__ inline int64_t packed_row_offset(int64_t r, int d, int64_t ndp) {
  const int64_t i = r / d;
  return packed_block_start(i, d, ndp) + (r - i * d) * (ndp - packed_c0(i, d));
}

__host__ __device__ inline int64_t packed_ndp(int n, int d) {
  return ((int64_t)n * d + kPackedG - 1) / kPackedG * kPackedG;
}

__host__ __device__ inline int64_t packed_elems(int n, int d) {
  return packed_block_start(n, d, packed_ndp(n, d));
}

// Monitors of one panel of the step kernel (FP64 for every storage format).
struct PanelStat {
  double dx2, x2, dmax, nonfinite;
};

// --------------------------------------------------------------------------
// Storage formats of A.  Every format is read as 16-byte vectors: V elements
// of one row per lane per load.
// --------------------------------------------------------------------------
template <int FMT> struct Fmt;

template <> struct Fmt<NSRGS_A_F64> {
  using acc_t = double;
  static constexpr int V = 2;
  static constexpr int kBytes = 8;
};
template <> struct Fmt<NSRGS_A_F32> {
  using acc_t = float;
  static constexpr int V = 4;
  static constexpr int kBytes = 4;
};
template <> struct Fmt<NSRGS_A_BF16> {
  using acc_t = float;
  static constexpr int V = 8;
  static constexpr int kBytes = 2;
};
template <> struct Fmt<NSRGS_A_BF16_SPLIT> {
  using acc_t = float;
  static constexpr int V = 8;
  static constexpr int kBytes = 4;   // hi + lo
};
template <> struct Fmt<NSRGS_A_FP8_E4M3> {
  using acc_t = float;
  static constexpr int V = 16;
  static constexpr int kBytes = 1;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 ld16(const void *p) {
  return *reinterpret_cast<const uint4 *>(p);
}
// Streaming read of A: non-temporal, so the reused X stays in cache.
__device__ __forceinline__ uint4 ld16_stream(const void *p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Expand one 16-byte vector of A (and its low part for the split format)
// into V values of the accumulation type.
template <int FMT>
__device__ __forceinline__ void expand(uint4 raw, uint4 raw_lo,
                                       typename Fmt<FMT>::acc_t *out) {
  if constexpr (FMT == NSRGS_A_F64) {
    out[0] = __hiloint2double((int)raw.y, (int)raw.x);
    out[1] = __hiloint2double((int)raw.w, (int)raw.z);
  } else if constexpr (FMT == NSRGS_A_F32) {
    out[0] = __uint_as_float(raw.x);
    out[1] = __uint_as_float(raw.y);
    out[2] = __uint_as_float(raw.z);
    out[3] = __uint_as_float(raw.w);
  } else if constexpr (FMT == NSRGS_A_BF16) {
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      out[2 * q] = bf16_lo(w[q]);
      out[2 * q + 1] = bf16_hi(w[q]);
    }
  } else if constexpr (FMT == NSRGS_A_BF16_SPLIT) {
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
    const uint32_t l[4] = {raw_lo.x, raw_lo.y, raw_lo.z, raw_lo.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      out[2 * q] = bf16_lo(w[q]) + bf16_lo(l[q]);       // exact in FP32
      out[2 * q + 1] = bf16_hi(w[q]) + bf16_hi(l[q]);
    }
  } else {
    static_assert(FMT == NSRGS_A_FP8_E4M3, "unknown format");
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // gfx950 converts OCP e4m3 codes exactly: two codes per instruction.
      auto lo2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], false);
      auto hi2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[q], true);
      out[4 * q + 0] = lo2[0];
      out[4 * q + 1] = lo2[1];
      out[4 * q + 2] = hi2[0];
      out[4 * q + 3] = hi2[1];
    }
  }
}

// Butterfly sum over the 64 lanes of a wave; every lane receives the total.
// The order of additions is fixed, so results are reproducible.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Sum of one value per thread over the whole workgroup (blockDim.x a multiple
// of 64, at most kMaxWaves waves).  `scratch` holds kMaxWaves entries.
// Every thread receives the result.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T s = 0;
  for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T *scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T s = scratch[0];
  for (int w = 1; w < nw; ++w) s = scratch[w] > s ? scratch[w] : s;
  return s;
}

// ---- transpose-reduce over the 64 lanes of a wave ------------------------
// (M values per lane, each to be summed over the wave)
// Each of 6 steps pairs lanes that differ in one bit: one lane of the pair
// keeps the lower half of its values, the other the upper half, and each adds
// the partner's copy of what it keeps (an odd middle value is kept and summed
// by both).  After the last step every value a lane holds is the full 64-lane
// sum of one entry; wave_tr_entry gives which.  The additions are in a fixed
// order, and lanes holding the same entry hold bitwise equal sums.
constexpr int wave_tr_count(int m, int steps) {
  return steps == 0 ? m : wave_tr_count(m / 2 + (m & 1), steps - 1);
}

template <typename T, int M, int STEP>
__device__ __forceinline__ void wave_tr_step(T *v, int lane) {
  if constexpr (STEP < 6) {
    constexpr int off = 32 >> STEP;
    constexpr int h = M / 2;
    const bool hi = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const T keep = hi ? v[h + i] : v[i];
      const T send = hi ? v[i] : v[h + i];
      v[i] = keep + __shfl_xor(send, off, kWave);
    }
    if constexpr (M & 1) v[h] = v[M - 1] + __shfl_xor(v[M - 1], off, kWave);
    wave_tr_step<T, h + (M & 1), STEP + 1>(v, lane);
  }
}

// For N <= 64 each lane ends with one value; the entry it holds, found by
// walking the steps backwards from position 0 (a value at position p < h
// after a step came from p, or from h + p in the lane that kept the upper
// half; the odd middle value came from the last position).
template <int N>
__device__ __forceinline__ int wave_tr_entry(int lane) {
  static_assert(wave_tr_count(N, 6) == 1, "one value per lane after the reduction");
  int p = 0;
#pragma unroll
  for (int st = 5; st >= 0; --st) {
    const int m = wave_tr_count(N, st);
    const int h = m / 2;
    const bool hi = ((lane >> (5 - st)) & 1) != 0;
    p = p < h ? (hi ? h + p : p) : m - 1;
  }
  return p;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// 4 x 32-bit multiply-xor bijection keyed by (k0, k1), key bumped between rounds.
struct U4 {
  uint32_t x, y, z, w;
};
__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c.x;
    const uint64_t p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Standard normal from one Philox output by Box-Muller on two 53-bit uniforms:
// u1 = (m1 + 1) 2^-53 in (0, 1], u2 = m2 2^-53 in [0, 1).
__device__ inline double normal_from(U4 o) {
  const uint64_t m1 = ((uint64_t)o.x << 21) | (o.y >> 11);
  const uint64_t m2 = ((uint64_t)o.z << 21) | (o.w >> 11);
  const double u1 = ((double)m1 + 1.0) * 0x1p-53;
  const double u2 = (double)m2 * 0x1p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace nsrgs
