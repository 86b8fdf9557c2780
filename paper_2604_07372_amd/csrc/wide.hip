// Kernels of the matrix-core path (block sizes up to d = 32; NS-RGS, exact
// polar and GPM retractions; the objective of eq. def:f).  See wide.h.
#include "device.h"
#include "host.h"
#include "kernels.h"
#include "wide.h"

namespace nsrgs {

template <typename T> struct WideT;
template <> struct WideT<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static constexpr int V = 2;     // elements per 16-byte load
};
template <> struct WideT<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static constexpr int V = 4;
};

// D = A B + C on one 16 x 16 x 4 matrix-core tile.  Lane l supplies A(l % 16,
// l / 16) and B(l / 16, l % 16); it holds D(4 (l / 16) + r, l % 16), r < 4,
// for FP32 and D(l / 16 + 4 r, l % 16) for FP64 (both measured on gfx950).
template <typename T>
__device__ __forceinline__ typename WideT<T>::v4 mfma4(T a, T b, typename WideT<T>::v4 c) {
  if constexpr (sizeof(T) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// KU: 16-byte column vectors per lane per tile row per step; a step covers
// 4 KU V columns.
template <typename T, int KU>
constexpr int wide_kstep() { return 4 * KU * WideT<T>::V; }

// ---------------------------------------------------------------------------
// Product kernel: partial[ks][r][c] = sum over the columns k of chunk ks of
// A[r][k] X[k][c], for the 128 rows of this workgroup and c < 16 NT.
//
// A step covers KSTEP = 4 KU V columns.  Lane (m = l % 16, q = l / 16) of a
// wave loads KU 16-byte vectors of each of its two tile rows, at columns
// kb + (u 4 + q) V .. + V (u < KU): the four lanes of a row read 64 bytes
// contiguously per load, a wave 16 rows x 64 bytes.  Element v of vector u is
// the lane's A operand of the tile product (u, v), so column kb + (u 4 + q) V
// + v is its k index.  The B operands come from Xs, a copy of X arranged in
// exactly that order by wide_xs_kernel: for each step and 16-column tile, lane
// l's KU V values are contiguous, so a wave reads them with KU V / (16 /
// sizeof(T)) 16-byte loads per tile, 64 lanes x 64 bytes contiguous.  Each
// wave works alone (no LDS, no barrier); the next two steps' A and B vectors
// are in flight during the current step's products.  A is read with ordinary
// (cached) loads: the two loads that share each 128-byte line arrive one
// instruction apart, and a load-only probe of this pattern streamed 9%
// faster cached than non-temporal.
// ---------------------------------------------------------------------------
// MT 16-row tiles per wave (64 MT rows per workgroup) and KU = 8 / MT
// vectors per tile row per step: each B operand serves MT tiles.
template <int MT> constexpr int wide_ku() { return 8 / MT; }

template <typename T, int NT, int MT>
__global__ void __launch_bounds__(256) wide_product_kernel(WideArgs a) {
  using v4 = typename WideT<T>::v4;
  constexpr int V = WideT<T>::V;
  constexpr int KU = wide_ku<MT>();
  constexpr int ROWS = 64 * MT;
  constexpr int KSTEP = wide_kstep<T, KU>();
  constexpr int BQ = KU * V * (int)sizeof(T) / 16;   // 16-byte B loads per tile per step
  __shared__ double s_scr[kMaxWaves];
  if (a.stop_flag) {
    if (__atomic_load_n(a.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = lane & 15, q = lane >> 4;
  const int nd = a.nd;
  // Workgroup b runs on XCD b % 8 (round-robin dispatch); the logical tiles
  // are ordered column-chunk major and dealt out so that each XCD works on a
  // contiguous range of them, i.e. on few column chunks, and its L2 holds
  // only those chunks' B operands.
  const int total = a.g.row_tiles * a.g.ks;
  int lin = blockIdx.x;
  if (a.g.xcd_remap) {
    const int per = (total + 7) / 8;
    lin = (blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  if (lin >= total) return;                          // uniform: padding workgroups of the remap
  const int rt = lin % a.g.row_tiles, ks = lin / a.g.row_tiles;
  const int kbeg = ks * a.g.kchunk;
  const int kend = min(nd, kbeg + a.g.kchunk);
  const int nsteps = kend > kbeg ? (kend - kbeg + KSTEP - 1) / KSTEP : 0;
  const int step0 = kbeg / KSTEP;
  const char *__restrict__ Ab = static_cast<const char *>(a.A);
  const uint4 *__restrict__ Xs = static_cast<const uint4 *>(a.xs);
  const bool want_ssq = a.sumsq != nullptr;

  int64_t roff[MT];
  bool rowok[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = rt * ROWS + wave * 16 * MT + mt * 16 + m;
    rowok[mt] = row < nd;
    roff[mt] = (int64_t)(row < nd ? row : nd - 1) * a.ld * (int64_t)sizeof(T);
  }

  v4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = v4{0, 0, 0, 0};
  double ssq = 0.0;

  auto load = [&](int s, uint4 (&ar)[MT][KU], uint4 (&br)[NT][BQ]) {
    const int kb = kbeg + s * KSTEP;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const uint4 *bp = Xs + ((int64_t)((step0 + s) * NT + nt) * 64 + lane) * BQ;
#pragma unroll
      for (int j = 0; j < BQ; ++j) br[nt][j] = bp[j];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int kc = kb + (u * 4 + q) * V;
        const int kcc = kc < nd ? kc : 0;            // a vector starting at or past nd reads column 0
        ar[mt][u] = ld16(Ab + roff[mt] + (int64_t)kcc * (int64_t)sizeof(T));
      }
  };
  auto compute = [&](int s, const uint4 (&ar)[MT][KU], const uint4 (&br)[NT][BQ]) {
    const int kb = kbeg + s * KSTEP;
    const bool ragged = kb + KSTEP > nd;             // uniform: only the matrix's last step
    T bv[NT][KU * V];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int j = 0; j < BQ; ++j) {
        if constexpr (sizeof(T) == 8) {
          bv[nt][2 * j] = __hiloint2double((int)br[nt][j].y, (int)br[nt][j].x);
          bv[nt][2 * j + 1] = __hiloint2double((int)br[nt][j].w, (int)br[nt][j].z);
        } else {
          bv[nt][4 * j] = __uint_as_float(br[nt][j].x);
          bv[nt][4 * j + 1] = __uint_as_float(br[nt][j].y);
          bv[nt][4 * j + 2] = __uint_as_float(br[nt][j].z);
          bv[nt][4 * j + 3] = __uint_as_float(br[nt][j].w);
        }
      }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      T av[MT][V];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if constexpr (sizeof(T) == 8) {
          av[mt][0] = __hiloint2double((int)ar[mt][u].y, (int)ar[mt][u].x);
          av[mt][1] = __hiloint2double((int)ar[mt][u].w, (int)ar[mt][u].z);
        } else {
          av[mt][0] = __uint_as_float(ar[mt][u].x);
          av[mt][1] = __uint_as_float(ar[mt][u].y);
          av[mt][2] = __uint_as_float(ar[mt][u].z);
          av[mt][3] = __uint_as_float(ar[mt][u].w);
        }
      }
      if (ragged) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < V; ++v) av[mt][v] = (kb + (u * 4 + q) * V + v < nd) ? av[mt][v] : T(0);
      }
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma4<T>(av[mt][v], bv[nt][u * V + v], acc[mt][nt]);
      if (want_ssq) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const double x = rowok[mt] ? (double)av[mt][v] : 0.0;
            ssq += x * x;
          }
      }
    }
  };

  // Register sets in a ring, unrolled so that they take turns without
  // copies: the loads of the next two (one 16-column tile, three sets) or
  // three (two tiles, four sets) steps are issued before a step's products.
  // (One wave per SIMD: the products of one step, about 2000 cycles, do not
  // cover the memory latency.  Two sets measured 10% slower than three; at
  // n = 500, d = 25 four sets took the product from 266 to 260 us (FP64) and
  // 134 to 131 us (FP32), while at d <= 16 they were 1% slower than three.
  // A branch-free variant of this loop, whose waits the compiler counts
  // exactly, measured slower still.)
  if constexpr (NT == 1) {
    uint4 ar0[MT][KU], ar1[MT][KU], ar2[MT][KU], br0[NT][BQ], br1[NT][BQ], br2[NT][BQ];
    if (nsteps > 0) load(0, ar0, br0);
    if (nsteps > 1) load(1, ar1, br1);
    for (int s = 0; s < nsteps; s += 3) {
      if (s + 2 < nsteps) load(s + 2, ar2, br2);
      __builtin_amdgcn_sched_barrier(0);
      compute(s, ar0, br0);
      if (s + 1 < nsteps) {
        if (s + 3 < nsteps) load(s + 3, ar0, br0);
        __builtin_amdgcn_sched_barrier(0);
        compute(s + 1, ar1, br1);
      }
      if (s + 2 < nsteps) {
        if (s + 4 < nsteps) load(s + 4, ar1, br1);
        __builtin_amdgcn_sched_barrier(0);
        compute(s + 2, ar2, br2);
      }
    }
  } else {
    uint4 ar0[MT][KU], ar1[MT][KU], ar2[MT][KU], ar3[MT][KU];
    uint4 br0[NT][BQ], br1[NT][BQ], br2[NT][BQ], br3[NT][BQ];
    if (nsteps > 0) load(0, ar0, br0);
    if (nsteps > 1) load(1, ar1, br1);
    if (nsteps > 2) load(2, ar2, br2);
    for (int s = 0; s < nsteps; s += 4) {
      if (s + 3 < nsteps) load(s + 3, ar3, br3);
      __builtin_amdgcn_sched_barrier(0);
      compute(s, ar0, br0);
      if (s + 1 < nsteps) {
        if (s + 4 < nsteps) load(s + 4, ar0, br0);
        __builtin_amdgcn_sched_barrier(0);
        compute(s + 1, ar1, br1);
      }
      if (s + 2 < nsteps) {
        if (s + 5 < nsteps) load(s + 5, ar1, br1);
        __builtin_amdgcn_sched_barrier(0);
        compute(s + 2, ar2, br2);
      }
      if (s + 3 < nsteps) {
        if (s + 6 < nsteps) load(s + 6, ar2, br2);
        __builtin_amdgcn_sched_barrier(0);
        compute(s + 3, ar3, br3);
      }
    }
  }

  T *__restrict__ P = static_cast<T *>(a.part) + (size_t)ks * a.g.rows_pad * 32;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * ROWS + wave * 16 * MT + mt * 16 + (sizeof(T) == 8 ? q + 4 * r : 4 * q + r);
        P[(size_t)row * 32 + nt * 16 + m] = acc[mt][nt][r];
      }
  if (want_ssq) {
    ssq = block_sum(ssq, s_scr);
    if (tid == 0) a.sumsq[(size_t)ks * a.g.row_tiles + rt] = ssq;
  }
}

// Xs: X in the product kernel's B-operand order.  Element (step, nt, l, j),
// j = u V + v, at ((step NT + nt) 64 + l) KU V + j holds X[k][c] with
// k = step KSTEP + (u 4 + l / 16) V + v and c = 16 nt + l % 16 (zero past nd
// or d).  One thread per element.
template <typename T, int NT, int MT>
__global__ void __launch_bounds__(256) wide_xs_kernel(const T *__restrict__ X, int nd, int d, int steps,
                                                      T *__restrict__ Xs, const int *stop_flag) {
  constexpr int V = WideT<T>::V;
  constexpr int KU = wide_ku<MT>();
  constexpr int KSTEP = wide_kstep<T, KU>();
  constexpr int PER = KU * V;
  if (stop_flag) {
    if (__atomic_load_n(stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)steps * NT * 64 * PER;
  if (e >= total) return;
  const int j = (int)(e % PER);
  const int l = (int)((e / PER) % 64);
  const int nt = (int)((e / (PER * 64)) % NT);
  const int step = (int)(e / ((int64_t)PER * 64 * NT));
  const int u = j / V, v = j % V;
  const int k = step * KSTEP + (u * 4 + l / 16) * V + v;
  const int c = 16 * nt + l % 16;
  const int kk = k < nd ? k : nd - 1, cc = c < d ? c : d - 1;
  const T x = X[(int64_t)kk * d + cc];
  Xs[e] = (k < nd && c < d) ? x : T(0);
}

// ---------------------------------------------------------------------------
// d x d helpers in FP64 on LDS, for every thread of a workgroup.
// ---------------------------------------------------------------------------
// out = op(A) op(B) for d x d FP64 matrices in LDS (row-major, stride d),
// op = transpose where TA / TB.  Blocks larger than 16 with at least four
// waves use the matrix cores: wave w < 4 owns the 16 x 16 output tile
// (w / 2, w % 2) and runs ceil(d / 4) FP64 16 x 16 x 4 steps, entries past d
// read as zero.  (Each entry's d products summed one by one took one LDS read
// of each operand per product, which bounds the per-block epilogue at
// d = 25.)  Otherwise each thread sums whole entries.  Ends with a barrier.
template <bool TA, bool TB>
__device__ __forceinline__ void wmm(double *out, const double *A, const double *B, int d) {
  static_assert(kWideMaxD <= 32, "2 x 2 output tiles and eight 4-wide steps cover d <= 32");
  const int dd = d * d;
  if (d > 16 && blockDim.x >= 4 * kWave) {   // uniform
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (w < 4) {
      const int r0 = (w >> 1) * 16, c0 = (w & 1) * 16;
      const int i = r0 + (lane & 15), c = c0 + (lane & 15), kq = lane >> 4;
      // every operand read is issued before the first product (clamped
      // in-bounds addresses, zero selected past d), so the eight steps wait
      // for LDS once
      const int ic = i < d ? i : 0, cc = c < d ? c : 0;
      double av[8], bv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = 4 * t + kq, kc = k < d ? k : 0;
        const double x = TA ? A[kc * d + ic] : A[ic * d + kc];
        const double y = TB ? B[cc * d + kc] : B[kc * d + cc];
        av[t] = (k < d && i < d) ? x : 0.0;
        bv[t] = (k < d && c < d) ? y : 0.0;
      }
      WideT<double>::v4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (4 * t < d) acc = mfma4<double>(av[t], bv[t], acc);   // uniform
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + kq + 4 * r;
        if (row < d && c < d) out[row * d + c] = acc[r];
      }
    }
    __syncthreads();
    return;
  }
  for (int e = threadIdx.x; e < dd; e += blockDim.x) {
    const int r = e / d, k = e % d;
    double s0 = 0.0, s1 = 0.0;
    int m = 0;
    for (; m + 1 < d; m += 2) {
      s0 += (TA ? A[m * d + r] : A[r * d + m]) * (TB ? B[k * d + m] : B[m * d + k]);
      s1 += (TA ? A[(m + 1) * d + r] : A[r * d + m + 1]) * (TB ? B[k * d + m + 1] : B[(m + 1) * d + k]);
    }
    if (m < d) s0 += (TA ? A[m * d + r] : A[r * d + m]) * (TB ? B[k * d + m] : B[m * d + k]);
    out[e] = s0 + s1;
  }
  __syncthreads();
}

// Sums of N values per thread over the workgroup in one pass (two barriers);
// every thread receives the N totals.  scr holds N * kMaxWaves doubles.
template <int N>
__device__ inline void block_sum_n(double (&v)[N], double *scr) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) scr[j * kMaxWaves + wave] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scr[j * kMaxWaves + w];
    v[j] = t;
  }
}

// ||I - M||_F of a d x d matrix in LDS (a block reduction).
__device__ inline double wdefect(const double *M, int d, double *scr) {
  double s = 0.0;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const double v = ((e / d) == (e % d) ? 1.0 : 0.0) - M[e];
    s += v * v;
  }
  return sqrt(block_sum(s, scr));
}

// The polar factor sgn(S) = U V^T of a nonsingular d x d matrix S = U Sigma V^T
// (Sec. 2.1), in place, to FP64 accuracy: Newton-Schulz from S scaled by
// 1 / sqrt(g), g the largest Gershgorin row sum of S^T S (an upper bound of
// sigma_max^2, so every scaled singular value lies in (0, 1], inside the
// region (0, sqrt 3) where the iteration converges to sgn), until
// ||I - S^T S||_F <= 64 d eps, then two more (quadratic) steps.  M, N are LDS
// scratch.  Returns the number of steps, or -1 if the matrix is singular or
// not finite (no convergence within 200 steps).
__device__ __forceinline__ int wide_polar(double *S, double *M, double *N, int d, double *scr) {
  const int dd = d * d;
  wmm<true, false>(M, S, S, d);
  double g = 0.0;
  for (int r = threadIdx.x; r < d; r += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += fabs(M[r * d + k]);
    g = s > g ? s : g;
  }
  g = block_max(g, scr);
  if (!(g > 0.0) || !isfinite(g)) return -1;
  const double sc = 1.0 / sqrt(g);
  for (int e = threadIdx.x; e < dd; e += blockDim.x) S[e] *= sc;
  __syncthreads();
  const double stop = 64.0 * d * 2.220446049250313e-16;
  int extra = -1;
  for (int it = 0; it < 200; ++it) {
    wmm<true, false>(M, S, S, d);
    const double def = wdefect(M, d, scr);
    if (!isfinite(def)) return -1;
    if (extra < 0 && def <= stop) extra = 2;
    if (extra == 0) return it;
    wmm<false, false>(N, S, M, d);
    for (int e = threadIdx.x; e < dd; e += blockDim.x) S[e] = 1.5 * S[e] - 0.5 * N[e];
    __syncthreads();
    if (extra > 0) --extra;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Epilogue: one workgroup per block i.  Step mode: C_i from the partials, the
// diagonal-block term, the retraction, X_i^{t+1} and the block's record.
// Init mode: W_i = (A Y)_i and the block's Grams Y_i^T W_i, W_i^T W_i.
// The d x d arithmetic is FP64 for every storage format.
// Dynamic LDS: seven d x d arrays, wide_epi_lds(d) bytes, and as many waves
// as d^2 entries need (up to four), so that small blocks do not hold a CU's
// LDS with a fixed 32 x 32 layout and idle threads.
// ---------------------------------------------------------------------------
__host__ __device__ inline int wide_epi_stride(int d) { return (d * d + 1) & ~1; }
inline size_t wide_epi_lds(int d) { return (size_t)7 * wide_epi_stride(d) * sizeof(double); }
inline int wide_epi_threads(int d) { return min(256, (d * d + kWave - 1) / kWave * kWave); }

template <typename T>
__global__ void __launch_bounds__(256) wide_epilogue_kernel(WideArgs a) {
  extern __shared__ double sm_dyn[];
  __shared__ double s_scr[kMaxWaves];
  __shared__ double s_scr7[7 * kMaxWaves];
  if (a.stop_flag) {
    if (__atomic_load_n(a.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int i = blockIdx.x, d = a.d, dd = d * d, tid = threadIdx.x;
  const int es = wide_epi_stride(d);
  double *X = sm_dyn, *C = X + es, *Ad = C + es, *G = Ad + es, *Tm = G + es, *F = Tm + es, *M = F + es;
  const T *__restrict__ Xin = static_cast<const T *>(a.X_in);
  const T *__restrict__ P = static_cast<const T *>(a.part);
  const T *__restrict__ A = static_cast<const T *>(a.A);
  for (int e = tid; e < dd; e += blockDim.x) {
    const int r = e / d, k = e % d;
    const int64_t row = (int64_t)i * d + r;
    X[e] = (double)Xin[row * d + k];
    double c = 0.0;
#pragma unroll 4
    for (int s = 0; s < a.g.ks; ++s) c += (double)P[((size_t)s * a.g.rows_pad + row) * 32 + k];
    C[e] = c;
    Ad[e] = a.no_diag ? 0.0 : (double)A[row * a.ld + (int64_t)i * d + k];
  }
  __syncthreads();

  if (a.mode == WIDE_INIT) {
    T *__restrict__ W = static_cast<T *>(a.X_out);
    for (int e = tid; e < dd; e += blockDim.x) W[((int64_t)i * d + e / d) * d + e % d] = (T)C[e];
    wmm<true, false>(G, X, C, d);       // Y_i^T W_i
    wmm<true, false>(Tm, C, C, d);      // W_i^T W_i
    double *out = a.igram + (size_t)i * 2 * dd;
    for (int e = tid; e < dd; e += blockDim.x) {
      out[e] = G[e];
      out[dd + e] = Tm[e];
    }
    return;
  }

  // Per-thread partial sums, reduced once at the end: ||X_i||^2 and the
  // objective pieces tr(X_i^T C_i) (C_i without the diagonal block),
  // ||X_i^T X_i||^2 and ||A_ii||^2 (the latter three only when F is evaluated).
  double red[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // x2 xc hh aii2 dx2 nonfin def2
  const bool need_diag = a.method != WIDE_GPM || a.objective;
  if (need_diag) wmm<false, false>(G, Ad, X, d);          // A_ii X_i
  if (a.objective) wmm<true, false>(Tm, X, X, d);         // X_i^T X_i
  for (int e = tid; e < dd; e += blockDim.x) {
    red[0] += X[e] * X[e];
    if (a.objective) {
      red[1] += X[e] * (C[e] - G[e]);
      red[2] += Tm[e] * Tm[e];
      red[3] += Ad[e] * Ad[e];
    }
  }

  double *S = F;         // the iterate being retracted
  int polar_steps = 0;
  if (a.method == WIDE_GPM) {
    for (int e = tid; e < dd; e += blockDim.x) S[e] = C[e];        // (A X)_i, diagonal block included
    __syncthreads();
    polar_steps = wide_polar(S, M, Tm, d, s_scr);
    wmm<true, false>(M, S, S, d);
  } else {
    const double nm1 = (double)(a.n - 1), mu = a.mu;
    for (int e = tid; e < dd; e += blockDim.x) G[e] = nm1 * X[e] - (C[e] - G[e]);   // G_i
    __syncthreads();
    wmm<true, false>(Tm, G, X, d);       // G_i^T X_i
    wmm<false, false>(M, X, Tm, d);      // X_i G_i^T X_i
    for (int e = tid; e < dd; e += blockDim.x) F[e] = X[e] - mu * 0.5 * (G[e] - M[e]);
    __syncthreads();
    wmm<true, false>(M, F, F, d);        // F_i^T F_i (also the first Newton-Schulz M)
  }
  // ||I - F_i^T F_i|| (for GPM: of the new iterate), summed with the rest
  for (int e = tid; e < dd; e += blockDim.x) {
    const double v = ((e / d) == (e % d) ? 1.0 : 0.0) - M[e];
    red[6] += v * v;
  }
  if (a.method == WIDE_POLAR) {
    __syncthreads();                     // M is rewritten by the polar iteration
    polar_steps = wide_polar(S, M, Tm, d, s_scr);
  } else if (a.method == WIDE_NS) {
    double *cur = F, *nxt = G;
    for (int st = 0; st < a.ns_steps; ++st) {
      if (st > 0) wmm<true, false>(M, cur, cur, d);
      wmm<false, false>(Tm, cur, M, d);
      for (int e = tid; e < dd; e += blockDim.x) nxt[e] = 1.5 * cur[e] - 0.5 * Tm[e];
      __syncthreads();
      double *t = cur;
      cur = nxt;
      nxt = t;
    }
    S = cur;
  }
  T *__restrict__ Xo = static_cast<T *>(a.X_out);
  // With xs_write the block's entries of X^{t+1} also go to their places in
  // the product's operand copy (the layout of wide_xs_kernel: entry (k, c) at
  // ((step NT + c / 16) 64 + l) KU V + j, step = k / KSTEP and, with
  // r = k mod KSTEP, l = 16 ((r / V) mod 4) + c mod 16, j = V (r / V / 4) + r mod V),
  // so the next step's product needs no staging launch.  Its zero padding
  // (columns past d, rows past n d) stays as the staging kernel wrote it.
  T *__restrict__ Xs = a.xs_write ? static_cast<T *>(a.xs) : nullptr;
  constexpr int V = WideT<T>::V;
  const int xs_per = a.g.ku * V, xs_nt = a.g.nt, xs_kstep = a.g.kstep;
  for (int e = tid; e < dd; e += blockDim.x) {
    const T v = (T)S[e];
    const int64_t k = (int64_t)i * d + e / d;
    const int c = e % d;
    Xo[k * d + c] = v;
    if (Xs) {
      const int step = (int)(k / xs_kstep), r = (int)(k % xs_kstep), g4 = r / V;
      const int l = (g4 % 4) * 16 + c % 16, j = (g4 / 4) * V + r % V;
      Xs[(((int64_t)step * xs_nt + c / 16) * 64 + l) * xs_per + j] = v;
    }
    const double dv = (double)v - X[e];
    red[4] += dv * dv;
    red[5] += isfinite(v) ? 0.0 : 1.0;
  }
  block_sum_n<7>(red, s_scr7);
  if (tid == 0) {
    const double dmax = sqrt(red[6]);
    a.stats[i] = WideStat{red[4], red[0], dmax, (red[5] != 0.0 || !isfinite(dmax)) ? 1.0 : 0.0, red[1], red[2],
                          red[3], polar_steps < 0 ? 1.0 : 0.0};
  }
}

// Partial X^T X over a slice of rows: workgroup g sums rows
// [g rpg, (g + 1) rpg) into gram[g] (FP64), d^2 entries.
template <typename T>
__global__ void __launch_bounds__(256) wide_gram_kernel(const T *__restrict__ X, int nd, int d,
                                                        double *gram, const int *stop_flag) {
  __shared__ double xs[32][kWideMaxD + 1];
  if (stop_flag) {
    if (__atomic_load_n(stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int g = blockIdx.x, tid = threadIdx.x, dd = d * d;
  const int rpg = (nd + gridDim.x - 1) / gridDim.x;
  const int r0 = g * rpg, r1 = min(nd, r0 + rpg);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int ea[4], eb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = tid + 256 * j;
    const int ee = e < dd ? e : 0;
    ea[j] = ee / d;
    eb[j] = ee % d;
  }
  for (int rb = r0; rb < r1; rb += 32) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      const int rr = e / kWideMaxD, c = e % kWideMaxD;
      const int row = rb + rr;
      const int rowc = row < nd ? row : nd - 1, cc = c < d ? c : d - 1;
      const double v = (double)X[(int64_t)rowc * d + cc];
      xs[rr][c] = (row < r1 && c < d) ? v : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int rr = 0; rr < 32; ++rr) acc[j] += xs[rr][ea[j]] * xs[rr][eb[j]];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int e = tid + 256 * j;
    if (e < dd) gram[(size_t)g * dd + e] = acc[j];
  }
}

// One workgroup after each step: FP64 reduction of the block records in a
// fixed order, the objective F(X^t) (eq. def:f) from its per-block pieces
//   F = (1/2)(||sum_i X_i^T X_i||^2 - sum_i ||X_i^T X_i||^2)
//       - sum_i tr(X_i^T C_i) + (1/2) sum_{i != j} ||A_ij||^2,
// and the stop rules: relative change ||X^{t+1} - X^t|| / ||X^t|| <= tol, or
// the paper's ratio R^{t-1} = (F(X^{t-1}) - F(X^t)) / F(X^t) < tol, which
// stops with X^t (this step's input) as the result.
// One workgroup of kWideFinishThreads (at most kMaxWaves waves: the
// reductions' scratch); the record loop is unrolled so that several records
// per thread are in flight (n records at 20000 blocks took 34 us one by one).
constexpr int kWideFinishThreads = kWave * kMaxWaves;
__global__ void __launch_bounds__(kWideFinishThreads) wide_finish_kernel(WideArgs a) {
  __shared__ double s_scr[kMaxWaves];
  __shared__ double s_scr7[7 * kMaxWaves];
  if (a.stop_flag) {
    if (__atomic_load_n(a.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int tid = threadIdx.x, d = a.d, dd = d * d;
  // sums in a fixed order; the non-finite and polar-failure flags are 0 / 1
  // per block, so their sums are counts
  double v[7] = {0, 0, 0, 0, 0, 0, 0}, dmax = 0;
#pragma unroll 4
  for (int p = tid; p < a.n; p += blockDim.x) {
    const WideStat s = a.stats[p];
    v[0] += s.dx2;
    v[1] += s.x2;
    v[2] += s.xc;
    v[3] += s.hh;
    v[4] += s.aii2;
    v[5] += s.nonfinite;
    v[6] += s.polar_bad;
    dmax = s.dmax > dmax ? s.dmax : dmax;
  }
  block_sum_n<7>(v, s_scr7);
  dmax = block_max(dmax, s_scr);
  const double dx2 = v[0], x2 = v[1], xc = v[2], hh = v[3], aii2 = v[4], nf = v[5], pb = v[6];
  double Fx = 0.0;
  if (a.objective) {
    double ss = 0.0;
    for (int e = tid; e < dd; e += blockDim.x) {
      double s = 0.0;
      for (int g = 0; g < kWideGramGroups; ++g) s += a.gram[(size_t)g * dd + e];
      ss += s * s;
    }
    ss = block_sum(ss, s_scr);
    double tot = 0.0;
    if (a.sumsq) {
      const int np = a.g.row_tiles * a.g.ks;
      for (int p = tid; p < np; p += blockDim.x) tot += a.sumsq[p];
      tot = block_sum(tot, s_scr);
    }
    if (tid == 0) {
      WideCtl *w = a.wctl;
      if (a.sumsq) {
        w->obj_const = 0.5 * (tot - aii2);
        w->have_const = 1;
      }
      Fx = 0.5 * (ss - hh) - xc + w->obj_const;
    }
  }
  if (tid == 0) {
    DevCtl *ctl = a.ctl;
    const double rel = x2 > 0.0 ? sqrt(dx2 / x2) : 0.0;
    ctl->sum_dx2 = dx2;
    ctl->sum_x2 = x2;
    ctl->rel_change = rel;
    ctl->max_defect = dmax;
    ctl->nonfinite = (nf != 0.0 || pb != 0.0) ? 1 : 0;
    ctl->iters = a.iter + 1;
    if (ctl->nonfinite || !isfinite(rel)) {
      ctl->nonfinite = 1;
      ctl->done = 1;
    } else if (a.stop_rule == 0 && a.tol > 0.0 && rel <= a.tol) {
      ctl->converged = 1;
      ctl->done = 1;
    }
    if (a.objective) {
      WideCtl *w = a.wctl;
      double R = NAN;
      if (a.iter >= 1) R = (w->obj - Fx) / Fx;
      w->obj_prev = w->obj;
      w->obj = Fx;
      w->obj_ratio = R;
      if (!ctl->done && a.stop_rule == 1 && a.tol > 0.0 && a.iter >= 1 && R < a.tol) {
        ctl->converged = 1;
        ctl->done = 1;
        ctl->iters = a.iter;         // X^t, this step's input, is the result
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Spectral initialization for d up to 32 (the same subspace iteration as the
// narrow path: W = A Y, Cholesky-QR of W in FP64, Rayleigh-Ritz values).
// ---------------------------------------------------------------------------
// Sum of the n per-block Grams (2 d^2 entries each) in FP64: workgroup g
// owns entries [64 g, 64 g + 64) (lane = entry, so every load is 512
// contiguous bytes); its four waves take every fourth block, then add their
// partial sums in wave order.
__global__ void __launch_bounds__(256) wide_igram_reduce_kernel(const double *igram, int n, int d,
                                                                double *sum, const DevCtl *ctl) {
  __shared__ double part[4][64];
  if (__atomic_load_n(&ctl->init_done, __ATOMIC_RELAXED)) return;   // uniform
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, ne = 2 * d * d;
  const int e = blockIdx.x * 64 + lane;
  const int ec = e < ne ? e : ne - 1;
  double s0 = 0.0, s1 = 0.0;
  int i = wave;
  for (; i + 4 < n; i += 8) {
    s0 += igram[(size_t)i * ne + ec];
    s1 += igram[(size_t)(i + 4) * ne + ec];
  }
  if (i < n) s0 += igram[(size_t)i * ne + ec];
  part[wave][lane] = s0 + s1;
  __syncthreads();
  if (wave == 0 && e < ne) sum[e] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// Rayleigh quotient T = sym(Y^T W) and the inverse Cholesky factor of W^T W
// (FP64) from the reduced Grams.
__global__ void __launch_bounds__(64) wide_gram_finish_kernel(const double *gsum, int d, DevCtl *ctl, WideCtl *w) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double G1[NE], G2[NE], Rm[NE];
  if (__atomic_load_n(&ctl->init_done, __ATOMIC_RELAXED)) return;   // uniform
  const int dd = d * d, tid = threadIdx.x;
  for (int e = tid; e < 2 * dd; e += blockDim.x) {
    const double s = gsum[e];
    if (e < dd) G1[e] = s; else G2[e - dd] = s;
  }
  __syncthreads();
  for (int e = tid; e < dd; e += blockDim.x) {
    const int r = e / d, k = e % d;
    w->T[e] = 0.5 * (G1[r * d + k] + G1[k * d + r]);
    Rm[e] = 0.0;
  }
  __syncthreads();
  // Cholesky W^T W = R^T R, one row of R per step: the pivot by one lane,
  // the rest of the row by lane k (one wave, so the barriers are cheap)
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  for (int j = 0; j < d; ++j) {
    if (tid == 0) {
      double s = G2[j * d + j];
      for (int q = 0; q < j; ++q) s -= Rm[q * d + j] * Rm[q * d + j];
      if (!(s > 0.0) || !isfinite(s)) { s_bad = 1; s = 1.0; }
      Rm[j * d + j] = sqrt(s);
    }
    __syncthreads();
    const int k = tid;
    if (k > j && k < d) {
      double t = G2[j * d + k];
      for (int q = 0; q < j; ++q) t -= Rm[q * d + j] * Rm[q * d + k];
      Rm[j * d + k] = t / Rm[j * d + j];
    }
    __syncthreads();
  }
  // R^{-1}: lane k solves column k by back substitution (in G1, free now)
  double *Ri = G1;
  for (int e = tid; e < dd; e += blockDim.x) Ri[e] = 0.0;
  __syncthreads();
  if (tid < d) {
    const int k = tid;
    Ri[k * d + k] = 1.0 / Rm[k * d + k];
    for (int r = k - 1; r >= 0; --r) {
      double s = 0.0;
      for (int q = r + 1; q <= k; ++q) s += Rm[r * d + q] * Ri[q * d + k];
      Ri[r * d + k] = -s / Rm[r * d + r];
    }
  }
  if (tid == 0 && s_bad) ctl->init_bad = 1;
  __syncthreads();
  for (int e = tid; e < dd; e += blockDim.x) w->Rinv[e] = G1[e];
}

// One thread per entry (row, k): Y_next = W R^{-1}, residual W - Y T.
template <typename T>
__global__ void __launch_bounds__(256) wide_init_apply_kernel(const T *W, const T *Y, T *Yn, int nd, int d,
                                                              double *part, int num_groups, DevCtl *ctl,
                                                              WideCtl *w, int iter, double tol) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double sR[NE], sT[NE];
  __shared__ double s_scr[kMaxWaves];
  if (__atomic_load_n(&ctl->init_done, __ATOMIC_RELAXED)) return;   // uniform
  const int tid = threadIdx.x, dd = d * d;
  for (int e = tid; e < dd; e += blockDim.x) {
    sR[e] = w->Rinv[e];
    sT[e] = w->T[e];
  }
  __syncthreads();
  const int64_t ent = (int64_t)blockIdx.x * blockDim.x + tid;
  const bool ok = ent < (int64_t)nd * d;
  const int64_t entc = ok ? ent : 0;
  const int64_t row = entc / d;
  const int k = (int)(entc % d);
  double s = 0.0, t = 0.0;
  for (int m = 0; m < d; ++m) {
    s += (double)W[row * d + m] * sR[m * d + k];
    t += (double)Y[row * d + m] * sT[m * d + k];
  }
  if (ok) Yn[ent] = (T)s;
  const double r = (double)W[entc] - t;
  double res2 = ok ? r * r : 0.0;
  const int bad = ok && !isfinite(s);
  res2 = block_sum(res2, s_scr);
  const double fbad = block_max((double)bad, s_scr);
  if (tid == 0) {
    part[2 * blockIdx.x] = res2;
    part[2 * blockIdx.x + 1] = fbad;
  }
}

// After the apply kernel (one workgroup; the kernel boundary orders the
// partials): the relative residual ||W - Y T||_F / ||T||_F and the stop test.
__global__ void __launch_bounds__(256) wide_init_check_kernel(const double *part, int num_groups, int d,
                                                              DevCtl *ctl, const WideCtl *w, int iter, double tol) {
  __shared__ double s_scr[kMaxWaves];
  if (__atomic_load_n(&ctl->init_done, __ATOMIC_RELAXED)) return;   // uniform
  const int tid = threadIdx.x, dd = d * d;
  {
    double sum = 0.0, b = 0.0;
    for (int g = tid; g < num_groups; g += blockDim.x) {
      sum += part[2 * g];
      b = part[2 * g + 1] > b ? part[2 * g + 1] : b;
    }
    double tn = 0.0;
    for (int e = tid; e < dd; e += blockDim.x) tn += w->T[e] * w->T[e];
    sum = block_sum(sum, s_scr);
    b = block_max(b, s_scr);
    tn = block_sum(tn, s_scr);
    if (tid == 0) {
      const double rel = tn > 0.0 ? sqrt(sum / tn) : 0.0;
      ctl->init_res = rel;
      ctl->init_iters = iter + 1;
      if (b != 0.0 || !isfinite(rel)) ctl->init_bad = 1;
      if (iter >= 1 && rel <= tol) ctl->init_done = 1;   // the first basis is random
      if (ctl->init_bad) ctl->init_done = 1;
    }
  }
}

// One workgroup per block: X0_i = sgn(Y_i) in FP64.
template <typename T>
__global__ void __launch_bounds__(256) wide_init_polar_kernel(const T *Y, T *X0, int n, int d, DevCtl *ctl) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double sS[NE], sM[NE], sN[NE];
  __shared__ double s_scr[kMaxWaves];
  const int b = blockIdx.x, dd = d * d;
  for (int e = threadIdx.x; e < dd; e += blockDim.x) sS[e] = (double)Y[(int64_t)b * dd + e];
  __syncthreads();
  const int steps = wide_polar(sS, sM, sN, d, s_scr);
  for (int e = threadIdx.x; e < dd; e += blockDim.x) X0[(int64_t)b * dd + e] = (T)sS[e];
  if (threadIdx.x == 0) {
    atomicMax(&ctl->polar_steps, steps);
    if (steps < 0) atomicOr(&ctl->init_bad, 1);
  }
}

// Ritz values: eigenvalues of T (FP64 cyclic Jacobi), descending.  One wave:
// every lane computes the same rotation, lane k updates entry k of the two
// rows, then of the two columns.
__global__ void __launch_bounds__(64) wide_init_finish_kernel(DevCtl *ctl, WideCtl *w, int d) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double M[NE];
  __shared__ double s_scr[kMaxWaves];
  const int k = threadIdx.x;
  for (int e = k; e < d * d; e += blockDim.x) M[e] = w->T[e];
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = k; e < d * d; e += blockDim.x) {
      const double v = M[e] * M[e];
      tot += v;
      if (e / d != e % d) off += v;
    }
    off = block_sum(off, s_scr);
    tot = block_sum(tot, s_scr);
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < d - 1; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = M[p * d + q];
        if (apq == 0.0) continue;                       // uniform: every lane reads the same value
        const double theta = (M[q * d + q] - M[p * d + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        __syncthreads();
        if (k < d) {                                    // rotate rows p, q
          const double mp = M[p * d + k], mq = M[q * d + k];
          M[p * d + k] = c * mp - sn * mq;
          M[q * d + k] = sn * mp + c * mq;
        }
        __syncthreads();
        if (k < d) {                                    // rotate columns p, q
          const double mp = M[k * d + p], mq = M[k * d + q];
          M[k * d + p] = c * mp - sn * mq;
          M[k * d + q] = sn * mp + c * mq;
        }
        __syncthreads();
      }
  }
  if (k == 0) {
    double wv[kWideMaxD];
    for (int i = 0; i < d; ++i) wv[i] = M[i * d + i];
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j)
        if (wv[j] > wv[i]) {
          const double t = wv[i];
          wv[i] = wv[j];
          wv[j] = t;
        }
    for (int i = 0; i < d; ++i) w->ritz[i] = wv[i];
    for (int i = 0; i < d && i < kMaxD; ++i) ctl->ritz[i] = wv[i];
  }
}

__global__ void wide_ctl_reset_kernel(WideCtl *w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  w->obj_const = 0.0;
  w->obj_prev = NAN;
  w->obj = NAN;
  w->obj_ratio = NAN;
  w->have_const = 0;
}


// ---------------------------------------------------------------------------
// NS-RGS on the Stiefel manifold St(p, d) = {S in R^{d x p} : S S^T = I_d},
// the extension of the method the paper names as future work (Sec. 6), for
// d <= p <= 32: every step of Algorithm 2 written for d x p blocks,
//   G_i = (n - 1) S_i - sum_{j != i} A_ij S_j
//   P_i = G_i - sym(G_i S_i^T) S_i          (projection onto T_S St)
//   F_i = S_i - mu P_i,   S_i <- Ts steps of S <- (3 S - S S^T S) / 2.
// At p = d and S_i in O(d) the projection is Algorithm 2's.
// ---------------------------------------------------------------------------
// out (r x c) = op(A) op(B) over an inner dimension m, row-major in LDS:
// A is r x m (m x r when TA), B is m x c (c x m when TB).  Ends with a barrier.
template <bool TA, bool TB>
__device__ inline void wmm_rect(double *out, const double *A, const double *B, int r, int m, int c) {
  for (int e = threadIdx.x; e < r * c; e += blockDim.x) {
    const int i = e / c, k = e % c;
    double s0 = 0.0, s1 = 0.0;
    int j = 0;
    for (; j + 1 < m; j += 2) {
      s0 += (TA ? A[j * r + i] : A[i * m + j]) * (TB ? B[k * m + j] : B[j * c + k]);
      s1 += (TA ? A[(j + 1) * r + i] : A[i * m + j + 1]) * (TB ? B[k * m + j + 1] : B[(j + 1) * c + k]);
    }
    if (j < m) s0 += (TA ? A[j * r + i] : A[i * m + j]) * (TB ? B[k * m + j] : B[j * c + k]);
    out[e] = s0 + s1;
  }
  __syncthreads();
}

// One workgroup per block i: C_i from the partials (diagonal block included,
// as the product streams whole rows), the Stiefel step in FP64, S_i^{t+1} and
// the block's monitors (||S^{t+1} - S^t||^2, ||S^t||^2, ||I - F_i F_i^T||_F).
// Dynamic LDS: seven d x p arrays (every d x d and d x p intermediate fits, as
// p >= d), wide_stiefel_epi_lds(d, p) bytes; launched with one wave when
// d p <= 64, so that small blocks do not hold a CU's LDS and threads idle.
__host__ __device__ inline int wide_stiefel_epi_stride(int d, int p) { return (d * p + 1) & ~1; }
inline size_t wide_stiefel_epi_lds(int d, int p) { return (size_t)7 * wide_stiefel_epi_stride(d, p) * sizeof(double); }
inline int wide_stiefel_epi_threads(int d, int p) { return d * p <= kWave ? kWave : 256; }

template <typename T>
__global__ void __launch_bounds__(256) wide_stiefel_epilogue_kernel(WideArgs a) {
  extern __shared__ double sm_dyn[];
  __shared__ double s_scr4[4 * kMaxWaves];
  if (a.stop_flag) {
    if (__atomic_load_n(a.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int i = blockIdx.x, d = a.d, p = a.p, dd = d * d, dp = d * p, tid = threadIdx.x;
  const int es = wide_stiefel_epi_stride(d, p);
  double *S = sm_dyn, *C = S + es, *Ad = C + es, *G = Ad + es, *F = G + es, *M = F + es, *W = M + es;
  const T *__restrict__ Sin = static_cast<const T *>(a.X_in);
  const T *__restrict__ Pp = static_cast<const T *>(a.part);
  const T *__restrict__ A = static_cast<const T *>(a.A);
  for (int e = tid; e < dp; e += blockDim.x) {
    const int r = e / p, k = e % p;
    const int64_t row = (int64_t)i * d + r;
    S[e] = (double)Sin[row * p + k];
    double c = 0.0;
    for (int s = 0; s < a.g.ks; ++s) c += (double)Pp[((size_t)s * a.g.rows_pad + row) * 32 + k];
    C[e] = c;
  }
  for (int e = tid; e < dd; e += blockDim.x) {
    const int64_t row = (int64_t)i * d + e / d;
    Ad[e] = (double)A[row * a.ld + (int64_t)i * d + e % d];
  }
  __syncthreads();
  wmm_rect<false, false>(W, Ad, S, d, d, p);                    // A_ii S_i
  const double nm1 = (double)(a.n - 1), mu = a.mu;
  for (int e = tid; e < dp; e += blockDim.x) G[e] = nm1 * S[e] - (C[e] - W[e]);
  __syncthreads();
  wmm_rect<false, true>(M, G, S, d, p, d);                      // G_i S_i^T
  for (int e = tid; e < dd; e += blockDim.x) Ad[e] = 0.5 * (M[e] + M[(e % d) * d + e / d]);
  __syncthreads();
  wmm_rect<false, false>(W, Ad, S, d, d, p);                    // sym(G_i S_i^T) S_i
  for (int e = tid; e < dp; e += blockDim.x) F[e] = S[e] - mu * (G[e] - W[e]);
  __syncthreads();
  wmm_rect<false, true>(M, F, F, d, p, d);                      // F_i F_i^T
  double red[4] = {0.0, 0.0, 0.0, 0.0};                         // x2 dx2 nonfin def2
  for (int e = tid; e < dd; e += blockDim.x) {
    const double v = ((e / d) == (e % d) ? 1.0 : 0.0) - M[e];
    red[3] += v * v;
  }
  double *cur = F, *nxt = G;
  for (int st = 0; st < a.ns_steps; ++st) {
    if (st > 0) wmm_rect<false, true>(M, cur, cur, d, p, d);
    wmm_rect<false, false>(W, M, cur, d, d, p);                 // (S S^T) S
    for (int e = tid; e < dp; e += blockDim.x) nxt[e] = 1.5 * cur[e] - 0.5 * W[e];
    __syncthreads();
    double *t = cur;
    cur = nxt;
    nxt = t;
  }
  T *__restrict__ So = static_cast<T *>(a.X_out);
  for (int e = tid; e < dp; e += blockDim.x) {
    const T v = (T)cur[e];
    So[((int64_t)i * d + e / p) * p + e % p] = v;
    const double dv = (double)v - S[e];
    red[0] += S[e] * S[e];
    red[1] += dv * dv;
    red[2] += isfinite(v) ? 0.0 : 1.0;
  }
  block_sum_n<4>(red, s_scr4);
  if (tid == 0) {
    const double dmax = sqrt(red[3]);
    a.stats[i] = WideStat{red[1], red[0], dmax, (red[2] != 0.0 || !isfinite(dmax)) ? 1.0 : 0.0, 0.0, 0.0, 0.0, 0.0};
  }
}

// One wave: the Gram S^T S from its partial sums, its eigenvectors by FP64
// cyclic Jacobi (rotations accumulated in E), and the d columns of the largest
// eigenvalues into basis (p x d, descending).
__global__ void __launch_bounds__(64) stiefel_basis_kernel(const double *gram, int p, int d, double *basis) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double M[NE], E[NE];
  __shared__ double s_scr[kMaxWaves];
  __shared__ int order[kWideMaxD];
  const int k = threadIdx.x, pp = p * p;
  for (int e = k; e < pp; e += blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < kWideGramGroups; ++g) s += gram[(size_t)g * pp + e];
    M[e] = s;
    E[e] = (e / p == e % p) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = k; e < pp; e += blockDim.x) {   // exact symmetry before the rotations
    const int r = e / p, c = e % p;
    if (r < c) {
      const double v = 0.5 * (M[e] + M[c * p + r]);
      M[e] = v;
      M[c * p + r] = v;
    }
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = k; e < pp; e += blockDim.x) {
      const double v = M[e] * M[e];
      tot += v;
      if (e / p != e % p) off += v;
    }
    off = block_sum(off, s_scr);
    tot = block_sum(tot, s_scr);
    if (off <= 1e-30 * tot) break;
    for (int a = 0; a < p - 1; ++a)
      for (int b = a + 1; b < p; ++b) {
        const double apq = M[a * p + b];
        if (apq == 0.0) continue;                       // uniform: every lane reads the same value
        const double theta = (M[b * p + b] - M[a * p + a]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        __syncthreads();
        if (k < p) {                                    // rows a, b of M
          const double ma = M[a * p + k], mb = M[b * p + k];
          M[a * p + k] = c * ma - sn * mb;
          M[b * p + k] = sn * ma + c * mb;
        }
        __syncthreads();
        if (k < p) {                                    // columns a, b of M and of E
          const double ma = M[k * p + a], mb = M[k * p + b];
          M[k * p + a] = c * ma - sn * mb;
          M[k * p + b] = sn * ma + c * mb;
          const double ea = E[k * p + a], eb = E[k * p + b];
          E[k * p + a] = c * ea - sn * eb;
          E[k * p + b] = sn * ea + c * eb;
        }
        __syncthreads();
      }
  }
  if (k == 0) {
    for (int j = 0; j < p; ++j) order[j] = j;
    for (int x = 0; x < p; ++x)
      for (int y = x + 1; y < p; ++y)
        if (M[order[y] * p + order[y]] > M[order[x] * p + order[x]]) {
          const int t = order[x];
          order[x] = order[y];
          order[y] = t;
        }
  }
  __syncthreads();
  for (int e = k; e < p * d; e += blockDim.x) basis[e] = E[(e / d) * p + order[e % d]];
}

// One workgroup per block: X_i = sgn(S_i V) (d x d, FP64 polar).
template <typename T>
__global__ void __launch_bounds__(256) stiefel_round_kernel(const T *S, const double *basis, T *X, int d, int p,
                                                            DevCtl *ctl) {
  constexpr int NE = kWideMaxD * kWideMaxD;
  __shared__ double sS[NE], sV[NE], sM[NE], sN[NE], sQ[NE];
  __shared__ double s_scr[kMaxWaves];
  const int b = blockIdx.x, dd = d * d;
  for (int e = threadIdx.x; e < d * p; e += blockDim.x) sS[e] = (double)S[(int64_t)b * d * p + e];
  for (int e = threadIdx.x; e < p * d; e += blockDim.x) sV[e] = basis[e];
  __syncthreads();
  wmm_rect<false, false>(sQ, sS, sV, d, p, d);
  const int steps = wide_polar(sQ, sM, sN, d, s_scr);
  for (int e = threadIdx.x; e < dd; e += blockDim.x) X[(int64_t)b * dd + e] = (T)sQ[e];
  if (threadIdx.x == 0 && steps < 0) atomicOr(&ctl->init_bad, 1);
}

// ---------------------------------------------------------------------------
// Geometry, workspace and launches.
// ---------------------------------------------------------------------------
int wide_supported_fmt(int fmt) { return fmt == NSRGS_A_F64 || fmt == NSRGS_A_F32; }

// The geometry and workspace depend on the iterate precision only: F64
// storage has FP64 partial products, every other format FP32 ones.
WideGeom wide_geom(int n, int d, int fmt) {
  WideGeom g{};
  const int nd = n * d;
  g.nt = d <= 16 ? 1 : 2;
  g.mt = env_int("NSRGS_WIDE_MT", 4) == 2 ? 2 : 4;
  g.ku = 8 / g.mt;
  g.xcd_remap = env_int("NSRGS_WIDE_XCD", 1) != 0;
  const int V = fmt == NSRGS_A_F64 ? 2 : 4;
  g.kstep = 4 * g.ku * V;
  g.rows = 64 * g.mt;
  g.row_tiles = (nd + g.rows - 1) / g.rows;
  g.rows_pad = g.row_tiles * g.rows;
  // Column chunks so that the grid fills the CUs once (256 workgroups of
  // 64 mt rows) without a part-empty last round; at most 32.  Measured at
  // n = 500, d = 25: one workgroup of 256 rows per CU beats 512 or 1024
  // workgroups of 128 or 256 rows (357 / 370 / 392 us per FP64 iteration).
  g.ks_max = 2048 / ((nd + 127) / 128);   // the same bound for either tile height
  g.ks_max = g.ks_max < 1 ? 1 : g.ks_max > 32 ? 32 : g.ks_max;   // sizes the workspace
  int slots = env_int("NSRGS_WIDE_SLOTS", 256);
  slots = slots < 1 ? 1 : slots > 2048 ? 2048 : slots;
  int ks = slots / g.row_tiles;
  ks = ks < 1 ? 1 : ks > g.ks_max ? g.ks_max : ks;
  const int forced = env_int("NSRGS_WIDE_KS", 0);
  if (forced >= 1) ks = forced < g.ks_max ? forced : g.ks_max;
  const int steps = (nd + g.kstep - 1) / g.kstep;
  const int steps_per = (steps + ks - 1) / ks;
  g.kchunk = steps_per * g.kstep;
  g.ks = (nd + g.kchunk - 1) / g.kchunk;
  g.steps = steps;
  return g;
}

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

WideLayout wide_layout(int n, int d, int fmt) {
  const WideGeom g = wide_geom(n, d, fmt);
  const size_t tb = fmt == NSRGS_A_F64 ? 8 : 4;
  WideLayout L{};
  size_t off = 0;
  L.ctl = off;   off += a256(sizeof(WideCtl));
  L.stats = off; off += a256((size_t)n * sizeof(WideStat));
  // sized for every tile height and step width (rows_pad and steps * kstep
  // are below n d + 256)
  const size_t nd_pad = (size_t)n * d + 256;
  L.part = off;  off += a256((size_t)g.ks_max * nd_pad * 32 * tb);
  L.xs = off;    off += a256(nd_pad * 32 * tb);                             // B operands, 2 tiles
  L.gram = off;  off += a256((size_t)kWideGramGroups * d * d * sizeof(double));
  L.sumsq = off; off += a256(((size_t)((n * d + 63) / 64) * g.ks_max + n) * sizeof(double));
  L.igram = off; off += a256((size_t)n * 2 * d * d * sizeof(double));
  L.total = off;
  return L;
}

template <typename T, int NT, int MT>
static void wide_launch_product_t(const WideArgs &a, hipStream_t s) {
  const int64_t xs_elems = (int64_t)a.g.steps * NT * 64 * (a.g.kstep / 4);
  const int total = a.g.row_tiles * a.g.ks;
  const int wgs = a.g.xcd_remap ? 8 * ((total + 7) / 8) : total;
  if (!a.xs_ready)
    hipLaunchKernelGGL((wide_xs_kernel<T, NT, MT>), dim3((unsigned)((xs_elems + 255) / 256)), dim3(256), 0, s,
                       static_cast<const T *>(a.X_in), a.nd, a.p, a.g.steps, static_cast<T *>(a.xs), a.stop_flag);
  hipLaunchKernelGGL((wide_product_kernel<T, NT, MT>), dim3(wgs), dim3(256), 0, s, a);
}

template <typename T>
static hipError_t wide_launch_product(const WideArgs &a, hipStream_t s) {
  if (a.g.nt == 1) {
    if (a.g.mt == 2) wide_launch_product_t<T, 1, 2>(a, s); else wide_launch_product_t<T, 1, 4>(a, s);
  } else {
    if (a.g.mt == 2) wide_launch_product_t<T, 2, 2>(a, s); else wide_launch_product_t<T, 2, 4>(a, s);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t wide_gram_t(const WideArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(wide_gram_kernel<T>, dim3(kWideGramGroups), dim3(256), 0, s,
                     static_cast<const T *>(a.X_in), a.nd, a.d, a.gram, a.stop_flag);
  return hipGetLastError();
}

template <typename T>
static hipError_t wide_post_t(const WideArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(wide_epilogue_kernel<T>, dim3(a.n), dim3(wide_epi_threads(a.d)), wide_epi_lds(a.d), s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wide_finish_kernel, dim3(1), dim3(kWideFinishThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t wide_init_post_t(const WideArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(wide_epilogue_kernel<T>, dim3(a.n), dim3(wide_epi_threads(a.d)), wide_epi_lds(a.d), s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ne = 2 * a.d * a.d;
  hipLaunchKernelGGL(wide_igram_reduce_kernel, dim3((ne + 63) / 64), dim3(256), 0, s, a.igram, a.n, a.d, a.gram,
                     a.ctl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(wide_gram_finish_kernel, dim3(1), dim3(64), 0, s, a.gram, a.d, a.ctl, a.wctl);
  return hipGetLastError();
}

hipError_t launch_wide_gram(int fmt, const WideArgs &a, hipStream_t s) {
  return fmt == NSRGS_A_F64 ? wide_gram_t<double>(a, s) : wide_gram_t<float>(a, s);
}
hipError_t launch_wide_post(int fmt, const WideArgs &a, hipStream_t s) {
  return fmt == NSRGS_A_F64 ? wide_post_t<double>(a, s) : wide_post_t<float>(a, s);
}
hipError_t launch_wide_init_post(int fmt, const WideArgs &a, hipStream_t s) {
  return fmt == NSRGS_A_F64 ? wide_init_post_t<double>(a, s) : wide_init_post_t<float>(a, s);
}

template <typename T>
static hipError_t wide_step_t(const WideArgs &a, hipStream_t s) {
  hipError_t e;
  if (a.objective && (e = wide_gram_t<T>(a, s)) != hipSuccess) return e;
  if ((e = wide_launch_product<T>(a, s)) != hipSuccess) return e;
  return wide_post_t<T>(a, s);
}

hipError_t launch_wide_step(int fmt, const WideArgs &a, hipStream_t s) {
  if (fmt == NSRGS_A_F64) return wide_step_t<double>(a, s);
  if (fmt == NSRGS_A_F32) return wide_step_t<float>(a, s);
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t wide_init_product_t(const WideArgs &a, hipStream_t s) {
  hipError_t e;
  if ((e = wide_launch_product<T>(a, s)) != hipSuccess) return e;
  return wide_init_post_t<T>(a, s);
}

hipError_t launch_wide_init_product(int fmt, const WideArgs &a, hipStream_t s) {
  if (fmt == NSRGS_A_F64) return wide_init_product_t<double>(a, s);
  if (fmt == NSRGS_A_F32) return wide_init_product_t<float>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_wide_init_apply(int fmt, const void *W, const void *Y, void *Y_next, int nd, int d,
                                  double *partials, int num_groups, DevCtl *ctl, WideCtl *wctl,
                                  int iter, double tol, hipStream_t s) {
  (void)num_groups;
  const int groups = (int)(((int64_t)nd * d + 255) / 256);   // one thread per entry
  num_groups = groups;
  const dim3 grid(groups), block(256);
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(wide_init_apply_kernel<double>, grid, block, 0, s, (const double *)W, (const double *)Y,
                       (double *)Y_next, nd, d, partials, num_groups, ctl, wctl, iter, tol);
  else
    hipLaunchKernelGGL(wide_init_apply_kernel<float>, grid, block, 0, s, (const float *)W, (const float *)Y,
                       (float *)Y_next, nd, d, partials, num_groups, ctl, wctl, iter, tol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wide_init_check_kernel, dim3(1), dim3(256), 0, s, partials, num_groups, d, ctl, wctl, iter, tol);
  return hipGetLastError();
}

hipError_t launch_wide_init_polar(int fmt, const void *Y, void *X0, int n, int d, DevCtl *ctl,
                                  hipStream_t s) {
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(wide_init_polar_kernel<double>, dim3(n), dim3(256), 0, s, (const double *)Y,
                       (double *)X0, n, d, ctl);
  else
    hipLaunchKernelGGL(wide_init_polar_kernel<float>, dim3(n), dim3(256), 0, s, (const float *)Y,
                       (float *)X0, n, d, ctl);
  return hipGetLastError();
}

hipError_t launch_wide_init_finish(DevCtl *ctl, WideCtl *wctl, int d, hipStream_t s) {
  hipLaunchKernelGGL(wide_init_finish_kernel, dim3(1), dim3(64), 0, s, ctl, wctl, d);
  return hipGetLastError();
}

hipError_t launch_wide_ctl_reset(WideCtl *wctl, hipStream_t s) {
  hipLaunchKernelGGL(wide_ctl_reset_kernel, dim3(1), dim3(64), 0, s, wctl);
  return hipGetLastError();
}

template <typename T>
static hipError_t wide_stiefel_step_t(const WideArgs &a, hipStream_t s) {
  hipError_t e;
  if ((e = wide_launch_product<T>(a, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(wide_stiefel_epilogue_kernel<T>, dim3(a.n), dim3(wide_stiefel_epi_threads(a.d, a.p)),
                     wide_stiefel_epi_lds(a.d, a.p), s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(wide_finish_kernel, dim3(1), dim3(kWideFinishThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wide_stiefel_step(int fmt, const WideArgs &a, hipStream_t s) {
  if (fmt == NSRGS_A_F64) return wide_stiefel_step_t<double>(a, s);
  if (fmt == NSRGS_A_F32) return wide_stiefel_step_t<float>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_stiefel_round(int fmt, const void *S, int n, int d, int p, double *gram, double *basis,
                                void *X, DevCtl *ctl, hipStream_t s) {
  hipError_t e;
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(wide_gram_kernel<double>, dim3(kWideGramGroups), dim3(256), 0, s,
                       static_cast<const double *>(S), n * d, p, gram, (const int *)nullptr);
  else
    hipLaunchKernelGGL(wide_gram_kernel<float>, dim3(kWideGramGroups), dim3(256), 0, s,
                       static_cast<const float *>(S), n * d, p, gram, (const int *)nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(stiefel_basis_kernel, dim3(1), dim3(64), 0, s, gram, p, d, basis);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(stiefel_round_kernel<double>, dim3(n), dim3(256), 0, s, static_cast<const double *>(S), basis,
                       static_cast<double *>(X), d, p, ctl);
  else
    hipLaunchKernelGGL(stiefel_round_kernel<float>, dim3(n), dim3(256), 0, s, static_cast<const float *>(S), basis,
                       static_cast<float *>(X), d, p, ctl);
  return hipGetLastError();
}

}  // namespace nsrgs
