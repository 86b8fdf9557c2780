// The streaming kernel of NS-RGS: one pass over A per iteration.
//
// Mode 0 (sync_step, Algorithm 2 of the paper, Sec. 2.2): for a panel of
// R = B d rows (B whole blocks) a workgroup forms
//     C_i = sum_{j != i} A_ij X_j                   (rows of the panel)
// with the diagonal blocks excluded inside the stream, then, on chip,
//     G_i = (n - 1) X_i - C_i
//     F_i = X_i - mu (G_i - X_i G_i^T X_i) / 2
//     X_i <- Newton-Schulz^{Ts}(F_i),  S <- 1.5 S - 0.5 S (S^T S)   (Alg. 1)
// and writes X^{t+1} plus per-panel monitors.  C, G and F never reach memory.
//
// Mode 1 (spectral initialization): the same stream computes W = A Y for the
// panel (no exclusion) and per-panel partial Grams Y^T W and W^T W; a
// one-workgroup kernel then reduces them in FP64 and factors W^T W = R^T R
// (Cholesky-QR).
//
// Data layout: A row-major (16-byte vectors along a row: lane l of a wave reads
// columns [c, c + V) of every panel row, consecutive lanes consecutive vectors,
// so a wave's loads of one row are 1 KB contiguous).  X is nd x d row-major;
// a lane reads the V x d slice of X matching its columns once per column group
// and reuses it for all R rows of the panel.  The W waves of a workgroup split
// the column groups round-robin; partial sums meet in LDS.
#pragma once
#include "device.h"
#include "kernels.h"

namespace nsrgs {

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

template <int FMT>
constexpr int elem_bytes() {
  return FMT == NSRGS_A_F64 ? 8 : FMT == NSRGS_A_F32 ? 4
       : (FMT == NSRGS_A_BF16 || FMT == NSRGS_A_BF16_SPLIT) ? 2 : 1;
}

// Accumulate one column vector [c, c + V) of every panel row, masking the
// matrix tail (columns >= nd) and, with EXCL, each row's own diagonal block.
// Used for the few column groups per panel that need masks, so it favours low
// register use over load batching: rows go in chunks of RC, and a scheduling
// barrier keeps the compiler from hoisting every row's load to the front.
// It has no divergent branch: every load goes to a clamped, in-bounds address
// and a select zeroes what lies outside, so it may be called with any c >= 0
// (c >= nd adds nothing).  (Exec-masked loads under this register pressure let
// the compiler place register copies at the join before the exec mask was
// restored, so the copies skipped the ragged lanes.)
template <int FMT, int D, int R, bool EXCL>
__device__ __forceinline__ void accum_masked(typename Fmt<FMT>::acc_t (&acc)[R][D],
                                             const char *__restrict__ Ab,
                                             const char *__restrict__ Alo,
                                             const int64_t (&rowoff)[R],
                                             const typename Fmt<FMT>::acc_t *__restrict__ X,
                                             int c, int nd, int row0) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  constexpr int EB = elem_bytes<FMT>();
  constexpr int RC = (R % 4 == 0) ? 4 : (R % 3 == 0) ? 3 : (R % 2 == 0) ? 2 : 1;
  T xv[V * D];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int cv = c + v;
    const int src = cv < nd ? cv : nd - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const T x = X[(int64_t)src * D + k];
      xv[v * D + k] = cv < nd ? x : T(0);
    }
  }
  // A rows are padded to whole 16-byte vectors, so a vector that starts below
  // nd stays inside the row; one that starts at or past nd reads column 0.
  const int64_t ca = (int64_t)(c < nd ? c : 0) * EB;
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += RC) {
    uint4 raw[RC], rawlo[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      raw[i] = ld16_stream(Ab + rowoff[r0 + i] + ca);
      if constexpr (FMT == NSRGS_A_BF16_SPLIT)
        rawlo[i] = ld16_stream(Alo + rowoff[r0 + i] + ca);
      else
        rawlo[i] = raw[i];
    }
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int r = r0 + i;
      T a[V];
      expand<FMT>(raw[i], rawlo[i], a);
      const int blk = (row0 + r) / D;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        bool ok = (c + v) < nd;
        if constexpr (EXCL) ok = ok && ((c + v) / D != blk);
        a[v] = ok ? a[v] : T(0);
      }
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = fmaT(a[v], xv[v * D + k], acc[r][k]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Unmasked accumulation of U column vectors per row: vector u of this lane
// starts at column c0 + u * 64 V, so each load instruction of the wave reads
// 1 KB of one row contiguously.  All R x U loads are issued before the
// first FMA.
template <int FMT, int D, int R, int U>
__device__ __forceinline__ void accum_full(typename Fmt<FMT>::acc_t (&acc)[R][D],
                                           const char *__restrict__ Ab,
                                           const char *__restrict__ Alo,
                                           const int64_t (&rowoff)[R],
                                           const typename Fmt<FMT>::acc_t *__restrict__ X,
                                           int c0) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  constexpr int EB = elem_bytes<FMT>();
  constexpr int NQ = V * D * (int)sizeof(T) / 16;
  uint4 xr[U][NQ];
  uint4 raw[U][R];
  uint4 rawlo[U][R];
  // X first, then the rows in the order they are used: the load counter
  // drains in issue order, so the arithmetic on row r can start as soon as
  // row r has arrived instead of waiting for the whole batch.
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int c = c0 + u * kWave * V;
    const uint4 *xp = reinterpret_cast<const uint4 *>(X + (int64_t)c * D);
#pragma unroll
    for (int q = 0; q < NQ; ++q) xr[u][q] = xp[q];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      raw[u][r] = ld16_stream(Ab + rowoff[r] + (int64_t)c * EB);
      if constexpr (FMT == NSRGS_A_BF16_SPLIT)
        rawlo[u][r] = ld16_stream(Alo + rowoff[r] + (int64_t)c * EB);
      else
        rawlo[u][r] = raw[u][r];
    }
  }
  // Keep every load of the group ahead of the arithmetic: left alone, the
  // scheduler sinks some of them below the first FMAs to save registers, and
  // their latency is then paid once per group with nothing else in flight.
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T xv[V * D];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if constexpr (sizeof(T) == 4) {
        xv[4 * q + 0] = __uint_as_float(xr[u][q].x);
        xv[4 * q + 1] = __uint_as_float(xr[u][q].y);
        xv[4 * q + 2] = __uint_as_float(xr[u][q].z);
        xv[4 * q + 3] = __uint_as_float(xr[u][q].w);
      } else {
        xv[2 * q + 0] = __hiloint2double((int)xr[u][q].y, (int)xr[u][q].x);
        xv[2 * q + 1] = __hiloint2double((int)xr[u][q].w, (int)xr[u][q].z);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T a[V];
      expand<FMT>(raw[u][r], rawlo[u][r], a);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = fmaT(a[v], xv[v * D + k], acc[r][k]);
    }
  }
}

// The two halves of one unmasked column vector per row, for the software
// pipeline of panel_compute: issue the R row loads and the X slice of the
// next column group, then accumulate the current one (loaded one round
// earlier) while those loads are in flight.  Loading the X slice with its
// group keeps the wait for the current operands from also waiting for the
// prefetch (the load counter drains in issue order).
template <int FMT, int D>
constexpr int x_quads() {
  return Fmt<FMT>::V * D * (int)sizeof(typename Fmt<FMT>::acc_t) / 16;
}

template <int FMT, int D, int R, int NQ>
__device__ __forceinline__ void load_group(uint4 (&raw)[R], uint4 (&rawlo)[R], uint4 (&xr)[NQ],
                                           const char *__restrict__ Ab, const char *__restrict__ Alo,
                                           const int64_t (&rowoff)[R],
                                           const typename Fmt<FMT>::acc_t *__restrict__ X, int c) {
  constexpr int EB = elem_bytes<FMT>();
  const uint4 *xp = reinterpret_cast<const uint4 *>(X + (int64_t)c * D);
#pragma unroll
  for (int q = 0; q < NQ; ++q) xr[q] = xp[q];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    raw[r] = ld16_stream(Ab + rowoff[r] + (int64_t)c * EB);
    if constexpr (FMT == NSRGS_A_BF16_SPLIT)
      rawlo[r] = ld16_stream(Alo + rowoff[r] + (int64_t)c * EB);
  }
  __builtin_amdgcn_sched_barrier(0);   // the prefetch stays ahead of the arithmetic
}

template <int FMT, int D, int R, int NQ>
__device__ __forceinline__ void fma_group(typename Fmt<FMT>::acc_t (&acc)[R][D], const uint4 (&raw)[R],
                                          const uint4 (&rawlo)[R], const uint4 (&xr)[NQ]) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  T xv[V * D];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const uint4 u = xr[q];
    if constexpr (sizeof(T) == 4) {
      xv[4 * q + 0] = __uint_as_float(u.x);
      xv[4 * q + 1] = __uint_as_float(u.y);
      xv[4 * q + 2] = __uint_as_float(u.z);
      xv[4 * q + 3] = __uint_as_float(u.w);
    } else {
      xv[2 * q + 0] = __hiloint2double((int)u.y, (int)u.x);
      xv[2 * q + 1] = __hiloint2double((int)u.w, (int)u.z);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T a[V];
    expand<FMT>(raw[r], FMT == NSRGS_A_BF16_SPLIT ? rawlo[r] : raw[r], a);
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int k = 0; k < D; ++k) acc[r][k] = fmaT(a[v], xv[v * D + k], acc[r][k]);
  }
}

// Per-block Riemannian step and Newton-Schulz retraction of B blocks whose
// C_i (sum over j != i of A_ij X_j) and X_i are in LDS (sC, sX: B d x d
// entries, row-major per block); sG, sT, sF, sM are LDS scratch of the same
// size.  Writes X^{t+1} for rows row0 .. row0 + B d - 1 (those below nd) and
// the blocks' monitors to *stat.  Every thread of the workgroup calls it.
template <typename T, int D, int B>
__device__ __forceinline__ void block_step_epilogue(int n, double mu_d, int ns_steps, int nd, int row0,
                                                    T *__restrict__ Xo, PanelStat *stat, T *sX, T *sC,
                                                    T *sG, T *sT, T *sF, T *sM, double *s_scr) {
  constexpr int NE = B * D * D;
  const int tid = threadIdx.x;
  // ---- fused per-block Riemannian step and Newton-Schulz retraction ----
  const T nm1 = T(n - 1);
  const T mu = T(mu_d);
  for (int e = tid; e < NE; e += blockDim.x) sG[e] = nm1 * sX[e] - sC[e];
  __syncthreads();
  // sT = G^T X  (per block)
  for (int e = tid; e < NE; e += blockDim.x) {
    const int bb = (e / (D * D)) * D * D, a = (e / D) % D, k = e % D;
    T s = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) s = fmaT(sG[bb + m * D + a], sX[bb + m * D + k], s);
    sT[e] = s;
  }
  __syncthreads();
  // F = X - mu (G - X (G^T X)) / 2
  for (int e = tid; e < NE; e += blockDim.x) {
    const int bb = (e / (D * D)) * D * D, a = (e / D) % D, k = e % D;
    T s = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) s = fmaT(sX[bb + a * D + m], sT[bb + m * D + k], s);
    const T P = T(0.5) * (sG[e] - s);
    sF[e] = sX[e] - mu * P;
  }
  __syncthreads();
  T *cur = sF;
  T *nxt = sT;
  const int steps = ns_steps;
  for (int st = 0; st < (steps > 0 ? steps : 1); ++st) {
    // M = S^T S
    for (int e = tid; e < NE; e += blockDim.x) {
      const int bb = (e / (D * D)) * D * D, a = (e / D) % D, k = e % D;
      T s = 0;
#pragma unroll
      for (int m = 0; m < D; ++m) s = fmaT(cur[bb + m * D + a], cur[bb + m * D + k], s);
      sM[e] = s;
      if (st == 0) {
        const T dlt = (a == k ? T(1) : T(0)) - s;
        sC[e] = dlt * dlt;                       // defect terms of F^T F
      }
    }
    __syncthreads();
    if (st < steps) {
      // S <- 1.5 S - 0.5 S M
      for (int e = tid; e < NE; e += blockDim.x) {
        const int bb = (e / (D * D)) * D * D, a = (e / D) % D, k = e % D;
        T s = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) s = fmaT(cur[bb + a * D + m], sM[bb + m * D + k], s);
        nxt[e] = T(1.5) * cur[e] - T(0.5) * s;
      }
      __syncthreads();
      T *tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
  }
  // ---- write X^{t+1} and the panel monitors ------------------------------
  double dx2 = 0.0, x2 = 0.0, dmax = 0.0;
  int nonfin = 0;
  for (int e = tid; e < NE; e += blockDim.x) {
    const int row = row0 + e / D;
    if (row < nd) {
      const T v = cur[e];
      Xo[(int64_t)row * D + (e % D)] = v;
      const double dv = (double)v - (double)sX[e];
      dx2 += dv * dv;
      x2 += (double)sX[e] * (double)sX[e];
      nonfin |= !isfinite(v);
    }
  }
  for (int b = tid; b < B; b += blockDim.x) {
    if (row0 + b * D < nd) {
      double s = 0.0;
      for (int j = 0; j < D * D; ++j) s += (double)sC[b * D * D + j];
      const double df = sqrt(s);
      dmax = df > dmax ? df : dmax;
      nonfin |= !isfinite(df);
    }
  }
  dx2 = block_sum(dx2, s_scr);
  x2 = block_sum(x2, s_scr);
  dmax = block_max(dmax, s_scr);
  const double nf = block_max((double)nonfin, s_scr);
  if (tid == 0) *stat = PanelStat{dx2, x2, dmax, nf};
}

// One panel of R = B d rows: what one workgroup does per column sweep.
struct PanelJob {
  const void *A;          // storage of this problem's A
  const void *A_lo;
  const float *scale;
  int64_t ld;
  const void *X_in;       // X^t (mode 0) or Y (mode 1)
  void *X_out;            // X^{t+1} (mode 0) or W = A Y (mode 1)
  int n, nd, panel;
  double mu;
  int ns_steps;
  PanelStat *stat;        // mode 0: where this panel's monitors go
  void *gram;             // mode 1: where this panel's 2 d^2 partial Grams go
};

// Stream the panel's rows of A once, reduce the per-lane sums over the
// workgroup, then (mode 0) run the per-block Riemannian step and
// Newton-Schulz retraction on chip and write X^{t+1} and the panel monitors,
// or (mode 1) write W = A Y and the panel's partial Grams.  Every thread of
// the workgroup must call it; it ends with a barrier, so LDS can be reused.
// LDS bytes panel_compute needs for a panel of B blocks of d x d.
template <int FMT, int D, int B>
constexpr int panel_lds_bytes() {
  using T = typename Fmt<FMT>::acc_t;
  return (int)(sizeof(double) * kMaxWaves + sizeof(T) * (kMaxWaves + 6) * B * D * D);
}

template <int FMT, int D, int B, int U, int MODE>
__device__ __forceinline__ void panel_compute(const PanelJob &job, char *lds) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  constexpr int R = B * D;
  constexpr int NE = R * D;              // panel entries of C (= B blocks of d x d)
  constexpr int UV = U > 0 ? U : 1;      // vectors per row per loop iteration
  constexpr int GROUP = kWave * V * UV;  // columns per wave per loop iteration
  constexpr int EB = elem_bytes<FMT>();
  constexpr bool EXCL = (MODE == 0);

  // LDS carve-up (caller-provided, panel_lds_bytes<FMT, D, B>() bytes, 8-aligned)
  double *s_scr = reinterpret_cast<double *>(lds);
  T (*s_red)[NE] = reinterpret_cast<T (*)[NE]>(lds + sizeof(double) * kMaxWaves);
  T *sX = reinterpret_cast<T *>(lds + sizeof(double) * kMaxWaves) + kMaxWaves * NE;
  T *sC = sX + NE, *sG = sC + NE, *sT = sG + NE, *sF = sT + NE, *sM = sF + NE;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  // wave index, provably uniform: the column-group loops below branch on it
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int nw = blockDim.x / kWave;
  const int nd = job.nd;
  const int row0 = job.panel * R;
  const T *__restrict__ X = static_cast<const T *>(job.X_in);
  const char *__restrict__ Ab = static_cast<const char *>(job.A);
  const char *__restrict__ Alo = static_cast<const char *>(job.A_lo);

  int64_t rowoff[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int row = (row0 + r < nd) ? row0 + r : nd - 1;   // clamp: tail rows unused
    rowoff[r] = (int64_t)row * job.ld * EB;
  }

  T acc[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[r][k] = T(0);

  // Column groups go round-robin to the waves.  The groups that hold this
  // panel's diagonal blocks (mode 0) and the ragged last group are taken out
  // of the main loop (a wave-uniform test) and done with masks afterwards.
  const int ngroups = (nd + GROUP - 1) / GROUP;
  const int nfull = nd / GROUP;
  int gd0 = -1, gd1 = -1;
  if constexpr (EXCL) {
    gd0 = row0 / GROUP;
    gd1 = min(row0 + R - 1, nd - 1) / GROUP;
  }
  if constexpr (U == 0) {
    // Software pipeline over this wave's full groups (diagonal groups skipped):
    // the loads of the next group are in flight while the current one is
    // accumulated.  g, gn are wave-uniform, so the branches are scalar.  The
    // skip is two selects, not a loop: gd1 <= gd0 + 1, so at most two steps
    // land on diagonal groups, and a loop nested in the pipelined one makes
    // the compiler drain every load in flight (the prefetch too) on entry.
    auto skip_diag = [&](int g) {
      g = (g == gd0 || g == gd1) ? g + nw : g;
      return (g == gd0 || g == gd1) ? g + nw : g;
    };
    // Two register buffers take turns (unrolled by two, so no copy hands one
    // over to the other).  The loop runs while two more groups remain, so
    // every load it issues is consumed on every path (by its own second half,
    // or by the next round or the tail): a prefetch that some path leaves
    // unused gets sunk past the branch by the compiler, behind the arithmetic
    // it was meant to overlap.
    constexpr int NQ = x_quads<FMT, D>();
    int g = skip_diag(wave);
    if (g < nfull) {
      uint4 b0[R], b0lo[R], x0[NQ], b1[R], b1lo[R], x1[NQ];
      load_group<FMT, D, R, NQ>(b0, b0lo, x0, Ab, Alo, rowoff, X, g * GROUP + lane * V);
      int ga = skip_diag(g + nw);
      int gb = skip_diag(ga + nw);
      while (gb < nfull) {                 // b0 holds g; ga < gb are the next two
        load_group<FMT, D, R, NQ>(b1, b1lo, x1, Ab, Alo, rowoff, X, ga * GROUP + lane * V);
        fma_group<FMT, D, R, NQ>(acc, b0, b0lo, x0);
        load_group<FMT, D, R, NQ>(b0, b0lo, x0, Ab, Alo, rowoff, X, gb * GROUP + lane * V);
        fma_group<FMT, D, R, NQ>(acc, b1, b1lo, x1);
        g = gb;
        ga = skip_diag(g + nw);
        gb = skip_diag(ga + nw);
      }
      if (ga < nfull) {                    // one more group
        load_group<FMT, D, R, NQ>(b1, b1lo, x1, Ab, Alo, rowoff, X, ga * GROUP + lane * V);
        fma_group<FMT, D, R, NQ>(acc, b0, b0lo, x0);
        fma_group<FMT, D, R, NQ>(acc, b1, b1lo, x1);
      } else {
        fma_group<FMT, D, R, NQ>(acc, b0, b0lo, x0);
      }
    }
  } else {
    // One path through the loop body (the diagonal groups are stepped over
    // by the induction, not by a branch in the body).
    auto skip_diag = [&](int g) {
      while (g < nfull && (g == gd0 || g == gd1)) g += nw;
      return g;
    };
    for (int g = skip_diag(wave); g < nfull; g = skip_diag(g + nw))
      accum_full<FMT, D, R, U>(acc, Ab, Alo, rowoff, X, g * GROUP + lane * V);
  }
  const int gt = nfull < ngroups ? nfull : -1;
  for (int q = 0; q < 3; ++q) {
    const int g = q == 0 ? gd0 : q == 1 ? gd1 : gt;
    if (g < 0 || g % nw != wave) continue;
    if (q == 1 && g == gd0) continue;
    if (q == 2 && (g == gd0 || g == gd1)) continue;
#pragma unroll
    for (int u = 0; u < UV; ++u) {
      const int c = g * GROUP + u * kWave * V + lane * V;
      accum_masked<FMT, D, R, EXCL>(acc, Ab, Alo, rowoff, X, c, nd, row0);
    }
  }

  // ---- reduce the panel sums over lanes, then over waves -----------------
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T v = wave_sum(acc[r][k]);
      if (lane == 0) s_red[wave][r * D + k] = v;
    }
  __syncthreads();
  for (int e = tid; e < NE; e += blockDim.x) {
    T s = s_red[0][e];
    for (int w = 1; w < nw; ++w) s += s_red[w][e];
    const int row = row0 + e / D;
    if constexpr (FMT == NSRGS_A_FP8_E4M3) s *= (row < nd) ? job.scale[row] : 0.0f;
    sC[e] = s;
    sX[e] = (row < nd) ? X[(int64_t)row * D + (e % D)] : T(0);
  }
  __syncthreads();

  if constexpr (MODE == 0) {
    block_step_epilogue<T, D, B>(job.n, job.mu, job.ns_steps, nd, row0, static_cast<T *>(job.X_out),
                                 job.stat, sX, sC, sG, sT, sF, sM, s_scr);
  } else {
    // ---- mode 1: W = A Y for the panel rows; partial Grams Y^T W, W^T W ----
    T *__restrict__ Wo = static_cast<T *>(job.X_out);
    for (int e = tid; e < NE; e += blockDim.x) {
      const int row = row0 + e / D;
      if (row < nd) Wo[(int64_t)row * D + (e % D)] = sC[e];
    }
    T *part = static_cast<T *>(job.gram);
    for (int e = tid; e < D * D; e += blockDim.x) {
      const int a = e / D, k = e % D;
      T g1 = 0, g2 = 0;
      for (int r = 0; r < R; ++r) {
        if (row0 + r < nd) {
          g1 = fmaT(sX[r * D + a], sC[r * D + k], g1);
          g2 = fmaT(sC[r * D + a], sC[r * D + k], g2);
        }
      }
      part[e] = g1;
      part[D * D + e] = g2;
    }
  }
  __syncthreads();
}

// After a mode-0 launch (one workgroup): reduce the panel monitors in a fixed
// order (FP64) into the control block and apply the stop rule.
__device__ inline void finish_step(const StreamArgs &args, double *s_scr) {
  const int tid = threadIdx.x;
  DevCtl *ctl = args.ctl;
  const PanelStat *part = static_cast<const PanelStat *>(args.partials);
  double a = 0.0, bsum = 0.0, m = 0.0, f = 0.0;
  for (int p = tid; p < args.num_panels; p += blockDim.x) {
    const PanelStat q = part[p];
    a += q.dx2;
    bsum += q.x2;
    m = q.dmax > m ? q.dmax : m;
    f = q.nonfinite > f ? q.nonfinite : f;
  }
  a = block_sum(a, s_scr);
  bsum = block_sum(bsum, s_scr);
  m = block_max(m, s_scr);
  f = block_max(f, s_scr);
  if (tid == 0) {
    const double rel = bsum > 0.0 ? sqrt(a / bsum) : 0.0;
    ctl->sum_dx2 = a;
    ctl->sum_x2 = bsum;
    ctl->rel_change = rel;
    ctl->max_defect = m;
    ctl->nonfinite = f != 0.0;
    ctl->iters = args.iter + 1;
    if (f != 0.0 || !isfinite(rel)) {
      ctl->nonfinite = 1;
      ctl->done = 1;
    } else if (args.tol > 0.0 && rel <= args.tol) {
      ctl->converged = 1;
      ctl->done = 1;
    }
    ctl->arrive = 0u;
  }
}

// After a mode-1 launch (one workgroup): FP64 reduction of the partial Grams,
// the Rayleigh quotient T = Y^T A Y and the Cholesky factor of W^T W.
template <typename T, int D>
__device__ inline void finish_gram(const StreamArgs &args) {
  __shared__ double G1[kMaxD * kMaxD], G2[kMaxD * kMaxD], Rm[kMaxD * kMaxD];
  const int tid = threadIdx.x;
  DevCtl *ctl = args.ctl;
  const T *all = static_cast<const T *>(args.partials);
  for (int e = tid; e < 2 * D * D; e += blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < args.num_panels; ++p) s += (double)all[(int64_t)p * 2 * D * D + e];
    if (e < D * D) G1[e] = s; else G2[e - D * D] = s;
  }
  __syncthreads();
  if (tid == 0) {
    int bad = 0;
    for (int a = 0; a < D; ++a)
      for (int k = 0; k < D; ++k) ctl->T[a * D + k] = 0.5 * (G1[a * D + k] + G1[k * D + a]);
    for (int j = 0; j < D * D; ++j) Rm[j] = 0.0;
    for (int j = 0; j < D; ++j) {
      double s = G2[j * D + j];
      for (int q = 0; q < j; ++q) s -= Rm[q * D + j] * Rm[q * D + j];
      if (!(s > 0.0) || !isfinite(s)) { bad = 1; s = 1.0; }
      const double rjj = sqrt(s);
      Rm[j * D + j] = rjj;
      for (int k = j + 1; k < D; ++k) {
        double t = G2[j * D + k];
        for (int q = 0; q < j; ++q) t -= Rm[q * D + j] * Rm[q * D + k];
        Rm[j * D + k] = t / rjj;
      }
    }
    // Rinv = R^{-1} (upper triangular), column by column.
    for (int j = 0; j < D * D; ++j) ctl->Rinv[j] = 0.0;
    for (int k = 0; k < D; ++k) {
      ctl->Rinv[k * D + k] = 1.0 / Rm[k * D + k];
      for (int i = k - 1; i >= 0; --i) {
        double s = 0.0;
        for (int q = i + 1; q <= k; ++q) s += Rm[i * D + q] * ctl->Rinv[q * D + k];
        ctl->Rinv[i * D + k] = -s / Rm[i * D + i];
      }
    }
    if (bad) ctl->init_bad = 1;
    ctl->arrive2 = 0u;
  }
}

template <int FMT, int D, int B, int U, int MODE>
__global__ void __launch_bounds__(kWave * (U == 0 ? kPipeMaxWaves : kMaxWaves))
stream_kernel(StreamArgs args) {
  using T = typename Fmt<FMT>::acc_t;
  __shared__ __attribute__((aligned(16))) char lds[panel_lds_bytes<FMT, D, B>()];
  if (args.stop_flag) {
    if (__atomic_load_n(args.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  PanelJob job;
  job.A = args.A;
  job.A_lo = args.A_lo;
  job.scale = args.scale;
  job.ld = args.ld;
  job.X_in = args.X_in;
  job.X_out = args.X_out;
  job.n = args.n;
  job.nd = args.nd;
  job.panel = blockIdx.x;
  job.mu = args.mu;
  job.ns_steps = args.ns_steps;
  job.stat = static_cast<PanelStat *>(args.partials) + blockIdx.x;
  job.gram = static_cast<T *>(args.partials) + (int64_t)blockIdx.x * 2 * D * D;
  panel_compute<FMT, D, B, U, MODE>(job, lds);
}

// The per-panel results are reduced by a second, one-workgroup kernel on the
// same stream: the kernel boundary orders every panel's writes before the
// reduction once per step.  (A last-arriving workgroup would need a release
// fence in every workgroup, and each of those writes back the L2; at
// thousands of panels per step that cost about a tenth of the stream.)
template <typename T, int D, int MODE>
__global__ void __launch_bounds__(256) stream_finish_kernel(StreamArgs args) {
  __shared__ double s_scr[kMaxWaves];
  if (args.stop_flag) {
    if (__atomic_load_n(args.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  if constexpr (MODE == 0) finish_step(args, s_scr);
  else finish_gram<T, D>(args);
}

// ---------------------------------------------------------------------------
// Instantiation table: (d, B, U) triples, R = B d rows per panel; U >= 1
// loads U vectors per row together (X slice first, every load ahead of the
// arithmetic) and then accumulates them; U = 0 is one vector per row per
// iteration with the next iteration's loads issued into a second register
// buffer before this one's arithmetic (software pipeline; it pays only while
// two buffers fit in registers, so only small d have it).  Mode 1 (the
// spectral-initialization product) uses the second table.
// ---------------------------------------------------------------------------
#define NSRGS_BOPTS(X)                                                                      \
  X(1, 8, 1) X(1, 16, 1) X(1, 8, 0) X(1, 8, 2)                                             \
  X(2, 4, 1) X(2, 8, 1) X(2, 4, 0) X(2, 4, 2)                                              \
  X(3, 4, 1) X(3, 2, 1) X(3, 8, 1) X(3, 4, 0) X(3, 2, 2) X(3, 4, 2) X(3, 1, 2) X(3, 1, 4)  \
  X(3, 2, 4)                                                                               \
  X(4, 2, 1) X(4, 4, 1) X(4, 2, 0) X(4, 2, 2) X(4, 1, 2)                                   \
  X(5, 1, 1) X(5, 2, 1) X(6, 1, 1) X(6, 2, 1) X(7, 1, 1) X(7, 2, 1) X(8, 1, 1) X(8, 2, 1)  \
  X(9, 1, 1) X(10, 1, 1) X(11, 1, 1) X(12, 1, 1) X(13, 1, 1) X(14, 1, 1) X(15, 1, 1)      \
  X(16, 1, 1)

#define NSRGS_BOPTS_INIT(X)                                                   \
  X(1, 8, 1) X(2, 4, 1) X(3, 4, 1) X(4, 2, 1) X(5, 1, 1) X(6, 1, 1) X(7, 1, 1) \
  X(8, 1, 1) X(9, 1, 1) X(10, 1, 1) X(11, 1, 1) X(12, 1, 1) X(13, 1, 1)        \
  X(14, 1, 1) X(15, 1, 1) X(16, 1, 1)

template <int MODE, int FMT, int D, int B, int U>
hipError_t launch_one(const StreamConfig &cfg, const StreamArgs &args, hipStream_t s) {
  using T = typename Fmt<FMT>::acc_t;
  // the pipelined shapes take at most kPipeMaxWaves waves per workgroup
  const int waves = U == 0 && cfg.waves > kPipeMaxWaves ? kPipeMaxWaves : cfg.waves;
  const dim3 grid(args.num_panels), block(kWave * waves);
  hipLaunchKernelGGL((stream_kernel<FMT, D, B, U, MODE>), grid, block, 0, s, args);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((stream_finish_kernel<T, D, MODE>), dim3(1), dim3(256), 0, s, args);
  return hipGetLastError();
}

// Dispatch to the compiled shapes with DLO <= d <= DHI (the step kernels of
// one format are split over two translation units by d so the library builds
// in parallel).
template <int MODE, int FMT, int DLO = 1, int DHI = kMaxD>
hipError_t launch_fmt_impl(const StreamConfig &cfg, const StreamArgs &args, hipStream_t s) {
#define NSRGS_CASE(DD, BB, UU)                                                          \
  if constexpr (DD >= DLO && DD <= DHI)                                                   \
    if (args.d == DD && cfg.blocks_per_panel == BB && cfg.unroll == UU)                   \
      return launch_one<MODE, FMT, DD, BB, UU>(cfg, args, s);
  if constexpr (MODE == 0) {
    NSRGS_BOPTS(NSRGS_CASE)
  } else {
    NSRGS_BOPTS_INIT(NSRGS_CASE)
  }
#undef NSRGS_CASE
  return hipErrorInvalidValue;
}

}  // namespace nsrgs
