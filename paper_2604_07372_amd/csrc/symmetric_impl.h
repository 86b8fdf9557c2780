// Symmetric half-stream step (the symmetric measurement matrix, Sec. 2.2:
// A_ji = A_ij^T).  Only the blocks above the block diagonal are streamed, and
// each element is used twice: C_i += A_ij X_j (row direction) and
// C_j += A_ij^T X_i (column direction), so one iteration reads about half of A.
//
// Work is cut into tiles: strips of H rows (a multiple of d) by chunks of
// CW = W * 64 * V * U columns, the tiles on or above the block diagonal.  In a
// tile each lane owns U column vectors for the whole strip and walks the
// strip's rows in panels of R rows:
//   * column direction: the lane's V x d sums over the strip's rows stay in
//     registers (X_i of the panel rows is wave-uniform);
//   * row direction: the R x d per-lane sums of a panel are reduced over the
//     wave by a transpose-reduce and kept in LDS per wave.
// At the end of the tile the row sums (H x d) go to prow[chunk] and the column
// sums (CW x d) to pcol[strip].  A second kernel adds, for each row, the row
// sums of its strip's tiles and the column sums of the tiles above it in its
// column, in a fixed order, and runs the per-block epilogue.  Elements on or
// below the block diagonal, or past nd, are masked with selects (no divergent
// branch), and only diagonal and ragged tiles take the masked path.
#pragma once

#include <limits.h>

#include "stream_impl.h"

namespace nsrgs {

struct SymArgs {
  const void *A;
  const void *A_lo;
  int64_t ld;             // elements; NSRGS_LD_PACKED: packed upper block triangle
  int64_t ndp;            // packed: n d rounded up to 64 (packed_ndp)
  const void *X_in;
  int nd;
  int H;          // strip height (rows), a multiple of d, of R and of the epilogue panel
  int CW;         // chunk width (columns) = waves * 64 * V * U
  int nchunks;
  int nstrips;
  void *prow;     // nchunks x nd x d: row sums of tile (strip(r), chunk) at row r
  void *pcol;     // nstrips x nd x d: column sums of tile (strip, chunk(c)) at column c
  const int *stop_flag;   // non-NULL: return at once when *stop_flag != 0
};

// Compiled tile shapes (d, R panel rows, U vectors per lane per row); the
// first one of each d is the default.  R d accumulators and R U loads per
// lane per panel; R d <= 64 (one value per lane after the transpose-reduce).
#define NSRGS_SYM_SHAPES(X)                                                                  \
  X(1, 16, 1) X(2, 16, 1) X(3, 12, 1) X(3, 16, 1) X(3, 12, 2) X(3, 6, 2) X(4, 12, 1) X(4, 8, 2) \
  X(4, 16, 1) X(5, 10, 1) X(6, 8, 1) X(7, 7, 1) X(8, 8, 1) X(9, 4, 1) X(10, 4, 1) X(11, 4, 1)    \
  X(12, 4, 1) X(13, 4, 1) X(14, 4, 1) X(15, 4, 1) X(16, 4, 1)

// Blocks per epilogue workgroup, per d.
constexpr int sym_epi_blocks(int d) { return d == 1 ? 64 : d == 2 ? 32 : d <= 4 ? 16 : d == 5 ? 8 : d == 6 ? 6 : 4; }
constexpr int kSymMaxD = 16;
// 2-byte formats: above d = 12 a lane's 8-element column slice and its sums
// (16 d values) spill, and the step measured slower than the full stream
// (n d = 30000, BF16: d = 13 2.01 ms against 1.59, d = 16 7.2 against 3.06).
constexpr int kSymMaxD2 = 12;

// The rows [strip0, strip1) of one tile for this wave's columns.
template <int FMT, int D, int R, int U, bool MASK>
__device__ __forceinline__ void sym_tile_rows(const SymArgs &a, const typename Fmt<FMT>::acc_t *__restrict__ X,
                                              int strip0, int strip1, int lane, int cw0,
                                              const int (&col)[U],
                                              const typename Fmt<FMT>::acc_t (&xc)[U][Fmt<FMT>::V][D],
                                              typename Fmt<FMT>::acc_t (&cacc)[U][Fmt<FMT>::V][D],
                                              typename Fmt<FMT>::acc_t *myrow) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  constexpr int EB = elem_bytes<FMT>();
  constexpr int N = R * D;
  constexpr int WCOLS = kWave * V * U;
  const int nd = a.nd;
  const char *__restrict__ Ab = static_cast<const char *>(a.A);
  const char *__restrict__ Alo = static_cast<const char *>(a.A_lo);

  const int ridx = wave_tr_entry<N>(lane);

  // masked path: block index of each column (-1 past nd, so nothing counts)
  int cblk[U][V];
  int cc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    cc[u] = (!MASK || col[u] < nd) ? col[u] : 0;   // clamped load column
#pragma unroll
    for (int v = 0; v < V; ++v) cblk[u][v] = (col[u] + v < nd) ? (col[u] + v) / D : -1;
  }
  // wave-uniform: the block of this wave's last column inside the matrix
  const int wlast_blk = cw0 < nd ? (min(cw0 + WCOLS, nd) - 1) / D : -1;

  // packed layout: element offset of the next panel's first row, carried from
  // panel to panel (-1: compute it from the closed form)
  int64_t next_off = -1;
  for (int row0 = strip0; row0 < strip1; row0 += R) {
    T *out = myrow + (row0 - strip0) * D;
    if (MASK && row0 / D >= wlast_blk) {
      // every element of this panel in this wave's columns is on or below the
      // block diagonal (or past nd): its sums are zero
      static_assert(N <= kWave, "one lane per panel entry");
      out[lane < N ? lane : N - 1] = T(0);
      next_off = -1;
      continue;
    }
    int64_t rowoff[R];
    if (a.ld == NSRGS_LD_PACKED) {
      // byte offset of column 0 of each row in the packed layout (columns left
      // of the row's stored range are never used: they lie below the block
      // diagonal, and a clamped column-0 read lands in earlier rows' storage)
      const int rfirst = (!MASK || row0 < nd) ? row0 : nd - 1;
      int64_t off = next_off >= 0 ? next_off : packed_row_offset(rfirst, D, a.ndp);
      int rlast = rfirst;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = (!MASK || row0 + r < nd) ? row0 + r : nd - 1;
        const int prev = r == 0 ? row : ((!MASK || row0 + r - 1 < nd) ? row0 + r - 1 : nd - 1);
        if (r > 0 && row != prev) off += a.ndp - packed_c0(prev / D, D);   // the previous row's length
        rowoff[r] = (off - packed_c0(row / D, D)) * EB;
        rlast = row;
      }
      // the next panel starts after this panel's last row (past nd: no next panel)
      next_off = off + a.ndp - packed_c0(rlast / D, D);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = (!MASK || row0 + r < nd) ? row0 + r : nd - 1;
        rowoff[r] = (int64_t)row * a.ld * EB;
      }
    }
    uint4 raw[R][U], rawlo[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        raw[r][u] = ld16_stream(Ab + rowoff[r] + (int64_t)cc[u] * EB);
        if constexpr (FMT == NSRGS_A_BF16_SPLIT) rawlo[r][u] = ld16_stream(Alo + rowoff[r] + (int64_t)cc[u] * EB);
        else rawlo[r][u] = make_uint4(0, 0, 0, 0);
      }
    T xr[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int row = (!MASK || row0 + r < nd) ? row0 + r : nd - 1;
#pragma unroll
      for (int k = 0; k < D; ++k) xr[r][k] = X[(int64_t)row * D + k];
    }
    __builtin_amdgcn_sched_barrier(0);

    T acc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int rblk = (row0 + r < nd) ? (row0 + r) / D : INT_MAX;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        T av[V];
        expand<FMT>(raw[r][u], rawlo[r][u], av);
        if constexpr (MASK) {
#pragma unroll
          for (int v = 0; v < V; ++v) av[v] = (rblk < cblk[u][v]) ? av[v] : T(0);
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int k = 0; k < D; ++k) {
            acc[r * D + k] = fmaT(av[v], xc[u][v][k], acc[r * D + k]);
            cacc[u][v][k] = fmaT(av[v], xr[r][k], cacc[u][v][k]);
          }
      }
    }
    wave_tr_step<T, N, 0>(acc, lane);
    out[ridx] = acc[0];
  }
}

// One tile per workgroup: blockIdx.x = chunk, blockIdx.y = strip; tiles left
// of the strip's diagonal chunk return at once.  Dynamic LDS: waves * H * d
// values of the accumulation type.
// X (= a.X_in) is also a separate read-only argument, so the wave-uniform
// reads of the panel rows' X_i can be scalar loads.
template <int FMT, int D, int R, int U>
__global__ void __launch_bounds__(kWave * kMaxWaves)
sym_tile_kernel(SymArgs a, const typename Fmt<FMT>::acc_t *__restrict__ X) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int V = Fmt<FMT>::V;
  constexpr int WCOLS = kWave * V * U;
  extern __shared__ __attribute__((aligned(16))) char sym_lds[];
  const int j = blockIdx.x, s = blockIdx.y;
  const int nd = a.nd, H = a.H, CW = a.CW;
  const int strip0 = s * H;
  if (j < strip0 / CW) return;                     // uniform
  if (a.stop_flag) {
    if (__atomic_load_n(a.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int strip1 = min(strip0 + H, nd);
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int nw = blockDim.x / kWave;
  const int cw0 = j * CW + wave * WCOLS;
  T *s_row = reinterpret_cast<T *>(sym_lds);
  T *myrow = s_row + (int64_t)wave * H * D;

  int col[U];
  T xc[U][V][D], cacc[U][V][D];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    col[u] = cw0 + u * kWave * V + lane * V;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = col[u] + v;
      const int cl = c < nd ? c : nd - 1;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const T x = X[(int64_t)cl * D + k];
        xc[u][v][k] = c < nd ? x : T(0);
        cacc[u][v][k] = T(0);
      }
    }
  }
  // masked path for tiles that reach the block diagonal or the matrix edge
  const bool mask = (j * CW) / D <= (strip1 - 1) / D || (j + 1) * CW > nd || strip0 + H > nd;
  if (mask) sym_tile_rows<FMT, D, R, U, true>(a, X, strip0, strip1, lane, cw0, col, xc, cacc, myrow);
  else sym_tile_rows<FMT, D, R, U, false>(a, X, strip0, strip1, lane, cw0, col, xc, cacc, myrow);
  __syncthreads();

  // row sums: the waves' partials added in wave order
  T *__restrict__ prow = static_cast<T *>(a.prow) + ((int64_t)j * nd + strip0) * D;
  const int nrow = (strip1 - strip0) * D;
  for (int e = tid; e < nrow; e += blockDim.x) {
    T v = s_row[e];
    for (int w = 1; w < nw; ++w) v += s_row[(int64_t)w * H * D + e];
    prow[e] = v;
  }
  // column sums of this lane's columns
  T *__restrict__ pcol = static_cast<T *>(a.pcol) + (int64_t)s * nd * D;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = col[u] + v;
      if (c < nd) {
#pragma unroll
        for (int k = 0; k < D; ++k) pcol[(int64_t)c * D + k] = cacc[u][v][k];
      }
    }
}

// One workgroup per BE blocks: C for each row = the row sums of the tiles of
// its strip (chunks in order) + the column sums of the tiles above it in its
// column (strips in order), then the per-block epilogue of the step.
// One element A(r, c) of the storage (full or packed), as the accumulation type.
template <int FMT>
__device__ __forceinline__ typename Fmt<FMT>::acc_t sym_elem(const SymArgs &a, int d, int r, int c) {
  using T = typename Fmt<FMT>::acc_t;
  const int64_t idx = a.ld == NSRGS_LD_PACKED ? packed_row_offset(r, d, a.ndp) + c - packed_c0(r / d, d)
                                               : (int64_t)r * a.ld + c;
  if constexpr (FMT == NSRGS_A_F64) {
    return static_cast<const double *>(a.A)[idx];
  } else if constexpr (FMT == NSRGS_A_F32) {
    return static_cast<const float *>(a.A)[idx];
  } else {
    const float hi = __uint_as_float((uint32_t)static_cast<const uint16_t *>(a.A)[idx] << 16);
    if constexpr (FMT == NSRGS_A_BF16_SPLIT)
      return hi + __uint_as_float((uint32_t)static_cast<const uint16_t *>(a.A_lo)[idx] << 16);
    else
      return (T)hi;
  }
}

template <int FMT, int D, int BE, int MODE>
__global__ void __launch_bounds__(256) sym_epilogue_kernel(SymArgs a, StreamArgs sa) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int NE = BE * D * D;
  __shared__ double s_scr[kMaxWaves];
  __shared__ T sbuf[6 * NE];
  if (sa.stop_flag) {
    if (__atomic_load_n(sa.stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int tid = threadIdx.x;
  const int nd = a.nd;
  const int row0 = blockIdx.x * BE * D;
  const int s = row0 / a.H;                 // BE d divides H: one strip per workgroup
  const int j0 = (s * a.H) / a.CW;
  T *sX = sbuf, *sC = sX + NE, *sG = sC + NE, *sT = sG + NE, *sF = sT + NE, *sM = sF + NE;
  const T *__restrict__ prow = static_cast<const T *>(a.prow);
  const T *__restrict__ pcol = static_cast<const T *>(a.pcol);
  const T *__restrict__ X = static_cast<const T *>(sa.X_in);
  const int64_t plane = (int64_t)nd * D;
  for (int e = tid; e < NE; e += blockDim.x) {
    const int row = row0 + e / D;
    const int rr = row < nd ? row : nd - 1;
    const int64_t o = (int64_t)rr * D + (e % D);
    // unrolled so that several loads are in flight; the additions stay in order
    T sum = T(0);
#pragma unroll 8
    for (int jj = j0; jj < a.nchunks; ++jj) sum += prow[jj * plane + o];
#pragma unroll 8
    for (int ss = 0; ss <= s; ++ss) sum += pcol[ss * plane + o];
    const T x = X[o];
    sC[e] = row < nd ? sum : T(0);
    sX[e] = row < nd ? x : T(0);
  }
  __syncthreads();
  if constexpr (MODE == 0) {
    block_step_epilogue<T, D, BE>(sa.n, sa.mu, sa.ns_steps, nd, row0, static_cast<T *>(sa.X_out),
                                  static_cast<PanelStat *>(sa.partials) + blockIdx.x, sX, sC, sG, sT, sF,
                                  sM, s_scr);
  } else {
    // W = A Y for the panel's rows: the off-diagonal sums plus A_ii Y_i (the
    // tiles leave the diagonal blocks out), and the panel's partial Grams
    // Y^T W and W^T W for the Cholesky-QR of the initialization.
    for (int e = tid; e < NE; e += blockDim.x) {
      const int row = row0 + e / D, k = e % D;
      const int b0 = (e / (D * D)) * D * D, ar = (e / D) % D;
      T s = T(0);
      if (row < nd) {
        const int ib = row / D;
#pragma unroll
        for (int m = 0; m < D; ++m) s = fmaT(sym_elem<FMT>(a, D, row, ib * D + m), sX[b0 + m * D + k], s);
      }
      sG[e] = sC[e] + s;
      (void)ar;
    }
    __syncthreads();
    T *__restrict__ Wo = static_cast<T *>(sa.X_out);
    for (int e = tid; e < NE; e += blockDim.x) {
      const int row = row0 + e / D;
      if (row < nd) Wo[(int64_t)row * D + (e % D)] = sG[e];
    }
    T *part = static_cast<T *>(sa.partials) + (int64_t)blockIdx.x * 2 * D * D;
    for (int e = tid; e < D * D; e += blockDim.x) {
      const int ar = e / D, k = e % D;
      T g1 = 0, g2 = 0;
      for (int r = 0; r < BE * D; ++r) {
        if (row0 + r < nd) {
          g1 = fmaT(sX[r * D + ar], sG[r * D + k], g1);
          g2 = fmaT(sG[r * D + ar], sG[r * D + k], g2);
        }
      }
      part[e] = g1;
      part[D * D + e] = g2;
    }
  }
}

// mode 0: one step (tile, epilogue, monitor reduction); mode 1: the
// initialization's product W = A Y with the partial Grams and their FP64
// reduction / Cholesky factor (finish_gram).
template <int FMT, int D, int R, int U>
hipError_t sym_launch_shape(const SymArgs &a, const StreamArgs &sa, int waves, int mode, hipStream_t s) {
  using T = typename Fmt<FMT>::acc_t;
  constexpr int BE = sym_epi_blocks(D);
  const size_t lds = (size_t)waves * a.H * D * sizeof(T);
  hipLaunchKernelGGL((sym_tile_kernel<FMT, D, R, U>), dim3(a.nchunks, a.nstrips), dim3(kWave * waves), lds,
                     s, a, static_cast<const T *>(a.X_in));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == 0) {
    hipLaunchKernelGGL((sym_epilogue_kernel<FMT, D, BE, 0>), dim3(sa.num_panels), dim3(256), 0, s, a, sa);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((stream_finish_kernel<T, D, 0>), dim3(1), dim3(256), 0, s, sa);
  } else {
    hipLaunchKernelGGL((sym_epilogue_kernel<FMT, D, BE, 1>), dim3(sa.num_panels), dim3(256), 0, s, a, sa);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((stream_finish_kernel<T, D, 1>), dim3(1), dim3(256), 0, s, sa);
  }
  return hipGetLastError();
}

// Dispatch over the compiled (d, R, U) shapes for one format.
template <int FMT>
hipError_t sym_launch_fmt(int d, int rows, int unroll, const SymArgs &a, const StreamArgs &sa, int waves,
                          int mode, hipStream_t s) {
#define NSRGS_SYM_CASE(DD, RR, UU) \
  if (d == DD && rows == RR && unroll == UU) return sym_launch_shape<FMT, DD, RR, UU>(a, sa, waves, mode, s);
  NSRGS_SYM_SHAPES(NSRGS_SYM_CASE)
#undef NSRGS_SYM_CASE
  return hipErrorInvalidValue;
}

}  // namespace nsrgs
