// The incomplete observation model (Sec. 4.1): each off-diagonal block pair
// (i, j) is observed with probability p, and A_ij = 0 otherwise; the iteration
// is Algorithm 2 on that A with mu = 1/(np).  Only observed blocks are stored
// (block-sparse rows), so an iteration reads about p of the dense bytes.
//
// Storage (nsrgs_bsr_matrix): block row i holds m_i = row_ptr[i+1] - row_ptr[i]
// blocks with ascending block columns col_idx[row_ptr[i] ..].  Its blocks are
// grouped by 64: group g = k / 64 holds w_g = min(64, m_i - 64 g) blocks,
// entry-major, so entry (a, b) of the k-th block is at
//     values[row_ptr[i] d^2 + 64 g d^2 + (a d + b) w_g + k mod 64].
// The loads of one entry over a group's blocks are one contiguous read, and
// a group's d^2 entries are one contiguous run of memory.
//
// Generator: the same elements as nsrgs_generate_measurement with the same
// observation mask, in three launches (count per block row, prefix sum, fill).
// Step: one wave per block row; lane l takes the row's blocks l, l + 64, ...,
// accumulates A_ij X_j (X_j, d x d, read from cache), the wave sums the d x d
// partials, and the workgroup runs the per-block epilogue of sync_step.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "host.h"
#include "kernels.h"
#include "nsrgs.h"
#include "stream_impl.h"

namespace nsrgs {
namespace {

// Offset of entry e of the k-th block of a block row of m blocks, from the
// row's first value (the grouped layout above).
__host__ __device__ __forceinline__ int64_t bsr_entry_off(int64_t k, int e, int64_t m, int d2) {
  const int64_t g0 = k & ~(int64_t)63, w = (m - g0) < 64 ? (m - g0) : 64;
  return g0 * d2 + (int64_t)e * w + (k & 63);
}

constexpr int kBsrRowsPerGroup = 4;   // block rows (waves) per step workgroup
constexpr int kBsrStepMaxD = 8;       // the fused one-wave-per-row step kernel
constexpr int kBsrMaxD = 32;          // storage, generator, and the step / solve through the wide epilogue

// Observation indicator of block pair (bi, bj), bi != bj: the generator's mask.
__device__ __forceinline__ bool observed(int bi, int bj, double p, uint32_t k0, uint32_t k1) {
  if (p >= 1.0) return true;
  const uint32_t blo = (uint32_t)(bi < bj ? bi : bj), bhi = (uint32_t)(bi < bj ? bj : bi);
  const U4 o = philox4x32_10(U4{bhi, blo, 1u, 0u}, k0, k1);
  return (double)o.x * 0x1p-32 < p;
}

// One workgroup per block row: number of observed off-diagonal blocks.
__global__ void __launch_bounds__(256)
bsr_count_kernel(int n, double p, uint32_t k0, uint32_t k1, int64_t *counts) {
  __shared__ double s_scr[kMaxWaves];
  const int i = blockIdx.x;
  double c = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) c += (j != i && observed(i, j, p, k0, k1)) ? 1.0 : 0.0;
  c = block_sum(c, s_scr);
  if (threadIdx.x == 0) counts[i] = (int64_t)c;
}

// One workgroup: exclusive prefix sum of n counts into row_ptr[0 .. n].
__global__ void __launch_bounds__(1024) bsr_scan_kernel(int n, const int64_t *counts, int64_t *row_ptr) {
  __shared__ int64_t s_part[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (n + T - 1) / T;
  const int b = t * per, e = min(n, b + per);
  int64_t s = 0;
  for (int i = b; i < e; ++i) s += counts[i];
  s_part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int u = 0; u < T; ++u) {
      const int64_t v = s_part[u];
      s_part[u] = run;
      run += v;
    }
    row_ptr[n] = run;
  }
  __syncthreads();
  int64_t run = s_part[t];
  for (int i = b; i < e; ++i) {
    row_ptr[i] = run;
    run += counts[i];
  }
}

template <typename T>
__device__ __forceinline__ T store_elem(double v);
template <>
__device__ __forceinline__ float store_elem<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ uint16_t store_elem<uint16_t>(double v) {
  // FP32 first, then BF16 round-to-nearest-even: the dense BF16 conversion's rounding
  const uint32_t u = __float_as_uint((float)v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7fc0u);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)(((u + 0x7fffu + lsb) >> 16) & 0xffffu);
}

// One workgroup per block row: the observed blocks' columns in ascending
// order (a ballot-based compaction of each 256-column stretch) and their
// elements, A_ij[a][b] = (Z Z^T)_rc + sigma W_rc with r = i d + a, c = j d + b.
template <typename T>
__global__ void __launch_bounds__(256)
bsr_fill_kernel(const double *__restrict__ Z, int n, int d, double sigma, double p, uint32_t k0, uint32_t k1,
                const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, T *__restrict__ values) {
  __shared__ int s_wave[kMaxWaves];
  __shared__ double zi[kBsrMaxD * kBsrMaxD];
  const int i = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave, nw = blockDim.x / kWave;
  const int64_t base = row_ptr[i];
  const int64_t m = row_ptr[i + 1] - base;
  const int d2 = d * d;
  for (int e = tid; e < d2; e += blockDim.x) zi[e] = Z[(int64_t)i * d2 + e];
  __syncthreads();
  int64_t done = 0;
  for (int j0 = 0; j0 < n; j0 += blockDim.x) {
    const int j = j0 + tid;
    const bool keep = j < n && j != i && observed(i, j, p, k0, k1);
    const uint64_t bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
      off += w < wave ? s_wave[w] : 0;
      tot += s_wave[w];
    }
    if (keep) {
      const int64_t k = done + off + before;
      col_idx[base + k] = j;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          const int r = i * d + a, c = j * d + b;
          double v = 0.0;
          for (int q = 0; q < d; ++q) v = fma(zi[a * d + q], Z[(int64_t)c * d + q], v);
          if (sigma != 0.0) {
            const uint32_t lo = (uint32_t)(r < c ? r : c), hi = (uint32_t)(r < c ? c : r);
            v += sigma * normal_from(philox4x32_10(U4{hi, lo, 0u, 0u}, k0, k1));
          }
          values[base * d2 + bsr_entry_off(k, a * d + b, m, d2)] = store_elem<T>(v);
        }
    }
    done += tot;
    __syncthreads();
  }
}

// Loads of the streamed arrays (values, column indices): non-temporal (NT) or
// ordinary.  An entry's 64-element run rarely starts on a cache line, so
// consecutive chunks of a block row share a line at each run's ends; an
// ordinary load keeps that line for the next chunk.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename E, bool NT>
__device__ __forceinline__ float load_elem(const E *p) {
  if constexpr (sizeof(E) == 4) return ld_stream<NT>(p);
  else return __uint_as_float((uint32_t)ld_stream<NT>(p) << 16);
}

// One wave per block row, kBsrRowsPerGroup block rows per workgroup.  Lane l
// takes the row's blocks k0 + l + 64 u (u < UN) of each chunk of 64 UN; the
// next chunk's column indices are loaded while this chunk's X_j gathers and
// products run, so the index -> gather dependence does not stall every chunk.
template <typename E, int D, bool NT, int UN>
__global__ void __launch_bounds__(kWave * kBsrRowsPerGroup)
bsr_step_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                const E *__restrict__ values, StreamArgs sa) {
  constexpr int D2 = D * D;
  constexpr int NB = kBsrRowsPerGroup;
  constexpr int NE = NB * D2;
  constexpr int CH = kWave * UN;
  __shared__ double s_scr[kMaxWaves];
  __shared__ float sbuf[6 * NE];
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int n = sa.n;
  const int i = blockIdx.x * NB + wave;                 // this wave's block row
  const int ic = i < n ? i : n - 1;
  const float *__restrict__ X = static_cast<const float *>(sa.X_in);
  const int64_t base = row_ptr[ic];
  const int64_t m = i < n ? row_ptr[ic + 1] - base : 0;   // wave-uniform
  const E *__restrict__ vals = values + base * D2;
  const int32_t *__restrict__ cols = col_idx + base;
  float acc[D2];
#pragma unroll
  for (int e = 0; e < D2; ++e) acc[e] = 0.0f;
  int jr_next[UN];
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t k = (int64_t)u * kWave + lane;
    jr_next[u] = m > 0 ? ld_stream<NT>(cols + (k < m ? k : m - 1)) : 0;
  }
  for (int64_t k0 = 0; k0 < m; k0 += CH) {
    int jr[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) jr[u] = jr_next[u];
    float a[UN][D2], x[UN][D2];
    bool use[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int64_t k = k0 + (int64_t)u * kWave + lane;
      const bool ok = k < m;
      const int64_t kc = ok ? k : m - 1;                // clamped: in-bounds, masked below
#pragma unroll
      for (int e = 0; e < D2; ++e) a[u][e] = load_elem<E, NT>(vals + bsr_entry_off(kc, e, m, D2));
      const int j = jr[u] < 0 ? 0 : (jr[u] < n ? jr[u] : n - 1);   // out-of-range indices read in bounds
      use[u] = ok && jr[u] == j && j != ic;             // and, like a stored diagonal block, count 0
#pragma unroll
      for (int e = 0; e < D2; ++e) x[u][e] = X[(int64_t)j * D2 + e];
    }
    if (k0 + CH < m) {                                  // wave-uniform
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const int64_t k = k0 + CH + (int64_t)u * kWave + lane;
        jr_next[u] = ld_stream<NT>(cols + (k < m ? k : m - 1));
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < UN; ++u) {
#pragma unroll
      for (int e = 0; e < D2; ++e) a[u][e] = use[u] ? a[u][e] : 0.0f;
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int b = 0; b < D; ++b)
#pragma unroll
          for (int c = 0; c < D; ++c) acc[r * D + c] = fmaf(a[u][r * D + b], x[u][b * D + c], acc[r * D + c]);
    }
  }
  float *sX = sbuf, *sC = sX + NE, *sG = sC + NE, *sT = sG + NE, *sF = sT + NE, *sM = sF + NE;
#pragma unroll
  for (int e = 0; e < D2; ++e) {
    const float v = wave_sum(acc[e]);
    if (lane == 0) sC[wave * D2 + e] = i < n ? v : 0.0f;
  }
  for (int e = lane; e < D2; e += kWave) sX[wave * D2 + e] = i < n ? X[(int64_t)ic * D2 + e] : 0.0f;
  __syncthreads();
  block_step_epilogue<float, D, NB>(n, sa.mu, sa.ns_steps, sa.nd, blockIdx.x * NB * D,
                                    static_cast<float *>(sa.X_out),
                                    static_cast<PanelStat *>(sa.partials) + blockIdx.x, sX, sC, sG, sT, sF, sM,
                                    s_scr);
}

// ---------------------------------------------------------------------------
// Sliced step (d <= 8).  The fused kernel above gathers X_j from the caches
// for every block; at the benchmark's size those gathers (36 B of scattered
// lines per 40 B of streamed A) cost as much cache bandwidth as the stream.
// Here the block columns are cut into slices of W blocks whose X fills 128
// KiB of LDS, and a workgroup (slice s, a group of 64 block rows, one per CU)
// loads X of its slice into LDS once, then streams its rows' blocks with
// columns in the slice (a contiguous range of each row, col_idx being
// ascending) and gathers X_j from LDS.  Each of its 16 waves takes 4 rows one
// after the other, with the next chunk of 64 blocks (the next row's first
// at a row's end) in flight while the current one is used.  Per-(slice, row)
// partial sums go to the workspace; an epilogue kernel adds them in slice
// order and runs the per-block step.  The row ranges of the slices come from
// a binary search per (slice, row).
// ---------------------------------------------------------------------------
constexpr int kBsrSliceBytes = 131072;
constexpr int kBsrSliceMaxD = 6;          // d >= 7 needs more registers than 8 waves per CU leave: fused kernel
constexpr int kBsrSliceRPW = 4;           // block rows per wave
// Waves per workgroup: 16 while a wave's chunk, X slice and sums fit 128
// VGPRs (d <= 4), else 8.
__host__ __device__ constexpr int bsr_slice_waves(int d) { return d <= 4 ? 16 : 8; }

__host__ __device__ constexpr int bsr_xs(int d) { return (d * d + 3) / 4 * 4; }   // floats per X_j in LDS
// Slice width in blocks: what the LDS slice holds, or less with NSRGS_BSR_SLICE_W.
inline int bsr_slice_w(int d) {
  const int w = kBsrSliceBytes / (4 * bsr_xs(d)), f = env_int("NSRGS_BSR_SLICE_W", 0);
  return (f > 0 && f < w) ? f : w;
}
inline int bsr_slices(int n, int d) { return (n + bsr_slice_w(d) - 1) / bsr_slice_w(d); }

// bounds[s n + i] = first k of block row i with col_idx >= s W, s = 0 .. S:
// one thread per (s, i).  The row's columns ascend over [0, n), so the entry
// sits near m s W / n when the stored blocks spread evenly (as the mask's do);
// the search probes that guess, gallops away from it in steps of 32, 64, ...
// entries until the answer is bracketed, and bisects the bracket.  The result
// is the unique first index whatever the spread (an uneven row costs only
// more gallop steps); about four cache lines per search against ten to
// fourteen for a bisection of the whole row.  (Searching all of a row's keys
// with one wave, each round probing 64 positions per key, measured three
// times slower: most probes are wasted.)
__global__ void __launch_bounds__(256)
bsr_bounds_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx, int n, int S, int W,
                  int32_t *__restrict__ bounds) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)(S + 1) * n) return;
  const int s = (int)(t / n), i = (int)(t % n);
  const int64_t base = row_ptr[i];
  const int64_t m = row_ptr[i + 1] - base;
  const int64_t key = (int64_t)s * W;
  const int32_t *__restrict__ c = col_idx + base;
  int64_t lo, hi;                                   // the answer lies in [lo, hi]
  if (m <= 0 || key <= 0) {
    lo = hi = 0;
  } else if (key >= n) {
    lo = hi = m;
  } else {
    const int64_t g = m * key / n;                  // < m
    if (c[g] < key) {                               // answer in (g, m]: gallop up
      lo = g + 1;
      hi = m;
      for (int64_t step = 32;; step *= 2) {
        const int64_t q = g + step;
        if (q >= m) break;
        if (c[q] >= key) { hi = q; break; }
        lo = q + 1;
      }
    } else {                                        // answer in [0, g]: gallop down
      lo = 0;
      hi = g;
      for (int64_t step = 32;; step *= 2) {
        const int64_t q = g - step;
        if (q < 0) break;
        if (c[q] < key) { lo = q + 1; break; }
        hi = q;
      }
    }
  }
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (c[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  bounds[t] = (int32_t)lo;
}

// One chunk of 64 UN blocks of a row: lane l's blocks k = k0 + l + 64 u
// (clamped to the row's range in this slice), their column indices and d^2
// values.  Buffer loads: the row's arrays are buffer resources (wave-uniform),
// the entry offset e m is a scalar offset and the lane's block offset the only
// per-lane address, so no per-lane 64-bit address arithmetic.  (The host runs
// this kernel only when a row's values span less than 2^31 bytes.)
struct BsrRow {
  __amdgpu_buffer_rsrc_t vals, cols;
  int64_t m;
};

template <typename E>
__device__ __forceinline__ BsrRow bsr_row(const E *values, const int32_t *col_idx, int64_t base, int64_t m, int d2) {
  // word 3 of a raw buffer resource on this GPU family; num_records in bytes
  // (loads past it read 0)
  constexpr int kRaw = 0x00020000;
  BsrRow r;
  r.vals = __builtin_amdgcn_make_buffer_rsrc((void *)(values + base * d2), (short)0,
                                             (int)(m * d2 * (int64_t)sizeof(E)), kRaw);
  r.cols = __builtin_amdgcn_make_buffer_rsrc((void *)(col_idx + base), (short)0, (int)(m * 4), kRaw);
  r.m = m;
  return r;
}

template <typename E, bool NT>
__device__ __forceinline__ float bsr_buf_elem(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  constexpr int aux = NT ? 2 : 0;                       // bit 1: non-temporal
  if constexpr (sizeof(E) == 4)
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, aux));
  else
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, aux) << 16);
}

template <typename E, int D, bool NT, int UN>
__device__ __forceinline__ void bsr_chunk_load(const BsrRow &row, int64_t k0, int64_t hi, int lane,
                                               float (&a)[UN][D * D], int (&jr)[UN]) {
  constexpr int aux = NT ? 2 : 0;
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t k = k0 + u * kWave + lane;
    const int kc = (int)(k < hi ? k : hi - 1);
    jr[u] = (int)__builtin_amdgcn_raw_buffer_load_b32(row.cols, kc * 4, 0, aux);
    // entry e of block kc: group start 64 g d^2 + k mod 64, then e w_g
    const int g0 = kc & ~63;
    const int w = (int)(row.m - g0 < 64 ? row.m - g0 : 64);
    int off = (g0 * (D * D) + (kc & 63)) * (int)sizeof(E);
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
      a[u][e] = bsr_buf_elem<E, NT>(row.vals, off, 0);
      off += w * (int)sizeof(E);
    }
  }
}

template <typename E, int D, bool NT, int UN, int NW, int MINW = 1>
__global__ void __launch_bounds__(kWave * NW, MINW)
bsr_slice_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                 const E *__restrict__ values, const int32_t *__restrict__ bounds, const float *__restrict__ X,
                 int n, int W, float *__restrict__ part, const int *stop_flag) {
  constexpr int D2 = D * D, XS = bsr_xs(D), XQ = XS / 4, RPW = kBsrSliceRPW, CH = kWave * UN;
  constexpr int ROWS = NW * kBsrSliceRPW;
  extern __shared__ float4 sX4[];
  if (stop_flag) {
    if (__atomic_load_n(stop_flag, __ATOMIC_RELAXED)) return;   // uniform: a solve has stopped
  }
  float *sXf = reinterpret_cast<float *>(sX4);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int g = blockIdx.x, s = blockIdx.y;
  const int j0 = s * W, jn = min(W, n - j0);
  // this wave's rows (wave-uniform), read while the slice of X is staged
  BsrRow row[RPW];
  int64_t rlo[RPW], rhi[RPW];
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = g * ROWS + q * NW + wave;
    const int ic = i < n ? i : n - 1;
    const int64_t b = row_ptr[ic];
    row[q] = bsr_row<E>(values, col_idx, b, row_ptr[ic + 1] - b, D2);
    rlo[q] = bounds[(int64_t)s * n + ic];
    rhi[q] = i < n ? bounds[(int64_t)(s + 1) * n + ic] : rlo[q];   // rows past n have no blocks
  }
  // the first chunk is in flight while the slice of X is staged
  float an[UN][D2];
  int jn_next[UN];
  bool have = false;                                    // wave-uniform: a chunk is in flight
  if (rhi[0] > rlo[0]) {
    bsr_chunk_load<E, D, NT, UN>(row[0], rlo[0], rhi[0], lane, an, jn_next);
    have = true;
  }
  for (int idx = tid; idx < jn * XS; idx += blockDim.x) {
    const int jl = idx / XS, e = idx % XS;
    sXf[idx] = e < D2 ? X[(int64_t)(j0 + jl) * D2 + e] : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = g * ROWS + q * NW + wave;
    float acc[D2];
#pragma unroll
    for (int e = 0; e < D2; ++e) acc[e] = 0.0f;
    if (!have && rhi[q] > rlo[q]) {                     // wave-uniform
      bsr_chunk_load<E, D, NT, UN>(row[q], rlo[q], rhi[q], lane, an, jn_next);
      have = true;
    }
    for (int64_t k0 = rlo[q]; k0 < rhi[q]; k0 += CH) {
      float a[UN][D2];
      int jr[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        jr[u] = jn_next[u];
#pragma unroll
        for (int e = 0; e < D2; ++e) a[u][e] = an[u][e];
      }
      have = false;
      if (k0 + CH < rhi[q]) {                           // wave-uniform: the row's next chunk in flight
        bsr_chunk_load<E, D, NT, UN>(row[q], k0 + CH, rhi[q], lane, an, jn_next);
        have = true;
      } else if (q + 1 < RPW) {
        if (rhi[q + 1] > rlo[q + 1]) {                  // or the next row's first
          bsr_chunk_load<E, D, NT, UN>(row[q + 1], rlo[q + 1], rhi[q + 1], lane, an, jn_next);
          have = true;
        }
      }
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        const bool ok = k0 + u * kWave + lane < rhi[q];
        const int jl = jr[u] - j0;
        const bool inside = jl >= 0 && jl < jn;         // ascending columns keep every stored one inside
        const bool use = ok && inside && jr[u] != i;
        const int jlc = inside ? jl : 0;
        float x[XS];
#pragma unroll
        for (int qq = 0; qq < XQ; ++qq) {
          const float4 v = sX4[jlc * XQ + qq];
          x[4 * qq] = v.x;
          x[4 * qq + 1] = v.y;
          x[4 * qq + 2] = v.z;
          x[4 * qq + 3] = v.w;
        }
#pragma unroll
        for (int e = 0; e < D2; ++e) a[u][e] = use ? a[u][e] : 0.0f;
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int b = 0; b < D; ++b)
#pragma unroll
            for (int c = 0; c < D; ++c) acc[r * D + c] = fmaf(a[u][r * D + b], x[b * D + c], acc[r * D + c]);
      }
    }
    // the row's d^2 sums over the wave by the transpose-reduce (a few shuffles
    // instead of six per entry); lanes holding the same entry hold equal sums
    wave_tr_step<float, D2, 0>(acc, lane);
    if (i < n) part[((int64_t)s * n + i) * D2 + wave_tr_entry<D2>(lane)] = acc[0];
  }
}

// C_i = the slices' partial sums in slice order, then the per-block step, for
// kBsrSliceEpiBlocks blocks per workgroup.
constexpr int kBsrSliceEpiBlocks = 16;
template <int D>
__global__ void __launch_bounds__(256)
bsr_slice_epilogue_kernel(const float *__restrict__ part, int S, StreamArgs sa) {
  constexpr int D2 = D * D;
  constexpr int NB = kBsrSliceEpiBlocks;
  constexpr int NE = NB * D2;
  __shared__ double s_scr[kMaxWaves];
  __shared__ float sbuf[6 * NE];
  if (sa.stop_flag) {
    if (__atomic_load_n(sa.stop_flag, __ATOMIC_RELAXED)) return;   // uniform: a solve has stopped
  }
  const int tid = threadIdx.x, n = sa.n;
  const float *__restrict__ X = static_cast<const float *>(sa.X_in);
  float *sX = sbuf, *sC = sX + NE, *sG = sC + NE, *sT = sG + NE, *sF = sT + NE, *sM = sF + NE;
  for (int t = tid; t < NE; t += blockDim.x) {
    const int i = blockIdx.x * NB + t / D2, e = t % D2;
    float c = 0.0f;
    if (i < n)
      for (int s = 0; s < S; ++s) c += part[((int64_t)s * n + i) * D2 + e];
    sC[t] = c;
    sX[t] = i < n ? X[(int64_t)i * D2 + e] : 0.0f;
  }
  __syncthreads();
  block_step_epilogue<float, D, NB>(n, sa.mu, sa.ns_steps, sa.nd, blockIdx.x * NB * D,
                                    static_cast<float *>(sa.X_out),
                                    static_cast<PanelStat *>(sa.partials) + blockIdx.x, sX, sC, sG, sT, sF, sM,
                                    s_scr);
}

hipError_t bsr_bounds_launch(const nsrgs_bsr_matrix &A, int n, int d, int32_t *bounds, hipStream_t s) {
  const int W = bsr_slice_w(d), S = bsr_slices(n, d);
  const int64_t nb = (int64_t)(S + 1) * n;
  hipLaunchKernelGGL(bsr_bounds_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, A.row_ptr, A.col_idx,
                     n, S, W, bounds);
  return hipGetLastError();
}

// The sliced product: part[s n + i] = slice s's share of block row i's
// C_i, from the bounds table of bsr_bounds_launch.
template <typename E, int D>
hipError_t bsr_slice_product_d(const nsrgs_bsr_matrix &A, int n, const float *Xf, const int32_t *bounds,
                               float *part, const int *stop_flag, hipStream_t s) {
  const int W = bsr_slice_w(D), S = bsr_slices(n, D);
  const size_t lds = (size_t)W * bsr_xs(D) * sizeof(float);
  const E *vals = static_cast<const E *>(A.values);
  // Load hint (NSRGS_BSR_NT, default ordinary loads: a chunk's first and last
  // cache lines are shared with its neighbours) and chunk size
  // (NSRGS_BSR_UN = 1, 2 or 4 blocks per lane, 2 and 4 for d <= 3 only; one by
  // default: two measured the same at p = 0.5 and slower at p = 0.2, four
  // needs 8 waves per CU and was slower).
  const bool nt = env_int("NSRGS_BSR_NT", 0) != 0;
  const int fu = env_int("NSRGS_BSR_UN", 1);
  const int un = D <= 3 && (fu == 2 || fu == 4) ? fu : 1;
#define NSRGS_BSR_SLICE(NTV, UNV, NWV, MINW)                                                               \
  {                                                                                                          \
    static const bool ok_ = hipFuncSetAttribute((const void *)bsr_slice_kernel<E, D, NTV, UNV, NWV, MINW>,   \
                                                hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                                kBsrSliceBytes) == hipSuccess;                               \
    if (!ok_) return hipErrorInvalidConfiguration;                                                         \
    const dim3 grid_((n + NWV * kBsrSliceRPW - 1) / (NWV * kBsrSliceRPW), S);                                \
    hipLaunchKernelGGL((bsr_slice_kernel<E, D, NTV, UNV, NWV, MINW>), grid_, dim3(kWave * NWV), lds, s,      \
                       A.row_ptr, A.col_idx, vals, bounds, Xf, n, W, part, stop_flag);                       \
  }
  // (more than 64 KiB of dynamic LDS has to be allowed per kernel, once)
  constexpr int NW1 = bsr_slice_waves(D);
  if (un == 4) {
    if constexpr (D <= 3) {
      if (nt) NSRGS_BSR_SLICE(true, 4, 8, 1) else NSRGS_BSR_SLICE(false, 4, 8, 1)
    }
  } else if (un == 2) {
    if constexpr (D <= 3) {
      if (nt) NSRGS_BSR_SLICE(true, 2, 16, 1) else NSRGS_BSR_SLICE(false, 2, 16, 1)
    }
  } else {
    if (nt) NSRGS_BSR_SLICE(true, 1, NW1, 1) else NSRGS_BSR_SLICE(false, 1, NW1, 1)
  }
#undef NSRGS_BSR_SLICE
  return hipGetLastError();
}

// One sliced step: the bounds (unless a solve found them already), the
// product, the epilogue and the monitor finish; sa.stop_flag (a solve's) ends
// every launch at once after the stop rule has fired.
template <typename E, int D>
hipError_t bsr_slice_launch_d(const nsrgs_bsr_matrix &A, const StreamArgs &sa, int32_t *bounds, float *part,
                              bool find_bounds, hipStream_t s) {
  const int n = sa.n, S = bsr_slices(n, D);
  hipError_t e;
  if (find_bounds && (e = bsr_bounds_launch(A, n, D, bounds, s)) != hipSuccess) return e;
  if ((e = bsr_slice_product_d<E, D>(A, n, static_cast<const float *>(sa.X_in), bounds, part, sa.stop_flag, s)) !=
      hipSuccess)
    return e;
  StreamArgs se = sa;
  se.num_panels = (n + kBsrSliceEpiBlocks - 1) / kBsrSliceEpiBlocks;
  hipLaunchKernelGGL((bsr_slice_epilogue_kernel<D>), dim3(se.num_panels), dim3(256), 0, s, part, S, se);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((stream_finish_kernel<float, D, 0>), dim3(1), dim3(256), 0, s, se);
  return hipGetLastError();
}

// C_i for the matrix-core path's epilogue: P[(i d + a) 32 + c] = the slices'
// partial sums of entry (a, c) in slice order (the order of the sliced step).
template <int D>
__global__ void __launch_bounds__(256)
bsr_slice_to_wide_kernel(const float *__restrict__ part, int S, int n, float *__restrict__ P, const int *stop_flag) {
  constexpr int D2 = D * D;
  if (stop_flag) {
    if (__atomic_load_n(stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * D2) return;
  const int i = (int)(t / D2), e = (int)(t % D2);
  float c = 0.0f;
  for (int s = 0; s < S; ++s) c += part[((int64_t)s * n + i) * D2 + e];
  P[((int64_t)i * D + e / D) * 32 + e % D] = c;
}

template <typename E, int D>
hipError_t bsr_slice_wide_d(const nsrgs_bsr_matrix &A, int n, const float *X, const int32_t *bounds, float *part,
                            float *P, const int *stop_flag, hipStream_t s) {
  hipError_t e = bsr_slice_product_d<E, D>(A, n, X, bounds, part, stop_flag, s);
  if (e != hipSuccess) return e;
  const int64_t nt = (int64_t)n * D * D;
  hipLaunchKernelGGL((bsr_slice_to_wide_kernel<D>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, part,
                     bsr_slices(n, D), n, P, stop_flag);
  return hipGetLastError();
}

template <typename E>
hipError_t bsr_slice_launch(int d, const nsrgs_bsr_matrix &A, const StreamArgs &sa, int32_t *bounds, float *part,
                            bool find_bounds, hipStream_t s) {
  switch (d) {
    case 1: return bsr_slice_launch_d<E, 1>(A, sa, bounds, part, find_bounds, s);
    case 2: return bsr_slice_launch_d<E, 2>(A, sa, bounds, part, find_bounds, s);
    case 3: return bsr_slice_launch_d<E, 3>(A, sa, bounds, part, find_bounds, s);
    case 4: return bsr_slice_launch_d<E, 4>(A, sa, bounds, part, find_bounds, s);
    case 5: return bsr_slice_launch_d<E, 5>(A, sa, bounds, part, find_bounds, s);
    case 6: return bsr_slice_launch_d<E, 6>(A, sa, bounds, part, find_bounds, s);
    default: return hipErrorInvalidValue;
  }
}

// Workspace of the sliced product: everything sync_workspace_bytes covers (the
// sync_step part and the matrix-core region a solve uses), then the slice
// bounds and the partial sums.
size_t bsr_slice_table_off(int n, int d) { return sync_workspace_bytes(n, d, NSRGS_A_F32); }
size_t bsr_slice_part_off(int n, int d) {
  return bsr_slice_table_off(n, d) + align256((size_t)(bsr_slices(n, d) + 1) * n * sizeof(int32_t));
}
size_t bsr_slice_ws_bytes(int n, int d) {
  return bsr_slice_part_off(n, d) + align256((size_t)bsr_slices(n, d) * n * d * d * sizeof(float));
}

// The product of block-sparse A with X for the matrix-core path's epilogue
// (any d <= 32): P[(i d + a) 32 + c] = sum over stored j != i of (A_ij X_j)[a][c],
// and the sum of squares of block row i's stored off-diagonal values into
// sumsq[i] (for the objective's constant).  One workgroup per block row.  The
// row's blocks go through LDS in chunks of KB: the values entry by entry (entry
// e of the chunk's blocks is KB consecutive elements of the entry-major
// layout), X_j of each block alongside.  Thread (g, c) accumulates column c of
// rows g, g + 8, g + 16, g + 24.  A stored diagonal block or a column index
// outside [0, n) contributes nothing (its values and X_j are staged as zeros).
template <typename E>
__global__ void __launch_bounds__(256)
bsr_wide_product_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                        const E *__restrict__ values, int n, int d, int KB, const float *__restrict__ X,
                        float *__restrict__ P, double *__restrict__ sumsq, const int *stop_flag) {
  extern __shared__ float s_dyn[];
  __shared__ double s_scr[kMaxWaves];
  if (stop_flag) {
    if (__atomic_load_n(stop_flag, __ATOMIC_RELAXED)) return;   // uniform
  }
  const int i = blockIdx.x, tid = threadIdx.x, dd = d * d;
  const int c = tid & 31, g = tid >> 5;
  const int cc = c < d ? c : 0;
  float *sA = s_dyn, *sX = s_dyn + KB * dd;
  const int64_t base = row_ptr[i];
  const int64_t m = row_ptr[i + 1] - base;
  const E *__restrict__ vals = values + base * dd;
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  int ar[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) ar[r] = (g + 8 * r) < d ? g + 8 * r : 0;   // clamped rows, results dropped
  double ssq = 0.0;
  for (int64_t k0 = 0; k0 < m; k0 += KB) {
    const int kb = (int)((m - k0) < KB ? (m - k0) : KB);
    for (int idx = tid; idx < KB * dd; idx += blockDim.x) {
      const int e = idx / KB, kk = idx % KB;
      const int kkc = kk < kb ? kk : kb - 1;
      const int jr = col_idx[base + k0 + kkc];
      const bool use = kk < kb && jr >= 0 && jr < n && jr != i;
      const float v = load_elem<E, true>(vals + bsr_entry_off(k0 + kkc, e, m, dd));
      const float va = use ? v : 0.0f;
      sA[kk * dd + e] = va;
      ssq += (double)va * (double)va;
    }
    for (int idx = tid; idx < KB * dd; idx += blockDim.x) {
      const int kk = idx / dd, e = idx % dd;
      const int kkc = kk < kb ? kk : kb - 1;
      const int jr = col_idx[base + k0 + kkc];
      const bool use = kk < kb && jr >= 0 && jr < n && jr != i;
      const int j = jr < 0 ? 0 : (jr < n ? jr : n - 1);
      const float x = X[(int64_t)j * dd + e];
      sX[kk * dd + e] = use ? x : 0.0f;
    }
    __syncthreads();
    for (int kk = 0; kk < kb; ++kk) {
      const float *a = sA + kk * dd, *x = sX + kk * dd;
      for (int b = 0; b < d; ++b) {
        const float xb = x[b * d + cc];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = fmaf(a[ar[r] * d + b], xb, acc[r]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int a = g + 8 * r;
    if (a < d && c < d) P[((int64_t)i * d + a) * 32 + c] = acc[r];
  }
  ssq = block_sum(ssq, s_scr);
  if (tid == 0 && sumsq) sumsq[i] = ssq;
}

// Load hint and blocks per lane per chunk: NSRGS_BSR_NT (1: non-temporal
// loads of the streamed arrays), NSRGS_BSR_UN (2: two blocks per lane, d <= 4).
template <typename E, int D>
hipError_t bsr_launch_d(const nsrgs_bsr_matrix &A, const StreamArgs &sa, hipStream_t s) {
  const bool nt = env_int("NSRGS_BSR_NT", 1) != 0;
  const int un = (D <= 4 && env_int("NSRGS_BSR_UN", 1) == 2) ? 2 : 1;
  const dim3 grid(sa.num_panels), block(kWave * kBsrRowsPerGroup);
  const E *vals = static_cast<const E *>(A.values);
  if (un == 2) {
    if constexpr (D <= 4) {
      if (nt) hipLaunchKernelGGL((bsr_step_kernel<E, D, true, 2>), grid, block, 0, s, A.row_ptr, A.col_idx, vals, sa);
      else hipLaunchKernelGGL((bsr_step_kernel<E, D, false, 2>), grid, block, 0, s, A.row_ptr, A.col_idx, vals, sa);
    }
  } else {
    if (nt) hipLaunchKernelGGL((bsr_step_kernel<E, D, true, 1>), grid, block, 0, s, A.row_ptr, A.col_idx, vals, sa);
    else hipLaunchKernelGGL((bsr_step_kernel<E, D, false, 1>), grid, block, 0, s, A.row_ptr, A.col_idx, vals, sa);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((stream_finish_kernel<float, D, 0>), dim3(1), dim3(256), 0, s, sa);
  return hipGetLastError();
}

template <typename E>
hipError_t bsr_launch(int d, const nsrgs_bsr_matrix &A, const StreamArgs &sa, hipStream_t s) {
  switch (d) {
    case 1: return bsr_launch_d<E, 1>(A, sa, s);
    case 2: return bsr_launch_d<E, 2>(A, sa, s);
    case 3: return bsr_launch_d<E, 3>(A, sa, s);
    case 4: return bsr_launch_d<E, 4>(A, sa, s);
    case 5: return bsr_launch_d<E, 5>(A, sa, s);
    case 6: return bsr_launch_d<E, 6>(A, sa, s);
    case 7: return bsr_launch_d<E, 7>(A, sa, s);
    case 8: return bsr_launch_d<E, 8>(A, sa, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Launch of the block-sparse product above for the matrix-core epilogue.
hipError_t launch_bsr_wide_product(const nsrgs_bsr_matrix &A, int n, int d, const float *X, float *P,
                                   double *sumsq, const int *stop_flag, hipStream_t s) {
  const int dd = d * d;
  int KB = 8192 / dd;                       // two KB x d^2 float buffers in 64 KiB of LDS
  KB = KB > 16 ? 16 : KB;
  const size_t lds = (size_t)2 * KB * dd * sizeof(float);
  if (A.fmt == NSRGS_A_F32)
    hipLaunchKernelGGL(bsr_wide_product_kernel<float>, dim3(n), dim3(256), lds, s, A.row_ptr, A.col_idx,
                       static_cast<const float *>(A.values), n, d, KB, X, P, sumsq, stop_flag);
  else
    hipLaunchKernelGGL(bsr_wide_product_kernel<uint16_t>, dim3(n), dim3(256), lds, s, A.row_ptr, A.col_idx,
                       static_cast<const uint16_t *>(A.values), n, d, KB, X, P, sumsq, stop_flag);
  return hipGetLastError();
}

bool bsr_sliced(int n, int d, size_t ws_bytes) {
  return d <= kBsrSliceMaxD && (int64_t)n * d * d * 4 < ((int64_t)1 << 31) && ws_bytes >= bsr_slice_ws_bytes(n, d) &&
         env_int("NSRGS_BSR_SLICED", 1) != 0;
}

hipError_t launch_bsr_slice_bounds(const nsrgs_bsr_matrix &A, int n, int d, void *ws, hipStream_t s) {
  return bsr_bounds_launch(A, n, d, reinterpret_cast<int32_t *>(static_cast<char *>(ws) + bsr_slice_table_off(n, d)),
                           s);
}

template <typename E>
static hipError_t slice_wide(const nsrgs_bsr_matrix &A, int n, int d, const float *X, const int32_t *bounds,
                             float *part, float *P, const int *stop_flag, hipStream_t s) {
  switch (d) {
    case 1: return bsr_slice_wide_d<E, 1>(A, n, X, bounds, part, P, stop_flag, s);
    case 2: return bsr_slice_wide_d<E, 2>(A, n, X, bounds, part, P, stop_flag, s);
    case 3: return bsr_slice_wide_d<E, 3>(A, n, X, bounds, part, P, stop_flag, s);
    case 4: return bsr_slice_wide_d<E, 4>(A, n, X, bounds, part, P, stop_flag, s);
    case 5: return bsr_slice_wide_d<E, 5>(A, n, X, bounds, part, P, stop_flag, s);
    case 6: return bsr_slice_wide_d<E, 6>(A, n, X, bounds, part, P, stop_flag, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bsr_slice_wide_product(const nsrgs_bsr_matrix &A, int n, int d, const float *X, float *P,
                                         void *ws, const int *stop_flag, hipStream_t s) {
  char *base = static_cast<char *>(ws);
  const int32_t *bounds = reinterpret_cast<const int32_t *>(base + bsr_slice_table_off(n, d));
  float *part = reinterpret_cast<float *>(base + bsr_slice_part_off(n, d));
  return A.fmt == NSRGS_A_F32 ? slice_wide<float>(A, n, d, X, bounds, part, P, stop_flag, s)
                              : slice_wide<uint16_t>(A, n, d, X, bounds, part, P, stop_flag, s);
}

int bsr_sliced_iterate(const nsrgs_bsr_matrix &A, int n, int d, double mu, int ns_steps, const void *X_in,
                       void *X_out, void *ws, hipStream_t s, int iter, double tol) {
  StreamArgs sa{};
  sa.X_in = X_in;
  sa.X_out = X_out;
  sa.n = n;
  sa.d = d;
  sa.nd = n * d;
  sa.mu = mu > 0.0 ? mu : 1.0 / n;
  sa.ns_steps = ns_steps;
  sa.partials = static_cast<char *>(ws) + step_ws_stats_offset(n, d, NSRGS_A_F32);
  sa.ctl = static_cast<DevCtl *>(ws);
  sa.iter = iter;
  sa.tol = tol;
  sa.stop_flag = &sa.ctl->done;
  char *base = static_cast<char *>(ws);
  int32_t *bounds = reinterpret_cast<int32_t *>(base + bsr_slice_table_off(n, d));
  float *part = reinterpret_cast<float *>(base + bsr_slice_part_off(n, d));
  const hipError_t e = A.fmt == NSRGS_A_F32 ? bsr_slice_launch<float>(d, A, sa, bounds, part, false, s)
                                            : bsr_slice_launch<uint16_t>(d, A, sa, bounds, part, false, s);
  NSRGS_HIP(e, "block-sparse step launch");
  return NSRGS_OK;
}

namespace {

int bsr_common(int n, int d, double p) {
  if (n < 2) return fail(NSRGS_ERR_INVALID_ARG, "n must be >= 2 (got %d)", n);
  if (d < 1 || d > kBsrMaxD) return fail(NSRGS_ERR_UNSUPPORTED, "block-sparse storage supports 1 <= d <= %d", kBsrMaxD);
  if (!(p >= 0.0 && p <= 1.0)) return fail(NSRGS_ERR_INVALID_ARG, "p must be in [0, 1]");
  if ((int64_t)n * d * d >= (int64_t)1 << 31) return fail(NSRGS_ERR_INVALID_ARG, "n*d*d too large");
  return NSRGS_OK;
}

}  // namespace
}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

int nsrgs_bsr_count(const double *Z, int n, int d, double p, uint64_t seed, int64_t *row_ptr, void *counts,
                    int64_t *nnzb, void *stream) {
  int st;
  if ((st = bsr_common(n, d, p))) return st;
  if (!Z || !row_ptr || !counts || !nnzb) return fail(NSRGS_ERR_INVALID_ARG, "NULL pointer argument");
  hipStream_t s = (hipStream_t)stream;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(bsr_count_kernel, dim3(n), dim3(256), 0, s, n, p, k0, k1, static_cast<int64_t *>(counts));
  NSRGS_HIP(hipGetLastError(), "bsr count launch");
  hipLaunchKernelGGL(bsr_scan_kernel, dim3(1), dim3(1024), 0, s, n, static_cast<const int64_t *>(counts), row_ptr);
  NSRGS_HIP(hipGetLastError(), "bsr scan launch");
  NSRGS_HIP(hipMemcpyAsync(nnzb, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s), "nnzb copy");
  NSRGS_HIP(hipStreamSynchronize(s), "stream sync");
  return NSRGS_OK;
}

int nsrgs_bsr_fill(const double *Z, int n, int d, double sigma, double p, uint64_t seed, const nsrgs_bsr_matrix *A,
                   void *stream) {
  int st;
  if ((st = bsr_common(n, d, p))) return st;
  if (!Z || !A || !A->row_ptr || !A->col_idx || !A->values) return fail(NSRGS_ERR_INVALID_ARG, "NULL pointer argument");
  if (!std::isfinite(sigma)) return fail(NSRGS_ERR_INVALID_ARG, "sigma must be finite");
  hipStream_t s = (hipStream_t)stream;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (A->fmt == NSRGS_A_F32)
    hipLaunchKernelGGL(bsr_fill_kernel<float>, dim3(n), dim3(256), 0, s, Z, n, d, sigma, p, k0, k1, A->row_ptr,
                       const_cast<int32_t *>(A->col_idx), (float *)A->values);
  else if (A->fmt == NSRGS_A_BF16)
    hipLaunchKernelGGL(bsr_fill_kernel<uint16_t>, dim3(n), dim3(256), 0, s, Z, n, d, sigma, p, k0, k1, A->row_ptr,
                       const_cast<int32_t *>(A->col_idx), (uint16_t *)A->values);
  else
    return fail(NSRGS_ERR_UNSUPPORTED, "block-sparse values must be F32 or BF16");
  NSRGS_HIP(hipGetLastError(), "bsr fill launch");
  return NSRGS_OK;
}

int sync_step_bsr(const nsrgs_bsr_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in, void *X_out,
                  void *ws, size_t ws_bytes, void *stream) {
  int st;
  if ((st = bsr_common(n, d, 0.0))) return st;
  if (!A || !A->row_ptr || !A->col_idx || !A->values) return fail(NSRGS_ERR_INVALID_ARG, "NULL matrix pointer");
  if (A->fmt != NSRGS_A_F32 && A->fmt != NSRGS_A_BF16)
    return fail(NSRGS_ERR_UNSUPPORTED, "block-sparse values must be F32 or BF16");
  if (!std::isfinite(mu)) return fail(NSRGS_ERR_INVALID_ARG, "mu must be finite");
  if (ns_steps < 0 || ns_steps > 64) return fail(NSRGS_ERR_INVALID_ARG, "ns_steps must be in [0, 64]");
  if (!X_in || !X_out || !aligned16(X_in) || !aligned16(X_out))
    return fail(NSRGS_ERR_INVALID_ARG, "X buffers must be non-NULL and 16-byte aligned");
  const size_t xb = (size_t)n * d * d * sizeof(float);
  const uintptr_t xi = (uintptr_t)X_in, xo = (uintptr_t)X_out;
  if (xi < xo + xb && xo < xi + xb) return fail(NSRGS_ERR_INVALID_ARG, "X_in and X_out overlap");
  if (!ws || ((uintptr_t)ws & 255u)) return fail(NSRGS_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (d > kBsrStepMaxD)
    return bsr_wide_step(A, n, d, mu, ns_steps, X_in, X_out, ws, ws_bytes, (hipStream_t)stream);
  const bool sliced = bsr_sliced(n, d, ws_bytes);
  const size_t need = narrow_ws_bytes(n, d, NSRGS_A_F32);
  if (ws_bytes < need) return fail(NSRGS_ERR_OUT_OF_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  StreamArgs sa{};
  sa.X_in = X_in;
  sa.X_out = X_out;
  sa.n = n;
  sa.d = d;
  sa.nd = n * d;
  sa.num_panels = (n + kBsrRowsPerGroup - 1) / kBsrRowsPerGroup;
  sa.mu = mu > 0.0 ? mu : 1.0 / n;
  sa.ns_steps = ns_steps;
  sa.partials = static_cast<char *>(ws) + step_ws_stats_offset(n, d, NSRGS_A_F32);
  sa.ctl = static_cast<DevCtl *>(ws);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (sliced) {
    char *base = static_cast<char *>(ws);
    int32_t *bounds = reinterpret_cast<int32_t *>(base + bsr_slice_table_off(n, d));
    float *part = reinterpret_cast<float *>(base + bsr_slice_part_off(n, d));
    e = A->fmt == NSRGS_A_F32 ? bsr_slice_launch<float>(d, *A, sa, bounds, part, true, s)
                              : bsr_slice_launch<uint16_t>(d, *A, sa, bounds, part, true, s);
  } else {
    e = A->fmt == NSRGS_A_F32 ? bsr_launch<float>(d, *A, sa, s) : bsr_launch<uint16_t>(d, *A, sa, s);
  }
  NSRGS_HIP(e, "bsr step launch");
  return NSRGS_OK;
}

size_t sync_step_bsr_workspace_bytes(int n, int d) {
  if (n < 2 || d < 1 || d > kBsrMaxD || (int64_t)n * d * d >= (int64_t)1 << 31) return 0;
  if (d > kBsrSliceMaxD || (int64_t)n * d * d * 4 >= ((int64_t)1 << 31)) return sync_workspace_bytes(n, d, NSRGS_A_F32);
  return bsr_slice_ws_bytes(n, d);
}

}  // extern "C"
