// The incomplete observation model (Sec. 4.1): each off-diagonal block pair
// (i, j) is observed with probability p, and A_ij = 0 otherwise; the iteration
// is Algorithm 2 on that A with mu = 1/(np).  Only observed blocks are stored
// (block-sparse rows), so an iteration reads about p of the dense bytes.
//
// Storage (nsrgs_bsr_matrix): block row i holds m_i = row_ptr[i+1] - row_ptr[i]
// blocks with ascending block columns col_idx[row_ptr[i] ..]; entry (a, b) of
// its k-th block is values[row_ptr[i] d^2 + (a d + b) m_i + k].  A block row's
// values are entry-major, so the loads of one entry over 64 consecutive
// blocks are one contiguous 64-element read.
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
          values[base * d2 + (int64_t)(a * d + b) * m + k] = store_elem<T>(v);
        }
    }
    done += tot;
    __syncthreads();
  }
}

template <typename E>
__device__ __forceinline__ float load_elem(const E *p);
template <>
__device__ __forceinline__ float load_elem<float>(const float *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float load_elem<uint16_t>(const uint16_t *p) {
  return __uint_as_float((uint32_t)__builtin_nontemporal_load(p) << 16);
}

// One wave per block row, kBsrRowsPerGroup block rows per workgroup.
template <typename E, int D>
__global__ void __launch_bounds__(kWave * kBsrRowsPerGroup)
bsr_step_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                const E *__restrict__ values, StreamArgs sa) {
  constexpr int D2 = D * D;
  constexpr int NB = kBsrRowsPerGroup;
  constexpr int NE = NB * D2;
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
  float acc[D2];
#pragma unroll
  for (int e = 0; e < D2; ++e) acc[e] = 0.0f;
  for (int64_t k0 = 0; k0 < m; k0 += kWave) {
    const int64_t k = k0 + lane;
    const bool ok = k < m;
    const int64_t kc = ok ? k : m - 1;                  // clamped: in-bounds, masked below
    // streamed once, non-temporal like the values, so that X stays in cache
    const int jr = __builtin_nontemporal_load(col_idx + base + kc);
    const int j = jr < 0 ? 0 : (jr < n ? jr : n - 1);   // out-of-range indices read in bounds
    const bool use = ok && jr == j && j != ic;          // and, like a stored diagonal block, count 0
    float a[D2], x[D2];
#pragma unroll
    for (int e = 0; e < D2; ++e) a[e] = load_elem<E>(vals + (int64_t)e * m + kc);
#pragma unroll
    for (int e = 0; e < D2; ++e) x[e] = X[(int64_t)j * D2 + e];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < D2; ++e) a[e] = use ? a[e] : 0.0f;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int b = 0; b < D; ++b)
#pragma unroll
        for (int c = 0; c < D; ++c) acc[r * D + c] = fmaf(a[r * D + b], x[b * D + c], acc[r * D + c]);
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
      const float v = load_elem<E>(vals + (int64_t)e * m + k0 + kkc);
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

template <typename E, int D>
hipError_t bsr_launch_d(const nsrgs_bsr_matrix &A, const StreamArgs &sa, hipStream_t s) {
  hipLaunchKernelGGL((bsr_step_kernel<E, D>), dim3(sa.num_panels), dim3(kWave * kBsrRowsPerGroup), 0, s,
                     A.row_ptr, A.col_idx, static_cast<const E *>(A.values), sa);
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
  const hipError_t e = A->fmt == NSRGS_A_F32 ? bsr_launch<float>(d, *A, sa, s) : bsr_launch<uint16_t>(d, *A, sa, s);
  NSRGS_HIP(e, "bsr step launch");
  return NSRGS_OK;
}

}  // extern "C"
