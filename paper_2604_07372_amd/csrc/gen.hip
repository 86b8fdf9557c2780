// Inputs on the device: the measurement matrix A = Z Z^T + sigma W of the
// paper's model (Sec. 2.2, eq. def:measurements; incomplete observations of
// Sec. 4.1) from a counter-based generator, and the one-time conversion of an
// FP32 A into the reduced storage formats of the precision forms.
#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "wide.h"

namespace nsrgs {

// One workgroup per row r; threads stride over the columns.  Element (r, c)
// is a pure function of (Z, sigma, seed, r, c): symmetric by construction.
// ld == NSRGS_LD_PACKED: A is the packed upper block triangle (row0 = 0); the
// row's columns [c0, ndp) are written, zeros past n d.
template <typename T>
__global__ void __launch_bounds__(256)
generate_kernel(const double *__restrict__ Z, int n, int d, double sigma, uint32_t k0,
                uint32_t k1, int zero_diag, double p, T *__restrict__ A, int64_t ld, int row0) {
  const int nd = n * d;
  const int r = row0 + (int)blockIdx.x;     // global row; A points at row row0
  double zr[kWideMaxD];
  for (int k = 0; k < d; ++k) zr[k] = Z[(int64_t)r * d + k];
  const int br = r / d;
  T *out;
  int cbeg, cend;
  if (ld == NSRGS_LD_PACKED) {
    const int64_t ndp = packed_ndp(n, d);
    cbeg = packed_c0(br, d);
    cend = (int)ndp;
    out = A + packed_row_offset(r, d, ndp) - cbeg;
  } else {
    cbeg = 0;
    cend = nd;
    out = A + (int64_t)blockIdx.x * ld;
  }
  for (int c = cbeg + (int)threadIdx.x; c < cend; c += blockDim.x) {
    if (c >= nd) {
      out[c] = T(0);
      continue;
    }
    double v = 0.0;
    for (int k = 0; k < d; ++k) v = fma(zr[k], Z[(int64_t)c * d + k], v);
    const int bc = c / d;
    const bool diag_blk = (br == bc);
    if (sigma != 0.0 && !(zero_diag && diag_blk)) {
      const uint32_t lo = (uint32_t)(r < c ? r : c), hi = (uint32_t)(r < c ? c : r);
      v += sigma * normal_from(philox4x32_10(U4{hi, lo, 0u, 0u}, k0, k1));
    }
    if (p < 1.0 && !diag_blk) {
      const uint32_t blo = (uint32_t)(br < bc ? br : bc), bhi = (uint32_t)(br < bc ? bc : br);
      const U4 o = philox4x32_10(U4{bhi, blo, 1u, 0u}, k0, k1);
      if (!((double)o.x * 0x1p-32 < p)) v = 0.0;
    }
    out[c] = (T)v;   // round to nearest even once
  }
}

// ---- storage-format conversion --------------------------------------------
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return ((u >> 16) & 0x8000u) | 0x7fc0u;   // NaN
  const uint32_t lsb = (u >> 16) & 1u;
  return ((u + 0x7fffu + lsb) >> 16) & 0xffffu;
}

// OCP e4m3 (bias 7, 3 mantissa bits, no infinities, 0x7f = NaN, max 448):
// round to nearest even, saturate to +-448.
__device__ __forceinline__ uint32_t e4m3_rne_sat(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = (u >> 24) & 0x80u;
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fu;
  const float a = fabsf(x);
  if (a >= 448.0f) return sign | 0x7eu;
  if (a < 0x1p-6f) {
    // subnormal grid: multiples of 2^-9; q in [0, 8], q = 8 is the smallest normal
    const uint32_t q = (uint32_t)rintf(a * 512.0f);
    return q ? (sign | q) : (sign ? 0x80u : 0u);
  }
  const uint32_t au = __float_as_uint(a);
  int e = (int)((au >> 23) & 0xffu) - 127;          // in [-6, 8]
  uint32_t m = au & 0x7fffffu;
  uint32_t q = m >> 20;
  const uint32_t rem = m & 0xfffffu;
  if (rem > 0x80000u || (rem == 0x80000u && (q & 1u))) ++q;
  if (q == 8u) {
    q = 0u;
    ++e;
  }
  return sign | ((uint32_t)(e + 7) << 3) | q;
}

__global__ void __launch_bounds__(256)
convert_bf16_kernel(const float *__restrict__ A, int nd, int64_t ld, uint16_t *__restrict__ hi,
                    uint16_t *__restrict__ lo, int row0) {
  const int r = row0 + (int)blockIdx.x;             // destination row; A points at row row0
  const float *src = A + (int64_t)blockIdx.x * ld;
  for (int c = threadIdx.x; c < nd; c += blockDim.x) {
    const float a = src[c];
    const uint32_t h = bf16_rne_bits(a);
    hi[(int64_t)r * ld + c] = (uint16_t)h;
    if (lo) {
      const float rem = a - __uint_as_float(h << 16);   // exact
      lo[(int64_t)r * ld + c] = (uint16_t)bf16_rne_bits(rem);
    }
  }
}

__global__ void __launch_bounds__(256)
convert_fp8_kernel(const float *__restrict__ A, int nd, int64_t ld, uint8_t *__restrict__ q,
                   float *__restrict__ scale, int row0) {
  __shared__ float s_scr[kMaxWaves];
  const int r = row0 + (int)blockIdx.x;             // destination row; A points at row row0
  const float *src = A + (int64_t)blockIdx.x * ld;
  float m = 0.0f;
  for (int c = threadIdx.x; c < nd; c += blockDim.x) m = fmaxf(m, fabsf(src[c]));
  m = block_max(m, s_scr);
  const float s = (m == 0.0f) ? 1.0f : m / 448.0f;
  if (threadIdx.x == 0) scale[r] = s;
  for (int c = threadIdx.x; c < nd; c += blockDim.x)
    q[(int64_t)r * ld + c] = (uint8_t)e4m3_rne_sat(src[c] / s);
}

__global__ void __launch_bounds__(256)
convert_bf16_flat_kernel(const float *__restrict__ A, int64_t count, uint16_t *__restrict__ hi,
                         uint16_t *__restrict__ lo) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float a = A[i];
    const uint32_t h = bf16_rne_bits(a);
    hi[i] = (uint16_t)h;
    if (lo) lo[i] = (uint16_t)bf16_rne_bits(a - __uint_as_float(h << 16));
  }
}

hipError_t launch_convert_flat(const float *A32, int64_t count, const nsrgs_matrix &out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (out.fmt != NSRGS_A_BF16 && out.fmt != NSRGS_A_BF16_SPLIT) return hipErrorInvalidValue;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(convert_bf16_flat_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A32, count,
                     (uint16_t *)out.data, out.fmt == NSRGS_A_BF16_SPLIT ? (uint16_t *)out.data_lo : nullptr);
  return hipGetLastError();
}

hipError_t launch_generate_rows(const double *Z, int n, int d, double sigma, uint64_t seed,
                                int zero_diag, double p, int fmt, void *A_rows, int64_t ld, int row0,
                                int nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const dim3 grid((unsigned)nrows), block(256);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(generate_kernel<double>, grid, block, 0, s, Z, n, d, sigma, k0, k1,
                       zero_diag, p, (double *)A_rows, ld, row0);
  else if (fmt == NSRGS_A_F32)
    hipLaunchKernelGGL(generate_kernel<float>, grid, block, 0, s, Z, n, d, sigma, k0, k1,
                       zero_diag, p, (float *)A_rows, ld, row0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_generate(const double *Z, int n, int d, double sigma, uint64_t seed,
                           int zero_diag, double p, int fmt, void *A, int64_t ld,
                           hipStream_t s) {
  return launch_generate_rows(Z, n, d, sigma, seed, zero_diag, p, fmt, A, ld, 0, n * d, s);
}

hipError_t launch_convert_rows(const float *A32_rows, int nd, int64_t ld, const nsrgs_matrix &out,
                               int row0, int nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const dim3 grid((unsigned)nrows), block(256);
  switch (out.fmt) {
    case NSRGS_A_BF16:
      hipLaunchKernelGGL(convert_bf16_kernel, grid, block, 0, s, A32_rows, nd, ld,
                         (uint16_t *)out.data, (uint16_t *)nullptr, row0);
      break;
    case NSRGS_A_BF16_SPLIT:
      hipLaunchKernelGGL(convert_bf16_kernel, grid, block, 0, s, A32_rows, nd, ld,
                         (uint16_t *)out.data, (uint16_t *)out.data_lo, row0);
      break;
    case NSRGS_A_FP8_E4M3:
      hipLaunchKernelGGL(convert_fp8_kernel, grid, block, 0, s, A32_rows, nd, ld,
                         (uint8_t *)out.data, (float *)out.row_scale, row0);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_convert(const float *A32, int nd, int64_t ld, const nsrgs_matrix &out,
                          hipStream_t s) {
  return launch_convert_rows(A32, nd, ld, out, 0, nd, s);
}

}  // namespace nsrgs
