// Spectral initialization of Algorithm 2 (paper Sec. 2.2): Y = top-d
// eigenvectors of A with Y^T Y = I, then X^0 = sgn(Y) blockwise.
//
// Block subspace iteration on d columns.  Each iteration is
//   (1) W = A Y_k, streamed by the NS-RGS streaming kernel in product mode,
//       which also reduces Y_k^T W (the Rayleigh quotient) and W^T W (FP64)
//       and factors W^T W = R^T R;
//   (2) this file's apply kernel: Y_{k+1} = W R^{-1} (Cholesky-QR) and the
//       residual ||W - Y_k T_k||_F, whose relative size ends the iteration.
// The polar kernel then forms sgn(Y_i) per block by FP64 Newton-Schulz from
// the Frobenius-scaled block (singular values in (0, 1]) until
// ||I - S^T S||_F <= 1e-13, plus two more quadratic steps.
#include "device.h"
#include "kernels.h"

namespace nsrgs {

template <typename T>
__global__ void init_random_kernel(T *Y, int nd, int d, uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nd * d) return;
  const uint32_t row = (uint32_t)(i / d), col = (uint32_t)(i % d);
  Y[i] = (T)normal_from(philox4x32_10(U4{row, col, 2u, 0u}, k0, k1));
}

// One thread per row: Y_next = W Rinv, residual W - Y T.
template <typename T, int D>
__global__ void __launch_bounds__(256) init_apply_kernel(InitArgs a) {
  __shared__ T sR[D * D], sT[D * D];
  __shared__ double s_scr[kMaxWaves];
  __shared__ int s_last;
  DevCtl *ctl = a.ctl;
  if (__atomic_load_n(&ctl->init_done, __ATOMIC_RELAXED)) return;   // uniform
  const int tid = threadIdx.x;
  for (int e = tid; e < D * D; e += blockDim.x) {
    sR[e] = (T)ctl->Rinv[e];
    sT[e] = (T)ctl->T[e];
  }
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + tid;
  double res2 = 0.0;
  int bad = 0;
  if (row < a.nd) {
    const T *W = static_cast<const T *>(a.W) + (int64_t)row * D;
    const T *Y = static_cast<const T *>(a.Y) + (int64_t)row * D;
    T *Yn = static_cast<T *>(a.Y_next) + (int64_t)row * D;
    T w[D], y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      w[k] = W[k];
      y[k] = Y[k];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T s = 0, t = 0;
#pragma unroll
      for (int m = 0; m < D; ++m) {
        s += w[m] * sR[m * D + k];
        t += y[m] * sT[m * D + k];
      }
      Yn[k] = s;
      const double r = (double)w[k] - (double)t;
      res2 += r * r;
      bad |= !isfinite(s);
    }
  }
  res2 = block_sum(res2, s_scr);
  const double fbad = block_max((double)bad, s_scr);
  double *part = static_cast<double *>(a.partials);
  if (tid == 0) {
    part[2 * blockIdx.x] = res2;
    part[2 * blockIdx.x + 1] = fbad;
  }
  // release: this workgroup's results before its arrival is counted (no L2
  // invalidate here: a full fence per workgroup keeps evicting the reused X)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(&ctl->arrive2, 1u) == (unsigned)a.num_groups - 1u);
  __syncthreads();
  if (s_last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every other workgroup's results
    double s = 0.0, b = 0.0;
    for (int g = tid; g < a.num_groups; g += blockDim.x) {
      s += part[2 * g];
      b = part[2 * g + 1] > b ? part[2 * g + 1] : b;
    }
    s = block_sum(s, s_scr);
    b = block_max(b, s_scr);
    if (tid == 0) {
      double tn = 0.0;
      for (int e = 0; e < D * D; ++e) tn += ctl->T[e] * ctl->T[e];
      const double rel = tn > 0.0 ? sqrt(s / tn) : 0.0;
      ctl->init_res = rel;
      ctl->init_iters = a.iter + 1;
      if (b != 0.0 || !isfinite(rel)) ctl->init_bad = 1;
      // The first basis is random, not orthonormal: no test at iteration 0.
      if (a.iter >= 1 && rel <= a.tol) ctl->init_done = 1;
      if (ctl->init_bad) ctl->init_done = 1;
      ctl->arrive2 = 0u;
    }
  }
}

// One workgroup (64 threads) per block: X0_i = sgn(Y_i) in FP64.
template <typename T, int D>
__global__ void __launch_bounds__(64) init_polar_kernel(const T *Y, T *X0, int n, DevCtl *ctl) {
  constexpr int NE = D * D;
  __shared__ double sS[NE], sM[NE], sN[NE];
  __shared__ double s_scr[kMaxWaves];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  double nrm = 0.0;
  for (int e = tid; e < NE; e += blockDim.x) {
    const double v = (double)Y[(int64_t)b * NE + e];
    sS[e] = v;
    nrm += v * v;
  }
  nrm = sqrt(block_sum(nrm, s_scr));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int e = tid; e < NE; e += blockDim.x) sS[e] *= inv;
  __syncthreads();
  double *cur = sS, *nxt = sN;
  int steps = 0, extra = -1;
  bool ok = false;
  for (int it = 0; it < 200; ++it) {
    double def = 0.0;
    for (int e = tid; e < NE; e += blockDim.x) {
      const int a = e / D, k = e % D;
      double s = 0.0;
      for (int m = 0; m < D; ++m) s += cur[m * D + a] * cur[m * D + k];
      sM[e] = s;
      const double dl = (a == k ? 1.0 : 0.0) - s;
      def += dl * dl;
    }
    def = sqrt(block_sum(def, s_scr));        // block_sum synchronises
    if (!isfinite(def)) break;
    if (extra < 0 && def <= 1e-13) extra = 2;
    if (extra == 0) {
      ok = true;
      break;
    }
    for (int e = tid; e < NE; e += blockDim.x) {
      const int a = e / D, k = e % D;
      double s = 0.0;
      for (int m = 0; m < D; ++m) s += cur[a * D + m] * sM[m * D + k];
      nxt[e] = 1.5 * cur[e] - 0.5 * s;
    }
    __syncthreads();
    double *t = cur;
    cur = nxt;
    nxt = t;
    ++steps;
    if (extra > 0) --extra;
  }
  for (int e = tid; e < NE; e += blockDim.x) X0[(int64_t)b * NE + e] = (T)cur[e];
  if (tid == 0) {
    atomicMax(&ctl->polar_steps, steps);
    if (!ok) atomicOr(&ctl->init_bad, 1);
  }
}

// Ritz values: eigenvalues of T (FP64 cyclic Jacobi), descending.
__global__ void init_finish_kernel(DevCtl *ctl, int d) {
  if (threadIdx.x != 0) return;
  __shared__ double M[kMaxD * kMaxD];
  for (int e = 0; e < d * d; ++e) M[e] = ctl->T[e];
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q) {
        tot += M[p * d + q] * M[p * d + q];
        if (p != q) off += M[p * d + q] * M[p * d + q];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < d - 1; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = M[p * d + q];
        if (apq == 0.0) continue;
        const double theta = (M[q * d + q] - M[p * d + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < d; ++k) {      // rotate rows p, q
          const double mp = M[p * d + k], mq = M[q * d + k];
          M[p * d + k] = c * mp - s * mq;
          M[q * d + k] = s * mp + c * mq;
        }
        for (int k = 0; k < d; ++k) {      // rotate columns p, q
          const double mp = M[k * d + p], mq = M[k * d + q];
          M[k * d + p] = c * mp - s * mq;
          M[k * d + q] = s * mp + c * mq;
        }
      }
  }
  double w[kMaxD];
  for (int i = 0; i < d; ++i) w[i] = M[i * d + i];
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j)
      if (w[j] > w[i]) {
        const double t = w[i];
        w[i] = w[j];
        w[j] = t;
      }
  for (int i = 0; i < d; ++i) ctl->ritz[i] = w[i];
}

// what: 0 = whole control block, 1 = solve fields, 2 = init fields.
__global__ void ctl_reset_kernel(DevCtl *ctl, int what) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (what == 0) {
    ctl->arrive = 0u;
    ctl->arrive2 = 0u;
  }
  if (what == 0 || what == 1) {
    ctl->done = 0;
    ctl->iters = 0;
    ctl->nonfinite = 0;
    ctl->converged = 0;
    ctl->rel_change = 0.0;
    ctl->max_defect = 0.0;
    ctl->sum_dx2 = 0.0;
    ctl->sum_x2 = 0.0;
  }
  if (what == 0 || what == 2) {
    ctl->init_done = 0;
    ctl->init_iters = 0;
    ctl->init_bad = 0;
    ctl->polar_steps = 0;
    ctl->init_res = 0.0;
    for (int i = 0; i < kMaxD; ++i) ctl->ritz[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------
#define NSRGS_D_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_init_random(int fmt, void *Y, int nd, int d, uint64_t seed, hipStream_t s) {
  const int64_t total = (int64_t)nd * d;
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (fmt == NSRGS_A_F64)
    hipLaunchKernelGGL(init_random_kernel<double>, grid, block, 0, s, (double *)Y, nd, d, k0, k1);
  else
    hipLaunchKernelGGL(init_random_kernel<float>, grid, block, 0, s, (float *)Y, nd, d, k0, k1);
  return hipGetLastError();
}

hipError_t launch_init_apply(int fmt, const InitArgs &a, hipStream_t s) {
  const dim3 block(256), grid((unsigned)a.num_groups);
#define NSRGS_AP(DD)                                                                   \
  if (a.d == DD) {                                                                     \
    if (fmt == NSRGS_A_F64)                                                            \
      hipLaunchKernelGGL((init_apply_kernel<double, DD>), grid, block, 0, s, a);       \
    else                                                                               \
      hipLaunchKernelGGL((init_apply_kernel<float, DD>), grid, block, 0, s, a);        \
    return hipGetLastError();                                                          \
  }
  NSRGS_D_LIST(NSRGS_AP)
#undef NSRGS_AP
  return hipErrorInvalidValue;
}

hipError_t launch_init_polar(int fmt, const void *Y, void *X0, int n, int d, DevCtl *ctl,
                             hipStream_t s) {
  const dim3 block(64), grid((unsigned)n);
#define NSRGS_PO(DD)                                                                   \
  if (d == DD) {                                                                       \
    if (fmt == NSRGS_A_F64)                                                            \
      hipLaunchKernelGGL((init_polar_kernel<double, DD>), grid, block, 0, s,           \
                         (const double *)Y, (double *)X0, n, ctl);                     \
    else                                                                               \
      hipLaunchKernelGGL((init_polar_kernel<float, DD>), grid, block, 0, s,            \
                         (const float *)Y, (float *)X0, n, ctl);                       \
    return hipGetLastError();                                                          \
  }
  NSRGS_D_LIST(NSRGS_PO)
#undef NSRGS_PO
  return hipErrorInvalidValue;
}

hipError_t launch_init_finish(DevCtl *ctl, int d, hipStream_t s) {
  hipLaunchKernelGGL(init_finish_kernel, dim3(1), dim3(64), 0, s, ctl, d);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(DevCtl *ctl, int what, hipStream_t s) {
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(64), 0, s, ctl, what);
  return hipGetLastError();
}

}  // namespace nsrgs
