// Batched small products of the sweep and of the apply: one workgroup per box
// (and per output block).  Operands stay in HBM/L2; each thread owns a strip
// of output entries and runs the full inner product in FP64.
#include "hbs_internal.h"

namespace hbs {
namespace {

constexpr int kNT = 256;

// C(i, j) = beta * C0(i, j) + alpha * sum_kk A(i, kk) B(kk, j) for i < M, j < N,
// with A(i, kk) = A[i * sar + kk * sac] and B(kk, j) = B[kk * sbr + j * sbc].
// C0 may alias C.  Called by every thread of the block.
__device__ __forceinline__ void bgemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                                      int64_t sar, int64_t sac, const double* __restrict__ B, int64_t sbr,
                                      int64_t sbc, double beta, const double* C0, int64_t ldc0, double* C,
                                      int64_t ldc) {
  for (int idx = threadIdx.x; idx < M * N; idx += blockDim.x) {
    const int i = idx / N, j = idx % N;
    const double* a = A + i * sar;
    const double* b = B + j * sbc;
    double acc0 = 0.0, acc1 = 0.0;
    int kk = 0;
    for (; kk + 1 < K; kk += 2) {
      acc0 += a[kk * sac] * b[kk * sbr];
      acc1 += a[(kk + 1) * sac] * b[(kk + 1) * sbr];
    }
    if (kk < K) acc0 += a[kk * sac] * b[kk * sbr];
    const double v = alpha * (acc0 + acc1);
    C[i * ldc + j] = (beta != 0.0) ? beta * C0[i * ldc0 + j] + v : v;
  }
}

// D_tau of eq. d_tau_formula, evaluated as
//   T1 = V^* X, X' = X - V T1 = (I - V V^*) X, E = X' U,
//   T2 = U^* W, D = W - U (T2 - E^*) = (I - U U^*) W + U (X' U)^*
//     = (I - U U^*) W + U U^* ((I - V V^*) X)^*.
__global__ void __launch_bounds__(kNT) combine_kernel(CombineArgs a) {
  const int box = blockIdx.x;
  const int m = a.mtau[box], k = a.k, mm = a.mmax;
  const double* U = a.U + (int64_t)box * mm * k;
  const double* V = a.V + (int64_t)box * mm * k;
  const double* W = a.W + (int64_t)box * mm * mm;
  const double* X = a.X + (int64_t)box * mm * mm;
  double* D = a.D + (int64_t)box * mm * mm;
  double* T1 = a.T + (int64_t)box * (mm * mm + 3 * mm * k);  // k x m
  double* Xp = T1 + mm * k;                                  // m x m
  double* E = Xp + mm * mm;                                  // m x k
  double* T2 = E + mm * k;                                   // k x m
  // T1 = V^* X
  bgemm(k, m, m, 1.0, V, 1, k, X, mm, 1, 0.0, nullptr, 0, T1, m);
  __syncthreads();
  // X' = X - V T1
  bgemm(m, m, k, -1.0, V, k, 1, T1, m, 1, 1.0, X, mm, Xp, m);
  __syncthreads();
  // E = X' U ; T2 = U^* W
  bgemm(m, k, m, 1.0, Xp, m, 1, U, k, 1, 0.0, nullptr, 0, E, k);
  bgemm(k, m, m, 1.0, U, 1, k, W, mm, 1, 0.0, nullptr, 0, T2, m);
  __syncthreads();
  // T2 <- T2 - E^*
  for (int idx = threadIdx.x; idx < k * m; idx += blockDim.x) {
    const int i = idx / m, j = idx % m;
    T2[i * m + j] -= E[j * k + i];
  }
  __syncthreads();
  // D = W - U T2
  bgemm(m, m, k, -1.0, U, k, 1, T2, m, 1, 1.0, W, mm, D, mm);
  // zero padding of D (rows/cols m .. mm-1)
  for (int idx = threadIdx.x; idx < mm * mm; idx += blockDim.x) {
    const int i = idx / mm, j = idx % mm;
    if (i >= m || j >= m) D[idx] = 0.0;
  }
}

// The four k x s blocks one child hands to its parent (eq.
// omega_tau_and_y_tau; Psi and Z rows as in Algorithm 2):
//   y = 0: V^* Omega_tau      y = 1: U^* (Y_tau - D_tau Omega_tau)
//   y = 2: U^* Psi_tau        y = 3: V^* (Z_tau - D_tau^* Psi_tau)
// Child t writes rows [k t, k t + k) of the next level's panels (ld = s).
__global__ void __launch_bounds__(kNT) parent_kernel(ParentArgs a) {
  const int box = blockIdx.x, which = blockIdx.y;
  const int m = a.mtau[box], k = a.k, s = a.s, mm = a.mmax;
  const int64_t ld = a.ld;
  const int64_t r0 = a.row0[box];
  const double* U = a.U + (int64_t)box * mm * k;
  const double* V = a.V + (int64_t)box * mm * k;
  const double* D = a.D + (int64_t)box * mm * mm;
  const double* Bas = (which == 0 || which == 3) ? V : U;
  const double* Tst = ((which < 2) ? a.Om : a.Ps) + r0 * ld;
  double* out = ((which == 0) ? a.nOm : (which == 1) ? a.nY : (which == 2) ? a.nPs : a.nZ) +
                (int64_t)box * k * s;
  if (which == 0 || which == 2) {
    bgemm(k, s, m, 1.0, Bas, 1, k, Tst, ld, 1, 0.0, nullptr, 0, out, s);
    return;
  }
  const double* Smp = ((which == 1) ? a.Y : a.Z) + r0 * ld;
  double* R = a.R + ((int64_t)box * 2 + (which == 3)) * mm * s;
  // R = Smp - D Tst  (or D^*)
  if (which == 1)
    bgemm(m, s, m, -1.0, D, mm, 1, Tst, ld, 1, 1.0, Smp, ld, R, s);
  else
    bgemm(m, s, m, -1.0, D, 1, mm, Tst, ld, 1, 1.0, Smp, ld, R, s);
  __syncthreads();
  bgemm(k, s, m, 1.0, Bas, 1, k, R, s, 1, 0.0, nullptr, 0, out, s);
}

// Upward pass of Algorithm 1 on one level: qhat_tau = B_tau^* in_tau, where
// in_tau is q(I_tau, :) at the leaves and [qhat_alpha; qhat_beta] above.
__global__ void __launch_bounds__(kNT) apply_up_kernel(ApplyArgs a) {
  const int box = blockIdx.x;
  const int m = a.mtau[box], k = a.k;
  const double* Bas = a.B1 + (int64_t)box * a.mmax * k;
  const double* in = a.in + (a.leaf ? a.row0[box] : (int64_t)box * m) * a.ld_in;
  double* out = a.out + (int64_t)box * k * a.ld_out;
  bgemm(k, (int)a.nvec, m, 1.0, Bas, 1, k, in, a.ld_in, 1, 0.0, nullptr, 0, out, a.ld_out);
}

// Downward pass of Algorithm 1 on one level:
//   out_tau = B_tau uhat_tau + D_tau qin_tau
// out_tau is [uhat_alpha; uhat_beta] above the leaves and u(I_tau, :) at them.
__global__ void __launch_bounds__(kNT) apply_down_kernel(ApplyArgs a) {
  const int box = blockIdx.x;
  const int m = a.mtau[box], k = a.k, mm = a.mmax;
  const int nv = (int)a.nvec;
  const double* Bas = a.B1 + (int64_t)box * mm * k;
  const double* D = a.Dm + (int64_t)box * mm * mm;
  const int64_t rows = a.leaf ? a.row0[box] : (int64_t)box * m;
  const double* uh = a.in + (int64_t)box * k * a.ld_in;
  const double* qin = a.qin + rows * a.ld_q;
  double* out = a.out + rows * a.ld_out;
  for (int idx = threadIdx.x; idx < m * nv; idx += blockDim.x) {
    const int i = idx / nv, j = idx % nv;
    double acc = 0.0;
    for (int kk = 0; kk < k; ++kk) acc += Bas[i * k + kk] * uh[kk * a.ld_in + j];
    if (a.transD)
      for (int kk = 0; kk < m; ++kk) acc += D[kk * mm + i] * qin[kk * a.ld_q + j];
    else
      for (int kk = 0; kk < m; ++kk) acc += D[i * mm + kk] * qin[kk * a.ld_q + j];
    out[i * a.ld_out + j] = acc;
  }
}

// Plain C = op(A) B for the root block (one workgroup per 64 rows).
__global__ void __launch_bounds__(kNT) dense_small_kernel(const double* A, int64_t lda, int32_t transA,
                                                          const double* Bm, int64_t ldb, double* C, int64_t ldc,
                                                          int32_t M, int32_t N, int32_t K) {
  const int r0 = blockIdx.x * 64;
  const int mrows = (M - r0) < 64 ? (M - r0) : 64;
  if (transA)
    bgemm(mrows, N, K, 1.0, A + r0, 1, lda, Bm, ldb, 1, 0.0, nullptr, 0, C + (int64_t)r0 * ldc, ldc);
  else
    bgemm(mrows, N, K, 1.0, A + (int64_t)r0 * lda, lda, 1, Bm, ldb, 1, 0.0, nullptr, 0, C + (int64_t)r0 * ldc,
          ldc);
}

}  // namespace

hipError_t launch_combine(const CombineArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(a.nodes), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_parent(const ParentArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(parent_kernel, dim3(a.nodes, 4), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_apply_up(const ApplyArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(apply_up_kernel, dim3(a.nodes), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_apply_down(const ApplyArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(apply_down_kernel, dim3(a.nodes), dim3(kNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dense_small(const double* A, int64_t lda, int32_t transA, const double* Bm, int64_t ldb,
                              double* C, int64_t ldc, int32_t M, int32_t N, int32_t K, hipStream_t st) {
  hipLaunchKernelGGL(dense_small_kernel, dim3((M + 63) / 64), dim3(kNT), 0, st, A, lda, transA, Bm, ldb, C, ldc,
                     M, N, K);
  return hipGetLastError();
}

}  // namespace hbs
