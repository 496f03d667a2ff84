// Batched small products of the apply (Algorithm 1): one workgroup per box,
// operands staged through LDS, FP64 register tiles.
#include "hbs_internal.h"

namespace hbs {
namespace {

constexpr int kNT = 256;

// Block-level FP64 product through LDS, called by all kNT threads:
//   C(i, j) = alpha * sum_kk A(i, kk) B(kk, j) + beta * C0(i, j),  i < M, j < N,
// with A(i, kk) = A[i * sar + kk * sac] and B(kk, j) = B[kk * sbr + j * sbc]
// (strides express transposes).  64 x 64 output tiles, 4 x 4 per thread,
// K staged in chunks of TK (deeper chunks: fewer memory round trips on the
// latency-bound levels near the root, more registers); global loads are coalesced along whichever index
// is contiguous.  C0 may alias C.  Ends with a barrier.
constexpr int TM = 64, TN = 64;
template <int TK>
struct GemmSmem {
  double As[TK][TM + 1];
  double Bs[TK][TN + 1];
};

template <int TK>
__device__ void tile_gemm(int M, int N, int K, double alpha, const double* __restrict__ A, int64_t sar,
                          int64_t sac, const double* __restrict__ B, int64_t sbr, int64_t sbc, double beta,
                          const double* C0, int64_t ldc0, double* C, int64_t ldc, GemmSmem<TK>& sm) {
  constexpr int LA = (TM * TK) / kNT, LB = (TN * TK) / kNT;
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  // per-thread element coordinates of the staged A and B chunks
  int ai[LA], ak[LA], bj[LB], bk[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int idx = tid + r * kNT;
    ai[r] = (sac == 1) ? idx / TK : idx % TM;
    ak[r] = (sac == 1) ? idx % TK : idx / TM;
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int idx = tid + r * kNT;
    bj[r] = (sbc == 1) ? idx % TN : idx / TK;
    bk[r] = (sbc == 1) ? idx / TN : idx % TK;
  }
  for (int i0 = 0; i0 < M; i0 += TM) {
    for (int j0 = 0; j0 < N; j0 += TN) {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      double pa[LA], pb[LB];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
          const int gi = i0 + ai[r], gk = k0 + ak[r];
          const bool ok = gi < M && gk < K;
          const double v = A[ok ? gi * sar + gk * sac : 0];
          pa[r] = ok ? v : 0.0;
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
          const int gj = j0 + bj[r], gk = k0 + bk[r];
          const bool ok = gj < N && gk < K;
          const double v = B[ok ? gk * sbr + gj * sbc : 0];
          pb[r] = ok ? v : 0.0;
        }
      };
      fetch(0);
      for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int r = 0; r < LA; ++r) sm.As[ak[r]][ai[r]] = pa[r];
#pragma unroll
        for (int r = 0; r < LB; ++r) sm.Bs[bk[r]][bj[r]] = pb[r];
        __syncthreads();
        if (k0 + TK < K) fetch(k0 + TK);  // next chunk in flight during the products
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) av[a] = sm.As[kk][ty + 16 * a];
#pragma unroll
          for (int b = 0; b < 4; ++b) bv[b] = sm.Bs[kk][tx + 16 * b];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int gi = i0 + ty + 16 * a;
        if (gi >= M) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int gj = j0 + tx + 16 * b;
          if (gj >= N) continue;
          const double v = alpha * acc[a][b];
          C[gi * ldc + gj] = (beta != 0.0) ? beta * C0[gi * ldc0 + gj] + v : v;
        }
      }
    }
  }
  __syncthreads();
}

// Upward pass of Algorithm 1 on one level: qhat_tau = B_tau^* in_tau, where
// in_tau is q(I_tau, :) at the leaves and [qhat_alpha; qhat_beta] above.
__global__ void __launch_bounds__(kNT) apply_up_kernel(ApplyArgs a) {
  const int box = blockIdx.x;
  const int m = a.mtau[box], k = a.k;
  const double* Bas = a.B1 + (int64_t)box * a.mmax * k;
  const double* in = a.in + (a.leaf ? a.row0[box] : (int64_t)box * m) * a.ld_in;
  double* out = a.out + (int64_t)box * k * a.ld_out;
  __shared__ GemmSmem<16> sm;
  tile_gemm(k, (int)a.nvec, m, 1.0, Bas, 1, k, in, a.ld_in, 1, 0.0, nullptr, 0, out, a.ld_out, sm);
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
  __shared__ GemmSmem<16> sm;
  // out = B uhat, then out += D qin (or D^* qin)
  tile_gemm(m, nv, k, 1.0, Bas, k, 1, uh, a.ld_in, 1, 0.0, nullptr, 0, out, a.ld_out, sm);
  if (a.transD)
    tile_gemm(m, nv, m, 1.0, D, 1, mm, qin, a.ld_q, 1, 1.0, out, a.ld_out, out, a.ld_out, sm);
  else
    tile_gemm(m, nv, m, 1.0, D, mm, 1, qin, a.ld_q, 1, 1.0, out, a.ld_out, out, a.ld_out, sm);
}

// Plain C = op(A) B for the root block (one workgroup per 64 rows).
__global__ void __launch_bounds__(kNT) dense_small_kernel(const double* A, int64_t lda, int32_t transA,
                                                          const double* Bm, int64_t ldb, double* C, int64_t ldc,
                                                          int32_t M, int32_t N, int32_t K) {
  __shared__ GemmSmem<16> sm;
  const int r0 = blockIdx.x * 64;
  const int mrows = (M - r0) < 64 ? (M - r0) : 64;
  if (transA)
    tile_gemm(mrows, N, K, 1.0, A + r0, 1, lda, Bm, ldb, 1, 0.0, nullptr, 0, C + (int64_t)r0 * ldc, ldc, sm);
  else
    tile_gemm(mrows, N, K, 1.0, A + (int64_t)r0 * lda, lda, 1, Bm, ldb, 1, 0.0, nullptr, 0, C + (int64_t)r0 * ldc,
              ldc, sm);
}

}  // namespace

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
