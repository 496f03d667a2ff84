// Matrix-free log-kernel sampler: [Y Z] = A [Omega Psi] with
// A(i, j) = log|x_i - x_j| (i != j), A(i, i) = 0, evaluated on the fly.
//
// FP64 path: v_mfma_f64_16x16x4_f64.  A workgroup owns 64 rows and one chunk
// of up to 160 sample columns of one side (Y or Z); each of its 4 waves owns
// 16 rows and 10 output tiles of 16 x 16.  The points are the reduction index:
// per chunk of 32 points the workgroup stages the sample-matrix rows in LDS,
// and every lane forms its own A-operand entry (row l % 16, point l / 16 of the
// 4-point step) from the coordinates, so A is never stored.
//
// Matrix-core operand layout (16x16x4, FP64), verified on gfx950:
//   A operand: lane l holds A(l % 16, l / 16)
//   B operand: lane l holds B(l / 16, l % 16)
//   result:    lane l, element r holds C(l / 16 + 4 r, l % 16)
//
// BF16 path: v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Every kernel
// entry (formed in FP32) and every test-matrix entry is carried as a pair of
// BF16 values hi + lo (hi = bf16(v), lo = bf16(v - hi): 16 significant bits),
// and each product is the sum of the three partial products hi hi, hi lo,
// lo hi, so the samples carry about 1e-5 relative error instead of the 4e-3
// of plain BF16 operands.  A workgroup owns 64 rows and 208 columns of the
// concatenation [Omega Psi], so each kernel entry it forms serves 208 columns.
// Lanes l supply 8 consecutive points (8 (l / 16) + r) of row l % 16 (A) and
// of column l % 16 (B); the result is C(4 (l / 16) + r, l % 16).
#include "hbs_internal.h"

namespace hbs {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;     // rows per workgroup
constexpr int kTiles = 10;    // 16-column tiles per wave
constexpr int kCols = 16 * kTiles;
constexpr int kKC = 32;       // points staged per chunk

__device__ __forceinline__ double logk(double xi, double yi, double xj, double yj, bool same) {
  const double dx = xi - xj, dy = yi - yj;
  return same ? 0.0 : 0.5 * log(dx * dx + dy * dy);
}

__global__ void __launch_bounds__(256) logkernel_f64(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y, const double* __restrict__ Om,
                                                     const double* __restrict__ Ps, double* __restrict__ Yo,
                                                     double* __restrict__ Zo, int32_t s, int64_t ld,
                                                     int32_t nchunk, int64_t row0, int64_t row1) {
  __shared__ double Bsh[kKC][kCols];
  __shared__ double xsh[kKC], ysh[kKC];
  const int side = blockIdx.y / nchunk;
  const int chunk = blockIdx.y % nchunk;
  const int col0 = chunk * kCols;
  const int ncol = (s - col0) < kCols ? (s - col0) : kCols;
  const double* __restrict__ Bsrc = side ? Ps : Om;
  double* __restrict__ Out = side ? Zo : Yo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row = row0 + (int64_t)blockIdx.x * kRows + wave * 16 + (lane & 15);  // A-operand row of this lane
  const bool rowok = row < row1;
  const double xi = rowok ? x[row] : 0.0, yi = rowok ? y[row] : 0.0;
  d4 acc[kTiles];
#pragma unroll
  for (int t = 0; t < kTiles; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (int64_t j0 = 0; j0 < n; j0 += kKC) {
    __syncthreads();
    for (int idx = tid; idx < kKC * kCols; idx += 256) {
      const int jj = idx / kCols, cc = idx % kCols;
      const int64_t j = j0 + jj;
      Bsh[jj][cc] = (j < n && cc < ncol) ? Bsrc[j * ld + col0 + cc] : 0.0;
    }
    if (tid < kKC) {
      const int64_t j = j0 + tid;
      xsh[tid] = (j < n) ? x[j] : 0.0;
      ysh[tid] = (j < n) ? y[j] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int st = 0; st < kKC / 4; ++st) {
      const int jj = st * 4 + (lane >> 4);
      const int64_t j = j0 + jj;
      const double av = (rowok && j < n) ? logk(xi, yi, xsh[jj], ysh[jj], j == row) : 0.0;
#pragma unroll
      for (int t = 0; t < kTiles; ++t) {
        const double bv = Bsh[jj][t * 16 + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  const int64_t rbase = row0 + (int64_t)blockIdx.x * kRows + wave * 16 + (lane >> 4);
#pragma unroll
  for (int t = 0; t < kTiles; ++t) {
    const int c = t * 16 + (lane & 15);
    if (c < ncol) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = rbase + 4 * r;
        if (rr < row1) Out[rr * ld + col0 + c] = acc[t][r];
      }
    }
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTB = 13;           // 16-column tiles per workgroup
constexpr int kColsB = 16 * kTB;  // columns of [Omega Psi] per workgroup
constexpr int kKB = 32;           // points per chunk (the MFMA depth)
constexpr int kBPad = kKB + 8;    // staged BF16 values per column (16 bytes of padding)

__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

__global__ void __launch_bounds__(256) logkernel_bf16(int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ Om,
                                                      const double* __restrict__ Ps, double* __restrict__ Yo,
                                                      double* __restrict__ Zo, int32_t s, int64_t ld, int64_t row0,
                                                      int64_t row1) {
  __shared__ __bf16 Bhi[kColsB][kBPad];
  __shared__ __bf16 Blo[kColsB][kBPad];
  __shared__ double xsh[kKB], ysh[kKB];
  const int c0 = blockIdx.y * kColsB;  // first column of [Omega Psi]
  const int ncol = min(kColsB, 2 * s - c0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row = row0 + (int64_t)blockIdx.x * kRows + wave * 16 + (lane & 15);  // A-operand row of this lane
  const bool rowok = row < row1;
  const double xi = rowok ? x[row] : 0.0, yi = rowok ? y[row] : 0.0;
  f32x4 acc[kTB];
#pragma unroll
  for (int t = 0; t < kTB; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t j0 = 0; j0 < n; j0 += kKB) {
    __syncthreads();
    for (int idx = tid; idx < kKB * kColsB; idx += 256) {
      const int jj = idx / kColsB, cc = idx % kColsB;
      const int64_t j = j0 + jj;
      const int c = c0 + cc;
      double v = 0.0;
      if (j < n && cc < ncol) v = (c < s) ? Om[j * ld + c] : Ps[j * ld + (c - s)];
      split_bf16((float)v, Bhi[cc][jj], Blo[cc][jj]);
    }
    if (tid < kKB) {
      const int64_t j = j0 + tid;
      xsh[tid] = (j < n) ? x[j] : 0.0;
      ysh[tid] = (j < n) ? y[j] : 0.0;
    }
    __syncthreads();
    bf16x8 ah, al;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int jj = 8 * (lane >> 4) + r;
      const int64_t j = j0 + jj;
      const double dx = xi - xsh[jj], dy = yi - ysh[jj];
      const float a = (rowok && j < n && j != row) ? 0.5f * logf((float)(dx * dx + dy * dy)) : 0.f;
      __bf16 h, l;
      split_bf16(a, h, l);
      ah[r] = h;
      al[r] = l;
    }
#pragma unroll
    for (int t = 0; t < kTB; ++t) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Bhi[t * 16 + (lane & 15)][8 * (lane >> 4)]);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Blo[t * 16 + (lane & 15)][8 * (lane >> 4)]);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[t], 0, 0, 0);
    }
  }
  const int64_t rbase = row0 + (int64_t)blockIdx.x * kRows + wave * 16 + 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < kTB; ++t) {
    const int cc = t * 16 + (lane & 15);
    if (cc < ncol) {
      const int c = c0 + cc;
      double* out = (c < s) ? Yo + c : Zo + (c - s);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = rbase + r;
        if (rr < row1) out[rr * ld] = (double)acc[t][r];
      }
    }
  }
}

}  // namespace

hipError_t launch_logkernel(int64_t n, const double* x, const double* y, const double* Om, const double* Ps,
                            double* Y, double* Z, int32_t s, int64_t ld, hbs_precision prec, hipStream_t st,
                            int64_t row0, int64_t row1) {
  if (row1 < 0) row1 = n;
  if (row0 < 0 || row1 > n || row0 > row1) return hipErrorInvalidValue;
  if (row0 == row1) return hipSuccess;
  const unsigned gx = (unsigned)((row1 - row0 + kRows - 1) / kRows);
  if (prec == HBS_BF16) {
    dim3 grid(gx, (2 * s + kColsB - 1) / kColsB);
    hipLaunchKernelGGL(logkernel_bf16, grid, dim3(256), 0, st, n, x, y, Om, Ps, Y, Z, s, ld, row0, row1);
    return hipGetLastError();
  }
  if (prec != HBS_FP64) return hipErrorInvalidValue;
  const int nchunk = (s + kCols - 1) / kCols;
  dim3 grid(gx, 2 * nchunk);
  hipLaunchKernelGGL(logkernel_f64, grid, dim3(256), 0, st, n, x, y, Om, Ps, Y, Z, s, ld, nchunk, row0, row1);
  return hipGetLastError();
}

}  // namespace hbs
