// Accuracy report of section 5: the operator-norm estimate by power
// iteration (20 steps in the paper) of the difference between the compressed
// operator and a black box, and a one-vector matvec of the log-kernel stand-in
// black box to drive it.
//
// The estimate for an operator E (E = A~ - B, or A~ or B alone):
//   v_0 given; v_i = E^* E (v_{i-1} / ||v_{i-1}||), i = 1 .. steps;
//   ||E||_2 ~= sqrt(||v_steps||).
// Sums of squares go through a fixed two-level reduction (no atomics), so
// the result does not depend on scheduling.
#include <algorithm>
#include <cmath>

#include "hbs_internal.h"

namespace hbs {
namespace {

constexpr int kRedBlocks = 256;  // partial sums per reduction
constexpr int kRedThreads = 256;

// part[b] = sum of v[i]^2 over the indices block b owns (grid-strided, in a
// fixed order), then a fixed LDS tree.
__global__ void __launch_bounds__(kRedThreads) sumsq_partial(const double* __restrict__ v, int64_t n,
                                                            double* __restrict__ part) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)kRedBlocks * kRedThreads)
    acc += v[i] * v[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The total of the kRedBlocks partial sums, in the same fixed tree order.
__device__ double sum_parts(const double* __restrict__ part, double* red) {
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

// x = v / ||v||, ||v||^2 being the sum of part[0 .. kRedBlocks - 1]; x = 0
// when v = 0 (E v_{i-1} vanished: the estimate is then 0).
__global__ void __launch_bounds__(kRedThreads) scale_unit(const double* __restrict__ v,
                                                         const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ x) {
  __shared__ double red[kRedThreads];
  const double ss = sum_parts(part, red);
  const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    x[i] = v[i] * inv;
}

// out[0] = sum of part[0 .. kRedBlocks - 1].
__global__ void __launch_bounds__(kRedThreads) sum_total(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  const double t = sum_parts(part, red);
  if (threadIdx.x == 0) out[0] = t;
}

// w -= t
__global__ void __launch_bounds__(kRedThreads) sub_inplace(double* __restrict__ w, const double* __restrict__ t,
                                                          int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    w[i] -= t[i];
}

// y = A v for the log kernel A(i, j) = log|p_i - p_j| = (1/2) log r_ij^2
// (i != j), A(i, i) = 0.  A workgroup owns 64 rows; its 4 waves take every
// fourth point of each staged chunk of 256 points, and their 4 partial sums
// are added in a fixed order at the end.
constexpr int kMvRows = 64;
constexpr int kMvChunk = 256;

__global__ void __launch_bounds__(256) logkernel_matvec(int64_t n, const double* __restrict__ px,
                                                       const double* __restrict__ py, const double* __restrict__ v,
                                                       double* __restrict__ y) {
  __shared__ double xs[kMvChunk], ys[kMvChunk], vs[kMvChunk];
  __shared__ double part[4][kMvRows];
  const int tid = threadIdx.x, r = tid & 63, q = tid >> 6;
  const int64_t i = (int64_t)blockIdx.x * kMvRows + r;
  const bool ok = i < n;
  const double xi = ok ? px[i] : 0.0, yi = ok ? py[i] : 0.0;
  double acc = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kMvChunk) {
    const int64_t j = j0 + tid;
    const bool jok = j < n;
    xs[tid] = jok ? px[j] : 0.0;
    ys[tid] = jok ? py[j] : 0.0;
    vs[tid] = jok ? v[j] : 0.0;
    __syncthreads();
    const int cnt = (n - j0) < kMvChunk ? (int)(n - j0) : kMvChunk;
    for (int u = q; u < cnt; u += 4) {
      const double dx = xi - xs[u], dy = yi - ys[u];
      const double term = 0.5 * log(dx * dx + dy * dy) * vs[u];
      acc += (j0 + u == i) ? 0.0 : term;
    }
    __syncthreads();
  }
  part[q][r] = acc;
  __syncthreads();
  if (q == 0 && ok) y[i] = ((part[0][r] + part[1][r]) + part[2][r]) + part[3][r];
}

}  // namespace
}  // namespace hbs

namespace {

#define MET_TRY(x)                                            \
  do {                                                        \
    hipError_t e_ = (x);                                      \
    if (e_ != hipSuccess) {                                   \
      st = (e_ == hipErrorOutOfMemory) ? HBS_ENOMEM : HBS_EDEVICE; \
      goto done;                                              \
    }                                                         \
  } while (0)
#define MET_CALL(x)          \
  do {                       \
    st = (x);                \
    if (st != HBS_OK) goto done; \
  } while (0)

// w = E x: A~ x and/or B x, their difference when both are present
hbs_status apply_e(hbs_factors* f, hbs_matvec bb, void* ctx, int transpose, const double* x, double* w,
                   double* t, int64_t n, hipStream_t s) {
  hbs_status st = HBS_OK;
  if (f) {
    st = hbs_apply(f, transpose, x, w, 1, 1, s);
    if (st != HBS_OK) return st;
  }
  if (bb) {
    st = bb(ctx, transpose, x, f ? t : w, s);
    if (st != HBS_OK) return st;
    if (f) {
      const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
      hipLaunchKernelGGL(hbs::sub_inplace, dim3(g), dim3(256), 0, s, w, t, n);
      if (hipGetLastError() != hipSuccess) return HBS_EDEVICE;
    }
  }
  return HBS_OK;
}

}  // namespace

extern "C" {

hbs_status hbs_power_norm(hbs_factors* f, hbs_matvec black_box, void* ctx, int64_t n, const double* v0,
                          int32_t steps, double* out, void* hip_stream) {
  if ((!f && !black_box) || n < 1 || !v0 || steps < 1 || !out) return HBS_EINVAL;
  if (f && hbs::factors_n(f) != n) return HBS_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  hbs_status st = HBS_OK;
  double *v = nullptr, *x = nullptr, *w = nullptr, *t = nullptr, *part = nullptr, *tot = nullptr;
  double h_tot = 0.0;
  const int g = (int)std::min<int64_t>((n + 255) / 256, 4096);
  MET_TRY(hipMalloc((void**)&v, sizeof(double) * n));
  MET_TRY(hipMalloc((void**)&x, sizeof(double) * n));
  MET_TRY(hipMalloc((void**)&w, sizeof(double) * n));
  MET_TRY(hipMalloc((void**)&t, sizeof(double) * n));
  MET_TRY(hipMalloc((void**)&part, sizeof(double) * (hbs::kRedBlocks + 1)));
  tot = part + hbs::kRedBlocks;
  MET_TRY(hipMemcpyAsync(v, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  for (int i = 0; i < steps; ++i) {
    hipLaunchKernelGGL(hbs::sumsq_partial, dim3(hbs::kRedBlocks), dim3(hbs::kRedThreads), 0, s, v, n, part);
    hipLaunchKernelGGL(hbs::scale_unit, dim3(g), dim3(hbs::kRedThreads), 0, s, v, part, n, x);
    MET_TRY(hipGetLastError());
    MET_CALL(apply_e(f, black_box, ctx, 0, x, w, t, n, s));  // w = E x
    MET_CALL(apply_e(f, black_box, ctx, 1, w, v, t, n, s));  // v = E^* w
  }
  hipLaunchKernelGGL(hbs::sumsq_partial, dim3(hbs::kRedBlocks), dim3(hbs::kRedThreads), 0, s, v, n, part);
  hipLaunchKernelGGL(hbs::sum_total, dim3(1), dim3(hbs::kRedThreads), 0, s, part, tot);
  MET_TRY(hipGetLastError());
  MET_TRY(hipMemcpyAsync(&h_tot, tot, sizeof(double), hipMemcpyDeviceToHost, s));
  MET_TRY(hipStreamSynchronize(s));
  *out = std::sqrt(std::sqrt(h_tot));
done:
  if (st != HBS_OK) (void)hipStreamSynchronize(s);
  (void)hipFree(v);
  (void)hipFree(x);
  (void)hipFree(w);
  (void)hipFree(t);
  (void)hipFree(part);
  return st;
}

hbs_status hbs_matvec_factors(void* ctx, int32_t transpose, const double* x, double* y, void* hip_stream) {
  if (!ctx) return HBS_EINVAL;
  return hbs_apply(static_cast<hbs_factors*>(ctx), transpose, x, y, 1, 1, hip_stream);
}

hbs_status hbs_matvec_logkernel(void* ctx, int32_t transpose, const double* x, double* y, void* hip_stream) {
  (void)transpose;  // the log kernel is symmetric
  const hbs_logkernel_points* p = static_cast<const hbs_logkernel_points*>(ctx);
  if (!p || p->n < 1 || !p->x || !p->y || !x || !y) return HBS_EINVAL;
  const int64_t nb = (p->n + hbs::kMvRows - 1) / hbs::kMvRows;
  hipLaunchKernelGGL(hbs::logkernel_matvec, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)hip_stream, p->n, p->x,
                     p->y, x, y);
  return hipGetLastError() == hipSuccess ? HBS_OK : HBS_EDEVICE;
}

}  // extern "C"
