// The per-box products that follow the bases U_tau, V_tau on one level:
// D_tau (eq. d_tau_formula) and the four k x s blocks each child hands to its
// parent (eq. omega_tau_and_y_tau; Psi and Z as in Algorithm 2).
//
// With W = Y_tau Omega_tau^dagger and X = Z_tau Psi_tau^dagger, eq.
// d_tau_formula reads D = W - U T with
//   E = (I - V V^*) X U,   T = U^* W - E^*.
// Since U^* U = V^* V = I, the two products that eq. omega_tau_and_y_tau
// takes with D simplify:
//   U^* D = U^* W - T = E^*,         so U^* (Y - D Omega) = U^* Y - E^* Omega,
//   D V   = W V - U U^* W V =: H,    so V^* (Z - D^* Psi) = V^* Z - H^* Psi,
// and the parent blocks no longer wait for D.  Three launches per level:
//   tail_a  F = X U, Q = W V, T0 = U^* W;
//   tail_b  G = V^* F, G2 = U^* Q, E = F - V G, H = Q - U G2, T = T0 - E^*
//           (two chains, split by rows);
//   tail_c  D = W - U T, and the parent blocks, one product per side and
//           64-column tile of s: Omega' = V^* Omega with Y' = U^* Y - E^* Omega,
//           Psi' = U^* Psi with Z' = V^* Z - H^* Psi (each panel read once).
// The parent blocks (every product with a test or sample panel) run in FP64
// on the matrix cores, or split-precision (parent_sliced) when the batch
// asks for it; everything that forms D stays FP64.
#include "hbs_gemm.h"
#include "hbs_internal.h"

namespace hbs {
namespace {

// Split-precision products cut every operand into S exact 7-bit slices (7 S
// bits: 8 gives FP64-level error per product); S = 0 is the FP64 path.
template <int S>
struct TailSmem {
  union {
    MfmaSmem<16> g;
    SliceSmem<S> sl;
  };
};
template <>
struct TailSmem<0> {
  MfmaSmem<16> g;
};

// Workspace of one box: F | Q | E | H (dld x k each) | T0 | T (k x dld each) |
// G: one k x k product per chain and row block (2 ceil(dld / 64) of them).
struct TailWs {
  double *F, *Q, *E, *H, *T0, *T, *G;
  __device__ TailWs(double* base, int dld, int k) {
    const int64_t mk = (int64_t)dld * k;
    F = base;
    Q = F + mk;
    E = Q + mk;
    H = E + mk;
    T0 = H + mk;
    T = T0 + mk;
    G = T + mk;
  }
};

// XCD-aware tile order (tail_a, tail_c).  The workgroups of a launch are
// dealt to the chip's 8 XCDs in turn, in dispatch order (workgroup i to XCD
// i % 8), and each XCD has its own L2.  The ny tiles of one box read the same
// basis, W, X and panels, so they are given consecutive slots on one XCD:
// box x + 8 (l / ny) and tile l % ny for workgroup i = 8 l + x.  The grid
// holds ny tiles for every box of the box count rounded up to 8; the padding
// workgroups return at once.  The x extent is capped at 2^21 workgroups (a
// multiple of 8, so i % 8 is still the XCD) and rows of y carry the rest,
// which keeps grid x times workgroup size within the 32-bit launch limit at
// any box count.  (tail_b's two chains share no operand and keep the plain
// two-dimensional grid, which measured faster.)
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kXcds = 8;
constexpr int64_t kXcdGridX = (int64_t)1 << 21;

struct XcdTile {
  int box, y;
};
__device__ __forceinline__ XcdTile xcd_tile(int ny) {
  // 32-bit index arithmetic: launch_tail refuses grids of 2^31 workgroups
  const unsigned i = blockIdx.x + gridDim.x * blockIdx.y, l = i / kXcds;
  return XcdTile{(int)(i % kXcds + kXcds * (l / (unsigned)ny)), (int)(l % (unsigned)ny)};
}
inline int64_t xcd_total(int nboxes, int ny) { return (int64_t)((nboxes + kXcds - 1) / kXcds) * kXcds * ny; }
inline dim3 xcd_grid(int nboxes, int ny) {
  const int64_t total = xcd_total(nboxes, ny);
  const int64_t gx = total < kXcdGridX ? total : kXcdGridX;
  return dim3((unsigned)gx, (unsigned)((total + gx - 1) / gx));
}

// The parent blocks of one side of a box for one 64-column tile of s.  Split
// products over boxes of more than 64 rows (two staging chunks) run as three
// separate products (P0 sliced twice): the fused product with two chunks
// needs more than the 256 registers a lane can have.
template <int S, int KCH>
__device__ __forceinline__ void parent(TailSmem<S>& sm, const ParentOp& op) {
  if constexpr (S > 0 && KCH > 1) {
    // (the scheduling barriers keep each product's loads from being hoisted
    // into the one before, which would exceed the register file)
    sliced_lt<S, KCH>(op.k, op.nc, op.m, 1.0, op.B1, op.k, op.P0, op.ld, 0.0, nullptr, 0, op.top, op.ldo, sm.sl);
    __builtin_amdgcn_sched_barrier(0);
    sliced_lt<S, KCH>(op.k, op.nc, op.m, 1.0, op.B3, op.k, op.P1, op.ld, 0.0, nullptr, 0, op.bot, op.ldo, sm.sl);
    __builtin_amdgcn_sched_barrier(0);
    sliced_lt<S, KCH>(op.k, op.nc, op.m, -1.0, op.B2, op.k, op.P0, op.ld, 1.0, op.bot, op.ldo, op.bot, op.ldo, sm.sl);
  } else if constexpr (S > 0) {
    parent_sliced<S, KCH>(op, sm.sl);
  } else {
    parent_mfma<16>(op, sm.g);
  }
}

// FP64 product by the workgroup of either tail variant
template <int S>
__device__ __forceinline__ void dgemm(TailSmem<S>& sm, int M, int N, int K, double alpha, const double* A, int sar,
                                      int sac, const double* B, int sbr, int sbc, double beta, const double* C0,
                                      int ldc0, double* C, int ldc) {
  mfma_gemm<16, (S > 0 ? kSliceThreads : kGemmThreads)>(M, N, K, alpha, A, sar, sac, B, sbr, sbc, beta, C0, ldc0, C,
                                                      ldc, sm.g);
}

template <int S>
constexpr int tail_threads() { return S > 0 ? kSliceThreads : kGemmThreads; }
// the fewest waves per SIMD the register allocation must leave room for (0:
// the compiler's choice): 4 for the one-chunk split products (at most 128
// registers a lane), so that two of their 8-wave workgroups share a compute
// unit and hide each other's slicing and barriers
template <int S, int KCH>
constexpr int tail_min_waves() { return 0; }

// grid (boxes, 3 mt): mt = row tiles of the box; FP64 on both paths (held to
// 4 waves per SIMD, which it fits in 128 registers without scratch)
__global__ void __launch_bounds__(kGemmThreads, 4) tail_a_kernel(SweepArgs a) {
  __shared__ MfmaSmem<16> sm;
  const int mt = (a.mmax + 63) / 64;
  const XcdTile tl = xcd_tile(3 * mt);
  if (tl.box >= a.nboxes) return;
  const BoxDesc& bx = a.box[tl.box];
  const int m = bx.m, k = a.k, dld = bx.dld;
  const int y = tl.y;
  const int which = y / mt, r0 = (y % mt) * 64;
  if (r0 >= m) return;
  const int nr = min(64, m - r0);
  TailWs ws(bx.T, dld, k);
  if (which == 0)  // F = X U (rows r0..)
    mfma_gemm<16>(nr, k, m, 1.0, bx.X + (int64_t)r0 * dld, dld, 1, bx.U, k, 1, 0.0, nullptr, 0,
                  ws.F + (int64_t)r0 * k, k, sm);
  else if (which == 1)  // Q = W V
    mfma_gemm<16>(nr, k, m, 1.0, bx.W + (int64_t)r0 * dld, dld, 1, bx.V, k, 1, 0.0, nullptr, 0,
                  ws.Q + (int64_t)r0 * k, k, sm);
  else  // T0 = U^* W (columns r0..)
    mfma_gemm<16>(k, nr, m, 1.0, bx.U, 1, k, bx.W + r0, dld, 1, 0.0, nullptr, 0, ws.T0 + r0, dld, sm);
}

// grid (boxes, 2 nrb): chain 0 forms G = V^* F, then rows of E = F - V G and
// the matching columns of T = T0 - E^*; chain 1 forms G2 = U^* Q, then rows of
// H = Q - U G2.  With nrb > 1 (levels of few boxes) every 64-row block
// recomputes its chain's k x k product (into its own slot) so that the blocks
// run independently.
// (the one-chunk-per-16 variant is held to 4 waves per SIMD, which it fits
// in 128 registers without scratch: twice the workgroups per compute unit to
// hide its load latencies)
template <int TK>
__global__ void __launch_bounds__(kGemmThreads, (TK == 16 ? 4 : 0)) tail_b_kernel(SweepArgs a) {
  __shared__ MfmaSmem<TK> sm;
  const BoxDesc& bx = a.box[blockIdx.x];
  const int m = bx.m, k = a.k, dld = bx.dld;
  const int nrb = gridDim.y / 2;  // row blocks per chain: 1, or one per 64 rows
  const int chain = blockIdx.y / nrb, rb = blockIdx.y % nrb, r0 = rb * 64;
  if (r0 >= m) return;
  const int nr = (nrb == 1) ? m : min(64, m - r0);
  TailWs ws(bx.T, dld, k);
  const double* B1 = chain ? bx.U : bx.V;   // basis of the k x k product
  const double* B2 = chain ? ws.Q : ws.F;   // its m x k partner
  double* Gs = ws.G + (int64_t)(chain * nrb + rb) * k * k;
  double* Out = chain ? ws.H : ws.E;
  mfma_gemm<TK>(k, k, m, 1.0, B1, 1, k, B2, k, 1, 0.0, nullptr, 0, Gs, k, sm);
  mfma_gemm<TK>(nr, k, k, -1.0, B1 + (int64_t)r0 * k, k, 1, Gs, k, 1, 1.0, B2 + (int64_t)r0 * k, k,
                Out + (int64_t)r0 * k, k, sm);
  if (chain == 0)
    for (int idx = threadIdx.x; idx < k * nr; idx += blockDim.x) {
      const int i = idx / nr, j = r0 + idx % nr;
      ws.T[i * dld + j] = ws.T0[i * dld + j] - ws.E[j * k + i];
    }
}

// tail_b for boxes of at most 64 rows and k <= 32 (variant 2), grid (boxes,
// 2 chains): both m x k operands of the chain are staged in LDS at once (all
// loads in flight together, one wait instead of one per 16-deep chunk), then
// G = B1^* B2 and Out = B2 - B1 G on the matrix cores from LDS, and for
// chain 0 T = T0 - E^* through LDS.  Rows past m and columns past k are zero.
constexpr int kSmallM = 64, kSmallK = 32;
struct SmallBSmem {
  double b1[kSmallM][kSmallK + 1];  // B1 = V or U (m x k); later E or H
  double b2[kSmallM][kSmallK + 1];  // B2 = F or Q (m x k)
  double g[kSmallK][kSmallK + 1];   // G = B1^* B2 (k x k)
};
__global__ void __launch_bounds__(kGemmThreads) tail_b_small_kernel(SweepArgs a) {
  __shared__ SmallBSmem sm;
  const BoxDesc& bx = a.box[blockIdx.x];
  const int m = bx.m, k = a.k, dld = bx.dld;
  const int chain = blockIdx.y;
  TailWs ws(bx.T, dld, k);
  const double* B1 = chain ? bx.U : bx.V;
  const double* B2 = chain ? ws.Q : ws.F;
  double* Out = chain ? ws.H : ws.E;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // ---- stage B1, B2 (row-major m x k, row stride k) ------------------------
  constexpr int PER = kSmallM * kSmallK / kGemmThreads;  // 8 per thread and operand
  double v1[PER], v2[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + kGemmThreads * q, i = idx / kSmallK, j = idx % kSmallK;
    const bool ok = i < m && j < k;
    const double x1 = B1[ok ? i * k + j : 0], x2 = B2[ok ? i * k + j : 0];
    v1[q] = ok ? x1 : 0.0;
    v2[q] = ok ? x2 : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + kGemmThreads * q, i = idx / kSmallK, j = idx % kSmallK;
    sm.b1[i][j] = v1[q];
    sm.b2[i][j] = v2[q];
  }
  __syncthreads();
  // ---- G = B1^* B2: 16 x 16 tiles of G, one per wave, K = 64 rows ---------
  // (v_mfma_f64_16x16x4f64: lane l supplies A(l % 16, l / 16), B(l / 16,
  // l % 16) and receives C(l / 16 + 4 e, l % 16) in element e)
  const int kt = (k + 15) / 16;
  if (wv < kt * kt) {
    const int i0 = 16 * (wv / kt), j0 = 16 * (wv % kt);
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kSmallM; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sm.b1[kk + lk][i0 + li], sm.b2[kk + lk][j0 + li], acc, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) sm.g[i0 + lk + 4 * e][j0 + li] = acc[e];
  }
  __syncthreads();
  // ---- Out = B2 - B1 G: (m/16) x (k/16) tiles dealt to the waves, K = k ----
  const int mtl = (m + 15) / 16, nt = mtl * kt;
  f64x4 oacc[2];  // at most 4 x 2 tiles over 4 waves
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    oacc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int tile = wv + 4 * t;
    if (tile < nt) {
      const int i0 = 16 * (tile / kt), j0 = 16 * (tile % kt);
#pragma unroll
      for (int kk = 0; kk < kSmallK; kk += 4)
        if (kk < 16 * kt)
          oacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sm.b1[i0 + li][kk + lk], sm.g[kk + lk][j0 + li], oacc[t],
                                                         0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read B1 before it is overwritten with Out
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int tile = wv + 4 * t;
    if (tile < nt) {
      const int i0 = 16 * (tile / kt), j0 = 16 * (tile % kt);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + lk + 4 * e, j = j0 + li;
        const double o = sm.b2[i][j] - oacc[t][e];
        sm.b1[i][j] = o;
        if (i < m && j < k) Out[i * k + j] = o;
      }
    }
  }
  if (chain == 0) {
    __syncthreads();
    // T = T0 - E^* (k x m, row stride dld)
    for (int idx = tid; idx < k * m; idx += kGemmThreads) {
      const int i = idx / m, j = idx % m;
      ws.T[i * dld + j] = ws.T0[i * dld + j] - sm.b1[j][i];
    }
  }
}

// grid (boxes, mt^2 + 2 st)
template <int S, int KCH = kSliceChunks>
__global__ void __launch_bounds__(tail_threads<S>(), (tail_min_waves<S, KCH>())) tail_c_kernel(SweepArgs a) {
  __shared__ TailSmem<S> sm;
  const int mt = (a.mmax + 63) / 64;
  const XcdTile tl = xcd_tile(mt * mt + 2 * ((a.s + 63) / 64));
  if (tl.box >= a.nboxes) return;
  const BoxDesc& bx = a.box[tl.box];
  const int m = bx.m, k = a.k, s = a.s, dld = bx.dld;
  const int y = tl.y;
  TailWs ws(bx.T, dld, k);
  if (y < mt * mt) {  // D = W - U T, one 64 x 64 tile
    const int r0 = (y / mt) * 64, c0 = (y % mt) * 64;
    if (r0 >= m || c0 >= m) return;
    dgemm<S>(sm, min(64, m - r0), min(64, m - c0), k, -1.0, bx.U + (int64_t)r0 * k, k, 1, ws.T + c0, dld, 1,
                 1.0, bx.W + (int64_t)r0 * dld + c0, dld, bx.D + (int64_t)r0 * dld + c0, dld);
    return;
  }
  const int st = (s + 63) / 64;
  const int q = y - mt * mt, side = q / st, c0 = (q % st) * 64;
  if (c0 >= s) return;
  const PanelSrc& ps = a.src[bx.src];
  // side 0: Omega' = V^* Omega, Y' = U^* Y - E^* Omega;
  // side 1: Psi' = U^* Psi, Z' = V^* Z - H^* Psi
  ParentOp op;
  op.B1 = side ? bx.U : bx.V;
  op.B2 = side ? ws.H : ws.E;
  op.B3 = side ? bx.V : bx.U;
  op.ld = ps.ld;
  op.P0 = ps.p[2 * side] + bx.row0 * op.ld + c0;
  op.P1 = ps.p[2 * side + 1] + bx.row0 * op.ld + c0;
  op.top = bx.np[2 * side] + c0;
  op.bot = bx.np[2 * side + 1] + c0;
  op.ldo = s;
  op.m = m;
  op.k = k;
  op.nc = min(64, s - c0);
  parent<S, KCH>(sm, op);
}

}  // namespace

size_t tail_workspace(int dld, int k) {
  return 6 * (size_t)dld * k + 2 * (size_t)((dld + 63) / 64) * k * k;
}

int tail_mixed_max_rows() { return kSliceChunks * kSliceK; }

// few boxes: latency bound, row blocks in parallel and deeper K chunks
int tail_b_default(const SweepArgs& a) { return a.nboxes < 256 ? 1 : 0; }
int tail_b_variants(const SweepArgs& a) { return (a.k <= kSmallK && a.mmax <= kSmallM) ? 3 : 2; }

namespace {

// the split-precision launch of tail_a or tail_c for S slices, with one
// staging chunk when the boxes have at most kSliceK rows
struct TailC {
  template <int S, int KCH>
  static void launch(dim3 grid, hipStream_t st, const SweepArgs& a) {
    hipLaunchKernelGGL((tail_c_kernel<S, KCH>), grid, dim3(kSliceThreads), 0, st, a);
  }
};
template <class K>
void launch_sliced(int slices, bool one_chunk, dim3 grid, hipStream_t st, const SweepArgs& a) {
  switch (slices * 2 + (one_chunk ? 1 : 0)) {
    case 12: K::template launch<6, kSliceChunks>(grid, st, a); break;
    case 13: K::template launch<6, 1>(grid, st, a); break;
    case 14: K::template launch<7, kSliceChunks>(grid, st, a); break;
    case 15: K::template launch<7, 1>(grid, st, a); break;
    case 16: K::template launch<8, kSliceChunks>(grid, st, a); break;
    default: K::template launch<8, 1>(grid, st, a); break;
  }
}

}  // namespace

hipError_t launch_tail(const SweepArgs& a, int part, int variant, hipStream_t st) {
  const int mt = (a.mmax + 63) / 64, sct = (a.s + 63) / 64;
  if (a.mixed && a.mmax > kSliceChunks * kSliceK) return hipErrorInvalidValue;  // split products contract over <= 128 rows
  if (xcd_total(a.nboxes, 3 * mt > mt * mt + 2 * sct ? 3 * mt : mt * mt + 2 * sct) >= ((int64_t)1 << 31))
    return hipErrorInvalidValue;
  if (a.mixed && (a.slices < 6 || a.slices > 8)) return hipErrorInvalidValue;
  if (part == 0) {
    hipLaunchKernelGGL(tail_a_kernel, xcd_grid(a.nboxes, 3 * mt), dim3(kGemmThreads), 0, st, a);
  } else if (part == 1) {
    if (variant < 0) variant = tail_b_default(a);
    if (variant == 2) {
      if (a.k > kSmallK || a.mmax > kSmallM) return hipErrorInvalidValue;
      hipLaunchKernelGGL(tail_b_small_kernel, dim3(a.nboxes, 2), dim3(kGemmThreads), 0, st, a);
    } else if (variant == 1)
      hipLaunchKernelGGL(tail_b_kernel<32>, dim3(a.nboxes, 2 * mt), dim3(kGemmThreads), 0, st, a);
    else
      hipLaunchKernelGGL(tail_b_kernel<16>, dim3(a.nboxes, 2), dim3(kGemmThreads), 0, st, a);
  } else {
    const dim3 grid = xcd_grid(a.nboxes, mt * mt + 2 * sct);
    if (!a.mixed)
      hipLaunchKernelGGL(tail_c_kernel<0>, grid, dim3(kGemmThreads), 0, st, a);
    else
      launch_sliced<TailC>(a.slices, a.mmax <= kSliceK, grid, st, a);
  }
  return hipGetLastError();
}

}  // namespace hbs
