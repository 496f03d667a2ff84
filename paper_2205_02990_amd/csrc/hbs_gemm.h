// Workgroup-level products on the matrix cores of gfx950, called by every
// thread of a workgroup:
//   mfma_gemm  FP64 products on v_mfma_f64_16x16x4f64;
//   sliced_lt  the split-precision product L^T R: both operands cut into
//              exact 7-bit integer slices (one power-of-two scale per row of
//              L^T and per column of R), the slice pairs multiplied exactly on
//              v_mfma_i32_16x16x64_i8 with 32-bit integer sums, recombined in
//              FP64 (error-free slicing in the manner of Ozaki, Ogita, Oishi
//              and Rump, with integer slices);
//   parent_mfma / parent_sliced  the two parent blocks of one side of a box
//              as one product over two blocks of contracted indices (FP64,
//              or sliced with scales of their own per block).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace hbs {

constexpr int kGemmThreads = 256;   // FP64 product workgroups
constexpr int kSliceThreads = 512;  // split-precision product workgroups

typedef double gemm_d4 __attribute__((ext_vector_type(4)));
typedef int gemm_i4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP64: C(i, j) = alpha * sum_kk A(i, kk) B(kk, j) + beta * C0(i, j), i < M,
// j < N, with A(i, kk) = A[i * sar + kk * sac], B(kk, j) = B[kk * sbr + j * sbc]
// (strides express transposes; all offsets within one box's blocks, so they
// are 32-bit, which keeps the address arithmetic in fewer registers).  64 x 64
// output tiles; with NT = 256 threads
// each wave owns a 32 x 32 quarter (2 x 2 MFMA blocks of 16 x 16), with 512 a
// 16 x 32 eighth (1 x 2 blocks).  K is staged through LDS
// in chunks of TK with the next chunk's global loads in flight during the
// products.  C0 may alias C.  Ends with a barrier.
//
// Lane layouts of v_mfma_f64_16x16x4f64: lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16) and receives C(l / 16 + 4 r, l % 16) in element r.
template <int TK>
struct MfmaSmem {
  double As[TK][65];  // As[kk][i]
  double Bs[TK][65];  // Bs[kk][j]
};

template <int TK, int NT = kGemmThreads>
__device__ __forceinline__ void mfma_gemm(int M, int N, int K, double alpha, const double* __restrict__ A, int sar,
                                          int sac, const double* __restrict__ B, int sbr, int sbc, double beta,
                                          const double* C0, int ldc0, double* C, int ldc, MfmaSmem<TK>& sm) {
  static_assert(TK % 4 == 0, "K chunk must be a multiple of the MFMA depth");
  static_assert(NT == 256 || NT == 512, "4 or 8 waves");
  constexpr int LA = 64 * TK / NT;
  constexpr int TR = (NT == 256) ? 2 : 1;  // 16-row blocks per wave
  static_assert(LA >= 1, "chunk too small for the workgroup");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rb = (wv >> 1) * 16 * TR, cb = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // staging coordinates: coalesced along whichever index is contiguous
  int ai[LA], ak[LA], bj[LA], bk[LA];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int idx = tid + r * NT;
    ai[r] = (sac == 1) ? idx / TK : idx % 64;
    ak[r] = (sac == 1) ? idx % TK : idx / 64;
    bj[r] = (sbc == 1) ? idx % 64 : idx / TK;
    bk[r] = (sbc == 1) ? idx / 64 : idx % TK;
  }
  for (int i0 = 0; i0 < M; i0 += 64) {
    for (int j0 = 0; j0 < N; j0 += 64) {
      gemm_d4 acc[TR][2];
#pragma unroll
      for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
      double pa[LA], pb[LA];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
          const int gi = i0 + ai[r], gk = k0 + ak[r];
          const bool ok = gi < M && gk < K;
          const double v = A[ok ? gi * sar + gk * sac : 0];
          pa[r] = ok ? v : 0.0;
        }
#pragma unroll
        for (int r = 0; r < LA; ++r) {
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
        for (int r = 0; r < LA; ++r) sm.Bs[bk[r]][bj[r]] = pb[r];
        __syncthreads();
        if (k0 + TK < K) fetch(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
          const double b0 = sm.Bs[kk + lk][cb + li], b1 = sm.Bs[kk + lk][cb + 16 + li];
#pragma unroll
          for (int a = 0; a < TR; ++a) {
            const double av = sm.As[kk + lk][rb + 16 * a + li];
            acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[a][0], 0, 0, 0);
            acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[a][1], 0, 0, 0);
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + rb + 16 * a + lk + 4 * r, gj = j0 + cb + 16 * b + li;
            if (gi < M && gj < N) {
              const double v = alpha * acc[a][b][r];
              C[gi * ldc + gj] = (beta != 0.0) ? beta * C0[gi * ldc0 + gj] + v : v;
            }
          }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Split precision: C(i, j) = alpha * sum_kk L(kk, i) R(kk, j) + beta * C0(i, j)
// for i < M, j < N, kk < K, with L(kk, i) = L[kk * ldl + i] and
// R(kk, j) = R[kk * ldr + j] (row-major, the output index contiguous).
//
// Row i of L^T is scaled by 2^-e_i with e_i the binary exponent of its
// largest magnitude (so every scaled entry lies in (-1, 1)), column j of R by
// 2^-f_j likewise.  A scaled entry t is cut into S integer slices
// q_p = trunc(128 t_p), t_{p+1} = 128 t_p - q_p (t_1 = t), so that
// t = sum_p q_p 2^(-7p) + a remainder below 2^(-7S); each q_p lies in
// [-127, 127].  Products of slice pairs (p, q) with p + q <= S + 1 are exact
// in 32-bit integer sums (at most S pairs per diagonal: |sum| <= S K 127^2,
// below 2^31 for K < 2^31 / (S 127^2), 16600 at S = 8) and
// are accumulated per diagonal p + q; the diagonals are combined in FP64:
//   C(i, j) ~ 2^(e_i + f_j) sum_d 2^(-7 d) acc_d(i, j).
// Dropped pairs and slice remainders bound the error of each entry by about
// (S + 3) K 2^(-7S) max|L(., i)| max|R(., j)|.
//
// Lane layouts of v_mfma_i32_16x16x64_i8: lane l supplies 16 bytes of row
// l % 16 of the left operand and of column l % 16 of the right operand, for
// the same 16 values of the contracted index (l / 16 selects which 16); it
// receives C(4 (l / 16) + r, l % 16) in element r.  Called by the 512
// threads of a workgroup; each of its 8 waves owns a 16 x 32 strip of each
// 64 x 64 output tile.
constexpr int kSliceK = 64;                       // contracted indices per LDS chunk
constexpr int kSliceRow = kSliceK / 4;            // int32 words per slice row
constexpr int kSliceGroups = kSliceThreads / 64;  // contracted-index groups in staging
constexpr int kSlicePer = kSliceK / kSliceGroups; // contracted indices per staging thread

// The 16-byte blocks of a slice row are stored XOR-swizzled by row so that
// the 16 rows one MFMA operand read touches fall in distinct LDS banks.
__device__ __forceinline__ int slice_word(int row, int word) {
  return ((((word >> 2) ^ (row >> 2)) & 3) << 2) | (word & 3);
}

template <int S>
struct SliceSmem {
  union {
    struct {
      int32_t As[S][64][kSliceRow];  // As[p][i][.]: four slices q_p of L(kk, i) per word
      int32_t Bs[S][64][kSliceRow];
    } q;
    double red[2][kSliceGroups][64];  // partial maxima (before any slicing)
  } u;
  int ea[64], eb[64];                 // scale exponents
};

// Cut 4 values (scaled by 2^-e) into S slices, one word of packed bytes each.
template <int S>
__device__ __forceinline__ void slice4(const double (&x)[4], int e, int32_t (&w)[S]) {
#pragma unroll
  for (int p = 0; p < S; ++p) w[p] = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double t = ldexp(x[c], -e);
#pragma unroll
    for (int p = 0; p < S; ++p) {
      const double v = t * 128.0;
      const double q = trunc(v);
      t = v - q;
      w[p] |= ((int32_t)q & 0xff) << (8 * c);
    }
  }
}

// Slice this thread's kSlicePer contracted indices [kSlicePer g, kSlicePer (g + 1))
// of one chunk of column c (values already in registers) into
// dst[p][c][words of those indices].
template <int S>
__device__ __forceinline__ void slice_regs(const double (&x)[kSlicePer], int c, int g, int e,
                                           int32_t (*dst)[64][kSliceRow]) {
#pragma unroll
  for (int w = 0; w < kSlicePer / 4; ++w) {
    const double x4[4] = {x[4 * w], x[4 * w + 1], x[4 * w + 2], x[4 * w + 3]};
    int32_t sw[S];
    slice4<S>(x4, e, sw);
    const int word = slice_word(c, (kSlicePer / 4) * g + w);
#pragma unroll
    for (int p = 0; p < S; ++p) dst[p][c][word] = sw[p];
  }
}

// Contracted lengths covered: the products here contract over the rows of one
// box (K = m_tau <= 128), at most two chunks of kSliceK; launches whose boxes
// have at most 64 rows instantiate one chunk (half the staging registers).
constexpr int kSliceChunks = 2;

template <int S, int KCH = kSliceChunks>
__device__ __forceinline__ void sliced_lt(int M, int N, int K, double alpha, const double* __restrict__ L, int64_t ldl,
                          const double* __restrict__ R, int64_t ldr, double beta, const double* C0, int64_t ldc0,
                          double* C, int64_t ldc, SliceSmem<S>& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rb = (wv >> 1) * 16, cb = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  const int c = tid & 63, g = tid >> 6;  // staging: output index c, contracted group g
  for (int i0 = 0; i0 < M; i0 += 64) {
    for (int j0 = 0; j0 < N; j0 += 64) {
      // this thread's operand values (column c of the L and R tiles, its
      // contracted indices of every chunk), all loads in flight together; the
      // scales (largest magnitude of each row of L^T and each column of R)
      // come from the same registers
      const bool oki = i0 + c < M, okj = j0 + c < N;
      double xa[KCH][kSlicePer], xb[KCH][kSlicePer];
      double ma = 0.0, mb = 0.0;
#pragma unroll
      for (int h = 0; h < KCH; ++h)
#pragma unroll
        for (int u = 0; u < kSlicePer; ++u) {
          const int kk = kSliceK * h + kSlicePer * g + u;
          const bool oka = oki && kk < K, okb = okj && kk < K;
          const double va = L[oka ? kk * ldl + i0 + c : 0];
          const double vb = R[okb ? kk * ldr + j0 + c : 0];
          xa[h][u] = oka ? va : 0.0;
          xb[h][u] = okb ? vb : 0.0;
          ma = fmax(ma, fabs(xa[h][u]));
          mb = fmax(mb, fabs(xb[h][u]));
        }
      {
        sm.u.red[0][g][c] = ma;
        sm.u.red[1][g][c] = mb;
        __syncthreads();
        if (tid < 128) {
          const int h = tid >> 6;
          double mx = 0.0;
#pragma unroll
          for (int q = 0; q < kSliceGroups; ++q) mx = fmax(mx, sm.u.red[h][q][c]);
          int e = 0;
          (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1); 0 for mx = 0
          (h ? sm.eb : sm.ea)[c] = e;
        }
        __syncthreads();
      }
      // recombine the S diagonal sums of column block b and store them
      auto finish = [&](int b, const gemm_i4 (&ac)[S]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ti = rb + 4 * lk + r, tj = cb + 16 * b + li;
          const int gi = i0 + ti, gj = j0 + tj;
          if (gi < M && gj < N) {
            double v = 0.0;
#pragma unroll
            for (int d = S - 1; d >= 0; --d) v += ldexp((double)ac[d][r], -7 * (d + 2));
            v = alpha * ldexp(v, sm.ea[ti] + sm.eb[tj]);
            C[gi * ldc + gj] = (beta != 0.0) ? beta * C0[gi * ldc0 + gj] + v : v;
          }
        }
      };
      if constexpr (KCH == 1) {
        // one chunk: the two column blocks one after the other, so that only
        // one block's S diagonal sums are live (half the accumulator
        // registers, twice the workgroups per compute unit)
        slice_regs<S>(xa[0], c, g, sm.ea[c], sm.u.q.As);
        slice_regs<S>(xb[0], c, g, sm.eb[c], sm.u.q.Bs);
        __syncthreads();
        gemm_i4 ap[S];
        const int wa = slice_word(rb + li, 4 * lk);
#pragma unroll
        for (int p = 0; p < S; ++p) ap[p] = *reinterpret_cast<const gemm_i4*>(&sm.u.q.As[p][rb + li][wa]);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          gemm_i4 ac[S];
#pragma unroll
          for (int d = 0; d < S; ++d) ac[d] = gemm_i4{0, 0, 0, 0};
          const int wb = slice_word(cb + 16 * b + li, 4 * lk);
#pragma unroll
          for (int q = 0; q < S; ++q) {
            const gemm_i4 bq = *reinterpret_cast<const gemm_i4*>(&sm.u.q.Bs[q][cb + 16 * b + li][wb]);
#pragma unroll
            for (int p = 0; p + q < S; ++p)
              ac[p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[p], bq, ac[p + q], 0, 0, 0);
          }
          finish(b, ac);
        }
        __syncthreads();
        continue;
      }
      gemm_i4 acc[2][S];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int d = 0; d < S; ++d) acc[b][d] = gemm_i4{0, 0, 0, 0};
#pragma unroll
      for (int h = 0; h < KCH; ++h) {
        if (kSliceK * h >= K) break;
        slice_regs<S>(xa[h], c, g, sm.ea[c], sm.u.q.As);
        slice_regs<S>(xb[h], c, g, sm.eb[c], sm.u.q.Bs);
        __syncthreads();
        gemm_i4 ap[S];
        const int wa = slice_word(rb + li, 4 * lk);
#pragma unroll
        for (int p = 0; p < S; ++p) ap[p] = *reinterpret_cast<const gemm_i4*>(&sm.u.q.As[p][rb + li][wa]);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int wb = slice_word(cb + 16 * b + li, 4 * lk);
#pragma unroll
          for (int q = 0; q < S; ++q) {
            const gemm_i4 bq = *reinterpret_cast<const gemm_i4*>(&sm.u.q.Bs[q][cb + 16 * b + li][wb]);
#pragma unroll
            for (int p = 0; p + q < S; ++p)
              acc[b][p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[p], bq, acc[b][p + q], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);  // one right-operand slice live at a time
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) finish(b, acc[b]);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// The parent blocks one side of a box hands up (eq. omega_tau_and_y_tau), for
// one tile of nc <= 64 columns of s:
//   top = B1^* P0,   bot = B3^* P1 - B2^* P0     (k x nc each, row stride ldo)
// with B1, B2, B3 m x k (row stride k) and P0, P1 m x nc (row stride ld).  It
// is one product with 2k output rows over two blocks of contracted indices:
// block 0 runs over the rows of P0 with left operand [B1 | -B2], block 1 over
// the rows of P1 with [0 | B3].  Each panel is read (and, split, sliced) once
// for both of its products.
struct ParentOp {
  const double *B1, *B2, *B3, *P0, *P1;
  int64_t ld;
  double *top, *bot;
  int64_t ldo;
  int m, k, nc;
};

// Where row i of block b's left operand L^T comes from: the entries
// L^T(i, kk) = sgn * src[kk * k] for kk < m (sgn = 0: a zero row).  Chosen
// once per thread and block from values already in registers.
struct ParentRow {
  const double* src;
  double sgn;
};
__device__ __forceinline__ ParentRow parent_row(int b, int i, int k, const double* B1, const double* B2,
                                                const double* B3) {
  const bool lo = i < k;
  const double* base = b ? B3 : (lo ? B1 : B2);
  return ParentRow{base + (lo ? i : i - k), b ? (lo ? 0.0 : 1.0) : (lo ? 1.0 : -1.0)};
}

// FP64: the product on v_mfma_f64_16x16x4f64, tiled as mfma_gemm (64 x 64
// output tiles, K staged in chunks of TK); block 1 starts at the contracted
// index mp = m rounded up to TK, so that no chunk mixes the blocks and the
// waves whose rows are the zero rows of block 1 skip its products.
template <int TK, int NT = kGemmThreads>
__device__ __forceinline__ void parent_mfma(const ParentOp& o, MfmaSmem<TK>& sm) {
  static_assert(TK % 4 == 0 && (NT == 256 || NT == 512), "tile");
  constexpr int LA = 64 * TK / NT;
  constexpr int TR = (NT == 256) ? 2 : 1;
  const double *B1 = o.B1, *B2 = o.B2, *B3 = o.B3, *P0 = o.P0, *P1 = o.P1;
  const int64_t ld = o.ld;
  const int m = o.m, k = o.k, M = 2 * k, N = o.nc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rb = (wv >> 1) * 16 * TR, cb = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  const int mp = (m + TK - 1) / TK * TK, K = mp + m;
  // staging: element idx = tid + r NT of a chunk is output index idx % 64 =
  // tid % 64 (the same for every r) and contracted index k0 + idx / 64;
  // both operands are contiguous along the output index
  const int ii = tid & 63;
  for (int i0 = 0; i0 < M; i0 += 64) {
    gemm_d4 acc[TR][2];
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = gemm_d4{0.0, 0.0, 0.0, 0.0};
    const bool oki = i0 + ii < M, okj = ii < N;
    double pa[LA], pb[LA];
    auto fetch = [&](int k0) {
      const int blk = k0 >= mp;
      const ParentRow lr = parent_row(blk, oki ? i0 + ii : 0, k, B1, B2, B3);
      const double* P = (blk ? P1 : P0) + ii;
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        const int kk = k0 - blk * mp + (tid + r * NT) / 64;
        const bool oka = oki && kk < m, okb = okj && kk < m;
        const double v = lr.src[oka ? (int64_t)kk * k : 0];
        const double w = P[okb ? (int64_t)kk * ld : 0];
        pa[r] = oka ? lr.sgn * v : 0.0;
        pb[r] = okb ? w : 0.0;
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        const int idx = tid + r * NT;
        sm.As[idx / 64][ii] = pa[r];
        sm.Bs[idx / 64][ii] = pb[r];
      }
      __syncthreads();
      if (k0 + TK < K) fetch(k0 + TK);  // block 0's chunks end at mp, where block 1's begin
      const bool blk1 = k0 >= mp;
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        const double b0 = sm.Bs[kk + lk][cb + li], b1 = sm.Bs[kk + lk][cb + 16 + li];
#pragma unroll
        for (int a = 0; a < TR; ++a) {
          const int r0 = i0 + rb + 16 * a;
          // wave-uniform: rows past the output, or block 1's zero rows
          if (r0 >= M || (blk1 && r0 + 16 <= k)) continue;
          const double av = sm.As[kk + lk][rb + 16 * a + li];
          acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[a][0], 0, 0, 0);
          acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[a][1], 0, 0, 0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = i0 + rb + 16 * a + lk + 4 * r, gj = cb + 16 * b + li;
          if (gi < M && gj < N) {
            double* dst = (gi < k) ? o.top + (int64_t)gi * o.ldo : o.bot + (int64_t)(gi - k) * o.ldo;
            dst[gj] = acc[a][b][r];
          }
        }
  }
  __syncthreads();
}

// Split precision: the same product with both operands cut into S slices as
// in sliced_lt, every block with scales of its own (the rows of P0 and P1,
// and of the left operand's blocks, may differ in magnitude by any amount),
// each block's exact integer sums recombined in FP64 and the two blocks
// added in FP64.  Called by the 512 threads of a workgroup (8 waves, each a
// 16 x 32 strip of a 64 x 64 output tile); K = m <= KCH kSliceK per block.
template <int S, int KCH = kSliceChunks>
__device__ __forceinline__ void parent_sliced(const ParentOp& o, SliceSmem<S>& sm) {
  const double *B1 = o.B1, *B2 = o.B2, *B3 = o.B3, *P0 = o.P0, *P1 = o.P1;
  const int64_t ld = o.ld;
  const int m = o.m, k = o.k, M = 2 * k, N = o.nc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rb = (wv >> 1) * 16, cb = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  const int c = tid & 63, g = tid >> 6;  // staging: output index c, contracted group g
  for (int i0 = 0; i0 < M; i0 += 64) {
    const bool wave_rows = i0 + rb < M;  // wave-uniform: some of this wave's rows are output rows
    const bool oki = i0 + c < M, okj = c < N;
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
      const ParentRow lr = parent_row(blk, oki ? i0 + c : 0, k, B1, B2, B3);
      const double* P = (blk ? P1 : P0) + c;
      // this thread's values of chunk h (masked), and their largest magnitudes
      double xa[kSlicePer], xb[kSlicePer];
      auto load = [&](int h) {
#pragma unroll
        for (int u = 0; u < kSlicePer; ++u) {
          const int kk = kSliceK * h + kSlicePer * g + u;
          const bool oka = oki && kk < m, okb = okj && kk < m;
          const double va = lr.src[oka ? (int64_t)kk * k : 0];
          const double vb = P[okb ? (int64_t)kk * ld : 0];
          xa[u] = oka ? lr.sgn * va : 0.0;
          xb[u] = okb ? vb : 0.0;
        }
      };
      double ma = 0.0, mb = 0.0;
#pragma unroll
      for (int h = KCH - 1; h >= 0; --h) {
        // the scales span every chunk; chunk 0's values stay loaded for its slicing
        load(h);
#pragma unroll
        for (int u = 0; u < kSlicePer; ++u) {
          ma = fmax(ma, fabs(xa[u]));
          mb = fmax(mb, fabs(xb[u]));
        }
      }
      sm.u.red[0][g][c] = ma;
      sm.u.red[1][g][c] = mb;
      __syncthreads();
      if (tid < 128) {
        const int h = tid >> 6;
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < kSliceGroups; ++q) mx = fmax(mx, sm.u.red[h][q][c]);
        int e = 0;
        (void)frexp(mx, &e);
        (h ? sm.eb : sm.ea)[c] = e;
      }
      __syncthreads();
      // this wave's rows take part in this block (block 1's first k rows are zero)
      const bool live = wave_rows && !(blk == 1 && i0 + rb + 16 <= k);
      // recombine this block's exact sums of column block b and store them
      // (block 0) or add them to what block 0 stored (block 1; the same lane)
      auto gather = [&](int b, const gemm_i4 (&ac)[S]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ti = rb + 4 * lk + r, tj = cb + 16 * b + li;
          const int gi = i0 + ti;
          if (gi < M && tj < N) {
            double v = 0.0;
#pragma unroll
            for (int d = S - 1; d >= 0; --d) v += ldexp((double)ac[d][r], -7 * (d + 2));
            v = ldexp(v, sm.ea[ti] + sm.eb[tj]);
            double* dst = (gi < k) ? o.top + (int64_t)gi * o.ldo : o.bot + (int64_t)(gi - k) * o.ldo;
            dst[tj] = blk ? dst[tj] + v : v;
          }
        }
      };
      if constexpr (KCH == 1) {
        slice_regs<S>(xa, c, g, sm.ea[c], sm.u.q.As);
        __builtin_amdgcn_sched_barrier(0);
        slice_regs<S>(xb, c, g, sm.eb[c], sm.u.q.Bs);
        __syncthreads();
        if (live) {
          gemm_i4 ap[S];
          const int wa = slice_word(rb + li, 4 * lk);
#pragma unroll
          for (int p = 0; p < S; ++p) ap[p] = *reinterpret_cast<const gemm_i4*>(&sm.u.q.As[p][rb + li][wa]);
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            gemm_i4 ac[S];
#pragma unroll
            for (int d = 0; d < S; ++d) ac[d] = gemm_i4{0, 0, 0, 0};
            const int wb = slice_word(cb + 16 * b + li, 4 * lk);
#pragma unroll
            for (int q = 0; q < S; ++q) {
              const gemm_i4 bq = *reinterpret_cast<const gemm_i4*>(&sm.u.q.Bs[q][cb + 16 * b + li][wb]);
#pragma unroll
              for (int p = 0; p + q < S; ++p)
                ac[p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[p], bq, ac[p + q], 0, 0, 0);
              // one slice of the right operand live at a time (the scheduler
              // would otherwise load all S ahead and exceed 128 registers)
              __builtin_amdgcn_sched_barrier(0);
            }
            gather(b, ac);
          }
        }
      } else {
        gemm_i4 acc[2][S];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int d = 0; d < S; ++d) acc[b][d] = gemm_i4{0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < KCH; ++h) {
          if (kSliceK * h >= m) break;
          if (h > 0) {
            __syncthreads();  // every wave has read the previous chunk's slices
            load(h);
          }
          slice_regs<S>(xa, c, g, sm.ea[c], sm.u.q.As);
          slice_regs<S>(xb, c, g, sm.eb[c], sm.u.q.Bs);
          __syncthreads();
          if (live) {
            gemm_i4 ap[S];
            const int wa = slice_word(rb + li, 4 * lk);
#pragma unroll
            for (int p = 0; p < S; ++p) ap[p] = *reinterpret_cast<const gemm_i4*>(&sm.u.q.As[p][rb + li][wa]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const int wb = slice_word(cb + 16 * b + li, 4 * lk);
#pragma unroll
              for (int q = 0; q < S; ++q) {
                const gemm_i4 bq = *reinterpret_cast<const gemm_i4*>(&sm.u.q.Bs[q][cb + 16 * b + li][wb]);
#pragma unroll
                for (int p = 0; p + q < S; ++p)
                  acc[b][p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ap[p], bq, acc[b][p + q], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);  // one right-operand slice live at a time
              }
            }
          }
        }
        if (live) {
#pragma unroll
          for (int b = 0; b < 2; ++b) gather(b, acc[b]);
        }
      }
      // the slices and scales are rewritten by the next block: every wave has used them
      __syncthreads();
    }
  }
}

}  // namespace hbs
