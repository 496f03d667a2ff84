// Internal declarations shared by the libhbs translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "../../include/hbs.h"

namespace hbs {

// Where a box's test and sample panels live: the caller's inputs of one
// instance, or the library's reduced panels of one level.  Row i of a box is
// at base + (row0 + i) * ld.
enum PanelKind { kOm = 0, kY = 1, kPs = 2, kZ = 3 };
struct PanelSrc {
  const double* p[4];  // Omega, Y, Psi, Z (indexed by PanelKind)
  int64_t ld;
};

// One box of one sweep launch.  Every launch covers the boxes of one aligned
// level of one or more instances that share (k, s).
struct BoxDesc {
  int64_t row0;   // first panel row of the box in its source
  int32_t src;    // index into the panel source table
  int32_t m;      // rows of the box (m_tau)
  int32_t dld;    // row stride of this box's D, W, X and sketch blocks (>= m)
  int32_t pad;
  double* U;      // basis outputs, m x k, row stride k
  double* V;
  double* D;      // m x m, stride dld
  double* W;      // workspace: Y Omega^dagger, m x m, stride dld
  double* X;      //            Z Psi^dagger
  double* Bt;     // workspace: [2][s][dld] transposed sketches
  double* T;      // workspace of the tail kernels, tail_workspace(dld, k) doubles
  double* np[4];  // parent panels Omega', Y', Psi', Z' (PanelKind order): k rows each, ld = s (null at the root)
};

struct SweepArgs {
  const BoxDesc* box;
  const PanelSrc* src;
  int32_t nboxes, k, s, mmax, mmin;
  int32_t root;   // 1: only W = Y Omega^dagger of each box (written to D)
  int32_t mixed;  // 1: split-precision bulk products in the tail kernels
  int32_t slices; // split precision: 7-bit slices per operand (6..8)
  int32_t svd;    // 1: bases by SVD truncation of the sketch, 0: truncated pivoted QR
  int32_t jac_sweeps;  // SVD truncation: most Jacobi sweeps per sketch
  int32_t* flag;
};

// Apply: one level of the upward or downward pass of Algorithm 1.
struct ApplyArgs {
  const int32_t* mtau;
  const int64_t* row0;   // rows of each node in the finest-level vector (leaf level)
  int32_t nodes, k, mmax;
  int64_t nvec;
  const double* B1;      // basis (V for up, U for down), [nodes][mmax][k]
  const double* Dm;      // [nodes][mmax][mmax]
  int32_t transD;        // use D^* instead of D
  const double* in;      // up: child block (leaf: q rows) ; down: parent uhat
  int64_t ld_in;
  const double* qin;     // down: q-hat of the children (inner) or q rows (leaf)
  int64_t ld_q;
  double* out;
  int64_t ld_out;
  int32_t leaf;          // 1: rows addressed through row0 (finest level)
};

bool side_supported(int mmin, int mmax, int s, int k, bool root, bool svd);
hipError_t prepare_side_kernels();
// Launch choices the autotuner picks among: a QR tile class (index into the
// compiled classes) with a number of sample-row chunks per box; cfg < 0 means
// the built-in heuristic.
struct LqChoice {
  int cfg, ns;
};
// The valid choices for a launch (up to max), the heuristic's, and the tile
// shape of a choice (lq: nt, cpr, ra, rs, cpl, ns, register cap in waves per
// SIMD or 0; col: nt, cpr, rpl, cpl, register cap).
int lq_candidates(const SweepArgs& a, LqChoice* out, int max);
// col modes: 0 truncated pivoted QR; for the SVD truncation, 1 its
// first-order correction (every box) then 2 Jacobi (boxes mode 1 flagged)
int col_candidates(const SweepArgs& a, int mode, int* out, int max);
LqChoice lq_default(const SweepArgs& a);
int col_default(const SweepArgs& a, int mode);
void lq_describe(LqChoice c, int* v);
void col_describe(int mode, int c, int* v);
// QR of the test blocks, reflectors applied to the samples, Y Omega^dagger
// (both sides of every box; the root's one side)
hipError_t launch_lq(const SweepArgs& a, LqChoice ch, hipStream_t st);
// N of a factor set's tree (host)
int64_t factors_n(const hbs_factors* f);
// the bases U_tau, V_tau from the nullspace sketches, kernel mode as above
// (cfg: index of a column tile class of that mode, < 0 for the heuristic)
hipError_t launch_col(const SweepArgs& a, int mode, int cfg, hipStream_t st);
// the products after the bases: part 0 (tail_a), 1 (tail_b), 2 (tail_c);
// variant (tail_b only): 0 one workgroup per chain, 1 row blocks in
// parallel with deeper K chunks, 2 small boxes staged whole, < 0 the
// heuristic (1 on levels of few boxes)
size_t tail_workspace(int dld, int k);
// the most box rows the split-precision products contract over
int tail_mixed_max_rows();
hipError_t launch_tail(const SweepArgs& a, int part, int variant, hipStream_t st);
int tail_b_default(const SweepArgs& a);
// tail_b variants valid for a launch: 0 and 1 always, 2 (both operands staged
// at once) for boxes of at most 64 rows with k <= 32
int tail_b_variants(const SweepArgs& a);
hipError_t launch_apply_up(const ApplyArgs& a, hipStream_t st);
hipError_t launch_apply_down(const ApplyArgs& a, hipStream_t st);
hipError_t launch_dense_small(const double* A, int64_t lda, int32_t transA, const double* Bm, int64_t ldb,
                              double* C, int64_t ldc, int32_t M, int32_t N, int32_t K, hipStream_t st);
// rows [row0, row1) of [Y Z] = A [Omega Psi] (the sum runs over all n points;
// row1 < 0: to n)
hipError_t launch_logkernel(int64_t n, const double* x, const double* y, const double* Om, const double* Ps,
                            double* Y, double* Z, int32_t s, int64_t ld, hbs_precision prec, hipStream_t st,
                            int64_t row0 = 0, int64_t row1 = -1);

}  // namespace hbs
