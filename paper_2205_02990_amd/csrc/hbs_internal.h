// Internal declarations shared by the libhbs translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "../../include/hbs.h"

namespace hbs {

// Per-level kernel arguments of the side kernel (QR of Omega_tau^*, nullspace
// sketch, pseudo-inverse solve, truncated QR of the sketch).
struct SideArgs {
  const double* Om;   // panel bases; row i of box b is at base + (row0[b] + i) * ld
  const double* Y;
  const double* Ps;
  const double* Z;
  int64_t ld;
  const int64_t* row0;  // device [nodes]
  const int32_t* mtau;  // device [nodes]
  int32_t nodes, s, k, mmax, mmin;
  double* U;  // [nodes][mmax][k]   (side 0 writes U, side 1 writes V)
  double* V;
  double* W;  // [nodes][mmax][mmax] Y_tau Omega_tau^dagger (side 0) / Z Psi^dagger (side 1)
  double* X;
  double* Bt;  // [nodes][2][s][mmax] transposed sketches (Y P)^*, (Z Q)^*
  int32_t* flag;
  int32_t root;  // 1: only W = Y Omega^dagger of the single box (written to W)
};

// Combine: D_tau from U, V, W, X (eq. d_tau_formula).
struct CombineArgs {
  const int32_t* mtau;
  int32_t nodes, k, mmax;
  const double* U;
  const double* V;
  const double* W;
  const double* X;
  double* D;     // [nodes][mmax][mmax]
  double* T;     // workspace [nodes][mmax * mmax + 3 * mmax * k]
};

// Parent samples: the four k x s blocks of eq. omega_tau_and_y_tau.
struct ParentArgs {
  const double* Om;
  const double* Y;
  const double* Ps;
  const double* Z;
  int64_t ld;
  const int64_t* row0;
  const int32_t* mtau;
  int32_t nodes, s, k, mmax;
  const double* U;
  const double* V;
  const double* D;
  double* R;         // workspace [nodes][2][mmax][s]
  double* nOm;       // next level panels, ld = s, box t writes rows [k t, k t + k)
  double* nY;
  double* nPs;
  double* nZ;
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

bool side_supported(int mmin, int mmax, int s, int k, bool root);
hipError_t launch_side(const SideArgs& a, hipStream_t st);
hipError_t launch_combine(const CombineArgs& a, hipStream_t st);
hipError_t launch_parent(const ParentArgs& a, hipStream_t st);
hipError_t launch_apply_up(const ApplyArgs& a, hipStream_t st);
hipError_t launch_apply_down(const ApplyArgs& a, hipStream_t st);
hipError_t launch_dense_small(const double* A, int64_t lda, int32_t transA, const double* Bm, int64_t ldb,
                              double* C, int64_t ldc, int32_t M, int32_t N, int32_t K, hipStream_t st);
hipError_t launch_logkernel(int64_t n, const double* x, const double* y, const double* Om, const double* Ps,
                            double* Y, double* Z, int32_t s, int64_t ld, hbs_precision prec, hipStream_t st);

}  // namespace hbs
