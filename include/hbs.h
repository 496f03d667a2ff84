/*
 * hbs.h -- C ABI of libhbs: black-box randomized compression of HBS
 * (hierarchically block separable) matrices on one AMD MI355X (gfx950).
 *
 * The method is Levitt & Martinsson, "Linear-complexity black-box randomized
 * compression of rank-structured matrices" (arXiv 2205.02990):
 *   - cluster tree ........................ section 3.1
 *   - HBS format, telescoping factorization  sections 3.2-3.3 (eqs.
 *     telescoping_leaf, telescoping_parent, define_d_tau)
 *   - compression from samples ............ section 4, Algorithm 2
 *   - apply of the factorization .......... Algorithm 1
 *
 * Conventions shared by every entry point
 *   - Matrices are FP64, row-major.  An "N x s panel with leading dimension
 *     ld" holds element (i, j) at p[i * ld + j]; ld >= s.
 *   - Every matrix pointer is a DEVICE pointer on the current HIP device
 *     unless stated otherwise.  Inputs are borrowed: read-only, and they must
 *     stay valid until the work enqueued on the caller's stream completes.
 *   - All device work is enqueued on `hip_stream` (a hipStream_t; NULL is the
 *     default stream).  Calls return when the work is enqueued, not finished.
 *   - Argument errors are reported synchronously, before anything is
 *     enqueued, as HBS_EINVAL (or HBS_EUNSUPPORTED for shapes no compiled
 *     kernel covers).  Numeric failures found on the device (a non-finite
 *     input value, or a test-matrix block that is numerically rank
 *     deficient) raise a per-factor-set flag that hbs_check() reports.
 *   - Objects are not thread safe; use one handle per host thread.
 */
#ifndef HBS_H
#define HBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HBS_OK = 0,
  HBS_EINVAL = -1,        /* bad argument (NULL, sizes, s too small ...)        */
  HBS_ENOMEM = -2,        /* device allocation failed                           */
  HBS_EDEVICE = -3,       /* a HIP runtime call failed                          */
  HBS_ENUMERIC = -4,      /* device flag: non-finite data or rank-deficient box */
  HBS_EUNSUPPORTED = -5   /* valid but not covered by a compiled kernel shape    */
} hbs_status;

typedef enum {
  HBS_FP64 = 0,           /* every product in FP64                              */
  HBS_FP32_SPLIT = 1,     /* split precision: every product with a test or
                           * sample block from exact 7-bit integer slices on
                           * the int8 matrix cores, recombined in FP64 (eight
                           * slices: FP64-level error per product); QR, bases, solves
                           * and D_tau stay FP64                               */
  HBS_BF16 = 2            /* log-kernel sampler only: BF16 hi/lo operand pairs,
                           * FP32 sums                                         */
} hbs_precision;

/* How col(B, k) of section 2.4 truncates the whole-nullspace sketch
 * B = Y_tau P_tau (m_tau x (s - m_tau)) to its k basis columns.  Given by
 * OR-ing one of these into the precision argument of hbs_factors_create,
 * hbs_compress, hbs_batch_create and hbs_compress_batched (HBS_TRUNC_QR
 * when none is given):
 *   HBS_TRUNC_QR   the truncated QR named in section 2.4: Householder QR
 *                  with column pivoting (largest remaining column first),
 *                  stopped after k steps; the k columns of Q it produced.
 *   HBS_TRUNC_SVD  the k leading left singular vectors of B (largest
 *                  singular value first), the truncation that minimises
 *                  ||B - Q Q^* B|| (section 2.3's goal).  Computed as the
 *                  pivoted QR run to min(m_tau, s - m_tau) steps, then
 *                  one-sided Jacobi on the triangular factor (at most 3
 *                  sweeps; HBS_JACOBI_SWEEPS in the environment at create
 *                  time sets another cap, 1..20).  The basis depends only on
 *                  B B^*, and rounding errors no longer grow from level to
 *                  level through the choice of k sketch columns. */
typedef enum {
  HBS_TRUNC_QR = 0,
  HBS_TRUNC_SVD = 0x100
} hbs_truncation;

typedef struct hbs_tree hbs_tree;        /* host-only, immutable after create */
typedef struct hbs_factors hbs_factors;  /* owns device memory                */
typedef struct hbs_batch hbs_batch;      /* owns device memory of many sets  */

/* Cluster tree of section 3.1 on the indices 0..n-1.  The root owns all of
 * them; a node [a, b) splits into [a, a + ceil((b-a)/2)) and [.., b); the
 * split goes on level by level until every node of the newest level has at
 * most leaf_max indices (so every leaf sits at depth L).  n >= 1,
 * leaf_max >= 1; a split that would create an empty node is HBS_EINVAL.
 * *out is owned by the caller and released with hbs_tree_destroy. */
hbs_status hbs_tree_create(int64_t n, int32_t leaf_max, hbs_tree** out);
void       hbs_tree_destroy(hbs_tree* t);
/* Depth L of the tree (0 when n <= leaf_max: the root is the only box). */
int32_t    hbs_tree_levels(const hbs_tree* t);
/* Host query: first index and size of node `node` (0-based, left to right)
 * on level `level`. */
hbs_status hbs_tree_node(const hbs_tree* t, int32_t level, int64_t node, int64_t* start, int64_t* size);

/* View of the factors of one level l = 1..L (section 3.3): the nodes of the
 * level left to right, each with U_tau, V_tau (m_tau x k) and the
 * discrepancy block D_tau (m_tau x m_tau).  Storage is padded to the largest
 * node: U and V are [nodes][m][k], D is [nodes][m][m], rows and columns past
 * m_tau hold zeros.  All pointers are device pointers owned by the factor
 * set (valid until hbs_factors_destroy); m_tau is a device int32 array. */
typedef struct {
  int32_t level, nodes, m, k;
  const int32_t* m_tau;
  const double* U;
  const double* V;
  const double* D;
} hbs_level_view;

/* Allocate a factor set (and the sweep's workspace) for compressing an
 * N x N matrix on tree `t` with bases of width k from s samples.  Every box
 * tau needs m_tau >= k and s - m_tau >= k (the nullspace of its m_tau x s test
 * matrix must hold a k-column sketch); the root needs s >= its row count (2k,
 * or N when L = 0).  `prec` selects the arithmetic of the bulk products,
 * optionally OR-ed with an hbs_truncation; unknown bits are HBS_EINVAL.
 * HBS_FP32_SPLIT needs every box to have at most 128 rows (largest leaf,
 * and 2k above the leaves), else HBS_EUNSUPPORTED.
 * Device memory is allocated here, once; hbs_compress_into calls no
 * hipMalloc (its first call captures the sweep as a HIP graph, later calls
 * replay it). */
hbs_status hbs_factors_create(const hbs_tree* t, int32_t k, int32_t s, hbs_precision prec,
                              hbs_factors** out);
void       hbs_factors_destroy(hbs_factors* f);

/* Algorithm 2 (section 4): from the test matrices Omega, Psi (N x s) and the
 * samples Y = A Omega, Z = A^* Psi (all four N x s, leading dimension ld)
 * build the telescoping factorization of A into `f`.  For every box of a
 * level at once: the full Householder QR of Omega_tau^* gives the nullspace
 * P_tau (its trailing s - m_tau columns, section 2.4) and Omega_tau^dagger;
 * U_tau = col(Y_tau P_tau, k) truncated as the factor set's hbs_truncation
 * says (eqs. u_tau_formula, v_tau_formula); D_tau by eq. d_tau_formula; then the
 * reduced test and sample matrices of eq. omega_tau_and_y_tau feed the next
 * level up; the root block is D^(0) = Y_root Omega_root^dagger.  The previous
 * contents of `f` are overwritten.  The first call on a factor set also
 * autotunes the tiles (see hbs_sweep_plan) and waits for the stream.
 * Ordering: the input pointers are captured at the call (a later call may
 * pass other inputs before this one has run), and every call on a factor
 * set or batch (compress, apply, import) runs after the previous one on the
 * device, also when they are made on different streams. */
hbs_status hbs_compress_into(hbs_factors* f, const double* Omega, const double* Y, const double* Psi,
                             const double* Z, int64_t ld, void* hip_stream);

/* hbs_factors_create followed by hbs_compress_into. */
hbs_status hbs_compress(const hbs_tree* t, int32_t k, int32_t s, const double* Omega, const double* Y,
                        const double* Psi, const double* Z, int64_t ld, hbs_precision prec,
                        void* hip_stream, hbs_factors** out);

/* Many independent compressions in one sweep (section 4 applied to each
 * matrix; the boxes of all of them at the same height above their leaves
 * share each kernel launch).  Instance i has tree trees[i], rank k[i] and
 * s[i] samples with the requirements of hbs_factors_create; instances of
 * different (k, s) run in separate launches of the same step.  The trees are
 * copied; *out is released with hbs_batch_destroy.  Device memory for every
 * instance's factors and for the shared workspace is allocated here. */
hbs_status hbs_batch_create(int32_t count, const hbs_tree* const* trees, const int32_t* k, const int32_t* s,
                            hbs_precision prec, hbs_batch** out);
void       hbs_batch_destroy(hbs_batch* b);
/* Algorithm 2 for every instance: Omega[i], Y[i], Psi[i], Z[i] are HOST
 * arrays of `count` device pointers to instance i's N_i x s_i panels with
 * leading dimension ld[i] >= s_i (ld is a host array).  Same semantics as
 * hbs_compress_into, per instance. */
hbs_status hbs_batch_compress(hbs_batch* b, const double* const* Omega, const double* const* Y,
                              const double* const* Psi, const double* const* Z, const int64_t* ld,
                              void* hip_stream);
/* A factor-set handle on instance i of the batch, usable with hbs_apply,
 * hbs_level, hbs_root, hbs_check and hbs_profile (the last two act on the
 * whole batch).  The instance's storage lives while the batch or any such
 * handle does; release the handle with hbs_factors_destroy. */
hbs_status hbs_batch_factors(hbs_batch* b, int32_t i, hbs_factors** out);
/* hbs_batch_create, hbs_batch_compress, then one factor-set handle per
 * instance written to out[0..count-1] (host array); the batch handle itself
 * is released before returning. */
hbs_status hbs_compress_batched(int32_t count, const hbs_tree* const* trees, const int32_t* k,
                                const int32_t* s, const double* const* Omega, const double* const* Y,
                                const double* const* Psi, const double* const* Z, const int64_t* ld,
                                hbs_precision prec, void* hip_stream, hbs_factors** out);

/* Algorithm 1: Out = A~ X (transpose = 0) or A~^* X (transpose != 0) for the
 * N x nvec block X; X and Out are N x nvec with leading dimension ldx >= nvec
 * and must not overlap.  Uses workspace sized on first use for nvec (the call
 * that grows it allocates). */
hbs_status hbs_apply(hbs_factors* f, int transpose, const double* X, double* Out, int64_t nvec,
                     int64_t ldx, void* hip_stream);

/* hbs_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation and kernels, but the level blocks of Algorithm 1 live in a
 * library-owned static device array of 64 MiB per GPU (held from module load
 * until the process ends) instead of memory allocated on first use; this
 * call never allocates.  nvec may be at most hbs_apply_static_max(f) (the
 * blocks of one vector take sum over levels l = 1..L of 2^l k doubles, twice);
 * larger requests return HBS_EUNSUPPORTED before anything is enqueued.  Every
 * call on a GPU shares that GPU's array: calls that overlap on the device
 * race (calls on one factor set are ordered by the library, calls on
 * different factor sets on different streams are not). */
hbs_status hbs_apply_static(hbs_factors* f, int transpose, const double* X, double* Out, int64_t nvec,
                            int64_t ldx, void* hip_stream);
/* The largest nvec hbs_apply_static accepts for f (INT64_MAX when L = 0:
 * no level blocks); -1 for NULL. */
int64_t    hbs_apply_static_max(const hbs_factors* f);

/* Wrap known factors as a factor set, e.g. the generators of a synthetic HBS
 * matrix, so that hbs_apply acts as its black box.  `levels` is a HOST array
 * of L views (levels[l-1] describes level l, layout as hbs_level_view, device
 * pointers with stride m = the tree's largest node on that level); D0 is the
 * device root block (2k x 2k, or N x N when L = 0).  The data are copied
 * (stream-ordered on hip_stream). */
hbs_status hbs_factors_import(const hbs_tree* t, int32_t k, const hbs_level_view* levels, const double* D0,
                              void* hip_stream, hbs_factors** out);

/* View of level `level` (1..L) of a factor set. */
hbs_status hbs_level(const hbs_factors* f, int32_t level, hbs_level_view* out);
/* Device pointer to the root block D^(0) and its size (rows = cols). */
hbs_status hbs_root(const hbs_factors* f, const double** D0, int32_t* rows);

/* Wait for the factor set's last enqueued work and report the device flag:
 * HBS_ENUMERIC if any box saw a non-finite value or a pivot of its test
 * matrix's QR below 64 eps ||Omega_tau||_F; HBS_OK otherwise.  Clears it. */
hbs_status hbs_check(hbs_factors* f);

const char* hbs_status_str(hbs_status s);

/* Kernel timing of the sweep (tracing, off by default).  With `enable` != 0,
 * every later sweep of the factor set's batch launches its kernels directly
 * (not through the captured graph) and brackets each launch with a pair of
 * HIP events on the caller's stream.  Kernel classes:
 *   0 QR of the test blocks, reflectors applied to the samples and the
 *     solve for Y_tau Omega_tau^dagger (sections 2.4, 4.1)
 *   1 truncated column-pivoted QR of the nullspace sketches: U_tau, V_tau
 *     (section 2.2, eqs. u_tau_formula, v_tau_formula)
 *   2 products of the bases with W, X and with the test and sample blocks
 *   3 the small k-wide terms of D_tau (eq. d_tau_formula)
 *   4 D_tau and the corrections of the parent blocks (eq.
 *     omega_tau_and_y_tau)
 *   5 root block D^(0) */
hbs_status hbs_profile(hbs_factors* f, int enable);
/* Wait for the recorded work, then write the summed device time in ms and
 * the launch count of each class (arrays of nclass <= 6 entries, host
 * memory) accumulated since the previous read, and reset them. */
hbs_status hbs_profile_read(hbs_factors* f, double* ms, int64_t* launches, int32_t nclass);

/* The tile plan of the sweep that computes a factor set (the whole batch's
 * sweep for a batch handle): one row of HBS_PLAN_COLS int32 per launch step,
 * written to the host array rows[max_rows][HBS_PLAN_COLS]; *nrows receives the
 * number of steps (rows beyond max_rows are not written).  Columns: step,
 * boxes, largest box rows, s, k, root step (0/1), tuned (1 once the
 * autotuner has chosen; until then the built-in heuristic's choice is
 * shown), QR tile (threads, lanes per row, test-row slots, sample-row slots,
 * column slots, sample-row chunks per box), pivoted-QR tile (threads, lanes
 * per row, sketch-row slots, column slots), tail_b variant (0 one
 * workgroup per chain, 1 row blocks in parallel), QR register cap (the
 * fewest waves per SIMD its registers leave room for; 0 for none),
 * pivoted-QR register cap.
 *
 * Autotuning: the first compression of a factor set or batch times every
 * valid QR, pivoted-QR and tail_b choice of each launch step on that step's
 * own data and keeps the fastest (cached per device and launch shape for
 * the life of the process); that call therefore waits for its stream and
 * must not be made while the stream is being captured.  A tile whose
 * compiled code spills registers to scratch is never timed, chosen or
 * launched, by the autotuner or the heuristic.  Setting the
 * environment variable HBS_AUTOTUNE=0 before creating the handle keeps the
 * built-in heuristic instead. */
#define HBS_PLAN_COLS 20
hbs_status hbs_sweep_plan(const hbs_factors* f, int32_t* rows, int32_t max_rows, int32_t* nrows);

/* Storage of the factors (quantity (4) of section 5): the number of FP64
 * values of every U_tau, V_tau (m_tau x k), D_tau (m_tau x m_tau) and of
 * D^(0), each counted at its own size (no padding), divided by N.  Host
 * arithmetic only; enqueues nothing. */
hbs_status hbs_floats_per_dof(const hbs_factors* f, double* out);

/* A black box for the accuracy estimate: y = B x (transpose = 0) or
 * y = B^* x (transpose != 0) for one device vector x of length n, enqueued on
 * hip_stream.  ctx is passed through unchanged. */
typedef hbs_status (*hbs_matvec)(void* ctx, int32_t transpose, const double* x, double* y, void* hip_stream);

/* Section 5's operator-norm estimate by power iteration: with
 * E = A~ - B (f and black_box both given), A~ (black_box NULL) or B (f NULL),
 *   v_i = E^* E (v_{i-1} / ||v_{i-1}||), i = 1 .. steps,
 * starting from the device vector v0 (length n, read only), writes
 * sqrt(||v_steps||) to *out (host); an iterate that vanishes (E = 0 on it)
 * stays 0, so *out is 0.  The paper's relative error is
 * hbs_power_norm(f, B) / hbs_power_norm(NULL, B), 20 steps each.  f's N must
 * equal n.  Allocates 4 n + 257 doubles of device workspace for the call and
 * waits for the stream before returning.  HBS_EINVAL if both f and
 * black_box are NULL, n < 1, steps < 1 or a pointer is NULL; a status
 * returned by black_box is passed on. */
hbs_status hbs_power_norm(hbs_factors* f, hbs_matvec black_box, void* ctx, int64_t n, const double* v0,
                          int32_t steps, double* out, void* hip_stream);

/* hbs_matvec over a factor set: ctx is an hbs_factors*; y = A~ x or A~^* x. */
hbs_status hbs_matvec_factors(void* ctx, int32_t transpose, const double* x, double* y, void* hip_stream);

/* hbs_matvec of the log-kernel black box below, one vector at a time (the
 * kernel is symmetric, so transpose is ignored).  ctx is a HOST pointer to
 * this struct, whose x and y are the device point coordinates. */
typedef struct {
  int64_t n;
  const double* x;
  const double* y;
} hbs_logkernel_points;
hbs_status hbs_matvec_logkernel(void* ctx, int32_t transpose, const double* x, double* y, void* hip_stream);

/* Stand-in black box: the log kernel A(i, j) = log|x_i - x_j| (i != j),
 * A(i, i) = 0, on points (x[i], y[i]) (device arrays of n FP64 values).
 * Writes Y = A Omega and Z = A^* Psi = A Psi (A is symmetric); Omega, Psi, Y,
 * Z are n x s with leading dimension ld.  The kernel is never stored: every
 * entry is formed on the fly inside the matrix-core product.  `prec`:
 * HBS_FP64 (FP64 entries and FP64 matrix-core products) or HBS_BF16 (entries
 * formed in FP32; entries and test-matrix values each carried as a BF16 pair
 * hi + lo, three BF16 matrix-core products per pair, FP32 accumulation: about
 * 1e-5 relative error in Y and Z).  HBS_FP32_SPLIT is HBS_EUNSUPPORTED here. */
hbs_status hbs_sample_logkernel(int64_t n, const double* x, const double* y, const double* Omega,
                                const double* Psi, double* Y, double* Z, int32_t s, int64_t ld,
                                hbs_precision prec, void* hip_stream);

/* Sampling and compression in one pass, streamed (section 1: the method reads
 * the black box once, and its leaf level needs only the sample rows of its own
 * boxes).  Writes Y and Z of the log-kernel black box above (points x, y,
 * test matrices Omega, Psi, all as in hbs_sample_logkernel with n = the tree's
 * N and s = the factor set's s; `sampler` is its precision, HBS_FP64 or
 * HBS_BF16) and compresses them into f (created by hbs_factors_create for the
 * tree of those n points), with the results of
 *   hbs_sample_logkernel(...); hbs_compress_into(f, Omega, Y, Psi, Z, ld, ...)
 * bit for bit.  The leaf boxes are split into `chunks` ranges of whole boxes:
 * the sampler writes one range's rows on hip_stream while the leaf level of
 * the range before runs on a second stream of the library's (default
 * priority), so that the leaf level consumes each range's samples right after
 * they are produced and overlaps the sampling of the next; the levels above
 * the leaves follow on hip_stream.  chunks = 1, a tree of one box, the factor
 * set's first compression (which times the tile choices step by step) and
 * event tracing (hbs_profile) run unstreamed; chunks above the number of
 * leaves count as that number.  Y and Z are caller-owned outputs (n x s, ld);
 * all other pointers are borrowed as in hbs_compress_into, and the call is
 * ordered after every earlier call on f as hbs_compress_into is.
 * HBS_EINVAL: NULL pointers, chunks < 1, ld < s, f imported or a batch
 * member; HBS_EUNSUPPORTED: sampler not HBS_FP64 or HBS_BF16. */
hbs_status hbs_compress_logkernel(hbs_factors* f, const double* x, const double* y, const double* Omega,
                                  const double* Psi, double* Y, double* Z, int64_t ld, hbs_precision sampler,
                                  int32_t chunks, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HBS_H */
