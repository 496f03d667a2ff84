// Host side of libhbs: cluster trees, factor storage, the level-by-level sweep
// schedule of Algorithm 2 (one set of launches per aligned level, shared by
// every instance of a batch), its capture in a HIP graph, the apply of
// Algorithm 1, and argument checking.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "hbs_internal.h"

struct hbs_tree {
  int64_t n = 0;
  int32_t leaf_max = 0;
  int32_t L = 0;
  std::vector<std::vector<int64_t>> start;  // start[l]: 2^l + 1 boundaries
};

namespace {

hbs_status from_hip(hipError_t e) {
  if (e == hipSuccess) return HBS_OK;
  if (e == hipErrorOutOfMemory) return HBS_ENOMEM;
  return HBS_EDEVICE;
}

#define HIP_TRY(x)                             \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

struct Level {
  int32_t nodes = 0, mmax = 0, mmin = 0;
  int32_t* mtau = nullptr;   // device [nodes]
  int64_t* row0 = nullptr;   // device [nodes]: leaf rows in the N-vector / 2k t above (apply)
  double* U = nullptr;       // device [nodes][mmax][k], zero padded
  double* V = nullptr;
  double* D = nullptr;       // device [nodes][mmax][mmax], zero padded
  // reduced test/sample panels consumed by this level's boxes (levels < L):
  // box t owns rows [2k t, 2k t + 2k), ld = s
  double* bOm = nullptr;
  double* bY = nullptr;
  double* bPs = nullptr;
  double* bZ = nullptr;
};

struct Instance {
  hbs_tree tree;
  int32_t k = 0, s = 0, L = 0;
  std::vector<Level> lev;  // 0..L
  double* D0 = nullptr;
  int32_t n0 = 0;
  int src_in = -1;              // panel-source slot of the caller's inputs
  std::vector<int> src_lev;     // panel-source slot of level l's reduced panels (l < L)
  // apply workspace
  double* qhat = nullptr;
  double* uhat = nullptr;
  int64_t apply_nvec = 0;
  std::vector<int64_t> hoff;  // row offset of level l's blocks in qhat/uhat
};

struct Launch {
  hbs::SweepArgs args;
  // tile choices (heuristic until the autotuner has run)
  hbs::LqChoice lq{-1, 0};
  int col = -1;    // tile of the basis kernel (mode 0, or mode 1 for the SVD truncation)
  int colj = -1;   // SVD truncation: tile of the Jacobi pass (mode 2)
  int tailb = -1;
};

struct Mark {
  hipEvent_t a, b;
  int cls;
};

}  // namespace

// A set of instances compressed together: one launch per aligned level and
// (k, s) class covers the boxes of all of them.
struct BatchImpl {
  std::vector<Instance> inst;
  hbs_precision prec = HBS_FP64;
  bool svd = false;       // bases by SVD truncation of the sketches (else truncated pivoted QR)
  int jac_sweeps = 3;     // SVD truncation: most Jacobi sweeps per sketch
  int slices = 8;         // split precision: 7-bit slices per operand
  std::vector<void*> allocs;
  // The panel-source table: the host template (callers' inputs are written
  // into it), and a ring of pinned copies, one per call, each reused only
  // after the event recorded behind its upload has completed, so that a
  // later call never rewrites the bytes an earlier call's copy still reads.
  std::vector<hbs::PanelSrc> h_src;
  static constexpr int kStage = 4;
  hbs::PanelSrc* h_stage[kStage] = {};
  hipEvent_t stage_ev[kStage] = {};
  bool stage_used[kStage] = {};
  int stage_next = 0;
  hbs::PanelSrc* d_src = nullptr;
  int nsrc = 0;
  // Every call on the batch (sweep or apply) records this event behind its
  // work; a call on another stream first waits for it, so calls on one
  // batch never overlap on the device (they share the workspace).
  hipEvent_t done_ev = nullptr;
  bool done_rec = false;
  hbs::BoxDesc* d_box = nullptr;
  std::vector<Launch> launches;
  int32_t* flag = nullptr;
  bool sweep_ready = false;  // workspace and launch plan exist
  hipStream_t last = nullptr;
  // graph of the whole sweep, captured on first use
  bool use_graph = true;
  bool autotune = true;  // time the tile choices on the first sweep
  bool tuned = false;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cstream = nullptr;  // capture stream
  // streamed sampling (hbs_compress_logkernel): the leaf level runs on this
  // stream, each chunk after the event recorded behind its sample rows
  hipStream_t sstream = nullptr;
  std::vector<hipEvent_t> chunk_ev;
  hipEvent_t join_ev = nullptr;
  // tracing
  bool prof = false;
  std::vector<Mark> marks;
  size_t nmarks = 0;

  hipError_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it == allocs.end()) return;
    allocs.erase(it);
    (void)hipFree(p);
  }
  hipError_t mark_begin(int cls, hipStream_t st) {
    if (!prof) return hipSuccess;
    if (nmarks == marks.size()) {
      Mark m{};
      hipError_t e = hipEventCreate(&m.a);
      if (e == hipSuccess) e = hipEventCreate(&m.b);
      if (e != hipSuccess) return e;
      marks.push_back(m);
    }
    marks[nmarks].cls = cls;
    return hipEventRecord(marks[nmarks].a, st);
  }
  hipError_t mark_end(hipStream_t st) {
    if (!prof) return hipSuccess;
    return hipEventRecord(marks[nmarks++].b, st);
  }
  ~BatchImpl() {
    (void)hipDeviceSynchronize();
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cstream) (void)hipStreamDestroy(cstream);
    if (sstream) (void)hipStreamDestroy(sstream);
    for (hipEvent_t e : chunk_ev) (void)hipEventDestroy(e);
    if (join_ev) (void)hipEventDestroy(join_ev);
    for (Mark& m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (int i = 0; i < kStage; ++i) {
      if (h_stage[i]) (void)hipHostFree(h_stage[i]);
      if (stage_ev[i]) (void)hipEventDestroy(stage_ev[i]);
    }
    if (done_ev) (void)hipEventDestroy(done_ev);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

// Order a call on stream st after the batch's previous call (any stream).
hipError_t batch_enter(BatchImpl* b, hipStream_t st) {
  if (b->done_rec && st != b->last) return hipStreamWaitEvent(st, b->done_ev, 0);
  return hipSuccess;
}
hipError_t batch_leave(BatchImpl* b, hipStream_t st) {
  b->last = st;
  hipError_t e = hipEventRecord(b->done_ev, st);
  if (e == hipSuccess) b->done_rec = true;
  return e;
}

}  // namespace

// The caller's batch handle: one more owner of the shared storage.
struct hbs_batch {
  std::shared_ptr<BatchImpl> b;
};

// A factor set is a handle on one instance of a batch (a batch of one for
// hbs_compress); the storage lives while the batch or any handle does.
struct hbs_factors {
  std::shared_ptr<BatchImpl> b;
  int idx = 0;
};

namespace {

hbs_status check_shape(const hbs_tree* t, int32_t k, int32_t s, bool mixed, bool svd) {
  if (!t || k < 1 || s < 1) return HBS_EINVAL;
  // the tiles' spill facts are read before any shape is judged (without a
  // device they stay unknown; the factor set's own set-up then fails)
  (void)hbs::prepare_side_kernels();
  const int L = t->L;
  if (L == 0) {
    if (s < t->n) return HBS_EINVAL;
    if (!hbs::side_supported((int)t->n, (int)t->n, s, k, true, svd)) return HBS_EUNSUPPORTED;
    return HBS_OK;
  }
  int64_t mmin = INT64_MAX, mmax = 0;
  for (size_t i = 0; i + 1 < t->start[L].size(); ++i) {
    const int64_t m = t->start[L][i + 1] - t->start[L][i];
    mmin = std::min(mmin, m);
    mmax = std::max(mmax, m);
  }
  if (mmin < k || s - mmax < k) return HBS_EINVAL;        // leaves
  if (L > 1 && s - 2 * (int64_t)k < k) return HBS_EINVAL;  // inner boxes of 2k rows
  if (s < 2 * (int64_t)k) return HBS_EINVAL;               // root
  if (!hbs::side_supported((int)mmin, (int)mmax, s, k, false, svd)) return HBS_EUNSUPPORTED;
  if (L > 1 && !hbs::side_supported(2 * k, 2 * k, s, k, false, svd)) return HBS_EUNSUPPORTED;
  if (!hbs::side_supported(2 * k, 2 * k, s, k, true, svd)) return HBS_EUNSUPPORTED;
  // the split products contract over at most tail_mixed_max_rows() box rows
  if (mixed && std::max<int64_t>(mmax, L > 1 ? 2 * (int64_t)k : 0) > hbs::tail_mixed_max_rows())
    return HBS_EUNSUPPORTED;
  return HBS_OK;
}

// Factor storage (and, for a compressible batch, the reduced panels) of one instance.
hbs_status build_instance(BatchImpl* b, Instance& in, bool with_panels) {
  const hbs_tree& t = in.tree;
  const int L = t.L, k = in.k, s = in.s;
  in.L = L;
  in.lev.assign(L + 1, Level{});
  for (int l = 0; l <= L; ++l) {
    Level& lv = in.lev[l];
    lv.nodes = 1 << l;
    std::vector<int32_t> mt(lv.nodes);
    std::vector<int64_t> r0(lv.nodes);
    for (int i = 0; i < lv.nodes; ++i) {
      if (l == L) {
        mt[i] = (int32_t)(t.start[l][i + 1] - t.start[l][i]);
        r0[i] = t.start[l][i];
      } else {
        mt[i] = 2 * k;
        r0[i] = (int64_t)2 * k * i;
      }
    }
    lv.mmax = *std::max_element(mt.begin(), mt.end());
    lv.mmin = *std::min_element(mt.begin(), mt.end());
    HIP_TRY(b->alloc((void**)&lv.mtau, sizeof(int32_t) * lv.nodes));
    HIP_TRY(b->alloc((void**)&lv.row0, sizeof(int64_t) * lv.nodes));
    HIP_TRY(hipMemcpy(lv.mtau, mt.data(), sizeof(int32_t) * lv.nodes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(lv.row0, r0.data(), sizeof(int64_t) * lv.nodes, hipMemcpyHostToDevice));
    if (l >= 1) {
      const size_t nb = (size_t)lv.nodes * lv.mmax * k * sizeof(double);
      const size_t nd = (size_t)lv.nodes * lv.mmax * lv.mmax * sizeof(double);
      HIP_TRY(b->alloc((void**)&lv.U, nb));
      HIP_TRY(b->alloc((void**)&lv.V, nb));
      HIP_TRY(b->alloc((void**)&lv.D, nd));
      // padding rows/columns past m_tau stay zero: the kernels write only m_tau x k and m_tau x m_tau
      HIP_TRY(hipMemset(lv.U, 0, nb));
      HIP_TRY(hipMemset(lv.V, 0, nb));
      HIP_TRY(hipMemset(lv.D, 0, nd));
    }
    if (with_panels && l < L) {
      const size_t nb = (size_t)lv.nodes * 2 * k * s * sizeof(double);
      HIP_TRY(b->alloc((void**)&lv.bOm, nb));
      HIP_TRY(b->alloc((void**)&lv.bY, nb));
      HIP_TRY(b->alloc((void**)&lv.bPs, nb));
      HIP_TRY(b->alloc((void**)&lv.bZ, nb));
    }
  }
  in.n0 = (L == 0) ? (int32_t)t.n : 2 * k;
  HIP_TRY(b->alloc((void**)&in.D0, sizeof(double) * (size_t)in.n0 * in.n0));
  in.hoff.assign(L + 2, 0);
  for (int l = 1; l <= L; ++l) in.hoff[l + 1] = in.hoff[l] + (int64_t)(1 << l) * k;
  return HBS_OK;
}

// Launch plan and workspace of the sweep: box descriptors for every aligned
// level and (k, s) class, built once.
hbs_status build_sweep(BatchImpl* b) {
  HIP_TRY(hbs::prepare_side_kernels());
  // panel-source slots: each instance's inputs, then its levels' reduced panels
  int nsrc = 0;
  for (Instance& in : b->inst) {
    in.src_in = nsrc++;
    in.src_lev.assign(in.L, -1);
    for (int l = 0; l < in.L; ++l) in.src_lev[l] = nsrc++;
  }
  b->nsrc = nsrc;
  b->h_src.assign(nsrc, hbs::PanelSrc{});
  for (int i = 0; i < BatchImpl::kStage; ++i) {
    HIP_TRY(hipHostMalloc((void**)&b->h_stage[i], sizeof(hbs::PanelSrc) * nsrc, hipHostMallocDefault));
    HIP_TRY(hipEventCreateWithFlags(&b->stage_ev[i], hipEventDisableTiming));
  }
  for (Instance& in : b->inst)
    for (int l = 0; l < in.L; ++l)
      b->h_src[in.src_lev[l]] = hbs::PanelSrc{{in.lev[l].bOm, in.lev[l].bY, in.lev[l].bPs, in.lev[l].bZ}, in.s};
  HIP_TRY(b->alloc((void**)&b->d_src, sizeof(hbs::PanelSrc) * nsrc));

  int maxL = 0;
  for (const Instance& in : b->inst) maxL = std::max(maxL, in.L);
  std::map<std::pair<int, int>, int> cls;  // (k, s) classes
  for (const Instance& in : b->inst) cls.emplace(std::make_pair(in.k, in.s), 0);
  // box lists per (step, class); step j handles level L_i - j of instance i,
  // the last step every root
  struct Group {
    int k, s;
    bool root;
    std::vector<hbs::BoxDesc> boxes;
    std::vector<size_t> ws;  // workspace doubles needed by each box
  };
  std::vector<std::vector<Group>> steps(maxL + 1);
  for (int j = 0; j <= maxL; ++j)
    for (auto& c : cls) steps[j].push_back(Group{c.first.first, c.first.second, j == maxL, {}, {}});
  auto group_of = [&](int j, const Instance& in) -> Group& {
    for (Group& g : steps[j])
      if (g.k == in.k && g.s == in.s) return g;
    return steps[j][0];
  };
  for (Instance& in : b->inst) {
    const int k = in.k, s = in.s;
    const hbs_tree& t = in.tree;
    for (int l = in.L; l >= 1; --l) {
      Level& lv = in.lev[l];
      Level& up = in.lev[l - 1];
      Group& g = group_of(in.L - l, in);
      for (int i = 0; i < lv.nodes; ++i) {
        hbs::BoxDesc d{};
        d.src = (l == in.L) ? in.src_in : in.src_lev[l];
        d.row0 = (l == in.L) ? t.start[l][i] : (int64_t)2 * k * i;
        d.m = (l == in.L) ? (int32_t)(t.start[l][i + 1] - t.start[l][i]) : 2 * k;
        d.dld = lv.mmax;
        d.U = lv.U + (size_t)i * lv.mmax * k;
        d.V = lv.V + (size_t)i * lv.mmax * k;
        d.D = lv.D + (size_t)i * lv.mmax * lv.mmax;
        d.np[hbs::kOm] = up.bOm + (size_t)k * i * s;
        d.np[hbs::kY] = up.bY + (size_t)k * i * s;
        d.np[hbs::kPs] = up.bPs + (size_t)k * i * s;
        d.np[hbs::kZ] = up.bZ + (size_t)k * i * s;
        const size_t dl = lv.mmax;
        g.boxes.push_back(d);
        g.ws.push_back(2 * dl * dl + 2 * dl * s + hbs::tail_workspace((int)dl, k));
      }
    }
    hbs::BoxDesc d{};
    d.src = (in.L == 0) ? in.src_in : in.src_lev[0];
    d.row0 = 0;
    d.m = in.n0;
    d.dld = in.n0;
    d.D = in.D0;
    group_of(maxL, in).boxes.push_back(d);
    group_of(maxL, in).ws.push_back(0);
  }
  // workspace: steps run one after another, so one pool sized for the largest step
  size_t wsmax = 0, nbox = 0;
  for (auto& st : steps) {
    size_t w = 0;
    for (Group& g : st) {
      for (size_t x : g.ws) w += x;
      nbox += g.boxes.size();
    }
    wsmax = std::max(wsmax, w);
  }
  double* ws = nullptr;
  HIP_TRY(b->alloc((void**)&ws, sizeof(double) * std::max<size_t>(wsmax, 1)));
  HIP_TRY(b->alloc((void**)&b->d_box, sizeof(hbs::BoxDesc) * std::max<size_t>(nbox, 1)));
  std::vector<hbs::BoxDesc> all;
  all.reserve(nbox);
  for (int j = 0; j <= maxL; ++j) {
    size_t off = 0;  // the groups of one step share the pool
    for (Group& g : steps[j]) {
      if (g.boxes.empty()) continue;
      const size_t first = all.size();
      int mmax = 0, mmin = INT_MAX;
      for (size_t q = 0; q < g.boxes.size(); ++q) {
        hbs::BoxDesc d = g.boxes[q];
        if (!g.root) {
          const size_t dl = d.dld, kk = g.k, ss = g.s;
          d.W = ws + off;
          d.X = d.W + dl * dl;
          d.Bt = d.X + dl * dl;
          d.T = d.Bt + 2 * ss * dl;
          off += g.ws[q];
        }
        mmax = std::max(mmax, d.m);
        mmin = std::min(mmin, d.m);
        all.push_back(d);
      }
      Launch ln{};
      ln.args.box = b->d_box + first;
      ln.args.src = b->d_src;
      ln.args.nboxes = (int32_t)g.boxes.size();
      ln.args.k = g.k;
      ln.args.s = g.s;
      ln.args.mmax = mmax;
      ln.args.mmin = mmin;
      ln.args.root = g.root ? 1 : 0;
      ln.args.mixed = b->prec == HBS_FP32_SPLIT ? 1 : 0;
      ln.args.svd = b->svd ? 1 : 0;
      ln.args.jac_sweeps = b->jac_sweeps;
      ln.args.slices = b->slices;
      ln.args.flag = b->flag;
      b->launches.push_back(ln);
    }
  }
  HIP_TRY(hipMemcpy(b->d_box, all.data(), sizeof(hbs::BoxDesc) * all.size(), hipMemcpyHostToDevice));
  b->sweep_ready = true;
  return HBS_OK;
}

// The kernels of one launch step (one aligned level of one (k, s) class, or
// a contiguous range of its boxes).
hbs_status enqueue_launch(BatchImpl* b, const Launch& ln, hipStream_t st) {
  HIP_TRY(b->mark_begin(ln.args.root ? 5 : 0, st));
  HIP_TRY(hbs::launch_lq(ln.args, ln.lq, st));
  HIP_TRY(b->mark_end(st));
  if (ln.args.root) return HBS_OK;
  HIP_TRY(b->mark_begin(1, st));
  HIP_TRY(hbs::launch_col(ln.args, ln.args.svd ? 1 : 0, ln.col, st));
  if (ln.args.svd) HIP_TRY(hbs::launch_col(ln.args, 2, ln.colj, st));
  HIP_TRY(b->mark_end(st));
  for (int part = 0; part < 3; ++part) {
    HIP_TRY(b->mark_begin(2 + part, st));
    HIP_TRY(hbs::launch_tail(ln.args, part, part == 1 ? ln.tailb : -1, st));
    HIP_TRY(b->mark_end(st));
  }
  return HBS_OK;
}

hbs_status enqueue_sweep(BatchImpl* b, hipStream_t st) {
  for (const Launch& ln : b->launches) {
    hbs_status r = enqueue_launch(b, ln, st);
    if (r != HBS_OK) return r;
  }
  return HBS_OK;
}

// ---- autotuner ----------------------------------------------------------
// The first sweep of a batch runs step by step; for the QR, the pivoted QR
// and the tail_b products it times every valid tile choice on the step's own
// data (twice each, the faster run counts) and keeps the fastest, then runs
// the chosen one so that the step's outputs are its.  (tail_a and tail_c run
// once: tail_c updates the parent panels in place.)  Choices are cached per
// device and launch shape for the life of the process, so later batches of
// the same shapes reuse them without timing.
struct TuneKey {
  int dev, kind, mmax, mmin, s, k, nboxes, mixed, root, svd, sweeps, slices;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, kind, mmax, mmin, s, k, nboxes, mixed, root, svd, sweeps, slices) <
           std::tie(o.dev, o.kind, o.mmax, o.mmin, o.s, o.k, o.nboxes, o.mixed, o.root, o.svd, o.sweeps, o.slices);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;  // kind 0: (lq cfg, ns); 1: (col cfg, 0); 2: (tail_b variant, 0);
                                                // 3: (Jacobi-pass col cfg, 0)

TuneKey tune_key(int dev, int kind, const hbs::SweepArgs& a) {
  return TuneKey{dev, kind, a.mmax, a.mmin, a.s, a.k, a.nboxes, a.mixed, a.root, a.svd, a.svd ? a.jac_sweeps : 0,
                 a.mixed ? a.slices : 0};
}

bool tune_lookup(const TuneKey& key, std::pair<int, int>* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

void tune_store(const TuneKey& key, std::pair<int, int> v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = v;
}

// Device time of fn() on the stream: the faster of two runs.
template <class F>
hipError_t time_twice(F fn, hipEvent_t e0, hipEvent_t e1, hipStream_t st, float* ms) {
  float best = 1e30f;
  for (int r = 0; r < 2; ++r) {
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return e;
    best = std::min(best, t);
  }
  *ms = best;
  return hipSuccess;
}

hipError_t tune_sweep(BatchImpl* b, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (Launch& ln : b->launches) {
    if (e != hipSuccess) break;
    const hbs::SweepArgs& a = ln.args;
    std::pair<int, int> v;
    // QR of the test blocks
    if (tune_lookup(tune_key(dev, 0, a), &v)) {
      ln.lq = hbs::LqChoice{v.first, v.second};
    } else {
      hbs::LqChoice cand[64];
      const int n = hbs::lq_candidates(a, cand, 64);
      float best = 1e30f;
      for (int i = 0; i < n && e == hipSuccess; ++i) {
        float t = 0.0f;
        e = time_twice([&] { return hbs::launch_lq(a, cand[i], st); }, e0, e1, st, &t);
        if (e == hipSuccess && t < best) best = t, ln.lq = cand[i];
      }
      if (e == hipSuccess && ln.lq.cfg >= 0) tune_store(tune_key(dev, 0, a), {ln.lq.cfg, ln.lq.ns});
    }
    if (e == hipSuccess) e = hbs::launch_lq(a, ln.lq, st);
    if (e != hipSuccess || a.root) continue;
    // the bases: truncated pivoted QR (and, for the SVD truncation, its
    // first-order correction, then the Jacobi pass over the flagged boxes)
    const int cmode = a.svd ? 1 : 0;
    if (tune_lookup(tune_key(dev, 1, a), &v)) {
      ln.col = v.first;
    } else {
      int cand[32];
      const int n = hbs::col_candidates(a, cmode, cand, 32);
      float best = 1e30f;
      for (int i = 0; i < n && e == hipSuccess; ++i) {
        float t = 0.0f;
        e = time_twice([&] { return hbs::launch_col(a, cmode, cand[i], st); }, e0, e1, st, &t);
        if (e == hipSuccess && t < best) best = t, ln.col = cand[i];
      }
      if (e == hipSuccess && ln.col >= 0) tune_store(tune_key(dev, 1, a), {ln.col, 0});
    }
    if (e == hipSuccess) e = hbs::launch_col(a, cmode, ln.col, st);
    if (a.svd && e == hipSuccess) {
      // (timed on this data: the flags the pass above left behind)
      if (tune_lookup(tune_key(dev, 3, a), &v)) {
        ln.colj = v.first;
      } else {
        int cand[32];
        const int n = hbs::col_candidates(a, 2, cand, 32);
        float best = 1e30f;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
          float t = 0.0f;
          e = time_twice([&] { return hbs::launch_col(a, 2, cand[i], st); }, e0, e1, st, &t);
          if (e == hipSuccess && t < best) best = t, ln.colj = cand[i];
        }
        if (e == hipSuccess && ln.colj >= 0) tune_store(tune_key(dev, 3, a), {ln.colj, 0});
      }
      if (e == hipSuccess) e = hbs::launch_col(a, 2, ln.colj, st);
    }
    if (e == hipSuccess) e = hbs::launch_tail(a, 0, -1, st);
    // the k-wide terms
    if (e == hipSuccess && tune_lookup(tune_key(dev, 2, a), &v)) {
      ln.tailb = v.first;
    } else if (e == hipSuccess) {
      float best = 1e30f;
      for (int var = 0; var < hbs::tail_b_variants(a) && e == hipSuccess; ++var) {
        float t = 0.0f;
        e = time_twice([&] { return hbs::launch_tail(a, 1, var, st); }, e0, e1, st, &t);
        if (e == hipSuccess && t < best) best = t, ln.tailb = var;
      }
      if (e == hipSuccess) tune_store(tune_key(dev, 2, a), {ln.tailb, 0});
    }
    if (e == hipSuccess) e = hbs::launch_tail(a, 1, ln.tailb, st);
    if (e == hipSuccess) e = hbs::launch_tail(a, 2, -1, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

hbs_status run_sweep_body(BatchImpl* b, hipStream_t st);

// Point the panel-source slots at the caller's inputs, then run the sweep:
// replay of the captured graph, or direct launches while tracing.
// Upload this call's panel-source table through the next pinned slot of the
// ring (stream-ordered: the slot is reused only after its earlier upload ran).
hipError_t stage_sources(BatchImpl* b, hipStream_t st) {
  const int i = b->stage_next;
  b->stage_next = (i + 1) % BatchImpl::kStage;
  if (b->stage_used[i]) {
    hipError_t e = hipEventSynchronize(b->stage_ev[i]);  // its earlier upload has run
    if (e != hipSuccess) return e;
  }
  std::memcpy(b->h_stage[i], b->h_src.data(), sizeof(hbs::PanelSrc) * b->nsrc);
  hipError_t e = hipMemcpyAsync(b->d_src, b->h_stage[i], sizeof(hbs::PanelSrc) * b->nsrc, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(b->stage_ev[i], st);
  if (e == hipSuccess) b->stage_used[i] = true;
  return e;
}

hbs_status run_sweep(BatchImpl* b, hipStream_t st) {
  HIP_TRY(batch_enter(b, st));
  HIP_TRY(stage_sources(b, st));
  hbs_status res = run_sweep_body(b, st);
  if (res != HBS_OK) return res;
  HIP_TRY(batch_leave(b, st));
  return HBS_OK;
}

hbs_status run_sweep_body(BatchImpl* b, hipStream_t st) {
  b->last = st;
  if (b->autotune && !b->tuned) {
    // the first sweep picks the tiles; the sweep below (graph capture or
    // direct launches) then runs with them
    HIP_TRY(tune_sweep(b, st));
    b->tuned = true;
  }
  if (b->prof || !b->use_graph) return enqueue_sweep(b, st);
  if (!b->gexec) {
    // captured once on a private stream (the default stream cannot be
    // captured); the graph then replays on whatever stream the caller passes
    if (!b->cstream) HIP_TRY(hipStreamCreateWithFlags(&b->cstream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cstream, hipStreamCaptureModeThreadLocal));
    hbs_status s1 = enqueue_sweep(b, b->cstream);
    hipError_t e = hipStreamEndCapture(b->cstream, &g);
    if (s1 != HBS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s1;
    }
    HIP_TRY(e);
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
  }
  HIP_TRY(hipGraphLaunch(b->gexec, st));
  return HBS_OK;
}

hbs_status make_batch(int32_t count, const hbs_tree* const* trees, const int32_t* k, const int32_t* s,
                      hbs_precision prec, bool with_sweep, std::shared_ptr<BatchImpl>* out) {
  if (count < 1 || !trees || !k || (with_sweep && !s)) return HBS_EINVAL;
  const int pflags = (int)prec;
  if (pflags & ~(0xff | HBS_TRUNC_SVD)) return HBS_EINVAL;
  const bool svd = (pflags & HBS_TRUNC_SVD) != 0;
  const hbs_precision pbase = (hbs_precision)(pflags & 0xff);
  if (pbase != HBS_FP64 && pbase != HBS_FP32_SPLIT) return HBS_EUNSUPPORTED;
  for (int i = 0; i < count; ++i) {
    if (with_sweep) {
      hbs_status st = check_shape(trees[i], k[i], s[i], pbase == HBS_FP32_SPLIT, svd);
      if (st != HBS_OK) return st;
    } else if (!trees[i] || k[i] < 1) {
      return HBS_EINVAL;
    }
  }
  std::shared_ptr<BatchImpl> b(new (std::nothrow) BatchImpl);
  if (!b) return HBS_ENOMEM;
  b->prec = pbase;
  b->svd = svd;
  {
    const char* ev = std::getenv("HBS_AUTOTUNE");  // "0": keep the built-in tile heuristic
    b->autotune = !(ev && ev[0] == '0');
    const char* js = std::getenv("HBS_JACOBI_SWEEPS");  // most Jacobi sweeps of the SVD truncation
    if (js) b->jac_sweeps = std::max(1, std::min(20, std::atoi(js)));
    const char* sl = std::getenv("HBS_SPLIT_SLICES");  // 7-bit slices per operand of the split path
    if (sl) b->slices = std::max(6, std::min(8, std::atoi(sl)));
  }
  HIP_TRY(b->alloc((void**)&b->flag, sizeof(int32_t)));
  HIP_TRY(hipMemset(b->flag, 0, sizeof(int32_t)));
  HIP_TRY(hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming));
  b->inst.resize(count);
  for (int i = 0; i < count; ++i) {
    Instance& in = b->inst[i];
    in.tree = *trees[i];
    in.k = k[i];
    in.s = with_sweep ? s[i] : 0;
    hbs_status st = build_instance(b.get(), in, with_sweep);
    if (st != HBS_OK) return st;
  }
  if (with_sweep) {
    hbs_status st = build_sweep(b.get());
    if (st != HBS_OK) return st;
  }
  *out = b;
  return HBS_OK;
}

Instance& inst_of(const hbs_factors* f) { return f->b->inst[f->idx]; }

hbs_status apply_body(hbs_factors* f, int transpose, const double* Xin, double* Out, int64_t nvec, int64_t ldx,
                      double* qhat, double* uhat, hipStream_t st);


}  // namespace

namespace hbs {
int64_t factors_n(const hbs_factors* f) { return inst_of(f).tree.n; }
}  // namespace hbs

// Device scratch of hbs_apply_static: the level blocks q-hat and u-hat of
// Algorithm 1 (two halves of kApplyScratch doubles / 2).  Every GPU the
// library runs on holds its own copy from module load until the process ends.
// Host code never passes this name to a kernel: it is a host-side stand-in;
// the device address comes from hipGetSymbolAddress (apply_scratch_ptr).
constexpr size_t kApplyScratch = (size_t)8 << 20;  // 64 MiB of doubles per device
static __device__ __align__(256) double scratch[kApplyScratch];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
hipError_t apply_scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* hbs_status_str(hbs_status s) {
  switch (s) {
    case HBS_OK: return "ok";
    case HBS_EINVAL: return "invalid argument";
    case HBS_ENOMEM: return "out of device memory";
    case HBS_EDEVICE: return "HIP runtime error";
    case HBS_ENUMERIC: return "numeric failure (non-finite data or rank-deficient test matrix)";
    case HBS_EUNSUPPORTED: return "shape not covered by a compiled kernel";
  }
  return "unknown status";
}

hbs_status hbs_tree_create(int64_t n, int32_t leaf_max, hbs_tree** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  if (n < 1 || leaf_max < 1) return HBS_EINVAL;
  hbs_tree* t = new (std::nothrow) hbs_tree;
  if (!t) return HBS_ENOMEM;
  t->n = n;
  t->leaf_max = leaf_max;
  t->start.push_back({0, n});
  for (;;) {
    const std::vector<int64_t>& cur = t->start.back();
    int64_t mx = 0;
    for (size_t i = 0; i + 1 < cur.size(); ++i) mx = std::max(mx, cur[i + 1] - cur[i]);
    if (mx <= leaf_max) break;
    if (t->start.size() > 40) {
      delete t;
      return HBS_EINVAL;
    }
    std::vector<int64_t> nxt;
    nxt.reserve(2 * cur.size() - 1);
    nxt.push_back(0);
    for (size_t i = 0; i + 1 < cur.size(); ++i) {
      const int64_t a = cur[i], bb = cur[i + 1];
      const int64_t half = (bb - a + 1) / 2;  // ceil((b - a) / 2)
      if (half == 0 || bb - a - half == 0) {
        delete t;
        return HBS_EINVAL;  // empty child
      }
      nxt.push_back(a + half);
      nxt.push_back(bb);
    }
    t->start.push_back(std::move(nxt));
  }
  t->L = (int32_t)t->start.size() - 1;
  *out = t;
  return HBS_OK;
}

void hbs_tree_destroy(hbs_tree* t) { delete t; }

int32_t hbs_tree_levels(const hbs_tree* t) { return t ? t->L : -1; }

hbs_status hbs_tree_node(const hbs_tree* t, int32_t level, int64_t node, int64_t* start, int64_t* size) {
  if (!t || level < 0 || level > t->L || node < 0 || node >= ((int64_t)1 << level) || !start || !size)
    return HBS_EINVAL;
  *start = t->start[level][node];
  *size = t->start[level][node + 1] - t->start[level][node];
  return HBS_OK;
}

hbs_status hbs_factors_create(const hbs_tree* t, int32_t k, int32_t s, hbs_precision prec, hbs_factors** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  std::shared_ptr<BatchImpl> b;
  hbs_status st = make_batch(1, &t, &k, &s, prec, true, &b);
  if (st != HBS_OK) return st;
  hbs_factors* f = new (std::nothrow) hbs_factors;
  if (!f) return HBS_ENOMEM;
  f->b = b;
  f->idx = 0;
  *out = f;
  return HBS_OK;
}

void hbs_factors_destroy(hbs_factors* f) { delete f; }

hbs_status hbs_compress_into(hbs_factors* f, const double* Omega, const double* Y, const double* Psi,
                             const double* Z, int64_t ld, void* hip_stream) {
  if (!f || !Omega || !Y || !Psi || !Z) return HBS_EINVAL;
  BatchImpl* b = f->b.get();
  if (!b->sweep_ready || b->inst.size() != 1) return HBS_EINVAL;  // imported sets, batch members
  Instance& in = b->inst[0];
  if (ld < in.s) return HBS_EINVAL;
  b->h_src[in.src_in] = hbs::PanelSrc{{Omega, Y, Psi, Z}, ld};
  return run_sweep(b, (hipStream_t)hip_stream);
}

hbs_status hbs_compress(const hbs_tree* t, int32_t k, int32_t s, const double* Omega, const double* Y,
                        const double* Psi, const double* Z, int64_t ld, hbs_precision prec, void* hip_stream,
                        hbs_factors** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  if (!Omega || !Y || !Psi || !Z || ld < s) return HBS_EINVAL;
  hbs_factors* f = nullptr;
  hbs_status st = hbs_factors_create(t, k, s, prec, &f);
  if (st != HBS_OK) return st;
  st = hbs_compress_into(f, Omega, Y, Psi, Z, ld, hip_stream);
  if (st != HBS_OK) {
    hbs_factors_destroy(f);
    return st;
  }
  *out = f;
  return HBS_OK;
}

hbs_status hbs_batch_create(int32_t count, const hbs_tree* const* trees, const int32_t* k, const int32_t* s,
                            hbs_precision prec, hbs_batch** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  std::shared_ptr<BatchImpl> b;
  hbs_status st = make_batch(count, trees, k, s, prec, true, &b);
  if (st != HBS_OK) return st;
  hbs_batch* h = new (std::nothrow) hbs_batch;
  if (!h) return HBS_ENOMEM;
  h->b = b;
  *out = h;
  return HBS_OK;
}

void hbs_batch_destroy(hbs_batch* h) { delete h; }

hbs_status hbs_batch_compress(hbs_batch* h, const double* const* Omega, const double* const* Y,
                              const double* const* Psi, const double* const* Z, const int64_t* ld,
                              void* hip_stream) {
  if (!h || !Omega || !Y || !Psi || !Z || !ld) return HBS_EINVAL;
  BatchImpl* b = h->b.get();
  for (size_t i = 0; i < b->inst.size(); ++i) {
    Instance& in = b->inst[i];
    if (!Omega[i] || !Y[i] || !Psi[i] || !Z[i] || ld[i] < in.s) return HBS_EINVAL;
  }
  for (size_t i = 0; i < b->inst.size(); ++i)
    b->h_src[b->inst[i].src_in] = hbs::PanelSrc{{Omega[i], Y[i], Psi[i], Z[i]}, ld[i]};
  return run_sweep(b, (hipStream_t)hip_stream);
}

hbs_status hbs_batch_factors(hbs_batch* h, int32_t i, hbs_factors** out) {
  if (!h || !out) return HBS_EINVAL;
  *out = nullptr;
  const std::shared_ptr<BatchImpl>& b = h->b;
  if (i < 0 || i >= (int32_t)b->inst.size()) return HBS_EINVAL;
  hbs_factors* f = new (std::nothrow) hbs_factors;
  if (!f) return HBS_ENOMEM;
  f->b = b;
  f->idx = i;
  *out = f;
  return HBS_OK;
}

hbs_status hbs_compress_batched(int32_t count, const hbs_tree* const* trees, const int32_t* k, const int32_t* s,
                                const double* const* Omega, const double* const* Y, const double* const* Psi,
                                const double* const* Z, const int64_t* ld, hbs_precision prec, void* hip_stream,
                                hbs_factors** out) {
  if (!out || count < 1) return HBS_EINVAL;
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  hbs_batch* h = nullptr;
  hbs_status st = hbs_batch_create(count, trees, k, s, prec, &h);
  if (st != HBS_OK) return st;
  st = hbs_batch_compress(h, Omega, Y, Psi, Z, ld, hip_stream);
  for (int i = 0; st == HBS_OK && i < count; ++i) st = hbs_batch_factors(h, i, &out[i]);
  if (st != HBS_OK)
    for (int i = 0; i < count; ++i) {
      hbs_factors_destroy(out[i]);
      out[i] = nullptr;
    }
  hbs_batch_destroy(h);
  return st;
}

hbs_status hbs_apply(hbs_factors* f, int transpose, const double* Xin, double* Out, int64_t nvec, int64_t ldx,
                     void* hip_stream) {
  if (!f || !Xin || !Out || nvec < 1 || ldx < nvec) return HBS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  BatchImpl* b = f->b.get();
  Instance& in = inst_of(f);
  HIP_TRY(batch_enter(b, st));
  if (in.L > 0 && nvec > in.apply_nvec) {
    HIP_TRY(hipStreamSynchronize(st));
    const size_t rows = (size_t)in.hoff[in.L + 1];
    void* q = nullptr;
    void* u = nullptr;
    f->b->release(in.qhat);
    f->b->release(in.uhat);
    in.qhat = in.uhat = nullptr;
    in.apply_nvec = 0;
    HIP_TRY(f->b->alloc(&q, sizeof(double) * rows * nvec));
    HIP_TRY(f->b->alloc(&u, sizeof(double) * rows * nvec));
    in.qhat = (double*)q;
    in.uhat = (double*)u;
    in.apply_nvec = nvec;
  }
  hbs_status res = apply_body(f, transpose, Xin, Out, nvec, ldx, in.qhat, in.uhat, st);
  if (res != HBS_OK) return res;
  HIP_TRY(batch_leave(b, st));
  return HBS_OK;
}

hbs_status hbs_apply_static(hbs_factors* f, int transpose, const double* Xin, double* Out, int64_t nvec,
                            int64_t ldx, void* hip_stream) {
  if (!f || !Xin || !Out || nvec < 1 || ldx < nvec) return HBS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  BatchImpl* b = f->b.get();
  Instance& in = inst_of(f);
  const size_t half = kApplyScratch / 2;
  if ((size_t)in.hoff[in.L + 1] * (size_t)nvec > half) return HBS_EUNSUPPORTED;
  double* sp = nullptr;
  HIP_TRY(apply_scratch_ptr(&sp));
  HIP_TRY(batch_enter(b, st));
  hbs_status res = apply_body(f, transpose, Xin, Out, nvec, ldx, sp, sp + half, st);
  if (res != HBS_OK) return res;
  HIP_TRY(batch_leave(b, st));
  return HBS_OK;
}

int64_t hbs_apply_static_max(const hbs_factors* f) {
  if (!f) return -1;
  const Instance& in = inst_of(f);
  const int64_t rows = in.hoff[in.L + 1];
  return rows > 0 ? (int64_t)(kApplyScratch / 2) / rows : INT64_MAX;
}

}  // extern "C"

namespace {

// Algorithm 1 with the level blocks q-hat and u-hat (hoff[L + 1] x nvec
// doubles each) in the given device buffers.
hbs_status apply_body(hbs_factors* f, int transpose, const double* Xin, double* Out, int64_t nvec, int64_t ldx,
                      double* qhat, double* uhat, hipStream_t st) {
  Instance& in = inst_of(f);
  const int L = in.L, k = in.k;
  if (L == 0) {
    HIP_TRY(hbs::launch_dense_small(in.D0, in.n0, transpose ? 1 : 0, Xin, ldx, Out, ldx, in.n0, (int)nvec, in.n0,
                                    st));
    return HBS_OK;
  }
  auto qh = [&](int l) { return qhat + in.hoff[l] * nvec; };
  auto uh = [&](int l) { return uhat + in.hoff[l] * nvec; };
  // upward pass
  for (int l = L; l >= 1; --l) {
    Level& lv = in.lev[l];
    hbs::ApplyArgs a{};
    a.mtau = lv.mtau;
    a.row0 = lv.row0;
    a.nodes = lv.nodes;
    a.k = k;
    a.mmax = lv.mmax;
    a.nvec = nvec;
    a.B1 = transpose ? lv.U : lv.V;
    a.in = (l == L) ? Xin : qh(l + 1);
    a.ld_in = (l == L) ? ldx : nvec;
    a.out = qh(l);
    a.ld_out = nvec;
    a.leaf = (l == L);
    HIP_TRY(hbs::launch_apply_up(a, st));
  }
  // root block
  HIP_TRY(hbs::launch_dense_small(in.D0, in.n0, transpose ? 1 : 0, qh(1), nvec, uh(1), nvec, in.n0, (int)nvec,
                                  in.n0, st));
  // downward pass
  for (int l = 1; l <= L; ++l) {
    Level& lv = in.lev[l];
    hbs::ApplyArgs a{};
    a.mtau = lv.mtau;
    a.row0 = lv.row0;
    a.nodes = lv.nodes;
    a.k = k;
    a.mmax = lv.mmax;
    a.nvec = nvec;
    a.B1 = transpose ? lv.V : lv.U;
    a.Dm = lv.D;
    a.transD = transpose ? 1 : 0;
    a.in = uh(l);
    a.ld_in = nvec;
    a.qin = (l == L) ? Xin : qh(l + 1);
    a.ld_q = (l == L) ? ldx : nvec;
    a.out = (l == L) ? Out : uh(l + 1);
    a.ld_out = (l == L) ? ldx : nvec;
    a.leaf = (l == L);
    HIP_TRY(hbs::launch_apply_down(a, st));
  }
  return HBS_OK;
}

}  // namespace

extern "C" {

hbs_status hbs_factors_import(const hbs_tree* t, int32_t k, const hbs_level_view* levels, const double* D0,
                              void* hip_stream, hbs_factors** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  if (!t || k < 1 || !D0 || (t->L > 0 && !levels)) return HBS_EINVAL;
  std::shared_ptr<BatchImpl> b;
  int32_t s0 = 0;
  hbs_status st = make_batch(1, &t, &k, &s0, HBS_FP64, false, &b);
  if (st != HBS_OK) return st;
  Instance& in = b->inst[0];
  hipStream_t hs = (hipStream_t)hip_stream;
  HIP_TRY(batch_enter(b.get(), hs));
  for (int l = 1; l <= in.L; ++l) {
    const hbs_level_view& v = levels[l - 1];
    Level& lv = in.lev[l];
    if (v.level != l || v.nodes != lv.nodes || v.m != lv.mmax || v.k != k || !v.U || !v.V || !v.D)
      return HBS_EINVAL;
    const size_t nb = (size_t)lv.nodes * lv.mmax * k * sizeof(double);
    const size_t nd = (size_t)lv.nodes * lv.mmax * lv.mmax * sizeof(double);
    HIP_TRY(hipMemcpyAsync(lv.U, v.U, nb, hipMemcpyDeviceToDevice, hs));
    HIP_TRY(hipMemcpyAsync(lv.V, v.V, nb, hipMemcpyDeviceToDevice, hs));
    HIP_TRY(hipMemcpyAsync(lv.D, v.D, nd, hipMemcpyDeviceToDevice, hs));
  }
  HIP_TRY(hipMemcpyAsync(in.D0, D0, sizeof(double) * (size_t)in.n0 * in.n0, hipMemcpyDeviceToDevice, hs));
  HIP_TRY(batch_leave(b.get(), hs));
  hbs_factors* f = new (std::nothrow) hbs_factors;
  if (!f) return HBS_ENOMEM;
  f->b = b;
  f->idx = 0;
  *out = f;
  return HBS_OK;
}

hbs_status hbs_level(const hbs_factors* f, int32_t level, hbs_level_view* out) {
  if (!f || !out) return HBS_EINVAL;
  const Instance& in = inst_of(f);
  if (level < 1 || level > in.L) return HBS_EINVAL;
  const Level& lv = in.lev[level];
  out->level = level;
  out->nodes = lv.nodes;
  out->m = lv.mmax;
  out->k = in.k;
  out->m_tau = lv.mtau;
  out->U = lv.U;
  out->V = lv.V;
  out->D = lv.D;
  return HBS_OK;
}

hbs_status hbs_root(const hbs_factors* f, const double** D0, int32_t* rows) {
  if (!f || !D0 || !rows) return HBS_EINVAL;
  const Instance& in = inst_of(f);
  *D0 = in.D0;
  *rows = in.n0;
  return HBS_OK;
}

hbs_status hbs_sweep_plan(const hbs_factors* f, int32_t* rows, int32_t max_rows, int32_t* nrows) {
  if (!f || !nrows || max_rows < 0 || (max_rows > 0 && !rows)) return HBS_EINVAL;
  const BatchImpl* b = f->b.get();
  *nrows = (int32_t)b->launches.size();
  for (int32_t i = 0; i < *nrows && i < max_rows; ++i) {
    const Launch& ln = b->launches[i];
    const hbs::SweepArgs& a = ln.args;
    int32_t* r = rows + (size_t)i * HBS_PLAN_COLS;
    for (int c = 0; c < HBS_PLAN_COLS; ++c) r[c] = 0;
    r[0] = i, r[1] = a.nboxes, r[2] = a.mmax, r[3] = a.s, r[4] = a.k, r[5] = a.root, r[6] = b->tuned ? 1 : 0;
    const hbs::LqChoice lq = ln.lq.cfg >= 0 ? ln.lq : hbs::lq_default(a);
    int v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (lq.cfg >= 0) hbs::lq_describe(lq, v);
    for (int c = 0; c < 6; ++c) r[7 + c] = v[c];
    r[18] = v[6];
    if (!a.root) {
      const int cmode = a.svd ? 1 : 0;
      const int col = ln.col >= 0 ? ln.col : hbs::col_default(a, cmode);
      int w[5] = {0, 0, 0, 0, 0};
      if (col >= 0) hbs::col_describe(cmode, col, w);
      for (int c = 0; c < 4; ++c) r[13 + c] = w[c];
      r[19] = w[4];
      r[17] = ln.tailb >= 0 ? ln.tailb : (a.nboxes < 256 ? 1 : 0);
    }
  }
  return HBS_OK;
}

hbs_status hbs_floats_per_dof(const hbs_factors* f, double* out) {
  if (!f || !out) return HBS_EINVAL;
  const Instance& in = inst_of(f);
  const hbs_tree& t = in.tree;
  const int64_t k = in.k;
  double total = (double)in.n0 * in.n0;  // D^(0)
  for (int l = 1; l <= in.L; ++l) {
    for (int64_t i = 0; i < ((int64_t)1 << l); ++i) {
      const int64_t m = (l == in.L) ? t.start[l][i + 1] - t.start[l][i] : 2 * k;
      total += (double)(2 * m * k + m * m);  // U_tau, V_tau, D_tau
    }
  }
  *out = total / (double)t.n;
  return HBS_OK;
}

hbs_status hbs_check(hbs_factors* f) {
  if (!f) return HBS_EINVAL;
  BatchImpl* b = f->b.get();
  HIP_TRY(hipStreamSynchronize(b->last));
  int32_t flag = 0;
  HIP_TRY(hipMemcpy(&flag, b->flag, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (flag) HIP_TRY(hipMemset(b->flag, 0, sizeof(int32_t)));
  return flag ? HBS_ENUMERIC : HBS_OK;
}

hbs_status hbs_profile(hbs_factors* f, int enable) {
  if (!f) return HBS_EINVAL;
  f->b->prof = enable != 0;
  return HBS_OK;
}

hbs_status hbs_profile_read(hbs_factors* f, double* ms, int64_t* launches, int32_t nclass) {
  if (!f || !ms || !launches || nclass < 1 || nclass > 6) return HBS_EINVAL;
  BatchImpl* b = f->b.get();
  for (int c = 0; c < nclass; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (size_t i = 0; i < b->nmarks; ++i) {
    const Mark& m = b->marks[i];
    HIP_TRY(hipEventSynchronize(m.b));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, m.a, m.b));
    if (m.cls < nclass) {
      ms[m.cls] += t;
      launches[m.cls] += 1;
    }
  }
  b->nmarks = 0;
  return HBS_OK;
}

hbs_status hbs_sample_logkernel(int64_t n, const double* x, const double* y, const double* Omega, const double* Psi,
                                double* Y, double* Z, int32_t s, int64_t ld, hbs_precision prec, void* hip_stream) {
  if (n < 1 || s < 1 || ld < s || !x || !y || !Omega || !Psi || !Y || !Z) return HBS_EINVAL;
  if (prec != HBS_FP64 && prec != HBS_BF16) return HBS_EUNSUPPORTED;
  HIP_TRY(hbs::launch_logkernel(n, x, y, Omega, Psi, Y, Z, s, ld, prec, (hipStream_t)hip_stream));
  return HBS_OK;
}

hbs_status hbs_compress_logkernel(hbs_factors* f, const double* x, const double* y, const double* Omega,
                                  const double* Psi, double* Y, double* Z, int64_t ld, hbs_precision sampler,
                                  int32_t chunks, void* hip_stream) {
  if (!f || !x || !y || !Omega || !Psi || !Y || !Z || chunks < 1) return HBS_EINVAL;
  if (sampler != HBS_FP64 && sampler != HBS_BF16) return HBS_EUNSUPPORTED;
  BatchImpl* b = f->b.get();
  if (!b->sweep_ready || b->inst.size() != 1) return HBS_EINVAL;  // imported sets, batch members
  Instance& in = b->inst[0];
  if (ld < in.s) return HBS_EINVAL;
  const hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = in.tree.n;
  const int L = in.L;
  b->h_src[in.src_in] = hbs::PanelSrc{{Omega, Y, Psi, Z}, ld};
  // unstreamed: one chunk, no leaf level, the first sweep (which times the
  // tiles step by step), or event tracing
  const int nleaf = L > 0 ? b->launches[0].args.nboxes : 0;
  if (chunks == 1 || L == 0 || (b->autotune && !b->tuned) || b->prof) {
    HIP_TRY(batch_enter(b, st));
    HIP_TRY(hbs::launch_logkernel(n, x, y, Omega, Psi, Y, Z, in.s, ld, sampler, st));
    return run_sweep(b, st);
  }
  chunks = std::min(chunks, nleaf);
  if (!b->sstream) HIP_TRY(hipStreamCreateWithFlags(&b->sstream, hipStreamNonBlocking));
  while ((int)b->chunk_ev.size() < chunks) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->chunk_ev.push_back(e);
  }
  if (!b->join_ev) HIP_TRY(hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming));
  HIP_TRY(batch_enter(b, st));
  HIP_TRY(stage_sources(b, st));
  b->last = st;
  // The leaf step (launch 0: the leaf boxes in tree order, rows contiguous)
  // in `chunks` ranges of whole boxes: the sampler writes a range's rows on
  // the caller's stream, the range's boxes run on the library's stream
  // behind it, while the sampler goes on to the next rows.
  const Launch& leaf = b->launches[0];
  const std::vector<int64_t>& bound = in.tree.start[L];
  for (int c = 0; c < chunks; ++c) {
    const int b0 = (int)((int64_t)nleaf * c / chunks), b1 = (int)((int64_t)nleaf * (c + 1) / chunks);
    HIP_TRY(hbs::launch_logkernel(n, x, y, Omega, Psi, Y, Z, in.s, ld, sampler, st, bound[b0], bound[b1]));
    HIP_TRY(hipEventRecord(b->chunk_ev[c], st));
    HIP_TRY(hipStreamWaitEvent(b->sstream, b->chunk_ev[c], 0));
    // the whole level's tile choices (the built-in heuristics depend on the
    // box count, so they are resolved for the level, not the range)
    Launch part = leaf;
    if (part.lq.cfg < 0) part.lq = hbs::lq_default(leaf.args);
    if (part.col < 0) part.col = hbs::col_default(leaf.args, leaf.args.svd ? 1 : 0);
    if (part.args.svd && part.colj < 0) part.colj = hbs::col_default(leaf.args, 2);
    if (part.tailb < 0) part.tailb = hbs::tail_b_default(leaf.args);
    part.args.box = leaf.args.box + b0;
    part.args.nboxes = b1 - b0;
    hbs_status r = enqueue_launch(b, part, b->sstream);
    if (r != HBS_OK) return r;
  }
  HIP_TRY(hipEventRecord(b->join_ev, b->sstream));
  HIP_TRY(hipStreamWaitEvent(st, b->join_ev, 0));
  for (size_t i = 1; i < b->launches.size(); ++i) {
    hbs_status r = enqueue_launch(b, b->launches[i], st);
    if (r != HBS_OK) return r;
  }
  HIP_TRY(batch_leave(b, st));
  return HBS_OK;
}

}  // extern "C"
