// Host side of libhbs: cluster tree, factor storage, the level-by-level sweep
// schedule of Algorithm 2, the apply of Algorithm 1, and argument checking.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hbs_internal.h"

struct hbs_tree {
  int64_t n = 0;
  int32_t leaf_max = 0;
  int32_t L = 0;
  std::vector<std::vector<int64_t>> start;  // start[l]: 2^l + 1 boundaries
};

namespace {

struct Level {
  int32_t nodes = 0, mmax = 0, mmin = 0;
  int32_t* mtau = nullptr;   // device [nodes]
  int64_t* row0 = nullptr;   // device [nodes]: first row of each box in its panels
  double* U = nullptr;       // device [nodes][mmax][k]
  double* V = nullptr;
  double* D = nullptr;       // device [nodes][mmax][mmax]
  // reduced test/sample panels consumed by this level's boxes (levels < L):
  // box t owns rows [2k t, 2k t + 2k), ld = s
  double* bOm = nullptr;
  double* bY = nullptr;
  double* bPs = nullptr;
  double* bZ = nullptr;
};

hbs_status from_hip(hipError_t e) {
  if (e == hipSuccess) return HBS_OK;
  if (e == hipErrorOutOfMemory) return HBS_ENOMEM;
  return HBS_EDEVICE;
}

}  // namespace

struct hbs_factors {
  hbs_tree tree;
  int32_t k = 0, s = 0, L = 0;
  hbs_precision prec = HBS_FP64;
  std::vector<Level> lev;  // 0..L (level 0 holds the root's panels)
  double* D0 = nullptr;
  int32_t n0 = 0;
  double* W = nullptr;
  double* X = nullptr;
  double* T = nullptr;
  double* R = nullptr;
  double* Bt = nullptr;
  int32_t* flag = nullptr;
  // apply workspace
  double* qhat = nullptr;
  double* uhat = nullptr;
  int64_t apply_nvec = 0;
  std::vector<int64_t> hoff;  // row offset of level l's blocks in qhat/uhat
  hipStream_t last = nullptr;
  std::vector<void*> allocs;
  // tracing: event pairs around launches (reused across sweeps)
  bool prof = false;
  struct Mark {
    hipEvent_t a, b;
    int cls;
  };
  std::vector<Mark> marks;
  size_t nmarks = 0;

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

  hipError_t alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
  ~hbs_factors() {
    for (Mark& m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

hbs_status build_levels(hbs_factors* f, bool with_workspace) {
  const hbs_tree& t = f->tree;
  const int L = t.L, k = f->k, s = f->s;
  f->lev.assign(L + 1, Level{});
  size_t wmax = 0, tmax = 0, rmax = 0, bmax = 0;
  for (int l = 0; l <= L; ++l) {
    Level& lv = f->lev[l];
    lv.nodes = 1 << l;
    std::vector<int32_t> mt(lv.nodes);
    std::vector<int64_t> r0(lv.nodes);
    if (l == L) {
      for (int i = 0; i < lv.nodes; ++i) {
        mt[i] = (int32_t)(t.start[l][i + 1] - t.start[l][i]);
        r0[i] = t.start[l][i];
      }
    } else {
      for (int i = 0; i < lv.nodes; ++i) {
        mt[i] = 2 * k;
        r0[i] = (int64_t)2 * k * i;
      }
    }
    lv.mmax = *std::max_element(mt.begin(), mt.end());
    lv.mmin = *std::min_element(mt.begin(), mt.end());
    hipError_t e;
    if ((e = f->alloc((void**)&lv.mtau, sizeof(int32_t) * lv.nodes)) != hipSuccess) return from_hip(e);
    if ((e = f->alloc((void**)&lv.row0, sizeof(int64_t) * lv.nodes)) != hipSuccess) return from_hip(e);
    if ((e = hipMemcpy(lv.mtau, mt.data(), sizeof(int32_t) * lv.nodes, hipMemcpyHostToDevice)) != hipSuccess)
      return from_hip(e);
    if ((e = hipMemcpy(lv.row0, r0.data(), sizeof(int64_t) * lv.nodes, hipMemcpyHostToDevice)) != hipSuccess)
      return from_hip(e);
    if (l >= 1) {
      const size_t nb = (size_t)lv.nodes * lv.mmax * k * sizeof(double);
      const size_t nd = (size_t)lv.nodes * lv.mmax * lv.mmax * sizeof(double);
      if ((e = f->alloc((void**)&lv.U, nb)) != hipSuccess) return from_hip(e);
      if ((e = f->alloc((void**)&lv.V, nb)) != hipSuccess) return from_hip(e);
      if ((e = f->alloc((void**)&lv.D, nd)) != hipSuccess) return from_hip(e);
      wmax = std::max(wmax, (size_t)lv.nodes * lv.mmax * lv.mmax);
      tmax = std::max(tmax, (size_t)lv.nodes * ((size_t)lv.mmax * lv.mmax + 3 * (size_t)lv.mmax * k));
      rmax = std::max(rmax, (size_t)lv.nodes * 2 * lv.mmax * s);
      bmax = std::max(bmax, (size_t)lv.nodes * 2 * s * lv.mmax);
    }
    if (with_workspace && l < L) {
      const size_t nb = (size_t)lv.nodes * 2 * k * s * sizeof(double);
      if ((e = f->alloc((void**)&lv.bOm, nb)) != hipSuccess) return from_hip(e);
      if ((e = f->alloc((void**)&lv.bY, nb)) != hipSuccess) return from_hip(e);
      if ((e = f->alloc((void**)&lv.bPs, nb)) != hipSuccess) return from_hip(e);
      if ((e = f->alloc((void**)&lv.bZ, nb)) != hipSuccess) return from_hip(e);
    }
  }
  f->n0 = (L == 0) ? (int32_t)t.n : 2 * k;
  hipError_t e;
  if ((e = f->alloc((void**)&f->D0, sizeof(double) * (size_t)f->n0 * f->n0)) != hipSuccess) return from_hip(e);
  if ((e = f->alloc((void**)&f->flag, sizeof(int32_t))) != hipSuccess) return from_hip(e);
  if ((e = hipMemset(f->flag, 0, sizeof(int32_t))) != hipSuccess) return from_hip(e);
  if (with_workspace) {
    if ((e = f->alloc((void**)&f->W, sizeof(double) * wmax)) != hipSuccess) return from_hip(e);
    if ((e = f->alloc((void**)&f->X, sizeof(double) * wmax)) != hipSuccess) return from_hip(e);
    if ((e = f->alloc((void**)&f->T, sizeof(double) * tmax)) != hipSuccess) return from_hip(e);
    if ((e = f->alloc((void**)&f->R, sizeof(double) * rmax)) != hipSuccess) return from_hip(e);
    if ((e = f->alloc((void**)&f->Bt, sizeof(double) * bmax)) != hipSuccess) return from_hip(e);
  }
  f->hoff.assign(L + 2, 0);
  for (int l = 1; l <= L; ++l) f->hoff[l + 1] = f->hoff[l] + (int64_t)(1 << l) * k;
  return HBS_OK;
}

hbs_status check_shape(const hbs_tree* t, int32_t k, int32_t s) {
  if (!t || k < 1 || s < 1) return HBS_EINVAL;
  const int L = t->L;
  if (L == 0) {
    if (s < t->n) return HBS_EINVAL;
    if (!hbs::side_supported((int)t->n, (int)t->n, s, k, true)) return HBS_EUNSUPPORTED;
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
  if (!hbs::side_supported((int)mmin, (int)mmax, s, k, false)) return HBS_EUNSUPPORTED;
  if (L > 1 && !hbs::side_supported(2 * k, 2 * k, s, k, false)) return HBS_EUNSUPPORTED;
  if (!hbs::side_supported(2 * k, 2 * k, s, k, true)) return HBS_EUNSUPPORTED;
  return HBS_OK;
}

#define HIP_TRY(x)                                \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) return from_hip(e_);    \
  } while (0)

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
      const int64_t a = cur[i], b = cur[i + 1];
      const int64_t half = (b - a + 1) / 2;  // ceil((b - a) / 2)
      if (half == 0 || b - a - half == 0) {
        delete t;
        return HBS_EINVAL;  // empty child
      }
      nxt.push_back(a + half);
      nxt.push_back(b);
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
  hbs_status st = check_shape(t, k, s);
  if (st != HBS_OK) return st;
  if (prec != HBS_FP64) return HBS_EUNSUPPORTED;
  hbs_factors* f = new (std::nothrow) hbs_factors;
  if (!f) return HBS_ENOMEM;
  f->tree = *t;
  f->k = k;
  f->s = s;
  f->L = t->L;
  f->prec = prec;
  st = build_levels(f, true);
  if (st != HBS_OK) {
    delete f;
    return st;
  }
  *out = f;
  return HBS_OK;
}

void hbs_factors_destroy(hbs_factors* f) {
  if (f) (void)hipDeviceSynchronize();
  delete f;
}

hbs_status hbs_compress_into(hbs_factors* f, const double* Omega, const double* Y, const double* Psi,
                             const double* Z, int64_t ld, void* hip_stream) {
  if (!f || !Omega || !Y || !Psi || !Z || ld < f->s) return HBS_EINVAL;
  if (!f->W) return HBS_EINVAL;  // imported factor sets have no sweep workspace
  hipStream_t st = (hipStream_t)hip_stream;
  f->last = st;
  const int L = f->L, k = f->k, s = f->s;
  for (int l = L; l >= 1; --l) {
    Level& lv = f->lev[l];
    Level& up = f->lev[l - 1];
    const bool leaf = (l == L);
    hbs::SideArgs sa{};
    sa.Om = leaf ? Omega : lv.bOm;
    sa.Y = leaf ? Y : lv.bY;
    sa.Ps = leaf ? Psi : lv.bPs;
    sa.Z = leaf ? Z : lv.bZ;
    sa.ld = leaf ? ld : s;
    sa.row0 = lv.row0;
    sa.mtau = lv.mtau;
    sa.nodes = lv.nodes;
    sa.s = s;
    sa.k = k;
    sa.mmax = lv.mmax;
    sa.mmin = lv.mmin;
    sa.U = lv.U;
    sa.V = lv.V;
    sa.W = f->W;
    sa.X = f->X;
    sa.Bt = f->Bt;
    sa.flag = f->flag;
    sa.root = 0;
    HIP_TRY(f->mark_begin(0, st));
    HIP_TRY(hbs::launch_side(sa, st));
    HIP_TRY(f->mark_end(st));
    hbs::CombineArgs ca{};
    ca.mtau = lv.mtau;
    ca.nodes = lv.nodes;
    ca.k = k;
    ca.mmax = lv.mmax;
    ca.U = lv.U;
    ca.V = lv.V;
    ca.W = f->W;
    ca.X = f->X;
    ca.D = lv.D;
    ca.T = f->T;
    HIP_TRY(f->mark_begin(1, st));
    HIP_TRY(hbs::launch_combine(ca, st));
    HIP_TRY(f->mark_end(st));
    hbs::ParentArgs pa{};
    pa.Om = sa.Om;
    pa.Y = sa.Y;
    pa.Ps = sa.Ps;
    pa.Z = sa.Z;
    pa.ld = sa.ld;
    pa.row0 = lv.row0;
    pa.mtau = lv.mtau;
    pa.nodes = lv.nodes;
    pa.s = s;
    pa.k = k;
    pa.mmax = lv.mmax;
    pa.U = lv.U;
    pa.V = lv.V;
    pa.D = lv.D;
    pa.R = f->R;
    pa.nOm = up.bOm;
    pa.nY = up.bY;
    pa.nPs = up.bPs;
    pa.nZ = up.bZ;
    HIP_TRY(f->mark_begin(2, st));
    HIP_TRY(hbs::launch_parent(pa, st));
    HIP_TRY(f->mark_end(st));
  }
  // root: D^(0) = Y_root Omega_root^dagger
  Level& rt = f->lev[0];
  hbs::SideArgs sa{};
  sa.Om = (L == 0) ? Omega : rt.bOm;
  sa.Y = (L == 0) ? Y : rt.bY;
  sa.Ps = sa.Om;
  sa.Z = sa.Y;
  sa.ld = (L == 0) ? ld : s;
  sa.row0 = rt.row0;
  sa.mtau = rt.mtau;
  sa.nodes = 1;
  sa.s = s;
  sa.k = k;
  sa.mmax = f->n0;
  sa.mmin = f->n0;
  sa.U = nullptr;
  sa.V = nullptr;
  sa.W = f->D0;
  sa.X = f->D0;
  sa.Bt = nullptr;
  sa.flag = f->flag;
  sa.root = 1;
  HIP_TRY(f->mark_begin(3, st));
  HIP_TRY(hbs::launch_side(sa, st));
  HIP_TRY(f->mark_end(st));
  return HBS_OK;
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

hbs_status hbs_apply(hbs_factors* f, int transpose, const double* Xin, double* Out, int64_t nvec, int64_t ldx,
                     void* hip_stream) {
  if (!f || !Xin || !Out || nvec < 1 || ldx < nvec) return HBS_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  f->last = st;
  const int L = f->L, k = f->k;
  if (L == 0) {
    HIP_TRY(hbs::launch_dense_small(f->D0, f->n0, transpose ? 1 : 0, Xin, ldx, Out, ldx, f->n0, (int)nvec, f->n0,
                                    st));
    return HBS_OK;
  }
  if (nvec > f->apply_nvec) {
    HIP_TRY(hipStreamSynchronize(st));
    const size_t rows = (size_t)f->hoff[L + 1];
    void* q = nullptr;
    void* u = nullptr;
    HIP_TRY(f->alloc(&q, sizeof(double) * rows * nvec));
    HIP_TRY(f->alloc(&u, sizeof(double) * rows * nvec));
    f->qhat = (double*)q;
    f->uhat = (double*)u;
    f->apply_nvec = nvec;
  }
  auto qh = [&](int l) { return f->qhat + f->hoff[l] * nvec; };
  auto uh = [&](int l) { return f->uhat + f->hoff[l] * nvec; };
  // upward pass
  for (int l = L; l >= 1; --l) {
    Level& lv = f->lev[l];
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
  HIP_TRY(hbs::launch_dense_small(f->D0, f->n0, transpose ? 1 : 0, qh(1), nvec, uh(1), nvec, f->n0, (int)nvec,
                                  f->n0, st));
  // downward pass
  for (int l = 1; l <= L; ++l) {
    Level& lv = f->lev[l];
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

hbs_status hbs_factors_import(const hbs_tree* t, int32_t k, const hbs_level_view* levels, const double* D0,
                              void* hip_stream, hbs_factors** out) {
  if (!out) return HBS_EINVAL;
  *out = nullptr;
  if (!t || k < 1 || !D0 || (t->L > 0 && !levels)) return HBS_EINVAL;
  hbs_factors* f = new (std::nothrow) hbs_factors;
  if (!f) return HBS_ENOMEM;
  f->tree = *t;
  f->k = k;
  f->s = 0;
  f->L = t->L;
  hbs_status st = build_levels(f, false);
  if (st != HBS_OK) {
    delete f;
    return st;
  }
  hipStream_t hs = (hipStream_t)hip_stream;
  for (int l = 1; l <= f->L; ++l) {
    const hbs_level_view& v = levels[l - 1];
    Level& lv = f->lev[l];
    if (v.level != l || v.nodes != lv.nodes || v.m != lv.mmax || v.k != k || !v.U || !v.V || !v.D) {
      delete f;
      return HBS_EINVAL;
    }
    const size_t nb = (size_t)lv.nodes * lv.mmax * k * sizeof(double);
    const size_t nd = (size_t)lv.nodes * lv.mmax * lv.mmax * sizeof(double);
    hipError_t e = hipMemcpyAsync(lv.U, v.U, nb, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(lv.V, v.V, nb, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(lv.D, v.D, nd, hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) {
      delete f;
      return from_hip(e);
    }
  }
  hipError_t e = hipMemcpyAsync(f->D0, D0, sizeof(double) * (size_t)f->n0 * f->n0, hipMemcpyDeviceToDevice, hs);
  if (e != hipSuccess) {
    delete f;
    return from_hip(e);
  }
  f->last = hs;
  *out = f;
  return HBS_OK;
}

hbs_status hbs_level(const hbs_factors* f, int32_t level, hbs_level_view* out) {
  if (!f || !out || level < 1 || level > f->L) return HBS_EINVAL;
  const Level& lv = f->lev[level];
  out->level = level;
  out->nodes = lv.nodes;
  out->m = lv.mmax;
  out->k = f->k;
  out->m_tau = lv.mtau;
  out->U = lv.U;
  out->V = lv.V;
  out->D = lv.D;
  return HBS_OK;
}

hbs_status hbs_root(const hbs_factors* f, const double** D0, int32_t* rows) {
  if (!f || !D0 || !rows) return HBS_EINVAL;
  *D0 = f->D0;
  *rows = f->n0;
  return HBS_OK;
}

hbs_status hbs_check(hbs_factors* f) {
  if (!f) return HBS_EINVAL;
  HIP_TRY(hipStreamSynchronize(f->last));
  int32_t flag = 0;
  HIP_TRY(hipMemcpy(&flag, f->flag, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (flag) HIP_TRY(hipMemset(f->flag, 0, sizeof(int32_t)));
  return flag ? HBS_ENUMERIC : HBS_OK;
}

hbs_status hbs_profile(hbs_factors* f, int enable) {
  if (!f) return HBS_EINVAL;
  f->prof = enable != 0;
  return HBS_OK;
}

hbs_status hbs_profile_read(hbs_factors* f, double* ms, int64_t* launches, int32_t nclass) {
  if (!f || !ms || !launches || nclass < 1 || nclass > 4) return HBS_EINVAL;
  for (int c = 0; c < nclass; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (size_t i = 0; i < f->nmarks; ++i) {
    const auto& m = f->marks[i];
    HIP_TRY(hipEventSynchronize(m.b));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, m.a, m.b));
    if (m.cls < nclass) {
      ms[m.cls] += t;
      launches[m.cls] += 1;
    }
  }
  f->nmarks = 0;
  return HBS_OK;
}

hbs_status hbs_sample_logkernel(int64_t n, const double* x, const double* y, const double* Omega, const double* Psi,
                                double* Y, double* Z, int32_t s, int64_t ld, hbs_precision prec, void* hip_stream) {
  if (n < 1 || s < 1 || ld < s || !x || !y || !Omega || !Psi || !Y || !Z) return HBS_EINVAL;
  if (prec != HBS_FP64) return HBS_EUNSUPPORTED;
  HIP_TRY(hbs::launch_logkernel(n, x, y, Omega, Psi, Y, Z, s, ld, prec, (hipStream_t)hip_stream));
  return HBS_OK;
}

}  // extern "C"
