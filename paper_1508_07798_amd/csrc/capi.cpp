// extern "C" entry points: argument checks, status codes, error messages.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "common.hpp"
#include "engine.hpp"
#include "planner.hpp"
#include "tuning.hpp"

namespace hss {
void mlp_forward(const float* w, const float* x, int n, float* y, hipStream_t st);
void mlp_grad(const float* w, const float* x, const float* t, int n, float* grad, double* loss, hipStream_t st);
void mlp_train(float* w, const float* x, const float* t, int n, int steps, float lr, float* loss_hist,
               hipStream_t st);
void mlp_grad_noalloc(const float* w, const float* x, const float* t, int n, float* grad, double* loss,
                      hipStream_t st);
std::vector<float> mlp_read(const char* path);
void rank_model_train(const float* feat, const float* rank, int n, const char* path, uint64_t seed);
int mlp_noalloc_max_n();
int panel_candidates(int scalar, int rows, int32_t* out, int cap);
}  // namespace hss

struct hss_ctx {
  std::vector<float> model;  // rank-model weights read from opts.rank_model_path
  std::unique_ptr<hss::EngineBase> eng;
};
struct hss_plan_ctx {
  hss::Plan plan;
};

namespace {
thread_local std::string g_err;

hss_status_t fail(int code, const std::string& msg) {
  g_err = msg;
  return (hss_status_t)code;
}

template <class F> hss_status_t guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const hss::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(HSS_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(HSS_EDEVICE, e.what());
  } catch (...) {
    return fail(HSS_EDEVICE, "unknown error");
  }
}

void check_finite_host(const hss_block_op_t& a) {
  if (a.vals_on_device) return;
  const int64_t nnzb = a.row_ptr[a.n_el];
  const int64_t cnt = nnzb * a.q * a.q * (a.dtype == HSS_C128 ? 2 : 1);
  const double* v = (const double*)a.vals;
  for (int64_t i = 0; i < cnt; ++i)
    if (!std::isfinite(v[i])) throw hss::Error(HSS_EINVAL, "operator holds a non-finite value");
}

void ensure_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) {
    (void)hipGetLastError();
    throw hss::Error(HSS_EDEVICE, "no HIP device available");
  }
}
}  // namespace

namespace {
// The planner's output depends on the structure only (block sparsity, q, tree), not
// on the values. The last plan is kept with a copy of the structure it came from, so
// that factorizations of new values on the same mesh and tree (a parameter sweep, a
// sequence of right-hand sides with new coefficients) skip the planner. The copy is
// compared element by element, never through a hash.
struct PlanCache {
  std::mutex mu;
  std::vector<int32_t> key;
  std::shared_ptr<const hss::Plan> plan;  // shared with the engines built on it
};
PlanCache& plan_cache() {
  static PlanCache c;
  return c;
}
// Visit the structure arrays in a fixed order (the caller has checked the pointers).
template <class F> void visit_structure(int nprob, const hss_block_op_t* A, const hss_tree_t* T, int leaf, F&& f) {
  const int32_t head[2] = {nprob, leaf};
  f(head, 2);
  for (int p = 0; p < nprob; ++p) {
    const hss_block_op_t& a = A[p];
    const hss_tree_t& t = T[p];
    const int32_t sz[4] = {a.n_el, a.q, (int32_t)a.dtype, t.n_leaves};
    f(sz, 4);
    f(a.row_ptr, (size_t)a.n_el + 1);
    f(a.col_idx, (size_t)a.row_ptr[a.n_el]);
    f(t.leaf_node, (size_t)t.n_leaves);
    f(t.leaf_ptr, (size_t)t.n_leaves + 1);
    f(t.leaf_elems, (size_t)a.n_el);
    f(t.elem_xy, 2 * (size_t)a.n_el);
  }
}
std::shared_ptr<const hss::Plan> plan_for(int nprob, const hss_block_op_t* A, const hss_tree_t* T, int leaf) {
  bool ok = nprob >= 1 && A && T;
  for (int p = 0; ok && p < nprob; ++p)
    ok = A[p].n_el >= 2 && A[p].row_ptr && A[p].col_idx && A[p].vals && T[p].n_leaves >= 2 && T[p].leaf_node &&
         T[p].leaf_ptr && T[p].leaf_elems && T[p].elem_xy && A[p].row_ptr[A[p].n_el] >= 0 &&
         T[p].leaf_ptr[T[p].n_leaves] == A[p].n_el;
  if (!ok) return std::make_shared<const hss::Plan>(hss::make_plan(nprob, A, T, leaf));  // reports the error
  PlanCache& c = plan_cache();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.plan) {
      size_t off = 0;
      bool same = true;
      visit_structure(nprob, A, T, leaf, [&](const int32_t* v, size_t n) {
        if (!same) return;
        same = off + n <= c.key.size() && std::memcmp(c.key.data() + off, v, n * sizeof(int32_t)) == 0;
        off += n;
      });
      if (same && off == c.key.size()) return c.plan;
    }
  }
  auto plan = std::make_shared<const hss::Plan>(hss::make_plan(nprob, A, T, leaf));
  std::vector<int32_t> key;
  visit_structure(nprob, A, T, leaf, [&](const int32_t* v, size_t n) { key.insert(key.end(), v, v + n); });
  std::lock_guard<std::mutex> lk(c.mu);
  c.key = std::move(key);
  c.plan = plan;
  return plan;
}
}  // namespace

extern "C" {

void hss_default_opts(hss_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->prec = HSS_PREC_FP32;
  o->p_os = 10;
  o->l0 = 32;
  o->max_attempts = 8;
  o->seed = 1508;
  o->rank_model = nullptr;
  o->kappa_h = 0.0;
  o->hip_stream = nullptr;
  o->profile = 0;
  o->apply_graph = 1;
  o->hss_leaf_elems = 4;
  o->rank_model_path = nullptr;
  o->keep_box = 0;
  o->ldu = 2;
  o->model_margin = 0.0;
}

const char* hss_last_error(void) { return g_err.c_str(); }

hss_status_t hss_factor_batched(int32_t nprob, const hss_block_op_t* A, const hss_tree_t* T, double tol,
                                const hss_opts_t* o, hss_handle_t* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> hss_status_t {
    if (!out) return fail(HSS_EINVAL, "out is null");
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(HSS_EINVAL, "tol must be finite and >= 0");
    hss_opts_t opts;
    hss_default_opts(&opts);
    if (o) opts = *o;
    if (opts.p_os < 1 || opts.l0 < 1 || opts.max_attempts < 1 || opts.hss_leaf_elems < 0 || opts.keep_box < 0 ||
        opts.ldu < 0 || opts.ldu > 2 || !(opts.model_margin == 0.0 || opts.model_margin >= 1.0) ||
        !std::isfinite(opts.model_margin))
      return fail(HSS_EINVAL, "bad options");
    const int leaf = opts.hss_leaf_elems > 0 ? opts.hss_leaf_elems : 4;
    if (opts.prec != HSS_PREC_FP64 && opts.prec != HSS_PREC_FP32 && opts.prec != HSS_PREC_BF16)
      return fail(HSS_EINVAL, "unknown precision");
    hss::tuning_load_default();
    std::shared_ptr<const hss::Plan> plan = plan_for(nprob, A, T, leaf);
    for (int p = 0; p < nprob; ++p) check_finite_host(A[p]);
    ensure_device();
    std::unique_ptr<hss_ctx> h(new hss_ctx);
    if (!opts.rank_model && opts.rank_model_path) {
      h->model = hss::mlp_read(opts.rank_model_path);
      opts.rank_model = h->model.data();
    }
    h->eng = hss::make_engine(std::move(plan), opts, A[0].dtype == HSS_C128);
    h->eng->factor(A, tol);
    *out = h.release();
    return HSS_OK;
  });
}

hss_status_t hss_factor(const hss_block_op_t* A, const hss_tree_t* T, double tol, const hss_opts_t* o,
                        hss_handle_t* out) {
  return hss_factor_batched(1, A, T, tol, o, out);
}

hss_status_t hss_apply(hss_handle_t h, int32_t nrhs, const void* x, int64_t ldx, void* y, int64_t ldy,
                       int32_t on_device) {
  return guarded([&]() -> hss_status_t {
    if (!h || !h->eng) return fail(HSS_EINVAL, "null handle");
    h->eng->apply(nrhs, x, ldx, y, ldy, on_device != 0);
    return HSS_OK;
  });
}

hss_status_t gmres_solve(hss_handle_t h, int32_t nrhs, const void* b, void* x, int64_t ld, double tol,
                         int32_t restart, int32_t maxit, int32_t on_device, hss_gmres_info_t* info) {
  return guarded([&]() -> hss_status_t {
    if (!h || !h->eng) return fail(HSS_EINVAL, "null handle");
    if (!info) return fail(HSS_EINVAL, "info is null");
    if (!(tol > 0)) return fail(HSS_EINVAL, "tol must be > 0");
    int s = h->eng->gmres(nrhs, b, x, ld, tol, restart, maxit, on_device != 0, info);
    if (s != HSS_OK) return fail(s, "GMRES did not reach the tolerance within maxit");
    return HSS_OK;
  });
}

hss_status_t hss_query(hss_handle_t h, const char* key, double* out, int64_t cap, int64_t* len) {
  return guarded([&]() -> hss_status_t {
    if (!h || !h->eng || !key) return fail(HSS_EINVAL, "null handle or key");
    std::vector<double> v;
    if (!h->eng->query(key, v)) return fail(HSS_EINVAL, std::string("unknown key ") + key);
    if (len) *len = (int64_t)v.size();
    for (int64_t i = 0; i < (int64_t)v.size() && i < cap && out; ++i) out[i] = v[i];
    return HSS_OK;
  });
}

void hss_destroy(hss_handle_t h) {
  try {
    delete h;
  } catch (...) {
  }
}

hss_status_t hss_plan_create(const hss_block_op_t* A, const hss_tree_t* T, int32_t hss_leaf_elems,
                             hss_plan_t* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> hss_status_t {
    if (!out) return fail(HSS_EINVAL, "out is null");
    if (hss_leaf_elems < 0) return fail(HSS_EINVAL, "HSS leaf size must be >= 0");
    std::unique_ptr<hss_plan_ctx> p(new hss_plan_ctx);
    p->plan = hss::make_plan(1, A, T, hss_leaf_elems > 0 ? hss_leaf_elems : 4);
    *out = p.release();
    return HSS_OK;
  });
}

hss_status_t hss_plan_query(hss_plan_t p, const char* key, int32_t node, int64_t* out, int64_t cap, int64_t* len) {
  return guarded([&]() -> hss_status_t {
    if (!p || !key) return fail(HSS_EINVAL, "null plan or key");
    std::vector<int64_t> v;
    const std::string k(key);
    if (k == "root") {
      v = p->plan.roots[0].dofs;
    } else {
      int g = p->plan.find(0, node);
      if (g < 0) return fail(HSS_EINVAL, "no such box");
      const hss::PNode& n = p->plan.nodes[g];
      if (k == "idof") v = n.idof;
      else if (k == "bdof") v = n.bdof;
      else if (k == "height") v = {n.height};
      else if (k == "hss") {
        for (auto& t : n.hss) {
          v.push_back(t.lo);
          v.push_back(t.hi);
          v.push_back(t.left);
          v.push_back(t.right);
        }
      } else {
        return fail(HSS_EINVAL, "unknown key " + k);
      }
    }
    if (len) *len = (int64_t)v.size();
    for (int64_t i = 0; i < (int64_t)v.size() && i < cap && out; ++i) out[i] = v[i];
    return HSS_OK;
  });
}

void hss_plan_destroy(hss_plan_t p) { delete p; }

hss_status_t hss_tuning_load(const char* path) {
  return guarded([&]() -> hss_status_t {
    if (!path) return fail(HSS_EINVAL, "null path");
    hss::tuning_load(path);
    return HSS_OK;
  });
}

hss_status_t hss_tuning_set(int32_t scalar, int32_t rows_class, int32_t nb, int32_t rpt, int32_t nt, int32_t block) {
  return guarded([&]() -> hss_status_t {
    if (nb < 0 || rpt < 0 || nt < 0 || block < -1) return fail(HSS_EINVAL, "bad tuning entry");
    hss::TuneEntry e;
    e.nb = nb;
    e.rpt = rpt;
    e.nt = nt;
    e.block = block;
    hss::tuning_set(scalar, rows_class, e);
    return HSS_OK;
  });
}

void hss_tuning_clear(void) { hss::tuning_clear(); }

hss_status_t hss_tuning_candidates(int32_t scalar, int32_t rows, int32_t* out, int32_t cap, int32_t* count) {
  return guarded([&]() -> hss_status_t {
    if (scalar < 0 || scalar > 3 || rows < 1 || !count || cap < 0) return fail(HSS_EINVAL, "bad arguments");
    *count = hss::panel_candidates(scalar, rows, out, cap);
    return HSS_OK;
  });
}

hss_status_t hss_mlp_forward(const float* w, const float* x, int32_t n, float* y, void* stream) {
  return guarded([&]() -> hss_status_t {
    if (!w || !x || !y || n < 1) return fail(HSS_EINVAL, "bad mlp arguments");
    ensure_device();
    hss::mlp_forward(w, x, n, y, (hipStream_t)stream);
    return HSS_OK;
  });
}

hss_status_t hss_mlp_grad(const float* w, const float* x, const float* t, int32_t n, float* grad, double* loss,
                          void* stream) {
  return guarded([&]() -> hss_status_t {
    if (!w || !x || !t || !grad || !loss || n < 1) return fail(HSS_EINVAL, "bad mlp arguments");
    ensure_device();
    hss::mlp_grad(w, x, t, n, grad, loss, (hipStream_t)stream);
    return HSS_OK;
  });
}

hss_status_t hss_mlp_grad_noalloc(const float* w, const float* x, const float* t, int32_t n, float* grad,
                                  double* loss, void* stream) {
  return guarded([&]() -> hss_status_t {
    if (!w || !x || !t || !grad || !loss || n < 1) return fail(HSS_EINVAL, "bad mlp arguments");
    if (n > HSS_MLP_NOALLOC_MAX_N || n > hss::mlp_noalloc_max_n())
      return fail(HSS_EINVAL, "hss_mlp_grad_noalloc takes at most " + std::to_string(HSS_MLP_NOALLOC_MAX_N) +
                                  " samples");
    ensure_device();
    hss::mlp_grad_noalloc(w, x, t, n, grad, loss, (hipStream_t)stream);
    return HSS_OK;
  });
}

hss_status_t hss_mlp_train(float* w, const float* x, const float* t, int32_t n, int32_t steps, float lr,
                           float* loss_hist, void* stream) {
  return guarded([&]() -> hss_status_t {
    if (!w || !x || !t || n < 1 || steps < 0 || !(lr > 0)) return fail(HSS_EINVAL, "bad mlp arguments");
    ensure_device();
    hss::mlp_train(w, x, t, n, steps, lr, loss_hist, (hipStream_t)stream);
    return HSS_OK;
  });
}

}  // extern "C"

#include "../../include/hss_debug.h"

namespace hss {
void debug_gemm(int scalar, int nb, const void* const* A, const void* const* B, void* const* C, const int32_t* M,
                const int32_t* N, const int32_t* K, const int32_t* lda, const int32_t* ldb, const int32_t* ldc,
                const double* al, const double* be, hipStream_t st);
void debug_gj(int scalar, int nb, void* const* Mat, const int32_t* n, const int32_t* m, int block,
              int32_t* singular, hipStream_t st);
void debug_row_id(int scalar, const void* Zt, int m, int l, double thresh, int p_os, int32_t* k, int32_t* skel,
                  void* U, float* tmax, hipStream_t st);
}  // namespace hss

extern "C" {
hss_status_t hss_debug_gemm(int32_t scalar, int32_t nbatch, const void* const* A, const void* const* B,
                            void* const* C, const int32_t* M, const int32_t* N, const int32_t* K,
                            const int32_t* lda, const int32_t* ldb, const int32_t* ldc, const double* alpha,
                            const double* beta, void* hip_stream) {
  return guarded([&]() -> hss_status_t {
    if (nbatch < 0 || !A || !B || !C || !M || !N || !K || !lda || !ldb || !ldc || !alpha || !beta)
      return fail(HSS_EINVAL, "bad gemm arguments");
    for (int b = 0; b < nbatch; ++b)
      if (M[b] < 0 || N[b] < 0 || K[b] < 0 || lda[b] < std::max(1, M[b]) || ldb[b] < std::max(1, K[b]) ||
          ldc[b] < std::max(1, M[b]))
        return fail(HSS_EINVAL, "bad gemm sizes");
    ensure_device();
    hss::debug_gemm(scalar, nbatch, A, B, C, M, N, K, lda, ldb, ldc, alpha, beta, (hipStream_t)hip_stream);
    return HSS_OK;
  });
}

hss_status_t hss_debug_gj(int32_t scalar, int32_t nbatch, void* const* Mat, const int32_t* n, const int32_t* m,
                          int32_t block, int32_t* singular, void* hip_stream) {
  return guarded([&]() -> hss_status_t {
    if (nbatch < 0 || !Mat || !n || !m || !singular) return fail(HSS_EINVAL, "bad gj arguments");
    if (block < 0 || block > 256) return fail(HSS_EINVAL, "gj block width must be in [0, 256]");
    for (int b = 0; b < nbatch; ++b)
      if (n[b] < 0 || m[b] < 0) return fail(HSS_EINVAL, "bad gj sizes");
    ensure_device();
    hss::tuning_load_default();
    hss::debug_gj(scalar, nbatch, Mat, n, m, block, singular, (hipStream_t)hip_stream);
    return HSS_OK;
  });
}

hss_status_t hss_debug_row_id(int32_t scalar, const void* Zt, int32_t m, int32_t l, double thresh, int32_t p_os,
                              int32_t* k, int32_t* skel, void* U, float* tmax, void* hip_stream) {
  return guarded([&]() -> hss_status_t {
    if (!Zt || !k || !skel || !U || !tmax) return fail(HSS_EINVAL, "bad row id arguments");
    if (m < 1 || m > 1024 || l < 1 || l > 512 || p_os < 0 || !(thresh >= 0) || !std::isfinite(thresh))
      return fail(HSS_EINVAL, "row id sizes out of range");
    ensure_device();
    hss::debug_row_id(scalar, Zt, m, l, thresh, p_os, k, skel, U, tmax, (hipStream_t)hip_stream);
    return HSS_OK;
  });
}

hss_status_t hss_rank_model_train(const float* feat, const float* rank, int32_t n, const char* out_path,
                                  uint64_t seed) {
  return guarded([&]() -> hss_status_t {
    if (!feat || !rank || !out_path || n < 1) return fail(HSS_EINVAL, "bad rank model arguments");
    ensure_device();
    hss::rank_model_train(feat, rank, n, out_path, seed);
    return HSS_OK;
  });
}
}  // extern "C"
