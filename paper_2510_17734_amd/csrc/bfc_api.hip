// extern "C" entry points of libbfc (declared in include/bfc.h).
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>

#include "bfc_device.h"

namespace bfc {

size_t inner_partial_bytes(int prec, int r);
size_t inner_factor_bytes(int r);

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {
// allocations that still succeed before one is made to fail; < 0: off
std::atomic<int64_t> g_fail_after{-1};
}

hipError_t lib_malloc(void** ptr, size_t bytes) {
  int64_t k = g_fail_after.load();
  while (k >= 0) {
    if (g_fail_after.compare_exchange_weak(k, k - 1)) {
      if (k == 0) {  // this one fails, as if the device were out of memory
        *ptr = nullptr;
        return hipErrorOutOfMemory;
      }
      break;
    }
  }
  return hipMalloc(ptr, bytes);
}

int64_t debug_fail_allocation_after(int64_t count) {
  return g_fail_after.exchange(count < 0 ? -1 : count);
}

bfc_status dev_alloc(Problem* P, void** ptr, size_t bytes) {
  hipError_t e = lib_malloc(ptr, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *ptr = nullptr;
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? BFC_ENOMEM : BFC_EHIP;
  }
  P->allocs.push_back(*ptr);
  return BFC_OK;
}

bfc_status dev_free(Problem* P, void* ptr) {
  for (size_t k = 0; k < P->allocs.size(); ++k)
    if (P->allocs[k] == ptr) {
      P->allocs.erase(P->allocs.begin() + k);
      BFC_HIP_TRY(hipDeviceSynchronize());  // no kernel may still use it
      BFC_HIP_TRY(hipFree(ptr));
      return BFC_OK;
    }
  set_error("internal: freeing an unknown allocation");
  return BFC_EHIP;
}

hipEvent_t Profiler::take() {
  if (pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = pool.back();
  pool.pop_back();
  return e;
}

ProfScope::ProfScope(Profiler* pr_, int kind_, hipStream_t st_) : pr(pr_), kind(kind_), st(st_) {
  if (!pr->on) return;
  a = pr->take();
  b = pr->take();
  if (a && b && hipEventRecord(a, st) == hipSuccess) return;
  a = b = nullptr;
}

ProfScope::~ProfScope() {
  if (!a || !b) return;
  if (hipEventRecord(b, st) == hipSuccess) pr->pending[kind].push_back({a, b});
}

}  // namespace bfc

struct bfc_problem : public bfc::Problem {};

namespace bfc {

static void release_events(Profiler& pr) {
  for (auto& v : pr.pending)
    for (auto& ab : v) {
      (void)hipEventDestroy(ab.first);
      (void)hipEventDestroy(ab.second);
    }
  for (auto& v : pr.pending) v.clear();
  for (hipEvent_t e : pr.pool) (void)hipEventDestroy(e);
  pr.pool.clear();
}

static void free_problem(bfc_problem* P) {
  (void)hipDeviceSynchronize();  // work enqueued before a failure may still use the buffers
  release_events(P->prof);
  if (P->sweep_exec) (void)hipGraphExecDestroy(P->sweep_exec);
  if (P->sweep_graph) (void)hipGraphDestroy(P->sweep_graph);
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  if (P->red_host) (void)hipHostFree(P->red_host);
  P->red_host = nullptr;
  delete P;
}

static bfc_status check_config(const bfc_config* cfg, int32_t* c_out) {
  if (!cfg) {
    set_error("null config");
    return BFC_EINVAL;
  }
  if (cfg->L < 0 || cfg->L > BFC_MAX_LEVELS) {
    set_error("L out of range");
    return BFC_EINVAL;
  }
  if (cfg->r < 1 || cfg->r > BFC_MAX_RANK) {
    set_error("r out of range [1, 12]");
    return BFC_EINVAL;
  }
  if (cfg->r > BFC_MAX_RANK_FULL && cfg->precision == BFC_C64_BF16GRAM) {
    set_error("the BF16-Gram mode supports r <= 8");
    return BFC_EINVAL;
  }
  const int64_t two_l = (int64_t)1 << cfg->L;
  if (cfg->n < 1 || cfg->n % two_l != 0 || cfg->n > 0x7FFFFFFF) {
    set_error("n must be a positive multiple of 2^L below 2^31");
    return BFC_EINVAL;
  }
  if (cfg->precision != BFC_C128 && cfg->precision != BFC_C64 &&
      cfg->precision != BFC_C64_BF16GRAM) {
    set_error("unknown precision");
    return BFC_EINVAL;
  }
  if (cfg->reg_mode != BFC_REG_PROXIMAL && cfg->reg_mode != BFC_REG_RIDGE) {
    set_error("unknown regularization mode");
    return BFC_EINVAL;
  }
  if (!(cfg->reg_rel >= 0.0)) {
    set_error("reg_rel must be >= 0");
    return BFC_EINVAL;
  }
  if (!(cfg->reg_floor >= 0.0 && cfg->reg_floor <= 0x1p-4)) {
    set_error("reg_floor must be in [0, 2^-4]");
    return BFC_EINVAL;
  }
  *c_out = (int32_t)(cfg->n / two_l);
  return BFC_OK;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int64_t bfc_num_params(int64_t n, int32_t L, int32_t r) { return bfc::num_params(n, L, r); }

const char* bfc_last_error(void) { return g_last_error.c_str(); }

bfc_status bfc_init_cores(const bfc_config* cfg, int64_t nnz, const int32_t* d_rows,
                          const int32_t* d_cols, const void* d_vals, const void* d_cores_init,
                          void* hip_stream, bfc_problem** out) {
  set_error("");
  if (!out) {
    set_error("null output pointer");
    return BFC_EINVAL;
  }
  *out = nullptr;
  int32_t c = 0;
  BFC_TRY(check_config(cfg, &c));
  if (nnz < 1 || nnz > 0x7FFFFFFF) {
    set_error("nnz must be in [1, 2^31)");
    return BFC_EINVAL;
  }
  if (!d_rows || !d_cols || !d_vals) {
    set_error("null entry array");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  bfc_problem* P = new (std::nothrow) bfc_problem();
  if (!P) {
    set_error("host allocation failed");
    return BFC_ENOMEM;
  }
  P->cfg = *cfg;
  P->n = cfg->n;
  P->L = cfg->L;
  P->r = cfg->r;
  P->c = c;
  P->prec = cfg->precision;
  P->nnz = nnz;
  P->elem = P->prec == BFC_C128 ? 16 : 8;
  P->nparams = num_params(P->n, P->L, P->r);
  bfc_status s = BFC_OK;
  auto fail = [&](bfc_status code) {
    free_problem(P);
    return code;
  };
  if ((s = dev_alloc(P, &P->cores, P->nparams * P->elem)) != BFC_OK) return fail(s);
  if ((s = dev_alloc(P, (void**)&P->flags, 64)) != BFC_OK) return fail(s);
  P->red_len = 2 * 2048;
  if ((s = dev_alloc(P, (void**)&P->red, (P->red_len + 2) * sizeof(double))) != BFC_OK)
    return fail(s);
  if (hipHostMalloc((void**)&P->red_host, 2 * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    set_error("hipHostMalloc failed");
    return fail(BFC_ENOMEM);
  }
  if (hipMemsetAsync(P->flags, 0, 64, st) != hipSuccess) {
    set_error("hipMemsetAsync failed");
    return fail(BFC_EHIP);
  }
  if ((s = build_layout(P, d_rows, d_cols, d_vals, st)) != BFC_OK) return fail(s);
  if ((s = dev_alloc(P, (void**)&P->fused_res, 2 * sizeof(double) * P->lay[P->L + 1].nblocks)) !=
      BFC_OK)
    return fail(s);
  if (P->max_items > 0) {
    P->partials_bytes = (size_t)P->max_items * inner_partial_bytes(P->prec, P->r);
    if ((s = dev_alloc(P, &P->partials, P->partials_bytes)) != BFC_OK) return fail(s);
    if (P->prec == BFC_C64_BF16GRAM) {
      const size_t d = (size_t)P->r * P->r, slices = (size_t)1 << (P->L + 1);
      if ((s = dev_alloc(P, &P->ir_part, (size_t)P->max_items * 2 * d * sizeof(float))) != BFC_OK)
        return fail(s);
      if ((s = dev_alloc(P, (void**)&P->ir_lam, slices * sizeof(double))) != BFC_OK)
        return fail(s);
      if ((s = dev_alloc(P, &P->ir_old, slices * d * 2 * sizeof(float))) != BFC_OK)
        return fail(s);
      if ((s = dev_alloc(P, &P->ir_fac, slices * inner_factor_bytes(P->r))) != BFC_OK)
        return fail(s);
    }
  }
  if (d_cores_init)
    s = launch_convert_cores(P, d_cores_init, nullptr, true, st);
  else
    s = launch_random_cores(P, cfg->seed, st);
  if (s != BFC_OK) return fail(s);
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error("hipStreamSynchronize failed");
    return fail(BFC_EHIP);
  }
  *out = P;
  return BFC_OK;
}

bfc_status bfc_sweep_core(bfc_problem* p, int32_t core, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  if (core < 0 || core > p->L + 1) {
    set_error("core index out of range [0, L+1]");
    return BFC_EINVAL;
  }
  return launch_sweep_core(p, core, (hipStream_t)hip_stream);
}

// The captured sweep recomputes every environment level it uses (the state
// a sweep reaches after any previous sweep), so replaying it is equivalent to
// issuing the L+2 core updates one by one.  After a sweep the left levels are
// current and the right levels stale, on either path.
static bfc_status sweep_via_graph(bfc_problem* p, hipStream_t st) {
  if (!p->sweep_exec) {
    invalidate_envs(p);
    BFC_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    bfc_status s = BFC_OK;
    for (int core = 0; core <= p->L + 1 && s == BFC_OK; ++core) s = launch_sweep_core(p, core, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != BFC_OK) {
      if (g) (void)hipGraphDestroy(g);
      invalidate_envs(p);
      return s;
    }
    BFC_HIP_TRY(e);
    // whether the captured last core update leaves the per-fiber residual
    // norms (the narrow ranks' outer kernel does, the wide ranks' does not)
    p->graph_fused_res = p->fused_res_valid;
    p->sweep_graph = g;
    BFC_HIP_TRY(hipGraphInstantiate(&p->sweep_exec, g, nullptr, nullptr, 0));
  }
  BFC_HIP_TRY(hipGraphLaunch(p->sweep_exec, st));
  // the state a sweep leaves (host-side bookkeeping the replay does not run)
  for (auto& E : p->rlev) E.valid = false;
  for (size_t q = 2; q < p->llev.size(); ++q) p->llev[q].valid = true;
  p->fused_res_valid = p->graph_fused_res;
  return BFC_OK;
}

bfc_status bfc_sweep(bfc_problem* p, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (p->use_graph && !p->prof.on && st != nullptr) return sweep_via_graph(p, st);
  for (int core = 0; core <= p->L + 1; ++core) BFC_TRY(launch_sweep_core(p, core, st));
  return BFC_OK;
}

bfc_status bfc_adam_sweep(bfc_problem* p, int32_t t, double alpha, double beta1, double beta2,
                          double sigma, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  if (t < 1 || !(alpha > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(sigma >= 0.0)) {
    set_error("bfc_adam_sweep: need t >= 1, alpha > 0, 0 <= beta1, beta2 < 1, sigma >= 0");
    return BFC_EINVAL;
  }
  if (p->r > BFC_MAX_RANK_FULL) {
    set_error("bfc_adam_sweep: supports r <= 8");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t real = p->elem / 2;
  if (!p->adam_m || !p->adam_v) {  // both moments or neither
    void *m = nullptr, *v = nullptr;
    BFC_TRY(dev_alloc(p, &m, (size_t)p->nparams * p->elem));
    const bfc_status sv = dev_alloc(p, &v, (size_t)p->nparams * real);
    if (sv != BFC_OK) {
      (void)dev_free(p, m);
      return sv;
    }
    if (p->adam_m) (void)dev_free(p, p->adam_m);
    if (p->adam_v) (void)dev_free(p, p->adam_v);
    p->adam_m = m;
    p->adam_v = v;
    BFC_HIP_TRY(hipMemsetAsync(p->adam_m, 0, (size_t)p->nparams * p->elem, st));
    BFC_HIP_TRY(hipMemsetAsync(p->adam_v, 0, (size_t)p->nparams * real, st));
  }
  if (p->L >= 1 && p->adam_part_items < p->max_items) {
    if (p->adam_part) BFC_TRY(dev_free(p, p->adam_part));
    p->adam_part = nullptr;
    BFC_TRY(dev_alloc(p, &p->adam_part,
                      (size_t)std::max(p->max_items, 1) * 2 * p->r * p->r * real));
    p->adam_part_items = std::max(p->max_items, 1);
  }
  for (int core = 0; core <= p->L + 1; ++core)
    BFC_TRY(launch_adam_core(p, core, t, alpha, beta1, beta2, sigma, st));
  return BFC_OK;
}

bfc_status bfc_adf_sweep(bfc_problem* p, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  if (p->r > BFC_MAX_RANK_FULL) {
    set_error("bfc_adf_sweep: supports r <= 8");
    return BFC_EINVAL;
  }
  if (p->c > 64 || p->c < p->r) {
    set_error("bfc_adf_sweep: the leaf blocks need r <= c = n / 2^L <= 64 rows");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t real = p->elem / 2;
  if (p->L >= 1 && p->adam_part_items < p->max_items) {
    if (p->adam_part) BFC_TRY(dev_free(p, p->adam_part));
    p->adam_part = nullptr;
    BFC_TRY(dev_alloc(p, &p->adam_part,
                      (size_t)std::max(p->max_items, 1) * 2 * p->r * p->r * real));
    p->adam_part_items = std::max(p->max_items, 1);
  }
  if (p->L >= 1 && !p->adf_dir)
    BFC_TRY(dev_alloc(p, &p->adf_dir, ((size_t)2 << p->L) * p->r * p->r * p->elem));
  return launch_adf_sweep(p, st);
}

bfc_status bfc_adam_reset(bfc_problem* p, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (p->adam_m) {
    BFC_HIP_TRY(hipMemsetAsync(p->adam_m, 0, (size_t)p->nparams * p->elem, st));
    BFC_HIP_TRY(hipMemsetAsync(p->adam_v, 0, (size_t)p->nparams * (p->elem / 2), st));
  }
  return BFC_OK;
}

bfc_status bfc_use_graphs(bfc_problem* p, int32_t enable) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  p->use_graph = enable != 0;
  return BFC_OK;
}

bfc_status bfc_predict_entries(const bfc_problem* p, int64_t m, const int32_t* d_rows,
                               const int32_t* d_cols, void* d_out, void* hip_stream) {
  if (!p || m < 0 || (m > 0 && (!d_rows || !d_cols || !d_out))) {
    set_error("bad predict arguments");
    return BFC_EINVAL;
  }
  return launch_predict(p, m, d_rows, d_cols, d_out, (hipStream_t)hip_stream);
}

bfc_status bfc_residual(const bfc_problem* p, int64_t m, const int32_t* d_rows,
                        const int32_t* d_cols, const void* d_vals, double out_sq[2],
                        void* hip_stream) {
  if (!p || m < 0 || !out_sq || (m > 0 && (!d_rows || !d_cols || !d_vals))) {
    set_error("bad residual arguments");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  double* dres = p->red + p->red_len;
  if (m == 0) {
    out_sq[0] = out_sq[1] = 0.0;
  } else {
    BFC_TRY(launch_residual(p, m, d_rows, d_cols, d_vals, dres, st));
    BFC_HIP_TRY(hipMemcpyAsync(p->red_host, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  int32_t nfail = 0;
  BFC_HIP_TRY(hipMemcpyAsync(&nfail, p->flags, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  if (m > 0) {
    out_sq[0] = p->red_host[0];
    out_sq[1] = p->red_host[1];
  }
  if (nfail) {
    BFC_HIP_TRY(hipMemsetAsync(p->flags, 0, 4, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    set_error("a regularized normal-equation matrix was not positive definite (" +
              std::to_string(nfail) + " blocks kept their values)");
    return BFC_ENOTSPD;
  }
  return BFC_OK;
}

// eq. (BF_convergence): sqrt(num / den) from the two norms, sqrt(num) when
// den = 0; the status of the residual call is passed on (ENOTSPD after
// filling *out).
static bfc_status relative_from(bfc_status s, const double sq[2], double* out) {
  if (s == BFC_OK || s == BFC_ENOTSPD) *out = sq[1] > 0.0 ? sqrt(sq[0] / sq[1]) : sqrt(sq[0]);
  return s;
}

bfc_status bfc_relative_error(const bfc_problem* p, int64_t m, const int32_t* d_rows,
                              const int32_t* d_cols, const void* d_vals, double* out,
                              void* hip_stream) {
  if (!out) {
    set_error("bad relative-error arguments");
    return BFC_EINVAL;
  }
  double sq[2] = {0.0, 0.0};
  return relative_from(bfc_residual(p, m, d_rows, d_cols, d_vals, sq, hip_stream), sq, out);
}

bfc_status bfc_relative_error_observed(bfc_problem* p, double* out, void* hip_stream) {
  if (!out) {
    set_error("bad relative-error arguments");
    return BFC_EINVAL;
  }
  double sq[2] = {0.0, 0.0};
  return relative_from(bfc_residual_observed(p, sq, hip_stream), sq, out);
}

bfc_status bfc_residual_observed(bfc_problem* p, double out_sq[2], void* hip_stream) {
  if (!p || !out_sq) {
    set_error("bad residual_observed arguments");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  double* dres = p->red + p->red_len;
  BFC_TRY(launch_residual_observed(p, dres, st));
  BFC_HIP_TRY(hipMemcpyAsync(p->red_host, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  int32_t nfail = 0;
  BFC_HIP_TRY(hipMemcpyAsync(&nfail, p->flags, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  out_sq[0] = p->red_host[0];
  out_sq[1] = p->red_host[1];
  if (nfail) {
    BFC_HIP_TRY(hipMemsetAsync(p->flags, 0, 4, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    set_error("a regularized normal-equation matrix was not positive definite (" +
              std::to_string(nfail) + " blocks kept their values)");
    return BFC_ENOTSPD;
  }
  return BFC_OK;
}

bfc_status bfc_get_cores(const bfc_problem* p, void* d_cores, void* hip_stream) {
  if (!p || !d_cores) {
    set_error("bad get_cores arguments");
    return BFC_EINVAL;
  }
  return launch_convert_cores(const_cast<bfc_problem*>(p), nullptr, d_cores, false,
                              (hipStream_t)hip_stream);
}

bfc_status bfc_set_cores(bfc_problem* p, const void* d_cores, void* hip_stream) {
  if (!p || !d_cores) {
    set_error("bad set_cores arguments");
    return BFC_EINVAL;
  }
  return launch_convert_cores(p, d_cores, nullptr, true, (hipStream_t)hip_stream);
}

bfc_status bfc_set_cores_f32(bfc_problem* p, const float* d_cores, void* hip_stream) {
  if (!p || !d_cores) {
    set_error("bad set_cores_f32 arguments");
    return BFC_EINVAL;
  }
  return launch_cores_from_f32(p, d_cores, (hipStream_t)hip_stream);
}

bfc_status bfc_set_values(bfc_problem* p, const void* d_vals, void* hip_stream) {
  if (!p || (!d_vals && p->nnz > 0)) {
    set_error("bad set_values arguments");
    return BFC_EINVAL;
  }
  if (!p->bad_flag) BFC_TRY(dev_alloc(p, (void**)&p->bad_flag, 4));
  return launch_set_values(p, d_vals, (hipStream_t)hip_stream);
}

bfc_status bfc_loss_gradient(bfc_problem* p, float scale, void* d_grad, int32_t grad_fp64,
                             double* loss, void* hip_stream) {
  if (!p || !d_grad || !(scale == scale)) {
    set_error("bad loss_gradient arguments");
    return BFC_EINVAL;
  }
  if (p->r > BFC_MAX_RANK_FULL) {
    set_error("bfc_loss_gradient: supports r <= 8");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t real = p->elem / 2;
  if (p->L >= 1 && p->adam_part_items < p->max_items) {
    if (p->adam_part) BFC_TRY(dev_free(p, p->adam_part));
    p->adam_part = nullptr;
    BFC_TRY(dev_alloc(p, &p->adam_part,
                      (size_t)std::max(p->max_items, 1) * 2 * p->r * p->r * real));
    p->adam_part_items = std::max(p->max_items, 1);
  }
  if (!p->grad) BFC_TRY(dev_alloc(p, &p->grad, (size_t)p->nparams * p->elem));
  BFC_TRY(launch_loss_gradient(p, scale, d_grad, grad_fp64 != 0, st));
  if (loss) {
    // the residual pass alone: pending solve-failure counts stay for
    // bfc_sync_status / bfc_residual_observed to report
    double* dres = p->red + p->red_len;
    BFC_TRY(launch_residual_observed(p, dres, st));
    BFC_HIP_TRY(hipMemcpyAsync(p->red_host, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    *loss = 0.5 * (double)scale * p->red_host[0];
  }
  return BFC_OK;
}

bfc_status bfc_loss_gradient_batch(bfc_problem* p, int32_t count, const void* const* d_vals,
                                   const float* const* d_cores, const float* scales,
                                   void* const* d_grads, int32_t grad_fp64, double* losses,
                                   void* hip_stream) {
  if (!p || count < 1 || !d_vals || !d_cores || !scales || !d_grads || !losses) {
    set_error("bad loss_gradient_batch arguments");
    return BFC_EINVAL;
  }
  for (int32_t b = 0; b < count; ++b)
    if (!d_vals[b] || !d_cores[b] || !d_grads[b] || !(scales[b] == scales[b])) {
      set_error("bfc_loss_gradient_batch: a NULL pointer or NaN scale at instance " +
                std::to_string(b));
      return BFC_EINVAL;
    }
  if (p->r > BFC_MAX_RANK_FULL) {
    set_error("bfc_loss_gradient_batch: supports r <= 8");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t real = p->elem / 2;
  if (p->L >= 1 && p->adam_part_items < p->max_items) {
    if (p->adam_part) BFC_TRY(dev_free(p, p->adam_part));
    p->adam_part = nullptr;
    BFC_TRY(dev_alloc(p, &p->adam_part,
                      (size_t)std::max(p->max_items, 1) * 2 * p->r * p->r * real));
    p->adam_part_items = std::max(p->max_items, 1);
  }
  if (!p->grad) BFC_TRY(dev_alloc(p, &p->grad, (size_t)p->nparams * p->elem));
  if (!p->bad_flag) BFC_TRY(dev_alloc(p, (void**)&p->bad_flag, 4));
  if (p->batch_res_cap < count) {
    void* fresh = nullptr;
    BFC_TRY(dev_alloc(p, &fresh, (size_t)count * 2 * sizeof(double)));
    if (p->batch_res) BFC_TRY(dev_free(p, p->batch_res));
    p->batch_res = (double*)fresh;
    p->batch_res_cap = count;
  }
  // the same launches as count calls of bfc_set_values, bfc_set_cores_f32
  // and bfc_loss_gradient, without their synchronizations
  BFC_HIP_TRY(hipMemsetAsync(p->bad_flag, 0, 4, st));
  for (int32_t b = 0; b < count; ++b) {
    BFC_TRY(enqueue_set_values(p, d_vals[b], st));
    BFC_TRY(launch_cores_from_f32(p, d_cores[b], st));
    BFC_TRY(launch_loss_gradient(p, scales[b], d_grads[b], grad_fp64 != 0, st));
    BFC_TRY(launch_residual_observed(p, p->batch_res + 2 * b, st));
  }
  std::vector<double> res((size_t)count * 2);
  int32_t bad = 0;
  BFC_HIP_TRY(hipMemcpyAsync(res.data(), p->batch_res, res.size() * sizeof(double),
                             hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipMemcpyAsync(&bad, p->bad_flag, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  for (int32_t b = 0; b < count; ++b) losses[b] = 0.5 * (double)scales[b] * res[2 * b];
  if (bad) {
    set_error("bfc_loss_gradient_batch: an instance's values hold a NaN or Inf");
    return BFC_ENONFINITE;
  }
  return BFC_OK;
}

bfc_status bfc_sync_status(bfc_problem* p, void* hip_stream) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  int32_t nfail = 0;
  BFC_HIP_TRY(hipMemcpyAsync(&nfail, p->flags, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  if (nfail) {
    BFC_HIP_TRY(hipMemsetAsync(p->flags, 0, 4, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
    set_error("a regularized normal-equation matrix was not positive definite (" +
              std::to_string(nfail) + " blocks kept their values)");
    return BFC_ENOTSPD;
  }
  return BFC_OK;
}

bfc_status bfc_profile_enable(bfc_problem* p, int32_t enable) {
  if (!p) {
    set_error("null problem");
    return BFC_EINVAL;
  }
  BFC_HIP_TRY(hipDeviceSynchronize());
  Profiler& pr = p->prof;
  for (auto& v : pr.pending) {
    for (auto& ab : v) {
      pr.pool.push_back(ab.first);
      pr.pool.push_back(ab.second);
    }
    v.clear();
  }
  for (int k = 0; k < KIND_COUNT; ++k) {
    pr.total_ms[k] = 0.0;
    pr.launches[k] = 0;
  }
  pr.on = enable != 0;
  return BFC_OK;
}

bfc_status bfc_profile_read(bfc_problem* p, int32_t kind, double* total_ms, int64_t* launches) {
  if (!p || kind < 0 || kind >= KIND_COUNT || !total_ms || !launches) {
    set_error("bad profile_read arguments");
    return BFC_EINVAL;
  }
  Profiler& pr = p->prof;
  for (int k = 0; k < KIND_COUNT; ++k) {
    for (auto& ab : pr.pending[k]) {
      BFC_HIP_TRY(hipEventSynchronize(ab.second));
      float ms = 0.f;
      BFC_HIP_TRY(hipEventElapsedTime(&ms, ab.first, ab.second));
      pr.total_ms[k] += ms;
      pr.launches[k] += 1;
      pr.pool.push_back(ab.first);
      pr.pool.push_back(ab.second);
    }
    pr.pending[k].clear();
  }
  *total_ms = pr.total_ms[kind];
  *launches = pr.launches[kind];
  return BFC_OK;
}

bfc_status bfc_solve_counters(bfc_problem* p, int32_t reset, int64_t out[2], void* hip_stream) {
  if (!p || !out) {
    set_error("bad solve_counters arguments");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  int32_t h[2] = {0, 0};
  BFC_HIP_TRY(hipMemcpyAsync(h, p->flags, 8, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  out[0] = h[0];
  out[1] = h[1];
  if (reset) {
    BFC_HIP_TRY(hipMemsetAsync(p->flags, 0, 8, st));
    BFC_HIP_TRY(hipStreamSynchronize(st));
  }
  return BFC_OK;
}

bfc_status bfc_core_stats(const bfc_problem* p, int32_t core, int64_t out[7]) {
  if (!p || !out || core < 0 || core > p->L + 1) {
    set_error("bad core_stats arguments");
    return BFC_EINVAL;
  }
  const CoreLayout& C = p->lay[core];
  const bool inner = core >= 1 && core <= p->L;
  out[0] = C.nblocks;
  out[1] = inner ? C.nruns : 0;
  out[2] = inner ? C.nsub : 0;
  out[3] = inner ? C.nitems : 0;
  out[4] = inner ? C.group_by_row : -1;
  out[5] = core <= p->L - 1 ? p->rlev[core].count : 0;
  out[6] = core >= 2 ? p->llev[core].count : 0;
  return BFC_OK;
}

void bfc_destroy(bfc_problem* p) {
  if (p) free_problem(p);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched sweeps
// ---------------------------------------------------------------------------
struct bfc_batch : public bfc::Batch {};

namespace bfc {
// Release the launch plan and its graph (the residual buffers stay).
void free_batch_plan(Batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  for (void* p : B->allocs)
    if (p != B->res) (void)hipFree(p);
  B->allocs.assign(1, B->res);
  B->sweep.clear();
  B->resid.clear();
  B->resid_fused.clear();
}
}  // namespace bfc

namespace {
void free_batch(bfc_batch* B) {
  free_batch_plan(B);
  if (B->res) (void)hipFree(B->res);
  if (B->res_host) (void)hipHostFree(B->res_host);
  delete B;
}

// Rebuild the plan when a problem's work items changed since it was made.
bfc_status refresh_batch(bfc_batch* B) {
  bool stale = false;
  for (size_t k = 0; k < B->probs.size(); ++k)
    stale = stale || B->versions[k] != B->probs[k]->layout_version;
  if (!stale) return BFC_OK;
  free_batch_plan(B);
  for (size_t k = 0; k < B->probs.size(); ++k) B->versions[k] = B->probs[k]->layout_version;
  return build_batch_plan(B);
}
}  // namespace

bfc_status bfc_batch_create(bfc_problem* const* problems, int32_t count, bfc_batch** out) {
  if (!out) {
    set_error("null output pointer");
    return BFC_EINVAL;
  }
  *out = nullptr;
  if (!problems || count < 1) {
    set_error("a batch needs at least one problem");
    return BFC_EINVAL;
  }
  for (int32_t k = 0; k < count; ++k) {
    if (!problems[k]) {
      set_error("null problem in batch");
      return BFC_EINVAL;
    }
    for (int32_t q = 0; q < k; ++q)
      if (problems[q] == problems[k]) {
        set_error("a problem appears twice in the batch");
        return BFC_EINVAL;
      }
    if (problems[k]->r > BFC_MAX_RANK_FULL) {
      set_error("bfc_batch_create: batches support r <= 8");
      return BFC_EINVAL;
    }
    if (problems[k]->prec != problems[0]->prec) {
      set_error("problems of one batch must share the arithmetic mode");
      return BFC_EINVAL;
    }
  }
  if (problems[0]->prec == BFC_C64_BF16GRAM) {
    set_error("batched sweeps take BFC_C128 or BFC_C64 problems");
    return BFC_EINVAL;
  }
  bfc_batch* B = new (std::nothrow) bfc_batch();
  if (!B) {
    set_error("host allocation failed");
    return BFC_ENOMEM;
  }
  B->prec = problems[0]->prec;
  for (int32_t k = 0; k < count; ++k) B->probs.push_back(problems[k]);
  bfc_status s = BFC_OK;
  if (lib_malloc((void**)&B->res, 2 * sizeof(double) * count) != hipSuccess ||
      hipHostMalloc((void**)&B->res_host, 2 * sizeof(double) * count, hipHostMallocDefault) !=
          hipSuccess) {
    if (B->res) (void)hipFree(B->res);
    B->res = nullptr;
    free_batch(B);
    set_error("batch allocation failed");
    return BFC_ENOMEM;
  }
  B->allocs.push_back(B->res);
  for (bfc::Problem* P : B->probs) B->versions.push_back(P->layout_version);
  if ((s = build_batch_plan(B)) != BFC_OK) {
    free_batch(B);
    return s;
  }
  *out = B;
  return BFC_OK;
}

bfc_status bfc_batch_sweep(bfc_batch* b, void* hip_stream) {
  if (!b) {
    set_error("null batch");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  BFC_TRY(refresh_batch(b));
  if (st != nullptr) {
    if (!b->exec) {
      BFC_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      bfc_status s = launch_batch(b->sweep, b->prec, st);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(st, &g);
      if (s != BFC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      BFC_HIP_TRY(e);
      b->graph = g;
      BFC_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    }
    BFC_HIP_TRY(hipGraphLaunch(b->exec, st));
  } else {
    BFC_TRY(launch_batch(b->sweep, b->prec, st));
  }
  // as after a single sweep: every right level is stale, every left level
  // current but the last one where the last core's update formed it itself
  for (bfc::Problem* P : b->probs) {
    for (auto& E : P->rlev) E.valid = false;
    for (size_t q = 2; q < P->llev.size(); ++q) P->llev[q].valid = true;
    if (P->lay[P->L + 1].up_node) P->llev[P->L + 1].valid = false;
    P->fused_res_valid = true;
  }
  return BFC_OK;
}

bfc_status bfc_batch_residuals(bfc_batch* b, double* out_sq, void* hip_stream) {
  if (!b || !out_sq) {
    set_error("bad batch_residuals arguments");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  BFC_TRY(refresh_batch(b));
  const size_t k = b->probs.size();
  // right after a (batched) sweep the last core's update has left per-fiber
  // norms; otherwise the residual reads the last left level of every problem
  bool fused = true;
  for (bfc::Problem* P : b->probs) fused = fused && P->fused_res_valid;
  if (fused) {
    BFC_TRY(launch_batch(b->resid_fused, b->prec, st));
  } else {
    for (bfc::Problem* P : b->probs) {
      bool stale = false;
      for (int q = 2; q <= P->L + 1; ++q) stale = stale || !P->llev[q].valid;
      if (stale) BFC_TRY(launch_residual_observed(P, P->red + P->red_len, st));
    }
    BFC_TRY(launch_batch(b->resid, b->prec, st));
  }
  BFC_HIP_TRY(hipMemcpyAsync(b->res_host, b->res, 2 * sizeof(double) * k, hipMemcpyDeviceToHost,
                             st));
  std::vector<int32_t> nfail(k, 0);
  for (size_t q = 0; q < k; ++q)
    BFC_HIP_TRY(hipMemcpyAsync(&nfail[q], b->probs[q]->flags, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  for (size_t q = 0; q < 2 * k; ++q) out_sq[q] = b->res_host[q];
  int64_t total = 0;
  for (size_t q = 0; q < k; ++q)
    if (nfail[q]) {
      total += nfail[q];
      BFC_HIP_TRY(hipMemsetAsync(b->probs[q]->flags, 0, 4, st));
    }
  if (total) {
    BFC_HIP_TRY(hipStreamSynchronize(st));
    set_error("a regularized normal-equation matrix was not positive definite (" +
              std::to_string(total) + " blocks kept their values)");
    return BFC_ENOTSPD;
  }
  return BFC_OK;
}

bfc_status bfc_batch_destroy(bfc_batch* b) {
  if (b) free_batch(b);
  return BFC_OK;
}

// ---------------------------------------------------------------------------
// work-item size and its autotuner
// ---------------------------------------------------------------------------
bfc_status bfc_set_item_size(bfc_problem* p, int32_t subgroups, void* hip_stream) {
  if (!p || subgroups < 0 || subgroups > 65536 || subgroups % 64 != 0) {
    set_error("item size must be 0 (automatic) or a multiple of 64 in [64, 65536]");
    return BFC_EINVAL;
  }
  if (p->r > BFC_MAX_RANK_FULL) {
    set_error("bfc_set_item_size (one work item per slice above r = 8): supports r <= 8");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  BFC_HIP_TRY(hipStreamSynchronize(st));
  // every core's new items planned on the host, every buffer that must grow
  // allocated, and only then the problem changed: a failed allocation leaves
  // it as it was
  const int L = p->L;
  std::vector<std::vector<WorkItem>> items(L + 1);
  std::vector<std::vector<int32_t>> tiles(L + 1);
  int32_t max_items = 0;
  for (int q = 1; q <= L; ++q) {
    plan_items(p, q, subgroups, items[q], tiles[q]);
    max_items = std::max(max_items, (int32_t)items[q].size());
  }
  std::vector<void*> fresh(L + 1, nullptr);
  void *partials = nullptr, *ir_part = nullptr;
  bfc_status s = BFC_OK;
  for (int q = 1; q <= L && s == BFC_OK; ++q)
    if ((int64_t)items[q].size() > p->lay[q].items_cap || !p->lay[q].items)
      s = dev_alloc(p, &fresh[q], std::max<size_t>(1, items[q].size()) * sizeof(WorkItem));
  const bool grow = max_items > p->max_items;
  if (s == BFC_OK && grow) {
    s = dev_alloc(p, &partials, (size_t)max_items * inner_partial_bytes(p->prec, p->r));
    if (s == BFC_OK && p->ir_part)
      s = dev_alloc(p, &ir_part, (size_t)max_items * 2 * p->r * p->r * sizeof(float));
  }
  if (s != BFC_OK) {
    const std::string msg = bfc_last_error();
    for (void* f : fresh)
      if (f) (void)dev_free(p, f);
    if (partials) (void)dev_free(p, partials);
    if (ir_part) (void)dev_free(p, ir_part);
    set_error(msg);
    return s;
  }
  for (int q = 1; q <= L; ++q) {
    CoreLayout& C = p->lay[q];
    if (fresh[q]) {
      if (C.items) BFC_TRY(dev_free(p, C.items));
      C.items = (WorkItem*)fresh[q];
      C.items_cap = (int32_t)std::max<size_t>(1, items[q].size());
    }
    BFC_TRY(install_items(p, q, items[q], tiles[q], st));
  }
  if (grow) {
    p->max_items = max_items;
    if (p->partials) BFC_TRY(dev_free(p, p->partials));
    p->partials = partials;
    p->partials_bytes = (size_t)max_items * inner_partial_bytes(p->prec, p->r);
    if (ir_part) {
      BFC_TRY(dev_free(p, p->ir_part));
      p->ir_part = ir_part;
    }
  }
  p->item_size = subgroups;
  // the captured sweep holds the old launch shapes and buffers
  if (p->sweep_exec) (void)hipGraphExecDestroy(p->sweep_exec);
  if (p->sweep_graph) (void)hipGraphDestroy(p->sweep_graph);
  p->sweep_exec = nullptr;
  p->sweep_graph = nullptr;
  ++p->layout_version;
  return BFC_OK;
}

bfc_status bfc_autotune_item_size(bfc_problem* const* problems, int32_t count, int32_t sweeps,
                                  const int32_t* candidates, int32_t ncand, int32_t* chosen,
                                  double* ms_per_sweep, void* hip_stream) {
  static const int32_t kDefault[] = {64, 128, 256, 512};
  if (!problems || count < 1 || sweeps < 1 || !chosen || (candidates && ncand < 1)) {
    set_error("bad autotune arguments");
    return BFC_EINVAL;
  }
  if (!candidates) {
    candidates = kDefault;
    ncand = 4;
  }
  for (int32_t c = 0; c < ncand; ++c)
    if (candidates[c] < 64 || candidates[c] % 64 != 0 || candidates[c] > 65536) {
      set_error("autotune candidates must be multiples of 64 in [64, 65536]");
      return BFC_EINVAL;
    }
  hipStream_t st = (hipStream_t)hip_stream;
  // the trial sweeps change the cores: keep a copy of every problem's cores
  std::vector<void*> saved(count, nullptr);
  auto release = [&]() {
    for (void* q : saved)
      if (q) (void)hipFree(q);
  };
  for (int32_t k = 0; k < count; ++k) {
    bfc_problem* P = problems[k];
    if (!P) {
      release();
      set_error("null problem");
      return BFC_EINVAL;
    }
    const size_t bytes = (size_t)P->nparams * P->elem;
    if (lib_malloc(&saved[k], bytes) != hipSuccess) {
      saved[k] = nullptr;
      release();
      set_error("autotune: no memory for the core copies");
      return BFC_ENOMEM;
    }
    if (hipMemcpyAsync(saved[k], P->cores, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      release();
      set_error("autotune: copy failed");
      return BFC_EHIP;
    }
  }
  auto restore = [&]() -> bfc_status {
    for (int32_t k = 0; k < count; ++k) {
      bfc_problem* P = problems[k];
      BFC_HIP_TRY(hipMemcpyAsync(P->cores, saved[k], (size_t)P->nparams * P->elem,
                                 hipMemcpyDeviceToDevice, st));
      BFC_HIP_TRY(hipMemsetAsync(P->flags, 0, 8, st));
      invalidate_envs(P);
    }
    BFC_HIP_TRY(hipStreamSynchronize(st));
    return BFC_OK;
  };
  bfc_batch* B = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bfc_status s = BFC_OK;
  double best = 0.0;
  int32_t best_size = candidates[0];
  do {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      set_error("autotune: hipEventCreate failed");
      s = BFC_EHIP;
      break;
    }
    if (count > 1 && (s = bfc_batch_create(problems, count, &B)) != BFC_OK) break;
    auto one_sweep = [&]() -> bfc_status {
      if (B) return bfc_batch_sweep(B, st);
      return bfc_sweep(problems[0], st);
    };
    for (int32_t c = 0; c < ncand && s == BFC_OK; ++c) {
      for (int32_t k = 0; k < count && s == BFC_OK; ++k)
        s = bfc_set_item_size(problems[k], candidates[c], st);
      if (s != BFC_OK) break;
      if ((s = one_sweep()) != BFC_OK) break;  // warm-up (and graph capture)
      if (hipEventRecord(e0, st) != hipSuccess) s = BFC_EHIP;
      for (int32_t t = 0; t < sweeps && s == BFC_OK; ++t) s = one_sweep();
      if (s != BFC_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        set_error("autotune: event timing failed");
        s = BFC_EHIP;
        break;
      }
      const double per = ms / sweeps;
      if (ms_per_sweep) ms_per_sweep[c] = per;
      if (c == 0 || per < best) {
        best = per;
        best_size = candidates[c];
      }
      if ((s = restore()) != BFC_OK) break;
    }
  } while (false);
  if (B) bfc_batch_destroy(B);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s == BFC_OK) {
    for (int32_t k = 0; k < count && s == BFC_OK; ++k)
      s = bfc_set_item_size(problems[k], best_size, st);
    if (s == BFC_OK) s = restore();
    if (s == BFC_OK) *chosen = best_size;
  } else {
    (void)restore();
  }
  release();
  return s;
}
