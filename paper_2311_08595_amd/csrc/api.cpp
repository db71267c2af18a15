// C ABI entry points (declared in include/sttsv.h).  Every function returns an
// STTSV_* code; C++ exceptions never cross this boundary.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "internal.hpp"

using sttsv::Plan;

struct sttsv_plan_s {
  Plan* p;
};

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return STTSV_ENOMEM;
  } catch (...) {
    return STTSV_EINVAL;
  }
}

template <typename S, typename D>
int copy_out(const std::vector<S>& src, void* out, int64_t count) {
  if ((int64_t)src.size() != count) return STTSV_EINVAL;
  D* o = static_cast<D*>(out);
  for (int64_t i = 0; i < count; ++i) o[i] = static_cast<D>(src[i]);
  return STTSV_OK;
}

}  // namespace

// Alg. 3 baseline launch sequence (naive.hip); contraction and SS-HOPM (sshopm.hip)
namespace sttsv {
hipError_t launch_sttsv_naive(Plan& p, const double* x, double* y, hipStream_t s);
int contract(Plan& p, const double* x, double* y, double* out);
int contract_noalloc(Plan& p, const double* x, double* y, double* out);
int zeig_sshopm(Plan& p, const double* x0, double alpha, double tol, int32_t max_iter, double* x,
                sttsv_zeig_info* info);
}

extern "C" {

int sttsv_plan(const int64_t* eptr, const int32_t* eidx, int64_t m, int32_t n, int32_t r,
               const sttsv_opts* opts, sttsv_plan_t* out) {
  if (out == nullptr) return STTSV_EINVAL;
  return guarded([&] {
    Plan* p = nullptr;
    const sttsv::GraphIn g{eptr, eidx, m, n, r, opts != nullptr ? opts->edge_weights : nullptr};
    const int rc = sttsv::build_plan(1, &g, opts, &p);
    if (rc != STTSV_OK) return rc;
    *out = new sttsv_plan_s{p};
    return STTSV_OK;
  });
}

int sttsv_plan_batch(int32_t G, const sttsv_graph_desc* gs, const sttsv_opts* opts, sttsv_plan_t* out) {
  if (out == nullptr || gs == nullptr || G < 1) return STTSV_EINVAL;
  if (opts != nullptr && opts->edge_weights != nullptr) return STTSV_EINVAL;   // weights come per graph
  return guarded([&] {
    std::vector<sttsv::GraphIn> in(G);
    for (int g = 0; g < G; ++g) in[g] = sttsv::GraphIn{gs[g].eptr, gs[g].eidx, gs[g].m, gs[g].n, gs[g].r, gs[g].w};
    Plan* p = nullptr;
    const int rc = sttsv::build_plan(G, in.data(), opts, &p);
    if (rc != STTSV_OK) return rc;
    *out = new sttsv_plan_s{p};
    return STTSV_OK;
  });
}

int sttsv_plan_graph_info(sttsv_plan_t plan, int32_t g, sttsv_graph_info* info) {
  if (plan == nullptr || plan->p == nullptr || info == nullptr) return STTSV_EINVAL;
  const Plan& p = *plan->p;
  if (g < 0 || g >= (int32_t)p.graphs.size()) return STTSV_EINVAL;
  const sttsv::GraphInfo& I = p.graphs[g];
  info->m = I.m;
  info->n = I.n;
  info->r = I.r;
  info->voff = I.voff;
  info->connected = I.connected ? 1 : 0;
  return STTSV_OK;
}

int sttsv_apply_prec(sttsv_plan_t plan, const double* x, double* y, int32_t precision) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr) return STTSV_EINVAL;
  if (precision != STTSV_PREC_FP64 && precision != STTSV_PREC_FP32) return STTSV_EINVAL;
  if (static_cast<const void*>(x) == static_cast<const void*>(y)) return STTSV_EINVAL;
  return guarded([&] {
    Plan& p = *plan->p;
    const hipError_t e = sttsv::launch_sttsv(p, x, y, precision, nullptr, p.stream);
    return e == hipSuccess ? STTSV_OK : STTSV_EHIP;
  });
}

int sttsv_apply_timed(sttsv_plan_t plan, const double* x, double* y, int32_t precision, int32_t cap,
                      int32_t* nstages, int32_t* kinds, int32_t* sizes, int64_t* counts, float* ms) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr || nstages == nullptr)
    return STTSV_EINVAL;
  if (precision != STTSV_PREC_FP64 && precision != STTSV_PREC_FP32) return STTSV_EINVAL;
  Plan& p = *plan->p;
  const int ns = sttsv::stage_count(p, precision);
  *nstages = ns;
  if (cap < ns || kinds == nullptr || sizes == nullptr || counts == nullptr || ms == nullptr) return STTSV_EINVAL;
  return guarded([&] {
    std::vector<hipEvent_t> ev(ns + 1, nullptr);
    int rc = STTSV_OK;
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) rc = STTSV_EHIP;
    if (rc == STTSV_OK && hipEventRecord(ev[0], p.stream) != hipSuccess) rc = STTSV_EHIP;
    for (int t = 0; t < ns && rc == STTSV_OK; ++t) {
      if (sttsv::launch_stage(p, t, x, y, precision, nullptr, p.stream) != hipSuccess) rc = STTSV_EHIP;
      if (rc == STTSV_OK && hipEventRecord(ev[t + 1], p.stream) != hipSuccess) rc = STTSV_EHIP;
    }
    if (rc == STTSV_OK && hipEventSynchronize(ev[ns]) != hipSuccess) rc = STTSV_EHIP;
    for (int t = 0; t < ns && rc == STTSV_OK; ++t) {
      sttsv::stage_desc(p, precision, t, &kinds[t], &sizes[t], &counts[t]);
      if (hipEventElapsedTime(&ms[t], ev[t], ev[t + 1]) != hipSuccess) rc = STTSV_EHIP;
    }
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    return rc;
  });
}

int sttsv_plan_autotune(sttsv_plan_t plan, const double* x, int32_t reps, const char* cache_path,
                        int32_t* tuned) {
  if (plan == nullptr || plan->p == nullptr) return STTSV_EINVAL;
  return guarded([&] { return sttsv::autotune(*plan->p, x, reps, cache_path, tuned); });
}

int sttsv_apply_naive(sttsv_plan_t plan, const double* x, double* y) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr) return STTSV_EINVAL;
  if (static_cast<const void*>(x) == static_cast<const void*>(y)) return STTSV_EINVAL;
  return guarded([&] {
    Plan& p = *plan->p;
    const hipError_t e = sttsv::launch_sttsv_naive(p, x, y, p.stream);
    return e == hipSuccess ? STTSV_OK : STTSV_EHIP;
  });
}

int sttsv_contract(sttsv_plan_t plan, const double* x, double* y, double* out) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr || out == nullptr) return STTSV_EINVAL;
  if (static_cast<const void*>(x) == static_cast<const void*>(y)) return STTSV_EINVAL;
  return guarded([&] { return sttsv::contract(*plan->p, x, y, out); });
}

int sttsv_ccss_build(sttsv_plan_t plan, sttsv_ccss_info* info) {
  if (plan == nullptr || plan->p == nullptr) return STTSV_EINVAL;
  return guarded([&] { return sttsv::build_ccss(*plan->p, info); });
}

int sttsv_apply_ccss(sttsv_plan_t plan, const double* x, double* y) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr) return STTSV_EINVAL;
  if (static_cast<const void*>(x) == static_cast<const void*>(y)) return STTSV_EINVAL;
  if (plan->p->ccss == nullptr) return STTSV_EINVAL;
  return guarded([&] {
    Plan& p = *plan->p;
    return sttsv::launch_ccss(p, x, y, p.stream) == hipSuccess ? STTSV_OK : STTSV_EHIP;
  });
}

int sttsv_cp_objective_grad(sttsv_plan_t plan, int32_t R, const double* A, const double* lambda, double* f,
                            double* dA, double* dlambda) {
  if (plan == nullptr || plan->p == nullptr || A == nullptr || lambda == nullptr || f == nullptr || dA == nullptr ||
      dlambda == nullptr)
    return STTSV_EINVAL;
  return guarded([&] { return sttsv::cp_objective_grad(*plan->p, R, A, lambda, f, dA, dlambda); });
}

int sym_cp_descent(sttsv_plan_t plan, int32_t R, double* A, double* lambda, int32_t iters, double step,
                   sttsv_cp_info* info) {
  if (plan == nullptr || plan->p == nullptr || A == nullptr || lambda == nullptr) return STTSV_EINVAL;
  return guarded([&] { return sttsv::cp_descent(*plan->p, R, A, lambda, iters, step, info); });
}

int sttsv_contract_noalloc(sttsv_plan_t plan, const double* x, double* y, double* out) {
  if (plan == nullptr || plan->p == nullptr || x == nullptr || y == nullptr || out == nullptr) return STTSV_EINVAL;
  if (static_cast<const void*>(x) == static_cast<const void*>(y)) return STTSV_EINVAL;
  return guarded([&] { return sttsv::contract_noalloc(*plan->p, x, y, out); });
}

int zeigvec_sshopm(sttsv_plan_t plan, const double* x0, double alpha, double tol, int32_t max_iter,
                   double* x_out, sttsv_zeig_info* info) {
  if (plan == nullptr || plan->p == nullptr || x_out == nullptr) return STTSV_EINVAL;
  if (!(alpha >= 0.0) || !(tol >= 0.0) || max_iter < 0) return STTSV_EINVAL;
  return guarded([&] { return sttsv::zeig_sshopm(*plan->p, x0, alpha, tol, max_iter, x_out, info); });
}

int sttsv_apply(sttsv_plan_t plan, const double* x, double* y) {
  if (plan == nullptr || plan->p == nullptr) return STTSV_EINVAL;
  return sttsv_apply_prec(plan, x, y, plan->p->precision);
}

int heigvec_solve_ex(sttsv_plan_t plan, const double* x0, double tol, const sttsv_solve_opts* opts,
                     double* x_out, sttsv_solve_info* info) {
  if (plan == nullptr || plan->p == nullptr) return STTSV_EINVAL;
  sttsv_solve_opts o;
  o.max_iter = 500;
  o.check_every = 8;
  o.schedule = STTSV_SOLVE_FP64;
  o.use_graph = 1;
  o.shift = 0.0;
  o.switch_tol = 1e-4;
  if (opts != nullptr) o = *opts;
  if (plan->p->graphs.size() != 1) return STTSV_EINVAL;   // batches: heigvec_solve_batch
  return guarded([&] { return sttsv::solve(*plan->p, x0, tol, o, x_out, info); });
}

int heigvec_solve_batch(sttsv_plan_t plan, const double* x0, double tol, const sttsv_solve_opts* opts,
                        double* x_out, sttsv_solve_info* infos) {
  if (plan == nullptr || plan->p == nullptr) return STTSV_EINVAL;
  sttsv_solve_opts o;
  o.max_iter = 500;
  o.check_every = 8;
  o.schedule = STTSV_SOLVE_FP64;
  o.use_graph = 1;
  o.shift = 0.0;
  o.switch_tol = 1e-4;
  if (opts != nullptr) o = *opts;
  return guarded([&] { return sttsv::solve(*plan->p, x0, tol, o, x_out, infos); });
}

int heigvec_solve(sttsv_plan_t plan, const double* x0, double tol, double* x_out, sttsv_solve_info* info) {
  return heigvec_solve_ex(plan, x0, tol, nullptr, x_out, info);
}

int sttsv_plan_get_info(sttsv_plan_t plan, sttsv_plan_info* info) {
  if (plan == nullptr || plan->p == nullptr || info == nullptr) return STTSV_EINVAL;
  const Plan& p = *plan->p;
  info->m = p.m;
  info->nnz = p.nnz;
  info->n = p.n;
  info->r = p.r;
  info->nbuckets = static_cast<int32_t>(p.buckets.size());
  info->connected = p.connected ? 1 : 0;
  info->device_bytes = p.device_bytes;
  info->graphs = static_cast<int32_t>(p.graphs.size());
  info->lanes = (p.flags & STTSV_FLAG_ONE_STREAM) || p.ev_fork == nullptr ? 1 : p.lanes[0];
  return STTSV_OK;
}

int sttsv_plan_query(sttsv_plan_t plan, int32_t what, void* out, int64_t count) {
  if (plan == nullptr || plan->p == nullptr || out == nullptr) return STTSV_EINVAL;
  return guarded([&] {
    const Plan& p = *plan->p;
    switch (what) {
      case STTSV_Q_PERM:
        return copy_out<int64_t, int64_t>(p.perm, out, count);
      case STTSV_Q_MEM:
        return copy_out<int32_t, int64_t>(p.mem, out, count);
      case STTSV_Q_TPTR:
        return copy_out<int64_t, int64_t>(p.tptr, out, count);
      case STTSV_Q_TSLOT:
        return copy_out<int32_t, int64_t>(p.tslot, out, count);
      case STTSV_Q_BUCKET_STACK: {
        std::vector<int64_t> v;
        for (const auto& b : p.buckets) {
          int64_t f = 0;
          for (int t = 0; t < 2; ++t) {
            const bool generic = b.k >= 4 && b.small_kind[t] < 0 && b.coop[t] == 0;
            if (generic && b.desc[t].lds_stack == 1) f |= (1 << t);
            if (generic && b.desc[t].lds_stack == sttsv::kStackFree) f |= (4 << t);
          }
          v.push_back(f);
        }
        return copy_out<int64_t, int64_t>(v, out, count);
      }
      case STTSV_Q_BUCKET_K:
      case STTSV_Q_BUCKET_M:
      case STTSV_Q_BUCKET_R:
      case STTSV_Q_BUCKET_RUNS:
      case STTSV_Q_BUCKET_LANES: {
        std::vector<int64_t> v;
        for (const auto& b : p.buckets)
          v.push_back(what == STTSV_Q_BUCKET_K      ? b.k
                      : what == STTSV_Q_BUCKET_M    ? b.m
                      : what == STTSV_Q_BUCKET_R    ? b.r
                      : what == STTSV_Q_BUCKET_LANES ? b.coop[0]
                                                    : (b.reuse ? b.desc[0].nruns : 0));
        return copy_out<int64_t, int64_t>(v, out, count);
      }
      case STTSV_Q_WEIGHTS:
        return copy_out<double, double>(p.weights, out, count);
      case STTSV_Q_CCSS_LEVEL_N:
      case STTSV_Q_CCSS_VERT:
      case STTSV_Q_CCSS_PARENT:
      case STTSV_Q_CCSS_LEAF: {
        std::vector<int64_t> v;
        const int rc = sttsv::ccss_query(p, what, v);
        return rc != STTSV_OK ? rc : copy_out<int64_t, int64_t>(v, out, count);
      }
      case STTSV_Q_CONTRIB: {
        if (count != p.nnz) return STTSV_EINVAL;
        std::vector<double> c(p.nnz), v(p.nnz);
        if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;
        if (p.contrib_compact) {
          // an FP32 apply left 32-bit words (upper halves of FP64 values)
          std::vector<uint32_t> w(p.nnz);
          if (p.nnz > 0 && hipMemcpy(w.data(), p.d_contrib32, sizeof(uint32_t) * p.nnz, hipMemcpyDeviceToHost) != hipSuccess)
            return STTSV_EHIP;
          for (int64_t q = 0; q < p.nnz; ++q) {
            const uint64_t u = static_cast<uint64_t>(w[p.glist[q]]) << 32;
            std::memcpy(&v[q], &u, sizeof(double));
          }
        } else {
          if (p.nnz > 0 && hipMemcpy(c.data(), p.d_contrib, sizeof(double) * p.nnz, hipMemcpyDeviceToHost) != hipSuccess)
            return STTSV_EHIP;
          for (int64_t q = 0; q < p.nnz; ++q) v[q] = c[p.glist[q]];
        }
        return copy_out<double, double>(v, out, count);
      }
      case STTSV_Q_SCALE_EXP: {
        const int r0 = p.graphs[0].r;
        std::vector<int64_t> v(r0 + 1, INT32_MIN);
        for (const auto& b : p.buckets)
          if (b.r == r0 && b.k > 1 && b.fp32_ok) v[b.k] = b.qexp32;
        return copy_out<int64_t, int64_t>(v, out, count);
      }
      default:
        return STTSV_EINVAL;
    }
  });
}

int sttsv_plan_destroy(sttsv_plan_t plan) {
  if (plan == nullptr) return STTSV_OK;
  if (plan->p != nullptr) {
    (void)hipStreamSynchronize(plan->p->stream);
    sttsv::free_plan(plan->p);
  }
  delete plan;
  return STTSV_OK;
}

const char* sttsv_strerror(int code) {
  switch (code) {
    case STTSV_OK: return "ok";
    case STTSV_EINVAL: return "invalid argument or malformed hypergraph";
    case STTSV_ENOMEM: return "out of memory";
    case STTSV_EDISCONNECTED: return "hypergraph not connected (H-eigenvector needs a connected hypergraph)";
    case STTSV_ENOTCONV: return "solver did not converge within max_iter";
    case STTSV_ENUMERIC: return "non-finite or non-positive value in the solve";
    case STTSV_EHIP: return "HIP runtime error";
    case STTSV_ENOTSUP: return "outside the supported range";
    default: return "unknown error";
  }
}

}  // extern "C"
