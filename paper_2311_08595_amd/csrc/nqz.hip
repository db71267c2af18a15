// NQZ iteration (Alg. 1) on the GPU.
//
// Every step of an iteration is a kernel whose decisions live in a device
// control block, so K iterations can be captured once in a hipGraph and
// replayed; the host only reads the control block between replays.
//
// Iteration t (x~ = current iterate scaled to max 1):
//   z = TTSV1(x~)                            edge kernels + node reduction
//   z' = z + alpha x~^[r-1]                  optional shift (alpha = 0: Alg. 1)
//   lambda_v = z'_v / x~_v^(r-1)             min / max over v
//   crit = (lambda_max - lambda_min) / lambda_min;  stop if crit < tol
//   w = z'^[1/(r-1)];  x~ <- w / max(w)      next iterate (Alg. 1 divides by
//                                            the l1 norm; TTSV1 and x^[r-1]
//                                            are both homogeneous of degree
//                                            r-1 so the ratio, the test and
//                                            the normalised x are unchanged)
// The returned x is the iterate whose TTSV1 met the test, divided by its l1
// norm (a fixed-shape, deterministic sum).
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>

#include "internal.hpp"

namespace sttsv {

struct Ctrl {
  int32_t done;
  int32_t skip64;   // FP64-series edge kernels skip this iteration
  int32_t skip32;   // FP32-series edge kernels skip this iteration
  int32_t status;
  int32_t iter, it32, it64;
  int32_t max_iter;
  double tol, switch_tol, shift;
  double lmin, lmax, crit, prev_crit;
  double inv_wmax;
};

struct Solver {
  int32_t n = 0;
  hipStream_t s = nullptr;
  double* x = nullptr;      // current iterate, max-normalised
  double* z = nullptr;
  double* w = nullptr;
  double* part = nullptr;   // per-block partials
  Ctrl* ctrl = nullptr;     // device
  Ctrl* hctrl = nullptr;    // pinned host mirror
  hipGraphExec_t exec = nullptr;
  int graph_iters = 0;
  int graph_sched = -1;
};

namespace {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 1024;   // fixed: reduction shape depends on n only

int red_grid(int n) { return std::max(1, std::min(kRedGrid, (n + kRedBlock - 1) / kRedBlock)); }

__device__ __forceinline__ double block_min(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Initial iterate: x~ = x0 / max(x0) (or all ones for the uniform start).
// part[b] = {min x0, max x0, bad}
__global__ void __launch_bounds__(kRedBlock) init_stats(const double* x0, int n, double* part) {
  __shared__ double sh[kRedBlock];
  double lo = INFINITY, hi = 0.0, bad = 0.0;
  for (int v = blockIdx.x * kRedBlock + threadIdx.x; v < n; v += gridDim.x * kRedBlock) {
    const double a = x0[v];
    if (!(a > 0.0) || !isfinite(a)) bad = 1.0;
    lo = fmin(lo, a);
    hi = fmax(hi, a);
  }
  lo = block_min(lo, sh);
  hi = block_max(hi, sh);
  bad = block_max(bad, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = lo;
    part[3 * blockIdx.x + 1] = hi;
    part[3 * blockIdx.x + 2] = bad;
  }
}

__global__ void __launch_bounds__(kRedBlock) init_final(const double* part, int G, Ctrl* c) {
  __shared__ double sh[kRedBlock];
  double hi = 0.0, bad = 0.0;
  for (int b = threadIdx.x; b < G; b += kRedBlock) {
    hi = fmax(hi, part[3 * b + 1]);
    bad = fmax(bad, part[3 * b + 2]);
  }
  hi = block_max(hi, sh);
  bad = block_max(bad, sh);
  if (threadIdx.x == 0) {
    if (bad > 0.0) {
      c->done = 1;
      c->skip64 = c->skip32 = 1;
      c->status = STTSV_EINVAL;
    }
    c->inv_wmax = 1.0 / hi;
  }
}

__global__ void __launch_bounds__(kRedBlock) scale_into(const double* src, double* dst, int n, const Ctrl* c) {
  if (c->done) return;
  const int v = blockIdx.x * kRedBlock + threadIdx.x;
  if (v < n) dst[v] = src[v] * c->inv_wmax;
}

__global__ void __launch_bounds__(kRedBlock) fill_ones(double* dst, int n) {
  const int v = blockIdx.x * kRedBlock + threadIdx.x;
  if (v < n) dst[v] = 1.0;
}

// Per-vertex step after TTSV1: shifted z, ratio lambda, next w.
// part[b] = {min lambda, max lambda, max w, bad}
template <bool LAMBDA>
__global__ void __launch_bounds__(kRedBlock) nqz_stats(const double* x, const double* z, double* w, int n,
                                                       int r, double* part, const Ctrl* c) {
  if (c->done) return;
  __shared__ double sh[kRedBlock];
  const double shift = c->shift;
  const double inv = 1.0 / double(r - 1);
  double lo = INFINITY, hi = -INFINITY, wm = 0.0, bad = 0.0;
  for (int v = blockIdx.x * kRedBlock + threadIdx.x; v < n; v += gridDim.x * kRedBlock) {
    const double xv = x[v];
    const double p = pow(xv, double(r - 1));
    const double zz = shift != 0.0 ? fma(shift, p, z[v]) : z[v];
    if (!(zz > 0.0) || !isfinite(zz)) bad = 1.0;
    if (LAMBDA) {
      const double lam = zz / p;
      lo = fmin(lo, lam);
      hi = fmax(hi, lam);
    }
    const double wv = pow(zz, inv);
    w[v] = wv;
    wm = fmax(wm, wv);
  }
  lo = block_min(lo, sh);
  hi = block_max(hi, sh);
  wm = block_max(wm, sh);
  bad = block_max(bad, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = lo;
    part[4 * blockIdx.x + 1] = hi;
    part[4 * blockIdx.x + 2] = wm;
    part[4 * blockIdx.x + 3] = bad;
  }
}

template <bool LAMBDA>
__global__ void __launch_bounds__(kRedBlock) nqz_final(const double* part, int G, Ctrl* c) {
  if (c->done) return;
  __shared__ double sh[kRedBlock];
  double lo = INFINITY, hi = -INFINITY, wm = 0.0, bad = 0.0;
  for (int b = threadIdx.x; b < G; b += kRedBlock) {
    lo = fmin(lo, part[4 * b]);
    hi = fmax(hi, part[4 * b + 1]);
    wm = fmax(wm, part[4 * b + 2]);
    bad = fmax(bad, part[4 * b + 3]);
  }
  lo = block_min(lo, sh);
  hi = block_max(hi, sh);
  wm = block_max(wm, sh);
  bad = block_max(bad, sh);
  if (threadIdx.x != 0) return;
  if (bad > 0.0 || !(wm > 0.0) || !isfinite(wm)) {
    c->done = 1;
    c->skip64 = c->skip32 = 1;
    c->status = STTSV_ENUMERIC;
    return;
  }
  c->inv_wmax = 1.0 / wm;
  if (!LAMBDA) return;
  const bool ran64 = c->skip64 == 0;
  const double crit = (hi - lo) / lo;
  c->iter += 1;
  if (ran64)
    c->it64 += 1;
  else
    c->it32 += 1;
  c->lmin = lo;
  c->lmax = hi;
  c->crit = crit;
  if (ran64) {
    if (crit < c->tol) {
      c->done = 1;
      c->status = STTSV_OK;
    }
  } else if (crit < c->switch_tol || crit < c->tol || crit > 0.8 * c->prev_crit) {
    c->skip64 = 0;   // FP32 series have done what they can: polish in FP64
    c->skip32 = 1;
  }
  c->prev_crit = crit;
  if (!c->done && c->iter >= c->max_iter) {
    c->done = 1;
    c->status = STTSV_ENOTCONV;
  }
  if (c->done) c->skip64 = c->skip32 = 1;
}

__global__ void __launch_bounds__(kRedBlock) sum_stage(const double* x, int n, double* part) {
  __shared__ double sh[kRedBlock];
  double acc = 0.0;
  for (int v = blockIdx.x * kRedBlock + threadIdx.x; v < n; v += gridDim.x * kRedBlock) acc += x[v];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kRedBlock) sum_final(const double* part, int G, double* out) {
  __shared__ double sh[kRedBlock];
  double acc = 0.0;
  for (int b = threadIdx.x; b < G; b += kRedBlock) acc += part[b];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = acc;
}

__global__ void __launch_bounds__(kRedBlock) divide_by(const double* x, const double* s, double* out, int n) {
  const int v = blockIdx.x * kRedBlock + threadIdx.x;
  if (v < n) out[v] = x[v] / *s;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? STTSV_OK : STTSV_EHIP; }

// One NQZ iteration (all launches on S.s).
hipError_t enqueue_iteration(Plan& p, Solver& S, int schedule) {
  hipError_t e;
  const int G = red_grid(S.n);
  if (schedule == STTSV_SOLVE_FP32_FP64) {
    if ((e = launch_sttsv(p, S.x, S.z, STTSV_PREC_FP32, &S.ctrl->skip32, S.s)) != hipSuccess) return e;
  }
  // FP64 pass: its edge kernels and its reduction run only when skip64 == 0,
  // those of the FP32 pass above only when skip32 == 0.
  if ((e = launch_sttsv(p, S.x, S.z, STTSV_PREC_FP64, &S.ctrl->skip64, S.s)) != hipSuccess) return e;
  hipLaunchKernelGGL((nqz_stats<true>), dim3(G), dim3(kRedBlock), 0, S.s, S.x, S.z, S.w, S.n, p.r, S.part, S.ctrl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((nqz_final<true>), dim3(1), dim3(kRedBlock), 0, S.s, S.part, G, S.ctrl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scale_into, dim3((S.n + kRedBlock - 1) / kRedBlock), dim3(kRedBlock), 0, S.s, S.w, S.x, S.n,
                     S.ctrl);
  return hipGetLastError();
}

}  // namespace

void free_solver(Plan& p) {
  Solver* S = p.solver;
  if (S == nullptr) return;
  if (S->exec) (void)hipGraphExecDestroy(S->exec);
  (void)hipFree(S->x);
  (void)hipFree(S->z);
  (void)hipFree(S->w);
  (void)hipFree(S->part);
  (void)hipFree(S->ctrl);
  if (S->hctrl) (void)hipHostFree(S->hctrl);
  if (S->s) (void)hipStreamDestroy(S->s);
  delete S;
  p.solver = nullptr;
}

static int ensure_solver(Plan& p) {
  if (p.solver != nullptr) return STTSV_OK;
  Solver* S = new Solver();
  p.solver = S;
  S->n = p.n;
  const size_t nb = size_t(p.n) * sizeof(double);
  if (hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) != hipSuccess) return STTSV_EHIP;
  if (hipMalloc(&S->x, nb) != hipSuccess || hipMalloc(&S->z, nb) != hipSuccess ||
      hipMalloc(&S->w, nb) != hipSuccess || hipMalloc(&S->part, 4 * kRedGrid * sizeof(double)) != hipSuccess ||
      hipMalloc(&S->ctrl, sizeof(Ctrl)) != hipSuccess)
    return STTSV_ENOMEM;
  if (hipHostMalloc(&S->hctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) return STTSV_ENOMEM;
  return STTSV_OK;
}

int solve(Plan& p, const double* x0, double tol, const sttsv_solve_opts& o, double* x_out,
          sttsv_solve_info* info) {
  if (!(tol > 0.0) || x_out == nullptr) return STTSV_EINVAL;
  if (o.max_iter < 1 || o.check_every < 1 || o.shift < 0.0) return STTSV_EINVAL;
  if (o.schedule != STTSV_SOLVE_FP64 && o.schedule != STTSV_SOLVE_FP32_FP64) return STTSV_EINVAL;
  if (!p.connected) return STTSV_EDISCONNECTED;
  int rc = ensure_solver(p);
  if (rc != STTSV_OK) return rc;
  Solver& S = *p.solver;
  const int n = p.n;
  const int G = red_grid(n);
  const dim3 gv((n + kRedBlock - 1) / kRedBlock);
  if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;

  // control block
  Ctrl c{};
  c.done = 0;
  c.skip64 = o.schedule == STTSV_SOLVE_FP32_FP64 ? 1 : 0;
  c.skip32 = o.schedule == STTSV_SOLVE_FP32_FP64 ? 0 : 1;
  c.status = STTSV_OK;
  c.max_iter = o.max_iter;
  c.tol = tol;
  c.switch_tol = o.switch_tol;
  c.shift = o.shift;
  c.prev_crit = INFINITY;
  c.crit = INFINITY;
  if (hipMemcpyAsync(S.ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, S.s) != hipSuccess) return STTSV_EHIP;

  // initial iterate (Alg. 1: y = 1/n, or the warm start), then z = TTSV1(y)
  // and the first x; scale of y is irrelevant (homogeneity), so y / max(y).
  if (x0 == nullptr) {
    hipLaunchKernelGGL(fill_ones, gv, dim3(kRedBlock), 0, S.s, S.x, n);
  } else {
    hipLaunchKernelGGL(init_stats, dim3(G), dim3(kRedBlock), 0, S.s, x0, n, S.part);
    hipLaunchKernelGGL(init_final, dim3(1), dim3(kRedBlock), 0, S.s, S.part, G, S.ctrl);
    hipLaunchKernelGGL(scale_into, gv, dim3(kRedBlock), 0, S.s, x0, S.x, n, S.ctrl);
  }
  const int first_prec = o.schedule == STTSV_SOLVE_FP32_FP64 ? STTSV_PREC_FP32 : STTSV_PREC_FP64;
  if ((rc = hip_rc(launch_sttsv(p, S.x, S.z, first_prec, &S.ctrl->done, S.s))) != STTSV_OK) return rc;
  hipLaunchKernelGGL((nqz_stats<false>), dim3(G), dim3(kRedBlock), 0, S.s, S.x, S.z, S.w, n, p.r, S.part, S.ctrl);
  hipLaunchKernelGGL((nqz_final<false>), dim3(1), dim3(kRedBlock), 0, S.s, S.part, G, S.ctrl);
  hipLaunchKernelGGL(scale_into, gv, dim3(kRedBlock), 0, S.s, S.w, S.x, n, S.ctrl);
  if (hipGetLastError() != hipSuccess) return STTSV_EHIP;

  // iterations: captured graph of check_every iterations, or direct launches
  const int K = o.check_every;
  if (o.use_graph) {
    if (S.exec == nullptr || S.graph_iters != K || S.graph_sched != o.schedule) {
      if (S.exec) {
        (void)hipGraphExecDestroy(S.exec);
        S.exec = nullptr;
      }
      if (hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(S.s, hipStreamCaptureModeThreadLocal) != hipSuccess) return STTSV_EHIP;
      hipError_t e = hipSuccess;
      for (int t = 0; t < K && e == hipSuccess; ++t) e = enqueue_iteration(p, S, o.schedule);
      hipError_t e2 = hipStreamEndCapture(S.s, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return STTSV_EHIP;
      }
      e = hipGraphInstantiate(&S.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        S.exec = nullptr;
        return STTSV_EHIP;
      }
      S.graph_iters = K;
      S.graph_sched = o.schedule;
    }
  }
  for (;;) {
    if (o.use_graph) {
      if (hipGraphLaunch(S.exec, S.s) != hipSuccess) return STTSV_EHIP;
    } else {
      for (int t = 0; t < K; ++t)
        if (enqueue_iteration(p, S, o.schedule) != hipSuccess) return STTSV_EHIP;
    }
    if (hipMemcpyAsync(S.hctrl, S.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, S.s) != hipSuccess) return STTSV_EHIP;
    if (hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;
    if (S.hctrl->done) break;
  }
  const Ctrl& h = *S.hctrl;
  if (h.status == STTSV_EINVAL) return STTSV_EINVAL;   // warm start not > 0 / finite

  // x_out = x~ / ||x~||_1
  double* dsum = S.part + 4 * kRedGrid - 1;
  hipLaunchKernelGGL(sum_stage, dim3(G), dim3(kRedBlock), 0, S.s, S.x, n, S.part);
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(kRedBlock), 0, S.s, S.part, G, dsum);
  hipLaunchKernelGGL(divide_by, gv, dim3(kRedBlock), 0, S.s, S.x, dsum, x_out, n);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;

  if (info != nullptr) {
    info->iterations = h.iter;
    info->iters_fp32 = h.it32;
    info->iters_fp64 = h.it64;
    info->converged = h.status == STTSV_OK && h.iter > 0 ? 1 : 0;
    info->lambda_min = h.lmin - o.shift;
    info->lambda_max = h.lmax - o.shift;
    info->criterion = h.crit;
  }
  return h.status;
}

}  // namespace sttsv
