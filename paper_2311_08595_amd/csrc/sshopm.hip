// Consumers of STTSV beyond H-eigenvector centrality (Sec. I names the
// shifted power method for tensor eigenpairs as one whose bottleneck is
// STTSV):
//  * the full contraction B x^r = x . (B x^(r-1));
//  * Z-eigenpairs (B x^(r-1) = lambda x, ||x||_2 = 1) by the shifted
//    symmetric higher-order power method of Kolda and Mayo, convex form:
//        w = B x^(r-1) + alpha x,  x <- w / ||w||_2,  lambda = x . B x^(r-1),
//    stopped when |lambda_k - lambda_(k-1)| <= tol |lambda_k| (tol = 0: after
//    max_iter updates).
// Every vector operation is a kernel here; the sums use a fixed grid and a
// fixed tree, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace sttsv {
namespace {

constexpr int kZBlock = 256;
constexpr int kZGrid = 512;   // fixed: the reduction tree does not depend on the device
static_assert(kZGrid == 2 * kZBlock, "z_final sums two partials per thread");

// Per-block partial sums of x.y, |y + alpha x|^2 and |y|^2 (grid-stride over
// v, then a fixed binary tree in LDS).  part[3 b + {0,1,2}].
__global__ void __launch_bounds__(kZBlock) z_stage(const double* x, const double* y,
                                                   int64_t n, double alpha, double* __restrict__ part) {
  __shared__ double sh[3][kZBlock];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t v = blockIdx.x * (int64_t)kZBlock + threadIdx.x; v < n; v += (int64_t)kZGrid * kZBlock) {
    const double xv = x[v], yv = y[v];
    const double w = yv + alpha * xv;
    a += xv * yv;
    b += w * w;
    c += yv * yv;
  }
  const int t = threadIdx.x;
  sh[0][t] = a;
  sh[1][t] = b;
  sh[2][t] = c;
  for (int s = kZBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s) {
      sh[0][t] += sh[0][t + s];
      sh[1][t] += sh[1][t + s];
      sh[2][t] += sh[2][t + s];
    }
  }
  if (t == 0) {
    part[3 * blockIdx.x + 0] = sh[0][0];
    part[3 * blockIdx.x + 1] = sh[1][0];
    part[3 * blockIdx.x + 2] = sh[2][0];
  }
}

// One block: the kZGrid partials of each quantity in a fixed tree -> st[0..2].
__global__ void __launch_bounds__(kZBlock) z_final(const double* __restrict__ part, double* __restrict__ st) {
  __shared__ double sh[3][kZBlock];
  const int t = threadIdx.x;
  for (int q = 0; q < 3; ++q) sh[q][t] = part[3 * t + q] + part[3 * (t + kZBlock) + q];
  for (int s = kZBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s)
      for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + s];
  }
  if (t == 0)
    for (int q = 0; q < 3; ++q) st[q] = sh[q][0];
}

// x <- (y + alpha x) / sqrt(st[1])   (or x <- y / sqrt(st[2]) with alpha unused
// when from_c: the first normalisation, y = x0)
// (y may be x itself in the first normalisation: each thread reads, then
// writes, only its own entry)
__global__ void __launch_bounds__(kZBlock) z_update(double* x, const double* y, int64_t n, double alpha,
                                                    const double* __restrict__ st, int from_c) {
  const int64_t v = blockIdx.x * (int64_t)kZBlock + threadIdx.x;
  if (v >= n) return;
  const double nrm = sqrt(from_c ? st[2] : st[1]);
  const double w = from_c ? y[v] : y[v] + alpha * x[v];
  x[v] = w / nrm;
}

__global__ void __launch_bounds__(kZBlock) z_fill(double* __restrict__ x, int64_t n, double val) {
  const int64_t v = blockIdx.x * (int64_t)kZBlock + threadIdx.x;
  if (v < n) x[v] = val;
}

struct ZScratch {
  double* part = nullptr;   // 3 kZGrid block partials
  double* st = nullptr;     // the three totals
};

// st[0..2] for (x, y, alpha), copied to host h[0..2] (synchronises the stream)
hipError_t reduce3(const double* x, const double* y, int64_t n, double alpha, const ZScratch& z, hipStream_t s,
                   double* h) {
  hipLaunchKernelGGL(z_stage, dim3(kZGrid), dim3(kZBlock), 0, s, x, y, n, alpha, z.part);
  hipLaunchKernelGGL(z_final, dim3(1), dim3(kZBlock), 0, s, (const double*)z.part, z.st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(h, z.st, 3 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

unsigned vgrid(int64_t n) { return static_cast<unsigned>((n + kZBlock - 1) / kZBlock); }

}  // namespace

// Per-plan SS-HOPM state, allocated on first use and kept until the plan is
// destroyed: the iterate, B x^(r-1), reduction partials, a device control
// block with its pinned host mirror, and the captured graph of kZSteps updates.
struct ZCtrl {
  double lam;        // lambda at the current iterate
  double alpha;      // shift
  double tol;        // stopping tolerance (0: run max_iter updates)
  int32_t iter;      // updates taken
  int32_t max_iter;
  int32_t done;      // no further update (converged, max_iter or numeric stop)
  int32_t conv;
  int32_t status;    // STTSV_OK or STTSV_ENUMERIC
  int32_t pad;
};

struct ZState {
  double* x = nullptr;
  double* y = nullptr;
  double* part = nullptr;
  double* st = nullptr;
  ZCtrl* ctrl = nullptr;
  ZCtrl* hctrl = nullptr;
  hipStream_t s = nullptr;      // own stream: the caller's may be the null stream, which cannot be captured
  hipGraphExec_t exec = nullptr;
};

constexpr int kZSteps = 8;   // updates per captured graph

namespace {

// The control step after each update's reductions (one thread): lambda, the
// stopping test, and the numeric check the next update needs (||w|| > 0).
__global__ void z_check(const double* __restrict__ st, ZCtrl* __restrict__ c) {
  if (c->done) return;
  const double lam = st[0];
  c->iter += 1;
  const bool conv = c->tol > 0.0 && fabs(lam - c->lam) <= c->tol * fabs(lam);
  c->lam = lam;
  if (conv) {
    c->conv = 1;
    c->done = 1;
  } else if (c->iter >= c->max_iter) {
    c->done = 1;
  } else if (!(st[1] > 0.0) || !isfinite(st[1])) {
    c->status = STTSV_ENUMERIC;
    c->done = 1;
  }
}

// The control block at the start: lambda_0 from the first reduction.
__global__ void z_ctrl_init(const double* __restrict__ st, ZCtrl* __restrict__ c, double alpha, double tol,
                            int32_t max_iter) {
  c->lam = st[0];
  c->alpha = alpha;
  c->tol = tol;
  c->iter = 0;
  c->max_iter = max_iter;
  c->conv = 0;
  c->status = STTSV_OK;
  c->done = max_iter <= 0 ? 1 : 0;
  if (!c->done && (!(st[1] > 0.0) || !isfinite(st[1]))) {
    c->status = STTSV_ENUMERIC;
    c->done = 1;
  }
}

// z_stage / z_final / z_update gated by the control block, shift read from it
__global__ void __launch_bounds__(kZBlock) z_stage_c(const double* x, const double* y, int64_t n,
                                                     const ZCtrl* __restrict__ c, double* __restrict__ part) {
  if (c->done) return;
  __shared__ double sh[3][kZBlock];
  const double alpha = c->alpha;
  double a = 0.0, b = 0.0, d = 0.0;
  for (int64_t v = blockIdx.x * (int64_t)kZBlock + threadIdx.x; v < n; v += (int64_t)kZGrid * kZBlock) {
    const double xv = x[v], yv = y[v];
    const double w = yv + alpha * xv;
    a += xv * yv;
    b += w * w;
    d += yv * yv;
  }
  const int t = threadIdx.x;
  sh[0][t] = a;
  sh[1][t] = b;
  sh[2][t] = d;
  for (int s = kZBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s) {
      sh[0][t] += sh[0][t + s];
      sh[1][t] += sh[1][t + s];
      sh[2][t] += sh[2][t + s];
    }
  }
  if (t == 0) {
    part[3 * blockIdx.x + 0] = sh[0][0];
    part[3 * blockIdx.x + 1] = sh[1][0];
    part[3 * blockIdx.x + 2] = sh[2][0];
  }
}

__global__ void __launch_bounds__(kZBlock) z_final_c(const double* __restrict__ part, const ZCtrl* __restrict__ c,
                                                     double* __restrict__ st) {
  if (c->done) return;
  __shared__ double sh[3][kZBlock];
  const int t = threadIdx.x;
  for (int q = 0; q < 3; ++q) sh[q][t] = part[3 * t + q] + part[3 * (t + kZBlock) + q];
  for (int s = kZBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s)
      for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + s];
  }
  if (t == 0)
    for (int q = 0; q < 3; ++q) st[q] = sh[q][0];
}

__global__ void __launch_bounds__(kZBlock) z_update_c(double* x, const double* y, int64_t n,
                                                      const double* __restrict__ st, const ZCtrl* __restrict__ c) {
  if (c->done) return;
  const int64_t v = blockIdx.x * (int64_t)kZBlock + threadIdx.x;
  if (v >= n) return;
  x[v] = (y[v] + c->alpha * x[v]) / sqrt(st[1]);
}

}  // namespace

void free_zstate(Plan& p) {
  ZState* z = p.zstate;
  if (z == nullptr) return;
  if (z->exec) (void)hipGraphExecDestroy(z->exec);
  for (void* q : {(void*)z->x, (void*)z->y, (void*)z->part, (void*)z->st, (void*)z->ctrl}) (void)hipFree(q);
  if (z->hctrl) (void)hipHostFree(z->hctrl);
  if (z->s) (void)hipStreamDestroy(z->s);
  delete z;
  p.zstate = nullptr;
}

static int get_zstate(Plan& p, ZState** out) {
  if (p.zstate == nullptr) {
    ZState* z = new ZState();
    p.zstate = z;
    const int64_t n = p.n;
    if (hipMalloc(&z->x, std::max<int64_t>(n, 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&z->y, std::max<int64_t>(n, 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&z->part, 3 * kZGrid * sizeof(double)) != hipSuccess ||
        hipMalloc(&z->st, 4 * sizeof(double)) != hipSuccess || hipMalloc(&z->ctrl, sizeof(ZCtrl)) != hipSuccess ||
        hipHostMalloc(&z->hctrl, sizeof(ZCtrl), hipHostMallocDefault) != hipSuccess) {
      free_zstate(p);
      return STTSV_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&z->s, hipStreamNonBlocking) != hipSuccess) {
      free_zstate(p);
      return STTSV_EHIP;
    }
    p.device_bytes += (2 * n + 3 * kZGrid + 4) * (int64_t)sizeof(double) + (int64_t)sizeof(ZCtrl);
  }
  *out = p.zstate;
  return STTSV_OK;
}

int contract(Plan& p, const double* x, double* y, double* out) {
  ZState* zs = nullptr;
  const int rc = get_zstate(p, &zs);
  if (rc != STTSV_OK) return rc;
  ZScratch z{zs->part, zs->st};
  hipStream_t s = p.stream;
  if (launch_sttsv(p, x, y, STTSV_PREC_FP64, nullptr, s) != hipSuccess) return STTSV_EHIP;
  double h[3];
  if (reduce3(x, y, p.n, 0.0, z, s, h) != hipSuccess) return STTSV_EHIP;
  *out = h[0];
  return STTSV_OK;
}

// ---- allocation-free contraction
// The reduction scratch of the contraction (kZGrid partials of three sums and
// the three totals) lives in one file-scope device array per GPU, so the entry
// point below calls no allocator.  Host code must not pass the array's name
// to a kernel: that name is a host-side stand-in.  The device address comes
// from hipGetSymbolAddress, taken once per device and kept in g_scratch_ptr.
constexpr int kScratchDoubles = 3 * kZGrid + 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int contract_noalloc(Plan& p, const double* x, double* y, double* out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return STTSV_EHIP;
  if (dev != p.device) return STTSV_EINVAL;               // the plan's device must be current
  if (dev < 0 || dev >= kMaxDevices) return STTSV_ENOTSUP;
  double* sp = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
      void* a = nullptr;
      if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || a == nullptr) return STTSV_EHIP;
      g_scratch_ptr[dev] = static_cast<double*>(a);
    }
    sp = g_scratch_ptr[dev];
  }
  // the scratch need does not grow with the plan: kZGrid partials of three
  // sums and three totals, every entry written before it is read
  static_assert(3 * kZGrid + 3 <= kScratchDoubles, "contraction scratch exceeds the static array");
  hipStream_t s = p.stream;
  if (launch_sttsv(p, x, y, STTSV_PREC_FP64, nullptr, s) != hipSuccess) return STTSV_EHIP;
  ZScratch z{sp, sp + 3 * kZGrid};
  double h[3];
  if (reduce3(x, y, p.n, 0.0, z, s, h) != hipSuccess) return STTSV_EHIP;
  *out = h[0];
  return STTSV_OK;
}

// One update: x <- (y + alpha x)/||.||, y = B x^(r-1), the three sums, the
// control step.  Every kernel (the STTSV's through its done flag) does nothing
// once the control block says done.
static hipError_t enqueue_update(Plan& p, ZState& z, hipStream_t s) {
  const int64_t n = p.n;
  hipLaunchKernelGGL(z_update_c, dim3(vgrid(n)), dim3(kZBlock), 0, s, z.x, (const double*)z.y, n,
                     (const double*)z.st, (const ZCtrl*)z.ctrl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_sttsv(p, z.x, z.y, STTSV_PREC_FP64, &z.ctrl->done, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(z_stage_c, dim3(kZGrid), dim3(kZBlock), 0, s, (const double*)z.x, (const double*)z.y, n,
                     (const ZCtrl*)z.ctrl, z.part);
  hipLaunchKernelGGL(z_final_c, dim3(1), dim3(kZBlock), 0, s, (const double*)z.part, (const ZCtrl*)z.ctrl, z.st);
  hipLaunchKernelGGL(z_check, dim3(1), dim3(1), 0, s, (const double*)z.st, z.ctrl);
  return hipGetLastError();
}

int zeig_sshopm(Plan& p, const double* x0, double alpha, double tol, int32_t max_iter, double* x,
                sttsv_zeig_info* info) {
  const int64_t n = p.n;
  ZState* zp = nullptr;
  int rc = get_zstate(p, &zp);
  if (rc != STTSV_OK) return rc;
  ZState& z = *zp;
  ZScratch zr{z.part, z.st};
  // x0 may still be in flight on the plan's stream; the iteration runs on the
  // state's own stream and the call returns after it has finished
  if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;
  hipStream_t s = z.s;
  double h[3];
  // x = x0 / ||x0||_2 (x0 = all ones when absent)
  const double* src = x0;
  if (src == nullptr) {
    hipLaunchKernelGGL(z_fill, dim3(vgrid(n)), dim3(kZBlock), 0, s, z.x, n, 1.0);
    src = z.x;
  }
  if (reduce3(src, src, n, 0.0, zr, s, h) != hipSuccess) return STTSV_EHIP;
  if (!(h[2] > 0.0) || !std::isfinite(h[2])) return STTSV_ENUMERIC;
  hipLaunchKernelGGL(z_update, dim3(vgrid(n)), dim3(kZBlock), 0, s, z.x, src, n, 0.0, (const double*)z.st, 1);
  // lambda_0 and the control block
  if (launch_sttsv(p, z.x, z.y, STTSV_PREC_FP64, nullptr, s) != hipSuccess) return STTSV_EHIP;
  hipLaunchKernelGGL(z_stage, dim3(kZGrid), dim3(kZBlock), 0, s, (const double*)z.x, (const double*)z.y, n, alpha,
                     z.part);
  hipLaunchKernelGGL(z_final, dim3(1), dim3(kZBlock), 0, s, (const double*)z.part, z.st);
  hipLaunchKernelGGL(z_ctrl_init, dim3(1), dim3(1), 0, s, (const double*)z.st, z.ctrl, alpha, tol, max_iter);
  if (hipGetLastError() != hipSuccess) return STTSV_EHIP;
  // updates: a captured graph of kZSteps updates (shift and tolerance live in
  // the control block, so one graph serves every call on the plan), replayed
  // until the control block says done
  if (z.exec == nullptr) {
    if (hipStreamSynchronize(s) != hipSuccess) return STTSV_EHIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return STTSV_EHIP;
    hipError_t e = hipSuccess;
    for (int t = 0; t < kZSteps && e == hipSuccess; ++t) e = enqueue_update(p, z, s);
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return STTSV_EHIP;
    }
    e = hipGraphInstantiate(&z.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      z.exec = nullptr;
      return STTSV_EHIP;
    }
  }
  for (;;) {
    if (hipMemcpyAsync(z.hctrl, z.ctrl, sizeof(ZCtrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return STTSV_EHIP;
    if (z.hctrl->done) break;
    if (hipGraphLaunch(z.exec, s) != hipSuccess) return STTSV_EHIP;
  }
  const ZCtrl c = *z.hctrl;
  if (c.status != STTSV_OK) return c.status;
  // the result, and the residual ||B x^(r-1) - lambda x||_2 at it
  if (hipMemcpyAsync(x, z.x, n * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) return STTSV_EHIP;
  if (reduce3(z.x, z.y, n, -c.lam, zr, s, h) != hipSuccess) return STTSV_EHIP;   // synchronises s
  if (info) {
    info->iterations = c.iter;
    info->converged = c.conv;
    info->lambda = c.lam;
    info->residual = std::sqrt(h[1]);
  }
  return c.conv ? STTSV_OK : STTSV_ENOTCONV;
}

}  // namespace sttsv
