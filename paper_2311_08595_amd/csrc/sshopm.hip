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
  double* y = nullptr;
  double* part = nullptr;
  double* st = nullptr;
  ~ZScratch() {
    if (y) (void)hipFree(y);
    if (part) (void)hipFree(part);
    if (st) (void)hipFree(st);
  }
};

// st[0..2] for (x, y, alpha), copied to host h[0..2] (synchronises the stream)
hipError_t reduce3(const double* x, const double* y, int64_t n, double alpha, ZScratch& z, hipStream_t s,
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

int contract(Plan& p, const double* x, double* y, double* out) {
  ZScratch z;
  if (hipMalloc(&z.part, 3 * kZGrid * sizeof(double)) != hipSuccess ||
      hipMalloc(&z.st, 4 * sizeof(double)) != hipSuccess)
    return STTSV_ENOMEM;
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
  ZScratch z;
  z.part = sp;
  z.st = sp + 3 * kZGrid;
  double h[3];
  const hipError_t e = reduce3(x, y, p.n, 0.0, z, s, h);
  z.part = nullptr;                                       // not owned: keep ~ZScratch from freeing it
  z.st = nullptr;
  if (e != hipSuccess) return STTSV_EHIP;
  *out = h[0];
  return STTSV_OK;
}

int zeig_sshopm(Plan& p, const double* x0, double alpha, double tol, int32_t max_iter, double* x,
                sttsv_zeig_info* info) {
  const int64_t n = p.n;
  ZScratch z;
  if (hipMalloc(&z.y, n * sizeof(double)) != hipSuccess ||
      hipMalloc(&z.part, 3 * kZGrid * sizeof(double)) != hipSuccess ||
      hipMalloc(&z.st, 4 * sizeof(double)) != hipSuccess)
    return STTSV_ENOMEM;
  hipStream_t s = p.stream;
  double h[3];
  // x = x0 / ||x0||_2 (x0 = all ones when absent)
  const double* src = x0;
  if (src == nullptr) {
    hipLaunchKernelGGL(z_fill, dim3(vgrid(n)), dim3(kZBlock), 0, s, x, n, 1.0);
    src = x;
  }
  if (reduce3(src, src, n, 0.0, z, s, h) != hipSuccess) return STTSV_EHIP;
  if (!(h[2] > 0.0) || !std::isfinite(h[2])) return STTSV_ENUMERIC;
  hipLaunchKernelGGL(z_update, dim3(vgrid(n)), dim3(kZBlock), 0, s, x, src, n, 0.0, (const double*)z.st, 1);
  // lambda_0
  if (launch_sttsv(p, x, z.y, STTSV_PREC_FP64, nullptr, s) != hipSuccess) return STTSV_EHIP;
  if (reduce3(x, z.y, n, alpha, z, s, h) != hipSuccess) return STTSV_EHIP;
  double lam = h[0];
  int32_t it = 0;
  bool conv = false;
  while (it < max_iter) {
    if (!(h[1] > 0.0) || !std::isfinite(h[1])) return STTSV_ENUMERIC;
    hipLaunchKernelGGL(z_update, dim3(vgrid(n)), dim3(kZBlock), 0, s, x, (const double*)z.y, n, alpha,
                       (const double*)z.st, 0);
    if (launch_sttsv(p, x, z.y, STTSV_PREC_FP64, nullptr, s) != hipSuccess) return STTSV_EHIP;
    if (reduce3(x, z.y, n, alpha, z, s, h) != hipSuccess) return STTSV_EHIP;
    ++it;
    const bool done = tol > 0.0 && std::fabs(h[0] - lam) <= tol * std::fabs(h[0]);
    lam = h[0];
    if (done) {
      conv = true;
      break;
    }
  }
  // residual ||B x^(r-1) - lambda x||_2 at the returned x
  if (reduce3(x, z.y, n, -lam, z, s, h) != hipSuccess) return STTSV_EHIP;
  if (info) {
    info->iterations = it;
    info->converged = conv ? 1 : 0;
    info->lambda = lam;
    info->residual = std::sqrt(h[1]);
  }
  return conv ? STTSV_OK : STTSV_ENOTCONV;
}

}  // namespace sttsv
