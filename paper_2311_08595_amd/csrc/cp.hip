// Symmetric CP decomposition of the blowup tensor (Sec. I names it among the
// algorithms whose bottleneck is STTSV): B ~ sum_l lambda_l a_l^(o r).
//   f(lambda, A) = ||B||^2 - 2 sum_l lambda_l c_l + sum_{l,m} lambda_l lambda_m G_lm^r
//   c_l = B a_l^r = a_l . y_l,  y_l = B a_l^(r-1) (one STTSV per column),
//   G = A^T A,
//   df/dlambda_l = -2 c_l + 2 sum_m G_lm^r lambda_m
//   df/da_l      = 2 r lambda_l (-y_l + sum_m lambda_m G_lm^(r-1) a_m)
// ||B||^2 = sum over distinct vertex sets of W_S^2 / |beta(S)| comes from the
// planner.  Every sum has a fixed shape (no atomics), so results are bitwise
// reproducible.  The optimiser is gradient descent with Armijo backtracking:
// halve the trial step t until f(x - t g) <= f(x) - 1e-4 t ||g||^2 (at most 40
// times), accept, double t for the next iteration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sttsv {
namespace {

constexpr int kCpBlock = 256;
constexpr int kCpGrid = 256;            // fixed: the reduction tree does not depend on the device
constexpr int kCpMaxR = STTSV_CP_MAX_R;

// Block partial of one inner product u . v over a grid-stride range (fixed
// order), then a fixed tree in LDS: part[pair * kCpGrid + block].
__global__ void __launch_bounds__(kCpBlock) cp_dots(const double* __restrict__ U, const double* __restrict__ V,
                                                    const int2* __restrict__ pairs, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[kCpBlock];
  const int2 pr = pairs[blockIdx.y];
  const double* u = U + (int64_t)pr.x * n;
  const double* v = V + (int64_t)pr.y * n;
  double a = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kCpBlock + threadIdx.x; i < n; i += (int64_t)kCpGrid * kCpBlock)
    a = fma(u[i], v[i], a);
  sh[threadIdx.x] = a;
  for (int s = kCpBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * kCpGrid + blockIdx.x] = sh[0];
}

// One block per pair: its kCpGrid partials in a fixed tree.
__global__ void __launch_bounds__(kCpBlock) cp_dots_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kCpBlock];
  sh[threadIdx.x] = part[(int64_t)blockIdx.x * kCpGrid + threadIdx.x];
  for (int s = kCpBlock / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__device__ double ipow(double b, int e) {
  double r = 1.0;
  while (e > 0) {
    if (e & 1) r *= b;
    b *= b;
    e >>= 1;
  }
  return r;
}

// Scalars of the objective from the dot products: dots = [G (R x R, row-major), c (R)].
// Writes f (scal[0]), dlambda (R) and C_lm = lambda_m G_lm^(r-1) (R x R).
__global__ void cp_scalars(const double* __restrict__ dots, const double* __restrict__ lambda, int R, int r,
                           double norm2, double* __restrict__ scal, double* __restrict__ dlambda,
                           double* __restrict__ C) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double* G = dots;
  const double* c = dots + R * R;
  double quad = 0.0, lin = 0.0;
  for (int l = 0; l < R; ++l) {
    double row = 0.0;
    for (int m = 0; m < R; ++m) {
      const double g = G[l * R + m];
      row = fma(ipow(g, r), lambda[m], row);
      C[l * R + m] = lambda[m] * ipow(g, r - 1);
    }
    dlambda[l] = -2.0 * c[l] + 2.0 * row;
    quad = fma(lambda[l], row, quad);
    lin = fma(lambda[l], c[l], lin);
  }
  scal[0] = norm2 - 2.0 * lin + quad;
}

// dA[l n + v] = 2 r lambda_l (-Y[l n + v] + sum_m C_lm A[m n + v])
__global__ void __launch_bounds__(kCpBlock) cp_grad_a(const double* __restrict__ A, const double* __restrict__ Y,
                                                      const double* __restrict__ C, const double* __restrict__ lambda,
                                                      int64_t n, int R, int r, double* __restrict__ dA) {
  const int64_t t = blockIdx.x * (int64_t)kCpBlock + threadIdx.x;
  if (t >= n * R) return;
  const int l = static_cast<int>(t / n);
  const int64_t v = t % n;
  double s = 0.0;
  for (int m = 0; m < R; ++m) s = fma(C[l * R + m], A[(int64_t)m * n + v], s);
  dA[t] = 2.0 * r * lambda[l] * (s - Y[t]);
}

// x_t = x - t g over cnt entries
__global__ void __launch_bounds__(kCpBlock) cp_axpy(const double* __restrict__ x, const double* __restrict__ g,
                                                    double t, int64_t cnt, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)kCpBlock + threadIdx.x;
  if (i < cnt) out[i] = x[i] - __dmul_rn(t, g[i]);   // two roundings, as written
}

unsigned cp_grid(int64_t cnt) { return static_cast<unsigned>((cnt + kCpBlock - 1) / kCpBlock); }

struct CpWork {
  int64_t n = 0;
  int R = 0;
  double* Y = nullptr;       // n x R: B a_l^(r-1)
  double* part = nullptr;    // block partials of the dot products
  double* dots = nullptr;    // G (R x R), c (R), then one slot per extra dot
  double* C = nullptr;       // R x R
  double* scal = nullptr;    // f
  int2* pairs = nullptr;     // all (l, m) for G, then (l, l) against Y for c
  int2* pairs_self = nullptr;
  double* At = nullptr;      // trial A and lambda
  double* lt = nullptr;
  double* dAt = nullptr;
  double* dlt = nullptr;
  ~CpWork() {
    for (void* q : {(void*)Y, (void*)part, (void*)dots, (void*)C, (void*)scal, (void*)pairs, (void*)pairs_self,
                    (void*)At, (void*)lt, (void*)dAt, (void*)dlt})
      (void)hipFree(q);
  }
  bool init(int64_t n_, int R_, bool trial) {
    n = n_;
    R = R_;
    const int np = R * R;
    std::vector<int2> pr;
    for (int l = 0; l < R; ++l)
      for (int m = 0; m < R; ++m) pr.push_back(make_int2(l, m));
    std::vector<int2> ps;
    for (int l = 0; l < R; ++l) ps.push_back(make_int2(l, l));
    bool ok = hipMalloc(&Y, sizeof(double) * n * R) == hipSuccess &&
              hipMalloc(&part, sizeof(double) * kCpGrid * (np + R)) == hipSuccess &&
              hipMalloc(&dots, sizeof(double) * (np + R + 2)) == hipSuccess &&
              hipMalloc(&C, sizeof(double) * np) == hipSuccess && hipMalloc(&scal, sizeof(double) * 4) == hipSuccess &&
              hipMalloc(&pairs, sizeof(int2) * np) == hipSuccess && hipMalloc(&pairs_self, sizeof(int2) * R) == hipSuccess;
    if (ok && trial)
      ok = hipMalloc(&At, sizeof(double) * n * R) == hipSuccess && hipMalloc(&lt, sizeof(double) * R) == hipSuccess &&
           hipMalloc(&dAt, sizeof(double) * n * R) == hipSuccess && hipMalloc(&dlt, sizeof(double) * R) == hipSuccess;
    ok = ok && hipMemcpy(pairs, pr.data(), sizeof(int2) * np, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(pairs_self, ps.data(), sizeof(int2) * R, hipMemcpyHostToDevice) == hipSuccess;
    return ok;
  }
};

// Fixed-shape dot products of the columns of U and V listed in pairs (on device)
// into out[0..npairs).
hipError_t dots(const double* U, const double* V, const int2* pairs, int npairs, int64_t n, double* part, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(cp_dots, dim3(kCpGrid, npairs), dim3(kCpBlock), 0, s, U, V, pairs, n, part);
  hipLaunchKernelGGL(cp_dots_final, dim3(npairs), dim3(kCpBlock), 0, s, (const double*)part, out);
  return hipGetLastError();
}

// f (to host), dlambda and dA at (A, lambda); Y, G, c and C in the work space.
int objective_grad(Plan& p, CpWork& w, const double* A, const double* lambda, int r, double* f_host, double* dA,
                   double* dlambda) {
  hipStream_t s = p.stream;
  const int64_t n = w.n;
  const int R = w.R;
  for (int l = 0; l < R; ++l)
    if (launch_sttsv(p, A + (int64_t)l * n, w.Y + (int64_t)l * n, STTSV_PREC_FP64, nullptr, s) != hipSuccess)
      return STTSV_EHIP;
  if (dots(A, A, w.pairs, R * R, n, w.part, w.dots, s) != hipSuccess ||
      dots(A, w.Y, w.pairs_self, R, n, w.part + (int64_t)kCpGrid * R * R, w.dots + R * R, s) != hipSuccess)
    return STTSV_EHIP;
  hipLaunchKernelGGL(cp_scalars, dim3(1), dim3(64), 0, s, (const double*)w.dots, lambda, R, r, p.graphs[0].norm2, w.scal,
                     dlambda, w.C);
  hipLaunchKernelGGL(cp_grad_a, dim3(cp_grid(n * R)), dim3(kCpBlock), 0, s, A, (const double*)w.Y,
                     (const double*)w.C, lambda, n, R, r, dA);
  if (hipGetLastError() != hipSuccess) return STTSV_EHIP;
  if (hipMemcpyAsync(f_host, w.scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return STTSV_EHIP;
  return STTSV_OK;
}

// ||dlambda||^2 + ||dA||^2 (fixed shape), to host
int grad_norm2(Plan& p, CpWork& w, const double* dA, const double* dlambda, double* out) {
  hipStream_t s = p.stream;
  const int64_t n = w.n;
  const int R = w.R;
  double* slot = w.dots + R * R + R;
  // dA viewed as one column of n R entries, dlambda as one of R entries
  // (the first pair of w.pairs is (0, 0))
  if (dots(dA, dA, w.pairs, 1, n * R, w.part, slot, s) != hipSuccess ||
      dots(dlambda, dlambda, w.pairs, 1, R, w.part + kCpGrid, slot + 1, s) != hipSuccess)
    return STTSV_EHIP;
  double h[2];
  if (hipMemcpyAsync(h, slot, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return STTSV_EHIP;
  *out = h[0] + h[1];
  return STTSV_OK;
}

}  // namespace

int cp_objective_grad(Plan& p, int32_t R, const double* A, const double* lambda, double* f, double* dA,
                      double* dlambda) {
  if (R < 1 || R > kCpMaxR) return STTSV_EINVAL;
  if (p.graphs.size() != 1) return STTSV_ENOTSUP;
  CpWork w;
  if (!w.init(p.n, R, false)) return STTSV_ENOMEM;
  return objective_grad(p, w, A, lambda, p.r, f, dA, dlambda);
}

int cp_descent(Plan& p, int32_t R, double* A, double* lambda, int32_t iters, double step, sttsv_cp_info* info) {
  if (R < 1 || R > kCpMaxR || iters < 0 || !(step > 0.0)) return STTSV_EINVAL;
  if (p.graphs.size() != 1) return STTSV_ENOTSUP;
  CpWork w;
  if (!w.init(p.n, R, true)) return STTSV_ENOMEM;
  hipStream_t s = p.stream;
  const int64_t n = p.n;
  double* dA = nullptr;
  double* dl = nullptr;
  if (hipMalloc(&dA, sizeof(double) * n * R) != hipSuccess || hipMalloc(&dl, sizeof(double) * R) != hipSuccess) {
    (void)hipFree(dA);
    return STTSV_ENOMEM;
  }
  struct Free {
    double* a;
    double* b;
    ~Free() {
      (void)hipFree(a);
      (void)hipFree(b);
    }
  } guard{dA, dl};
  double f = 0.0;
  int rc = objective_grad(p, w, A, lambda, p.r, &f, dA, dl);
  if (rc != STTSV_OK) return rc;
  const double f0 = f;
  double t = step;
  int32_t it = 0, halv = 0;
  for (; it < iters; ++it) {
    double gg = 0.0;
    if ((rc = grad_norm2(p, w, dA, dl, &gg)) != STTSV_OK) return rc;
    double ft = 0.0;
    for (int h = 0;; ++h) {
      hipLaunchKernelGGL(cp_axpy, dim3(cp_grid(n * R)), dim3(kCpBlock), 0, s, (const double*)A, (const double*)dA, t,
                         n * R, w.At);
      hipLaunchKernelGGL(cp_axpy, dim3(cp_grid(R)), dim3(kCpBlock), 0, s, (const double*)lambda, (const double*)dl, t,
                         (int64_t)R, w.lt);
      if (hipGetLastError() != hipSuccess) return STTSV_EHIP;
      if ((rc = objective_grad(p, w, w.At, w.lt, p.r, &ft, w.dAt, w.dlt)) != STTSV_OK) return rc;
      if (ft <= f - 1e-4 * t * gg || h >= 40) {
        halv += h;
        break;
      }
      t *= 0.5;
    }
    if (hipMemcpyAsync(A, w.At, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(lambda, w.lt, sizeof(double) * R, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dA, w.dAt, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dl, w.dlt, sizeof(double) * R, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return STTSV_EHIP;
    f = ft;
    t *= 2.0;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return STTSV_EHIP;
  if (info != nullptr) {
    info->iterations = it;
    info->halvings = halv;
    info->f = f;
    info->f0 = f0;
    info->norm2 = p.graphs[0].norm2;
  }
  return STTSV_OK;
}

}  // namespace sttsv
