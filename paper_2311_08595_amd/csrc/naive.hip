// The paper's NAIVE baseline (Alg. 3) on the GPU: every (edge, member) pair
// forms its own generating-function product, in FP64, with nothing shared
// between the members of an edge or between edges.  It exists to measure what
// the memoised kernels save, not as a production path.
//
// For edge e (k = |e|) and member v (Alg. 2 / Eq. (2), w(e) = |e|, Sec. II):
//
//   c_v = w/|beta| (r-1)! [t^(r-1)] e^{x_v t} prod_{u in e, u != v} (e^{x_u t} - 1)
//
// computed in the ordinary power basis with full-length series (degrees
// 0..r-1): start from e^{x_v t}, then k-1 truncated products, one per other
// member.  That is k(k-1) truncated products per edge (Sec. IV's count for
// Alg. 3), against 2(k-3) windowed ones in the memoised kernels.  The x values
// of the edge are scaled by a power of two so the largest is in [0.5, 1); the
// term is homogeneous of degree r-1 (Eq. (2)), so the scale comes back out as
// an exact ldexp.  All terms are non-negative for x >= 0.
#include "internal.hpp"

namespace sttsv {
namespace {

// One thread per member slot of a size bucket: slot t is member j = t / m of
// edge i = t % m, so consecutive threads read consecutive SoA entries.
// RC: series capacity (a multiple of 8, >= r); degrees >= r are never formed.
template <int RC>
__global__ void __launch_bounds__(64) edge_naive(EdgeCall c, BucketDesc b) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= b.m * b.k) return;
  const int64_t i = t % b.m;
  const int j = static_cast<int>(t / b.m);
  const int r = b.r, k = b.k;

  double mx = 0.0;
  for (int u = 0; u < k; ++u) mx = fmax(mx, fabs(c.x[b.mem[(int64_t)u * b.m + i]]));
  int e2 = 0;
  (void)frexp(mx, &e2);                                 // mx = f 2^e2, f in [0.5, 1)
  const double coef = ldexp(b.wgt != nullptr ? b.wgt[i] : b.wk, (r - 1) * e2);   // w/|beta| (r-1)! 2^((r-1) e2)

  // s <- e^{z_v t}: s[n] = z_v^n / n!
  double s[RC], p[RC];
  const double zv = ldexp(c.x[b.mem[(int64_t)j * b.m + i]], -e2);
  s[0] = 1.0;
#pragma unroll
  for (int n = 1; n < RC; ++n)
    if (n < r) s[n] = s[n - 1] * (zv * (1.0 / double(n)));

  for (int u = 0; u < k; ++u) {
    if (u == j) continue;
    // p <- e^{z_u t} - 1: p[0] = 0, p[a] = z_u^a / a!
    const double zu = ldexp(c.x[b.mem[(int64_t)u * b.m + i]], -e2);
    p[0] = 0.0;
    if (r > 1) p[1] = zu;
#pragma unroll
    for (int a = 2; a < RC; ++a)
      if (a < r) p[a] = p[a - 1] * (zu * (1.0 / double(a)));
    // s <- s * p truncated to degrees 0..r-1, in place from the top degree down
#pragma unroll
    for (int n = RC - 1; n >= 0; --n) {
      if (n < r) {
        double acc = 0.0;
#pragma unroll
        for (int a = 1; a <= n; ++a) acc = fma(s[n - a], p[a], acc);
        s[n] = acc;
      }
    }
  }
  double top = 0.0;
#pragma unroll
  for (int n = 0; n < RC; ++n)
    if (n == r - 1) top = s[n];
  c.contrib[b.loc[(int64_t)j * b.m + i]] = coef * top;
}

// x into the plan's degree-rank order, which the member slots index.
__global__ void __launch_bounds__(256) naive_permute(const double* __restrict__ x, const int32_t* __restrict__ rid,
                                                     int64_t n, double* __restrict__ xr) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) xr[q] = x[rid[q]];
}

template <int RC>
hipError_t launch_naive_rc(const EdgeCall& c, const BucketDesc& b, hipStream_t s) {
  const int64_t slots = b.m * b.k;
  const dim3 grid(static_cast<unsigned>((slots + 63) / 64));
  hipLaunchKernelGGL((edge_naive<RC>), grid, dim3(64), 0, s, c, b);
  return hipGetLastError();
}

hipError_t launch_naive_bucket(const EdgeCall& c, const BucketDesc& b, hipStream_t s) {
  if (b.m == 0) return hipSuccess;
  switch ((b.r + 7) / 8) {
    case 1: return launch_naive_rc<8>(c, b, s);
    case 2: return launch_naive_rc<16>(c, b, s);
    case 3: return launch_naive_rc<24>(c, b, s);
    case 4: return launch_naive_rc<32>(c, b, s);
    case 5: return launch_naive_rc<40>(c, b, s);
    case 6: return launch_naive_rc<48>(c, b, s);
    case 7: return launch_naive_rc<56>(c, b, s);
    case 8: return launch_naive_rc<64>(c, b, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// y = B x^(r-1) by Alg. 3: permute, one naive launch per bucket, then the
// plan's deterministic reduction (the same one the memoised path uses).
hipError_t launch_sttsv_naive(Plan& p, const double* x, double* y, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (p.n > 0) {
    hipLaunchKernelGGL(naive_permute, dim3(static_cast<unsigned>((p.n + 255) / 256)), dim3(256), 0, s, x,
                       (const int32_t*)p.d_rid, (int64_t)p.n, p.d_xr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const EdgeCall c{p.d_xr, p.d_contrib, nullptr, nullptr};
  p.contrib_compact = false;                     // FP64 contributions
  for (const Bucket& B : p.buckets)
    if ((e = launch_naive_bucket(c, B.desc[0], s)) != hipSuccess) return e;
  return launch_reduction(p, y, nullptr, s);
}

}  // namespace sttsv
