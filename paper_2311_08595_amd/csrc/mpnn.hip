// Warm-start message-passing network: forward, loss, backward and Adam, all
// on the GPU.  Definition (H = 64; d_v degree, E(v) edges containing v):
//   features F (n x 4): log(1+d), mean log|e|, log(d)/(r-1), log(1+sum(|e|-1))
//   H0 = relu(F W0 + b0)
//   for l = 1, 2:  Ed = vertex->edge mean of H_{l-1};  A = edge->vertex mean of Ed
//                  H_l = relu([H_{l-1}, A] W_l + b_l)
//   s = H2 w_out + b_out   (score ~ log x),   x0 = exp(s - max s) / sum
//   loss L = mean(u^2), u = (s - mean s) - (log x* - mean log x*)
// Dense products run on BF16 MFMA (v_mfma_f32_16x16x16_bf16) with FP32
// accumulation: inputs ([H, A], the weights, and dZ for the input gradient)
// are rounded to bfloat16 (nearest even); everything else is FP32.  Every
// reduction has a fixed order (no atomics), so training is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace sttsv {
namespace mpnn {

constexpr int HD = 64;                     // hidden width
constexpr int KF = 16;                     // padded feature width (4 used)
constexpr int NF = 4;
// packed parameter vector: W0 (KF x HD, rows >= NF zero), b0, W1 (2HD x HD),
// b1, W2 (2HD x HD), b2, wout (HD), bout (1)
constexpr int OFF_W0 = 0;
constexpr int OFF_B0 = OFF_W0 + KF * HD;
constexpr int OFF_W1 = OFF_B0 + HD;
constexpr int OFF_B1 = OFF_W1 + 2 * HD * HD;
constexpr int OFF_W2 = OFF_B1 + HD;
constexpr int OFF_B2 = OFF_W2 + 2 * HD * HD;
constexpr int OFF_WO = OFF_B2 + HD;
constexpr int OFF_BO = OFF_WO + HD;
constexpr int NPARAM = OFF_BO + 1;
constexpr int kTile = 256;                 // vertices per partial of weight gradients

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);          // round to nearest even (finite inputs)
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// ------------------------------------------------------------------ graph
struct Graph {
  int32_t n = 0, r = 0;
  int64_t m = 0, nnz = 0;
  int32_t* eptr = nullptr;    // m+1 (edge -> members)
  int32_t* eidx = nullptr;
  int32_t* nptr = nullptr;    // n+1 (vertex -> edges)
  int32_t* nedge = nullptr;
  float* inv_size = nullptr;  // 1/|e|
  float* inv_deg = nullptr;   // 1/d_v
  uint16_t* X0 = nullptr;     // n x KF features (bf16)
  // vertex-side sums over E(v) in fixed-shape chunks (level 0 reads edges
  // through nedge, level l > 0 reads the partial rows of level l-1)
  static constexpr int kMaxLevels = 6;
  int nlev = 0;
  int32_t nchunk[kMaxLevels] = {};
  int32_t* cstart[kMaxLevels] = {};
  int32_t* clen[kMaxLevels] = {};
  int32_t* cdst[kMaxLevels] = {};   // >= 0 vertex (final); < 0: -(partial row)-1
  int32_t npart[kMaxLevels] = {};   // partial rows written by level l
};

struct Net {
  float* p = nullptr;         // FP32 master parameters (NPARAM)
  float* g = nullptr;         // gradients
  float* am = nullptr;        // Adam moments
  float* av = nullptr;
  uint16_t* wt[3] = {nullptr, nullptr, nullptr};   // W_l^T bf16 (HD x K)
  uint16_t* wr[3] = {nullptr, nullptr, nullptr};   // W_l   bf16 (K x HD)
  int64_t steps = 0;
  // workspace, grown to the largest graph seen
  int64_t cap_n = 0, cap_m = 0;
  float *Z[3] = {}, *Hh[3] = {};                    // n x HD
  uint16_t* X[3] = {};                              // X0 (graph), X1, X2: n x 2HD bf16
  uint16_t* dZb = nullptr;                          // n x HD bf16
  float *dZ = nullptr, *dH = nullptr, *dA = nullptr; // n x HD
  float *E = nullptr, *dE = nullptr;                // m x HD
  float *s = nullptr, *ds = nullptr;                // n
  float* part = nullptr;                            // partials
  int64_t part_cap = 0;
  float* vpart[2] = {nullptr, nullptr};             // vertex-sum partial rows (ping-pong)
  int64_t vpart_cap = 0;
  float* scal = nullptr;                            // small scalars
};

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return __shfl(v, 0, 64);
}

// features (one wave per vertex: lane l sums the vertex's edges l, l + 64,
// ..., then a fixed halving reduction across the wave)
__global__ void __launch_bounds__(256) feat_kernel(Graph g) {
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (v >= g.n) return;                         // uniform per wave
  const int a = g.nptr[v], b = g.nptr[v + 1];
  double slog = 0.0, sco = 0.0;
  for (int q = a + lane; q < b; q += 64) {
    const int e = g.nedge[q];
    const double k = double(g.eptr[e + 1] - g.eptr[e]);
    slog += log(k);
    sco += k - 1.0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    slog += __shfl_down(slog, o);
    sco += __shfl_down(sco, o);
  }
  if (lane != 0) return;
  const double d = double(b - a);
  float f[KF] = {};
  f[0] = float(log1p(d));
  f[1] = d > 0 ? float(slog / d) : 0.f;
  f[2] = d > 0 ? float(log(d) / double(g.r - 1)) : 0.f;
  f[3] = float(log1p(sco));
  for (int c = 0; c < KF; ++c) g.X0[(int64_t)v * KF + c] = to_bf16(f[c]);
  g.inv_deg[v] = d > 0 ? float(1.0 / d) : 0.f;
}

__global__ void inv_size_kernel(Graph g) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < g.m) g.inv_size[e] = 1.0f / float(g.eptr[e + 1] - g.eptr[e]);
}

// Z = X W + b (X: n x K bf16 row stride ldx, W^T: HD x K bf16), H = relu(Z);
// optionally H -> bf16 into the left half of the next layer's input.
// One wave per 16 rows.
template <int K>
__global__ void __launch_bounds__(256) dense_fwd(const uint16_t* __restrict__ X, int ldx,
                                                 const uint16_t* __restrict__ Wt, const float* __restrict__ b, int n,
                                                 float* __restrict__ Z, float* __restrict__ Hh,
                                                 uint16_t* __restrict__ Xnext) {
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (row0 >= n) return;                              // whole wave
  float4_t acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  const int ar = row0 + (lane & 15);
  const int kq = 4 * (lane >> 4);
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    short4_t a = {0, 0, 0, 0};
    if (ar < n) a = *reinterpret_cast<const short4_t*>(X + (int64_t)ar * ldx + k0 + kq);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const short4_t bb = *reinterpret_cast<const short4_t*>(Wt + (int64_t)(cb * 16 + (lane & 15)) * K + k0 + kq);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row0 + kq + j;
      const int col = cb * 16 + (lane & 15);
      if (row < n) {
        const float z = acc[cb][j] + b[col];
        const float h = fmaxf(z, 0.f);
        Z[(int64_t)row * HD + col] = z;
        Hh[(int64_t)row * HD + col] = h;
        if (Xnext != nullptr) Xnext[(int64_t)row * 2 * HD + col] = to_bf16(h);
      }
    }
}

// dX = dZ W^T (dZ: n x HD bf16, W: K x HD bf16) -> left half to dHprev,
// right half to dA (K = 2HD).  One wave per 16 rows.
__global__ void __launch_bounds__(256) dense_bwd_dx(const uint16_t* __restrict__ dZb,
                                                    const uint16_t* __restrict__ W, int n,
                                                    float* __restrict__ dHprev, float* __restrict__ dA) {
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (row0 >= n) return;
  const int ar = row0 + (lane & 15);
  const int kq = 4 * (lane >> 4);
  float4_t acc[8];
#pragma unroll
  for (int cb = 0; cb < 8; ++cb) acc[cb] = float4_t{0, 0, 0, 0};
#pragma unroll
  for (int j0 = 0; j0 < HD; j0 += 16) {
    short4_t a = {0, 0, 0, 0};
    if (ar < n) a = *reinterpret_cast<const short4_t*>(dZb + (int64_t)ar * HD + j0 + kq);
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const short4_t bb = *reinterpret_cast<const short4_t*>(W + (int64_t)(cb * 16 + (lane & 15)) * HD + j0 + kq);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 8; ++cb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row0 + kq + j;
      const int col = cb * 16 + (lane & 15);
      if (row < n) {
        if (col < HD)
          dHprev[(int64_t)row * HD + col] = acc[cb][j];
        else
          dA[(int64_t)row * HD + col - HD] = acc[cb][j];
      }
    }
}

// Ed_e = (1/|e|) sum_{v in e} H_v.  16 lanes per edge, 4 features per lane
// (one 16-byte load per lane and row: a wave gathers 4 rows at once).
__global__ void __launch_bounds__(256) edge_mean(Graph g, const float* __restrict__ Hh, float* __restrict__ E) {
  const int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
  const int c = 4 * (threadIdx.x & 15);
  if (e >= g.m) return;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int q = g.eptr[e]; q < g.eptr[e + 1]; ++q)
    acc += *reinterpret_cast<const float4_t*>(Hh + (int64_t)g.eidx[q] * HD + c);
  *reinterpret_cast<float4_t*>(E + e * HD + c) = acc * g.inv_size[e];
}

// Vertex-side sums over E(v), one wave per chunk of at most kVChunk terms,
// lane = feature.  MODE 0 (edge->vertex mean): terms Ed_e, final value
// bf16(sum / d_v) into the right half of X.  MODE 1 (adjoint of the
// vertex->edge mean): terms dE_e / |e|, final value added to dH_v.
constexpr int kVChunk = 128;

template <int MODE>
__global__ void __launch_bounds__(256) vsum_level(int nchunk, const int32_t* __restrict__ cstart,
                                                  const int32_t* __restrict__ clen, const int32_t* __restrict__ cdst,
                                                  const int32_t* __restrict__ nedge, const float* __restrict__ inv_size,
                                                  const float* __restrict__ inv_deg, const float* __restrict__ src,
                                                  const float* __restrict__ prev, float* __restrict__ part,
                                                  uint16_t* __restrict__ X, float* __restrict__ dH) {
  // 16 lanes per chunk, 4 features per lane
  const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
  const int f = 4 * (threadIdx.x & 15);
  if (c >= nchunk) return;
  const int32_t st = cstart[c], ln = clen[c], d = cdst[c];
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  if (prev == nullptr) {
    for (int q = 0; q < ln; ++q) {
      const int e = nedge[st + q];
      const float4_t t = *reinterpret_cast<const float4_t*>(src + (int64_t)e * HD + f);
      if (MODE == 0)
        acc += t;
      else
        acc += t * inv_size[e];
    }
  } else {
    for (int q = 0; q < ln; ++q) acc += *reinterpret_cast<const float4_t*>(prev + (int64_t)(st + q) * HD + f);
  }
  if (d < 0) {
    *reinterpret_cast<float4_t*>(part + (int64_t)(-(int64_t)d - 1) * HD + f) = acc;
  } else if (MODE == 0) {
    const float id = inv_deg[d];
    uint16_t* xo = X + (int64_t)d * 2 * HD + HD + f;
    for (int j = 0; j < 4; ++j) xo[j] = to_bf16(acc[j] * id);
  } else {
    float4_t* o = reinterpret_cast<float4_t*>(dH + (int64_t)d * HD + f);
    *o = *o + acc;
  }
}

// adjoint of node_mean: dE_e = sum_{v in e} dA_v / d_v (16 lanes per edge,
// 4 features per lane)
__global__ void __launch_bounds__(256) node_mean_T(Graph g, const float* __restrict__ dA, float* __restrict__ dE) {
  const int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
  const int c = 4 * (threadIdx.x & 15);
  if (e >= g.m) return;
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  for (int q = g.eptr[e]; q < g.eptr[e + 1]; ++q) {
    const int v = g.eidx[q];
    acc += *reinterpret_cast<const float4_t*>(dA + (int64_t)v * HD + c) * g.inv_deg[v];
  }
  *reinterpret_cast<float4_t*>(dE + e * HD + c) = acc;
}

// s_v = H2_v . wout + bout  (one wave per vertex)
__global__ void __launch_bounds__(256) score(const float* __restrict__ H2, const float* __restrict__ p, int n,
                                             float* __restrict__ s) {
  const int64_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  if (v >= n) return;
  const float t = wave_sum(H2[v * HD + c] * p[OFF_WO + c]);
  if (c == 0) s[v] = t + p[OFF_BO];
}

// block sums of a and b over [0, n): part[2*blk], part[2*blk+1]
__global__ void __launch_bounds__(256) sum2_stage(const float* a, const double* bsrc, int n, float* part,
                                                  bool log_b) {
  __shared__ float sh[2][256];
  float sa = 0.f, sb = 0.f;
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    sa += a[v];
    if (bsrc != nullptr) sb += log_b ? float(log(bsrc[v])) : float(bsrc[v]);
  }
  sh[0][threadIdx.x] = sa;
  sh[1][threadIdx.x] = sb;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void sum2_final(const float* part, int nb, float* out) {
  if (threadIdx.x != 0) return;
  float a = 0.f, b = 0.f;
  for (int q = 0; q < nb; ++q) {
    a += part[2 * q];
    b += part[2 * q + 1];
  }
  out[0] = a;
  out[1] = b;
}

// u_v = (s_v - smean) - (log x*_v - tmean);  ds_v = 2 u_v / n;  part: sum u^2 per block
__global__ void __launch_bounds__(256) loss_grad(const float* s, const double* xstar, int n, const float* means,
                                                 float* ds, float* part) {
  __shared__ float sh[256];
  const float sm = means[0] / float(n), tm = means[1] / float(n);
  float acc = 0.f;
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    const float u = (s[v] - sm) - (float(log(xstar[v])) - tm);
    ds[v] = 2.f * u / float(n);
    acc += u * u;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[2 * blockIdx.x] = sh[0];
}

// dH2 = ds (x) wout; dZ = dH2 * [Z2 > 0] handled by relu_bwd
__global__ void __launch_bounds__(256) score_bwd(const float* ds, const float* p, int n, float* dH) {
  const int64_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  if (v >= n) return;
  dH[v * HD + c] = ds[v] * p[OFF_WO + c];
}

// dZ = dH * [Z > 0] (fp32 and bf16)
__global__ void __launch_bounds__(256) relu_bwd(const float* dH, const float* Z, int64_t cnt, float* dZ,
                                                uint16_t* dZb) {
  const int64_t q = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (q >= cnt) return;
  const float d = Z[q] > 0.f ? dH[q] : 0.f;
  dZ[q] = d;
  dZb[q] = to_bf16(d);
}

// Weight-gradient partials of one tile of kTile vertices:
//   dW[k][j] = sum_v X[v][k] dZ[v][j] (K rows), db[j] = sum_v dZ[v][j],
//   and, for the output layer, dwout[j] = sum_v H2[v][j] ds[v], dbout = sum ds.
// part layout per tile: K*HD + HD floats.  Thread t owns columns j = t % HD
// and rows k = t / HD, t/HD + 4, ...
template <int K>
__global__ void __launch_bounds__(256) wgrad_tile(const uint16_t* __restrict__ X, int ldx,
                                                  const float* __restrict__ dZ, int n, float* __restrict__ part) {
  const int tile = blockIdx.x;
  const int j = threadIdx.x % HD;
  const int k0 = threadIdx.x / HD;
  const int v0 = tile * kTile, v1 = min(n, v0 + kTile);
  float* out = part + (int64_t)tile * (K * HD + HD);
  for (int k = k0; k < K; k += 4) {
    float acc = 0.f;
    for (int v = v0; v < v1; ++v) acc += from_bf16(X[(int64_t)v * ldx + k]) * dZ[(int64_t)v * HD + j];
    out[k * HD + j] = acc;
  }
  if (k0 == 0) {
    float acc = 0.f;
    for (int v = v0; v < v1; ++v) acc += dZ[(int64_t)v * HD + j];
    out[K * HD + j] = acc;
  }
}

__global__ void __launch_bounds__(256) outgrad_tile(const float* __restrict__ H2, const float* __restrict__ ds, int n,
                                                    float* __restrict__ part) {
  const int tile = blockIdx.x;
  const int j = threadIdx.x;
  const int v0 = tile * kTile, v1 = min(n, v0 + kTile);
  float* out = part + (int64_t)tile * (HD + 1);
  if (j < HD) {
    float acc = 0.f;
    for (int v = v0; v < v1; ++v) acc += H2[(int64_t)v * HD + j] * ds[v];
    out[j] = acc;
  } else if (j == HD) {
    float acc = 0.f;
    for (int v = v0; v < v1; ++v) acc += ds[v];
    out[HD] = acc;
  }
}

// g[off + q] = sum over tiles of part[tile*stride + q], q < len (tile order)
__global__ void __launch_bounds__(256) sum_tiles(const float* part, int tiles, int stride, int len, float* g) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= len) return;
  float acc = 0.f;
  for (int t = 0; t < tiles; ++t) acc += part[(int64_t)t * stride + q];
  g[q] = acc;
}

__global__ void __launch_bounds__(256) adam(float* p, const float* g, float* m, float* v, int cnt, float lr,
                                            float b1, float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= cnt) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// bf16 copies of W_l: W^T (HD x K) and W (K x HD)
__global__ void __launch_bounds__(256) weights_bf16(const float* W, int K, uint16_t* wt, uint16_t* wr) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= K * HD) return;
  const int k = q / HD, j = q % HD;
  const uint16_t h = to_bf16(W[q]);
  wr[q] = h;
  wt[j * K + k] = h;
}

// x0 = exp(s - max s) / sum: block maxima, then exponentials and block
// sums, then the division (fixed-shape reductions)
__global__ void __launch_bounds__(256) warm_max(const float* s, int n, double* part) {
  __shared__ double sh[256];
  double mx = -INFINITY;
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) mx = fmax(mx, double(s[v]));
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) warm_exp(const float* s, int n, const double* part, int nb, double* x0,
                                                double* psum) {
  __shared__ double sh[256];
  double mx = -INFINITY;
  for (int q = 0; q < nb; ++q) mx = fmax(mx, part[q]);
  double acc = 0.0;
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    const double e = exp(double(s[v]) - mx);
    x0[v] = e;
    acc += e;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) psum[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) warm_div(int n, const double* psum, int nb, double* x0) {
  double tot = 0.0;
  for (int q = 0; q < nb; ++q) tot += psum[q];
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) x0[v] = x0[v] / tot;
}

// ------------------------------------------------------------------ host side
int ok(hipError_t e) { return e == hipSuccess ? STTSV_OK : STTSV_EHIP; }

template <typename T>
bool dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) == hipSuccess;
}

int ensure_workspace(Net& N, const Graph& g) {
  if (g.n <= N.cap_n && g.m <= N.cap_m) return STTSV_OK;
  const int64_t n = std::max<int64_t>(g.n, N.cap_n), m = std::max<int64_t>(g.m, N.cap_m);
  for (int l = 0; l < 3; ++l) {
    (void)hipFree(N.Z[l]);
    (void)hipFree(N.Hh[l]);
  }
  for (int l = 1; l < 3; ++l) (void)hipFree(N.X[l]);
  for (void* q : {(void*)N.dZb, (void*)N.dZ, (void*)N.dH, (void*)N.dA, (void*)N.E, (void*)N.dE, (void*)N.s,
                  (void*)N.ds, (void*)N.part})
    (void)hipFree(q);
  bool good = true;
  for (int l = 0; l < 3; ++l) good = good && dalloc(&N.Z[l], n * HD) && dalloc(&N.Hh[l], n * HD);
  for (int l = 1; l < 3; ++l) good = good && dalloc(&N.X[l], n * 2 * HD);
  good = good && dalloc(&N.dZb, n * HD) && dalloc(&N.dZ, n * HD) && dalloc(&N.dH, n * HD) &&
         dalloc(&N.dA, n * HD) && dalloc(&N.E, m * HD) && dalloc(&N.dE, m * HD) && dalloc(&N.s, n) &&
         dalloc(&N.ds, n);
  const int64_t tiles = (n + kTile - 1) / kTile;
  N.part_cap = std::max<int64_t>(tiles * (2 * HD * HD + HD), 2 * 1024);
  good = good && dalloc(&N.part, N.part_cap);
  N.cap_n = n;
  N.cap_m = m;
  return good ? STTSV_OK : STTSV_ENOMEM;
}

int ensure_vpart(Net& N, const Graph& g) {
  int64_t need = 1;
  for (int l = 0; l < g.nlev; ++l) need = std::max<int64_t>(need, g.npart[l]);
  if (need <= N.vpart_cap) return STTSV_OK;
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(N.vpart[i]);
    if (!dalloc(&N.vpart[i], (size_t)need * HD)) return STTSV_ENOMEM;
  }
  N.vpart_cap = need;
  return STTSV_OK;
}

template <int MODE>
void vertex_sums(Net& N, const Graph& g, const float* src, uint16_t* X, float* dH, hipStream_t s) {
  for (int l = 0; l < g.nlev; ++l) {
    const float* prev = l == 0 ? nullptr : N.vpart[(l - 1) & 1];
    float* part = N.vpart[l & 1];
    hipLaunchKernelGGL((vsum_level<MODE>), dim3((g.nchunk[l] + 15) / 16), dim3(256), 0, s, g.nchunk[l],
                       (const int32_t*)g.cstart[l], (const int32_t*)g.clen[l], (const int32_t*)g.cdst[l],
                       (const int32_t*)g.nedge, (const float*)g.inv_size, (const float*)g.inv_deg, src, prev, part, X,
                       dH);
  }
}

int refresh_bf16(Net& N, hipStream_t s) {
  const int K[3] = {KF, 2 * HD, 2 * HD};
  const int off[3] = {OFF_W0, OFF_W1, OFF_W2};
  for (int l = 0; l < 3; ++l)
    hipLaunchKernelGGL(weights_bf16, dim3((K[l] * HD + 255) / 256), dim3(256), 0, s, N.p + off[l], K[l], N.wt[l],
                       N.wr[l]);
  return ok(hipGetLastError());
}

int forward(Net& N, const Graph& g, hipStream_t s) {
  int rc = ensure_workspace(N, g);
  if (rc == STTSV_OK) rc = ensure_vpart(N, g);
  if (rc != STTSV_OK) return rc;
  const dim3 gd((g.n + 63) / 64), ge((g.m + 15) / 16), gv((g.n + 3) / 4);
  hipLaunchKernelGGL((dense_fwd<KF>), gd, dim3(256), 0, s, g.X0, KF, N.wt[0], N.p + OFF_B0, g.n, N.Z[0], N.Hh[0],
                     N.X[1]);
  for (int l = 1; l <= 2; ++l) {
    hipLaunchKernelGGL(edge_mean, ge, dim3(256), 0, s, g, (const float*)N.Hh[l - 1], N.E);
    vertex_sums<0>(N, g, (const float*)N.E, N.X[l], nullptr, s);
    hipLaunchKernelGGL((dense_fwd<2 * HD>), gd, dim3(256), 0, s, N.X[l], 2 * HD, N.wt[l],
                       N.p + (l == 1 ? OFF_B1 : OFF_B2), g.n, N.Z[l], N.Hh[l], l == 1 ? N.X[2] : nullptr);
  }
  hipLaunchKernelGGL(score, gv, dim3(256), 0, s, (const float*)N.Hh[2], (const float*)N.p, g.n, N.s);
  return ok(hipGetLastError());
}

int loss_and_grad(Net& N, const Graph& g, const double* xstar, float* loss_host, hipStream_t s) {
  int rc = forward(N, g, s);
  if (rc != STTSV_OK) return rc;
  const int nb = std::max(1, std::min(1024, (g.n + 255) / 256));
  hipLaunchKernelGGL(sum2_stage, dim3(nb), dim3(256), 0, s, (const float*)N.s, xstar, g.n, N.part, true);
  hipLaunchKernelGGL(sum2_final, dim3(1), dim3(64), 0, s, (const float*)N.part, nb, N.scal);
  hipLaunchKernelGGL(loss_grad, dim3(nb), dim3(256), 0, s, (const float*)N.s, xstar, g.n, (const float*)N.scal,
                     N.ds, N.part);
  hipLaunchKernelGGL(sum2_final, dim3(1), dim3(64), 0, s, (const float*)N.part, nb, N.scal + 2);
  // output layer
  const int tiles = (g.n + kTile - 1) / kTile;
  hipLaunchKernelGGL(outgrad_tile, dim3(tiles), dim3(256), 0, s, (const float*)N.Hh[2], (const float*)N.ds, g.n,
                     N.part);
  hipLaunchKernelGGL(sum_tiles, dim3(1), dim3(256), 0, s, (const float*)N.part, tiles, HD + 1, HD + 1, N.g + OFF_WO);
  const dim3 gd((g.n + 63) / 64), ge((g.m + 15) / 16), gv((g.n + 3) / 4);
  const int64_t cnt = (int64_t)g.n * HD;
  const dim3 gc((unsigned)((cnt + 255) / 256));
  hipLaunchKernelGGL(score_bwd, gv, dim3(256), 0, s, (const float*)N.ds, (const float*)N.p, g.n, N.dH);
  for (int l = 2; l >= 1; --l) {
    hipLaunchKernelGGL(relu_bwd, gc, dim3(256), 0, s, (const float*)N.dH, (const float*)N.Z[l], cnt, N.dZ, N.dZb);
    hipLaunchKernelGGL((wgrad_tile<2 * HD>), dim3(tiles), dim3(256), 0, s, (const uint16_t*)N.X[l], 2 * HD,
                       (const float*)N.dZ, g.n, N.part);
    const int off = l == 2 ? OFF_W2 : OFF_W1;
    hipLaunchKernelGGL(sum_tiles, dim3((2 * HD * HD + HD + 255) / 256), dim3(256), 0, s, (const float*)N.part, tiles,
                       2 * HD * HD + HD, 2 * HD * HD + HD, N.g + off);
    hipLaunchKernelGGL(dense_bwd_dx, gd, dim3(256), 0, s, (const uint16_t*)N.dZb, (const uint16_t*)N.wr[l], g.n,
                       N.dH, N.dA);
    hipLaunchKernelGGL(node_mean_T, ge, dim3(256), 0, s, g, (const float*)N.dA, N.dE);
    vertex_sums<1>(N, g, (const float*)N.dE, nullptr, N.dH, s);
  }
  hipLaunchKernelGGL(relu_bwd, gc, dim3(256), 0, s, (const float*)N.dH, (const float*)N.Z[0], cnt, N.dZ, N.dZb);
  hipLaunchKernelGGL((wgrad_tile<KF>), dim3(tiles), dim3(256), 0, s, (const uint16_t*)g.X0, KF, (const float*)N.dZ,
                     g.n, N.part);
  hipLaunchKernelGGL(sum_tiles, dim3((KF * HD + HD + 255) / 256), dim3(256), 0, s, (const float*)N.part, tiles,
                     KF * HD + HD, KF * HD + HD, N.g + OFF_W0);
  if ((rc = ok(hipGetLastError())) != STTSV_OK) return rc;
  if (loss_host != nullptr) {
    float sc[4];
    if (hipMemcpyAsync(sc, N.scal, sizeof(sc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return STTSV_EHIP;
    *loss_host = sc[2] / float(g.n);
  }
  return STTSV_OK;
}

}  // namespace mpnn
}  // namespace sttsv

using sttsv::mpnn::Graph;
using sttsv::mpnn::Net;

struct sttsv_mpnn_graph_s {
  Graph g;
};
struct sttsv_mpnn_s {
  Net n;
};

extern "C" {

int sttsv_mpnn_graph(const int64_t* eptr, const int32_t* eidx, int64_t m, int32_t n, int32_t r,
                     sttsv_mpnn_graph_t* out) {
  using namespace sttsv::mpnn;
  if (eptr == nullptr || eidx == nullptr || out == nullptr || m < 1 || n < 1 || r < 2) return STTSV_EINVAL;
  const int64_t nnz = eptr[m];
  if (nnz > INT32_MAX || m > INT32_MAX) return STTSV_ENOTSUP;
  std::vector<int32_t> ep(m + 1), np(n + 1, 0), ne(nnz);
  for (int64_t e = 0; e <= m; ++e) ep[e] = static_cast<int32_t>(eptr[e]);
  for (int64_t q = 0; q < nnz; ++q) {
    if (eidx[q] < 0 || eidx[q] >= n) return STTSV_EINVAL;
    np[eidx[q] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) np[v + 1] += np[v];
  {
    std::vector<int32_t> cur(np.begin(), np.end() - 1);
    for (int64_t e = 0; e < m; ++e)
      for (int64_t q = eptr[e]; q < eptr[e + 1]; ++q) ne[cur[eidx[q]]++] = static_cast<int32_t>(e);
  }
  auto* G = new sttsv_mpnn_graph_s();
  Graph& g = G->g;
  g.n = n;
  g.m = m;
  g.r = r;
  g.nnz = nnz;
  bool good = dalloc(&g.eptr, m + 1) && dalloc(&g.eidx, nnz) && dalloc(&g.nptr, (size_t)n + 1) &&
              dalloc(&g.nedge, nnz) && dalloc(&g.inv_size, m) && dalloc(&g.inv_deg, n) &&
              dalloc(&g.X0, (size_t)n * KF);
  good = good && hipMemcpy(g.eptr, ep.data(), 4 * (m + 1), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g.eidx, eidx, 4 * nnz, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g.nptr, np.data(), 4 * ((size_t)n + 1), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g.nedge, ne.data(), 4 * nnz, hipMemcpyHostToDevice) == hipSuccess;
  // chunk levels of the vertex-side sums: a vertex's edges in chunks of
  // kVChunk; if it has several, their partial rows are summed the same way
  if (good) {
    std::vector<int64_t> seg_start(n), seg_len(n);
    std::vector<int32_t> seg_node(n);
    for (int32_t v = 0; v < n; ++v) {
      seg_start[v] = np[v];
      seg_len[v] = np[v + 1] - np[v];
      seg_node[v] = v;
    }
    while (!seg_node.empty() && good) {
      if (g.nlev == Graph::kMaxLevels) {
        good = false;
        break;
      }
      std::vector<int32_t> st, ln, ds;
      std::vector<int64_t> nst, nln;
      std::vector<int32_t> nnd;
      int64_t next = 0;
      for (size_t q = 0; q < seg_node.size(); ++q) {
        const int64_t d = seg_len[q];
        const int64_t nch = d <= kVChunk ? 1 : (d + kVChunk - 1) / kVChunk;
        if (nch == 1) {
          st.push_back(static_cast<int32_t>(seg_start[q]));
          ln.push_back(static_cast<int32_t>(d));
          ds.push_back(seg_node[q]);
        } else {
          for (int64_t c = 0; c < nch; ++c) {
            st.push_back(static_cast<int32_t>(seg_start[q] + c * kVChunk));
            ln.push_back(static_cast<int32_t>(std::min<int64_t>(kVChunk, d - c * kVChunk)));
            ds.push_back(static_cast<int32_t>(-(next + c) - 1));
          }
          nst.push_back(next);
          nln.push_back(nch);
          nnd.push_back(seg_node[q]);
          next += nch;
        }
      }
      const int l = g.nlev++;
      g.nchunk[l] = static_cast<int32_t>(st.size());
      g.npart[l] = static_cast<int32_t>(next);
      good = dalloc(&g.cstart[l], st.size()) && dalloc(&g.clen[l], st.size()) && dalloc(&g.cdst[l], st.size()) &&
             hipMemcpy(g.cstart[l], st.data(), 4 * st.size(), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(g.clen[l], ln.data(), 4 * ln.size(), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(g.cdst[l], ds.data(), 4 * ds.size(), hipMemcpyHostToDevice) == hipSuccess;
      seg_start = std::move(nst);
      seg_len = std::move(nln);
      seg_node = std::move(nnd);
    }
  }
  if (good) {
    hipLaunchKernelGGL(feat_kernel, dim3((n + 3) / 4), dim3(256), 0, 0, g);
    hipLaunchKernelGGL(inv_size_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, 0, g);
    good = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  }
  if (!good) {
    sttsv_mpnn_graph_destroy(G);
    return STTSV_ENOMEM;
  }
  *out = G;
  return STTSV_OK;
}

int sttsv_mpnn_graph_destroy(sttsv_mpnn_graph_t G) {
  if (G == nullptr) return STTSV_OK;
  Graph& g = G->g;
  for (void* q : {(void*)g.eptr, (void*)g.eidx, (void*)g.nptr, (void*)g.nedge, (void*)g.inv_size, (void*)g.inv_deg,
                  (void*)g.X0})
    (void)hipFree(q);
  for (int l = 0; l < g.nlev; ++l) {
    (void)hipFree(g.cstart[l]);
    (void)hipFree(g.clen[l]);
    (void)hipFree(g.cdst[l]);
  }
  delete G;
  return STTSV_OK;
}

int sttsv_mpnn_create(const float* params, sttsv_mpnn_t* out) {
  using namespace sttsv::mpnn;
  if (params == nullptr || out == nullptr) return STTSV_EINVAL;
  auto* M = new sttsv_mpnn_s();
  Net& N = M->n;
  const int K[3] = {KF, 2 * HD, 2 * HD};
  bool good = dalloc(&N.p, NPARAM) && dalloc(&N.g, NPARAM) && dalloc(&N.am, NPARAM) && dalloc(&N.av, NPARAM) &&
              dalloc(&N.scal, 8);
  for (int l = 0; l < 3; ++l) good = good && dalloc(&N.wt[l], (size_t)K[l] * HD) && dalloc(&N.wr[l], (size_t)K[l] * HD);
  good = good && hipMemcpy(N.p, params, 4 * NPARAM, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(N.am, 0, 4 * NPARAM) == hipSuccess && hipMemset(N.av, 0, 4 * NPARAM) == hipSuccess &&
         hipMemset(N.g, 0, 4 * NPARAM) == hipSuccess;
  good = good && refresh_bf16(N, 0) == STTSV_OK && hipDeviceSynchronize() == hipSuccess;
  if (!good) {
    sttsv_mpnn_destroy(M);
    return STTSV_ENOMEM;
  }
  *out = M;
  return STTSV_OK;
}

int sttsv_mpnn_params(sttsv_mpnn_t M, float* params_out, float* grads_out) {
  using namespace sttsv::mpnn;
  if (M == nullptr) return STTSV_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return STTSV_EHIP;
  if (params_out && hipMemcpy(params_out, M->n.p, 4 * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return STTSV_EHIP;
  if (grads_out && hipMemcpy(grads_out, M->n.g, 4 * NPARAM, hipMemcpyDeviceToHost) != hipSuccess) return STTSV_EHIP;
  return STTSV_OK;
}

int sttsv_mpnn_forward(sttsv_mpnn_t M, sttsv_mpnn_graph_t G, float* scores) {
  if (M == nullptr || G == nullptr) return STTSV_EINVAL;
  int rc = sttsv::mpnn::forward(M->n, G->g, 0);
  if (rc != STTSV_OK) return rc;
  if (scores != nullptr &&
      hipMemcpyAsync(scores, M->n.s, 4 * (size_t)G->g.n, hipMemcpyDeviceToDevice, 0) != hipSuccess)
    return STTSV_EHIP;
  return sttsv::mpnn::ok(hipGetLastError());
}

int sttsv_mpnn_loss_grad(sttsv_mpnn_t M, sttsv_mpnn_graph_t G, const double* xstar, float* loss) {
  if (M == nullptr || G == nullptr || xstar == nullptr) return STTSV_EINVAL;
  return sttsv::mpnn::loss_and_grad(M->n, G->g, xstar, loss, 0);
}

int sttsv_mpnn_adam(sttsv_mpnn_t M, float lr, float beta1, float beta2, float eps) {
  using namespace sttsv::mpnn;
  if (M == nullptr || !(lr > 0.f)) return STTSV_EINVAL;
  Net& N = M->n;
  N.steps += 1;
  const float c1 = 1.f - std::pow(beta1, (float)N.steps), c2 = 1.f - std::pow(beta2, (float)N.steps);
  hipLaunchKernelGGL(adam, dim3((NPARAM + 255) / 256), dim3(256), 0, 0, N.p, (const float*)N.g, N.am, N.av, NPARAM,
                     lr, beta1, beta2, eps, c1, c2);
  const int rc = refresh_bf16(N, 0);
  return rc != STTSV_OK ? rc : ok(hipGetLastError());
}

int sttsv_mpnn_warm_start(sttsv_mpnn_t M, sttsv_mpnn_graph_t G, double* x0) {
  if (M == nullptr || G == nullptr || x0 == nullptr) return STTSV_EINVAL;
  int rc = sttsv::mpnn::forward(M->n, G->g, 0);
  if (rc != STTSV_OK) return rc;
  using namespace sttsv::mpnn;
  const int nb = std::max(1, std::min(512, (G->g.n + 255) / 256));
  double* buf = reinterpret_cast<double*>(M->n.part);          // >= 2048 floats = 1024 doubles
  hipLaunchKernelGGL(warm_max, dim3(nb), dim3(256), 0, 0, (const float*)M->n.s, G->g.n, buf);
  hipLaunchKernelGGL(warm_exp, dim3(nb), dim3(256), 0, 0, (const float*)M->n.s, G->g.n, (const double*)buf, nb, x0,
                     buf + 512);
  hipLaunchKernelGGL(warm_div, dim3(nb), dim3(256), 0, 0, G->g.n, (const double*)(buf + 512), nb, x0);
  return sttsv::mpnn::ok(hipGetLastError());
}

int sttsv_mpnn_query(sttsv_mpnn_t M, sttsv_mpnn_graph_t G, int32_t what, float* out, int64_t count) {
  using namespace sttsv::mpnn;
  if (M == nullptr || G == nullptr || out == nullptr) return STTSV_EINVAL;
  const Net& N = M->n;
  const Graph& g = G->g;
  if (N.cap_n < g.n || N.cap_m < g.m) return STTSV_EINVAL;      // nothing computed for a graph this size
  const float* f = nullptr;
  const uint16_t* h = nullptr;
  int64_t len = 0;
  switch (what) {
    case STTSV_MQ_Z0: case STTSV_MQ_Z1: case STTSV_MQ_Z2:
      f = N.Z[what - STTSV_MQ_Z0]; len = (int64_t)g.n * HD; break;
    case STTSV_MQ_X1: case STTSV_MQ_X2:
      h = N.X[what - STTSV_MQ_X1 + 1]; len = (int64_t)g.n * 2 * HD; break;
    case STTSV_MQ_X0: h = g.X0; len = (int64_t)g.n * KF; break;
    case STTSV_MQ_S: f = N.s; len = g.n; break;
    case STTSV_MQ_DS: f = N.ds; len = g.n; break;
    case STTSV_MQ_DZ: f = N.dZ; len = (int64_t)g.n * HD; break;
    case STTSV_MQ_DA: f = N.dA; len = (int64_t)g.n * HD; break;
    case STTSV_MQ_DE: f = N.dE; len = g.m * HD; break;
    case STTSV_MQ_DH: f = N.dH; len = (int64_t)g.n * HD; break;
    default: return STTSV_EINVAL;
  }
  if (count != len) return STTSV_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return STTSV_EHIP;
  if (f != nullptr) return hipMemcpy(out, f, 4 * (size_t)len, hipMemcpyDeviceToHost) == hipSuccess ? STTSV_OK : STTSV_EHIP;
  std::vector<uint16_t> tmp(len);
  if (hipMemcpy(tmp.data(), h, 2 * (size_t)len, hipMemcpyDeviceToHost) != hipSuccess) return STTSV_EHIP;
  for (int64_t q = 0; q < len; ++q) {
    const uint32_t u = static_cast<uint32_t>(tmp[q]) << 16;
    std::memcpy(out + q, &u, 4);
  }
  return STTSV_OK;
}

int sttsv_mpnn_destroy(sttsv_mpnn_t M) {
  if (M == nullptr) return STTSV_OK;
  Net& N = M->n;
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)N.p, (void*)N.g, (void*)N.am, (void*)N.av, (void*)N.scal, (void*)N.dZb, (void*)N.dZ,
                  (void*)N.dH, (void*)N.dA, (void*)N.E, (void*)N.dE, (void*)N.s, (void*)N.ds, (void*)N.part})
    (void)hipFree(q);
  for (int l = 0; l < 3; ++l) {
    (void)hipFree(N.wt[l]);
    (void)hipFree(N.wr[l]);
    (void)hipFree(N.Z[l]);
    (void)hipFree(N.Hh[l]);
  }
  (void)hipFree(N.X[1]);
  (void)hipFree(N.X[2]);
  (void)hipFree(N.vpart[0]);
  (void)hipFree(N.vpart[1]);
  delete M;
  return STTSV_OK;
}

}  // extern "C"
