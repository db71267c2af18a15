// NQZ iteration (Alg. 1) on the GPU, for every hypergraph of a plan at once.
//
// Every step of an iteration is a kernel whose decisions live in device
// control blocks (one per graph plus one per solve), so K iterations can be
// captured once in a hipGraph and replayed; the host only reads the solve's
// "all done" flag between replays.
//
// Iteration t for graph g (x~ = its current iterate scaled to max 1):
//   z = TTSV1(x~)                            edge kernels + node reduction
//   z' = z + alpha x~^[r-1]                  optional shift (alpha = 0: Alg. 1)
//   lambda_v = z'_v / x~_v^(r-1)             min / max over g's vertices
//   crit = (lambda_max - lambda_min) / lambda_min;  g stops when crit < tol
//   w = z'^[1/(r-1)];  x~ <- w / max(w)      next iterate (Alg. 1 divides by
//                                            the l1 norm; TTSV1 and x^[r-1]
//                                            are both homogeneous of degree
//                                            r-1, so the ratio, the test and
//                                            the normalised x are unchanged)
// A finished graph is masked: its edges are skipped and its x is frozen.
// The returned x of each graph is the iterate whose TTSV1 met the test,
// divided by its l1 norm (fixed-shape, deterministic sum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sttsv {

struct GCtrl {            // per graph
  int32_t done, status;
  int32_t iter, it32, it64;
  int32_t r;
  double lmin, lmax, crit, prev_crit;
  double inv_wmax;
};

struct SCtrl {            // per solve
  int32_t all_done;
  int32_t max_iter;
  double tol, switch_tol, shift;
  int32_t no32;          // no open graph runs FP32 series again (a graph never switches back)
  int32_t pad;
};

struct Solver {
  int32_t n = 0, G = 0, nblk = 0;
  hipStream_t s = nullptr;
  double* x = nullptr;        // current iterates, max-normalised per graph
  float* x32 = nullptr;       // the same rounded to FP32 (compact FP32 series of the mixed schedule)
  double* z = nullptr;
  double* w = nullptr;
  double* part = nullptr;     // per-block partials (4 per block)
  double* sums = nullptr;     // per-graph l1 norms
  int32_t* bgraph = nullptr;  // graph of each vertex block
  int32_t* bsub = nullptr;    // block index inside its graph
  int32_t* gblk0 = nullptr;   // first block of each graph
  int32_t* gnblk = nullptr;   // blocks of each graph
  int32_t* voff = nullptr;    // first vertex of each graph
  int32_t* gn = nullptr;      // vertices of each graph
  int32_t* skip64 = nullptr;  // graph skips the FP64-series edge launches
  int32_t* skip32 = nullptr;  // graph skips the FP32-series edge launches
  // Batched plans: per edge stage (slot q = sequence * gate_stride + stage
  // index; sequence 0 = FP64 apply, 1 = FP32-series apply) the graphs whose
  // edges it may process, gate_graph[gate_ptr[q] .. gate_ptr[q + 1]), and
  // gate[q] = 1 when none of them runs that sequence in the next iteration:
  // the stage's kernels then leave at once instead of testing every edge.
  int32_t* gate = nullptr;
  int32_t* gate_ptr = nullptr;
  int32_t* gate_graph = nullptr;
  int32_t gate_stride = 0, ngate = 0;
  GCtrl* ctrl = nullptr;
  SCtrl* sctrl = nullptr;
  GCtrl* hctrl = nullptr;     // pinned host mirrors
  SCtrl* hsctrl = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphExec_t exec64 = nullptr;   // FP64-only iterations: the FP32->FP64 schedule once no32
  int graph_iters = 0;
  int graph_sched = -1;
  int graph64_iters = 0;
};

namespace {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 1024;   // blocks per graph at most: shapes depend on n_g only

int blocks_of(int n) { return std::max(1, std::min(kRedGrid, (n + kRedBlock - 1) / kRedBlock)); }

template <typename F>
__device__ __forceinline__ double block_reduce(double v, double* sh, F op) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRedBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
struct OpMin {
  __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct OpAdd {
  __device__ double operator()(double a, double b) const { return a + b; }
};

struct VBlock {         // vertex range of one block: v = v0 + tid + j*stride
  int32_t g, v0, vend, stride;
};

__device__ __forceinline__ VBlock vblock(const Solver& S) {
  VBlock b;
  b.g = S.bgraph[blockIdx.x];
  const int32_t sub = S.bsub[blockIdx.x];
  b.v0 = S.voff[b.g] + sub * kRedBlock + threadIdx.x;
  b.vend = S.voff[b.g] + S.gn[b.g];
  b.stride = S.gnblk[b.g] * kRedBlock;
  return b;
}

// Initial iterate: x~ = x0 / max(x0) per graph.  part[b] = {max, bad}
__global__ void __launch_bounds__(kRedBlock) init_stats(Solver S, const double* x0) {
  __shared__ double sh[kRedBlock];
  const VBlock vb = vblock(S);
  double hi = 0.0, bad = 0.0;
  for (int v = vb.v0; v < vb.vend; v += vb.stride) {
    const double a = x0[v];
    if (!(a > 0.0) || !isfinite(a)) bad = 1.0;
    hi = fmax(hi, a);
  }
  hi = block_reduce(hi, sh, OpMax());
  bad = block_reduce(bad, sh, OpMax());
  if (threadIdx.x == 0) {
    S.part[4 * blockIdx.x] = hi;
    S.part[4 * blockIdx.x + 1] = bad;
  }
}

__global__ void __launch_bounds__(kRedBlock) init_final(Solver S) {
  __shared__ double sh[kRedBlock];
  const int g = blockIdx.x;
  const int b0 = S.gblk0[g], nb = S.gnblk[g];
  double hi = 0.0, bad = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedBlock) {
    hi = fmax(hi, S.part[4 * (b0 + b)]);
    bad = fmax(bad, S.part[4 * (b0 + b) + 1]);
  }
  hi = block_reduce(hi, sh, OpMax());
  bad = block_reduce(bad, sh, OpMax());
  if (threadIdx.x == 0) {
    GCtrl& c = S.ctrl[g];
    if (bad > 0.0) {
      c.done = 1;
      c.status = STTSV_EINVAL;
      S.skip64[g] = S.skip32[g] = 1;
    }
    c.inv_wmax = 1.0 / hi;
  }
}

// dst = src / max per graph (and rounded to FP32 into dst32 when given)
__global__ void __launch_bounds__(kRedBlock) scale_into(Solver S, const double* src, double* dst, float* dst32) {
  const VBlock vb = vblock(S);
  const GCtrl& c = S.ctrl[vb.g];
  if (c.done) return;
  const double f = c.inv_wmax;
  for (int v = vb.v0; v < vb.vend; v += vb.stride) {
    const double t = src[v] * f;
    dst[v] = t;
    if (dst32 != nullptr) dst32[v] = static_cast<float>(t);
  }
}

// The solver keeps x, z, w in degree-rank order (position q holds vertex
// rid[q]; each graph's positions are its own vertex range), so its STTSV
// needs no reordering: these two kernels convert at entry and exit.
__global__ void __launch_bounds__(kRedBlock) scale_from_vertex_order(Solver S, const double* src,
                                                                     const int32_t* __restrict__ rid, double* dst) {
  const VBlock vb = vblock(S);
  const GCtrl& c = S.ctrl[vb.g];
  if (c.done) return;
  const double f = c.inv_wmax;
  for (int v = vb.v0; v < vb.vend; v += vb.stride) dst[v] = src[rid[v]] * f;
}

__global__ void __launch_bounds__(kRedBlock) divide_to_vertex_order(Solver S, const double* x,
                                                                    const int32_t* __restrict__ rid, double* out) {
  const VBlock vb = vblock(S);
  const double s = S.sums[vb.g];
  for (int v = vb.v0; v < vb.vend; v += vb.stride) out[rid[v]] = x[v] / s;
}

__global__ void __launch_bounds__(kRedBlock) fill_ones(double* dst, int n) {
  const int v = blockIdx.x * kRedBlock + threadIdx.x;
  if (v < n) dst[v] = 1.0;
}

// Per-vertex step after TTSV1: shifted z, ratio lambda, next w.
// part[b] = {min lambda, max lambda, max w, bad}
template <bool LAMBDA>
__global__ void __launch_bounds__(kRedBlock) nqz_stats(Solver S) {
  __shared__ double sh[kRedBlock];
  const VBlock vb = vblock(S);
  const GCtrl& c = S.ctrl[vb.g];
  if (c.done) return;                               // uniform per block
  const double shift = S.sctrl->shift;
  const int r = c.r;
  const double inv = 1.0 / double(r - 1);
  double lo = INFINITY, hi = -INFINITY, wm = 0.0, bad = 0.0;
  for (int v = vb.v0; v < vb.vend; v += vb.stride) {
    const double xv = S.x[v];
    const double p = pow(xv, double(r - 1));
    const double zz = shift != 0.0 ? fma(shift, p, S.z[v]) : S.z[v];
    if (!(zz > 0.0) || !isfinite(zz)) bad = 1.0;
    if (LAMBDA) {
      const double lam = zz / p;
      lo = fmin(lo, lam);
      hi = fmax(hi, lam);
    }
    const double wv = pow(zz, inv);
    S.w[v] = wv;
    wm = fmax(wm, wv);
  }
  lo = block_reduce(lo, sh, OpMin());
  hi = block_reduce(hi, sh, OpMax());
  wm = block_reduce(wm, sh, OpMax());
  bad = block_reduce(bad, sh, OpMax());
  if (threadIdx.x == 0) {
    S.part[4 * blockIdx.x] = lo;
    S.part[4 * blockIdx.x + 1] = hi;
    S.part[4 * blockIdx.x + 2] = wm;
    S.part[4 * blockIdx.x + 3] = bad;
  }
}

template <bool LAMBDA>
__global__ void __launch_bounds__(kRedBlock) nqz_final(Solver S) {
  __shared__ double sh[kRedBlock];
  const int g = blockIdx.x;
  GCtrl& c = S.ctrl[g];
  if (c.done) {
    if (threadIdx.x == 0 && S.G == 1) S.sctrl->all_done = 1;
    return;
  }
  const int b0 = S.gblk0[g], nb = S.gnblk[g];
  double lo = INFINITY, hi = -INFINITY, wm = 0.0, bad = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedBlock) {
    lo = fmin(lo, S.part[4 * (b0 + b)]);
    hi = fmax(hi, S.part[4 * (b0 + b) + 1]);
    wm = fmax(wm, S.part[4 * (b0 + b) + 2]);
    bad = fmax(bad, S.part[4 * (b0 + b) + 3]);
  }
  lo = block_reduce(lo, sh, OpMin());
  hi = block_reduce(hi, sh, OpMax());
  wm = block_reduce(wm, sh, OpMax());
  bad = block_reduce(bad, sh, OpMax());
  if (threadIdx.x != 0) return;
  if (bad > 0.0 || !(wm > 0.0) || !isfinite(wm)) {
    c.done = 1;
    c.status = STTSV_ENUMERIC;
    S.skip64[g] = S.skip32[g] = 1;
    if (S.G == 1) {                         // one graph: no separate all-done pass
      S.sctrl->all_done = 1;
      S.sctrl->no32 = 1;
    }
    return;
  }
  c.inv_wmax = 1.0 / wm;
  if (!LAMBDA) return;
  const bool ran64 = S.skip64[g] == 0;
  const double crit = (hi - lo) / lo;
  c.iter += 1;
  if (ran64)
    c.it64 += 1;
  else
    c.it32 += 1;
  c.lmin = lo;
  c.lmax = hi;
  c.crit = crit;
  if (ran64) {
    if (crit < S.sctrl->tol) {
      c.done = 1;
      c.status = STTSV_OK;
    }
  } else if (crit < S.sctrl->switch_tol || crit < S.sctrl->tol || crit > 0.8 * c.prev_crit) {
    S.skip64[g] = 0;   // FP32 series have done what they can: polish in FP64
    S.skip32[g] = 1;
  }
  c.prev_crit = crit;
  if (!c.done && c.iter >= S.sctrl->max_iter) {
    c.done = 1;
    c.status = STTSV_ENOTCONV;
  }
  if (c.done) S.skip64[g] = S.skip32[g] = 1;
  if (S.G == 1) {
    S.sctrl->all_done = c.done;
    S.sctrl->no32 = S.skip32[g];
  }
}

// Block 0: all_done = every graph done, no32 = no open graph runs FP32
// series.  Block 1 + q: the gate of edge stage slot q (a done graph skips
// both sequences, so all_done closes every gate).
__global__ void __launch_bounds__(kRedBlock) all_done_check(Solver S) {
  __shared__ double sh[kRedBlock];
  if (blockIdx.x > 0) {
    const int q = static_cast<int>(blockIdx.x) - 1;
    const int32_t* skip = q < S.gate_stride ? S.skip64 : S.skip32;
    double run = 0.0;
    for (int t = S.gate_ptr[q] + static_cast<int>(threadIdx.x); t < S.gate_ptr[q + 1]; t += kRedBlock)
      run = fmax(run, skip[S.gate_graph[t]] ? 0.0 : 1.0);
    run = block_reduce(run, sh, OpMax());
    if (threadIdx.x == 0) S.gate[q] = run > 0.0 ? 0 : 1;
    return;
  }
  double open = 0.0, open32 = 0.0;
  for (int g = threadIdx.x; g < S.G; g += kRedBlock) {
    open = fmax(open, S.ctrl[g].done ? 0.0 : 1.0);
    open32 = fmax(open32, S.skip32[g] ? 0.0 : 1.0);
  }
  open = block_reduce(open, sh, OpMax());
  open32 = block_reduce(open32, sh, OpMax());
  if (threadIdx.x == 0) {
    S.sctrl->all_done = open > 0.0 ? 0 : 1;
    S.sctrl->no32 = open32 > 0.0 ? 0 : 1;
  }
}

__global__ void __launch_bounds__(kRedBlock) sum_stage(Solver S, const double* x) {
  __shared__ double sh[kRedBlock];
  const VBlock vb = vblock(S);
  double acc = 0.0;
  for (int v = vb.v0; v < vb.vend; v += vb.stride) acc += x[v];
  acc = block_reduce(acc, sh, OpAdd());
  if (threadIdx.x == 0) S.part[4 * blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kRedBlock) sum_final(Solver S) {
  __shared__ double sh[kRedBlock];
  const int g = blockIdx.x;
  const int b0 = S.gblk0[g], nb = S.gnblk[g];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedBlock) acc += S.part[4 * (b0 + b)];
  acc = block_reduce(acc, sh, OpAdd());
  if (threadIdx.x == 0) S.sums[g] = acc;
}

// FP32-series iterations of the mixed schedule run compact (FP32 x,
// 32-bit contributions) when every FP32-list edge stage has FP32 series.
bool compact_mixed(const Plan& p, int schedule) { return schedule == STTSV_SOLVE_FP32_FP64 && p.compact_ok; }

// One NQZ iteration (all launches on S.s).
hipError_t enqueue_iteration(Plan& p, Solver& S, int schedule) {
  hipError_t e;
  const int32_t* all_done = &S.sctrl->all_done;
  const bool cmp = compact_mixed(p, schedule);
  const int32_t* gate64 = S.gate;                                          // null for one graph
  const int32_t* gate32 = S.gate != nullptr ? S.gate + S.gate_stride : nullptr;
  if (schedule == STTSV_SOLVE_FP32_FP64)
    e = launch_edges_both(p, S.x, all_done, S.skip32, S.skip64, S.s, cmp ? S.x32 : nullptr, gate32, gate64);
  else
    e = launch_edges(p, S.x, STTSV_PREC_FP64, all_done, S.skip64, S.s, XOrder::kRank, false, gate64);
  if (e != hipSuccess) return e;
  // a graph's level-0 workgroups read words while it runs FP32 series (skip32 == 0)
  e = cmp ? launch_reduction_phased(p, S.z, S.skip32, all_done, S.s, true)
          : launch_reduction(p, S.z, all_done, S.s, true);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((nqz_stats<true>), dim3(S.nblk), dim3(kRedBlock), 0, S.s, S);
  hipLaunchKernelGGL((nqz_final<true>), dim3(S.G), dim3(kRedBlock), 0, S.s, S);
  if (S.G > 1) hipLaunchKernelGGL(all_done_check, dim3(1 + S.ngate), dim3(kRedBlock), 0, S.s, S);
  hipLaunchKernelGGL(scale_into, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, (const double*)S.w, S.x,
                     cmp ? S.x32 : nullptr);
  return hipGetLastError();
}

int hip_rc(hipError_t e) { return e == hipSuccess ? STTSV_OK : STTSV_EHIP; }

}  // namespace

void free_solver(Plan& p) {
  Solver* S = p.solver;
  if (S == nullptr) return;
  if (S->exec) (void)hipGraphExecDestroy(S->exec);
  if (S->exec64) (void)hipGraphExecDestroy(S->exec64);
  for (void* q : {(void*)S->x, (void*)S->x32, (void*)S->z, (void*)S->w, (void*)S->part, (void*)S->sums, (void*)S->bgraph,
                  (void*)S->bsub, (void*)S->gblk0, (void*)S->gnblk, (void*)S->voff, (void*)S->gn,
                  (void*)S->skip64, (void*)S->skip32, (void*)S->ctrl, (void*)S->sctrl, (void*)S->gate,
                  (void*)S->gate_ptr, (void*)S->gate_graph})
    (void)hipFree(q);
  if (S->hctrl) (void)hipHostFree(S->hctrl);
  if (S->hsctrl) (void)hipHostFree(S->hsctrl);
  if (S->s) (void)hipStreamDestroy(S->s);
  delete S;
  p.solver = nullptr;
}

static int ensure_solver(Plan& p) {
  if (p.solver != nullptr) return STTSV_OK;
  Solver* S = new Solver();
  p.solver = S;
  const int G = static_cast<int>(p.graphs.size());
  S->n = p.n;
  S->G = G;
  std::vector<int32_t> bgraph, bsub, gblk0(G), gnblk(G), voff(G), gn(G);
  for (int g = 0; g < G; ++g) {
    gblk0[g] = static_cast<int32_t>(bgraph.size());
    gnblk[g] = blocks_of(p.graphs[g].n);
    voff[g] = p.graphs[g].voff;
    gn[g] = p.graphs[g].n;
    for (int b = 0; b < gnblk[g]; ++b) {
      bgraph.push_back(g);
      bsub.push_back(b);
    }
  }
  S->nblk = static_cast<int32_t>(bgraph.size());
  const size_t nb = size_t(p.n) * sizeof(double);
  if (hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) != hipSuccess) return STTSV_EHIP;
  auto alloc = [](auto** ptr, size_t bytes) { return hipMalloc(reinterpret_cast<void**>(ptr), bytes) == hipSuccess; };
  if (!alloc(&S->x, nb) || !alloc(&S->x32, nb / 2) || !alloc(&S->z, nb) || !alloc(&S->w, nb) ||
      !alloc(&S->part, 4 * sizeof(double) * S->nblk) || !alloc(&S->sums, sizeof(double) * G) ||
      !alloc(&S->bgraph, 4 * S->nblk) || !alloc(&S->bsub, 4 * S->nblk) || !alloc(&S->gblk0, 4 * G) ||
      !alloc(&S->gnblk, 4 * G) || !alloc(&S->voff, 4 * G) || !alloc(&S->gn, 4 * G) ||
      !alloc(&S->skip64, 4 * G) || !alloc(&S->skip32, 4 * G) || !alloc(&S->ctrl, sizeof(GCtrl) * G) ||
      !alloc(&S->sctrl, sizeof(SCtrl)))
    return STTSV_ENOMEM;
  if (hipHostMalloc(&S->hctrl, sizeof(GCtrl) * G, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&S->hsctrl, sizeof(SCtrl), hipHostMallocDefault) != hipSuccess)
    return STTSV_ENOMEM;
  auto up = [](void* d, const void* h, size_t bytes) { return hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) == hipSuccess; };
  if (!up(S->bgraph, bgraph.data(), 4 * bgraph.size()) || !up(S->bsub, bsub.data(), 4 * bsub.size()) ||
      !up(S->gblk0, gblk0.data(), 4 * G) || !up(S->gnblk, gnblk.data(), 4 * G) || !up(S->voff, voff.data(), 4 * G) ||
      !up(S->gn, gn.data(), 4 * G))
    return STTSV_EHIP;
  if (G > 1) {
    // graphs of every edge stage: those of the stage's buckets' order r (a
    // superset of the graphs with edges there, so a closed gate never skips
    // an edge that runs)
    const size_t ns = std::max(p.stages[0].size(), p.stages[1].size());
    S->gate_stride = static_cast<int32_t>(ns);
    S->ngate = static_cast<int32_t>(2 * ns);
    std::vector<int32_t> ptr(1, 0), gl;
    std::vector<char> in(G);
    for (int seq = 0; seq < 2; ++seq)
      for (size_t si = 0; si < ns; ++si) {
        std::fill(in.begin(), in.end(), 0);
        if (si < p.stages[seq].size()) {
          const Stage& st = p.stages[seq][si];
          std::vector<int> bl;
          if (st.type == 0)
            bl.push_back(st.index);
          else if (st.type == 1)
            bl = p.groups[st.index].buckets;
          for (int b : bl)
            for (int g = 0; g < G; ++g)
              if (p.graphs[g].r == p.buckets[b].r) in[g] = 1;
        }
        for (int g = 0; g < G; ++g)
          if (in[g]) gl.push_back(g);
        ptr.push_back(static_cast<int32_t>(gl.size()));
      }
    if (gl.empty()) gl.push_back(0);
    if (!alloc(&S->gate, 4 * std::max<size_t>(1, S->ngate)) || !alloc(&S->gate_ptr, 4 * ptr.size()) ||
        !alloc(&S->gate_graph, 4 * gl.size()))
      return STTSV_ENOMEM;
    if (!up(S->gate_ptr, ptr.data(), 4 * ptr.size()) || !up(S->gate_graph, gl.data(), 4 * gl.size()))
      return STTSV_EHIP;
  }
  return STTSV_OK;
}

int solve(Plan& p, const double* x0, double tol, const sttsv_solve_opts& o, double* x_out,
          sttsv_solve_info* infos) {
  if (!(tol > 0.0) || x_out == nullptr) return STTSV_EINVAL;
  if (o.max_iter < 1 || o.check_every < 1 || !(o.shift >= 0.0)) return STTSV_EINVAL;
  if (o.schedule != STTSV_SOLVE_FP64 && o.schedule != STTSV_SOLVE_FP32_FP64) return STTSV_EINVAL;
  if (!p.connected) return STTSV_EDISCONNECTED;
  int rc = ensure_solver(p);
  if (rc != STTSV_OK) return rc;
  Solver& S = *p.solver;
  const int G = S.G;
  const int n = p.n;
  if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;

  // control blocks
  std::vector<GCtrl> c(G);
  std::vector<int32_t> s64(G), s32(G);
  for (int g = 0; g < G; ++g) {
    c[g] = GCtrl{};
    c[g].status = STTSV_OK;
    c[g].r = p.graphs[g].r;
    c[g].prev_crit = INFINITY;
    c[g].crit = INFINITY;
    s64[g] = o.schedule == STTSV_SOLVE_FP32_FP64 ? 1 : 0;
    s32[g] = o.schedule == STTSV_SOLVE_FP32_FP64 ? 0 : 1;
  }
  SCtrl sc{};
  sc.all_done = 0;
  sc.max_iter = o.max_iter;
  sc.tol = tol;
  sc.switch_tol = o.switch_tol;
  sc.shift = o.shift;
  sc.no32 = o.schedule == STTSV_SOLVE_FP32_FP64 ? 0 : 1;
  if (hipMemcpyAsync(S.ctrl, c.data(), sizeof(GCtrl) * G, hipMemcpyHostToDevice, S.s) != hipSuccess ||
      hipMemcpyAsync(S.sctrl, &sc, sizeof(SCtrl), hipMemcpyHostToDevice, S.s) != hipSuccess ||
      hipMemcpyAsync(S.skip64, s64.data(), 4 * G, hipMemcpyHostToDevice, S.s) != hipSuccess ||
      hipMemcpyAsync(S.skip32, s32.data(), 4 * G, hipMemcpyHostToDevice, S.s) != hipSuccess)
    return STTSV_EHIP;

  // initial iterate (Alg. 1: y = 1/n, or the warm start), then z = TTSV1(y)
  // and the first x; the scale of y is irrelevant (homogeneity), so y / max(y)
  if (x0 == nullptr) {
    hipLaunchKernelGGL(fill_ones, dim3((n + kRedBlock - 1) / kRedBlock), dim3(kRedBlock), 0, S.s, S.x, n);
  } else {
    hipLaunchKernelGGL(init_stats, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, x0);
    hipLaunchKernelGGL(init_final, dim3(G), dim3(kRedBlock), 0, S.s, S);
    hipLaunchKernelGGL(scale_from_vertex_order, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, x0,
                       (const int32_t*)p.d_rid, S.x);
  }
  const int first_prec = o.schedule == STTSV_SOLVE_FP32_FP64 ? STTSV_PREC_FP32 : STTSV_PREC_FP64;
  const int32_t* first_skip = first_prec == STTSV_PREC_FP32 ? S.skip32 : S.skip64;
  if ((rc = hip_rc(launch_edges(p, S.x, first_prec, nullptr, first_skip, S.s, XOrder::kRank))) != STTSV_OK) return rc;
  if ((rc = hip_rc(launch_reduction(p, S.z, nullptr, S.s, true))) != STTSV_OK) return rc;
  hipLaunchKernelGGL((nqz_stats<false>), dim3(S.nblk), dim3(kRedBlock), 0, S.s, S);
  hipLaunchKernelGGL((nqz_final<false>), dim3(G), dim3(kRedBlock), 0, S.s, S);
  if (G > 1) hipLaunchKernelGGL(all_done_check, dim3(1 + S.ngate), dim3(kRedBlock), 0, S.s, S);
  hipLaunchKernelGGL(scale_into, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, (const double*)S.w, S.x,
                     compact_mixed(p, o.schedule) ? S.x32 : nullptr);
  if (hipGetLastError() != hipSuccess) return STTSV_EHIP;

  // iterations: captured graph of check_every iterations, or direct launches.
  // Under the FP32 -> FP64 schedule, once no open graph runs FP32 series any
  // more (a graph never switches back) the FP32 launches would all exit at
  // once: the remaining iterations run the FP64-only sequence instead, which
  // computes the same bits.
  const int K = o.check_every;
  auto capture = [&](int sched, hipGraphExec_t* exec) -> int {
    if (*exec) {
      (void)hipGraphExecDestroy(*exec);
      *exec = nullptr;
    }
    if (hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(S.s, hipStreamCaptureModeThreadLocal) != hipSuccess) return STTSV_EHIP;
    hipError_t e = hipSuccess;
    for (int t = 0; t < K && e == hipSuccess; ++t) e = enqueue_iteration(p, S, sched);
    const hipError_t e2 = hipStreamEndCapture(S.s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return STTSV_EHIP;
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *exec = nullptr;
      return STTSV_EHIP;
    }
    return STTSV_OK;
  };
  if (o.use_graph && (S.exec == nullptr || S.graph_iters != K || S.graph_sched != o.schedule)) {
    if ((rc = capture(o.schedule, &S.exec)) != STTSV_OK) return rc;
    S.graph_iters = K;
    S.graph_sched = o.schedule;
  }
  bool only64 = o.schedule != STTSV_SOLVE_FP32_FP64;
  for (;;) {
    const int sched = only64 ? STTSV_SOLVE_FP64 : o.schedule;
    if (o.use_graph) {
      hipGraphExec_t* ex = &S.exec;
      if (sched != o.schedule) {
        if (S.exec64 == nullptr || S.graph64_iters != K) {
          if ((rc = capture(STTSV_SOLVE_FP64, &S.exec64)) != STTSV_OK) return rc;
          S.graph64_iters = K;
        }
        ex = &S.exec64;
      }
      if (hipGraphLaunch(*ex, S.s) != hipSuccess) return STTSV_EHIP;
    } else {
      for (int t = 0; t < K; ++t)
        if (enqueue_iteration(p, S, sched) != hipSuccess) return STTSV_EHIP;
    }
    if (hipMemcpyAsync(S.hsctrl, S.sctrl, sizeof(SCtrl), hipMemcpyDeviceToHost, S.s) != hipSuccess) return STTSV_EHIP;
    if (hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;
    if (S.hsctrl->all_done) break;
    only64 = only64 || S.hsctrl->no32 != 0;
  }
  if (hipMemcpy(S.hctrl, S.ctrl, sizeof(GCtrl) * G, hipMemcpyDeviceToHost) != hipSuccess) return STTSV_EHIP;

  // x_out = x~ / ||x~||_1 per graph
  hipLaunchKernelGGL(sum_stage, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, (const double*)S.x);
  hipLaunchKernelGGL(sum_final, dim3(G), dim3(kRedBlock), 0, S.s, S);
  hipLaunchKernelGGL(divide_to_vertex_order, dim3(S.nblk), dim3(kRedBlock), 0, S.s, S, (const double*)S.x,
                     (const int32_t*)p.d_rid, x_out);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(S.s) != hipSuccess) return STTSV_EHIP;

  // overall status: the worst of the graphs' (EINVAL > ENUMERIC > ENOTCONV > OK)
  int worst = STTSV_OK;
  auto severity = [](int st) {
    return st == STTSV_EINVAL ? 3 : st == STTSV_ENUMERIC ? 2 : st == STTSV_ENOTCONV ? 1 : 0;
  };
  for (int g = 0; g < G; ++g) {
    const GCtrl& h = S.hctrl[g];
    if (severity(h.status) > severity(worst)) worst = h.status;
    if (infos != nullptr) {
      infos[g].iterations = h.iter;
      infos[g].iters_fp32 = h.it32;
      infos[g].iters_fp64 = h.it64;
      infos[g].converged = h.status == STTSV_OK && h.iter > 0 ? 1 : 0;
      infos[g].lambda_min = h.lmin - o.shift;
      infos[g].lambda_max = h.lmax - o.shift;
      infos[g].criterion = h.crit;
    }
  }
  return worst;
}

}  // namespace sttsv
