// STTSV launch sequence: one edge-major launch per size bucket (kernel picked
// by edge size and series window), then the deterministic node reduction.
#include "internal.hpp"

namespace sttsv {

void fill_edge_part0(EdgeTables&);
void fill_edge_part1(EdgeTables&);
void fill_edge_part2(EdgeTables&);
void fill_edge_part3(EdgeTables&);
void fill_edge_part4(EdgeTables&);
void fill_edge_part5(EdgeTables&);
void fill_edge_part6(EdgeTables&);
void fill_edge_part7(EdgeTables&);

namespace {

// Size-1 edges {v}: beta = {(v,..,v)}, value 1, so the term is x_v^(r-1).
__global__ void __launch_bounds__(256) edge_k1(EdgeLaunch a) {
  if (a.done != nullptr && *a.done) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.m) return;
  const double xv = a.x[a.mem[i]];
  int e2 = 0;
  const double f = frexp(xv, &e2);          // xv = f 2^e2
  double p = 1.0;
  for (int j = 0; j < a.r - 1; ++j) p *= f;
  a.contrib[i] = ldexp(p, (a.r - 1) * e2);
}

hipError_t launch_k1(const EdgeLaunch& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.m + 255) / 256));
  hipLaunchKernelGGL(edge_k1, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

EdgeTables build_tables() {
  EdgeTables t{};
  fill_edge_part0(t);
  fill_edge_part1(t);
  fill_edge_part2(t);
  fill_edge_part3(t);
  fill_edge_part4(t);
  fill_edge_part5(t);
  fill_edge_part6(t);
  fill_edge_part7(t);
  for (int w = 0; w <= kMaxW; ++w) {
    t.f64[KIND_K1][w] = &launch_k1;
    t.f32[KIND_K1][w] = &launch_k1;
  }
  return t;
}

}  // namespace

const EdgeTables& edge_tables() {
  static const EdgeTables t = build_tables();
  return t;
}

static int kind_of(int k) { return k == 1 ? KIND_K1 : k == 2 ? KIND_K2 : k == 3 ? KIND_K3 : KIND_KG; }

int stage_count(const Plan& p) { return static_cast<int>(p.buckets.size() + p.levels.size()); }

hipError_t launch_stage(Plan& p, int stage, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s) {
  const int nb = static_cast<int>(p.buckets.size());
  if (stage < nb) {
    const EdgeTables& tab = edge_tables();
    const Bucket& b = p.buckets[stage];
    const bool f32 = precision == STTSV_PREC_FP32 && b.fp32_ok && b.k > 1;
    EdgeLaunch a;
    a.x = x;
    a.mem = p.d_mem + b.slot_off;
    a.contrib = p.d_contrib + b.slot_off;
    a.done = done;
    a.m = b.m;
    a.k = b.k;
    a.r = p.r;
    a.qexp = f32 ? b.qexp32 : 0;
    a.lds_stack = f32 ? b.lds32 : b.lds64;
    a.gstack = f32 ? b.gstack32 : b.gstack64;
    a.wk = p.weights[b.k];
    const int W = p.r - b.k + 1;
    const int kind = kind_of(b.k);
    const int wi = kind == KIND_K1 ? 0 : W;
    EdgeLaunchFn fn = f32 ? tab.f32[kind][wi] : tab.f64[kind][wi];
    if (fn == nullptr) return hipErrorInvalidValue;
    return fn(a, s);
  }
  const size_t l = static_cast<size_t>(stage - nb);
  const double* in = l == 0 ? p.d_contrib : p.d_partials[l - 1];
  double* next = l < p.d_partials.size() ? p.d_partials[l] : nullptr;
  return launch_reduce_level(p.levels[l], static_cast<int>(l), in, p.d_tslot, y, next, done, s);
}

hipError_t launch_sttsv(Plan& p, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s) {
  const int ns = stage_count(p);
  for (int t = 0; t < ns; ++t) {
    const hipError_t e = launch_stage(p, t, x, y, precision, done, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void stage_desc(const Plan& p, int stage, int32_t* kind, int32_t* size, int64_t* count) {
  const int nb = static_cast<int>(p.buckets.size());
  if (stage < nb) {
    *kind = 0;
    *size = p.buckets[stage].k;
    *count = p.buckets[stage].m;
  } else {
    *kind = 1;
    *size = stage - nb;
    *count = p.levels[stage - nb].nchunks;
  }
}

}  // namespace sttsv
