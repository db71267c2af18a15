// STTSV launch sequence: per-bucket edge kernels (k = 1, 2, 3 and the
// register-resident k <= 7 kernels), one fused launch per window range for the
// generic buckets, then the deterministic node reduction.
#include <algorithm>
#include <utility>

#include <cmath>

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
void fill_edge_gen0(EdgeTables&);
void fill_edge_gen1(EdgeTables&);
void fill_edge_gen2(EdgeTables&);
void fill_edge_gen3(EdgeTables&);
void fill_edge_gen4(EdgeTables&);
void fill_edge_gen5(EdgeTables&);
void fill_edge_gen6(EdgeTables&);
void fill_edge_gen7(EdgeTables&);
void fill_edge_coop0(EdgeTables&);
void fill_edge_coop1(EdgeTables&);
void fill_edge_coop2(EdgeTables&);
void fill_edge_coop3(EdgeTables&);
void fill_edge_cpart0(EdgeTables&);
void fill_edge_cpart1(EdgeTables&);
void fill_edge_cpart2(EdgeTables&);
void fill_edge_cpart3(EdgeTables&);
void fill_edge_cpart4(EdgeTables&);
void fill_edge_cpart5(EdgeTables&);
void fill_edge_cpart6(EdgeTables&);
void fill_edge_cpart7(EdgeTables&);
void fill_edge_cgen0(EdgeTables&);
void fill_edge_cgen1(EdgeTables&);
void fill_edge_ccoop0(EdgeTables&);
void fill_edge_ccoop1(EdgeTables&);

namespace {

// Size-1 edges {v}: beta = {(v,..,v)}, value w(e), so the term is
// w(e) x_v^(r-1) (w(e) = |e| = 1 by default; an edge-weighted plan stores
// w(e) (r-1)!, and the table value for size 1 is (r-1)!).
__global__ void __launch_bounds__(256) edge_k1(EdgeCall c, BucketDesc b) {
  if (c.done != nullptr && *c.done) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= b.m) return;
  if (c.gskip != nullptr && c.gskip[b.gid != nullptr ? b.gid[i] : 0]) return;
  const double xv = c.x[b.mem[i]];
  int e2 = 0;
  const double f = frexp(xv, &e2);          // xv = f 2^e2
  double p = 1.0;
  for (int j = 0; j < b.r - 1; ++j) p *= f;
  if (b.wgt != nullptr) p *= b.wgt[i] / b.wk;
  store_contrib(c, b.loc[i], ldexp(p, (b.r - 1) * e2));
}

// x into degree-rank order: xr[p] = x[rid[p]] (and rounded to FP32 into
// xr32 when it is not null).
__global__ void __launch_bounds__(256) permute_x(const double* __restrict__ x, const int32_t* __restrict__ rid,
                                                 int64_t n, double* __restrict__ xr, float* __restrict__ xr32,
                                                 const int32_t* done) {
  if (done != nullptr && *done) return;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double v = x[rid[p]];
  xr[p] = v;
  if (xr32 != nullptr) xr32[p] = static_cast<float>(v);
}

hipError_t launch_k1(const EdgeCall& c, const BucketDesc& b, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((b.m + 255) / 256));
  hipLaunchKernelGGL(edge_k1, grid, dim3(256), 0, s, c, b);
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
  fill_edge_gen0(t);
  fill_edge_gen1(t);
  fill_edge_gen2(t);
  fill_edge_gen3(t);
  fill_edge_gen4(t);
  fill_edge_gen5(t);
  fill_edge_gen6(t);
  fill_edge_gen7(t);
  fill_edge_coop0(t);
  fill_edge_coop1(t);
  fill_edge_coop2(t);
  fill_edge_coop3(t);
  fill_edge_cpart0(t);
  fill_edge_cpart1(t);
  fill_edge_cpart2(t);
  fill_edge_cpart3(t);
  fill_edge_cpart4(t);
  fill_edge_cpart5(t);
  fill_edge_cpart6(t);
  fill_edge_cpart7(t);
  fill_edge_cgen0(t);
  fill_edge_cgen1(t);
  fill_edge_ccoop0(t);
  fill_edge_ccoop1(t);
  t.k1 = &launch_k1;
  return t;
}

}  // namespace

const EdgeTables& edge_tables() {
  static const EdgeTables t = build_tables();
  return t;
}

namespace {

// Rough time of an edge launch (s): a fixed launch cost, the incidence bytes
// at a random-access bandwidth, and the series FMAs at a fraction of the
// FP64 issue rate.  Only used to balance the stream lanes.
double edge_cost(int k, int r, int64_t m) {
  const double W = r - k + 1;
  double fma = 0.0;
  if (k == 2) fma = W;
  else if (k == 3) fma = 3.0 * W + W * (W - 1) / 2;
  else if (k > 3) fma = (k - 3) * W * (W - 1) + (k + 1) * W;
  return static_cast<double>(m) * (20.0 * k / 3.2e12 + 2.0 * fma / 3e13);
}

// Estimated edge work (s, launch costs excluded) below which a plan keeps
// all edge launches on its own stream.
constexpr double kLaneMinWork = 20e-6;

// Longest-first greedy assignment of every precision's edge stages to lanes.
void assign_lanes(Plan& p) {
  for (int seq = 0; seq < 2; ++seq) {
    std::vector<Stage>& st = p.stages[seq];
    std::vector<std::pair<double, size_t>> work;
    for (size_t t = 0; t < st.size(); ++t) {
      const Stage& S = st[t];
      double c = 5e-6;
      if (S.type == 0) {
        const Bucket& B = p.buckets[S.index];
        c += edge_cost(B.k, B.r, B.m);
      } else if (S.type == 1) {
        const GenGroup& G = p.groups[S.index];
        for (int b : G.buckets) {
          const Bucket& B = p.buckets[b];
          const int L = B.coop[G.f64 ? 0 : 1];
          if (G.coop)   // lane groups: 2 log2 L products per lane instead of 2(k-3) per edge
            c += edge_cost(B.k, B.r, B.m) * 1.5 * std::log2((double)L) * L / std::max(1, 2 * (B.k - 3));
          else          // the runtime-k kernel runs at about half the FMA rate of the others
            c += 2.0 * edge_cost(B.k, B.r, B.m);
        }
      } else {
        continue;
      }
      work.emplace_back(c, t);
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const std::pair<double, size_t>& a, const std::pair<double, size_t>& b) {
                       return a.first > b.first;
                     });
    // small plans: the fork / join costs more than the overlap can win
    double total = 0.0;
    for (const auto& w : work) total += w.first - 5e-6;
    const int nl = total < kLaneMinWork ? 1 : std::max(1, std::min<int>(kLanes, static_cast<int>(work.size())));
    std::vector<double> load(nl, 0.0);
    for (const auto& w : work) {
      const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      st[w.second].lane = l;
      load[l] += w.first;
    }
    // the plan's own stream takes the heaviest lane: it then tends to finish
    // last, and the join waits on helper lanes that are already done
    const int heavy = static_cast<int>(std::max_element(load.begin(), load.end()) - load.begin());
    if (heavy != 0)
      for (const auto& w : work) {
        int& l = st[w.second].lane;
        l = l == heavy ? 0 : l == 0 ? heavy : l;
      }
    p.lanes[seq] = nl;
  }
}

}  // namespace

void build_stages(Plan& p) {
  for (int seq = 0; seq < 2; ++seq) {
    std::vector<Stage>& st = p.stages[seq];
    st.clear();
    st.push_back(Stage{3, 0, true});
    for (size_t b = 0; b < p.buckets.size(); ++b) {
      const Bucket& B = p.buckets[b];
      const bool f64 = seq == 0 || !B.fp32_ok || B.k == 1;
      if (B.k == 1 || B.small_kind[f64 ? 0 : 1] >= 0) st.push_back(Stage{0, static_cast<int>(b), f64});
    }
    for (size_t g = 0; g < p.groups.size(); ++g)
      if (p.groups[g].seq == seq) st.push_back(Stage{1, static_cast<int>(g), p.groups[g].f64});
    for (size_t l = 0; l < p.levels.size(); ++l) st.push_back(Stage{2, static_cast<int>(l), true});
  }
  // FP32 applies run compact unless an edge stage of size >= 2 falls back to
  // FP64 series (its kernels store FP64 contributions); size-1 edges store
  // either form
  p.compact_ok = true;
  for (const Stage& S : p.stages[1]) {
    if (S.type == 0 && S.f64 && p.buckets[S.index].k != 1) p.compact_ok = false;
    if (S.type == 1 && S.f64) p.compact_ok = false;
  }
  assign_lanes(p);
}

int stage_count(const Plan& p, int precision) {
  return static_cast<int>(p.stages[precision == STTSV_PREC_FP32 ? 1 : 0].size());
}

static hipError_t launch_permute(Plan& p, const double* x, const int32_t* done, hipStream_t s, bool compact) {
  if (p.n == 0) return hipSuccess;
  hipLaunchKernelGGL(permute_x, dim3(static_cast<unsigned>((p.n + 255) / 256)), dim3(256), 0, s, x,
                     (const int32_t*)p.d_rid, (int64_t)p.n, p.d_xr, compact ? p.d_xr32 : nullptr, done);
  return hipGetLastError();
}

hipError_t launch_permute_x(Plan& p, const double* x, hipStream_t s) {
  return launch_permute(p, x, nullptr, s, false);
}

// The edge-launch arguments: compact (FP32 x from x32, 32-bit contributions)
// when x32 is given, else FP64 x and contributions.
static EdgeCall edge_call(Plan& p, const double* xr, const int32_t* done, const int32_t* gskip, const float* x32) {
  return EdgeCall{xr, p.d_contrib, done, gskip, x32, x32 != nullptr ? p.d_contrib32 : nullptr};
}

// c.x: the caller's x for the permute stage, the rank-ordered copy for edge stages
static hipError_t launch_stage_call(Plan& p, const Stage& S, const EdgeCall& c, double* y, hipStream_t s) {
  const EdgeTables& tab = edge_tables();
  const bool compact = c.contrib32 != nullptr;
  if (S.type == 3) return launch_permute(p, c.x, c.done, s, compact);
  if (S.type == 0) {
    const Bucket& B = p.buckets[S.index];
    const BucketDesc& d = B.desc[S.f64 ? 0 : 1];
    if (B.k == 1) return tab.k1(c, d, s);
    if (S.f64 && B.reuse) {
      const SmallLaunchFn fr = tab.run64[B.k - 4][d.W];
      return fr ? fr(c, d, s) : hipErrorInvalidValue;
    }
    if (compact && S.f64) return hipErrorInvalidValue;     // the plan's compact_ok rules this out
    const SmallLaunchFn fn = S.f64 ? tab.small64[B.small_kind[0]][d.W]
                                   : (compact ? tab.small32c : tab.small32)[B.small_kind[1]][d.W];
    return fn ? fn(c, d, s) : hipErrorInvalidValue;
  }
  if (S.type == 1) {
    const GenGroup& G = p.groups[S.index];
    if (compact && G.f64) return hipErrorInvalidValue;
    const GenLaunchFn fn = G.coop ? (G.f64 ? tab.coop64[G.range] : (compact ? tab.coop32c : tab.coop32)[G.range])
                                  : (G.f64 ? tab.gen64[G.range] : (compact ? tab.gen32c : tab.gen32)[G.range]);
    return fn ? fn(c, G.d_bks, G.d_tasks, G.ntasks, G.lds, s) : hipErrorInvalidValue;
  }
  const size_t l = static_cast<size_t>(S.index);
  const void* in = l > 0 ? static_cast<const void*>(p.d_partials[l - 1])
                         : compact ? static_cast<const void*>(p.d_contrib32) : static_cast<const void*>(p.d_contrib);
  double* next = l < p.d_partials.size() ? p.d_partials[l] : nullptr;
  return launch_reduce_level(p.levels[l], in, y, next, c.done, s, false, compact && l == 0);
}

hipError_t launch_stage(Plan& p, int stage, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s) {
  const Stage& S = p.stages[precision == STTSV_PREC_FP32 ? 1 : 0][stage];
  const bool compact = precision == STTSV_PREC_FP32 && p.compact_ok;
  if (S.type != 2) p.contrib_compact = compact;
  return launch_stage_call(p, S, edge_call(p, S.type == 3 ? x : p.d_xr, done, nullptr, compact ? p.d_xr32 : nullptr),
                           y, s);
}

hipError_t launch_sttsv(Plan& p, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s) {
  const bool compact = precision == STTSV_PREC_FP32 && p.compact_ok;
  const hipError_t e = launch_edges(p, x, precision, done, nullptr, s, XOrder::kVertex, compact);
  return e != hipSuccess ? e : launch_reduction(p, y, done, s, false, compact);
}

int init_lanes(Plan& p) {
  if (hipEventCreateWithFlags(&p.ev_fork, hipEventDisableTiming) != hipSuccess) return STTSV_EHIP;
  for (int l = 0; l < kLanes - 1; ++l)
    if (hipStreamCreateWithFlags(&p.aux[l], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p.ev_join[l], hipEventDisableTiming) != hipSuccess)
      return STTSV_EHIP;
  return STTSV_OK;
}

// Edge stages of np precisions (precs[i] with per-graph skip flags skips[i])
// inside one fork/join of the stream lanes.
// x32 (nullable): the FP32 stages run compact, gathering from it.
// gates[i] (nullable): per-stage flags of precision i, used as the stage's
// done flag.
static hipError_t launch_edge_sets(Plan& p, const double* x, const int* precs, const int32_t* const* skips, int np,
                                   const int32_t* done, hipStream_t s, XOrder order, const float* x32,
                                   const int32_t* const* gates) {
  const double* xr = order == XOrder::kRank ? x : p.d_xr;
  const bool multi = !(p.flags & STTSV_FLAG_ONE_STREAM) && p.ev_fork != nullptr;
  int nl = 1;
  if (multi)
    for (int i = 0; i < np; ++i) nl = std::max(nl, p.lanes[precs[i] == STTSV_PREC_FP32 ? 1 : 0]);
  hipError_t e = order == XOrder::kVertex ? launch_permute(p, x, done, s, x32 != nullptr) : hipSuccess;
  if (e != hipSuccess) return e;
  if (nl > 1) {
    // fork: every helper lane starts after the work already on s
    if ((e = hipEventRecord(p.ev_fork, s)) != hipSuccess) return e;
    for (int l = 0; l < nl - 1; ++l)
      if ((e = hipStreamWaitEvent(p.aux[l], p.ev_fork, 0)) != hipSuccess) return e;
  }
  for (int i = 0; i < np && e == hipSuccess; ++i) {
    const int seq = precs[i] == STTSV_PREC_FP32 ? 1 : 0;
    const bool lanes = nl > 1 && p.lanes[seq] > 1;
    EdgeCall c = edge_call(p, xr, done, skips[i], precs[i] == STTSV_PREC_FP32 ? x32 : nullptr);
    const int32_t* gate = gates != nullptr ? gates[i] : nullptr;
    for (size_t si = 0; si < p.stages[seq].size(); ++si) {
      const Stage& S = p.stages[seq][si];
      if (S.type == 2 || S.type == 3) continue;
      const hipStream_t ls = lanes && S.lane > 0 ? p.aux[S.lane - 1] : s;
      if (gate != nullptr) c.done = gate + si;
      if ((e = launch_stage_call(p, S, c, nullptr, ls)) != hipSuccess) break;
    }
  }
  if (nl > 1) {
    // join (also after a failed launch, so no helper lane is left forked):
    // helper l waits for helper l-1, and the plan's stream waits for the
    // last helper only, so only one cross-queue wait sits on its path
    hipError_t w = hipSuccess;
    for (int l = 0; l < nl - 1 && w == hipSuccess; ++l) {
      if (l > 0) w = hipStreamWaitEvent(p.aux[l], p.ev_join[l - 1], 0);
      if (w == hipSuccess) w = hipEventRecord(p.ev_join[l], p.aux[l]);
    }
    if (w == hipSuccess) w = hipStreamWaitEvent(s, p.ev_join[nl - 2], 0);
    if (e == hipSuccess) e = w;
  }
  return e;
}

hipError_t launch_edges(Plan& p, const double* x, int precision, const int32_t* done, const int32_t* gskip,
                        hipStream_t s, XOrder order, bool compact, const int32_t* gate) {
  // a compact launch needs the FP32 copy of x, which only the permute makes
  if (compact && (precision != STTSV_PREC_FP32 || order != XOrder::kVertex || !p.compact_ok))
    return hipErrorInvalidValue;
  p.contrib_compact = compact;
  return launch_edge_sets(p, x, &precision, &gskip, 1, done, s, order, compact ? p.d_xr32 : nullptr, &gate);
}

hipError_t launch_edges_both(Plan& p, const double* x, const int32_t* done, const int32_t* skip32,
                             const int32_t* skip64, hipStream_t s, const float* x32, const int32_t* gate32,
                             const int32_t* gate64) {
  const int precs[2] = {STTSV_PREC_FP32, STTSV_PREC_FP64};
  const int32_t* skips[2] = {skip32, skip64};
  const int32_t* gates[2] = {gate32, gate64};
  if (x32 != nullptr && !p.compact_ok) return hipErrorInvalidValue;
  p.contrib_compact = false;
  return launch_edge_sets(p, x, precs, skips, 2, done, s, XOrder::kRank, x32, gates);
}

hipError_t launch_reduction_phased(Plan& p, double* y, const int32_t* phase32, const int32_t* done, hipStream_t s,
                                   bool rank_out) {
  for (size_t l = 0; l < p.levels.size(); ++l) {
    double* next = l < p.d_partials.size() ? p.d_partials[l] : nullptr;
    const hipError_t e = l == 0 ? launch_reduce_level0_phased(p.levels[0], p.d_contrib, p.d_contrib32, phase32, y,
                                                              next, done, s, rank_out)
                                : launch_reduce_level(p.levels[l], p.d_partials[l - 1], y, next, done, s, rank_out);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduction(Plan& p, double* y, const int32_t* done, hipStream_t s, bool rank_out, bool compact) {
  for (size_t l = 0; l < p.levels.size(); ++l) {
    const void* in = l > 0 ? static_cast<const void*>(p.d_partials[l - 1])
                           : compact ? static_cast<const void*>(p.d_contrib32) : static_cast<const void*>(p.d_contrib);
    double* next = l < p.d_partials.size() ? p.d_partials[l] : nullptr;
    const hipError_t e = launch_reduce_level(p.levels[l], in, y, next, done, s, rank_out, compact && l == 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void stage_desc(const Plan& p, int precision, int stage, int32_t* kind, int32_t* size, int64_t* count) {
  const Stage& S = p.stages[precision == STTSV_PREC_FP32 ? 1 : 0][stage];
  *kind = S.type;
  if (S.type == 0) {
    *size = p.buckets[S.index].k;
    *count = p.buckets[S.index].m;
  } else if (S.type == 1) {
    if (p.groups[S.index].coop)
      *kind = 4;
    else if (p.groups[S.index].stack_free)
      *kind = 6;                                 // generic kernel without suffix stacks
    else if (p.groups[S.index].lds == 0)
      *kind = 5;                                 // generic kernel, suffix stacks in global memory
    *size = p.groups[S.index].range;
    int64_t m = 0;
    for (int b : p.groups[S.index].buckets) m += p.buckets[b].m;
    *count = m;
  } else if (S.type == 2) {
    *size = S.index;
    *count = p.levels[S.index].nchunks;
  } else {
    *size = 0;
    *count = p.n;
  }
}

}  // namespace sttsv
