// Host planner: validate the hypergraph, build the canonical layout, the
// weight table, the reduction schedule, and upload everything to the GPU.
//
// Canonical layout (the library's format; the paper's CCSS forest, Sec. III,
// is its prior art -- edges are sorted vertex sequences, Sec. II-B, grouped by
// size like the levels L_k of Sec. III):
//  1. deg(v) = number of edges containing v;
//  2. vertex order by (deg descending, id ascending); rank(v) = position;
//  3. every edge lists its members by increasing rank (hubs first);
//  4. canonical edge order by (size, member-rank sequence, input index);
//  5. buckets of equal size k, m_k edges each;
//  6. member slots in structure-of-arrays form: member j of the i-th edge of
//     bucket k at slot_off(k) + j m_k + i, slot_off(k) = sum_{k'<k} k' m_k';
//  7. node-major incidence lists: for each v the slots holding v, in
//     canonical edge order;
//  7a. the edge kernels gather x in degree-rank order (hubs first, so the hot
//     part of x shares cache lines): on the device, member slots hold rank
//     positions voff + rank, and every STTSV first copies x into that order;
//  8. contribution storage: vertices (in index order) form blocks of at
//     most kStageTerms incidences (a vertex with more forms a block of its
//     own); each block owns a contiguous region, split into one part per die
//     (workgroup w of a launch runs on die w mod 8), and the incidences that
//     one die's edge workgroups produce for the block take consecutive
//     places in its part, in (bucket, edge, member) order.  The edge
//     kernels' stores then advance write fronts, each filled by one die's
//     L2, instead of landing anywhere in the array, and a level-0 reduction
//     workgroup copies one block's region (or, for a larger vertex, at most
//     one range per die part) into LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace sttsv {
namespace {

// ---- host parallelism.  Every parallel loop below writes disjoint outputs
// or combines per-chunk results in a fixed order, so the layout is the same
// whatever the thread count.
int host_threads() {
  static const int t = [] {
    const unsigned h = std::thread::hardware_concurrency();
    return static_cast<int>(std::max(1u, std::min(16u, h)));
  }();
  return t;
}

thread_local bool t_in_parallel = false;   // loops nested in a parallel loop run inline

// f(chunk, begin, end) over [0, n) cut into at most host_threads() contiguous
// chunks (chunk index in order); small ranges, and loops inside another
// parallel loop, run inline.
template <typename F>
void parallel_chunks(int64_t n, F&& f, int64_t min_per_chunk = 1 << 15) {
  const int64_t T = t_in_parallel ? 1
                                  : std::max<int64_t>(1, std::min<int64_t>(host_threads(),
                                                                           n / std::max<int64_t>(1, min_per_chunk)));
  if (T <= 1) {
    f(0, int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T - 1);
  for (int64_t t = 1; t < T; ++t)
    th.emplace_back([&, t] {
      t_in_parallel = true;
      f(static_cast<int>(t), n * t / T, n * (t + 1) / T);
    });
  t_in_parallel = true;
  f(0, int64_t(0), n / T);
  t_in_parallel = false;
  for (auto& x : th) x.join();
}
int chunk_count(int64_t n, int64_t min_per_chunk = 1 << 15) {
  if (t_in_parallel) return 1;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / std::max<int64_t>(1, min_per_chunk))));
}

// Sort with a strict total order (equal keys impossible), in parallel: sorted
// chunks merged pairwise.  The order is unique, so the result equals
// std::sort's.
template <typename T, typename Less>
void parallel_sort(std::vector<T>& v, Less less) {
  const int64_t n = static_cast<int64_t>(v.size());
  const int T0 = chunk_count(n, 1 << 16);
  if (T0 <= 1) {
    std::sort(v.begin(), v.end(), less);
    return;
  }
  std::vector<int64_t> cut(T0 + 1);
  for (int t = 0; t <= T0; ++t) cut[t] = n * t / T0;
  {
    std::vector<std::thread> th;
    for (int t = 0; t < T0; ++t)
      th.emplace_back([&, t] { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1], less); });
    for (auto& x : th) x.join();
  }
  std::vector<T> tmp(v.size());
  std::vector<T>* src = &v;
  std::vector<T>* dst = &tmp;
  while (cut.size() > 2) {
    std::vector<int64_t> next;
    std::vector<std::thread> th;
    for (size_t q = 0; q + 1 < cut.size(); q += 2) {
      if (q + 2 < cut.size()) {
        const int64_t a = cut[q], b = cut[q + 1], e = cut[q + 2];
        th.emplace_back([=, &less] {
          std::merge(src->begin() + a, src->begin() + b, src->begin() + b, src->begin() + e, dst->begin() + a, less);
        });
        next.push_back(a);
      } else {                                  // an odd run out: copied as is
        const int64_t a = cut[q], e = cut[q + 1];
        th.emplace_back([=] { std::copy(src->begin() + a, src->begin() + e, dst->begin() + a); });
        next.push_back(a);
      }
    }
    for (auto& x : th) x.join();
    next.push_back(n);
    cut.swap(next);
    std::swap(src, dst);
  }
  if (src != &v) v.swap(*src);
}

// One level of the reduction schedule (host side).
struct HostLevel {
  std::vector<int32_t> start, len, dst;
  int64_t in_len = 0;
};

// Lanes that sum one level-0 chunk of length l: 8 for long chunks, fewer for
// chunks that fit (the kernel then adds the missing partial sums as the
// zeros they are, so the tree and its bits do not change).
int group_lanes(int32_t l) { return l <= 1 ? 1 : l == 2 ? 2 : l <= 4 ? 4 : 8; }
int lane_class(int32_t l) { return group_lanes(l) == 8 ? 0 : group_lanes(l) == 4 ? 1 : group_lanes(l) == 2 ? 2 : 3; }

// Level-0 chunks of a vertex of degree d, counted per lane class (8, 4, 2, 1).
void add_chunks(int64_t d, int64_t cnt[4]) {
  if (d <= kChunk) {
    cnt[lane_class(static_cast<int32_t>(d))]++;
    return;
  }
  const int64_t nch = (d + kChunk - 1) / kChunk;
  cnt[0] += nch - 1;
  cnt[lane_class(static_cast<int32_t>(d - (nch - 1) * kChunk))]++;
}

// Passes a level-0 workgroup makes over chunks counted per lane class.
int64_t stage_passes(const int64_t cnt[4]) {
  int64_t p = 0;
  for (int q = 0; q < 4; ++q) {
    const int64_t per = kStageThreads / (8 >> q);
    p += (cnt[q] + per - 1) / per;
  }
  return p;
}

// Launch order of reduction level 0.  One workgroup per vertex block (at
// most kStageTerms incidences and kStagePasses passes), and one per
// kStageTerms / kChunk consecutive chunks of a larger vertex (its own
// block); inside a workgroup the chunks go longest first, so they fall into
// runs of equal lane counts (8, 4, 2, 1); workgroups go heaviest first.
// Fills P.l0_* and returns the level with its chunks in that order.
HostLevel level0_schedule(Plan& P, const HostLevel& L, const std::vector<int32_t>& cblock) {
  const int64_t nc = static_cast<int64_t>(L.len.size());
  int32_t nb = 0;
  for (int64_t c = 0; c < nc; ++c) nb = std::max(nb, cblock[c] + 1);
  std::vector<std::vector<int64_t>> bc(nb);
  for (int64_t c = 0; c < nc; ++c) bc[cblock[c]].push_back(c);
  struct Wg {
    int32_t block;
    int64_t first, count, terms;   // chunks [first, first + count) of the block's list
  };
  std::vector<Wg> wgs;
  constexpr int64_t kPiece = kStageTerms / kChunk;
  for (int32_t b = 0; b < nb; ++b) {
    const auto& v = bc[b];
    const int64_t nv = static_cast<int64_t>(v.size());
    const int64_t step = P.region[b + 1] - P.region[b] > kStageTerms ? kPiece : std::max<int64_t>(nv, 1);
    for (int64_t i = 0; i < nv; i += step) {
      const int64_t cnt = std::min(step, nv - i);
      int64_t t = 0;
      for (int64_t q = i; q < i + cnt; ++q) t += L.len[v[q]];
      wgs.push_back(Wg{b, i, cnt, t});
    }
  }
  std::stable_sort(wgs.begin(), wgs.end(), [](const Wg& a, const Wg& q) { return a.terms > q.terms; });
  HostLevel R;
  R.in_len = L.in_len;
  P.l0_wg.clear();
  P.l0_n1.clear();
  P.l0_base.clear();
  P.l0_terms.clear();
  P.l0_graph.clear();
  for (const Wg& w : wgs) {
    std::vector<int64_t> v(bc[w.block].begin() + w.first, bc[w.block].begin() + w.first + w.count);
    std::stable_sort(v.begin(), v.end(), [&](int64_t a, int64_t q) { return L.len[a] > L.len[q]; });
    int64_t cnt[4] = {0, 0, 0, 0};
    int64_t base = INT64_MAX;
    for (int64_t c : v) {
      cnt[lane_class(L.len[c])]++;
      if (L.len[c] > 0) base = std::min<int64_t>(base, L.start[c]);
    }
    P.l0_wg.push_back(make_int4(static_cast<int32_t>(R.len.size()), static_cast<int32_t>(cnt[0]),
                                static_cast<int32_t>(cnt[1]), static_cast<int32_t>(cnt[2])));
    P.l0_n1.push_back(static_cast<int32_t>(cnt[3]));
    P.l0_graph.push_back(P.block_graph[w.block]);
    P.l0_base.push_back(base == INT64_MAX ? 0 : base);
    P.l0_terms.push_back(w.terms);
    for (int64_t c : v) {
      R.start.push_back(L.start[c]);
      R.len.push_back(L.len[c]);
      R.dst.push_back(L.dst[c]);
    }
  }
  return R;
}

// Level-0 LDS layout for the current places: the terms of a workgroup are
// the node-major incidences [base, base + terms); it copies the maximal runs
// of consecutive places they occupy (one run for a block of small vertices,
// at most one per die part for a piece of a large vertex), each term to LDS
// offset (its node-major index - base).
int stage_level0(Plan& P) {
  if (P.levels.empty() || P.levels[0].d_wg == nullptr) return STTSV_OK;
  ReduceLevel& D = P.levels[0];
  const size_t nwg = P.l0_wg.size();
  std::vector<int4> wg(2 * nwg);
  std::vector<int2> ranges;
  std::vector<uint16_t> lpos(P.nnz, 0);
  // per workgroup (in parallel): LDS offsets of its terms and the runs of
  // consecutive places it copies; then the runs are laid out in workgroup order
  std::vector<std::vector<int2>> wr(nwg);
  std::vector<int> bad(nwg, 0);
  parallel_chunks(static_cast<int64_t>(nwg), [&](int, int64_t w0, int64_t w1) {
    std::vector<int32_t> pl;
    for (int64_t w = w0; w < w1; ++w) {
      const int64_t base = P.l0_base[w], terms = P.l0_terms[w];
      const int64_t cnt[4] = {P.l0_wg[w].y, P.l0_wg[w].z, P.l0_wg[w].w, P.l0_n1[w]};
      if (terms > kStageTerms || base + terms > P.nnz || stage_passes(cnt) > kStagePasses) {
        bad[w] = 1;
        continue;
      }
      pl.resize(terms);
      for (int64_t q = 0; q < terms; ++q) {
        pl[q] = P.glist[base + q];
        lpos[pl[q]] = static_cast<uint16_t>(q);
      }
      std::sort(pl.begin(), pl.end());
      for (int64_t i = 0; i < terms; ++i) {
        if (i > 0 && pl[i] == pl[i - 1]) {          // two terms in one place
          bad[w] = 1;
          break;
        }
        if (i == 0 || pl[i] != pl[i - 1] + 1) wr[w].push_back(make_int2(pl[i], 0));
        wr[w].back().y++;
      }
      if (wr[w].size() > static_cast<size_t>(kStageRuns)) bad[w] = 1;
    }
  }, 16);
  for (size_t w = 0; w < nwg; ++w) {
    if (bad[w]) return STTSV_EINVAL;
    const int32_t r0 = static_cast<int32_t>(ranges.size());
    ranges.insert(ranges.end(), wr[w].begin(), wr[w].end());
    wg[2 * w] = P.l0_wg[w];
    wg[2 * w + 1] = make_int4(P.l0_n1[w], r0, static_cast<int32_t>(wr[w].size()), P.l0_graph[w]);
  }
  if (hipMemcpy(D.d_wg, wg.data(), sizeof(int4) * wg.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (!ranges.empty() &&
       hipMemcpy(D.d_ranges, ranges.data(), sizeof(int2) * ranges.size(), hipMemcpyHostToDevice) != hipSuccess) ||
      (P.nnz > 0 && hipMemcpy(D.d_lpos, lpos.data(), sizeof(uint16_t) * P.nnz, hipMemcpyHostToDevice) != hipSuccess))
    return STTSV_EHIP;
  return STTSV_OK;
}

struct Dsu {
  std::vector<int32_t> p;
  explicit Dsu(int32_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int32_t find(int32_t a) {
    while (p[a] != a) {
      p[a] = p[p[a]];
      a = p[a];
    }
    return a;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

// w(e)/|beta(e)| (r-1)! = (r-1)! / ((k-1)! S(r,k)) for every k <= r
// (w(e) = |e| and |beta(e)| = |e|! S(r,|e|), Sec. II).  Stirling numbers by
// their recurrence in extended precision; one rounding to double at the end.
std::vector<double> weight_table(int r) {
  std::vector<std::vector<long double>> S(r + 1, std::vector<long double>(r + 1, 0.0L));
  S[0][0] = 1.0L;
  for (int a = 1; a <= r; ++a)
    for (int b = 1; b <= a; ++b) S[a][b] = (long double)b * S[a - 1][b] + S[a - 1][b - 1];
  std::vector<double> w(r + 1, 0.0);
  for (int k = 1; k <= r; ++k) {
    long double num = 1.0L;  // (r-1)!/(k-1)!
    for (int j = k; j <= r - 1; ++j) num *= (long double)j;
    w[k] = static_cast<double>(num / S[r][k]);
  }
  return w;
}

// w(e)/|beta(e)| (r-1)! for an edge of size k with weight w: w times
// (r-1)!/(k! S(r,k)) in extended precision, one rounding to double.
std::vector<long double> unit_weight_table(int r) {
  std::vector<std::vector<long double>> S(r + 1, std::vector<long double>(r + 1, 0.0L));
  S[0][0] = 1.0L;
  for (int a = 1; a <= r; ++a)
    for (int b = 1; b <= a; ++b) S[a][b] = (long double)b * S[a - 1][b] + S[a - 1][b - 1];
  std::vector<long double> u(r + 1, 0.0L);
  for (int k = 1; k <= r; ++k) {
    long double num = 1.0L;  // (r-1)!/k!
    for (int j = k + 1; j <= r - 1; ++j) num *= (long double)j;
    if (k == r) num = 1.0L / (long double)r;
    u[k] = num / S[r][k];
  }
  return u;
}

double log2_fact(int a) {
  double s = 0.0;
  for (int j = 2; j <= a; ++j) s += std::log2((double)j);
  return s;
}

// FP32 series range check for edges of size k in an order-r tensor.  With
// z_i <= rho = 2^q and max z_i > rho/2, every coefficient met is at most
// max_{d<W} (k rho)^d / d! and the coefficients that matter (g_j, P) are at
// least (rho/2)^(W-1)/W!.  Pick q to centre that range inside FP32's; report
// false if it does not fit with margin.
bool fp32_scale(int r, int k, int* qout) {
  const int W = r - k + 1;
  double best = -1e300;
  int bq = 0;
  for (int q = -8; q <= 12; ++q) {
    double hi = 0.0;
    for (int d = 0; d < W; ++d) hi = std::max(hi, d * (std::log2((double)k) + q) - log2_fact(d));
    double lo = (W - 1) * (q - 1.0) - log2_fact(W);
    if (W >= 2) lo = std::min(lo, (W - 2) * (q - 1.0) - log2_fact(W - 1));
    const double margin = std::min(120.0 - hi, lo + 110.0);
    if (margin > best) {
      best = margin;
      bq = q;
    }
  }
  *qout = bq;
  return best >= 0.0;
}

template <typename T>
int upload(T** dptr, const T* src, size_t count, int64_t* acct) {
  *dptr = nullptr;
  if (count == 0) return STTSV_OK;
  if (hipMalloc(reinterpret_cast<void**>(dptr), count * sizeof(T)) != hipSuccess) {
    *dptr = nullptr;
    return STTSV_ENOMEM;
  }
  *acct += (int64_t)(count * sizeof(T));
  if (src != nullptr && hipMemcpy(*dptr, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return STTSV_EHIP;
  return STTSV_OK;
}

}  // namespace

void free_plan(Plan* p) {
  if (p == nullptr) return;
  free_solver(*p);
  free_zstate(*p);
  free_ccss(*p);
  (void)hipFree(p->d_mem);
  (void)hipFree(p->d_rid);
  (void)hipFree(p->d_xr);
  (void)hipFree(p->d_xr32);
  (void)hipFree(p->d_contrib32);
  (void)hipFree(p->d_loc);
  (void)hipFree(p->d_gid);
  (void)hipFree(p->d_wgt);
  (void)hipFree(p->d_contrib);
  for (auto& g : p->groups) {
    (void)hipFree(g.d_bks);
    (void)hipFree(g.d_tasks);
  }
  for (auto& L : p->levels) {
    (void)hipFree(L.d_desc);
    (void)hipFree(L.d_wg);
    (void)hipFree(L.d_ranges);
    (void)hipFree(L.d_lpos);
    (void)hipFree(L.d_desc0[0]);
    (void)hipFree(L.d_desc0[1]);
  }
  for (double* d : p->d_partials) (void)hipFree(d);
  for (auto& b : p->buckets) {
    (void)hipFree(b.gstack[0]);
    (void)hipFree(b.gstack[1]);
    (void)hipFree(b.d_runs);
  }
  for (int l = 0; l < kLanes - 1; ++l) {
    if (p->aux[l]) (void)hipStreamDestroy(p->aux[l]);
    if (p->ev_join[l]) (void)hipEventDestroy(p->ev_join[l]);
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  delete p;
}

namespace {

// Checks of one hypergraph (problem statement of Sec. II: a set system of
// non-empty vertex subsets of size <= r).  Fills deg on success.
int validate_graph(const GraphIn& g, std::vector<int64_t>& deg) {
  if (g.eptr == nullptr || g.eidx == nullptr) return STTSV_EINVAL;
  if (g.m < 1 || g.n < 1) return STTSV_EINVAL;
  if (g.r < 2 || g.r > STTSV_MAX_ORDER) return STTSV_ENOTSUP;
  if (g.eptr[0] != 0) return STTSV_EINVAL;
  for (int64_t e = 0; e < g.m; ++e) {
    const int64_t k = g.eptr[e + 1] - g.eptr[e];
    if (k < 1 || k > g.r) return STTSV_EINVAL;
  }
  if (g.w != nullptr)
    for (int64_t e = 0; e < g.m; ++e)
      if (!(std::isfinite(g.w[e]) && g.w[e] > 0.0)) return STTSV_EINVAL;   // w(e) finite and positive
  deg.assign(g.n, 0);
  std::vector<int64_t> seen(g.n, -1);
  for (int64_t e = 0; e < g.m; ++e) {
    for (int64_t p = g.eptr[e]; p < g.eptr[e + 1]; ++p) {
      const int32_t v = g.eidx[p];
      if (v < 0 || v >= g.n) return STTSV_EINVAL;
      if (seen[v] == e) return STTSV_EINVAL;   // repeated vertex in an edge
      seen[v] = e;
      deg[v]++;
    }
  }
  return STTSV_OK;
}

// Canonical order of one graph: vertex ranks (degree descending, id
// ascending), members of every edge by rank, and for every size k the edges
// sorted by (member-rank sequence, input index).  rk holds each edge's
// member ranks, sorted, at the edge's CSR offsets.
struct Canon {
  std::vector<int32_t> inv_rank;                 // rank -> vertex
  std::vector<int32_t> rk;
  std::vector<std::vector<int64_t>> order;       // [k] -> input edges, canonical
};

void canonicalise(const GraphIn& g, const std::vector<int64_t>& deg, Canon& c) {
  const int32_t n = g.n;
  std::vector<int32_t> rank(n);
  int64_t maxd = 0;
  for (int64_t d : deg) maxd = std::max(maxd, d);
  std::vector<int64_t> cnt(maxd + 2, 0);
  for (int64_t d : deg) cnt[maxd - d + 1]++;
  for (int64_t i = 1; i < (int64_t)cnt.size(); ++i) cnt[i] += cnt[i - 1];
  for (int32_t v = 0; v < n; ++v) rank[v] = static_cast<int32_t>(cnt[maxd - deg[v]]++);
  c.inv_rank.assign(n, 0);
  for (int32_t v = 0; v < n; ++v) c.inv_rank[rank[v]] = v;
  const int64_t nnz = g.eptr[g.m];
  c.rk.assign(nnz, 0);
  parallel_chunks(g.m, [&](int, int64_t e0, int64_t e1) {
    for (int64_t e = e0; e < e1; ++e) {
      int32_t* a = c.rk.data() + g.eptr[e];
      const int64_t k = g.eptr[e + 1] - g.eptr[e];
      for (int64_t j = 0; j < k; ++j) a[j] = rank[g.eidx[g.eptr[e] + j]];
      std::sort(a, a + k);
    }
  });
  c.order.assign(g.r + 1, {});
  for (int64_t e = 0; e < g.m; ++e) c.order[g.eptr[e + 1] - g.eptr[e]].push_back(e);
  for (int k = 1; k <= g.r; ++k) {
    auto& ids = c.order[k];
    if (ids.empty()) continue;
    struct Key {
      uint64_t head;
      int64_t id;
    };
    std::vector<Key> keys(ids.size());
    parallel_chunks(static_cast<int64_t>(ids.size()), [&](int, int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) {
        const int32_t* a = c.rk.data() + g.eptr[ids[t]];
        const uint64_t r0 = (uint64_t)(uint32_t)a[0];
        const uint64_t r1 = k > 1 ? (uint64_t)(uint32_t)a[1] : 0;
        keys[t] = Key{(r0 << 32) | r1, ids[t]};
      }
    });
    parallel_sort(keys, [&](const Key& x, const Key& y) {
      if (x.head != y.head) return x.head < y.head;
      const int32_t* a = c.rk.data() + g.eptr[x.id];
      const int32_t* b = c.rk.data() + g.eptr[y.id];
      for (int j = 2; j < k; ++j)
        if (a[j] != b[j]) return a[j] < b[j];
      return x.id < y.id;
    });
    parallel_chunks(static_cast<int64_t>(ids.size()), [&](int, int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t) ids[t] = keys[t].id;
    });
  }
}

// ||B||^2 = sum over distinct vertex sets S of W_S^2 / |beta(S)| (Sec. II:
// every entry of the blowup of S holds W_S / |beta(S)|, and edges on one
// vertex set add to the same entries); |beta(S)| = |S|! S(r, |S|).  The
// canonical order puts edges on one vertex set next to each other.
double blowup_norm2(const GraphIn& g, const Canon& c) {
  std::vector<std::vector<long double>> S(g.r + 1, std::vector<long double>(g.r + 1, 0.0L));
  S[0][0] = 1.0L;
  for (int a = 1; a <= g.r; ++a)
    for (int b = 1; b <= a; ++b) S[a][b] = (long double)b * S[a - 1][b] + S[a - 1][b - 1];
  // groups of equal vertex sets are summed in blocks of a fixed number of
  // edges (a block starts at the first group beginning in it), the block
  // sums added in order: the value does not depend on the thread count
  constexpr int64_t kBlk = 1 << 16;
  long double tot = 0.0L, fact = 1.0L;
  for (int k = 1; k <= g.r; ++k) {
    fact *= (long double)k;
    const long double beta = fact * S[g.r][k];
    const auto& ids = c.order[k];
    const int64_t ne = static_cast<int64_t>(ids.size());
    auto same = [&](int64_t a, int64_t b) {
      return std::equal(c.rk.data() + g.eptr[ids[a]], c.rk.data() + g.eptr[ids[a]] + k, c.rk.data() + g.eptr[ids[b]]);
    };
    auto group_start = [&](int64_t t) {   // first group that begins at or after t
      while (t > 0 && t < ne && same(t, t - 1)) ++t;
      return t;
    };
    const int64_t nb = (ne + kBlk - 1) / kBlk;
    std::vector<long double> part(nb, 0.0L);
    parallel_chunks(nb, [&](int, int64_t b0, int64_t b1) {
      for (int64_t b = b0; b < b1; ++b) {
        int64_t t = group_start(b * kBlk);
        const int64_t end = group_start(std::min(ne, (b + 1) * kBlk));
        long double acc = 0.0L;
        while (t < end) {
          long double W = 0.0L;
          int64_t u = t;
          for (; u < ne; ++u) {
            if (u > t && !same(u, t)) break;
            W += g.w != nullptr ? (long double)g.w[ids[u]] : (long double)k;
          }
          acc += W * W / beta;
          t = u;
        }
        part[b] = acc;
      }
    }, 1);
    for (int64_t b = 0; b < nb; ++b) tot += part[b];
  }
  return static_cast<double>(tot);
}

bool connected_graph(const GraphIn& g, const std::vector<int64_t>& deg) {
  Dsu d(g.n);
  for (int64_t e = 0; e < g.m; ++e)
    for (int64_t p = g.eptr[e] + 1; p < g.eptr[e + 1]; ++p) d.unite(g.eidx[g.eptr[e]], g.eidx[p]);
  for (int32_t v = 0; v < g.n; ++v)
    if (deg[v] == 0 || d.find(v) != 0) return false;
  return true;
}

}  // namespace

// Lane groups pay where one lane per edge leaves the chip idle: the one-lane
// kernel runs an edge's 2(k-3) products one after another, with a dependent
// gather, store and reload per member, a group of L lanes 2 log2(L) products
// per lane.  They are taken for sizes k >= 8 whose chain shrinks by more than
// the group's 1.5x shuffle and idle-lane cost, when all of the graph's edges
// in the same window range would make fewer one-lane waves than half the
// chip's SIMDs (else the fused one-lane launch keeps the chip busy and its
// total work is lower).
int coop_lanes(int r, int k, int64_t range_waves) {
  constexpr int64_t kHalfSimds = 512;
  (void)r;
  if (k < 8 || k > 64) return 0;
  int L = 8;
  while (L < k) L <<= 1;
  if (k - 3.0 <= 1.5 * std::log2((double)L)) return 0;
  return range_waves < kHalfSimds ? L : 0;
}

// Fused generic launches: every bucket of size >= 4 without a per-bucket
// kernel, grouped by (launch sequence, series type, window range).  Frees
// and rebuilds the groups; stage lists must be rebuilt afterwards.
int build_groups(Plan& P) {
  for (auto& g : P.groups) {
    (void)hipFree(g.d_bks);
    (void)hipFree(g.d_tasks);
    P.device_bytes -= g.bytes;
  }
  P.groups.clear();
  for (Bucket& B : P.buckets) B.task0 = -1;
  int rc = STTSV_OK;
  for (int seq = 0; seq < 2; ++seq) {
    for (int rg = 0; rg < kGenRanges; ++rg) {
      for (int t = 0; t < 2; ++t) {
       for (int cp = 0; cp < 2; ++cp) {
        GenGroup grp;
        grp.range = rg;
        grp.seq = seq;
        grp.f64 = t == 0;
        grp.coop = cp == 1;
        for (size_t b = 0; b < P.buckets.size(); ++b) {
          const Bucket& B = P.buckets[b];
          const int type = (seq == 0 || !B.fp32_ok || B.k == 1) ? 0 : 1;
          if (type != t || B.k < 4 || B.small_kind[t] >= 0 || (B.coop[t] > 0) != grp.coop) continue;
          if (gen_range_of(B.r - B.k + 1) != rg) continue;
          grp.buckets.push_back(static_cast<int>(b));
        }
        if (grp.buckets.empty()) continue;
        if (grp.coop) {
          // lane groups: the largest per-lane work (log2(L) W^2) first
          std::stable_sort(grp.buckets.begin(), grp.buckets.end(), [&](int a, int b) {
            const Bucket& A = P.buckets[a];
            const Bucket& B = P.buckets[b];
            const int64_t wa = (int64_t)A.coop[t] * (A.r - A.k + 1) * (A.r - A.k + 1);
            const int64_t wb = (int64_t)B.coop[t] * (B.r - B.k + 1) * (B.r - B.k + 1);
            return wa > wb;
          });
          std::vector<BucketDesc> bks;
          std::vector<GenTask> tasks;
          for (size_t q = 0; q < grp.buckets.size(); ++q) {
            Bucket& B = P.buckets[grp.buckets[q]];
            if (seq == 0 && t == 0) B.task0 = static_cast<int64_t>(tasks.size());
            bks.push_back(B.desc[t]);
            const int64_t per = kCoopBlock / B.coop[t];
            const int64_t nblk = (B.m + per - 1) / per;
            for (int64_t blk = 0; blk < nblk; ++blk)
              tasks.push_back(GenTask{static_cast<int32_t>(q), static_cast<int32_t>(blk)});
          }
          grp.ntasks = (int64_t)tasks.size();
          P.groups.push_back(std::move(grp));
          GenGroup& H = P.groups.back();
          const int64_t before = P.device_bytes;
          if ((rc = upload(&H.d_bks, bks.data(), bks.size(), &P.device_bytes)) != STTSV_OK) return rc;
          if ((rc = upload(&H.d_tasks, tasks.data(), tasks.size(), &P.device_bytes)) != STTSV_OK) return rc;
          H.bytes = P.device_bytes - before;
          continue;
        }
        // longest per-edge work first, so the slow blocks start early
        std::stable_sort(grp.buckets.begin(), grp.buckets.end(), [&](int a, int b) {
          const Bucket& A = P.buckets[a];
          const Bucket& B = P.buckets[b];
          const int64_t wa = (int64_t)(A.k - 3) * (A.r - A.k + 1) * (A.r - A.k + 1);
          const int64_t wb = (int64_t)(B.k - 3) * (B.r - B.k + 1) * (B.r - B.k + 1);
          return wa > wb;
        });
        const size_t tsz = t == 0 ? sizeof(double) : sizeof(float);
        auto need_of = [&](const Bucket& B) {
          return (int64_t)kGenBlock * kg_stack_bytes(B.k, B.r - B.k + 1, static_cast<int>(tsz));
        };
        auto free_ok = [&](const Bucket& B) {   // the stack-free variant exists and its scalars fit
          return stack_free_ok(B.r - B.k + 1, static_cast<int>(tsz)) &&
                 (int64_t)kGenBlock * kg_scalar_bytes(B.k) <= kLdsMax;
        };
        // placement: 0 = stack in LDS, 1 = in global memory, 2 = no stack
        // (tuner choices; without one, LDS when it fits the default budget)
        auto place_of = [&](const Bucket& B) {
          const int64_t need = need_of(B);
          const int pref = B.lds_pref[t];
          if (pref == kStackFree) return free_ok(B) ? 2 : need <= kLdsBudget ? 0 : 1;
          return pref >= 0 ? (pref == 1 && need <= kLdsMax ? 0 : 1) : (need <= kLdsBudget ? 0 : 1);
        };
        // a launch reserves its largest LDS need for every block, so buckets
        // of different placements get launches of their own (else global-
        // stack buckets would run at the LDS-limited occupancy of the others)
        std::vector<int> parts[3];
        for (int b : grp.buckets) parts[place_of(P.buckets[b])].push_back(b);
        for (int part = 0; part < 3; ++part) {
          const std::vector<int>& list = parts[part];
          if (list.empty()) continue;
          GenGroup sub;
          sub.range = grp.range;
          sub.seq = grp.seq;
          sub.f64 = grp.f64;
          sub.coop = false;
          sub.stack_free = part == 2;
          sub.buckets = list;
          std::vector<BucketDesc> bks;
          std::vector<GenTask> tasks;
          for (size_t q = 0; q < sub.buckets.size(); ++q) {
            Bucket& B = P.buckets[sub.buckets[q]];
            if (seq == 0 && t == 0) B.task0 = static_cast<int64_t>(tasks.size());
            const int W = B.r - B.k + 1;
            BucketDesc& d = B.desc[t];
            if (part == 0) {
              d.lds_stack = 1;
              sub.lds = std::max(sub.lds, static_cast<size_t>(need_of(B)));
            } else if (part == 2) {
              d.lds_stack = kStackFree;
              sub.lds = std::max(sub.lds, static_cast<size_t>((int64_t)kGenBlock * kg_scalar_bytes(B.k)));
            } else {
              d.lds_stack = 0;
              if (B.gstack[t] == nullptr) {
                const size_t bytes = (size_t)kg_stack_bytes(B.k, W, static_cast<int>(tsz)) * (size_t)B.m;
                if (hipMalloc(&B.gstack[t], bytes) != hipSuccess) return STTSV_ENOMEM;
                P.device_bytes += (int64_t)bytes;
              }
              d.gstack = B.gstack[t];
            }
            bks.push_back(d);
            const int64_t nblk = (B.m + kGenBlock - 1) / kGenBlock;
            for (int64_t blk = 0; blk < nblk; ++blk)
              tasks.push_back(GenTask{static_cast<int32_t>(q), static_cast<int32_t>(blk)});
          }
          sub.ntasks = (int64_t)tasks.size();
          P.groups.push_back(std::move(sub));
          GenGroup& H = P.groups.back();
          const int64_t before = P.device_bytes;
          if ((rc = upload(&H.d_bks, bks.data(), bks.size(), &P.device_bytes)) != STTSV_OK) return rc;
          if ((rc = upload(&H.d_tasks, tasks.data(), tasks.size(), &P.device_bytes)) != STTSV_OK) return rc;
          H.bytes = P.device_bytes - before;
        }
       }
      }
    }
  }
  return STTSV_OK;
}

// Smallest binary exponent of min(z_0, z_1) (both shifts) for which every
// value of the FP64 product phi(z_0 t) phi(z_1 t) truncated to W terms stays
// normal with a margin of 2^16: z^(W-1) / W! >= 2^(-1006).
static int reuse_emin(int W) {
  if (W < 2) return INT32_MIN / 2;
  double lf = 0.0;   // log2(W!)
  for (int q = 2; q <= W; ++q) lf += std::log2(static_cast<double>(q));
  return static_cast<int>(std::ceil((-1006.0 + lf) / (W - 1)));
}

// Prefix reuse for one bucket: runs of at most kRunMax consecutive canonical
// edges whose first two members agree (hence also their graph), longest
// first.  Only FP64 register-resident buckets take it.
int set_reuse(Plan& P, Bucket& B, bool by_flag) {
  const bool want = B.reuse_pref >= 0 ? B.reuse_pref == 1 : by_flag;
  const bool ok = B.small_kind[0] >= SK_R4 && B.small_kind[0] <= SK_R7 &&
                  edge_tables().run64[B.k - 4][B.r - B.k + 1] != nullptr;
  B.reuse = want && ok;
  BucketDesc& d = B.desc[0];
  if (!B.reuse) {
    d.run_start = nullptr;
    d.nruns = 0;
    return STTSV_OK;
  }
  if (B.d_runs == nullptr) {
    std::vector<std::vector<int32_t>> by_len(kRunMax + 1);
    const int32_t* m0 = P.mem.data() + B.slot_off;
    const int32_t* m1 = m0 + B.m;
    for (int64_t i = 0; i < B.m;) {
      int64_t j = i + 1;
      while (j < B.m && j - i < kRunMax && m0[j] == m0[i] && m1[j] == m1[i]) ++j;
      by_len[j - i].push_back(static_cast<int32_t>(i));
      i = j;
    }
    B.runs.clear();
    for (int L = kRunMax; L >= 1; --L) {
      d.run_cnt[kRunMax - L] = static_cast<int32_t>(by_len[L].size());
      B.runs.insert(B.runs.end(), by_len[L].begin(), by_len[L].end());
    }
    int rc = upload(&B.d_runs, B.runs.data(), B.runs.size(), &P.device_bytes);
    if (rc != STTSV_OK) return rc;
  }
  d.run_start = B.d_runs;
  d.nruns = static_cast<int64_t>(B.runs.size());
  return STTSV_OK;
}

// Die of every edge of bucket B in the FP64 launch sequence (workgroup w of
// a launch runs on die w mod kXcd).
static void edge_dies(const Bucket& B, std::vector<uint8_t>& die) {
  die.assign(B.m, 0);
  if (B.reuse) {
    int64_t t = 0;
    for (int q = 0; q < kRunMax; ++q)
      for (int32_t c = 0; c < B.desc[0].run_cnt[q]; ++c, ++t)
        for (int u = 0; u < kRunMax - q; ++u)
          die[B.runs[t] + u] = static_cast<uint8_t>((t / kSmallBlock) % kXcd);
    return;
  }
  for (int64_t i = 0; i < B.m; ++i) {
    if (B.coop[0] > 0)
      die[i] = static_cast<uint8_t>((B.task0 + i / (kCoopBlock / B.coop[0])) % kXcd);
    else if (B.k == 1 || B.small_kind[0] >= 0)
      die[i] = static_cast<uint8_t>((i / kSmallBlock) % kXcd);
    else if (B.task0 >= 0)
      die[i] = static_cast<uint8_t>((B.task0 + i / kGenBlock) % kXcd);
  }
}

int assign_places(Plan& P) {
  const int64_t nnz = P.nnz;
  const int32_t nb = static_cast<int32_t>(P.region.size()) - 1;
  std::vector<int64_t> cur((size_t)nb * kXcd, 0);
  std::vector<std::vector<uint8_t>> dies(P.buckets.size());
  for (size_t bi = 0; bi < P.buckets.size(); ++bi) edge_dies(P.buckets[bi], dies[bi]);
  for (size_t bi = 0; bi < P.buckets.size(); ++bi) {
    const Bucket& B = P.buckets[bi];
    for (int64_t i = 0; i < B.m; ++i) {
      const int x = dies[bi][i];
      for (int j = 0; j < B.k; ++j) cur[(size_t)P.vblock[P.mem[B.slot_off + (int64_t)j * B.m + i]] * kXcd + x]++;
    }
  }
  for (int32_t b = 0; b < nb; ++b) {
    int64_t at = P.region[b];
    for (int x = 0; x < kXcd; ++x) {
      const int64_t c = cur[(size_t)b * kXcd + x];
      cur[(size_t)b * kXcd + x] = at;
      at += c;
    }
  }
  std::vector<int32_t> loc(nnz);
  for (size_t bi = 0; bi < P.buckets.size(); ++bi) {
    const Bucket& B = P.buckets[bi];
    for (int64_t i = 0; i < B.m; ++i) {
      const int x = dies[bi][i];
      for (int j = 0; j < B.k; ++j) {
        const int64_t s = B.slot_off + (int64_t)j * B.m + i;
        loc[s] = static_cast<int32_t>(cur[(size_t)P.vblock[P.mem[s]] * kXcd + x]++);
      }
    }
  }
  std::vector<int32_t> glist(nnz);
  parallel_chunks(nnz, [&](int, int64_t q0, int64_t q1) {
    for (int64_t q = q0; q < q1; ++q) glist[q] = loc[P.tslot[q]];
  });
  if (nnz > 0 && hipMemcpy(P.d_loc, loc.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice) != hipSuccess)
    return STTSV_EHIP;
  P.glist = std::move(glist);
  return stage_level0(P);
}

// Node-major incidence lists: for every vertex u, the slots holding u in
// canonical edge order (a vertex occurs once per edge).  Counting sort by
// vertex over the canonical edges, in chunks of consecutive edges: per-chunk
// counts, per-vertex offsets chunk by chunk, then each chunk scatters its
// slots in edge order -- the lists a sequential pass would make.
static void build_node_major(Plan& P, int32_t n) {
  const int64_t m = P.m;
  const int T = std::min(8, chunk_count(m, 1 << 16));
  std::vector<int64_t> cut(T + 1);
  for (int t = 0; t <= T; ++t) cut[t] = m * t / T;
  // first bucket of every chunk (buckets are in canonical edge order)
  auto bucket_of = [&](int64_t cidx) {
    size_t lo = 0, hi = P.buckets.size();
    while (hi - lo > 1) {
      const size_t mid = (lo + hi) / 2;
      if (P.buckets[mid].edge_off <= cidx) lo = mid; else hi = mid;
    }
    return lo;
  };
  auto each_slot = [&](int64_t c0, int64_t c1, auto&& f) {
    size_t b = bucket_of(c0);
    for (int64_t cidx = c0; cidx < c1; ++cidx) {
      while (cidx >= P.buckets[b].edge_off + P.buckets[b].m) ++b;
      const Bucket& B = P.buckets[b];
      const int64_t i = cidx - B.edge_off;
      for (int j = 0; j < B.k; ++j) f(B.slot_off + (int64_t)j * B.m + i);
    }
  };
  std::vector<std::vector<int32_t>> cnt(T, std::vector<int32_t>(T > 1 ? (size_t)n : 0, 0));
  if (T == 1) {
    std::vector<int64_t> cur(P.tptr.begin(), P.tptr.end() - 1);
    each_slot(0, m, [&](int64_t s) { P.tslot[cur[P.mem[s]]++] = static_cast<int32_t>(s); });
    return;
  }
  {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] { each_slot(cut[t], cut[t + 1], [&](int64_t s) { cnt[t][P.mem[s]]++; }); });
    for (auto& x : th) x.join();
  }
  parallel_chunks(n, [&](int, int64_t u0, int64_t u1) {
    for (int64_t u = u0; u < u1; ++u) {
      int64_t run = P.tptr[u];
      for (int t = 0; t < T; ++t) {
        const int32_t c = cnt[t][u];
        cnt[t][u] = static_cast<int32_t>(run - P.tptr[u]);   // offset inside u's list
        run += c;
      }
    }
  });
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      each_slot(cut[t], cut[t + 1], [&](int64_t s) {
        const int32_t u = P.mem[s];
        P.tslot[P.tptr[u] + cnt[t][u]++] = static_cast<int32_t>(s);
      });
    });
  for (auto& x : th) x.join();
}

int build_plan(int G, const GraphIn* gs, const sttsv_opts* opts, Plan** out) {
  if (G < 1 || gs == nullptr || out == nullptr) return STTSV_EINVAL;
  if (opts != nullptr && opts->precision != STTSV_PREC_FP64 && opts->precision != STTSV_PREC_FP32)
    return STTSV_EINVAL;
  // ---- validation, sizes
  std::vector<std::vector<int64_t>> degs(G);
  int64_t m = 0, nnz = 0, n64 = 0;
  int32_t rmax = 0;
  for (int g = 0; g < G; ++g) {
    const int rc = validate_graph(gs[g], degs[g]);
    if (rc != STTSV_OK) return rc;
    m += gs[g].m;
    nnz += gs[g].eptr[gs[g].m];
    n64 += gs[g].n;
    rmax = std::max(rmax, gs[g].r);
  }
  if (nnz > INT32_MAX || n64 > INT32_MAX || m > INT32_MAX) return STTSV_ENOTSUP;
  const int32_t n = static_cast<int32_t>(n64);

  Plan* P = new Plan();
  P->m = m;
  P->nnz = nnz;
  P->n = n;
  P->r = rmax;
  P->precision = opts ? opts->precision : STTSV_PREC_FP64;
  P->flags = opts ? opts->flags : 0;
  P->stream = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
  (void)hipGetDevice(&P->device);
  P->graphs.resize(G);
  {
    int32_t voff = 0;
    int64_t eoff = 0;
    for (int g = 0; g < G; ++g) {
      GraphInfo& I = P->graphs[g];
      I.m = gs[g].m;
      I.nnz = gs[g].eptr[gs[g].m];
      I.n = gs[g].n;
      I.r = gs[g].r;
      I.voff = voff;
      I.eoff = eoff;
      voff += gs[g].n;
      eoff += gs[g].m;
    }
  }

  // ---- buckets keyed by (r, k, lanes per edge); every graph's edges of
  // size k form a contiguous run of one bucket, in the graph's own canonical
  // order.  The lanes per edge (one, or a lane group) follow from the graph's
  // own edge count of that size, so each graph's results are those of its
  // single-graph plan, whatever else is in the batch.
  constexpr int kModes = 5;                       // lanes per edge: 1 (mode 0), 8, 16, 32, 64
  auto mode_of = [](int L) { return L == 0 ? 0 : L == 8 ? 1 : L == 16 ? 2 : L == 32 ? 3 : 4; };
  const int mode_lanes[kModes] = {0, 8, 16, 32, 64};
  std::vector<std::vector<std::vector<int64_t>>> cnt(
      rmax + 1, std::vector<std::vector<int64_t>>(rmax + 1, std::vector<int64_t>(kModes, 0)));
  std::vector<std::vector<int64_t>> goff(G, std::vector<int64_t>(rmax + 1, 0));
  std::vector<std::vector<int>> gmode(G, std::vector<int>(rmax + 1, 0));
  for (int g = 0; g < G; ++g) {
    std::vector<int64_t> mk(gs[g].r + 1, 0);
    for (int64_t e = 0; e < gs[g].m; ++e) mk[gs[g].eptr[e + 1] - gs[g].eptr[e]]++;
    std::vector<int64_t> rwaves(kGenRanges, 0);   // one-lane waves of the graph's sizes >= 4 per window range
    for (int k = 4; k <= gs[g].r; ++k)
      if (mk[k] > 0) rwaves[gen_range_of(gs[g].r - k + 1)] += (mk[k] + 63) / 64;
    for (int k = 1; k <= gs[g].r; ++k) {
      const int md = k >= 4 && mk[k] > 0 ? mode_of(coop_lanes(gs[g].r, k, rwaves[gen_range_of(gs[g].r - k + 1)])) : 0;
      gmode[g][k] = md;
      goff[g][k] = cnt[gs[g].r][k][md];
      cnt[gs[g].r][k][md] += mk[k];
    }
  }
  std::vector<std::vector<std::vector<int>>> bidx(rmax + 1,
                                                  std::vector<std::vector<int>>(rmax + 1, std::vector<int>(kModes, -1)));
  {
    int64_t edge_off = 0, slot_off = 0;
    for (int r = 2; r <= rmax; ++r)
      for (int k = 1; k <= r; ++k)
        for (int md = 0; md < kModes; ++md) {
          if (cnt[r][k][md] == 0) continue;
          Bucket B;
          B.r = r;
          B.k = k;
          B.m = cnt[r][k][md];
          B.edge_off = edge_off;
          B.slot_off = slot_off;
          B.lanes_per_edge = mode_lanes[md];
          if (k > 1) B.fp32_ok = fp32_scale(r, k, &B.qexp32);
          bidx[r][k][md] = static_cast<int>(P->buckets.size());
          P->buckets.push_back(B);
          edge_off += B.m;
          slot_off += (int64_t)k * B.m;
        }
  }

  // ---- member slots, canonical permutation, graph ids, node-major lists
  P->perm.assign(m, 0);
  P->mem.assign(nnz, 0);
  P->tptr.assign((size_t)n + 1, 0);
  for (int g = 0; g < G; ++g)
    for (int32_t v = 0; v < gs[g].n; ++v) {
      const int64_t u = (int64_t)P->graphs[g].voff + v;
      P->tptr[u + 1] = P->tptr[u] + degs[g][v];
    }
  P->tslot.assign(nnz, 0);
  std::vector<int32_t> memr(nnz, 0), rid(n, 0);
  std::vector<int32_t> gid;
  if (G > 1) gid.assign(m, 0);
  bool weighted = false;
  for (int g = 0; g < G; ++g) weighted = weighted || gs[g].w != nullptr;
  std::vector<double> wgt;
  std::vector<std::vector<long double>> utab(rmax + 1);
  std::vector<std::vector<double>> dtab(rmax + 1);
  if (weighted) wgt.assign(m, 0.0);
  if (weighted)
    for (int g = 0; g < G; ++g) {
      if (gs[g].w == nullptr && dtab[gs[g].r].empty()) dtab[gs[g].r] = weight_table(gs[g].r);
      if (gs[g].w != nullptr && utab[gs[g].r].empty()) utab[gs[g].r] = unit_weight_table(gs[g].r);
    }
  {
    // graphs of a batch in parallel (each writes its own edges, slots and
    // vertices); inside a graph the loops are parallel again
    auto one_graph = [&](int g) {
      const GraphIn& in = gs[g];
      const GraphInfo& I = P->graphs[g];
      Canon c;
      canonicalise(in, degs[g], c);
      for (int32_t q = 0; q < in.n; ++q) rid[I.voff + q] = I.voff + c.inv_rank[q];
      for (int k = 1; k <= in.r; ++k) {
        const auto& ids = c.order[k];
        if (ids.empty()) continue;
        const Bucket& B = P->buckets[bidx[in.r][k][gmode[g][k]]];
        const int64_t base = goff[g][k];
        parallel_chunks(static_cast<int64_t>(ids.size()), [&](int, int64_t t0, int64_t t1) {
          for (int64_t t = t0; t < t1; ++t) {
            const int64_t e = ids[t];
            const int64_t i = base + t;                           // edge index in the bucket
            P->perm[B.edge_off + i] = I.eoff + e;
            if (G > 1) gid[B.edge_off + i] = g;
            if (weighted)
              wgt[B.edge_off + i] = in.w == nullptr ? dtab[in.r][k]
                                                    : static_cast<double>((long double)in.w[e] * utab[in.r][k]);
            const int32_t* a = c.rk.data() + in.eptr[e];
            for (int j = 0; j < k; ++j) {
              const int64_t s = B.slot_off + (int64_t)j * B.m + i;
              P->mem[s] = I.voff + c.inv_rank[a[j]];
              memr[s] = I.voff + a[j];
            }
          }
        });
      }
      P->graphs[g].connected = connected_graph(in, degs[g]);
      P->graphs[g].norm2 = blowup_norm2(in, c);
    };
    if (G == 1) {
      one_graph(0);
    } else {
      parallel_chunks(G, [&](int, int64_t g0, int64_t g1) {
        for (int64_t g = g0; g < g1; ++g) one_graph(static_cast<int>(g));
      }, 1);
    }
    build_node_major(*P, n);
  }
  P->connected = true;
  for (const GraphInfo& I : P->graphs) P->connected = P->connected && I.connected;
  P->weights = weight_table(gs[0].r);
  std::vector<int64_t> deg(n);
  for (int g = 0; g < G; ++g)
    for (int32_t v = 0; v < gs[g].n; ++v) deg[(int64_t)P->graphs[g].voff + v] = degs[g][v];
  degs.clear();

  // ---- vertex blocks (layout item 8; places are assigned once the kernels are chosen)
  std::vector<int32_t>& vblock = P->vblock;
  vblock.assign(n, 0);
  {
    int64_t acc = 0;
    int32_t b = 0;
    P->region.assign(1, 0);
    int64_t nv = 0;                   // vertices in the current block
    int64_t cnt[4] = {0, 0, 0, 0};    // its level-0 chunks per lane class
    int g = 0;
    for (int32_t u = 0; u < n; ++u) {
      int64_t with[4] = {cnt[0], cnt[1], cnt[2], cnt[3]};
      add_chunks(deg[u], with);
      // a block holds one graph's vertices only: its level-0 workgroups can
      // then read the contribution format of that graph's solver phase
      bool new_graph = false;
      while (g + 1 < G && u >= P->graphs[g + 1].voff) {
        ++g;
        new_graph = true;
      }
      if (nv > 0 && (new_graph || acc + deg[u] > kStageTerms || stage_passes(with) > kStagePasses)) {
        P->region.push_back(P->region.back() + acc);
        ++b;
        acc = 0;
        nv = 0;
        for (int q = 0; q < 4; ++q) with[q] = 0;
        add_chunks(deg[u], with);
      }
      vblock[u] = b;
      acc += deg[u];
      ++nv;
      for (int q = 0; q < 4; ++q) cnt[q] = with[q];
    }
    P->region.push_back(nnz);
    // graph of every block (blocks never straddle graphs)
    P->block_graph.assign(P->region.size() - 1, 0);
    for (int gi = 0; gi < G; ++gi)
      for (int32_t v = 0; v < P->graphs[gi].n; ++v) P->block_graph[vblock[P->graphs[gi].voff + v]] = gi;
  }

  // ---- reduction schedule
  std::vector<HostLevel> hl;
  {
    // level 0 input: contributions gathered through tslot; segment of v = [tptr[v], tptr[v+1])
    std::vector<int64_t> seg_start(n), seg_len(n);
    std::vector<int32_t> seg_node(n);
    for (int32_t v = 0; v < n; ++v) {
      seg_start[v] = P->tptr[v];
      seg_len[v] = deg[v];
      seg_node[v] = v;
    }
    int64_t in_len = nnz;
    bool first = true;
    while (!seg_node.empty()) {
      HostLevel L;
      L.in_len = in_len;
      std::vector<int64_t> nstart, nlen;
      std::vector<int32_t> nnode;
      int64_t next_len = 0;
      std::vector<int32_t> cblock;   // level 0: vertex block of every chunk
      for (size_t q = 0; q < seg_node.size(); ++q) {
        const int64_t d = seg_len[q];
        const int64_t nch = d <= kChunk ? 1 : (d + kChunk - 1) / kChunk;
        if (first) cblock.insert(cblock.end(), nch, vblock[seg_node[q]]);
        if (nch == 1) {
          L.start.push_back(static_cast<int32_t>(d > 0 ? seg_start[q] : 0));
          L.len.push_back(static_cast<int32_t>(d));
          L.dst.push_back(seg_node[q]);
        } else {
          for (int64_t c = 0; c < nch; ++c) {
            L.start.push_back(static_cast<int32_t>(seg_start[q] + c * kChunk));
            L.len.push_back(static_cast<int32_t>(std::min<int64_t>(kChunk, d - c * kChunk)));
            L.dst.push_back(static_cast<int32_t>(-(next_len + c) - 1));
          }
          nstart.push_back(next_len);
          nlen.push_back(nch);
          nnode.push_back(seg_node[q]);
          next_len += nch;
        }
      }
      if (first) {
        L = level0_schedule(*P, L, cblock);
        first = false;
      }
      hl.push_back(std::move(L));
      seg_start = std::move(nstart);
      seg_len = std::move(nlen);
      seg_node = std::move(nnode);
      in_len = next_len;
    }
  }

  // ---- device uploads
  int rc = STTSV_OK;
  auto fail = [&](int code) {
    free_plan(P);
    return code;
  };
  if ((rc = upload(&P->d_mem, memr.data(), nnz, &P->device_bytes)) != STTSV_OK) return fail(rc);
  memr.clear();
  memr.shrink_to_fit();
  if ((rc = upload(&P->d_rid, rid.data(), n, &P->device_bytes)) != STTSV_OK) return fail(rc);
  std::vector<int32_t> rpos(n);   // degree-rank position of every vertex
  for (int32_t q = 0; q < n; ++q) rpos[rid[q]] = q;
  if ((rc = upload<double>(&P->d_xr, nullptr, n, &P->device_bytes)) != STTSV_OK) return fail(rc);
  if ((rc = upload<float>(&P->d_xr32, nullptr, n, &P->device_bytes)) != STTSV_OK) return fail(rc);
  if ((rc = upload<uint32_t>(&P->d_contrib32, nullptr, nnz, &P->device_bytes)) != STTSV_OK) return fail(rc);
  if ((rc = upload<int32_t>(&P->d_loc, nullptr, nnz, &P->device_bytes)) != STTSV_OK) return fail(rc);
  if ((rc = upload<double>(&P->d_contrib, nullptr, nnz, &P->device_bytes)) != STTSV_OK) return fail(rc);
  if (G > 1 && (rc = upload(&P->d_gid, gid.data(), gid.size(), &P->device_bytes)) != STTSV_OK) return fail(rc);
  if (weighted && (rc = upload(&P->d_wgt, wgt.data(), wgt.size(), &P->device_bytes)) != STTSV_OK) return fail(rc);
  for (size_t l = 0; l < hl.size(); ++l) {
    ReduceLevel L;
    L.nchunks = (int64_t)hl[l].len.size();
    L.in_len = hl[l].in_len;
    P->levels.push_back(L);
    ReduceLevel& D = P->levels.back();
    if (l > 0) {
      std::vector<int4> desc(D.nchunks);
      for (int64_t c = 0; c < D.nchunks; ++c) {
        const int32_t d = hl[l].dst[c];
        desc[c] = make_int4(hl[l].start[c], hl[l].len[c], d, d >= 0 ? rpos[d] : d);
      }
      if ((rc = upload(&D.d_desc, desc.data(), D.nchunks, &P->device_bytes)) != STTSV_OK) return fail(rc);
    } else {
      // packed level-0 descriptors: LDS offset within the workgroup's terms | length << 16
      std::vector<int2> dv(D.nchunks), dr(D.nchunks);
      for (size_t w = 0; w < P->l0_wg.size(); ++w) {
        const int4 a = P->l0_wg[w];
        const int64_t nch = (int64_t)a.y + a.z + a.w + P->l0_n1[w];
        for (int64_t c = a.x; c < a.x + nch; ++c) {
          const int64_t off = hl[0].len[c] > 0 ? hl[0].start[c] - P->l0_base[w] : 0;
          if (off < 0 || off + hl[0].len[c] > P->l0_terms[w]) return fail(STTSV_EINVAL);
          const int32_t x = static_cast<int32_t>(off | ((int64_t)hl[0].len[c] << 16));
          const int32_t d = hl[0].dst[c];
          dv[c] = make_int2(x, d);
          dr[c] = make_int2(x, d >= 0 ? rpos[d] : d);
        }
      }
      if ((rc = upload(&D.d_desc0[0], dv.data(), D.nchunks, &P->device_bytes)) != STTSV_OK ||
          (rc = upload(&D.d_desc0[1], dr.data(), D.nchunks, &P->device_bytes)) != STTSV_OK)
        return fail(rc);
    }
    if (l == 0 && !P->l0_wg.empty()) {
      D.nwg = static_cast<int64_t>(P->l0_wg.size());
      if ((rc = upload<int4>(&D.d_wg, nullptr, 2 * D.nwg, &P->device_bytes)) != STTSV_OK ||
          (rc = upload<int2>(&D.d_ranges, nullptr, kStageRuns * D.nwg, &P->device_bytes)) != STTSV_OK ||
          (rc = upload<uint16_t>(&D.d_lpos, nullptr, nnz, &P->device_bytes)) != STTSV_OK)
        return fail(rc);
    }
    if (l + 1 < hl.size()) {
      double* part = nullptr;
      if ((rc = upload<double>(&part, nullptr, hl[l + 1].in_len, &P->device_bytes)) != STTSV_OK) return fail(rc);
      P->d_partials.push_back(part);
    }
  }
  // ---- kernel selection, bucket descriptors, fused generic groups
  const EdgeTables& tab = edge_tables();
  std::vector<std::vector<double>> wtab(rmax + 1);
  for (Bucket& B : P->buckets) {
    const int r = B.r;
    const int W = r - B.k + 1;
    if (wtab[r].empty()) wtab[r] = weight_table(r);
    for (int t = 0; t < 2; ++t) {
      BucketDesc& d = B.desc[t];
      d.mem = P->d_mem + B.slot_off;
      d.loc = P->d_loc + B.slot_off;
      d.gid = P->d_gid != nullptr ? P->d_gid + B.edge_off : nullptr;
      d.gstack = nullptr;
      d.m = B.m;
      d.k = B.k;
      d.r = r;
      d.W = W;
      d.qexp = t == 1 ? B.qexp32 : 0;
      d.lds_stack = 1;
      d.reuse_emin = reuse_emin(W);
      d.wk = wtab[r][B.k];
      d.wgt = P->d_wgt != nullptr ? P->d_wgt + B.edge_off : nullptr;
      d.run_start = nullptr;
      d.nruns = 0;
      for (int q = 0; q < kRunMax; ++q) d.run_cnt[q] = 0;
      const auto& small = t == 0 ? tab.small64 : tab.small32;
      const auto& coop = t == 0 ? tab.coop64 : tab.coop32;
      B.coop[t] = B.lanes_per_edge > 0 && W <= (t == 0 ? kCoopMaxW64 : kCoopMaxW32) && coop[gen_range_of(W)] != nullptr
                      ? B.lanes_per_edge : 0;
      d.lanes = B.coop[t];
      int kind = -1;
      if (B.k == 2) kind = SK_K2;
      if (B.k == 3) kind = SK_K3;
      if (B.k >= 4 && B.k <= 7 && !(P->flags & STTSV_FLAG_GENERIC_ONLY) && small[SK_R4 + (B.k - 4)][W] != nullptr &&
          kr_default(B.k, W, t == 0 ? 8 : 4))
        kind = SK_R4 + (B.k - 4);
      B.small_kind[t] = kind;
    }
  }
  for (Bucket& B : P->buckets)
    if ((rc = set_reuse(*P, B, (P->flags & STTSV_FLAG_PREFIX_REUSE) != 0)) != STTSV_OK) return fail(rc);
  if ((rc = build_groups(*P)) != STTSV_OK) return fail(rc);
  if ((rc = assign_places(*P)) != STTSV_OK) return fail(rc);
  build_stages(*P);
  if (!(P->flags & STTSV_FLAG_ONE_STREAM) && (rc = init_lanes(*P)) != STTSV_OK) return fail(rc);
  if (hipDeviceSynchronize() != hipSuccess) return fail(STTSV_EHIP);
  *out = P;
  return STTSV_OK;
}

}  // namespace sttsv
