// The Compound CSS forest (Sec. III) built on the device, and Alg. 4's
// memoised STTSV over it (Sec. IV-B).
//
// Forest: for every member slot (edge e, member u) of an edge of size k >= 2
// the path e \ {u}, its members in degree-rank order (the plan's member
// order; the paper lists them by vertex index, any order gives the same
// tensor), is a root-to-level-(k-1) path; the slot is a special leaf of the
// node that ends it.  The forest is the trie of all paths.  Level d is built
// from level d-1 by one radix sort of the keys (parent node, d-th vertex) of
// the paths still longer than d, a head flag where the key changes, and a
// prefix sum that numbers the distinct keys: nodes of a level come out in
// (parent, vertex) order, and the paths that end at level d, sorted by their
// node, are that level's special leaves.
//
// STTSV (FP64): level by level, a node's workspace is its parent's times
// phi(z_v t) -- in the phi basis, prod over the path of Ebar(x_i t) equals
// (prod x_i) t^d prod phi(x_i t), so a depth-d node keeps the W = r - d
// coefficients its own leaves need (its children need one fewer) -- one
// truncated product per forest edge, never repeated for another edge or
// another edge size sharing the prefix.  Each node keeps its workspace and
// the product Z of its path's z on its path's own power-of-two scale
// 2^E (E = max exponent of |x| on the path), rescaled exactly when a child or
// a leaf has a larger x.  A special leaf (e, u) at depth k - 1 adds
//     w(e)/|beta(e)| (r-1)! 2^(E (r-1)) Z sum_a z_u^a / a! Phi[W-1-a]
// (the coefficient of t^(r-1) in e^(x_u t) times its path's product).  The
// leaf values go to the plan's contribution places and the plan's
// deterministic node reduction sums them.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <vector>

#include "edge_kernels.inc"

namespace sttsv {

struct CcssForest {
  int levels = 0;
  int r = 0;
  std::vector<int64_t> n_at;         // nodes per level (level d = depth d + 1)
  std::vector<int32_t*> vert;        // device, per level: degree-rank position of the node's vertex
  std::vector<int32_t*> parent;      // device, per level: parent index in the level above (-1 at depth 1)
  std::vector<int32_t*> leaf_slots;  // device, per level: slots whose path ends there, in node order
  std::vector<int64_t> n_leaf;
  int32_t* leaf_node = nullptr;      // device, per slot: owning node (-1 for size-1 edges)
  double* buf[2] = {nullptr, nullptr};   // workspaces of two consecutive levels (W doubles per node)
  int32_t* ebuf[2] = {nullptr, nullptr}; // scale exponents
  double* zbuf[2] = {nullptr, nullptr};  // products of the path's z
  int64_t device_bytes = 0;
  double build_ms = 0.0;
};

namespace {

constexpr int kCcssBlock = 256;

// per-slot geometry: first member slot of its edge, stride (bucket edges),
// member position and edge size
struct SlotGeo {
  int32_t base;
  int32_t m;
  int32_t j;
  int32_t k;
};

__global__ void slot_geo(SlotGeo* geo, int32_t* act, int64_t slot_off, int64_t m, int k, int64_t act_off) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * k) return;
  const int64_t s = slot_off + t;
  geo[s] = SlotGeo{static_cast<int32_t>(slot_off + t % m), static_cast<int32_t>(m), static_cast<int32_t>(t / m), k};
  act[act_off + t] = static_cast<int32_t>(s);
}

// key of every active path at level d: (node at level d-1) * n + its d-th member
__global__ void level_keys(const int32_t* __restrict__ act, int64_t A, const SlotGeo* __restrict__ geo,
                           const int32_t* __restrict__ mem, const int32_t* __restrict__ node_of, int d, int64_t n,
                           uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A) return;
  const int32_t s = act[t];
  const SlotGeo g = geo[s];
  const int idx = d < g.j ? d : d + 1;                     // member d of e \ {u}
  const int64_t e = mem[g.base + (int64_t)idx * g.m];
  const int64_t par = d > 0 ? node_of[s] : 0;
  keys[t] = static_cast<uint64_t>(par * n + e);
  vals[t] = s;
}

__global__ void head_flags(const uint64_t* __restrict__ keys, int64_t A, int32_t* __restrict__ flag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A) return;
  flag[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

// number nodes, record each node's vertex and parent, each path's node; mark
// the paths that end at this level
__global__ void level_nodes(const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                            const int32_t* __restrict__ flag, const int32_t* __restrict__ id, int64_t A, int d,
                            int64_t n, const SlotGeo* __restrict__ geo, int32_t* __restrict__ node_of,
                            int32_t* __restrict__ vert, int32_t* __restrict__ parent, int32_t* __restrict__ leaf_node,
                            uint8_t* __restrict__ fin, uint8_t* __restrict__ cont) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= A) return;
  const int32_t s = vals[t];
  const int32_t q = id[t] - 1;
  node_of[s] = q;
  if (flag[t]) {
    vert[q] = static_cast<int32_t>(keys[t] % static_cast<uint64_t>(n));
    parent[q] = d > 0 ? static_cast<int32_t>(keys[t] / static_cast<uint64_t>(n)) : -1;
  }
  const bool ends = geo[s].k - 1 == d + 1;
  if (ends) leaf_node[s] = q;
  fin[t] = ends ? 1 : 0;
  cont[t] = ends ? 0 : 1;
}

__global__ void fill_i32(int32_t* p, int64_t count, int32_t v) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

unsigned grid_of(int64_t count) { return static_cast<unsigned>((count + kCcssBlock - 1) / kCcssBlock); }

// ---------------------------------------------------------------- STTSV over the forest
// Node of depth `depth`: W = r - depth coefficients; the parent keeps W + 1.
template <int W>
__global__ void __launch_bounds__(kCcssBlock) node_step(const double* __restrict__ xr, const int32_t* __restrict__ vert,
                                                        const int32_t* __restrict__ parent, int64_t N, int depth,
                                                        const double* __restrict__ pbuf, const int32_t* __restrict__ pexp,
                                                        const double* __restrict__ pz, double* __restrict__ cbuf,
                                                        int32_t* __restrict__ cexp, double* __restrict__ cz) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= N) return;
  const double xv = xr[vert[q]];
  int ev = 0;
  (void)frexp(fabs(xv), &ev);
  double L[W];
  int E = ev;
  double Z = 1.0;
  if (depth == 1) {
#pragma unroll
    for (int c = 0; c < W; ++c) L[c] = c == 0 ? 1.0 : 0.0;
  } else {
    const int64_t p = parent[q];
    const int Ep = pexp[p];
    E = Ep > ev ? Ep : ev;
    const int sh = Ep - E;                                   // <= 0: exact power-of-two rescale
#pragma unroll
    for (int c = 0; c < W; ++c) L[c] = ldexp(pbuf[p * (W + 1) + c], sh * c);
    Z = ldexp(pz[p], sh * (depth - 1));
  }
  const double z = ldexp(xv, -E);
  double f[W];
  phi_series<double, W>(z, f);
  series_mul<double, W>(L, f);
#pragma unroll
  for (int c = 0; c < W; ++c) cbuf[q * W + c] = L[c];
  cexp[q] = E;
  cz[q] = Z * z;
}

// Special leaves of edges of size k (depth k - 1, W = r - k + 1) of bucket b.
template <int W>
__global__ void __launch_bounds__(kCcssBlock) leaf_step(EdgeCall c, BucketDesc b, const int32_t* __restrict__ slots,
                                                        int64_t NL, int64_t slot_off,
                                                        const int32_t* __restrict__ leaf_node,
                                                        const double* __restrict__ cbuf, const int32_t* __restrict__ cexp,
                                                        const double* __restrict__ cz) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= NL) return;
  const int64_t s = slots[t];
  const int64_t rel = s - slot_off;
  const int64_t i = rel % b.m;                              // edge in the bucket
  const int j = static_cast<int>(rel / b.m);                 // member
  const int64_t q = leaf_node[s];
  const double xu = c.x[b.mem[rel]];
  int eu = 0;
  (void)frexp(fabs(xu), &eu);
  const int Eq = cexp[q];
  const int E = Eq > eu ? Eq : eu;
  const int sh = Eq - E;
  const double zu = ldexp(xu, -E);
  // sum_a z_u^a / a! Phi[W-1-a], all terms >= 0 for x >= 0
  double acc = 0.0, pw = 1.0;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    acc = fma(pw, ldexp(cbuf[q * W + (W - 1 - a)], sh * (W - 1 - a)), acc);
    pw = pw * (zu * (1.0 / double(a + 1)));
  }
  const double Z = ldexp(cz[q], sh * (b.k - 1));
  const double coef = ldexp(b.wgt != nullptr ? b.wgt[i] : b.wk, (b.r - 1) * E);
  c.contrib[b.loc[(int64_t)j * b.m + i]] = coef * (Z * acc);
}

using NodeLaunch = hipError_t (*)(const double*, const int32_t*, const int32_t*, int64_t, int, const double*,
                                  const int32_t*, const double*, double*, int32_t*, double*, hipStream_t);
using LeafLaunch = hipError_t (*)(const EdgeCall&, const BucketDesc&, const int32_t*, int64_t, int64_t, const int32_t*,
                                  const double*, const int32_t*, const double*, hipStream_t);

template <int W>
hipError_t launch_node(const double* xr, const int32_t* vert, const int32_t* parent, int64_t N, int depth,
                       const double* pbuf, const int32_t* pexp, const double* pz, double* cbuf, int32_t* cexp,
                       double* cz, hipStream_t s) {
  hipLaunchKernelGGL((node_step<W>), dim3(grid_of(N)), dim3(kCcssBlock), 0, s, xr, vert, parent, N, depth, pbuf, pexp,
                     pz, cbuf, cexp, cz);
  return hipGetLastError();
}

template <int W>
hipError_t launch_leaf(const EdgeCall& c, const BucketDesc& b, const int32_t* slots, int64_t NL, int64_t slot_off,
                       const int32_t* leaf_node, const double* cbuf, const int32_t* cexp, const double* cz,
                       hipStream_t s) {
  hipLaunchKernelGGL((leaf_step<W>), dim3(grid_of(NL)), dim3(kCcssBlock), 0, s, c, b, slots, NL, slot_off, leaf_node,
                     cbuf, cexp, cz);
  return hipGetLastError();
}

struct CcssTables {
  NodeLaunch node[kMaxW + 1];
  LeafLaunch leaf[kMaxW + 1];
};

template <int W>
void fill_ccss(CcssTables& t) {
  if constexpr (W >= 1) {
    t.node[W] = &launch_node<W>;
    t.leaf[W] = &launch_leaf<W>;
    fill_ccss<W - 1>(t);
  }
}

const CcssTables& ccss_tables() {
  static const CcssTables t = [] {
    CcssTables x{};
    fill_ccss<kMaxW - 1>(x);
    return x;
  }();
  return t;
}

template <typename T>
bool dalloc(T** p, size_t count, int64_t* acct) {
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) return false;
  *acct += (int64_t)(count * sizeof(T));
  return true;
}

}  // namespace

void free_ccss(Plan& p) {
  CcssForest* f = p.ccss;
  if (f == nullptr) return;
  (void)hipStreamSynchronize(p.stream);
  for (auto* q : f->vert) (void)hipFree(q);
  for (auto* q : f->parent) (void)hipFree(q);
  for (auto* q : f->leaf_slots) (void)hipFree(q);
  (void)hipFree(f->leaf_node);
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(f->buf[i]);
    (void)hipFree(f->ebuf[i]);
    (void)hipFree(f->zbuf[i]);
  }
  delete f;
  p.ccss = nullptr;
}

int build_ccss(Plan& p, sttsv_ccss_info* info) {
  if (p.graphs.size() != 1) return STTSV_ENOTSUP;   // one hypergraph: windows follow its order r
  free_ccss(p);
  const auto t0 = std::chrono::steady_clock::now();
  auto* f = new CcssForest();
  p.ccss = f;
  f->r = p.r;
  hipStream_t s = p.stream;
  const int64_t nnz = p.nnz;
  int64_t scratch_bytes = 0;
  // paths: every slot of an edge of size >= 2
  int64_t A = 0;
  int kmax = 1;
  for (const Bucket& B : p.buckets)
    if (B.k >= 2) {
      A += B.m * B.k;
      kmax = std::max(kmax, B.k);
    }
  SlotGeo* geo = nullptr;
  int32_t *act = nullptr, *vals = nullptr, *vals2 = nullptr, *flag = nullptr, *id = nullptr, *node_of = nullptr;
  uint64_t *keys = nullptr, *keys2 = nullptr;
  uint8_t *fin = nullptr, *cont = nullptr;
  int32_t* nsel = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int rc = STTSV_OK;
  auto cleanup = [&]() {
    for (void* q : {(void*)geo, (void*)act, (void*)vals, (void*)vals2, (void*)flag, (void*)id, (void*)node_of,
                    (void*)keys, (void*)keys2, (void*)fin, (void*)cont, (void*)nsel, tmp})
      (void)hipFree(q);
  };
  if (!dalloc(&geo, nnz, &scratch_bytes) || !dalloc(&act, A, &scratch_bytes) || !dalloc(&vals, A, &scratch_bytes) ||
      !dalloc(&vals2, A, &scratch_bytes) || !dalloc(&flag, A, &scratch_bytes) || !dalloc(&id, A, &scratch_bytes) ||
      !dalloc(&node_of, nnz, &scratch_bytes) || !dalloc(&keys, A, &scratch_bytes) ||
      !dalloc(&keys2, A, &scratch_bytes) || !dalloc(&fin, A, &scratch_bytes) || !dalloc(&cont, A, &scratch_bytes) ||
      !dalloc(&nsel, 2, &scratch_bytes) || !dalloc(&f->leaf_node, nnz, &f->device_bytes)) {
    cleanup();
    free_ccss(p);
    return STTSV_ENOMEM;
  }
  // temporary storage of the library sort, scan and selection (largest of the three)
  {
    size_t a = 0, b = 0, c = 0;
    int bits = 1;
    while (bits < 63 && ((uint64_t)1 << bits) <= (uint64_t)(nnz + 1) * (uint64_t)p.n) ++bits;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, keys, keys2, vals, vals2, static_cast<int>(A), 0, bits, s);
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, b, flag, id, static_cast<int>(A), s);
    (void)hipcub::DeviceSelect::Flagged(nullptr, c, vals2, fin, vals, nsel, static_cast<int>(A), s);
    tmp_bytes = std::max(a, std::max(b, c));
    if (hipMalloc(&tmp, tmp_bytes) != hipSuccess) {
      cleanup();
      free_ccss(p);
      return STTSV_ENOMEM;
    }
  }
  hipLaunchKernelGGL(fill_i32, dim3(grid_of(nnz)), dim3(kCcssBlock), 0, s, f->leaf_node, nnz, -1);
  {
    int64_t off = 0;
    for (const Bucket& B : p.buckets) {
      if (B.k < 2) continue;
      hipLaunchKernelGGL(slot_geo, dim3(grid_of(B.m * B.k)), dim3(kCcssBlock), 0, s, geo, act, B.slot_off, B.m,
                         B.k, off);
      off += B.m * B.k;
    }
  }
  int bits = 1;
  while (bits < 63 && ((uint64_t)1 << bits) <= (uint64_t)(nnz + 1) * (uint64_t)p.n) ++bits;
  int64_t max_work = 0;   // largest level workspace (doubles)
  for (int d = 0; A > 0 && rc == STTSV_OK; ++d) {
    const unsigned g = grid_of(A);
    hipLaunchKernelGGL(level_keys, dim3(g), dim3(kCcssBlock), 0, s, act, A, geo, p.d_mem, node_of, d, (int64_t)p.n,
                       keys, vals);
    size_t tb = tmp_bytes;
    if (hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys2, vals, vals2, static_cast<int>(A), 0, bits, s) !=
        hipSuccess) {
      rc = STTSV_EHIP;
      break;
    }
    hipLaunchKernelGGL(head_flags, dim3(g), dim3(kCcssBlock), 0, s, keys2, A, flag);
    tb = tmp_bytes;
    if (hipcub::DeviceScan::InclusiveSum(tmp, tb, flag, id, static_cast<int>(A), s) != hipSuccess) {
      rc = STTSV_EHIP;
      break;
    }
    int32_t N = 0;
    if (hipMemcpyAsync(&N, id + (A - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = STTSV_EHIP;
      break;
    }
    int32_t *vt = nullptr, *pa = nullptr, *ls = nullptr;
    if (!dalloc(&vt, N, &f->device_bytes) || !dalloc(&pa, N, &f->device_bytes)) {
      (void)hipFree(vt);
      rc = STTSV_ENOMEM;
      break;
    }
    f->vert.push_back(vt);
    f->parent.push_back(pa);
    f->n_at.push_back(N);
    max_work = std::max(max_work, (int64_t)N * (p.r - (d + 1)));
    hipLaunchKernelGGL(level_nodes, dim3(g), dim3(kCcssBlock), 0, s, keys2, vals2, flag, id, A, d, (int64_t)p.n,
                       geo, node_of, vt, pa, f->leaf_node, fin, cont);
    // this level's leaves (in node order) and the paths that go on
    tb = tmp_bytes;
    int32_t cnt[2] = {0, 0};
    if (hipcub::DeviceSelect::Flagged(tmp, tb, vals2, fin, vals, nsel, static_cast<int>(A), s) != hipSuccess ||
        hipMemcpyAsync(&cnt[0], nsel, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = STTSV_EHIP;
      break;
    }
    if (!dalloc(&ls, cnt[0], &f->device_bytes)) {
      rc = STTSV_ENOMEM;
      break;
    }
    if (cnt[0] > 0 && hipMemcpyAsync(ls, vals, sizeof(int32_t) * cnt[0], hipMemcpyDeviceToDevice, s) != hipSuccess) {
      (void)hipFree(ls);
      rc = STTSV_EHIP;
      break;
    }
    f->leaf_slots.push_back(ls);
    f->n_leaf.push_back(cnt[0]);
    tb = tmp_bytes;
    if (hipcub::DeviceSelect::Flagged(tmp, tb, vals2, cont, act, nsel, static_cast<int>(A), s) != hipSuccess ||
        hipMemcpyAsync(&cnt[1], nsel, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = STTSV_EHIP;
      break;
    }
    A = cnt[1];
    f->levels = d + 1;
  }
  cleanup();
  if (rc == STTSV_OK) {
    for (int i = 0; i < 2 && rc == STTSV_OK; ++i) {
      int64_t maxn = 0;
      for (int64_t n_d : f->n_at) maxn = std::max(maxn, n_d);
      if (!dalloc(&f->buf[i], max_work, &f->device_bytes) || !dalloc(&f->ebuf[i], maxn, &f->device_bytes) ||
          !dalloc(&f->zbuf[i], maxn, &f->device_bytes))
        rc = STTSV_ENOMEM;
    }
  }
  if (rc == STTSV_OK && hipStreamSynchronize(s) != hipSuccess) rc = STTSV_EHIP;
  if (rc != STTSV_OK) {
    free_ccss(p);
    return rc;
  }
  f->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info != nullptr) {
    info->levels = f->levels;
    info->nodes = 0;
    for (int64_t n_d : f->n_at) info->nodes += n_d;
    info->roots = f->n_at.empty() ? 0 : f->n_at[0];
    info->convolutions = info->nodes - info->roots;
    info->leaves = 0;
    for (int64_t l : f->n_leaf) info->leaves += l;
    info->device_bytes = f->device_bytes;
    info->build_ms = f->build_ms;
  }
  return STTSV_OK;
}

hipError_t launch_ccss(Plan& p, const double* x, double* y, hipStream_t s) {
  CcssForest* f = p.ccss;
  const CcssTables& tab = ccss_tables();
  hipError_t e = launch_permute_x(p, x, s);
  if (e != hipSuccess) return e;
  const EdgeCall c{p.d_xr, p.d_contrib, nullptr, nullptr};
  p.contrib_compact = false;                     // FP64 contributions
  // size-1 edges: their own kernel (no path)
  for (const Bucket& B : p.buckets)
    if (B.k == 1 && (e = edge_tables().k1(c, B.desc[0], s)) != hipSuccess) return e;
  for (int d = 0; d < f->levels; ++d) {
    const int depth = d + 1;
    const int W = f->r - depth;
    if (W < 1) break;
    const int cur = d & 1, prv = cur ^ 1;
    const int64_t N = f->n_at[d];
    if (N > 0 && (e = tab.node[W](p.d_xr, f->vert[d], f->parent[d], N, depth, f->buf[prv], f->ebuf[prv],
                                  f->zbuf[prv], f->buf[cur], f->ebuf[cur], f->zbuf[cur], s)) != hipSuccess)
      return e;
    const int64_t NL = f->n_leaf[d];
    if (NL > 0) {
      const int k = depth + 1;
      for (const Bucket& B : p.buckets) {
        if (B.k != k) continue;
        if ((e = tab.leaf[W](c, B.desc[0], f->leaf_slots[d], NL, B.slot_off, f->leaf_node, f->buf[cur],
                             f->ebuf[cur], f->zbuf[cur], s)) != hipSuccess)
          return e;
      }
    }
  }
  return launch_reduction(p, y, nullptr, s);
}

int ccss_query(const Plan& p, int32_t what, std::vector<int64_t>& out) {
  const CcssForest* f = p.ccss;
  if (f == nullptr) return STTSV_EINVAL;
  out.clear();
  if (what == STTSV_Q_CCSS_LEVEL_N) {
    out.assign(f->n_at.begin(), f->n_at.end());
    return STTSV_OK;
  }
  if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;
  std::vector<int32_t> h;
  if (what == STTSV_Q_CCSS_VERT || what == STTSV_Q_CCSS_PARENT) {
    std::vector<int32_t> rid(p.n);
    if (p.n > 0 && hipMemcpy(rid.data(), p.d_rid, sizeof(int32_t) * p.n, hipMemcpyDeviceToHost) != hipSuccess)
      return STTSV_EHIP;
    for (int d = 0; d < f->levels; ++d) {
      h.resize(f->n_at[d]);
      const int32_t* src = what == STTSV_Q_CCSS_VERT ? f->vert[d] : f->parent[d];
      if (!h.empty() && hipMemcpy(h.data(), src, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return STTSV_EHIP;
      for (int32_t v : h) out.push_back(what == STTSV_Q_CCSS_VERT ? rid[v] : v);
    }
    return STTSV_OK;
  }
  if (what == STTSV_Q_CCSS_LEAF) {
    h.resize(p.nnz);
    if (p.nnz > 0 && hipMemcpy(h.data(), f->leaf_node, sizeof(int32_t) * p.nnz, hipMemcpyDeviceToHost) != hipSuccess)
      return STTSV_EHIP;
    out.assign(h.begin(), h.end());
    return STTSV_OK;
  }
  return STTSV_EINVAL;
}

}  // namespace sttsv
