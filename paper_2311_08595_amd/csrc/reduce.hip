// Deterministic node-major reduction y_v = sum of v's per-incidence
// contributions (replaces the AtomicAdd accumulation of Alg. 3 / Alg. 4).
//
// The summation tree of every vertex is fixed by its incidence list alone:
// the list (canonical edge order) is cut into chunks of kChunk = 32
// consecutive terms.  A chunk is summed by a group of 8 lanes: lane j adds
// terms j, j+8, j+16, j+24 in that order (missing terms are exact zeros),
// then the 8 lane sums are combined by a halving butterfly (offsets 4, 2, 1).
// If a vertex has more than one chunk, the chunk sums are the input of the
// next level and are cut the same way.  No launch parameter enters the tree,
// so y is bitwise identical across runs, launch shapes and devices.
//
// The first level reads the contributions, which the edge kernels leave in
// one contiguous region per block of vertices (at most kStageTerms of them
// per block, or one vertex with more).  A level-0 workgroup owns one block,
// or kStageTerms consecutive terms of a larger vertex, i.e. a run of
// consecutive node-major incidences.  It copies its contributions into LDS
// with coalesced loads, each term to its node-major offset, and then sums
// every chunk from a run of LDS; the descriptors of all its passes are
// loaded up front, so no pass waits for global memory.  Gathering straight
// from global memory made every lane fetch its own cache line.
#include "internal.hpp"

namespace sttsv {
namespace {

constexpr int kGroup = 8;                   // lanes per chunk
constexpr int kPerLane = kChunk / kGroup;   // terms per lane
constexpr int kCopyDepth = 4;                // loads in flight per thread while staging
static_assert(kChunk % kGroup == 0, "chunk must split evenly over the group");
static_assert(kStageTerms <= 65536, "LDS offsets are 16-bit");
static_assert(kGroup == 8, "pass_at assumes lane classes 8, 4, 2, 1");

// v from lane i + K of the same row of 16 lanes (DPP row shift; lanes whose
// source lies outside the row get 0).  Chunk groups of 8, 4 and 2 lanes are
// aligned within rows, and a lane only ever reads a lane of its own group
// whose value the tree still needs.
template <int K>
__device__ __forceinline__ double lane_down(double v) {
  static_assert(K >= 1 && K <= 15, "row shift");
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x100 + K, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x100 + K, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// A term as stored: FP64, or (compact FP32 applies) the upper 32 bits of the
// FP64 value, which widen back exactly.
__device__ __forceinline__ double term(double v) { return v; }
__device__ __forceinline__ double term(uint32_t w) { return __hiloint2double(static_cast<int>(w), 0); }

// Levels >= 1: chunk c of the level is summed by lanes 8c .. 8c+7.
template <bool RANK, typename In>
__global__ void __launch_bounds__(256) reduce_level(const int4* __restrict__ desc, int64_t nchunks,
                                                    const In* __restrict__ in,
                                                    double* __restrict__ y, double* __restrict__ next,
                                                    const int32_t* done) {
  if (done != nullptr && *done) return;     // uniform: every lane leaves together
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = gid / kGroup;
  const int j = static_cast<int>(gid % kGroup);
  int4 dsc = make_int4(0, 0, kNoDst, 0);
  if (c < nchunks) dsc = desc[c];
  const int32_t s = dsc.x, l = dsc.y;
  double t[kPerLane];
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {   // all loads first; an absent term re-reads the chunk's first
    const int p = j + q * kGroup;
    t[q] = term(in[p < l ? s + p : s]);
  }
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) v = j + q * kGroup < l ? v + t[q] : v;
  v += lane_down<4>(v);
  v += lane_down<2>(v);
  v += lane_down<1>(v);
  if (j == 0 && c < nchunks) {
    const int32_t d = RANK ? dsc.w : dsc.z;
    if (d >= 0)
      y[d] = v;
    else if (d != kNoDst)
      next[-(int64_t)d - 1] = v;
  }
}

// Copy src[0 .. len) into LDS, term i to st[pos[i]], kCopyDepth loads in
// flight per thread.
template <typename In>
__device__ __forceinline__ void stage_range(const In* __restrict__ src, const uint16_t* __restrict__ pos,
                                            double* st, int len) {
  for (int i0 = 0; i0 < len; i0 += kStageThreads * kCopyDepth) {
    In t[kCopyDepth];
    int k[kCopyDepth];
#pragma unroll
    for (int u = 0; u < kCopyDepth; ++u) {   // unconditional loads (index clamped): all in flight at once
      const int i = i0 + u * kStageThreads + static_cast<int>(threadIdx.x);
      const int ic = i < len ? i : len - 1;
      t[u] = src[ic];
      k[u] = i < len ? static_cast<int>(pos[ic]) : -1;
    }
#pragma unroll
    for (int u = 0; u < kCopyDepth; ++u)
      if (k[u] >= 0) st[k[u]] = term(t[u]);
  }
}

// Pass p of a level-0 workgroup (uniform): lanes per chunk G (0: no such
// pass), first chunk of the pass and end of its lane class.
struct PassAt {
  int G, lg, first, end;   // lg = log2 G
};
__device__ __forceinline__ PassAt pass_at(int p, int4 a, int n1) {
  int c = a.x;
  const int n[4] = {a.y, a.z, a.w, n1};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int G = kGroup >> q, per = kStageThreads / G;
    const int np = (n[q] + per - 1) / per;
    if (p < np) return PassAt{G, 3 - q, c + p * per, c + n[q]};
    p -= np;
    c += n[q];
  }
  return PassAt{0, 0, 0, 0};
}

// One pass: every group of G lanes sums one chunk from LDS.  G = 8: lane j
// adds terms j, j+8, j+16, j+24 (the present ones, in that order), then the
// halving butterfly.  G < 8 (chunks of at most G terms): lane j holds s_j =
// 0.0 + t_j (or 0.0), and every partial sum the 8-lane tree would take from
// an absent lane is added as the +0.0 it is, so the bits are those of the
// 8-lane tree.  All LDS reads of a lane are issued before the first add
// (indices clamped into the array; absent terms are not added).
__device__ __forceinline__ void stage_pass(int G, int2 d, const double* st, double* __restrict__ y,
                                           double* __restrict__ next) {
  const int j = static_cast<int>(threadIdx.x) & (G - 1);
  const int s = d.x & 0xffff, l = d.x >> 16;
  double v = 0.0;
  if (G == kGroup) {
    double t[kPerLane];
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) t[q] = st[min(s + j + q * kGroup, kStageTerms - 1)];
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) v = j + q * kGroup < l ? v + t[q] : v;
    v += lane_down<4>(v);
    v += lane_down<2>(v);
    v += lane_down<1>(v);
  } else {
    const double t = st[min(s + j, kStageTerms - 1)];
    v = j < l ? v + t : v;
    v = v + 0.0;                                                    // + s_{j+4}
    if (G >= 4) v += lane_down<2>(v); else v = v + 0.0;
    if (G >= 2) v += lane_down<1>(v); else v = v + 0.0;
  }
  if (j == 0) {
    if (d.y >= 0)
      y[d.y] = v;
    else if (d.y != kNoDst)
      next[-(int64_t)d.y - 1] = v;
  }
}

// One level-0 workgroup: stage its contributions (format In) into LDS, then
// its passes.
template <typename In>
__device__ __forceinline__ void level0_body(double* st, const int2* __restrict__ desc, int4 a, int4 b,
                                            const int2* __restrict__ ranges, const uint16_t* __restrict__ lpos,
                                            const In* __restrict__ in, double* __restrict__ y,
                                            double* __restrict__ next) {
  int2 d[kStagePasses];
#pragma unroll
  for (int p = 0; p < kStagePasses; ++p) {
    const PassAt P = pass_at(p, a, b.x);
    const int c = P.first + (static_cast<int>(threadIdx.x) >> P.lg);
    d[p] = P.G > 0 && c < P.end ? desc[c] : make_int2(0, kNoDst);
  }
  for (int r = 0; r < b.z; ++r) {
    const int2 rg = ranges[b.y + r];
    stage_range(in + rg.x, lpos + rg.x, st, rg.y);
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kStagePasses; ++p) {
    const PassAt P = pass_at(p, a, b.x);
    if (P.G == 0) break;
    stage_pass(P.G, d[p], st, y, next);
  }
}

template <typename In>
__global__ void __launch_bounds__(kStageThreads) reduce_level0(const int2* __restrict__ desc,
                                                               const int4* __restrict__ wg,
                                                               const int2* __restrict__ ranges,
                                                               const uint16_t* __restrict__ lpos,
                                                               const In* __restrict__ in,
                                                               double* __restrict__ y, double* __restrict__ next,
                                                               const int32_t* done) {
  if (done != nullptr && *done) return;
  __shared__ double st[kStageTerms];
  level0_body<In>(st, desc, wg[2 * blockIdx.x], wg[2 * blockIdx.x + 1], ranges, lpos, in, y, next);
}

// Mixed formats: the workgroup's block belongs to graph b.w, whose
// contributions this iteration are 32-bit words when phase32[b.w] == 0 (the
// graph ran FP32 series) and FP64 otherwise (uniform per workgroup).
__global__ void __launch_bounds__(kStageThreads) reduce_level0_phased(const int2* __restrict__ desc,
                                                                      const int4* __restrict__ wg,
                                                                      const int2* __restrict__ ranges,
                                                                      const uint16_t* __restrict__ lpos,
                                                                      const double* __restrict__ in64,
                                                                      const uint32_t* __restrict__ in32,
                                                                      const int32_t* __restrict__ phase32,
                                                                      double* __restrict__ y,
                                                                      double* __restrict__ next, const int32_t* done) {
  if (done != nullptr && *done) return;
  __shared__ double st[kStageTerms];
  const int4 a = wg[2 * blockIdx.x], b = wg[2 * blockIdx.x + 1];
  if (phase32[b.w] == 0)
    level0_body<uint32_t>(st, desc, a, b, ranges, lpos, in32, y, next);
  else
    level0_body<double>(st, desc, a, b, ranges, lpos, in64, y, next);
}

}  // namespace

template <typename In>
hipError_t launch_level(const ReduceLevel& L, const In* in, double* y, double* next, const int32_t* done,
                        hipStream_t s, bool rank_out) {
  if (L.d_wg != nullptr) {
    hipLaunchKernelGGL((reduce_level0<In>), dim3(static_cast<unsigned>(L.nwg)), dim3(kStageThreads), 0, s,
                       L.d_desc0[rank_out ? 1 : 0], L.d_wg, L.d_ranges, L.d_lpos, in, y, next, done);
    return hipGetLastError();
  }
  const int64_t threads = L.nchunks * kGroup;
  const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
  if (rank_out)
    hipLaunchKernelGGL((reduce_level<true, In>), grid, dim3(256), 0, s, L.d_desc, L.nchunks, in, y, next, done);
  else
    hipLaunchKernelGGL((reduce_level<false, In>), grid, dim3(256), 0, s, L.d_desc, L.nchunks, in, y, next, done);
  return hipGetLastError();
}

hipError_t launch_reduce_level0_phased(const ReduceLevel& L, const double* in64, const uint32_t* in32,
                                       const int32_t* phase32, double* y, double* next, const int32_t* done,
                                       hipStream_t s, bool rank_out) {
  if (L.nchunks == 0) return hipSuccess;
  if (L.d_wg == nullptr) return hipErrorInvalidValue;    // level 0 is always staged when it has chunks
  hipLaunchKernelGGL(reduce_level0_phased, dim3(static_cast<unsigned>(L.nwg)), dim3(kStageThreads), 0, s,
                     L.d_desc0[rank_out ? 1 : 0], L.d_wg, L.d_ranges, L.d_lpos, in64, in32, phase32, y, next, done);
  return hipGetLastError();
}

hipError_t launch_reduce_level(const ReduceLevel& L, const void* in, double* y, double* next,
                               const int32_t* done, hipStream_t s, bool rank_out, bool compact) {
  if (L.nchunks == 0) return hipSuccess;
  return compact ? launch_level(L, static_cast<const uint32_t*>(in), y, next, done, s, rank_out)
                 : launch_level(L, static_cast<const double*>(in), y, next, done, s, rank_out);
}

}  // namespace sttsv
