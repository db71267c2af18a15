// Deterministic node-major reduction y_v = sum of v's per-incidence
// contributions (replaces the AtomicAdd accumulation of Alg. 3 / Alg. 4).
// Contributions live in one region per vertex block (about 1 MiB each, see
// the planner); the first level gathers each vertex's terms from its block's
// region, and its workgroups are ordered so that every die works through
// its own blocks one at a time, keeping the gathered region in its L2.
//
// The summation tree of every vertex is fixed by its incidence list alone:
// the list (canonical edge order) is cut into chunks of kChunk = 32
// consecutive terms.  A chunk is summed by a group of 8 lanes: lane j adds
// terms j, j+8, j+16, j+24 in that order (missing terms are exact zeros),
// then the 8 lane sums are combined by a halving butterfly (offsets 4, 2, 1).
// If a vertex has more than one chunk, the chunk sums are the input of the
// next level and are cut the same way.  No launch parameter enters the tree,
// so y is bitwise identical across runs, launch shapes and devices.
#include "internal.hpp"

namespace sttsv {
namespace {

constexpr int kGroup = 8;                   // lanes per chunk
constexpr int kPerLane = kChunk / kGroup;   // terms per lane
static_assert(kChunk % kGroup == 0, "chunk must split evenly over the group");

template <bool GATHER, bool RANK>
__global__ void __launch_bounds__(256) reduce_level(const int4* __restrict__ desc, int64_t nchunks,
                                                    const int32_t* __restrict__ gather,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ y, double* __restrict__ next,
                                                    const int32_t* done) {
  if (done != nullptr && *done) return;     // uniform: every lane leaves together
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = gid / kGroup;
  const int j = static_cast<int>(gid % kGroup);
  int4 dsc = make_int4(0, 0, kNoDst, 0);
  if (c < nchunks) dsc = desc[c];
  const int32_t s = dsc.x, l = dsc.y;
  int32_t idx[kPerLane];
#pragma unroll
  for (int q = 0; q < kPerLane; ++q) {
    const int p = j + q * kGroup;
    idx[q] = p < l ? (GATHER ? gather[s + p] : s + p) : -1;
  }
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < kPerLane; ++q)
    if (idx[q] >= 0) v += in[idx[q]];
  v += __shfl_down(v, 4, kGroup);
  v += __shfl_down(v, 2, kGroup);
  v += __shfl_down(v, 1, kGroup);
  if (j == 0 && c < nchunks) {
    const int32_t d = RANK ? dsc.w : dsc.z;
    if (d >= 0)
      y[d] = v;
    else if (d != kNoDst)
      next[-(int64_t)d - 1] = v;
  }
}

// A chunk of at most G < 8 terms summed by G lanes with the same tree: lane
// j holds s_j (0.0 + t_j, or 0.0), and every partial sum the 8-lane tree
// would take from an absent lane is added as the +0.0 it is.
template <int G, bool GATHER>
__device__ __forceinline__ double short_chunk(int4 d, int j, const int32_t* __restrict__ gather,
                                              const double* __restrict__ in) {
  double v = 0.0;
  if (j < d.y) v += in[GATHER ? gather[d.x + j] : d.x + j];
  v = v + 0.0;                                                    // + s_{j+4}
  if constexpr (G >= 4) v += __shfl_down(v, 2, G); else v = v + 0.0;
  if constexpr (G >= 2) v += __shfl_down(v, 1, G); else v = v + 0.0;
  return v;
}

template <int G, bool GATHER, bool RANK>
__device__ __forceinline__ void level0_group(const int4* __restrict__ desc, int4 w, const int32_t* __restrict__ gather,
                                             const double* __restrict__ in, double* __restrict__ y,
                                             double* __restrict__ next) {
  const int lc = threadIdx.x / G, j = threadIdx.x % G;
  const bool active = lc < w.z;                 // whole groups of G lanes agree
  const int4 d = active ? desc[w.x + lc] : make_int4(0, 0, kNoDst, kNoDst);
  double v;
  if constexpr (G == kGroup) {
    int32_t idx[kPerLane];
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int p = j + q * kGroup;
      idx[q] = p < d.y ? (GATHER ? gather[d.x + p] : d.x + p) : -1;
    }
    v = 0.0;
#pragma unroll
    for (int q = 0; q < kPerLane; ++q)
      if (idx[q] >= 0) v += in[idx[q]];
    v += __shfl_down(v, 4, kGroup);
    v += __shfl_down(v, 2, kGroup);
    v += __shfl_down(v, 1, kGroup);
  } else {
    v = short_chunk<G, GATHER>(d, j, gather, in);
  }
  if (j == 0 && active) {
    const int32_t t = RANK ? d.w : d.z;
    if (t >= 0)
      y[t] = v;
    else if (t != kNoDst)
      next[-(int64_t)t - 1] = v;
  }
}

// Level 0 with the workgroup table: workgroup b takes chunks
// [wg[b].x, +wg[b].z), wg[b].y lanes each (uniform within the workgroup).
template <bool GATHER, bool RANK>
__global__ void __launch_bounds__(256) reduce_level0(const int4* __restrict__ desc, const int4* __restrict__ wg,
                                                     const int32_t* __restrict__ gather,
                                                     const double* __restrict__ in, double* __restrict__ y,
                                                     double* __restrict__ next, const int32_t* done) {
  if (done != nullptr && *done) return;
  const int4 w = wg[blockIdx.x];
  switch (w.y) {
    case 1: level0_group<1, GATHER, RANK>(desc, w, gather, in, y, next); break;
    case 2: level0_group<2, GATHER, RANK>(desc, w, gather, in, y, next); break;
    case 4: level0_group<4, GATHER, RANK>(desc, w, gather, in, y, next); break;
    default: level0_group<kGroup, GATHER, RANK>(desc, w, gather, in, y, next); break;
  }
}

}  // namespace

hipError_t launch_reduce_level(const ReduceLevel& L, const double* in, double* y, double* next,
                               const int32_t* done, hipStream_t s, bool rank_out) {
  if (L.nchunks == 0) return hipSuccess;
  if (L.d_wg != nullptr) {
    const dim3 grid(static_cast<unsigned>(L.nwg));
    const int4* d = L.d_desc;
    const int4* w = L.d_wg;
    if (L.d_gather != nullptr && rank_out)
      hipLaunchKernelGGL((reduce_level0<true, true>), grid, dim3(256), 0, s, d, w, L.d_gather, in, y, next, done);
    else if (L.d_gather != nullptr)
      hipLaunchKernelGGL((reduce_level0<true, false>), grid, dim3(256), 0, s, d, w, L.d_gather, in, y, next, done);
    else if (rank_out)
      hipLaunchKernelGGL((reduce_level0<false, true>), grid, dim3(256), 0, s, d, w, nullptr, in, y, next, done);
    else
      hipLaunchKernelGGL((reduce_level0<false, false>), grid, dim3(256), 0, s, d, w, nullptr, in, y, next, done);
    return hipGetLastError();
  }
  const int64_t threads = L.nchunks * kGroup;
  const dim3 grid(static_cast<unsigned>((threads + 255) / 256));
  const int4* d = L.d_desc;
  if (L.d_gather != nullptr) {
    if (rank_out)
      hipLaunchKernelGGL((reduce_level<true, true>), grid, dim3(256), 0, s, d, L.nchunks, L.d_gather, in, y, next, done);
    else
      hipLaunchKernelGGL((reduce_level<true, false>), grid, dim3(256), 0, s, d, L.nchunks, L.d_gather, in, y, next,
                         done);
  } else {
    if (rank_out)
      hipLaunchKernelGGL((reduce_level<false, true>), grid, dim3(256), 0, s, d, L.nchunks, nullptr, in, y, next, done);
    else
      hipLaunchKernelGGL((reduce_level<false, false>), grid, dim3(256), 0, s, d, L.nchunks, nullptr, in, y, next,
                         done);
  }
  return hipGetLastError();
}

}  // namespace sttsv
