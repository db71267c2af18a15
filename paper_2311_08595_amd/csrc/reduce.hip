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

}  // namespace

hipError_t launch_reduce_level(const ReduceLevel& L, const double* in, double* y, double* next,
                               const int32_t* done, hipStream_t s, bool rank_out) {
  if (L.nchunks == 0) return hipSuccess;
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
