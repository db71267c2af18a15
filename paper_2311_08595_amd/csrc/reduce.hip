// Deterministic node-major reduction y_v = sum of v's per-incidence
// contributions (replaces the AtomicAdd accumulation of Alg. 3 / Alg. 4).
//
// The summation tree of every vertex is fixed by its degree alone: the
// incidences of v, in canonical edge order, are cut into chunks of kChunk
// consecutive terms summed left to right; if there is more than one chunk,
// the chunk sums form the input of the next level and are cut the same way.
// So y is bitwise identical across runs, launch shapes and devices.
#include "internal.hpp"

namespace sttsv {
namespace {

template <bool GATHER>
__global__ void __launch_bounds__(256) reduce_level(const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ len,
                                                    const int32_t* __restrict__ dst, int64_t nchunks,
                                                    const double* __restrict__ in,
                                                    const int32_t* __restrict__ tslot,
                                                    double* __restrict__ y, double* __restrict__ next,
                                                    const int32_t* done) {
  if (done != nullptr && *done) return;
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  const int32_t s = start[c];
  const int32_t l = len[c];
  double acc = 0.0;
  if (l > 0) {
    acc = GATHER ? in[tslot[s]] : in[s];
    for (int32_t p = 1; p < l; ++p) acc += GATHER ? in[tslot[s + p]] : in[s + p];
  }
  const int32_t d = dst[c];
  if (d >= 0)
    y[d] = acc;
  else
    next[-(int64_t)d - 1] = acc;
}

}  // namespace

hipError_t launch_reduce_level(const ReduceLevel& L, int level, const double* in,
                               const int32_t* tslot, double* y, double* next,
                               const int32_t* done, hipStream_t s) {
  if (L.nchunks == 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((L.nchunks + 255) / 256));
  if (level == 0)
    hipLaunchKernelGGL((reduce_level<true>), grid, dim3(256), 0, s, L.d_start, L.d_len, L.d_dst,
                       L.nchunks, in, tslot, y, next, done);
  else
    hipLaunchKernelGGL((reduce_level<false>), grid, dim3(256), 0, s, L.d_start, L.d_len, L.d_dst,
                       L.nchunks, in, tslot, y, next, done);
  return hipGetLastError();
}

}  // namespace sttsv
