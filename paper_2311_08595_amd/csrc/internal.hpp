// Internal declarations shared by the host planner, the kernel launchers and
// the C ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/sttsv.h"

namespace sttsv {

// Kinds of edge kernels (by edge size k).
enum EdgeKind : int { KIND_K1 = 0, KIND_K2 = 1, KIND_K3 = 2, KIND_KG = 3, KIND_COUNT = 4 };

constexpr int kMaxW = STTSV_MAX_ORDER;   // windows W = r - k + 1 <= r - 1 for k >= 2
constexpr int kGenBlock = 64;            // threads per block of the generic kernel
constexpr int kSmallBlock = 256;         // threads per block of the k <= 3 kernels
constexpr int kChunk = 32;               // reduction chunk length (fixed: part of the format)

// Arguments of one bucket launch (all device pointers already offset to the
// bucket's slot range).
struct EdgeLaunch {
  const double* x;      // input vector
  const int32_t* mem;   // member slots of the bucket, SoA: mem[j*m + i]
  double* contrib;      // contributions, same slot layout as mem
  void* gstack;         // global suffix stack for the generic kernel (or null)
  const int32_t* done;  // early-exit flag (solver), nullable
  int64_t m;            // edges in the bucket
  int32_t k;            // edge size
  int32_t r;            // tensor order
  int32_t qexp;         // series scale exponent (rho = 2^qexp)
  int32_t lds_stack;    // 1: suffix stack in LDS, 0: in gstack
  double wk;            // w(e)/|beta(e)| (r-1)!
};

using EdgeLaunchFn = hipError_t (*)(const EdgeLaunch&, hipStream_t);

// Function tables indexed [kind][W], filled by the instantiation units.
struct EdgeTables {
  EdgeLaunchFn f64[KIND_COUNT][kMaxW + 1];
  EdgeLaunchFn f32[KIND_COUNT][kMaxW + 1];
};
const EdgeTables& edge_tables();

// One level of the deterministic node reduction.
struct ReduceLevel {
  int64_t nchunks = 0;
  int32_t* d_start = nullptr;   // first input index of each chunk
  int32_t* d_len = nullptr;     // chunk length (0 for an isolated vertex)
  int32_t* d_dst = nullptr;     // >= 0: vertex id (final); < 0: -(partial index)-1
  int64_t in_len = 0;           // length of this level's input array
};

struct Bucket {
  int32_t k = 0;
  int64_t m = 0;
  int64_t edge_off = 0;   // first canonical edge
  int64_t slot_off = 0;   // first member slot
  int32_t qexp32 = 0;     // FP32 series scale exponent
  bool fp32_ok = true;    // FP32 series representable for this size
  int32_t lds64 = 1, lds32 = 1;  // stack placement per precision (generic kind)
  void* gstack64 = nullptr;
  void* gstack32 = nullptr;
};

struct Plan {
  int64_t m = 0, nnz = 0;
  int32_t n = 0, r = 0;
  int32_t precision = STTSV_PREC_FP64;
  hipStream_t stream = nullptr;
  int device = 0;
  bool connected = false;
  int64_t device_bytes = 0;

  std::vector<Bucket> buckets;
  std::vector<double> weights;      // index k = 0..r

  // host copies of the canonical layout (introspection)
  std::vector<int64_t> perm;
  std::vector<int32_t> mem;
  std::vector<int64_t> tptr;
  std::vector<int32_t> tslot;

  // device buffers
  int32_t* d_mem = nullptr;
  int32_t* d_tslot = nullptr;
  double* d_contrib = nullptr;
  std::vector<ReduceLevel> levels;
  std::vector<double*> d_partials;   // partial arrays for levels >= 1

  // solver scratch (allocated on first solve)
  struct Solver* solver = nullptr;
};

// planner (plan.cpp)
int build_plan(const int64_t* eptr, const int32_t* eidx, int64_t m, int32_t n, int32_t r,
               const sttsv_opts* opts, Plan** out);
void free_plan(Plan* p);

// STTSV launch sequence (apply.hip): one stage per size bucket (edge
// kernel), then one stage per reduction level.
hipError_t launch_sttsv(Plan& p, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s);
int stage_count(const Plan& p);
hipError_t launch_stage(Plan& p, int stage, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s);
void stage_desc(const Plan& p, int stage, int32_t* kind, int32_t* size, int64_t* count);

// reduction kernels (reduce.hip)
hipError_t launch_reduce_level(const ReduceLevel& L, int level, const double* in,
                               const int32_t* tslot, double* y, double* next,
                               const int32_t* done, hipStream_t s);

// solver (nqz.hip)
int solve(Plan& p, const double* x0, double tol, const sttsv_solve_opts& o, double* x_out,
          sttsv_solve_info* info);
void free_solver(Plan& p);

}  // namespace sttsv
