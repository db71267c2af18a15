// Internal declarations shared by the host planner, the kernel launchers and
// the C ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/sttsv.h"

namespace sttsv {

// Edge kernels by edge size k: k = 1, 2, 3 have their own kernels; for
// 4 <= k <= 7 a register-resident kernel with k fixed at compile time is used
// where its series fit in registers; every other k >= 4 runs the generic
// kernel (runtime k, suffix stack in LDS or global memory), whose buckets are
// fused into one launch per window range.  All variants perform the same
// operations in the same order, so their contributions are bitwise identical.
enum SmallKind : int { SK_K2 = 0, SK_K3 = 1, SK_R4 = 2, SK_R5 = 3, SK_R6 = 4, SK_R7 = 5, SK_COUNT = 6 };

constexpr int kMaxW = STTSV_MAX_ORDER;   // windows W = r - k + 1 <= r - 1 for k >= 2
constexpr int kGenBlock = 64;            // threads per block of the generic kernel
constexpr int kSmallBlock = 256;         // threads per block of the other edge kernels
constexpr int kChunk = 32;               // reduction chunk length (fixed: part of the format)
constexpr int kXcd = 8;                  // accelerator dies (XCDs); workgroups go round-robin over them
constexpr int kStageTerms = 20480;       // contributions one level-0 workgroup stages in LDS (160 KiB, all of it)
constexpr int kStageThreads = 1024;      // threads of a level-0 workgroup
constexpr int kStagePasses = 16;         // passes over its chunks a level-0 workgroup makes (at most)
constexpr int kStageRuns = kXcd;         // contiguous contribution ranges per level-0 workgroup (at most)
constexpr int32_t kNoDst = INT32_MIN;    // padding chunk of the reduction schedule: no output
constexpr int kRunMax = 4;               // prefix reuse: edges per run (per thread)
constexpr int kGenRanges = 8;            // window ranges of the fused generic kernels
constexpr int kGenLo[kGenRanges] = {1, 9, 17, 25, 33, 41, 49, 57};
constexpr int kGenHi[kGenRanges] = {8, 16, 24, 32, 40, 48, 56, 63};
constexpr int64_t kLdsBudget = 40 * 1024;  // LDS per generic block by default (>= 4 blocks per CU)
constexpr int64_t kLdsMax = 64 * 1024;     // largest LDS per generic block the tuner may choose
constexpr int kKrBytes = 1024;           // register-resident kernels by default only where (k-1) W sizeof(T) fits
constexpr bool kr_default(int k, int W, int tsz) { return (k - 1) * W * tsz <= kKrBytes; }
constexpr int kCoopBlock = 256;          // threads per block of the lane-group edge kernel
constexpr int kCoopMaxW64 = 48;          // largest window of its FP64 variant (three series in registers)
constexpr int kCoopMaxW32 = 63;          // ... and of its FP32 variant

// Generic kernel: suffix checkpoint interval C for window W and series size
// tsz bytes (C + 2 live series within about 160 VGPRs, at most 4), and the
// per-thread stack it needs (z values and suffix products of z in FP64, then
// one checkpoint series per C forward steps).
constexpr int kg_checkpoint(int W, int tsz) {
  return (640 / (W * tsz) - 2) >= 4 ? 4 : (640 / (W * tsz) - 2) >= 1 ? (640 / (W * tsz) - 2) : 1;
}
constexpr int64_t kg_stack_bytes(int k, int W, int tsz) {
  return 16LL * k + (int64_t)((k - 3 + kg_checkpoint(W, tsz) - 1) / kg_checkpoint(W, tsz)) * W * tsz;
}
// Stack-free generic variant (suffix series recomputed, scalars in LDS):
// compiled for windows >= kStackFreeMinW, and for FP64 series up to
// kStackFreeMaxW64 (its three live series fit the registers there without
// scratch; longer FP64 windows would spill).
constexpr int kStackFree = 2;
constexpr int kStackFreeMinW = 9;
constexpr int kStackFreeMaxW64 = 48;
constexpr bool stack_free_ok(int W, int tsz) { return W >= kStackFreeMinW && (tsz == 4 || W <= kStackFreeMaxW64); }
constexpr int64_t kg_scalar_bytes(int k) { return 16LL * k; }

inline int gen_range_of(int W) {
  for (int g = 0; g < kGenRanges; ++g)
    if (W >= kGenLo[g] && W <= kGenHi[g]) return g;
  return -1;
}

// Per-call arguments of the edge kernels.
struct EdgeCall {
  const double* x;      // input vector
  double* contrib;      // per-incidence contributions (one region per vertex block)
  const int32_t* done;  // whole launch is skipped when *done != 0 (nullable)
  const int32_t* gskip; // per-graph skip flags indexed by BucketDesc::gid (nullable)
  // compact FP32 series (both null otherwise): FP32-series kernels gather x
  // from x32 and store each contribution as the upper 32 bits of its FP64
  // value, rounded, at the same place in contrib32 (a buffer of its own)
  const float* x32;
  uint32_t* contrib32;
};

#if defined(__HIP__)
// A contribution as a compact FP32 apply stores it: the upper 32 bits of the
// FP64 value rounded to nearest (ties away from zero), i.e. FP64's sign and
// exponent range with 21 significant bits; the reduction widens it back
// exactly.
__device__ __forceinline__ uint32_t contrib_word(double v) {
  return static_cast<uint32_t>((static_cast<uint64_t>(__double_as_longlong(v)) + 0x80000000ull) >> 32);
}

// Store at place q in the call's format (run-time choice: for the size-1
// kernel only; the series kernels choose at compile time).
__device__ __forceinline__ void store_contrib(const EdgeCall& c, int64_t q, double v) {
  if (c.contrib32 != nullptr)
    c.contrib32[q] = contrib_word(v);
  else
    c.contrib[q] = v;
}
#endif

// Plan-time description of one size bucket (device pointers offset to the
// bucket's slot range).
struct BucketDesc {
  const int32_t* mem;   // member ids, SoA: mem[j*m + i]
  const int32_t* loc;   // contribution index of each member slot, SoA like mem
  const int32_t* gid;   // graph of each edge (batched plans), or null
  void* gstack;         // generic kernel: per-edge global stack (when not in LDS)
  int64_t m;            // edges in the bucket
  int32_t k, r, W;      // edge size, tensor order, series window r - k + 1
  int32_t qexp;         // series scale exponent (rho = 2^qexp)
  int32_t lds_stack;    // generic kernel: 1 = stack in LDS, 0 = in global memory, kStackFree = none
  int32_t reuse_emin;   // prefix reuse: smallest exponent of z_0, z_1 with an exact rescale
  int32_t lanes;        // lane-group kernel: lanes per edge (power of two >= k, <= 64)
  double wk;            // w(e)/|beta(e)| (r-1)! for w(e) = |e|
  const double* wgt;    // per-edge w(e)/|beta(e)| (r-1)! (edge-weighted plans), or null
  // prefix reuse (FP64 register-resident kernels): runs of consecutive edges
  // with the same first two members, longest first; run_cnt[L] runs of
  // kRunMax - L edges
  const int32_t* run_start;
  int64_t nruns;
  int32_t run_cnt[4];
};

// One block of a fused generic launch: 64 consecutive edges of a bucket.
struct GenTask {
  int32_t bucket;
  int32_t block;
};

using SmallLaunchFn = hipError_t (*)(const EdgeCall&, const BucketDesc&, hipStream_t);
using GenLaunchFn = hipError_t (*)(const EdgeCall&, const BucketDesc* bks, const GenTask* tasks,
                                   int64_t ntasks, size_t lds, hipStream_t);

struct EdgeTables {
  SmallLaunchFn small64[SK_COUNT][kMaxW + 1];
  SmallLaunchFn small32[SK_COUNT][kMaxW + 1];
  SmallLaunchFn small32c[SK_COUNT][kMaxW + 1];   // compact FP32-apply variants (FP32 x, 32-bit contributions)
  SmallLaunchFn run64[4][kMaxW + 1];     // prefix-reuse variants, k = 4..7, FP64
  GenLaunchFn gen64[kGenRanges];
  GenLaunchFn gen32[kGenRanges];
  GenLaunchFn gen32c[kGenRanges];
  GenLaunchFn coop64[kGenRanges];        // fused lane-group kernels by window range (FP64, FP32 series)
  GenLaunchFn coop32[kGenRanges];
  GenLaunchFn coop32c[kGenRanges];
  SmallLaunchFn k1;
};

// Lanes per edge of the lane-group kernel for edges of size k in an order-r
// tensor (0: one lane per edge), given how many one-lane waves the graph's
// edges of every size with the same window range would make.  A pure
// function of the graph, so a graph's results do not depend on the plan it
// is part of.
int coop_lanes(int r, int k, int64_t range_waves);
const EdgeTables& edge_tables();

// One level of the deterministic node reduction.
struct ReduceLevel {
  int64_t nchunks = 0;
  // one 16-byte descriptor per chunk (a single load for the 8 lanes of a
  // chunk): x = first input index, y = length (0 for an isolated vertex),
  // z = destination (>= 0: vertex id, final; < 0: -(partial index)-1;
  // kNoDst: padding), w = the same with the vertex's degree-rank position
  // in place of its id (the solver keeps its vectors in that order)
  int4* d_desc = nullptr;
  // level 0 only (null for the other levels, which use 8 lanes per chunk):
  // two int4 per workgroup, {first chunk, chunks summed by 8 lanes, by 4,
  // by 2} and {chunks summed by 1 lane, first range, ranges, 0}.  The
  // workgroup's terms are consecutive node-major incidences; it copies its
  // contribution ranges (int2 {first place, length}) into LDS, every term
  // to its node-major offset (d_lpos, one per place), so each chunk is a
  // run of LDS.  Its chunk descriptors are int2 {LDS offset | length << 16,
  // destination}, with vertex ids [0] or degree-rank positions [1] as
  // destinations.
  int4* d_wg = nullptr;
  int64_t nwg = 0;
  int2* d_ranges = nullptr;
  uint16_t* d_lpos = nullptr;
  int2* d_desc0[2] = {nullptr, nullptr};
  int64_t in_len = 0;           // length of this level's input array
};

struct Bucket {
  int32_t r = 0;          // tensor order of the graphs in this bucket
  int32_t k = 0;
  int64_t m = 0;
  int64_t edge_off = 0;   // first canonical edge
  int64_t slot_off = 0;   // first member slot
  int64_t task0 = -1;     // first workgroup of the bucket in its FP64 fused generic launch
  int32_t qexp32 = 0;     // FP32 series scale exponent
  bool fp32_ok = true;    // FP32 series representable for this size
  void* gstack[2] = {nullptr, nullptr};  // generic-kernel global stacks [fp64, fp32]
  BucketDesc desc[2];     // [fp64 series, fp32 series]
  int small_kind[2] = {-1, -1};          // SmallKind, or -1: generic / k = 1
  int lanes_per_edge = 0;                // lane-group kernel: lanes per edge (0: not this kernel)
  int coop[2] = {0, 0};                  // lanes per edge per series type (0 where W is above its cap)
  int lds_pref[2] = {-1, -1};            // generic stack placement: -1 auto, 0 global, 1 LDS
  bool reuse = false;                    // FP64 register-resident kernel with prefix reuse
  int reuse_pref = -1;                   // tuner choice: -1 flag decides, 0 off, 1 on
  std::vector<int32_t> runs;             // host copy of the run starts (longest first)
  int32_t* d_runs = nullptr;
};

// A fused generic launch: all generic buckets of one precision whose window
// falls in one range.
struct GenGroup {
  int range = 0;
  bool coop = false;    // lane-group kernel (else the one-lane generic kernel)
  bool stack_free = false;   // one-lane generic kernel without suffix stacks
  int seq = 0;          // launch sequence: 0 = FP64 apply, 1 = FP32-series apply
  bool f64 = true;      // series type of the group's kernels
  int64_t ntasks = 0;
  size_t lds = 0;
  BucketDesc* d_bks = nullptr;
  GenTask* d_tasks = nullptr;
  int64_t bytes = 0;
  std::vector<int> buckets;
};

// One launch of the STTSV sequence.
struct Stage {
  int type;      // 0 = per-bucket edge kernel, 1 = fused generic group, 2 = reduction level,
                 // 3 = x into degree-rank order
  int index;     // bucket, group or level
  bool f64;      // series type of an edge stage
  int lane = 0;  // stream lane of an edge stage (0 = the plan's stream)
};

// Edge launches run on up to kLanes streams: the plan's own and kLanes - 1
// helpers of default priority, forked from and joined back to the plan's
// stream with events.
constexpr int kLanes = 3;

// One hypergraph of a (possibly batched) plan.
struct GraphInfo {
  int64_t m = 0, nnz = 0;
  int32_t n = 0, r = 0;
  int32_t voff = 0;       // first vertex in the plan's vertex numbering
  int64_t eoff = 0;       // first input edge in the plan's edge numbering
  bool connected = false;
  double norm2 = 0.0;     // ||B||^2 of the graph's blowup tensor
};

struct Plan {
  int64_t m = 0, nnz = 0;
  int32_t n = 0, r = 0;   // r: the largest tensor order of the plan's graphs
  std::vector<GraphInfo> graphs;
  int32_t precision = STTSV_PREC_FP64;
  int32_t flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  bool connected = false;
  int64_t device_bytes = 0;

  std::vector<Bucket> buckets;      // ordered by (r, k)
  std::vector<double> weights;      // w/|beta| (r-1)! for k = 0..r of the first graph's r

  // host copies of the canonical layout (introspection)
  std::vector<int64_t> perm;
  std::vector<int32_t> mem;
  std::vector<int64_t> tptr;
  std::vector<int32_t> tslot;

  // device buffers
  int32_t* d_mem = nullptr;       // member slots as degree-rank positions (what the kernels gather by)
  int32_t* d_rid = nullptr;       // vertex id at every degree-rank position
  double* d_xr = nullptr;         // x in degree-rank order (written by the permute stage)
  float* d_xr32 = nullptr;        // ... and rounded to FP32 (compact FP32 applies)
  std::vector<int32_t> vblock;    // vertex block of every vertex
  std::vector<int64_t> region;    // first contribution index of every block (+ nnz at the end)
  int32_t* d_loc = nullptr;       // contribution index of every member slot
  std::vector<int32_t> glist;     // contribution index of every node-major incidence (host)
  // level-0 schedule on the host: per workgroup {first chunk, 8-, 4-, 2-lane
  // chunks}, its 1-lane chunk count and its first node-major incidence.  The
  // LDS ranges and offsets follow from the places, so they are rebuilt
  // whenever the places change.
  std::vector<int4> l0_wg;
  std::vector<int32_t> l0_n1;
  std::vector<int32_t> l0_graph;     // graph of each level-0 workgroup's block
  std::vector<int32_t> block_graph;  // graph of every vertex block
  std::vector<int64_t> l0_base, l0_terms;
  int32_t* d_gid = nullptr;       // graph of every edge (batched plans only)
  double* d_wgt = nullptr;        // per canonical edge w(e)/|beta(e)| (r-1)! (edge-weighted plans only)
  double* d_contrib = nullptr;    // contributions, one region per vertex block
  uint32_t* d_contrib32 = nullptr; // the same places as 32-bit words (compact FP32 series)
  bool contrib_compact = false;   // the last apply stored 32-bit contributions (FP32 apply)
  bool compact_ok = false;        // every FP32-list edge stage (k >= 2) runs FP32 series: FP32 applies run compact
  std::vector<GenGroup> groups;   // fused generic launches (both precisions)
  std::vector<Stage> stages[2];   // launch sequence per precision [fp64, fp32]
  int lanes[2] = {1, 1};          // stream lanes the edge stages use, per precision
  hipStream_t aux[kLanes - 1] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kLanes - 1] = {};
  std::vector<ReduceLevel> levels;
  std::vector<double*> d_partials;   // partial arrays for levels >= 1

  // solver scratch (allocated on first solve)
  struct Solver* solver = nullptr;
  // the CCSS forest (built on request, ccss.hip)
  struct CcssForest* ccss = nullptr;
  // SS-HOPM / contraction scratch and captured updates (first use, sshopm.hip)
  struct ZState* zstate = nullptr;
};

// planner (plan.cpp): a plan over the disjoint union of G hypergraphs
struct GraphIn {
  const int64_t* eptr;
  const int32_t* eidx;
  int64_t m;
  int32_t n, r;
  const double* w;        // edge weights (nullable: w(e) = |e|)
};
int build_plan(int G, const GraphIn* gs, const sttsv_opts* opts, Plan** out);
void free_plan(Plan* p);

// STTSV launch sequence (apply.hip): per-bucket edge kernels and fused
// generic groups, then one stage per reduction level.
// An FP32 apply (precision STTSV_PREC_FP32) runs compact: FP32 copy of x,
// 32-bit contributions and a level-0 reduction that reads them.
hipError_t launch_sttsv(Plan& p, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s);
int stage_count(const Plan& p, int precision);
hipError_t launch_stage(Plan& p, int stage, const double* x, double* y, int precision,
                        const int32_t* done, hipStream_t s);
void stage_desc(const Plan& p, int precision, int stage, int32_t* kind, int32_t* size, int64_t* count);
void build_stages(Plan& p);   // fills p.stages from buckets, groups and levels
int init_lanes(Plan& p);      // helper streams and events of the edge lanes
int build_groups(Plan& p);    // (re)builds the fused generic groups (plan.cpp)
int assign_places(Plan& p);   // contribution places (and the level-0 LDS slots) for the current kernel choice
int set_reuse(Plan& p, Bucket& b, bool by_flag);   // prefix-reuse runs of a bucket (plan.cpp)
// The edge launches of one precision (per-graph skip flags, nullable), and
// the reduction alone: the solver runs both precisions' edge launches then
// one reduction per iteration.  launch_edges first copies x into degree-rank
// order unless permute is false (the copy of an earlier call is still valid).
// x order of an edge launch: the caller's vertex order (copied into rank
// order first), already in rank order, or copied by an earlier launch.
enum class XOrder { kVertex, kRank, kCopied };
// gate (nullable): one flag per edge stage of the precision's sequence
// (indexed as the plan's stage list); a stage's kernels leave at once when
// its flag is set, in place of done.
hipError_t launch_edges(Plan& p, const double* x, int precision, const int32_t* done, const int32_t* gskip,
                        hipStream_t s, XOrder order = XOrder::kVertex, bool compact = false,
                        const int32_t* gate = nullptr);
// rank_out: write y in degree-rank order instead of vertex order.
hipError_t launch_reduction(Plan& p, double* y, const int32_t* done, hipStream_t s, bool rank_out = false,
                            bool compact = false);
// The solver's mixed schedule with compact FP32 series: graph g's level-0
// workgroups read 32-bit words when phase32[g] == 0 (the graph runs FP32
// series this iteration), FP64 contributions otherwise.
hipError_t launch_reduction_phased(Plan& p, double* y, const int32_t* phase32, const int32_t* done, hipStream_t s,
                                   bool rank_out);
// FP32- and FP64-series edge stages (x already in rank order) inside one
// fork/join, each gated by its own per-graph skip flags: the solver's mixed
// schedule, where each graph runs one of the two per iteration.  With x32
// (the iterate in rank order, rounded to FP32) the FP32 stages run compact.
hipError_t launch_edges_both(Plan& p, const double* x, const int32_t* done, const int32_t* skip32,
                             const int32_t* skip64, hipStream_t s, const float* x32,
                             const int32_t* gate32 = nullptr, const int32_t* gate64 = nullptr);

// x into degree-rank order (the copy the edge kernels gather from)
hipError_t launch_permute_x(Plan& p, const double* x, hipStream_t s);

// the CCSS forest and Alg. 4 over it (ccss.hip)
int build_ccss(Plan& p, sttsv_ccss_info* info);
hipError_t launch_ccss(Plan& p, const double* x, double* y, hipStream_t s);
int ccss_query(const Plan& p, int32_t what, std::vector<int64_t>& out);
void free_ccss(Plan& p);
void free_zstate(Plan& p);

// symmetric CP decomposition of the blowup tensor over the STTSV (cp.hip)
int cp_objective_grad(Plan& p, int32_t R, const double* A, const double* lambda, double* f, double* dA,
                      double* dlambda);
int cp_descent(Plan& p, int32_t R, double* A, double* lambda, int32_t iters, double step, sttsv_cp_info* info);

// reduction kernels (reduce.hip)
hipError_t launch_reduce_level(const ReduceLevel& L, const void* in, double* y, double* next,
                               const int32_t* done, hipStream_t s, bool rank_out = false, bool compact = false);
hipError_t launch_reduce_level0_phased(const ReduceLevel& L, const double* in64, const uint32_t* in32,
                                       const int32_t* phase32, double* y, double* next, const int32_t* done,
                                       hipStream_t s, bool rank_out);

// autotuner (tune.cpp)
int autotune(Plan& p, const double* x, int reps, const char* cache_path, int32_t* tuned);

// solver (nqz.hip): every graph of the plan; infos has one entry per graph
int solve(Plan& p, const double* x0, double tol, const sttsv_solve_opts& o, double* x_out,
          sttsv_solve_info* infos);
void free_solver(Plan& p);

}  // namespace sttsv
