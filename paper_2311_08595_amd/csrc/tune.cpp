// Autotuner: picks, per size bucket and series type, among kernel variants
// that compute bitwise-identical contributions (so tuning never changes y):
//   * 4 <= k <= 7: register-resident kernel vs the generic kernel;
//   * generic buckets: suffix stack in LDS vs in global memory vs no stack
//     (suffix series recomputed; long windows only);
//   * FP64 register-resident buckets: with or without prefix reuse;
// and then the stream lane of every edge launch (whole applies timed).
// Each kernel candidate is launched alone on the plan's stream with the caller's x
// and timed with hipEvents (median of reps); the choices are kept in the plan
// and in a cache keyed by (series type, r, k, round(log2 m)), which can be
// read from and appended to a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace sttsv {
namespace {

struct Choice {
  int use_kr;   // -1 not applicable, 0 generic, 1 register-resident
  int lds;      // -1 not applicable, 0 global stack, 1 LDS stack, kStackFree no stack
  int reuse;    // -1 not applicable, 0 off, 1 prefix reuse
};

std::mutex g_mu;
std::map<std::string, Choice> g_cache;

std::string key_of(int t, const Bucket& B) {
  char buf[96];
  std::snprintf(buf, sizeof(buf), "t%d_r%d_k%d_m%d", t, B.r, B.k,
                static_cast<int>(std::lround(std::log2(std::max<double>(1.0, (double)B.m)))));
  return buf;
}

void load_cache(const char* path) {
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return;
  char key[96];
  int a = 0, b = 0, c = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  while (std::fscanf(f, "%95s %d %d %d", key, &a, &b, &c) == 4) g_cache[key] = Choice{a, b, c};
  std::fclose(f);
}

void append_cache(const char* path, const std::string& key, const Choice& c) {
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "a");
  if (f == nullptr) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), c.use_kr, c.lds, c.reuse);
  std::fclose(f);
}

template <typename F>
float time_median(F&& launch, int reps, hipStream_t s) {
  std::vector<float> t;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1e30f;
  (void)launch();                                   // warm-up
  for (int i = 0; i < reps; ++i) {
    float ms = 0.f;
    if (hipEventRecord(a, s) != hipSuccess || launch() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
        hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      ms = 1e30f;
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

// A one-bucket generic launch with the given stack placement (0 global,
// 1 LDS, kStackFree none).
float time_generic(Plan& p, Bucket& B, int t, int place, const EdgeCall& c, int reps) {
  const EdgeTables& tab = edge_tables();
  const int W = B.r - B.k + 1;
  const int tsz = t == 0 ? 8 : 4;
  const int64_t need = place == kStackFree ? (int64_t)kGenBlock * kg_scalar_bytes(B.k)
                                           : (int64_t)kGenBlock * kg_stack_bytes(B.k, W, tsz);
  if (place != 0 && need > kLdsMax) return 1e30f;
  if (place == kStackFree && !stack_free_ok(W, tsz)) return 1e30f;
  BucketDesc d = B.desc[t];
  void* tmp = nullptr;
  d.lds_stack = place;
  if (place == 0) {
    if (B.gstack[t] != nullptr) {
      d.gstack = B.gstack[t];
    } else {
      if (hipMalloc(&tmp, (size_t)kg_stack_bytes(B.k, W, tsz) * (size_t)B.m) != hipSuccess) return 1e30f;
      d.gstack = tmp;
    }
  }
  std::vector<GenTask> tasks;
  for (int64_t blk = 0; blk < (B.m + kGenBlock - 1) / kGenBlock; ++blk)
    tasks.push_back(GenTask{0, static_cast<int32_t>(blk)});
  BucketDesc* d_b = nullptr;
  GenTask* d_t = nullptr;
  float ms = 1e30f;
  if (hipMalloc(&d_b, sizeof(BucketDesc)) == hipSuccess &&
      hipMalloc(&d_t, sizeof(GenTask) * tasks.size()) == hipSuccess &&
      hipMemcpy(d_b, &d, sizeof(BucketDesc), hipMemcpyHostToDevice) == hipSuccess &&
      hipMemcpy(d_t, tasks.data(), sizeof(GenTask) * tasks.size(), hipMemcpyHostToDevice) == hipSuccess) {
    const GenLaunchFn fn = t == 0 ? tab.gen64[gen_range_of(W)]
                                  : (c.contrib32 != nullptr ? tab.gen32c : tab.gen32)[gen_range_of(W)];
    const size_t ldsb = place != 0 ? static_cast<size_t>(need) : 0;
    if (fn != nullptr)
      ms = time_median([&] { return fn(c, d_b, d_t, (int64_t)tasks.size(), ldsb, p.stream); }, reps, p.stream);
  }
  (void)hipFree(d_b);
  (void)hipFree(d_t);
  (void)hipFree(tmp);
  return ms;
}

// Stream lanes by measurement: starting from the cost-model assignment, move
// one edge stage at a time to another lane and keep the move when the whole
// apply gets faster by more than 0.5 %; repeat while a round finds a move (at
// most four rounds).  A sample is kLaneBatch back-to-back applies (the steady
// state of repeated applies, whose launches overlap across applies), timed
// with hipEvents on the plan's stream; a candidate's time is the median of
// max(reps, 5) samples.  The search's result is then timed against the
// starting assignment in alternation and kept only if it wins, so timing
// noise cannot leave a slower assignment than the cost model's.  The lanes
// never change any bit of y.
constexpr int kLaneBatch = 2;
constexpr float kTuneMargin = 0.97f;   // a stack placement other than the default must be 3 % faster
int tune_lanes(Plan& p, const double* x, int reps) {
  if ((p.flags & STTSV_FLAG_ONE_STREAM) || p.ev_fork == nullptr) return STTSV_OK;
  double* y = nullptr;
  if (hipMalloc(&y, sizeof(double) * static_cast<size_t>(p.n)) != hipSuccess) return STTSV_ENOMEM;
  reps = std::max(reps, 5);
  for (int seq = 0; seq < 2; ++seq) {
    const int nl = p.lanes[seq];
    if (nl < 2) continue;
    const int prec = seq == 0 ? STTSV_PREC_FP64 : STTSV_PREC_FP32;
    auto apply = [&] {
      hipError_t e = hipSuccess;
      for (int q = 0; q < kLaneBatch && e == hipSuccess; ++q) e = launch_sttsv(p, x, y, prec, nullptr, p.stream);
      return e;
    };
    auto lanes_now = [&] {
      std::vector<int> v;
      for (const Stage& S : p.stages[seq]) v.push_back(S.lane);
      return v;
    };
    auto set_lanes = [&](const std::vector<int>& v) {
      for (size_t i = 0; i < v.size(); ++i) p.stages[seq][i].lane = v[i];
    };
    const std::vector<int> start = lanes_now();
    float best = time_median(apply, reps, p.stream);
    for (int round = 0; round < 4; ++round) {
      bool moved = false;
      for (Stage& S : p.stages[seq]) {
        if (S.type != 0 && S.type != 1) continue;
        const int from = S.lane;
        for (int l = 0; l < nl; ++l) {
          if (l == from || S.lane != from) continue;
          S.lane = l;
          const float t = time_median(apply, reps, p.stream);
          if (t < 0.995f * best) {
            best = t;
            moved = true;
          } else {
            S.lane = from;
          }
        }
      }
      if (!moved) break;
    }
    const std::vector<int> found = lanes_now();
    if (found != start) {
      float t_found = 0.f, t_start = 0.f;
      for (int round = 0; round < 3; ++round) {
        set_lanes(start);
        t_start += time_median(apply, reps, p.stream);
        set_lanes(found);
        t_found += time_median(apply, reps, p.stream);
      }
      if (!(t_found < t_start)) set_lanes(start);
    }
  }
  const hipError_t e = hipStreamSynchronize(p.stream);
  (void)hipFree(y);
  return e == hipSuccess ? STTSV_OK : STTSV_EHIP;
}

}  // namespace

int autotune(Plan& p, const double* x, int reps, const char* cache_path, int32_t* tuned) {
  if (x == nullptr || reps < 1) return STTSV_EINVAL;
  load_cache(cache_path);
  const EdgeTables& tab = edge_tables();
  // the edge kernels gather from the rank-ordered copies of x: the first
  // stage of an FP32 apply makes both (FP64 and FP32, when the plan's FP32
  // applies run compact); FP32-series kernels are timed as an FP32 apply
  // runs them
  if (launch_stage(p, 0, x, nullptr, STTSV_PREC_FP32, nullptr, p.stream) != hipSuccess) return STTSV_EHIP;
  const EdgeCall c64{p.d_xr, p.d_contrib, nullptr, nullptr, nullptr, nullptr};
  const EdgeCall c32 = p.compact_ok ? EdgeCall{p.d_xr, p.d_contrib, nullptr, nullptr, p.d_xr32, p.d_contrib32} : c64;
  int count = 0;
  for (Bucket& B : p.buckets) {
    if (B.k < 4) continue;
    const int W = B.r - B.k + 1;
    for (int t = 0; t < 2; ++t) {
      if (t == 1 && !B.fp32_ok) continue;
      if (B.coop[t] > 0) continue;        // lane-group kernel: no bit-identical alternative
      const std::string key = key_of(t, B);
      Choice ch{-1, -1, -1};
      bool cached = false;
      {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
          ch = it->second;
          cached = true;
        }
      }
      const EdgeCall& c = t == 0 ? c64 : c32;
      const auto& small = t == 0 ? tab.small64 : (c.contrib32 != nullptr ? tab.small32c : tab.small32);
      const SmallLaunchFn kr = (B.k <= 7 && !(p.flags & STTSV_FLAG_GENERIC_ONLY)) ? small[SK_R4 + (B.k - 4)][W] : nullptr;
      if (!cached) {
        const float g_lds = time_generic(p, B, t, 1, c, reps);
        const float g_glb = time_generic(p, B, t, 0, c, reps);
        const float g_free = stack_free_ok(W, t == 0 ? 8 : 4) ? time_generic(p, B, t, kStackFree, c, reps) : 1e30f;
        const float g_best = std::min(g_lds, std::min(g_glb, g_free));
        // the planner's default placement unless another is clearly faster
        // (near-ties would flip with timing noise from run to run)
        const int tsz = t == 0 ? 8 : 4;
        const bool def_lds = (int64_t)kGenBlock * kg_stack_bytes(B.k, W, tsz) <= kLdsBudget;
        const float g_def = def_lds ? g_lds : g_glb;
        if (g_best < kTuneMargin * g_def)
          ch.lds = g_lds == g_best ? 1 : g_free == g_best ? kStackFree : 0;
        else
          ch.lds = def_lds ? 1 : 0;
        ch.use_kr = -1;
        if (kr != nullptr) {
          const BucketDesc d = B.desc[t];
          float t_kr = time_median([&] { return kr(c, d, p.stream); }, reps, p.stream);
          const SmallLaunchFn fr = t == 0 ? tab.run64[B.k - 4][W] : nullptr;
          if (fr != nullptr) {
            const int saved_kind = B.small_kind[0], saved_pref = B.reuse_pref;
            B.small_kind[0] = SK_R4 + (B.k - 4);
            B.reuse_pref = 1;
            int rc = set_reuse(p, B, false);
            float t_run = 1e30f;
            if (rc == STTSV_OK && B.reuse) {
              const BucketDesc dr = B.desc[0];
              t_run = time_median([&] { return fr(c, dr, p.stream); }, reps, p.stream);
            }
            B.small_kind[0] = saved_kind;
            B.reuse_pref = saved_pref;
            ch.reuse = t_run < t_kr ? 1 : 0;
            t_kr = std::min(t_kr, t_run);
          }
          const float g_chosen = ch.lds == 1 ? g_lds : ch.lds == kStackFree ? g_free : g_glb;
          ch.use_kr = t_kr <= g_chosen ? 1 : 0;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = ch;
        append_cache(cache_path, key, ch);
      }
      if (kr != nullptr && ch.use_kr >= 0) B.small_kind[t] = ch.use_kr == 1 ? SK_R4 + (B.k - 4) : -1;
      if (ch.lds >= 0) B.lds_pref[t] = ch.lds;
      if (t == 0 && ch.reuse >= 0) B.reuse_pref = ch.reuse;
      ++count;
    }
  }
  if (hipStreamSynchronize(p.stream) != hipSuccess) return STTSV_EHIP;
  free_solver(p);                 // the captured launch sequences change
  free_zstate(p);
  int rc = STTSV_OK;
  for (Bucket& B : p.buckets)
    if (rc == STTSV_OK) rc = set_reuse(p, B, (p.flags & STTSV_FLAG_PREFIX_REUSE) != 0);
  if (rc == STTSV_OK) rc = build_groups(p);
  if (rc == STTSV_OK) rc = assign_places(p);   // the die of an edge follows its kernel
  if (rc != STTSV_OK) return rc;
  build_stages(p);
  if ((rc = tune_lanes(p, x, reps)) != STTSV_OK) return rc;
  if (tuned != nullptr) *tuned = count;
  return STTSV_OK;
}

}  // namespace sttsv
