// Declarations shared by the batched path (ds_batched.hip) and the batched
// learned method (ds_learned.hip).
#pragma once

#include "ds_internal.h"

namespace ds {

constexpr int32_t kBmInvalid = -1;   // report value: X_k not strictly increasing or not finite
constexpr int32_t kBmTrivial = -2;   // report value: N_k <= 0
constexpr int kNumQueues = 8;        // one tile queue per XCD
constexpr int kRouterParams = 1153;  // 1 -> 32 -> 32 -> 1 router
constexpr int kSegFitBytes = 32;
constexpr int kBatchLearnSamples = 2048;  // training samples per array and step
// Training steps of a batched model when none are asked for.  From the quantile
// starting point (init_params_kernel) more steps do not narrow the windows:
// on the 256-array mixture the search takes the same time after 1 to 40
// steps, and each step costs about 44 us for 256 models.
constexpr int kBatchLearnStepsDefault = 2;
constexpr int kBatchMaxSegments = 4096;   // the search stages a model's fits, steps and grid in LDS

template <typename T>
struct alignas(16) ArrMeta {
  T H, W, X0, XN;
  int64_t x_off;    // first value of the array in X_packed
  int64_t q_off;    // first query
  int64_t q_end;    // one past the last query
  int64_t w_off;    // first RANKCODE word in the word pool
  int64_t c_off;    // first code in the code pool
  int64_t t_off;    // first tile of the array
  int32_t N, R, jmin, nW;
  int32_t method;   // DS_METHOD_DIRECT, _BSEARCH_OFFSET, _LEARNED, kBmInvalid, kBmTrivial
  int32_t n_updates;
  int32_t slot;     // learned: index of the array's model
  int32_t pad;
  // build accumulators, merged by atomics across the chunks of the array
  unsigned long long gbits;  // bits of the minimum rounded gap (a float >= 0)
  uint32_t flags;            // 1 not finite, 2 not increasing, 4 X_i - X_0 not increasing
  int32_t first_bad;         // first i whose cell equals that of X_{i-1} at the starting H
};

struct PlanTotals {
  int64_t total_tiles;
  int64_t learned_tiles;        // tiles of learned arrays (the rest are Direct / binary search)
  int64_t words_used;
  uint32_t queue[kNumQueues];   // Direct / binary-search tiles
  uint32_t lqueue[kNumQueues];  // learned tiles
  int32_t n_learned;
  uint32_t long_segs;  // long segments queued by the learned fit (batched learned build)
  unsigned long long fallbacks;  // learned queries that left their window
};

// per learned array: the feature's constants and where its keys are
struct alignas(16) LearnMeta {
  double X0, XN, delta, flo, fscale;
  int64_t x_off;
  int32_t N;
  int32_t k;   // array index
};

// A segment whose fit range holds more than kFitLongKeys keys is fitted by a
// whole workgroup (seg_fit_long_kernel); the build queues it as (model slot,
// segment).  Such a segment holds at least kFitLongKeys - 1 keys of its own,
// so a batch of total_x keys queues at most total_x / (kFitLongKeys - 1).
constexpr int kFitLongKeys = 8192;
struct LongSeg {
  int32_t slot, s;
};

// device pointers of the batched learned method inside the workspace
struct BatchLearned {
  const void* meta;        // ArrMeta<T>[K]
  const int64_t* tile_off;
  PlanTotals* tot;
  int32_t K;
  int32_t nseg;
  int32_t steps;     // training steps (0 with the identity router)
  int32_t identity;  // 1: no network, segments of the feature itself (the ablation)
  int32_t log2g;     // cells of each model's router grid (2^log2g)
  int32_t pad_;
  uint64_t seed;
  int64_t tile;
  int64_t total_x;         // values in the packed X (reads never pass its end)
  const void* X;
  const void* z;
  int32_t* out;
  LearnMeta* lmeta;        // [K] (first n_learned used)
  float* params;           // [K][kRouterParams]
  float* adam_m;
  float* adam_v;
  float* steps_tab;        // [K][nseg] compiled router steps
  uint32_t* grid;          // [K][2^log2g] compiled router grid
  void* segs;              // [K][nseg] segment fits
  int32_t* first;          // [K][nseg + 1]
  LongSeg* longs;          // queue of long segments, total_x / (kFitLongKeys - 1) + 1 entries
  void* samples;           // first value of every 64-byte block of X, then +inf
};

// The largest k in [0, n) with off[k] <= g (off non-decreasing, off[0] <= g),
// found by one whole wave with 64 probes per round: log64 n dependent loads
// instead of log2 n.  Every lane of the wave must call it; all get the answer.
__device__ __forceinline__ int32_t wave_last_le(const int64_t* __restrict__ off, int32_t n, int64_t g) {
  const int lane = threadIdx.x & 63;
  int32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int32_t stride = (hi - lo + 63) / 64;
    const int64_t p = int64_t(lo) + int64_t(lane) * stride;
    // the probes at or below the answer are a prefix of the lanes
    const int c = __popcll(__ballot(p < hi && off[p] <= g));
    lo += (c > 0 ? c - 1 : 0) * stride;
    hi = (hi - lo < stride) ? hi : lo + stride;
  }
  return lo;
}

// implemented in ds_learned.hip
int32_t batch_grid_log2(int32_t nseg);  // grid cells of a batched model's compiled router (log2)
ds_status batched_learned_build(const BatchLearned& b, int dtype, hipStream_t s);
ds_status batched_learned_search(const BatchLearned& b, int dtype, hipStream_t s);

}  // namespace ds
