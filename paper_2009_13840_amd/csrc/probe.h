// Live timing of selected kernel launches during a solve.  While a class of
// kernels is armed, every `stride`-th launch of it (per class and level) carries
// a start and a stop HIP event that the runtime stamps from the kernel's own
// dispatch (hipExtLaunchKernelGGL), on the launch's stream, so the elapsed time
// is the kernel's execution without the dispatch latency that separately
// recorded events would add; after the stream has finished the host sums the
// elapsed times per (class, level).  Sampling keeps the host's event calls from
// slowing a stream of short launches.  Events come from a pool that is reused
// from one read to the next.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hho {

constexpr int kProbeClasses = 10, kProbeLevels = 16;

struct KernelProbe {
  unsigned mask = 0;  // armed classes (HHO_PROBE_* bits)
  int stride = 1;     // time one launch in `stride` of each (class, level)
  int64_t seen[kProbeClasses][kProbeLevels] = {};  // launches of each armed (class, level)
  struct Rec {
    int kind, level;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;       // recorded pairs since the last read
  std::vector<hipEvent_t> pool;  // created events, reused
  size_t next = 0;             // next free event of the pool
  bool failed = false;         // an event call failed: the read reports it

  hipEvent_t take() {
    if (next == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        failed = true;
        return nullptr;
      }
      pool.push_back(e);
    }
    return pool[next++];
  }
  static int class_index(int kind) {
    int i = 0;
    while (i < kProbeClasses && !((unsigned)kind & (1u << i))) ++i;
    return i;
  }
  // returns the index of the opened record, or -1 when the class is not armed
  // or this launch is not sampled; the events wait in the thread's launch slot
  // for the next HHO_LAUNCH
  int begin(int kind, int level) {
    if (!(mask & (unsigned)kind)) return -1;
    const int ci = class_index(kind), li = level < 0 ? 0 : (level < kProbeLevels ? level : kProbeLevels - 1);
    if (ci >= kProbeClasses || seen[ci][li]++ % stride != 0) return -1;
    hipEvent_t a = take(), b = take();
    if (!a || !b) return -1;
    recs.push_back({kind, level, a, b});
    launch_slot() = {a, b};
    return (int)recs.size() - 1;
  }
  // after the launch statement: a slot still holding the events means that no
  // HHO_LAUNCH consumed them, so the record is dropped
  void end(int idx) {
    if (idx < 0) return;
    LaunchSlot &ls = launch_slot();
    if (ls.a) {
      ls = {};
      recs.pop_back();
    }
  }
  struct LaunchSlot {
    hipEvent_t a = nullptr, b = nullptr;
  };
  static LaunchSlot &launch_slot() {
    static thread_local LaunchSlot slot;
    return slot;
  }
  void reset() {
    launch_slot() = {};
    recs.clear();
    next = 0;
    failed = false;
    for (auto &row : seen)
      for (int64_t &c : row) c = 0;
  }
  ~KernelProbe() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// times one launch statement (when its class is armed and the launch sampled)
#define HHO_PROBED(probe, kind, level, stream, launch)                          \
  do {                                                                          \
    const int pidx_ = (probe) ? (probe)->begin((kind), (level)) : -1;           \
    launch;                                                                     \
    if (pidx_ >= 0) (probe)->end(pidx_);                                        \
  } while (0)

// a kernel launch that takes the events a probe left in the thread's slot
#define HHO_LAUNCH(kernel, grid, block, shmem, stream, ...)                                          \
  do {                                                                                               \
    ::hho::KernelProbe::LaunchSlot &ls_ = ::hho::KernelProbe::launch_slot();                         \
    if (ls_.a) {                                                                                     \
      const hipEvent_t a_ = ls_.a, b_ = ls_.b;                                                       \
      ls_ = {};                                                                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, a_, b_, 0, __VA_ARGS__);             \
    } else {                                                                                         \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                           \
    }                                                                                                \
  } while (0)

}  // namespace hho
