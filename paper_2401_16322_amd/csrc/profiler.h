// Optional per-launch timing of the library's kernels with HIP events on the
// launch stream, plus the algorithmic HBM bytes of each launch (every operand
// array counted once per launch, halos not counted).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "expwave.h"

namespace expw {

class Profiler {
 public:
  // The destructor makes no HIP call (a handle may be destroyed while the
  // process exits, after the runtime has shut down); release() frees the
  // events while the runtime is alive.
  void release() {
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
    pool_.clear();
    recs_.clear();
    used_ = 0;
  }

  bool active() const { return mask_ != 0; }

  // mask: bit k enables timing of kernel class k (0 = off)
  void enable(uint32_t mask) {
    mask_ = mask;
    recs_.clear();
    used_ = 0;
    for (int k = 0; k < EXPW_KERNEL_CLASSES; ++k) {
      ms_[k] = 0.0;
      bytes_[k] = 0.0;
      launches_[k] = 0;
    }
  }

  // A start/stop event pair for the next launch of class kind, to be attached
  // to the dispatch itself; returns its slot (-1 when that class is not timed).
  int acquire(int kind, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!(mask_ >> kind & 1u)) return -1;
    while (pool_.size() < used_ + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool_.push_back(e);
    }
    const int slot = static_cast<int>(used_);
    used_ += 2;
    *e0 = pool_[slot];
    *e1 = pool_[slot + 1];
    return slot;
  }

  void commit(int slot, int kind, double bytes) {
    if (slot >= 0) recs_.push_back({kind, slot, bytes});
  }

  // Waits for the recorded launches and folds them into the per-class totals.
  bool collect() {
    for (const Rec& r : recs_) {
      if (hipEventSynchronize(pool_[r.slot + 1]) != hipSuccess) return false;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pool_[r.slot], pool_[r.slot + 1]) != hipSuccess) return false;
      ms_[r.kind] += ms;
      bytes_[r.kind] += r.bytes;
      launches_[r.kind] += 1;
    }
    recs_.clear();
    used_ = 0;
    return true;
  }

  double ms(int k) const { return ms_[k]; }
  double bytes(int k) const { return bytes_[k]; }
  int64_t launches(int k) const { return launches_[k]; }

 private:
  struct Rec {
    int kind;
    int slot;
    double bytes;
  };
  uint32_t mask_ = 0;
  std::vector<hipEvent_t> pool_;
  size_t used_ = 0;
  std::vector<Rec> recs_;
  double ms_[EXPW_KERNEL_CLASSES] = {};
  double bytes_[EXPW_KERNEL_CLASSES] = {};
  int64_t launches_[EXPW_KERNEL_CLASSES] = {};
};

// Launches kernel on stream st. When kind is a timed class, the profiler's
// events are attached to the dispatch (hipExtLaunchKernel), so they hold the
// kernel's own start and end times.
// Launch errors surface through hipGetLastError() at the caller's next check.
template <typename F, typename... Args>
void launch_timed(Profiler* prof, hipStream_t st, int kind, double bytes, F kernel, dim3 grid,
                  dim3 block, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int slot = prof ? prof->acquire(kind, &e0, &e1) : -1;
  if (slot < 0) {
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
  prof->commit(slot, kind, bytes);
}

}  // namespace expw
