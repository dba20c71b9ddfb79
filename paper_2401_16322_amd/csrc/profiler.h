// Optional per-launch timing of the library's kernels with HIP events on the
// launch stream, plus the algorithmic HBM bytes of each launch (every operand
// array counted once per launch, halos not counted).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "expwave.h"

namespace expw {

class Profiler {
 public:
  ~Profiler() {
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
  }

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

  // Records a start event before a launch of class kind; returns its slot
  // (-1 when that class is not timed).
  int begin(hipStream_t st, int kind) {
    if (!(mask_ >> kind & 1u)) return -1;
    while (pool_.size() < used_ + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      pool_.push_back(e);
    }
    const int slot = static_cast<int>(used_);
    used_ += 2;
    (void)hipEventRecord(pool_[slot], st);
    return slot;
  }

  void end(hipStream_t st, int slot, int kind, double bytes) {
    if (slot < 0) return;
    (void)hipEventRecord(pool_[slot + 1], st);
    recs_.push_back({kind, slot, bytes});
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

}  // namespace expw
