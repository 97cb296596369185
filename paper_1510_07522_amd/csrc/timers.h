// Optional per-kernel-class timing with HIP events on the launching stream.
// When enabled, launches wrapped in KernelTimer record an event pair; the
// totals are read (after a stream synchronisation) through the C ABI.
#pragma once
#include "common.h"

namespace rsrr {

bool timers_on();
// Brackets one launch: construct before, destroy after the launch.
struct KernelTimer {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  double flops, bytes;
  KernelTimer(const char* n, hipStream_t st, double fl = 0, double by = 0);
  ~KernelTimer();
};

}  // namespace rsrr
