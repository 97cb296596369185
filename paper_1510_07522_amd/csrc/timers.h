// Optional per-kernel-class timing with HIP events on the launching stream.
// When enabled, launches wrapped in KernelTimer record an event pair; the
// totals are read (after a stream synchronisation) through the C ABI.
#pragma once
#include <string>

#include "common.h"

namespace rsrr {

bool timers_on();
// Brackets one launch: construct before, destroy after the launch.
// `sym` (optional) names the kernel function as a profiler lists it; the
// launch is then also accumulated under "sym:<sym>".
struct KernelTimer {
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  double flops, bytes;
  std::string sym;
  KernelTimer(const char* n, hipStream_t st, double fl = 0, double by = 0, std::string symbol = std::string());
  ~KernelTimer();
};

}  // namespace rsrr
