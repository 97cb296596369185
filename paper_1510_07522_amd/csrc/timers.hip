// Per-kernel-class timers (HIP events) and their C ABI.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rsrr.h"
#include "timers.h"

namespace rsrr {

namespace {
struct Rec { hipEvent_t a, b; double flops, bytes; std::string sym; };
struct Acc { long launches = 0; double ms = 0, flops = 0, bytes = 0; };
std::mutex g_mu;
bool g_on = false;
std::string g_only;   // when set, only launches of this kernel function are timed
std::map<std::string, std::vector<Rec>> g_pending;
std::map<std::string, Acc> g_acc;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
  if (!g_pool.empty()) { hipEvent_t e = g_pool.back(); g_pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  return e;
}

void drain() {   // caller holds g_mu
  for (auto& kv : g_pending) {
    Acc& acc = g_acc[kv.first];
    for (auto& r : kv.second) {
      float ms = 0;
      if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
          hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        acc.launches += 1;
        acc.ms += ms;
        acc.flops += r.flops;
        acc.bytes += r.bytes;
        if (!r.sym.empty()) {
          Acc& as = g_acc["sym:" + r.sym];
          as.launches += 1;
          as.ms += ms;
          as.flops += r.flops;
          as.bytes += r.bytes;
        }
      }
      if (r.a) g_pool.push_back(r.a);
      if (r.b) g_pool.push_back(r.b);
    }
    kv.second.clear();
  }
}
}  // namespace

bool timers_on() { return g_on; }

KernelTimer::KernelTimer(const char* n, hipStream_t st, double fl, double by, std::string symbol)
    : name(n), s(st), flops(fl), bytes(by), sym(std::move(symbol)) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_only.empty() && sym != g_only) return;
  a = take();
  if (a) (void)hipEventRecord(a, s);
}

KernelTimer::~KernelTimer() {
  if (!g_on || !a) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = take();
  if (b) (void)hipEventRecord(b, s);
  g_pending[name].push_back(Rec{a, b, flops, bytes, sym});
}

}  // namespace rsrr

using namespace rsrr;

extern "C" {

void rsrr_timers_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
}

void rsrr_timers_only(const char* sym) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_only = sym ? sym : "";
}

void rsrr_timers_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain();
  g_acc.clear();
}

int rsrr_timers_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain();
  return (int)g_acc.size();
}

int rsrr_timers_get(int index, char* name, int name_len, long long* launches, double* total_ms,
                    double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain();
  if (index < 0 || index >= (int)g_acc.size()) return set_error(ST_EINVAL, "timer index out of range");
  auto it = g_acc.begin();
  std::advance(it, index);
  if (name && name_len > 0) {
    snprintf(name, name_len, "%s", it->first.c_str());
  }
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  if (flops) *flops = it->second.flops;
  if (bytes) *bytes = it->second.bytes;
  return ST_OK;
}

}  // extern "C"
