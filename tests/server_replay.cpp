// Host-only replay of the serving loop's scheduler (server_sched.h) with a
// mock device side: each request "runs" by sleeping for a modelled latency
// and keeps an arena of a fixed fraction of its admission bound, so the
// admission, memory-release and wake-up logic runs exactly as in the library,
// without a GPU.  Request needs come from the library's own workspace bound.
//
// Input (stdin): "budget_gib slots time_scale watchdog_s" on the first line,
// then one request per line: "t_arrival family n N L" (family 0 QEP, 1 delay,
// 2 BEM).  Requests are submitted at their (scaled) arrival times from one
// thread and waited for in order with a bounded wait.  Exit 0 when every
// request finished and the held memory never exceeded the budget; prints one
// line per request and a summary.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "../paper_1510_07522_amd/csrc/bounds.h"
#include "../paper_1510_07522_amd/csrc/server_sched.h"

namespace {

struct Req {
  double t = 0;
  int family = 0, n = 0, N = 0, L = 0;
  size_t need = 0;
  double latency = 0;
};

struct MockOps : rsrr::sched::SlotOps {
  std::vector<size_t> arena;
  std::mutex mu;
  size_t held = 0, peak = 0, budget = 0;
  std::atomic<int> running{0}, max_running{0};
  bool over = false;
  double scale = 1.0;

  explicit MockOps(int slots) : arena(slots, 0) {}
  size_t arena_bytes(int s) override {
    std::lock_guard<std::mutex> lk(mu);
    return arena[s];
  }
  void release_arena(int s) override {
    std::lock_guard<std::mutex> lk(mu);
    held -= arena[s];
    arena[s] = 0;
  }
  int run(int s, void* payload) override {
    const Req& r = *(const Req*)payload;
    {
      // the solve grows the slot's arena to what it actually uses (a fraction
      // of the bound, as measured on the device)
      std::lock_guard<std::mutex> lk(mu);
      const size_t use = (size_t)(0.7 * r.need);
      if (use > arena[s]) {
        held += use - arena[s];
        arena[s] = use;
      }
      peak = std::max(peak, held);
      if (held > budget) over = true;
    }
    const int now_running = ++running;
    int prev = max_running.load();
    while (now_running > prev && !max_running.compare_exchange_weak(prev, now_running)) {}
    std::this_thread::sleep_for(std::chrono::duration<double>(r.latency * scale));
    --running;
    return 0;
  }
};

double modelled_latency(const Req& r) {
  // seconds on the device, roughly: a fixed part plus the n^3 work of the
  // sampling LUs and of the reduced problem (k_S = min(n, N L))
  const double n = r.n, kS = std::min<double>(r.n, (double)r.N * r.L);
  return 0.2 + 1.5 * r.N / 48.0 * std::pow(n / 2048.0, 3) + 2.5 * std::pow(kS / 2048.0, 3);
}

}  // namespace

int main() {
  double budget_gib = 0, scale = 1, dog = 0;
  int slots = 0;
  if (scanf("%lf %d %lf %lf", &budget_gib, &slots, &scale, &dog) != 4) return 2;
  std::vector<Req> reqs;
  Req r;
  while (scanf("%lf %d %d %d %d", &r.t, &r.family, &r.n, &r.N, &r.L) == 5) reqs.push_back(r);
  rsrr_params prm;
  memset(&prm, 0, sizeof(prm));
  prm.NS = 512;
  prm.K = 2;
  prm.nb = 64;
  prm.precision = RSRR_PREC_C64_IR;
  prm.cheb_degree = 40;
  prm.chunk_gib = 24.0;
  for (Req& q : reqs) {
    prm.N = q.N;
    prm.L = q.L;
    const size_t U = (size_t)q.n * q.L * 16;
    q.need = rsrr::workspace_bound(q.n, 3, q.family == 2, &prm) + U;
    q.latency = modelled_latency(q);
  }
  const size_t budget = (size_t)(budget_gib * 1073741824.0);
  MockOps ops(slots);
  ops.budget = budget;
  ops.scale = scale;
  rsrr::sched::Scheduler sch(budget, slots, &ops, dog);
  sch.start();
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  std::vector<uint64_t> tickets(reqs.size(), 0);
  std::vector<int> refused(reqs.size(), 0);
  std::thread submitter([&] {
    for (size_t i = 0; i < reqs.size(); ++i) {
      std::this_thread::sleep_until(t0 + std::chrono::duration_cast<clk::duration>(
                                             std::chrono::duration<double>(reqs[i].t * scale)));
      void* pl = &reqs[i];
      if (sch.submit(reqs[i].need, pl, &tickets[i]) != rsrr::sched::SUBMIT_OK) refused[i] = 1;
    }
  });
  submitter.join();
  int done = 0, timeouts = 0;
  double lat_max = 0;
  for (size_t i = 0; i < reqs.size(); ++i) {
    if (refused[i]) {
      printf("request %zu refused (needs %.1f GiB)\n", i + 1, reqs[i].need / 1073741824.0);
      continue;
    }
    void* pl = nullptr;
    int st = 0;
    double lat = 0;
    // generous bound: the whole stream's modelled work, scaled
    double total = 0;
    for (const Req& q : reqs) total += q.latency;
    const int w = sch.wait(tickets[i], 10.0 + 2.0 * total * scale, &pl, &st, &lat);
    if (w != rsrr::sched::WAIT_DONE) {
      ++timeouts;
      printf("request %zu: wait ended without a result (%d)\n%s", i + 1, w, sch.state().c_str());
      break;
    }
    ++done;
    lat_max = std::max(lat_max, lat / scale);
    printf("request %zu: family %d n %d L %d need %.1f GiB latency %.3f (modelled s)\n", i + 1,
           reqs[i].family, reqs[i].n, reqs[i].L, reqs[i].need / 1073741824.0, lat / scale);
  }
  // two waiters of one ticket: one receives the result, the other learns
  // that the ticket is gone (no access to a removed job)
  Req extra;
  extra.need = 1;
  extra.latency = 0.05;
  uint64_t tk = 0;
  bool dbl_ok = sch.submit(extra.need, &extra, &tk) == rsrr::sched::SUBMIT_OK;
  int wa = -1, wb = -1;
  if (dbl_ok) {
    std::thread ta([&] {
      void* p = nullptr;
      int st = 0;
      double l = 0;
      wa = sch.wait(tk, 30.0, &p, &st, &l);
    });
    std::thread tb([&] {
      void* p = nullptr;
      int st = 0;
      double l = 0;
      wb = sch.wait(tk, 30.0, &p, &st, &l);
    });
    ta.join();
    tb.join();
    dbl_ok = (wa == rsrr::sched::WAIT_DONE) != (wb == rsrr::sched::WAIT_DONE) &&
             (wa == rsrr::sched::WAIT_UNKNOWN || wb == rsrr::sched::WAIT_UNKNOWN);
  }
  printf("double wait: %s (%d, %d)\n", dbl_ok ? "ok" : "FAILED", wa, wb);
  sch.stop();
  int nref = 0;
  for (int v : refused) nref += v;
  printf("summary: %d done, %d refused, %d timeouts, peak held %.1f of %.1f GiB, max concurrent %d, "
         "max latency %.2f, over budget %d\n", done, nref, timeouts, ops.peak / 1073741824.0, budget_gib,
         ops.max_running.load(), lat_max, ops.over ? 1 : 0);
  return (timeouts == 0 && done + nref == (int)reqs.size() && !ops.over && dbl_ok) ? 0 : 1;
}
