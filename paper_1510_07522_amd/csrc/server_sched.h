// Admission and slot scheduling of the serving loop, independent of the
// device: the device side supplies a SlotOps (run one request on a slot, the
// memory a slot keeps between requests, give that memory back), so the same
// logic runs in the library and, with a mock SlotOps, in a host-only test.
//
// A scheduler owns `slots` worker threads.  Requests wait in one FIFO queue
// and are admitted, in order, as soon as a slot is free and their device
// memory fits the budget:
//
//   sum over the other slots of held(t)  +  max(need(r), arena(s))  <=  budget
//
// held(t) is max(need, arena) for a running slot and the arena it keeps for an
// idle one.  An idle slot gives its arena back when the head of the queue is
// waiting for memory.  A request whose need alone exceeds the budget is
// refused at submission.  Waits can be bounded; a watchdog thread prints the
// queue and slot state when nothing has been admitted or finished for a while
// although work is pending.
#pragma once
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace rsrr {
namespace sched {

struct SlotOps {
  virtual ~SlotOps() = default;
  // device memory slot `slot` holds between requests (its arena)
  virtual size_t arena_bytes(int slot) = 0;
  // gives that memory back; called only while the slot is idle
  virtual void release_arena(int slot) = 0;
  // runs one request on the slot (no scheduler lock held); returns its status
  virtual int run(int slot, void* payload) = 0;
};

enum { SUBMIT_OK = 0, SUBMIT_TOO_BIG = 1, SUBMIT_STOPPED = 2 };
enum { WAIT_DONE = 0, WAIT_TIMEOUT = 1, WAIT_UNKNOWN = 2 };

class Scheduler {
 public:
  Scheduler(size_t budget, int slots, SlotOps* ops, double watchdog_s)
      : budget_(budget), ops_(ops), watchdog_s_(watchdog_s), slots_(slots) {}
  ~Scheduler() { stop(); }

  void start() {
    t_event_ = now();
    for (int i = 0; i < (int)slots_.size(); ++i) slots_[i].th = std::thread(&Scheduler::worker, this, i);
    if (watchdog_s_ > 0) dog_ = std::thread(&Scheduler::watchdog, this);
  }

  // Queues a request of `need` bytes; *ticket receives its ticket.
  int submit(size_t need, void* payload, uint64_t* ticket) {
    if (need > budget_) return SUBMIT_TOO_BIG;
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return SUBMIT_STOPPED;
    const uint64_t t = next_++;
    Job& j = jobs_[t];
    j.need = need;
    j.payload = payload;
    j.t_submit = now();
    queue_.push_back(t);
    *ticket = t;
    cv_.notify_all();
    return SUBMIT_OK;
  }

  // Waits until the request has run (timeout_s <= 0: no limit).  On WAIT_DONE
  // the job is forgotten and its payload, status and latency are returned.
  int wait(uint64_t ticket, double timeout_s, void** payload, int* status, double* latency) {
    std::unique_lock<std::mutex> lk(mu_);
    if (jobs_.find(ticket) == jobs_.end()) return WAIT_UNKNOWN;
    // the job is looked up again at every wake-up: another waiter of the same
    // ticket, or stop(), may have removed it meanwhile
    auto done = [&] {
      auto f = jobs_.find(ticket);
      return f == jobs_.end() || f->second.done;
    };
    if (timeout_s > 0) {
      if (!cv_.wait_until(lk, deadline(timeout_s), done)) return WAIT_TIMEOUT;
    } else {
      cv_.wait(lk, done);
    }
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return WAIT_UNKNOWN;
    *payload = it->second.payload;
    *status = it->second.status;
    *latency = it->second.latency;
    jobs_.erase(it);
    return WAIT_DONE;
  }

  void pending(int* queued, int* running) {
    std::lock_guard<std::mutex> lk(mu_);
    int run = 0;
    for (const Slot& s : slots_) run += s.busy ? 1 : 0;
    *queued = (int)queue_.size();
    *running = run;
  }

  // Runs everything already submitted, then joins the workers.  Returns the
  // payloads of jobs nobody waited for (the caller frees them).
  std::vector<void*> stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_) return {};
      stop_ = true;
    }
    cv_.notify_all();
    for (Slot& s : slots_)
      if (s.th.joinable()) s.th.join();
    {
      std::lock_guard<std::mutex> lk(mu_);
      dog_stop_ = true;
    }
    dog_cv_.notify_all();
    if (dog_.joinable()) dog_.join();
    std::lock_guard<std::mutex> lk(mu_);
    stopped_ = true;
    std::vector<void*> left;
    for (auto& kv : jobs_) left.push_back(kv.second.payload);
    jobs_.clear();
    return left;
  }

  // One line per slot and one for the queue (the watchdog's report).
  std::string state() {
    std::lock_guard<std::mutex> lk(mu_);
    return state_locked();
  }

 private:
  struct Job {
    size_t need = 0;
    void* payload = nullptr;
    double t_submit = 0, latency = 0;
    int status = 0;
    bool done = false;
  };
  struct Slot {
    std::thread th;
    size_t held = 0;
    bool busy = false;
    uint64_t ticket = 0;
    double t_start = 0;
  };

  // Timed waits use the system clock: libstdc++ then waits with
  // pthread_cond_timedwait, which thread checkers follow (its steady-clock
  // waits use a call they do not intercept and report false races).
  static std::chrono::system_clock::time_point deadline(double seconds) {
    return std::chrono::system_clock::now() +
           std::chrono::duration_cast<std::chrono::system_clock::duration>(std::chrono::duration<double>(seconds));
  }

  static double now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
  }

  size_t others_held(int self) const {
    size_t b = 0;
    for (int i = 0; i < (int)slots_.size(); ++i)
      if (i != self) b += slots_[i].held;
    return b;
  }

  void bump() {   // memory freed, a request admitted or finished: waiting slots look again
    ++gen_;
    t_event_ = now();
    cv_.notify_all();
  }

  void worker(int id) {
    Slot& sl = slots_[id];
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
      if (queue_.empty()) break;                         // stop and drained
      const uint64_t ticket = queue_.front();
      Job& r = jobs_[ticket];
      lk.unlock();
      const size_t own = ops_->arena_bytes(id);          // idle: only this thread touches it
      lk.lock();
      if (queue_.empty() || queue_.front() != ticket) continue;   // taken meanwhile
      sl.held = own;
      if (others_held(id) + std::max(r.need, own) > budget_) {
        if (own > 0) {                                   // give the idle arena back first
          lk.unlock();
          ops_->release_arena(id);
          lk.lock();
          sl.held = 0;
          bump();
          continue;
        }
        const uint64_t g0 = gen_;                        // wait for memory to be freed
        cv_.wait(lk, [&] { return gen_ != g0 || stop_ || queue_.empty() || queue_.front() != ticket; });
        continue;
      }
      queue_.pop_front();
      sl.busy = true;
      sl.ticket = ticket;
      sl.t_start = now();
      sl.held = std::max(r.need, own);
      void* payload = r.payload;
      bump();                                            // the head changed: others look again
      lk.unlock();

      const int st = ops_->run(id, payload);
      const size_t arena = ops_->arena_bytes(id);

      lk.lock();
      Job& rr = jobs_[ticket];
      rr.status = st;
      rr.latency = now() - rr.t_submit;
      rr.done = true;
      sl.busy = false;
      sl.ticket = 0;
      sl.held = arena;
      bump();
    }
  }

  std::string state_locked() const {
    char buf[256];
    std::string s;
    const double t = now();
    size_t held = 0;
    for (int i = 0; i < (int)slots_.size(); ++i) {
      const Slot& sl = slots_[i];
      held += sl.held;
      snprintf(buf, sizeof(buf), "slot %d: %s ticket %llu held %.2f GiB%s\n", i, sl.busy ? "busy" : "idle",
               (unsigned long long)sl.ticket, sl.held / 1073741824.0, "");
      s += buf;
      if (sl.busy) {
        snprintf(buf, sizeof(buf), "  running for %.1f s\n", t - sl.t_start);
        s += buf;
      }
    }
    const Job* head = nullptr;
    if (!queue_.empty()) {
      auto it = jobs_.find(queue_.front());
      if (it != jobs_.end()) head = &it->second;
    }
    snprintf(buf, sizeof(buf), "queue %zu (head ticket %llu needs %.2f GiB), held %.2f of %.2f GiB, gen %llu, "
             "%.1f s since the last admission or completion\n", queue_.size(),
             (unsigned long long)(queue_.empty() ? 0 : queue_.front()), head ? head->need / 1073741824.0 : 0.0,
             held / 1073741824.0, budget_ / 1073741824.0, (unsigned long long)gen_, t - t_event_);
    s += buf;
    return s;
  }

  void watchdog() {
    std::unique_lock<std::mutex> lk(mu_);
    double reported = 0;
    while (!dog_stop_) {
      dog_cv_.wait_until(lk, deadline(std::min(1.0, watchdog_s_)));
      if (dog_stop_) break;
      bool work = !queue_.empty();
      for (const Slot& s : slots_) work |= s.busy;
      const double quiet = now() - t_event_;
      if (work && quiet >= watchdog_s_ && t_event_ != reported) {
        reported = t_event_;
        const std::string st = state_locked();
        fprintf(stderr, "[rsrr server] nothing admitted or finished for %.0f s:\n%s", quiet, st.c_str());
        fflush(stderr);
      }
    }
  }

  std::mutex mu_;
  std::condition_variable cv_, dog_cv_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, Job> jobs_;
  size_t budget_;
  SlotOps* ops_;
  double watchdog_s_;
  std::vector<Slot> slots_;
  std::thread dog_;
  uint64_t next_ = 1, gen_ = 0;
  double t_event_ = 0;
  bool stop_ = false, dog_stop_ = false, stopped_ = false;
};

}  // namespace sched
}  // namespace rsrr
