// Serving: continuous batching of complete solves (Alg. 2) on one device.
//
// A server owns max_slots execution slots.  Each slot is one host worker
// thread with its own non-blocking, default-priority HIP stream and its own
// device workspace; a slot runs one request at a time, so up to max_slots
// solves overlap on the device.  Requests wait in one FIFO queue and are
// admitted, in order, as soon as a slot is free and their device memory fits
// the budget:
//
//   sum over the other slots of held(t)  +  max(need(r), arena(s))  <=  budget
//
// need(r) is the workspace bound of the request (solve_workspace_bound);
// held(t) is max(need, arena) for a running slot and the arena it keeps for
// an idle one.  An idle slot gives its arena back when the head of the queue
// is waiting for memory.  A request whose bound alone exceeds the budget is
// refused at submission (RSRR_EBUSY).  Every kernel on the path is
// deterministic (no floating-point atomics, fixed reduction orders), so a
// request returns bit-identical results alone or in a mix.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "driver.h"

using namespace rsrr;

namespace {

struct Request {
  rsrr_problem* p = nullptr;
  rsrr_contour c{};
  rsrr_params prm{};
  std::vector<c128> U;          // host copy of the probing matrix (empty: seeded)
  size_t need = 0;
  double t_submit = 0, latency = 0;
  int status = 0;
  bool done = false;
  rsrr_result* res = nullptr;
  std::string err;
};

struct Slot {
  std::thread th;
  hipStream_t stream = nullptr;
  rsrr_problem view;            // aliases the request's problem; owns only the workspace
  size_t held = 0;
  bool busy = false;
};

}  // namespace

struct rsrr_server {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Request> reqs;
  std::vector<Slot*> slots;
  size_t budget = 0;
  uint64_t next_ticket = 1;
  uint64_t gen = 0;             // bumped whenever memory is freed or a request ends
  bool stop = false;
  int device = 0;
};

namespace {

// The view shares the problem's device data (coefficients, BEM points) and
// host descriptors; it never frees them.
void bind_view(rsrr_problem* v, const rsrr_problem* p, hipStream_t s) {
  v->n = p->n;
  v->J = p->J;
  v->bem = p->bem;
  v->kinds = p->kinds;
  v->fns = p->fns;
  v->mats = p->mats;
  v->gram = p->gram;
  v->xyz = p->xyz;
  v->h = p->h;
  v->stream = s;
}

void unbind_view(rsrr_problem* v) {
  v->mats.clear();
  v->xyz = nullptr;
}

size_t others_held(const rsrr_server* srv, const Slot* self) {
  size_t b = 0;
  for (const Slot* t : srv->slots)
    if (t != self) b += t->held;
  return b;
}

void worker(rsrr_server* srv, Slot* sl) {
  (void)hipSetDevice(srv->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    srv->cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
    if (srv->queue.empty()) break;                       // stop and drained
    const uint64_t ticket = srv->queue.front();
    Request& r = srv->reqs[ticket];
    const size_t own = sl->view.ws.bytes();
    const size_t others = others_held(srv, sl);
    if (others + std::max(r.need, own) > srv->budget) {
      if (own > 0) {                                     // give the idle arena back first
        lk.unlock();
        sl->view.ws.release();
        lk.lock();
        sl->held = 0;
        ++srv->gen;
        srv->cv.notify_all();
        continue;
      }
      const uint64_t g0 = srv->gen;                      // wait for memory to be freed
      srv->cv.wait(lk, [&] { return srv->gen != g0 || srv->queue.empty() || srv->queue.front() != ticket; });
      continue;
    }
    srv->queue.pop_front();
    sl->busy = true;
    sl->held = std::max(r.need, own);
    ++srv->gen;                                          // the head changed: others look again
    srv->cv.notify_all();
    lk.unlock();

    bind_view(&sl->view, r.p, sl->stream);
    rsrr_result* res = new rsrr_result();
    memset(&res->info, 0, sizeof(res->info));
    const c128* Ud = nullptr;
    int st = ST_OK;
    if (!r.U.empty()) {
      c128* d = nullptr;
      st = sl->view.ws.get<c128>("srv_U", r.U.size(), &d);
      if (st == ST_OK && hipMemcpyAsync(d, r.U.data(), r.U.size() * sizeof(c128), hipMemcpyHostToDevice,
                                        sl->stream) != hipSuccess)
        st = set_error(ST_EHIP, "server: upload of U failed");
      Ud = d;
    }
    if (st == ST_OK) st = solve_impl(&sl->view, &r.c, &r.prm, Ud, res);
    (void)hipStreamSynchronize(sl->stream);
    unbind_view(&sl->view);
    const char* msg = st < 0 ? rsrr_last_error() : "";
    const size_t arena = sl->view.ws.bytes();

    lk.lock();
    Request& rr = srv->reqs[ticket];
    rr.status = st;
    rr.latency = now_s() - rr.t_submit;
    if (st < 0) {
      rr.err = msg;
      delete res;
    } else {
      res->info.status = st;
      rr.res = res;
    }
    rr.done = true;
    sl->busy = false;
    sl->held = arena;
    ++srv->gen;
    srv->cv.notify_all();
  }
}

}  // namespace

int rsrr_server_create(rsrr_server** out, size_t hbm_budget_bytes, int max_slots) {
  if (!out) return set_error(ST_EINVAL, "rsrr_server_create: null output");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16) return set_error(ST_EINVAL, "max_slots=%d outside [1, 16]", max_slots);
  if (hbm_budget_bytes == 0) return set_error(ST_EINVAL, "zero memory budget");
  rsrr_server* srv = new rsrr_server();
  srv->budget = hbm_budget_bytes;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return set_error(ST_EHIP, "hipGetDevice failed");
  }
  for (int i = 0; i < max_slots; ++i) {
    Slot* sl = new Slot();
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      delete sl;
      rsrr_server_destroy(srv);
      return set_error(ST_EHIP, "cannot create a slot stream");
    }
    srv->slots.push_back(sl);
  }
  for (Slot* sl : srv->slots) sl->th = std::thread(worker, srv, sl);
  *out = srv;
  return ST_OK;
}

int rsrr_server_submit(rsrr_server* srv, rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                       const rsrr_complex* U_host, uint64_t* ticket) {
  if (!srv || !ticket) return set_error(ST_EINVAL, "rsrr_server_submit: null argument");
  RSRR_TRY(check_params(p, c, prm));
  Request r;
  r.p = p;
  r.c = *c;
  r.prm = *prm;
  if (U_host) r.U.assign((const c128*)U_host, (const c128*)U_host + (size_t)p->n * prm->L);
  r.need = solve_workspace_bound(p, prm) + r.U.size() * sizeof(c128);
  if (r.need > srv->budget)
    return set_error(ST_EBUSY, "request needs up to %zu bytes of workspace, budget %zu", r.need, srv->budget);
  r.t_submit = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return set_error(ST_EINVAL, "server is shutting down");
  const uint64_t t = srv->next_ticket++;
  srv->reqs.emplace(t, std::move(r));
  srv->queue.push_back(t);
  *ticket = t;
  srv->cv.notify_all();
  return ST_OK;
}

int rsrr_server_wait(rsrr_server* srv, uint64_t ticket, rsrr_result** out, double* latency_s) {
  if (!srv || !out) return set_error(ST_EINVAL, "rsrr_server_wait: null argument");
  *out = nullptr;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return set_error(ST_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  srv->cv.wait(lk, [&] { return it->second.done; });
  Request& r = it->second;
  const int st = r.status;
  if (latency_s) *latency_s = r.latency;
  *out = r.res;
  const std::string err = r.err;
  srv->reqs.erase(it);
  lk.unlock();
  if (st < 0) return set_error(st, "%s", err.c_str());
  return st;
}

int rsrr_server_pending(rsrr_server* srv, int* queued, int* running) {
  if (!srv) return set_error(ST_EINVAL, "rsrr_server_pending: null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  int run = 0;
  for (const Slot* s : srv->slots) run += s->busy ? 1 : 0;
  if (queued) *queued = (int)srv->queue.size();
  if (running) *running = run;
  return ST_OK;
}

void rsrr_server_destroy(rsrr_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  for (Slot* sl : srv->slots)
    if (sl->th.joinable()) sl->th.join();
  for (Slot* sl : srv->slots) {
    sl->view.ws.release();
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    delete sl;
  }
  for (auto& kv : srv->reqs) delete kv.second.res;   // results nobody waited for
  delete srv;
}
