// Serving: continuous batching of complete solves (Alg. 2) on one device.
//
// The scheduling (FIFO admission by device-memory budget, slots, bounded
// waits, watchdog) is server_sched.h; this file supplies its device side.
// Each slot is one host worker thread with its own non-blocking,
// default-priority HIP stream and its own device workspace; a slot runs one
// request at a time, so up to max_slots solves overlap on the device.
//
// Slots run the LU factorisations without the look-ahead stream: a slot uses
// exactly one stream and never makes it wait for another.  With several slots
// there are more streams than hardware queues (four by default), and streams
// that share a hardware queue are served in submission order; a cross-stream
// wait in one slot could then sit in front of the work another slot's wait
// depends on, and two such waits in two queues block each other for good.
// Every kernel on the path is deterministic (no floating-point atomics, fixed
// reduction orders) and the look-ahead only reorders independent launches, so
// a request returns bit-identical results alone or in a mix.
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "driver.h"
#include "server_sched.h"

using namespace rsrr;

namespace {

struct Request {
  rsrr_problem* p = nullptr;
  rsrr_contour c{};
  rsrr_params prm{};
  std::vector<c128> U;          // host copy of the probing matrix (empty: seeded)
  rsrr_result* res = nullptr;
  std::string err;
};

struct DeviceSlot {
  hipStream_t stream = nullptr;
  rsrr_problem view;            // aliases the request's problem; owns only the workspace
};

struct DeviceOps : sched::SlotOps {
  int device = 0;
  std::vector<DeviceSlot*> slots;

  size_t arena_bytes(int i) override { return slots[i]->view.ws.bytes(); }
  void release_arena(int i) override {
    (void)hipSetDevice(device);
    slots[i]->view.ws.release();
  }
  int run(int i, void* payload) override {
    (void)hipSetDevice(device);
    DeviceSlot* sl = slots[i];
    Request& r = *(Request*)payload;
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
    if (st < 0) {
      r.err = rsrr_last_error();
      delete res;
    } else {
      res->info.status = st;
      r.res = res;
    }
    return st;
  }
};

double watchdog_seconds() {
  const char* e = getenv("RSRR_SERVER_WATCHDOG_S");
  if (!e || !*e) return 120.0;
  return atof(e);
}

}  // namespace

struct rsrr_server {
  DeviceOps ops;
  sched::Scheduler* sch = nullptr;
};

int rsrr_server_create(rsrr_server** out, size_t hbm_budget_bytes, int max_slots) {
  if (!out) return set_error(ST_EINVAL, "rsrr_server_create: null output");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16) return set_error(ST_EINVAL, "max_slots=%d outside [1, 16]", max_slots);
  if (hbm_budget_bytes == 0) return set_error(ST_EINVAL, "zero memory budget");
  rsrr_server* srv = new rsrr_server();
  if (hipGetDevice(&srv->ops.device) != hipSuccess) {
    delete srv;
    return set_error(ST_EHIP, "hipGetDevice failed");
  }
  for (int i = 0; i < max_slots; ++i) {
    DeviceSlot* sl = new DeviceSlot();
    sl->view.ws.no_aux = true;   // one stream per slot (see the note at the top)
    srv->ops.slots.push_back(sl);
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      sl->stream = nullptr;
      rsrr_server_destroy(srv);
      return set_error(ST_EHIP, "cannot create a slot stream");
    }
  }
  srv->sch = new sched::Scheduler(hbm_budget_bytes, max_slots, &srv->ops, watchdog_seconds());
  srv->sch->start();
  *out = srv;
  return ST_OK;
}

int rsrr_server_submit(rsrr_server* srv, rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                       const rsrr_complex* U_host, uint64_t* ticket) {
  if (!srv || !ticket) return set_error(ST_EINVAL, "rsrr_server_submit: null argument");
  RSRR_TRY(check_params(p, c, prm));
  Request* r = new Request();
  r->p = p;
  r->c = *c;
  r->prm = resolve_params(p, prm);
  if (U_host) r->U.assign((const c128*)U_host, (const c128*)U_host + (size_t)p->n * prm->L);
  const size_t need = solve_workspace_bound(p, &r->prm) + r->U.size() * sizeof(c128);
  const int st = srv->sch->submit(need, r, ticket);
  if (st == sched::SUBMIT_OK) return ST_OK;
  delete r;
  if (st == sched::SUBMIT_TOO_BIG)
    return set_error(ST_EBUSY, "request needs up to %zu bytes of workspace, beyond the budget", need);
  return set_error(ST_EINVAL, "server is shutting down");
}

int rsrr_server_wait(rsrr_server* srv, uint64_t ticket, double timeout_s, rsrr_result** out, double* latency_s) {
  if (!srv || !out) return set_error(ST_EINVAL, "rsrr_server_wait: null argument");
  *out = nullptr;
  void* payload = nullptr;
  int st = 0;
  double lat = 0;
  const int w = srv->sch->wait(ticket, timeout_s, &payload, &st, &lat);
  if (w == sched::WAIT_UNKNOWN) return set_error(ST_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (w == sched::WAIT_TIMEOUT) {
    const std::string s = srv->sch->state();
    return set_error(ST_ETIMEDOUT, "request %llu not finished after %.1f s; server state:\n%s",
                     (unsigned long long)ticket, timeout_s, s.c_str());
  }
  Request* r = (Request*)payload;
  if (latency_s) *latency_s = lat;
  *out = r->res;
  const std::string err = r->err;
  delete r;
  if (st < 0) return set_error(st, "%s", err.c_str());
  return st;
}

int rsrr_server_pending(rsrr_server* srv, int* queued, int* running) {
  if (!srv) return set_error(ST_EINVAL, "rsrr_server_pending: null server");
  int q = 0, r = 0;
  srv->sch->pending(&q, &r);
  if (queued) *queued = q;
  if (running) *running = r;
  return ST_OK;
}

void rsrr_server_destroy(rsrr_server* srv) {
  if (!srv) return;
  if (srv->sch) {
    for (void* pl : srv->sch->stop()) {       // results nobody waited for
      Request* r = (Request*)pl;
      delete r->res;
      delete r;
    }
    delete srv->sch;
  }
  (void)hipSetDevice(srv->ops.device);
  for (DeviceSlot* sl : srv->ops.slots) {
    sl->view.ws.release();
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    delete sl;
  }
  delete srv;
}
