// Autotuning of the LU panel width nb for the sampling factorisations.
//
// rsrr_tune_lu times the batched factorisation (blocks of panels, look-ahead
// stream) of `batch` synthetic matrices of order n for every candidate panel
// width and keeps the fastest in a process-wide table keyed by precision,
// order and batch size; rsrr_tune_save / rsrr_tune_load persist the table as
// JSON.  A solve whose rsrr_params.nb is 0 takes its panel width from the
// table (the entry of the same precision with the nearest order, then the
// nearest batch), or 64 when the table has no entry of that precision.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "driver.h"

namespace rsrr {

namespace {

struct TuneEntry {
  int precision, n, batch, nb;
  double ms;
};
std::mutex g_tmu;
std::vector<TuneEntry> g_table;

constexpr int CANDIDATES[] = {16, 32, 64};

// Deterministic test matrices: entries from a counter hash (splitmix64
// finaliser) in [-1, 1), plus 2 sqrt(n) on the diagonal.
template <typename R>
__global__ __launch_bounds__(256) void tune_fill_kernel(cplx<R>* A, int n, long total, uint64_t seed) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  uint64_t z = seed + (uint64_t)e * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double re = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  const double im = (double)((z * 0x2545F4914F6CDD1Dull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  const long q = e % ((long)n * n);
  const bool diag = (q % n) == (q / n);
  A[e] = mk<R>((R)(re + (diag ? 2.0 * sqrt((double)n) : 0.0)), (R)im);
}

template <typename R>
int tune_one(int n, int batch, int* nb_best, double* ms_best, double* ms_all) {
  hipStream_t s = nullptr;
  Arena ws;
  const long nn = (long)n * n;
  cplx<R>* A = nullptr;
  int *ipiv = nullptr, *info = nullptr;
  cplx<R>* dinv = nullptr;
  RSRR_TRY(ws.get<cplx<R>>("t_A", (size_t)batch * nn, &A));
  RSRR_TRY(ws.get<int>("t_ipiv", (size_t)batch * n, &ipiv));
  RSRR_TRY(ws.get<int>("t_info", batch, &info));
  RSRR_TRY(ws.get<cplx<R>>("t_dinv", LUWork<R>::dinv_elems(n, 64, batch), &dinv));
  struct Events {               // destroyed on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  RSRR_HIP(hipEventCreate(&ev.e0));
  RSRR_HIP(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  int best = 64;
  double tbest = INFINITY;
  int ci = 0;
  for (int nb : CANDIDATES) {
    LUWork<R> w;
    w.n = n; w.nb = nb; w.batch = batch; w.lda = n; w.sA = nn; w.A = A;
    w.ipiv = ipiv; w.dinv = dinv; w.info = info;
    w.tag = "tune_lu";
    w.pair = true;
    w.gauss3m = sizeof(R) == 4;
    RSRR_TRY(ws.aux_stream(&w.aux, &w.ev_main, &w.ev_aux));
    double t = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {        // the first is a warm-up
      hipLaunchKernelGGL((tune_fill_kernel<R>), dim3((unsigned)cdivl(batch * nn, 256)), dim3(256), 0, s, A, n,
                         batch * nn, (uint64_t)(n * 131 + rep));
      RSRR_LAUNCH_CHECK();
      RSRR_HIP(hipEventRecord(e0, s));
      RSRR_TRY(lu_factor<R>(w, s));
      RSRR_HIP(hipEventRecord(e1, s));
      RSRR_HIP(hipEventSynchronize(e1));
      float ms = 0;
      RSRR_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) t = std::min(t, (double)ms);
    }
    if (ms_all) ms_all[ci] = t;
    ++ci;
    if (t < tbest) { tbest = t; best = nb; }
  }
  *nb_best = best;
  *ms_best = tbest;
  return ST_OK;
}

}  // namespace

int tuned_nb(int precision, int n, int batch) {
  std::lock_guard<std::mutex> lk(g_tmu);
  const TuneEntry* pick = nullptr;
  for (const TuneEntry& e : g_table) {
    if (e.precision != precision) continue;
    if (!pick) { pick = &e; continue; }
    const double dn = std::fabs(std::log((double)e.n / n)), dp = std::fabs(std::log((double)pick->n / n));
    const double db = std::fabs(std::log((double)e.batch / batch)), dq = std::fabs(std::log((double)pick->batch / batch));
    if (dn < dp || (dn == dp && db < dq)) pick = &e;
  }
  return pick ? pick->nb : 64;
}

}  // namespace rsrr

using namespace rsrr;

extern "C" {

int rsrr_tune_lu(int precision, int n, int batch, int* nb_best, double* ms_best) {
  if (precision != RSRR_PREC_C128 && precision != RSRR_PREC_C64_IR)
    return set_error(ST_EINVAL, "rsrr_tune_lu: unknown precision %d", precision);
  const int nmax = precision == RSRR_PREC_C128 ? LU_MAX_N_C128 : LU_MAX_N_C64;
  if (n < 1 || n > nmax || batch < 1 || !nb_best) return set_error(ST_EINVAL, "rsrr_tune_lu: bad arguments");
  double ms = 0, all[3] = {0, 0, 0};
  int nb = 64;
  const int st = precision == RSRR_PREC_C128 ? tune_one<double>(n, batch, &nb, &ms, all)
                                              : tune_one<float>(n, batch, &nb, &ms, all);
  if (st < 0) return st;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    bool found = false;
    for (TuneEntry& e : g_table)
      if (e.precision == precision && e.n == n && e.batch == batch) { e.nb = nb; e.ms = ms; found = true; }
    if (!found) g_table.push_back(TuneEntry{precision, n, batch, nb, ms});
  }
  vlog("tune lu precision %d n %d batch %d: nb 16 %.3f ms, 32 %.3f ms, 64 %.3f ms -> %d", precision, n, batch,
       all[0], all[1], all[2], nb);
  *nb_best = nb;
  if (ms_best) *ms_best = ms;
  return ST_OK;
}

int rsrr_tune_save(const char* path) {
  if (!path) return set_error(ST_EINVAL, "rsrr_tune_save: null path");
  std::lock_guard<std::mutex> lk(g_tmu);
  FILE* f = fopen(path, "w");
  if (!f) return set_error(ST_EINVAL, "rsrr_tune_save: cannot write %s", path);
  fprintf(f, "{\"lu_panel_width\": [\n");
  for (size_t i = 0; i < g_table.size(); ++i) {
    const TuneEntry& e = g_table[i];
    fprintf(f, "  {\"precision\": \"%s\", \"n\": %d, \"batch\": %d, \"nb\": %d, \"ms\": %.6f}%s\n",
            e.precision == RSRR_PREC_C128 ? "c128" : "c64_ir", e.n, e.batch, e.nb, e.ms,
            i + 1 < g_table.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return ST_OK;
}

// Reads the file rsrr_tune_save writes (one entry per line); entries replace
// those of the same precision, order and batch.
int rsrr_tune_load(const char* path) {
  if (!path) return set_error(ST_EINVAL, "rsrr_tune_load: null path");
  FILE* f = fopen(path, "r");
  if (!f) return set_error(ST_EINVAL, "rsrr_tune_load: cannot read %s", path);
  char line[512];
  int loaded = 0;
  std::vector<TuneEntry> got;
  while (fgets(line, sizeof(line), f)) {
    char prec[16] = "";
    TuneEntry e{};
    if (sscanf(line, " {\"precision\": \"%15[^\"]\", \"n\": %d, \"batch\": %d, \"nb\": %d, \"ms\": %lf", prec, &e.n,
               &e.batch, &e.nb, &e.ms) == 5) {
      e.precision = strcmp(prec, "c128") == 0 ? RSRR_PREC_C128 : RSRR_PREC_C64_IR;
      if (e.nb < 1 || e.nb > 64 || e.n < 1 || e.batch < 1) continue;
      got.push_back(e);
      ++loaded;
    }
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tmu);
  for (const TuneEntry& e : got) {
    bool found = false;
    for (TuneEntry& t : g_table)
      if (t.precision == e.precision && t.n == e.n && t.batch == e.batch) { t = e; found = true; }
    if (!found) g_table.push_back(e);
  }
  return loaded;
}

}  // extern "C"
