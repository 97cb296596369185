// The batched LU solve of rsrr_gesv_batched with its work space in a fixed,
// file-scope device array instead of device allocations, for callers that
// cannot allocate (code under stream capture, tight serving loops, hosts that
// forbid allocation calls).
//
// The array is `scratch` below (SCRATCH_BYTES, 256-byte aligned); every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel: its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and kept in
// g_scratch[device]; that address is what the kernels receive.  All calls on
// one device share the array, so calls that overlap in time on one device
// (other host threads, other streams) race; each call writes every byte it
// reads (per-matrix status cleared by a kernel, pivots and diagonal-block
// inverses written by the factorisation) before reading it.
#include <mutex>

#include "driver.h"

using namespace rsrr;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once).
int scratch_address(void** out) {
  int dev = -1;
  RSRR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return set_error(ST_EINVAL, "device %d outside [0, %d)", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(ST_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return ST_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename R>
int gesv_noalloc(int n, int nrhs, void* A, int lda, long long sA, void* B, int ldb, long long sB, int batch,
                 int nb, int* info_host, void* stream) {
  if (n < 1 || n > lu_max_order<R>() || nrhs < 0 || batch < 1 || lda < n || ldb < n || nb < 1 || nb > 64)
    return set_error(ST_EINVAL, "gesv_noalloc: bad arguments");
  if (!A || (nrhs > 0 && !B)) return set_error(ST_EINVAL, "gesv_noalloc: null pointer");
  const size_t b_info = round256((size_t)batch * sizeof(int));
  const size_t b_ipiv = round256((size_t)batch * n * sizeof(int));
  const size_t b_dinv = round256(LUWork<R>::dinv_elems(n, nb, batch) * sizeof(cplx<R>));
  const size_t need = b_info + b_ipiv + b_dinv;
  if (need > SCRATCH_BYTES)
    return set_error(ST_EINVAL, "gesv_noalloc: needs %zu bytes of work space; the fixed scratch holds %zu "
                     "(use fewer matrices per call or rsrr_gesv_batched)", need, SCRATCH_BYTES);
  void* base = nullptr;
  RSRR_TRY(scratch_address(&base));
  char* p = (char*)base;
  hipStream_t s = (hipStream_t)stream;
  LUWork<R> w;
  w.n = n; w.nb = nb; w.batch = batch; w.lda = lda; w.sA = sA; w.A = (cplx<R>*)A;
  w.pair = true;
  w.info = (int*)p;
  w.ipiv = (int*)(p + b_info);
  w.dinv = (cplx<R>*)(p + b_info + b_ipiv);
  RSRR_TRY(lu_factor<R>(w, s));      // clears the status words first
  if (nrhs > 0) RSRR_TRY(lu_solve<R>(w, (cplx<R>*)B, ldb, sB, nrhs, s));
  // without a status buffer the call only enqueues kernels (no copy, no wait:
  // it can be recorded under stream capture); zero pivots are then not reported
  if (!info_host) return ST_OK;
  // per-matrix status through a fixed host buffer
  int first_bad = -1, bad_at = 0;
  int h[256];
  for (int b0 = 0; b0 < batch; b0 += 256) {
    const int cnt = batch - b0 < 256 ? batch - b0 : 256;
    RSRR_HIP(hipMemcpyAsync(h, w.info + b0, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < cnt; ++q) {
      info_host[b0 + q] = h[q];
      if (h[q] && first_bad < 0) { first_bad = b0 + q; bad_at = h[q]; }
    }
  }
  if (first_bad >= 0) return set_error(ST_ESINGULAR, "gesv_noalloc: matrix %d has a zero pivot at %d", first_bad, bad_at);
  return ST_OK;
}

}  // namespace

extern "C" {

int rsrr_gesv_batched_noalloc(int precision, int n, int nrhs, void* A, int lda, long long sA, void* B, int ldb,
                              long long sB, int batch, int nb, int* info_host, void* stream) {
  if (precision == RSRR_PREC_C128)
    return gesv_noalloc<double>(n, nrhs, A, lda, sA, B, ldb, sB, batch, nb, info_host, stream);
  if (precision == RSRR_PREC_C64_IR)
    return gesv_noalloc<float>(n, nrhs, A, lda, sA, B, ldb, sB, batch, nb, info_host, stream);
  return set_error(ST_EINVAL, "gesv_noalloc: unknown precision %d", precision);
}

}  // extern "C"
