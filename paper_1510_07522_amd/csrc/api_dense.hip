// C ABI of the dense building blocks (batched GEMM, batched LU solve).
#include "driver.h"

using namespace rsrr;

namespace {

template <typename R>
int gemm_entry(int opA, int opB, int M, int N, int K, rsrr_complex alpha, const void* A, int lda,
               long long sA, const void* B, int ldb, long long sB, rsrr_complex beta, void* C,
               int ldc, long long sC, int batch, bool g3m, void* stream) {
  if (opA < 0 || opA > 2 || opB < 0 || opB > 2) return set_error(ST_EINVAL, "gemm: bad op");
  if (M < 0 || N < 0 || K < 0 || batch < 0) return set_error(ST_EINVAL, "gemm: negative size");
  const int ra = (opA == OP_N) ? M : K, rb = (opB == OP_N) ? K : N;
  if ((ra > 0 && lda < ra) || (rb > 0 && ldb < rb) || (M > 0 && ldc < M))
    return set_error(ST_EINVAL, "gemm: leading dimension too small");
  if ((M && N && batch) && (!C || (K && (!A || !B)))) return set_error(ST_EINVAL, "gemm: null pointer");
  GemmBatch<R> g;
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = mk<R>((R)alpha.re, (R)alpha.im);
  g.beta = mk<R>((R)beta.re, (R)beta.im);
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = (const cplx<R>*)B; g.ldb = ldb; g.sB = sB;
  g.C = (cplx<R>*)C; g.ldc = ldc; g.sC = sC;
  g.batch = batch;
  g.gauss3m = g3m;
  RSRR_TRY(gemm_batched<R>(g, (hipStream_t)stream));
  RSRR_HIP(hipStreamSynchronize((hipStream_t)stream));
  return ST_OK;
}

template <typename R>
int gesv_entry(int n, int nrhs, void* A, int lda, long long sA, void* B, int ldb, long long sB,
               int batch, int nb, int* info_host, void* stream) {
  if (n < 1 || n > lu_max_order<R>() || nrhs < 0 || batch < 1 || lda < n || ldb < n || nb < 1 || nb > 64)
    return set_error(ST_EINVAL, "gesv: bad arguments");
  if (!A || (nrhs > 0 && !B)) return set_error(ST_EINVAL, "gesv: null pointer");
  hipStream_t s = (hipStream_t)stream;
  int *ipiv = nullptr, *info = nullptr;
  cplx<R>* dinv = nullptr;
  const size_t de = LUWork<R>::dinv_elems(n, nb, batch);
  if (hipMalloc(&ipiv, (size_t)batch * n * sizeof(int)) != hipSuccess ||
      hipMalloc(&info, (size_t)batch * sizeof(int)) != hipSuccess ||
      hipMalloc(&dinv, de * sizeof(cplx<R>)) != hipSuccess) {
    (void)hipGetLastError();
    if (ipiv) (void)hipFree(ipiv);
    if (info) (void)hipFree(info);
    return set_error(ST_ENOMEM, "gesv: workspace allocation failed");
  }
  LUWork<R> w;
  w.n = n; w.nb = nb; w.batch = batch; w.lda = lda; w.sA = sA; w.A = (cplx<R>*)A;
  w.pair = true;
  w.ipiv = ipiv; w.dinv = dinv; w.info = info;
  int st = lu_factor<R>(w, s);
  if (st == ST_OK && nrhs > 0) st = lu_solve<R>(w, (cplx<R>*)B, ldb, sB, nrhs, s);
  std::vector<int> h(batch, 0);
  if (st == ST_OK) {
    if (hipMemcpyAsync(h.data(), info, batch * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = set_error(ST_EHIP, "gesv: synchronisation failed");
  }
  (void)hipFree(ipiv);
  (void)hipFree(info);
  (void)hipFree(dinv);
  if (st < 0) return st;
  if (info_host) for (int b = 0; b < batch; ++b) info_host[b] = h[b];
  for (int b = 0; b < batch; ++b)
    if (h[b]) return set_error(ST_ESINGULAR, "gesv: matrix %d has a zero pivot at %d", b, h[b]);
  return ST_OK;
}

}  // namespace

extern "C" {

int rsrr_zgemm_batched(int opA, int opB, int M, int N, int K, rsrr_complex alpha,
                       const rsrr_complex* A, int lda, long long sA, const rsrr_complex* B, int ldb,
                       long long sB, rsrr_complex beta, rsrr_complex* C, int ldc, long long sC,
                       int batch, void* stream) {
  return gemm_entry<double>(opA, opB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                            batch, false, stream);
}

int rsrr_cgemm_batched(int opA, int opB, int M, int N, int K, rsrr_complex alpha, const void* A,
                       int lda, long long sA, const void* B, int ldb, long long sB,
                       rsrr_complex beta, void* C, int ldc, long long sC, int batch, int gauss3m,
                       void* stream) {
  return gemm_entry<float>(opA, opB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                           batch, gauss3m != 0, stream);
}

int rsrr_gesv_batched(int precision, int n, int nrhs, void* A, int lda, long long sA, void* B,
                      int ldb, long long sB, int batch, int nb, int* info_host, void* stream) {
  if (precision == RSRR_PREC_C128)
    return gesv_entry<double>(n, nrhs, A, lda, sA, B, ldb, sB, batch, nb, info_host, stream);
  if (precision == RSRR_PREC_C64_IR)
    return gesv_entry<float>(n, nrhs, A, lda, sA, B, ldb, sB, batch, nb, info_host, stream);
  return set_error(ST_EINVAL, "gesv: unknown precision %d", precision);
}

}  // extern "C"
