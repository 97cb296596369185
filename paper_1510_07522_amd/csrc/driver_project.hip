// Alg. 2, Step 4 (first half): the reduced coefficients.
//   coefficient form (eq. eq-Zs-expr): B_k = Q^H A_k Q
//   BEM, Chebyshev (eq. eq-Ts-coefs): P_j = w_j sum_k cos(j theta_k) Q^H T(x_k) Q
//   at the d+1 first-kind Chebyshev points x_k of [c - a, c + a], with
//   w_0 = 1/(d+1) and w_j = 2/(d+1) (the standard interpolant);
//   BEM, circle: P_j = (1/(d+1)) sum_k w^(-jk) Q^H T(z_k) Q at the points
//   z_k = c + R w^k, w = exp(2 pi i/(d+1)), for the basis ((z - c)/R)^j.
// Either way the samples Q^H T(x_k) Q are formed first (T generated on the
// fly, in batches that fit chunk_gib) and combined by one product with the
// (d+1) x (d+1) weight matrix.
#include <algorithm>
#include <cmath>

#include "driver.h"

namespace rsrr {

static int zgemm(int opA, int opB, int M, int N, int K, c128 alpha, const void* A, long lda, long sA,
                 const c128* B, long ldb, long sB, c128 beta, c128* C, long ldc, long sC, int batch,
                 bool a_real, hipStream_t s, bool gauss3m = false) {
  GemmBatch<double> g;
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.batch = batch; g.a_real = a_real; g.gauss3m = gauss3m;
  g.tag = "project_gemm";
  return gemm_batched<double>(g, s);
}

int project_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* Q,
                 long ldq, int kS, c128* B, int* J_out) {
  hipStream_t s = p->stream;
  const int n = p->n;
  const c128 one = {1, 0}, zero = {0, 0};
  const long kk = (long)kS * kS;
  c128* W = nullptr;
  if (!p->bem) {
    RSRR_TRY(p->ws.get<c128>("pj_W", (size_t)n * kS, &W));
    for (int k = 0; k < p->J; ++k) {
      const c128* src = W;
      switch (p->kinds[k]) {
        case RSRR_MAT_IDENTITY: src = Q; break;
        case RSRR_MAT_DIAG:
          RSRR_TRY(diag_scale((const c128*)p->mats[k], Q, ldq, W, n, n, kS, s));
          break;
        default:
          RSRR_TRY(zgemm(OP_N, OP_N, n, kS, n, one, p->mats[k], n, 0, Q, ldq, 0, zero, W, n, 0, 1,
                         p->kinds[k] == RSRR_MAT_REAL, s));
      }
      const long lds = (src == Q) ? ldq : n;
      RSRR_TRY(zgemm(OP_C, OP_N, kS, kS, n, one, Q, ldq, 0, src, lds, 0, zero, B + k * kk, kS, 0, 1,
                     false, s));
    }
    if (J_out) *J_out = p->J;
    RSRR_HIP(hipStreamSynchronize(s));
    return ST_OK;
  }
  // ---- interpolation of the BEM matrix: Chebyshev on [c - a, c + a] or a circle
  const int d = prm->cheb_degree > 0 ? prm->cheb_degree : 40;
  const int nd = d + 1;
  const double cx = c->center.re, a = c->a;
  double Rc = 0;
  const bool circle = bem_circle_interp(c, prm, &Rc);
  std::vector<double> theta(nd);
  std::vector<c128> xk(nd);
  for (int k = 0; k < nd; ++k) {
    if (circle) {
      theta[k] = 2.0 * M_PI * k / nd;
      xk[k] = mk<double>(c->center.re + Rc * cos(theta[k]), c->center.im + Rc * sin(theta[k]));
    } else {
      theta[k] = (k + 0.5) * M_PI / nd;
      xk[k] = mk<double>(cx + a * cos(theta[k]), 0.0);
    }
  }
  const size_t per = (size_t)n * n * sizeof(c128);
  const int ch = (int)std::max<size_t>(1, std::min<size_t>(nd, (size_t)(prm->chunk_gib * 1073741824.0) / per));
  c128 *T = nullptr, *Mk = nullptr, *zd = nullptr, *Cw = nullptr;
  RSRR_TRY(p->ws.get<c128>("pj_T", (size_t)ch * n * n, &T));
  RSRR_TRY(p->ws.get<c128>("pj_W", (size_t)ch * n * kS, &W));
  RSRR_TRY(p->ws.get<c128>("pj_M", (size_t)nd * kk, &Mk));
  RSRR_TRY(p->ws.get<c128>("pj_z", nd, &zd));
  RSRR_TRY(p->ws.get<c128>("pj_C", (size_t)nd * nd, &Cw));
  RSRR_HIP(hipMemcpyAsync(zd, xk.data(), nd * sizeof(c128), hipMemcpyHostToDevice, s));
  for (int k0 = 0; k0 < nd; k0 += ch) {
    const int cnt = std::min(ch, nd - k0);
    RSRR_TRY(assemble_bem<double>(n, p->xyz, p->h, cnt, zd + k0, T, n, (long)n * n, s));
    // T(x_k) Q, the bulk of the projection's work (8 n^2 k_S per point), with
    // 3 real products per complex one (normwise stable; the coefficients are
    // then used by the reduced problem, whose eigenpairs are checked against
    // the exact T by their residuals)
    RSRR_TRY(zgemm(OP_N, OP_N, n, kS, n, one, T, n, (long)n * n, Q, ldq, 0, zero, W, n, (long)n * kS,
                   cnt, false, s, true));
    RSRR_TRY(zgemm(OP_C, OP_N, kS, kS, n, one, Q, ldq, 0, W, n, (long)n * kS, zero, Mk + k0 * kk, kS,
                   kk, cnt, false, s));
  }
  // P (kk x nd) = M (kk x nd) C,  C[k][j] = w_j cos(j theta_k) (Chebyshev) or
  // exp(-i j theta_k)/(d+1) (circle)
  std::vector<c128> Ch((size_t)nd * nd);
  for (int j = 0; j < nd; ++j)
    for (int k = 0; k < nd; ++k)
      Ch[k + (size_t)j * nd] = circle ? mk<double>(cos(j * theta[k]) / nd, -sin(j * theta[k]) / nd)
                                      : mk<double>((j == 0 ? 1.0 : 2.0) / nd * cos(j * theta[k]), 0.0);
  RSRR_HIP(hipMemcpyAsync(Cw, Ch.data(), Ch.size() * sizeof(c128), hipMemcpyHostToDevice, s));
  RSRR_TRY(zgemm(OP_N, OP_N, (int)kk, nd, nd, one, Mk, kk, 0, Cw, nd, 0, zero, B, kk, 0, 1, false, s));
  if (J_out) *J_out = nd;
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

}  // namespace rsrr
