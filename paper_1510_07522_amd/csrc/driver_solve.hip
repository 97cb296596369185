// Alg. 2 end to end on the device: sampling, basis, projection, the modified
// block Sakurai-Sugiura method on the reduced problem (Alg. 1), eigenvector
// recovery, and the residual filter.
//
//   moments   A_a = 1/(2 pi i) sum_m dz_m ((zeta_m - gamma)/rho)^a T_S(zeta_m)^{-1},
//             a < 2K, with the contour's quadrature weights dz_m (ellipse:
//             dz_m = (2 pi/NS) phi'(theta_m), which is eq. eq-Ap-num;
//             rectangle: Gauss-Legendre on each side), as one GEMM per chunk of
//             nodes over the batched inverses;
//   winding   n = 1/(2 pi i) sum_m dz_m tr(T_S(zeta_m)^{-1} T_S'(zeta_m)) (eq. eq-ncs);
//   Hankel    H = [A_{i+j}], H^< = [A_{i+j+1}] (eq. eq-HH); SVD of H (eq. eq-svdH);
//   gap       argmax sigma_j / sigma_{j+1} if >= tol_gap (eq. eq-gap);
//   extract   A = V0^H H^< W0 S0^{-1} (eq. eq-A), lambda = rho l' + gamma,
//             g = H_r W0 S0^{-1} g' (eq. eq-eigens), v = Q g (Alg. 2 Step 5).
// Readings: all Hankel singular values above hankel_tol * sigma_1 are kept;
// the eigenvalues strictly inside the contour whose residual
// ||T(l) v|| / (||T(l)||_F ||v||) is at most tol_res are returned.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "bounds.h"
#include "driver.h"
#include "eig.h"
#include "reduced.h"

namespace rsrr {

static const c128 ONE = {1, 0}, ZERO = {0, 0};

static int zgemm(int opA, int opB, int M, int N, int K, c128 alpha, const void* A, long lda,
                 const c128* B, long ldb, c128 beta, c128* C, long ldc, hipStream_t s,
                 bool a_real = false, const char* tag = "reduced_gemm") {
  GemmBatch<double> g;
  g.tag = tag;
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.a_real = a_real;
  return gemm_batched<double>(g, s);
}

// splitmix64 (Steele, Lea, Flood 2014) and Box-Muller: complex Gaussian
// (x + i y)/sqrt(2) entries for the probing matrix when none is supplied.
static uint64_t splitmix64(uint64_t* st) {
  uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static void gaussian_probe(int n, int L, uint64_t seed, std::vector<c128>* U) {
  U->resize((size_t)n * L);
  uint64_t st = seed;
  for (size_t e = 0; e < U->size(); ++e) {
    const double u1 = ((splitmix64(&st) >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix64(&st) >> 11) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(u1));
    (*U)[e] = mk<double>(r * cos(2 * M_PI * u2) / sqrt(2.0), r * sin(2 * M_PI * u2) / sqrt(2.0));
  }
}

// g_k(z_q), g_k'(z_q) of the reduced problem at m nodes (row q holds J values):
// the f_k themselves, or for the BEM interpolant the Chebyshev polynomials
// tau_j((z - c)/a) or the powers ((z - c)/R)^j.  Returns 1 (g filled, dg
// zero) when the caller's scalar functions come without derivatives.
static int reduced_scalars(const rsrr_problem* p, int J, const rsrr_contour* c, const rsrr_params* prm,
                           const cd* z, size_t m, std::vector<cd>* g, std::vector<cd>* dg) {
  g->assign(m * J, cd(0, 0));
  dg->assign(m * J, cd(0, 0));
  if (!p->bem) {
    const int st = eval_scalars(p, z, m, g->data(), dg->data());
    if (st == 1) dg->assign(m * J, cd(0, 0));
    return st;
  }
  double Rc = 0;
  if (bem_circle_interp(c, prm, &Rc)) {
    const cd ctr(c->center.re, c->center.im);
    for (size_t q = 0; q < m; ++q) {
      cd* gq = g->data() + q * J;
      cd* dq = dg->data() + q * J;
      const cd sq = (z[q] - ctr) / Rc;
      gq[0] = 1.0;
      for (int j = 1; j < J; ++j) {
        gq[j] = gq[j - 1] * sq;
        dq[j] = (double)j * gq[j - 1] / Rc;
      }
    }
    return ST_OK;
  }
  const double cx = c->center.re, a = c->a;
  for (size_t q = 0; q < m; ++q) {
    cd* gq = g->data() + q * J;
    cd* dq = dg->data() + q * J;
    const cd t = (z[q] - cx) / a;
    gq[0] = 1.0;
    if (J > 1) { gq[1] = t; dq[1] = 1.0; }
    for (int j = 2; j < J; ++j) {
      gq[j] = 2.0 * t * gq[j - 1] - gq[j - 2];
      dq[j] = 2.0 * gq[j - 1] + 2.0 * t * dq[j - 1] - dq[j - 2];
    }
    for (int j = 0; j < J; ++j) dq[j] /= a;
  }
  return ST_OK;
}

size_t solve_workspace_bound(const rsrr_problem* p, const rsrr_params* prm) {
  return workspace_bound(p->n, p->J, p->bem, prm);
}

size_t Arena::bytes() const {
  size_t b = 0;
  for (const auto& kv : bufs) b += kv.second.second;
  return b;
}

int solve_begin(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* Uin,
                rsrr_result* res, SamplePlan* sp) {
  hipStream_t s = p->stream;
  Arena& ws = p->ws;
  const int n = p->n, L = prm->L;
  const long NL = (long)prm->N * L;
  // ---- Alg. 2, Steps 1-2: probing matrix and the sampled system matrices
  const c128* U = Uin;
  if (!U) {
    std::vector<c128> hU;
    gaussian_probe(n, L, prm->seed, &hU);
    c128* dU = nullptr;
    RSRR_TRY(ws.get<c128>("sv_U", hU.size(), &dU));
    RSRR_HIP(hipMemcpyAsync(dU, hU.data(), hU.size() * sizeof(c128), hipMemcpyHostToDevice, s));
    RSRR_HIP(hipStreamSynchronize(s));
    U = dU;
  }
  c128* Shat = nullptr;
  RSRR_TRY(ws.get<c128>("sv_Shat", (size_t)n * NL, &Shat));
  return sample_begin(p, c, prm, U, n, Shat, n, &res->info, sp);
}

int solve_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* Uin,
               rsrr_result* res) {
  SamplePlan sp;
  RSRR_TRY(solve_begin(p, c, prm, Uin, res, &sp));
  RSRR_TRY(sample_factor(&sp));
  return solve_end(p, c, prm, res, &sp);
}

int solve_end(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, rsrr_result* res,
              SamplePlan* sp) {
  hipStream_t s = p->stream;
  Arena& ws = p->ws;
  const int n = p->n, N = prm->N, L = prm->L, NS = prm->NS, K = prm->K;
  const long NL = (long)N * L;
  rsrr_info& info = res->info;
  int warn = 0;
  const cd gamma(c->center.re, c->center.im);
  const double rho = std::max(c->a, c->b);
  c128* Shat = sp->S;
  int st = sample_end(sp);
  if (st < 0) return st;
  warn |= st;

  // ---- Step 3: orthonormal basis of S_hat, or of the moment matrix M_hat
  // (SSRR moment scheme: S_hat replaced by M_hat = S_hat D Z)
  double t0 = now_s();
  const c128* Sbase = Shat;
  long ncols = NL;
  if (prm->scheme == RSRR_SCHEME_MOMENT) {
    ncols = (long)(prm->Kp > 0 ? prm->Kp : N) * L;
    c128* Mhat = nullptr;
    RSRR_TRY(ws.get<c128>("sv_Mhat", (size_t)n * ncols, &Mhat));
    RSRR_TRY(moment_impl(p, c, prm, Shat, n, Mhat, n));
    Sbase = Mhat;
  }
  const int kmax = (int)std::min<long>(n, ncols);
  c128* Q = nullptr;
  RSRR_TRY(ws.get<c128>("sv_Q", (size_t)n * kmax, &Q));
  int kS = 0;
  // three levels: the sampling matrix's singular values reach delta sigma_1
  RSRR_TRY(ortho_impl(n, (int)ncols, Sbase, n, prm->delta, Q, n, &kS, ws, s, 3));
  info.k_S = kS;
  info.t_basis = now_s() - t0;
  vlog("sample %.3fs (ir %d, fallback %d), basis k_S=%d %.3fs", info.t_sample, info.ir_iters,
       info.ir_fallback, kS, info.t_basis);
  if (kS == 0) return set_error(ST_ENOTCONV, "sampling matrix is numerically zero");
  if (kS == ncols && ncols < n) warn |= RSRR_WARN_RANK_SATURATED;

  // ---- Step 4: reduced coefficients
  t0 = now_s();
  const int Jmax = p->bem ? (prm->cheb_degree > 0 ? prm->cheb_degree : 40) + 1 : p->J;
  const long kk = (long)kS * kS;
  c128 *B = nullptr, *BT = nullptr;
  RSRR_TRY(ws.get<c128>("sv_B", (size_t)Jmax * kk, &B));
  RSRR_TRY(ws.get<c128>("sv_BT", (size_t)Jmax * kk, &BT));
  int J = 0;
  RSRR_TRY(project_impl(p, c, prm, Q, n, kS, B, &J));
  RSRR_TRY(transpose_blocks(B, BT, kS, J, s));
  info.t_project = now_s() - t0;
  vlog("project J=%d %.3fs", J, info.t_project);

  // ---- Alg. 1: moments of T_S^{-1} and the winding number
  t0 = now_s();
  std::vector<cd> zeta, dzeta;
  contour_nodes(c, NS, false, &zeta, &dzeta);
  const size_t per = (size_t)kk * sizeof(c128) * 2;
  // nodes per batch: as many as the chunk memory holds, balanced over the batches
  const int ch = chunk_count(NS, per, prm->chunk_gib).second;
  c128 *TS = nullptr, *X = nullptr, *Amom = nullptr, *gdev = nullptr, *cw = nullptr, *dinv = nullptr,
       *part = nullptr;
  int *ipiv = nullptr, *linfo = nullptr;
  const int nchunk = 64;
  RSRR_TRY(ws.get<c128>("rd_TS", (size_t)ch * kk, &TS));
  RSRR_TRY(ws.get<c128>("rd_X", (size_t)ch * kk, &X));
  RSRR_TRY(ws.get<c128>("rd_A", (size_t)2 * K * kk, &Amom));
  RSRR_TRY(ws.get<c128>("rd_g", (size_t)2 * ch * J, &gdev));
  RSRR_TRY(ws.get<c128>("rd_cw", (size_t)ch * 2 * K, &cw));
  // panel width of the reduced LUs (their own: the tuned width is the sampling's)
  const int nbr = reduced_nb(prm);
  RSRR_TRY(ws.get<c128>("rd_dinv", LUWork<double>::dinv_elems(kS, nbr, ch), &dinv));
  RSRR_TRY(ws.get<c128>("rd_part", (size_t)ch * nchunk, &part));
  // moments and winding traces in one pass over the inverses when the sizes
  // allow it (2K <= 8, J <= 4, the batch's wave sums in LDS)
  const bool fused = 2 * K <= 8 && J <= 4 && (size_t)4 * ch * J * sizeof(c128) <= 60 * 1024;
  c128* dpart = nullptr;
  if (fused) RSRR_TRY(ws.get<c128>("rd_dpart", (size_t)moments_wind_parts(kk, ch, J), &dpart));
  RSRR_TRY(ws.get<int>("rd_ipiv", (size_t)ch * kS, &ipiv));
  int* iperm = nullptr;
  RSRR_TRY(ws.get<int>("rd_perm", (size_t)ch * kS, &iperm));
  int* lperm = nullptr;
  RSRR_TRY(ws.get<int>("rd_lperm", (size_t)ch * ((kS + nbr - 1) / nbr) * kS, &lperm));
  RSRR_TRY(ws.get<int>("rd_info", ch, &linfo));
  cd wind(0, 0);
  std::vector<cd> g, dg;
  const int sst = reduced_scalars(p, J, c, prm, zeta.data(), NS, &g, &dg);
  if (sst < 0) return sst;
  const bool have_wind = sst == ST_OK;
  if (!have_wind) warn |= RSRR_WARN_NO_WINDING;
  std::vector<c128> hg((size_t)ch * J), hdg((size_t)ch * J), hcw((size_t)ch * 2 * K), hpart;
  for (int m0 = 0; m0 < NS; m0 += ch) {
    const int cnt = std::min(ch, NS - m0);
    for (int q = 0; q < cnt; ++q) {
      for (int k = 0; k < J; ++k) {
        const cd gv = g[(size_t)(m0 + q) * J + k], dv = dg[(size_t)(m0 + q) * J + k];
        hg[(size_t)q * J + k] = mk<double>(gv.real(), gv.imag());
        hdg[(size_t)q * J + k] = mk<double>(dv.real(), dv.imag());
      }
      const cd w = dzeta[m0 + q] / cd(0, 2.0 * M_PI);
      const cd sm = (zeta[m0 + q] - gamma) / rho;
      cd pw(1, 0);
      for (int a = 0; a < 2 * K; ++a) {
        const cd v = w * pw;
        hcw[q + (size_t)a * cnt] = mk<double>(v.real(), v.imag());
        pw *= sm;
      }
    }
    RSRR_HIP(hipMemcpyAsync(gdev, hg.data(), (size_t)cnt * J * sizeof(c128), hipMemcpyHostToDevice, s));
    RSRR_HIP(hipMemcpyAsync(gdev + (size_t)ch * J, hdg.data(), (size_t)cnt * J * sizeof(c128),
                            hipMemcpyHostToDevice, s));
    RSRR_HIP(hipMemcpyAsync(cw, hcw.data(), (size_t)cnt * 2 * K * sizeof(c128), hipMemcpyHostToDevice, s));
    // T_S(zeta_q) = sum_k g_k(zeta_q) B_k for the chunk: (kk x J) (J x cnt)
    RSRR_TRY(zgemm(OP_N, OP_N, (int)kk, cnt, J, ONE, B, kk, gdev, J, ZERO, TS, kk, s));
    LUWork<double> w;
    w.n = kS; w.nb = nbr; w.batch = cnt; w.lda = kS; w.sA = kk; w.A = TS;
    w.ipiv = ipiv; w.dinv = dinv; w.info = linfo;
    w.tag = "reduced_lu_c128";
    RSRR_TRY(ws.aux_stream(&w.aux, &w.ev_main, &w.ev_aux));
    w.gauss3m = true;
    w.full_swap = true;
    w.lperm = lperm;
    w.pair = true;
    RSRR_TRY(lu_factor<double>(w, s));
    // the inverses replace the factors in TS once the solves are done; X is
    // the work space of the solves
    RSRR_TRY(lu_inverse<double>(w, X, TS, kS, kk, iperm, s));
    // moments: [A_0 .. A_{2K-1}] += [X_m] cw   (kk x cnt) (cnt x 2K), X_m in TS;
    // winding: tr(X_m T_S'(zeta_m)) = sum_k g_k'(zeta_m) sum_e X_m[e] (B_k^T)[e]
    std::vector<int> hinfo(cnt);
    if (fused) {
      RSRR_TRY(moments_wind(TS, kk, cnt, cw, 2 * K, BT, J, Amom, m0 != 0, dpart, part, s));
      hpart.resize((size_t)cnt * J);
      RSRR_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(c128), hipMemcpyDeviceToHost, s));
    } else {
      RSRR_TRY(zgemm(OP_N, OP_N, (int)kk, 2 * K, cnt, ONE, TS, kk, cw, cnt, m0 == 0 ? ZERO : ONE, Amom, kk, s));
      // T_S'(zeta_m) into X, then sum_e X_m[e] (T_S'(zeta_m)^T)[e] in chunks
      RSRR_TRY(zgemm(OP_N, OP_N, (int)kk, cnt, J, ONE, BT, kk, gdev + (size_t)ch * J, J, ZERO, X, kk, s));
      RSRR_TRY(dot_partials(TS, X, kk, cnt, nchunk, part, s));
      hpart.resize((size_t)cnt * nchunk);
      RSRR_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(c128), hipMemcpyDeviceToHost, s));
    }
    RSRR_HIP(hipMemcpyAsync(hinfo.data(), linfo, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < cnt; ++q)
      if (hinfo[q]) return set_error(ST_ESINGULAR, "reduced matrix singular at node %d", m0 + q);
    for (int q = 0; q < cnt; ++q) {
      cd tr(0, 0);
      if (fused) {
        for (int k = 0; k < J; ++k)
          tr += cd(hdg[(size_t)q * J + k].re, hdg[(size_t)q * J + k].im) *
                cd(hpart[(size_t)q * J + k].re, hpart[(size_t)q * J + k].im);
      } else {
        for (int t = 0; t < nchunk; ++t) tr += cd(hpart[(size_t)q * nchunk + t].re, hpart[(size_t)q * nchunk + t].im);
      }
      wind += dzeta[m0 + q] / cd(0, 2.0 * M_PI) * tr;
    }
  }
  info.wind_re = have_wind ? wind.real() : std::nan("");
  info.wind_im = have_wind ? wind.imag() : std::nan("");
  info.n_wind = have_wind ? (int)std::lround(wind.real()) : -1;
  vlog("moments NS=%d chunk=%d winding %.6f%+.2ei %.3fs", NS, ch, wind.real(), wind.imag(), now_s() - t0);

  // ---- Hankel matrices and the SVD of H
  const int M = K * kS;
  c128 *H = nullptr, *Hs = nullptr, *Uh = nullptr, *Wh = nullptr;
  RSRR_TRY(ws.get<c128>("rd_H", (size_t)M * M, &H));
  RSRR_TRY(ws.get<c128>("rd_Hs", (size_t)M * M, &Hs));
  RSRR_TRY(ws.get<c128>("rd_Uh", (size_t)M * M, &Uh));
  RSRR_TRY(ws.get<c128>("rd_Wh", (size_t)M * M, &Wh));
  RSRR_TRY(build_hankel(Amom, kS, K, 0, H, M, s));
  RSRR_TRY(build_hankel(Amom, kS, K, 1, Hs, M, s));
  std::vector<double> sigma;
  int rH = 0;
  // basis of range(H) down to a tenth of the truncation level
  RSRR_TRY(hankel_svd(H, M, 0.1 * prm->hankel_tol, prm->hankel_tol, Uh, M, Wh, M, &sigma, &rH, ws, s));
  if (rH == 0) return set_error(ST_ESINGULAR, "Hankel matrix is zero: no eigenvalue inside the contour");
  sigma.resize(M, 0.0);   // directions outside the numerical range: zero
  res->hankel_sigma = sigma;
  vlog("hankel svd M=%d rank %d %.3fs", M, rH, now_s() - t0);
  // gap count (eq. eq-gap), reading: zero tail excluded, smallest j on ties
  {
    const double floor_ = 10.0 * 1.1102230246251565e-16 * M * sigma[0];
    double best = 0;
    int bj = -1;
    for (int j = 0; j + 1 < M; ++j) {
      if (!(sigma[j + 1] > floor_)) break;
      const double r = sigma[j] / sigma[j + 1];
      if (r > best) { best = r; bj = j + 1; }
    }
    info.n_gap = (best >= prm->tol_gap) ? bj : -1;
  }
  int m = 0;
  for (int j = 0; j < rH; ++j) if (sigma[j] > prm->hankel_tol * sigma[0]) ++m;
  info.m = m;
  // every singular value retained: H may not have the rank Alg. 1 needs
  // (K k_S at least the number of eigenvalues inside, eq. eq-ranks)
  if (m == M) warn |= RSRR_WARN_HANKEL_FULL;

  // ---- A = V0^H H^< W0 S0^{-1}; eig; recovery
  c128 *W0s = nullptr, *T1 = nullptr, *Ar = nullptr, *Gp = nullptr, *T2 = nullptr, *Gv = nullptr, *Vv = nullptr;
  double* invs = nullptr;
  RSRR_TRY(ws.get<c128>("rd_W0s", (size_t)M * m, &W0s));
  RSRR_TRY(ws.get<c128>("rd_T1", (size_t)M * m, &T1));
  RSRR_TRY(ws.get<c128>("rd_Ar", (size_t)m * m, &Ar));
  RSRR_TRY(ws.get<c128>("rd_Gp", (size_t)m * m, &Gp));
  RSRR_TRY(ws.get<c128>("rd_T2", (size_t)M * m, &T2));
  RSRR_TRY(ws.get<c128>("rd_Gv", (size_t)kS * m, &Gv));
  RSRR_TRY(ws.get<c128>("rd_Vv", (size_t)n * m, &Vv));
  RSRR_TRY(ws.get<double>("rd_invs", m, &invs));
  std::vector<double> hinv(m);
  for (int j = 0; j < m; ++j) hinv[j] = 1.0 / sigma[j];
  RSRR_HIP(hipMemcpyAsync(invs, hinv.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
  RSRR_TRY(gather_scale_cols(Wh, M, nullptr, invs, M, m, W0s, M, s));
  RSRR_TRY(zgemm(OP_N, OP_N, M, m, M, ONE, Hs, M, W0s, M, ZERO, T1, M, s));
  RSRR_TRY(zgemm(OP_C, OP_N, m, m, M, ONE, Uh, M, T1, M, ZERO, Ar, m, s));
  std::vector<cd> lamp;
  vlog("extraction m=%d gap=%d", m, info.n_gap);
  // spectral splits whose dropped coupling could bring residuals within a
  // tenth of the acceptance level are followed by a first-order correction
  RSRR_TRY(eig_general(Ar, m, m, &lamp, Gp, m, ws, s, 0.1 * prm->tol_res));
  vlog("eig m=%d %.3fs", m, now_s() - t0);
  RSRR_TRY(zgemm(OP_N, OP_N, M, m, m, ONE, W0s, M, Gp, m, ZERO, T2, M, s));
  // H_r = [A_0 ... A_{K-1}] is the first block row of H: rows 0..kS-1 of the
  // Hankel layout, i.e. Amom blocks 0..K-1 side by side (ld kS).
  RSRR_TRY(zgemm(OP_N, OP_N, kS, m, M, ONE, Amom, kS, T2, M, ZERO, Gv, kS, s));
  RSRR_TRY(zgemm(OP_N, OP_N, n, m, kS, ONE, Q, n, Gv, kS, ZERO, Vv, n, s));
  info.t_reduced = now_s() - t0;

  // ---- inside filter, normalisation and residuals (a8)
  t0 = now_s();
  std::vector<cd> lam(m);
  std::vector<int> inside;
  for (int j = 0; j < m; ++j) {
    lam[j] = rho * lamp[j] + gamma;
    if (contour_inside(c, lam[j])) inside.push_back(j);
  }
  const int nin = (int)inside.size();
  info.n_candidates = nin;
  std::vector<double> rel, raw;
  c128* Vin = nullptr;
  if (nin > 0) {
    int* pin = nullptr;
    c128 *Rr = nullptr, *zerov = nullptr, *coef = nullptr;
    double* nrm = nullptr;
    RSRR_TRY(ws.get<c128>("fi_V", (size_t)n * nin, &Vin));
    RSRR_TRY(ws.get<int>("fi_perm", nin, &pin));
    RSRR_TRY(ws.get<c128>("fi_R", (size_t)n * nin, &Rr));
    RSRR_TRY(ws.get<c128>("fi_zero", n, &zerov));
    RSRR_TRY(ws.get<double>("fi_nrm", 2 * (size_t)nin, &nrm));
    RSRR_HIP(hipMemcpyAsync(pin, inside.data(), nin * sizeof(int), hipMemcpyHostToDevice, s));
    RSRR_TRY(gather_scale_cols(Vv, n, pin, nullptr, n, nin, Vin, n, s));
    RSRR_TRY(normalize_cols(Vin, n, n, nin, s));
    RSRR_TRY(fill_c128(zerov, n, ZERO, s));
    std::vector<double> fro2(nin);
    std::vector<c128> lz(nin);
    for (int q = 0; q < nin; ++q) lz[q] = mk<double>(lam[inside[q]].real(), lam[inside[q]].imag());
    if (p->bem) {
      c128* zl = nullptr;
      double* partb = nullptr;
      RSRR_TRY(ws.get<c128>("fi_z", nin, &zl));
      RSRR_TRY(ws.get<double>("fi_bpart", (size_t)nin * n, &partb));
      RSRR_HIP(hipMemcpyAsync(zl, lz.data(), nin * sizeof(c128), hipMemcpyHostToDevice, s));
      RSRR_TRY(bem_residual(n, p->xyz, p->h, nin, zl, zerov, n, Vin, n, n, 1, Rr, n, n, s));
      RSRR_TRY(bem_fro2(n, p->xyz, p->h, nin, zl, partb, nrm + nin, s));
      RSRR_HIP(hipMemcpyAsync(fro2.data(), nrm + nin, nin * sizeof(double), hipMemcpyDeviceToHost, s));
    } else {
      std::vector<const c128*> P(p->J);
      for (int k = 0; k < p->J; ++k) {
        c128* Pk = nullptr;
        char name[32];
        snprintf(name, sizeof(name), "fi_P%d", k);
        RSRR_TRY(ws.get<c128>(name, (size_t)n * nin, &Pk));
        switch (p->kinds[k]) {
          case RSRR_MAT_IDENTITY:
            RSRR_TRY((convert<double, double>(Vin, n, 0, Pk, n, 0, n, nin, 1, s)));
            break;
          case RSRR_MAT_DIAG:
            RSRR_TRY(diag_scale((const c128*)p->mats[k], Vin, n, Pk, n, n, nin, s));
            break;
          default:
            RSRR_TRY(zgemm(OP_N, OP_N, n, nin, n, ONE, p->mats[k], n, Vin, n, ZERO, Pk, n, s,
                           p->kinds[k] == RSRR_MAT_REAL));
        }
        P[k] = Pk;
      }
      std::vector<c128> hc((size_t)nin * p->J);
      {
        std::vector<cd> zl(nin), fv((size_t)nin * p->J);
        for (int q = 0; q < nin; ++q) zl[q] = lam[inside[q]];
        RSRR_TRY(eval_scalars(p, zl.data(), nin, fv.data(), nullptr));
        for (size_t e = 0; e < fv.size(); ++e) hc[e] = mk<double>(fv[e].real(), fv[e].imag());
      }
      RSRR_TRY(ws.get<c128>("fi_coef", hc.size(), &coef));
      RSRR_HIP(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      RSRR_TRY(combine_residual(zerov, n, P.data(), p->J, coef, n, 1, nin, Rr, n, s));
      for (int q = 0; q < nin; ++q) {
        cd ss(0, 0);
        for (int k = 0; k < p->J; ++k)
          for (int l = 0; l < p->J; ++l) {
            const cd gkl(p->gram[2 * (k * p->J + l)], p->gram[2 * (k * p->J + l) + 1]);
            const cd fk(hc[(size_t)q * p->J + k].re, hc[(size_t)q * p->J + k].im);
            const cd fl(hc[(size_t)q * p->J + l].re, hc[(size_t)q * p->J + l].im);
            ss += std::conj(fk) * fl * gkl;
          }
        fro2[q] = std::max(0.0, ss.real());
      }
    }
    RSRR_TRY(block_fro2(Rr, n, n, n, 1, nin, nrm, nullptr, s));
    std::vector<double> r2(nin);
    RSRR_HIP(hipMemcpyAsync(r2.data(), nrm, nin * sizeof(double), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    rel.resize(nin);
    raw.resize(nin);
    for (int q = 0; q < nin; ++q) {
      raw[q] = sqrt(r2[q]);                         // ||v|| = 1
      rel[q] = raw[q] / sqrt(fro2[q]);
    }
  }
  // keep, sort by (Re, Im), copy out
  std::vector<int> keep;
  for (int q = 0; q < nin; ++q)
    if (rel[q] <= prm->tol_res) keep.push_back(q);
  std::sort(keep.begin(), keep.end(), [&](int x, int y) {
    const cd a = lam[inside[x]], b = lam[inside[y]];
    return a.real() < b.real() || (a.real() == b.real() && a.imag() < b.imag());
  });
  const int ne = (int)keep.size();
  info.n_eig = ne;
  res->lambda.resize(ne);
  res->resid.resize(ne);
  res->resid_paper.resize(ne);
  res->V.resize((size_t)n * ne);
  for (int q = 0; q < ne; ++q) {
    const cd l = lam[inside[keep[q]]];
    res->lambda[q].re = l.real();
    res->lambda[q].im = l.imag();
    res->resid[q] = rel[keep[q]];
    res->resid_paper[q] = raw[keep[q]];
    RSRR_HIP(hipMemcpyAsync(res->V.data() + (size_t)q * n, Vin + (size_t)keep[q] * n,
                            n * sizeof(c128), hipMemcpyDeviceToHost, s));
  }
  RSRR_HIP(hipStreamSynchronize(s));
  info.t_residual = now_s() - t0;
  info.ws_bytes = (double)ws.bytes();
  if (have_wind && ne != info.n_wind) warn |= RSRR_WARN_COUNT_MISMATCH;
  return warn;
}

}  // namespace rsrr
