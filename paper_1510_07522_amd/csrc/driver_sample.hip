// Alg. 2, Steps 1-2: the sampling matrix S_hat = [T(z_0)^{-1} U ... T(z_{N-1})^{-1} U].
//
// complex128 form: assemble T(z_j) for all j, one batched LU, one batched solve.
// complex64 + refinement form: the same in complex64, then fp64 iterative
// refinement  R_j = U - T(z_j) Y_j (fp64),  D_j = T~_j^{-1} R_j (complex64),
// Y_j += D_j, with eta_j = ||R_j||_F / (||T(z_j)||_F ||Y_j||_F + ||U||_F).  A node
// is refined until eta_j reaches the fp64 floor (4 u) or stops falling (a sweep
// that does not halve it), at most ir_max_iter sweeps: the sampled blocks carry
// the accuracy a complex128 factorisation would give them, which clustered
// eigenvalues of the reduced problem need.  Nodes left above ir_tol are
// factored again in complex128.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bounds.h"
#include "driver.h"
#include "timers.h"

namespace rsrr {

// Scalar coefficients f_k(z_j) for the given nodes (row j holds J values).
static int node_coefs(const rsrr_problem* p, const std::vector<cd>& z, std::vector<c128>* f) {
  std::vector<cd> v(z.size() * p->J);
  const int st = eval_scalars(p, z.data(), z.size(), v.data(), nullptr);
  if (st < 0) return st;
  f->resize(v.size());
  for (size_t e = 0; e < v.size(); ++e) (*f)[e] = mk<double>(v[e].real(), v[e].imag());
  return ST_OK;
}

// ||T(z_j)||_F^2 for coefficient-form problems from the coefficient Gram.
static double fro2_coeff(const rsrr_problem* p, const c128* f) {
  cd s(0, 0);
  for (int k = 0; k < p->J; ++k)
    for (int l = 0; l < p->J; ++l) {
      const cd g(p->gram[2 * (k * p->J + l)], p->gram[2 * (k * p->J + l) + 1]);
      s += std::conj(cd(f[k].re, f[k].im)) * cd(f[l].re, f[l].im) * g;
    }
  return std::max(0.0, s.real());
}

template <typename R>
static int assemble_nodes(rsrr_problem* p, int nz, const c128* f_dev, const c128* z_dev,
                          cplx<R>* T, hipStream_t s) {
  const long n = p->n;
  if (p->bem) return assemble_bem<R>(p->n, p->xyz, p->h, nz, z_dev, T, n, n * n, s);
  std::vector<const void*> mats(p->mats.begin(), p->mats.end());
  CoeffSet cs;
  cs.n = p->n;
  cs.J = p->J;
  cs.kinds_host = p->kinds.data();
  cs.mats = mats.data();
  return assemble_coeff<R>(cs, nz, f_dev, T, n, n * n, s);
}

static int check_info(const int* info_dev, int batch, hipStream_t s, const std::vector<cd>& z) {
  std::vector<int> h(batch);
  RSRR_HIP(hipMemcpyAsync(h.data(), info_dev, batch * sizeof(int), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < batch; ++j)
    if (h[j] != 0)
      return set_error(ST_ESINGULAR, "T(z) is exactly singular at node %d (z = %.17g%+.17gi, pivot %d)",
                       j, z[j].real(), z[j].imag(), h[j]);
  return ST_OK;
}

// Residual R = U - T(z_j) Y_j (fp64) for all nodes; P is scratch for A_k Y.
// dst[:, q*L + c] = src[:, idx[q]*L + c]   (the columns of the listed nodes)
__global__ __launch_bounds__(256) void gather_node_cols_kernel(const c128* src, long lds, int rows, int L,
                                                               const int* idx, int count, c128* dst, long ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * L * count) return;
  const int r = (int)(e % rows);
  const long col = e / rows;
  const int q = (int)(col / L), c = (int)(col % L);
  dst[r + col * ldd] = src[r + ((long)idx[q] * L + c) * lds];
}

// dst[:, idx[q]*L + c] = (complex64) src[:, q*L + c]
__global__ __launch_bounds__(256) void scatter_node_cols_c64_kernel(const c128* src, long lds, int rows, int L,
                                                                    const int* idx, int count, c64* dst,
                                                                    long ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * L * count) return;
  const int r = (int)(e % rows);
  const long col = e / rows;
  const int q = (int)(col / L), c = (int)(col % L);
  const c128 v = src[r + col * lds];
  dst[r + ((long)idx[q] * L + c) * ldd] = mk<float>((float)v.re, (float)v.im);
}

// R_j = U - T(z_j) Y_j in fp64 for the N nodes whose solutions are the
// column blocks of Y.  BEM: the fp64 matrices of all sampling nodes are
// resident in Tres (node j at Tres + j n^2), and nodes[q] (host; none: q)
// names the node of block q.  Coefficient form: f_dev holds the N nodes'
// coefficients.
static int residual_fp64(rsrr_problem* p, int N, int L, const c128* f_dev, const c128* U, long ldu,
                         const c128* Y, long ldy, c128* Rb, hipStream_t s, const c128* Tres = nullptr,
                         const int* nodes = nullptr) {
  const int n = p->n;
  const long cols = (long)N * L;
  if (p->bem && Tres) {
    const long nn = (long)n * n;
    RSRR_TRY((convert<double, double>(U, ldu, 0, Rb, n, (long)L * n, n, L, N, s)));
    for (int q = 0; q < N; q += nodes ? 1 : N) {
      GemmBatch<double> g;
      g.M = n; g.N = L; g.K = n;
      g.alpha = mk<double>(-1, 0); g.beta = mk<double>(1, 0);
      g.A = Tres + (nodes ? nodes[q] : 0) * nn; g.lda = n; g.sA = nn;
      g.B = Y + (long)q * L * ldy; g.ldb = ldy; g.sB = (long)L * ldy;
      g.C = Rb + (long)q * L * n; g.ldc = n; g.sC = (long)L * n;
      g.batch = nodes ? 1 : N;
      g.gauss3m = true;        // normwise stable, which is what the backward error needs
      g.tag = "ir_residual_gemm";
      RSRR_TRY(gemm_batched<double>(g, s));
    }
    return ST_OK;
  }
  if (p->bem) return set_error(ST_EINVAL, "residual: the BEM matrices are not resident");
  std::vector<const c128*> P(p->J);
  for (int k = 0; k < p->J; ++k) {
    c128* Pk = nullptr;
    char name[32];
    snprintf(name, sizeof(name), "ir_P%d", k);
    RSRR_TRY(p->ws.get<c128>(name, (size_t)n * cols, &Pk));
    switch (p->kinds[k]) {
      case RSRR_MAT_IDENTITY:
        RSRR_TRY((convert<double, double>(Y, ldy, 0, Pk, n, 0, n, (int)cols, 1, s)));
        break;
      case RSRR_MAT_DIAG:
        RSRR_TRY(diag_scale((const c128*)p->mats[k], Y, ldy, Pk, n, n, (int)cols, s));
        break;
      default: {
        GemmBatch<double> g;
        g.M = n; g.N = (int)cols; g.K = n;
        g.A = p->mats[k]; g.lda = n;
        g.a_real = (p->kinds[k] == RSRR_MAT_REAL);
        g.B = Y; g.ldb = ldy;
        g.C = Pk; g.ldc = n;
        g.tag = "ir_residual_gemm";
        RSRR_TRY(gemm_batched<double>(g, s));
      }
    }
    P[k] = Pk;
  }
  return combine_residual(U, ldu, P.data(), p->J, f_dev, n, L, N, Rb, n, s);
}

// M_alpha = sum_i w_i s_i^alpha Y_i (eq. eq-malpha-qud).  For each probe column
// l, [M_0(:,l) ... M_{K'-1}(:,l)] = [Y_0(:,l) ... Y_{N-1}(:,l)] C with
// C[i][alpha] = w_i s_i^alpha: an n x N by N x K' product, batched over l
// (column l of block i sits at S + (i L + l) lds).
int moment_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* S, long lds,
                c128* M, long ldm) {
  hipStream_t s = p->stream;
  const int n = p->n, N = prm->N, L = prm->L, Kp = prm->Kp > 0 ? prm->Kp : prm->N;
  std::vector<cd> z, dz;
  contour_nodes(c, N, true, &z, &dz);
  const cd gamma(c->center.re, c->center.im);
  const double rho = std::max(c->a, c->b);
  std::vector<c128> hC((size_t)N * Kp);
  for (int i = 0; i < N; ++i) {
    const cd si = (z[i] - gamma) / rho;
    cd v = dz[i] / cd(0, 2.0 * M_PI);
    for (int a = 0; a < Kp; ++a) {
      hC[i + (size_t)a * N] = mk<double>(v.real(), v.imag());
      v *= si;
    }
  }
  c128* dC = nullptr;
  RSRR_TRY(p->ws.get<c128>("mm_C", hC.size(), &dC));
  RSRR_HIP(hipMemcpyAsync(dC, hC.data(), hC.size() * sizeof(c128), hipMemcpyHostToDevice, s));
  GemmBatch<double> g;
  g.tag = "moment_gemm";
  g.M = n; g.N = Kp; g.K = N;
  g.A = S; g.lda = (long)L * lds; g.sA = lds;
  g.B = dC; g.ldb = N; g.sB = 0;
  g.C = M; g.ldc = (long)L * ldm; g.sC = ldm;
  g.batch = L;
  RSRR_TRY(gemm_batched<double>(g, s));
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

int sample_begin(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* U, long ldu,
                 c128* S, long lds, rsrr_info* info, SamplePlan* sp) {
  SamplePlan& P = *sp;
  P.p = p; P.c = c; P.prm = prm; P.U = U; P.ldu = ldu; P.S = S; P.lds = lds; P.info = info;
  P.t0 = now_s();
  hipStream_t s = p->stream;
  const int n = p->n, N = prm->N, nb = prm->nb;
  const long nn = (long)n * n;
  contour_nodes(c, N, true, &P.z, nullptr);
  P.zc.assign(N, mk<double>(0, 0));
  for (int j = 0; j < N; ++j) P.zc[j] = mk<double>(P.z[j].real(), P.z[j].imag());
  P.f.clear();
  if (!p->bem) RSRR_TRY(node_coefs(p, P.z, &P.f));
  RSRR_TRY(p->ws.get<c128>("s_f", std::max<size_t>(1, P.f.size()), &P.f_dev));
  RSRR_TRY(p->ws.get<c128>("s_z", N, &P.z_dev));
  RSRR_TRY(p->ws.get<int>("s_ipiv", (size_t)N * n, &P.ipiv));
  RSRR_TRY(p->ws.get<int>("s_info", N, &P.infod));
  if (!P.f.empty())
    RSRR_HIP(hipMemcpyAsync(P.f_dev, P.f.data(), P.f.size() * sizeof(c128), hipMemcpyHostToDevice, s));
  RSRR_HIP(hipMemcpyAsync(P.z_dev, P.zc.data(), N * sizeof(c128), hipMemcpyHostToDevice, s));
  P.c64 = prm->precision != RSRR_PREC_C128;
  if (!P.c64) {
    c128 *T = nullptr, *dinv = nullptr;
    RSRR_TRY(p->ws.get<c128>("s_T128", (size_t)N * nn, &T));
    RSRR_TRY(p->ws.get<c128>("s_dinv128", LUWork<double>::dinv_elems(n, nb, N), &dinv));
    LUWork<double>& w = P.w128;
    w = LUWork<double>();
    w.n = n; w.nb = nb; w.batch = N; w.lda = n; w.sA = nn; w.A = T;
    w.ipiv = P.ipiv; w.dinv = dinv; w.info = P.infod;
    w.tag = "sample_lu_c128";
    w.pair = true;
    RSRR_TRY(p->ws.aux_stream(&w.aux, &w.ev_main, &w.ev_aux));
  } else {
    c64 *T = nullptr, *dinv = nullptr;
    RSRR_TRY(p->ws.get<c64>("s_T64", (size_t)N * nn, &T));
    RSRR_TRY(p->ws.get<c64>("s_dinv64", LUWork<float>::dinv_elems(n, nb, N), &dinv));
    LUWork<float>& w = P.w64;
    w = LUWork<float>();
    w.n = n; w.nb = nb; w.batch = N; w.lda = n; w.sA = nn; w.A = T;
    w.ipiv = P.ipiv; w.dinv = dinv; w.info = P.infod;
    w.tag = "sample_lu_c64";
    w.pair = true;
    RSRR_TRY(p->ws.aux_stream(&w.aux, &w.ev_main, &w.ev_aux));
    w.gauss3m = true;          // errors are removed by the fp64 refinement
  }
  return ST_OK;
}

int sample_assemble(SamplePlan* sp, hipStream_t s) {
  rsrr_problem* p = sp->p;
  const int N = sp->prm->N;
  if (sp->c64) return assemble_nodes<float>(p, N, sp->f_dev, sp->z_dev, sp->w64.A, s);
  return assemble_nodes<double>(p, N, sp->f_dev, sp->z_dev, sp->w128.A, s);
}

// Assembly and factorisation of the sampled matrices on stream s.
static int assemble_and_factor(SamplePlan* sp, hipStream_t s) {
  RSRR_TRY(sample_assemble(sp, s));
  if (sp->c64) return lu_factor<float>(sp->w64, s);
  return lu_factor<double>(sp->w128, s);
}

// Everything that decides the launches of assemble_and_factor: a graph
// captured for one key is replayed only for the same key.
static std::vector<long long> graph_key(const SamplePlan* sp) {
  const rsrr_problem* p = sp->p;
  std::vector<long long> k = {p->n, p->J, p->bem ? 1 : 0, sp->prm->N, sp->prm->nb, sp->c64 ? 1 : 0,
                              (long long)sp->f_dev, (long long)sp->z_dev, (long long)sp->ipiv, (long long)sp->infod,
                              (long long)p->xyz};
  long long hb;
  memcpy(&hb, &p->h, sizeof(hb));
  k.push_back(hb);
  for (int q = 0; q < p->J; ++q) {
    k.push_back(p->kinds[q]);
    k.push_back((long long)p->mats[q]);
  }
  if (sp->c64) {
    k.push_back((long long)sp->w64.A); k.push_back((long long)sp->w64.dinv);
    k.push_back((long long)sp->w64.aux);
  } else {
    k.push_back((long long)sp->w128.A); k.push_back((long long)sp->w128.dinv);
    k.push_back((long long)sp->w128.aux);
  }
  return k;
}

void SampleGraph::reset() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  key.clear();
}

SampleGraph::~SampleGraph() {
  reset();
  if (cap) (void)hipStreamDestroy(cap);
}

int sample_factor(SamplePlan* sp) {
  rsrr_problem* p = sp->p;
  hipStream_t s = p->stream;
  if (!sp->prm->graph || timers_on()) return assemble_and_factor(sp, s);
  // captured once per key on the handle's capture stream (the uploads the
  // launches read are complete first), replayed on the problem's stream
  SampleGraph& G = p->sgraph;
  std::vector<long long> key = graph_key(sp);
  if (!G.exec || G.key != key) {
    G.reset();
    if (!G.cap) RSRR_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    RSRR_HIP(hipStreamSynchronize(s));
    RSRR_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    const int st = assemble_and_factor(sp, G.cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(G.cap, &g);
    if (st < 0) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return set_error(ST_EHIP, "capture of the sampling launches: %s", hipGetErrorString(e));
    G.graph = g;
    RSRR_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    G.key = key;
  }
  RSRR_HIP(hipGraphLaunch(G.exec, s));
  return ST_OK;
}

int sample_end(SamplePlan* sp) {
  SamplePlan& P = *sp;
  rsrr_problem* p = P.p;
  const rsrr_params* prm = P.prm;
  const c128* U = P.U;
  const long ldu = P.ldu, lds = P.lds;
  c128* S = P.S;
  hipStream_t s = p->stream;
  const int n = p->n, N = prm->N, L = prm->L, nb = prm->nb;
  const long nn = (long)n * n;
  const std::vector<cd>& z = P.z;
  const std::vector<c128>& f = P.f;
  const std::vector<c128>& zc = P.zc;
  c128 *f_dev = P.f_dev, *z_dev = P.z_dev;
  int *ipiv = P.ipiv, *infod = P.infod;
  int ir_iters = 0, fallback = 0, warn = 0;
  (void)f_dev;

  if (!P.c64) {
    LUWork<double>& w = P.w128;
    RSRR_TRY(check_info(infod, N, s, z));
    RSRR_TRY(replicate<double>(U, ldu, S, lds, (long)L * lds, n, L, N, s));
    RSRR_TRY(lu_solve<double>(w, S, lds, (long)L * lds, L, s));
  } else {
    c64* Y32 = nullptr;
    c128* Rb = nullptr;
    double* nrm = nullptr;
    int* active_dev = nullptr;
    const long cols = (long)N * L;
    RSRR_TRY(p->ws.get<c64>("s_Y32", (size_t)n * cols, &Y32));
    RSRR_TRY(p->ws.get<c128>("s_R", (size_t)n * cols, &Rb));
    RSRR_TRY(p->ws.get<double>("s_nrm", 3 * (size_t)N + 1, &nrm));
    RSRR_TRY(p->ws.get<int>("s_active", N, &active_dev));
    double* fpart = nullptr;
    RSRR_TRY(p->ws.get<double>("s_fpart", (size_t)N * BLOCK_FRO2_PARTS, &fpart));
    LUWork<float>& w = P.w64;
    RSRR_TRY(check_info(infod, N, s, z));
    // Y0 = T~^{-1} U in complex64, widened to fp64
    RSRR_TRY((convert<float, double>(U, ldu, 0, Y32, n, (long)L * n, n, L, N, s)));
    RSRR_TRY(lu_solve<float>(w, Y32, n, (long)L * n, L, s));
    RSRR_TRY((convert<double, float>(Y32, n, (long)L * n, S, lds, (long)L * lds, n, L, N, s)));
    // normalisation terms of the backward error
    std::vector<double> fro2(N), u2(1);
    if (p->bem) {
      double* part = nullptr;
      RSRR_TRY(p->ws.get<double>("s_bempart", (size_t)N * n, &part));
      RSRR_TRY(bem_fro2(n, p->xyz, p->h, N, z_dev, part, nrm, s));
      RSRR_HIP(hipMemcpyAsync(fro2.data(), nrm, N * sizeof(double), hipMemcpyDeviceToHost, s));
    } else {
      for (int j = 0; j < N; ++j) fro2[j] = fro2_coeff(p, &f[(size_t)j * p->J]);
    }
    RSRR_TRY(block_fro2(U, ldu, 0, n, L, 1, nrm + 3 * N, fpart, s));
    RSRR_HIP(hipMemcpyAsync(u2.data(), nrm + 3 * N, sizeof(double), hipMemcpyDeviceToHost, s));
    // BEM: the fp64 T(z_j) of every node assembled once for all refinement
    // sweeps, in the buffer a complex128 fallback factors them in
    c128* Tres = nullptr;
    if (p->bem) {
      RSRR_TRY(p->ws.get<c128>("s_T128", (size_t)N * nn, &Tres));
      RSRR_TRY(assemble_bem<double>(n, p->xyz, p->h, N, z_dev, Tres, n, nn, s));
    }
    std::vector<int> active(N, 1);
    std::vector<double> r2(N), y2(N), eta_v(N, INFINITY);
    const double eta_floor = 4 * 1.1102230246251565e-16;
    // after the first sweep only the nodes still above ir_tol are refined:
    // their columns are gathered for the fp64 residual, and the solves skip
    // the others
    int *idx_dev = nullptr;
    c128 *Sa = nullptr, *Ra = nullptr, *fa_dev = nullptr;
    RSRR_TRY(p->ws.get<int>("s_idx", N, &idx_dev));
    std::vector<int> idx;
    int nact = N;
    for (int it = 0;; ++it) {
      // residuals of the nodes corrected in the last sweep (all in the first)
      const bool res_full = (nact == N);
      if (res_full) {
        RSRR_TRY(residual_fp64(p, N, L, f_dev, U, ldu, S, lds, Rb, s, Tres));
        RSRR_TRY(block_fro2(Rb, n, (long)L * n, n, L, N, nrm, fpart, s));
        RSRR_TRY(block_fro2(S, lds, (long)L * lds, n, L, N, nrm + N, fpart, s));
        RSRR_HIP(hipMemcpyAsync(r2.data(), nrm, N * sizeof(double), hipMemcpyDeviceToHost, s));
        RSRR_HIP(hipMemcpyAsync(y2.data(), nrm + N, N * sizeof(double), hipMemcpyDeviceToHost, s));
        RSRR_HIP(hipStreamSynchronize(s));
      } else {
        const int na = (int)idx.size();
        const long ca = (long)na * L;
        RSRR_TRY(p->ws.get<c128>("s_Sa", (size_t)n * ca, &Sa));
        RSRR_TRY(p->ws.get<c128>("s_Ra", (size_t)n * ca, &Ra));
        std::vector<c128> fa(p->bem ? 0 : (size_t)na * p->J);
        if (!p->bem)
          for (int q = 0; q < na; ++q)
            for (int k = 0; k < p->J; ++k) fa[(size_t)q * p->J + k] = f[(size_t)idx[q] * p->J + k];
        RSRR_TRY(p->ws.get<c128>("s_fa", std::max<size_t>(1, fa.size()), &fa_dev));
        if (!fa.empty())
          RSRR_HIP(hipMemcpyAsync(fa_dev, fa.data(), fa.size() * sizeof(c128), hipMemcpyHostToDevice, s));
        RSRR_HIP(hipMemcpyAsync(idx_dev, idx.data(), na * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_node_cols_kernel, dim3((unsigned)cdivl((long)n * ca, 256)), dim3(256), 0, s, S,
                           lds, n, L, idx_dev, na, Sa, (long)n);
        RSRR_LAUNCH_CHECK();
        RSRR_TRY(residual_fp64(p, na, L, fa_dev, U, ldu, Sa, n, Ra, s, Tres, idx.data()));
        RSRR_TRY(block_fro2(Ra, n, (long)L * n, n, L, na, nrm, fpart, s));
        RSRR_TRY(block_fro2(Sa, n, (long)L * n, n, L, na, nrm + N, fpart, s));
        std::vector<double> ra(na), ya(na);
        RSRR_HIP(hipMemcpyAsync(ra.data(), nrm, na * sizeof(double), hipMemcpyDeviceToHost, s));
        RSRR_HIP(hipMemcpyAsync(ya.data(), nrm + N, na * sizeof(double), hipMemcpyDeviceToHost, s));
        RSRR_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < na; ++q) { r2[idx[q]] = ra[q]; y2[idx[q]] = ya[q]; }
      }
      // only the nodes tested in this sweep can stay active
      const std::vector<int> was(active);
      nact = 0;
      double emax = 0;
      for (int j = 0; j < N; ++j) {
        if (!was[j]) continue;
        const double eta = sqrt(r2[j]) / (sqrt(fro2[j]) * sqrt(y2[j]) + sqrt(u2[0]));
        const bool falling = !(eta > 0.5 * eta_v[j]);
        active[j] = !(eta == eta) || (eta > eta_floor && falling);
        eta_v[j] = eta;
        nact += active[j];
        emax = std::max(emax, eta);
      }
      vlog("refinement sweep %d: %d of %d nodes still refined, max eta %.2e", it, nact, N, emax);
      if (nact == 0 || it >= prm->ir_max_iter) break;
      ir_iters = it + 1;
      const std::vector<int> tested(idx);
      idx.clear();
      for (int j = 0; j < N; ++j) if (active[j]) idx.push_back(j);
      RSRR_HIP(hipMemcpyAsync(active_dev, active.data(), N * sizeof(int), hipMemcpyHostToDevice, s));
      if (nact == N) {
        RSRR_TRY((convert<float, double>(Rb, n, (long)L * n, Y32, n, (long)L * n, n, L, N, s)));
        RSRR_TRY(lu_solve<float>(w, Y32, n, (long)L * n, L, s));
      } else {
        // residual columns of the active nodes, compacted into Rk in the order of idx
        std::vector<int> src;
        if (res_full) {
          src = idx;
        } else {
          for (size_t q = 0; q < tested.size(); ++q) if (active[tested[q]]) src.push_back((int)q);
        }
        const long ck = (long)src.size() * L;
        c128* Rk = nullptr;
        RSRR_TRY(p->ws.get<c128>("s_Rk", (size_t)n * ck, &Rk));
        RSRR_HIP(hipMemcpyAsync(idx_dev, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_node_cols_kernel, dim3((unsigned)cdivl((long)n * ck, 256)), dim3(256), 0, s,
                           res_full ? Rb : Ra, (long)n, n, L, idx_dev, (int)src.size(), Rk, (long)n);
        RSRR_LAUNCH_CHECK();
        RSRR_HIP(hipMemcpyAsync(idx_dev, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(scatter_node_cols_c64_kernel, dim3((unsigned)cdivl((long)n * ck, 256)), dim3(256), 0, s,
                           Rk, (long)n, n, L, idx_dev, (int)idx.size(), Y32, (long)n);
        RSRR_LAUNCH_CHECK();
        RSRR_TRY(lu_solve<float>(w, Y32, n, (long)L * n, L, s, active_dev));
      }
      RSRR_TRY(add_correction(S, lds, (long)L * lds, Y32, n, (long)L * n, n, L, N, active_dev, s));
    }
    // complex128 fallback for the nodes left above ir_tol
    std::vector<int> bad;
    for (int j = 0; j < N; ++j) if (!(eta_v[j] <= prm->ir_tol)) bad.push_back(j);
    if (!bad.empty() && n > LU_MAX_N_C128)
      return set_error(ST_ENOTCONV, "refinement left %d node(s) above ir_tol=%g and the complex128 fallback "
                       "goes up to order %d (n=%d)", (int)bad.size(), prm->ir_tol, LU_MAX_N_C128, n);
    if (!bad.empty()) {
      fallback = (int)bad.size();
      warn |= RSRR_WARN_IR_FALLBACK;
      const int nbad = (int)bad.size();
      std::vector<cd> zb(nbad);
      std::vector<c128> zbc(nbad), fb;
      for (int q = 0; q < nbad; ++q) { zb[q] = z[bad[q]]; zbc[q] = zc[bad[q]]; }
      if (!p->bem) RSRR_TRY(node_coefs(p, zb, &fb));
      c128 *Tb = nullptr, *dinvb = nullptr, *Yb = nullptr, *fbd = nullptr, *zbd = nullptr;
      RSRR_TRY(p->ws.get<c128>("s_T128", (size_t)nbad * nn, &Tb));
      RSRR_TRY(p->ws.get<c128>("s_dinv128", LUWork<double>::dinv_elems(n, nb, nbad), &dinvb));
      RSRR_TRY(p->ws.get<c128>("s_Yfb", (size_t)nbad * n * L, &Yb));
      RSRR_TRY(p->ws.get<c128>("s_ffb", std::max<size_t>(1, fb.size()), &fbd));
      RSRR_TRY(p->ws.get<c128>("s_zfb", nbad, &zbd));
      if (!fb.empty()) RSRR_HIP(hipMemcpyAsync(fbd, fb.data(), fb.size() * sizeof(c128), hipMemcpyHostToDevice, s));
      RSRR_HIP(hipMemcpyAsync(zbd, zbc.data(), nbad * sizeof(c128), hipMemcpyHostToDevice, s));
      RSRR_TRY(assemble_nodes<double>(p, nbad, fbd, zbd, Tb, s));
      LUWork<double> wb;
      wb.n = n; wb.nb = nb; wb.batch = nbad; wb.lda = n; wb.sA = nn; wb.A = Tb;
      wb.ipiv = ipiv; wb.dinv = dinvb; wb.info = infod;
      wb.tag = "fallback_lu_c128";
      wb.pair = true;
      RSRR_TRY(p->ws.aux_stream(&wb.aux, &wb.ev_main, &wb.ev_aux));
      RSRR_TRY(lu_factor<double>(wb, s));
      RSRR_TRY(check_info(infod, nbad, s, zb));
      RSRR_TRY(replicate<double>(U, ldu, Yb, n, (long)n * L, n, L, nbad, s));
      RSRR_TRY(lu_solve<double>(wb, Yb, n, (long)n * L, L, s));
      for (int q = 0; q < nbad; ++q)
        RSRR_TRY((convert<double, double>(Yb + (long)q * n * L, n, 0, S + (long)bad[q] * L * lds, lds,
                                          0, n, L, 1, s)));
    }
  }
  RSRR_HIP(hipStreamSynchronize(s));
  if (P.info) {
    P.info->n = n;
    P.info->N = N;
    P.info->L = L;
    P.info->ir_iters = ir_iters;
    P.info->ir_fallback = fallback;
    P.info->t_sample = now_s() - P.t0;
  }
  return warn;
}

int sample_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* U,
                long ldu, c128* S, long lds, rsrr_info* info) {
  SamplePlan sp;
  RSRR_TRY(sample_begin(p, c, prm, U, ldu, S, lds, info, &sp));
  RSRR_TRY(sample_factor(&sp));
  return sample_end(&sp);
}

}  // namespace rsrr
