// Schur decomposition A = Z T Z^H of a large dense complex matrix by spectral
// divide and conquer, followed by eigenvectors of T.
//
// A diagonal block B of the current T is split along a line through the mean
// of its eigenvalues: the matrix sign function S = sign(B - sigma I) (or of
// -i (B - i sigma I) for a horizontal line) is computed by the scaled Newton
// iteration X <- (mu X + X^{-1}/mu)/2, mu = sqrt(||X^{-1}||_F / ||X||_F);
// P = (I + S)/2 projects on the eigenvalues right of (above) the line, rank
// k = tr P.  Q = [Q1 Q2] with Q1 an orthonormal basis of range(P) and Q2 of its
// orthogonal complement makes Q^H B Q block upper triangular; T and Z are
// updated with GEMMs and both diagonal blocks are split further.  Blocks of
// at most DC_LEAF rows are put in Schur form concurrently, one workgroup each.
// Inversions use the batched LU of the sampling step; bases use the pivoted
// Cholesky / Cholesky-QR routines of the orthonormalisation step.
#include <algorithm>
#include <complex>
#include <cmath>
#include <vector>

#include "driver.h"
#include "eig.h"
#include "timers.h"

namespace rsrr {

static const c128 ONE = {1, 0}, ZERO = {0, 0}, MONE = {-1, 0};

static int zg(int opA, int opB, int M, int N, int K, c128 alpha, const c128* A, long lda,
              const c128* B, long ldb, c128 beta, c128* C, long ldc, hipStream_t s) {
  GemmBatch<double> g;
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.tag = "dc_gemm";
  g.gauss3m = true;
  return gemm_batched<double>(g, s);
}

// dst = rot * (src - shift I)   (len x len)
__global__ __launch_bounds__(256) void shift_copy_kernel(const c128* src, long lds, c128* dst, long ldd,
                                                         int len, c128 shift, c128 rot) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)len * len) return;
  const int r = (int)(e % len), c = (int)(e / len);
  c128 v = src[r + (long)c * lds];
  if (r == c) v = v - shift;
  dst[r + (long)c * ldd] = rot * v;
}

// per-workgroup partial sums over column ranges: out[2*blk] = sum |X|^2,
// out[2*blk+1] = sum |Y - X|^2 (when Y given)
constexpr int FCOLS = 8;
__global__ __launch_bounds__(256) void fro_partial_kernel(const c128* X, const c128* Y, long ld, int rows,
                                                          int cols, double* out, int sub_identity = 0) {
  __shared__ double r0[256], r1[256];
  const int c0 = blockIdx.x * FCOLS;
  double a = 0, b = 0;
  for (int c = c0; c < min(cols, c0 + FCOLS); ++c)
    for (int r = threadIdx.x; r < rows; r += 256) {
      c128 x = X[r + (long)c * ld];
      if (sub_identity && r == c) x.re -= 1.0;
      a += abs2(x);
      if (Y) b += abs2(Y[r + (long)c * ld] - x);
    }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) { r0[threadIdx.x] += r0[threadIdx.x + o]; r1[threadIdx.x] += r1[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[2 * blockIdx.x] = r0[0]; out[2 * blockIdx.x + 1] = r1[0]; }
}

// Y <- a X + b Y
__global__ __launch_bounds__(256) void axpby_kernel(const c128* X, c128* Y, long ld, int len, double a,
                                                    double b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)len * len) return;
  const int r = (int)(e % len), c = (int)(e / len);
  const c128 x = X[r + (long)c * ld], y = Y[r + (long)c * ld];
  Y[r + (long)c * ld] = mk<double>(a * x.re + b * y.re, a * x.im + b * y.im);
}

// P = (I + S)/2 in place; diagonal copied to diag[]
__global__ __launch_bounds__(256) void projector_kernel(c128* S, long ld, int len, c128* diag) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)len * len) return;
  const int r = (int)(e % len), c = (int)(e / len);
  c128 v = 0.5 * S[r + (long)c * ld];
  if (r == c) { v.re += 0.5; diag[r] = v; }
  S[r + (long)c * ld] = v;
}

__global__ void diag_copy_kernel(const c128* A, long lda, int len, c128* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = A[i + (long)i * lda];
}

__global__ __launch_bounds__(256) void zero_block_kernel(c128* A, long lda, int rows, int cols) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  A[(e % rows) + (e / rows) * lda] = mk<double>(0, 0);
}

static unsigned nblk(long cnt) { return (unsigned)cdivl(cnt, 256); }

struct DcWork {
  c128 *X, *Y, *LU, *dinv, *Q, *tmp, *tmp2, *diag;
  int *ipiv, *info;
  double* part;
  int cap;
};

static int fro_sums(const c128* X, const c128* Y, long ld, int len, DcWork& w, hipStream_t s,
                    double* fx, double* fd, int sub_identity = 0) {
  const int nb = (len + FCOLS - 1) / FCOLS;
  hipLaunchKernelGGL(fro_partial_kernel, dim3(nb), dim3(256), 0, s, X, Y, ld, len, len, w.part, sub_identity);
  RSRR_LAUNCH_CHECK();
  std::vector<double> h(2 * nb);
  RSRR_HIP(hipMemcpyAsync(h.data(), w.part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  double a = 0, b = 0;
  for (int i = 0; i < nb; ++i) { a += h[2 * i]; b += h[2 * i + 1]; }
  *fx = a;
  if (fd) *fd = b;
  return ST_OK;
}

static int host_diag(const c128* A, long lda, int len, DcWork& w, hipStream_t s, std::vector<c128>* d) {
  hipLaunchKernelGGL(diag_copy_kernel, dim3((unsigned)cdivl(len, 256)), dim3(256), 0, s, A, lda, len, w.diag);
  RSRR_LAUNCH_CHECK();
  d->resize(len);
  RSRR_HIP(hipMemcpyAsync(d->data(), w.diag, len * sizeof(c128), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

// Sign function of X (len x len, in w.X, destroyed); result in w.X.
// Scaled Newton X <- (mu X + X^{-1}/mu)/2 while far from convergence; once the
// relative change is below 1e-2 and ||X^2 - I||_F / sqrt(len) < 0.5, the
// inverse-free Newton-Schulz step X <- X (3I - X^2)/2 (two GEMMs) finishes.
// Returns -1 if X became singular or the iteration did not converge.
static int newton_sign(int len, DcWork& w, Arena& ws, hipStream_t s, int* iters) {
  const long ll = (long)len * len;
  const double sq = sqrt((double)len);
  LUWork<double> lw;
  // one matrix: the single-workgroup panel dominates, and a narrower panel
  // re-reads fewer columns per micro-panel (measured best of 16 / 32 / 64)
  lw.n = len; lw.nb = 32; lw.batch = 1; lw.lda = len; lw.sA = ll;
  lw.ipiv = w.ipiv; lw.dinv = w.dinv; lw.info = w.info;
  lw.tag = "dc_lu";
  lw.gauss3m = true;
  lw.pair = true;
  RSRR_TRY(ws.aux_stream(&lw.aux, &lw.ev_main, &lw.ev_aux));
  bool scaling = true, schulz = false;
  double prev_r = 1e300;
  for (int it = 0; it < 100; ++it) {
    if (schulz) {
      RSRR_TRY(zg(OP_N, OP_N, len, len, len, ONE, w.X, len, w.X, len, ZERO, w.Y, len, s));   // X^2
      double r2 = 0;
      RSRR_TRY(fro_sums(w.Y, nullptr, len, len, w, s, &r2, nullptr, 1));
      const double r = sqrt(r2) / sq;
      if (r < 1e-13) { *iters = it; return ST_OK; }
      // stagnation at the rounding level of a non-normal S: converged
      if (r < 1e-8 && r > 0.5 * prev_r) { *iters = it; return ST_OK; }
      prev_r = r;
      if (!(r < 0.5)) { schulz = false; prev_r = 1e300; continue; }   // back to Newton
      RSRR_TRY(zg(OP_N, OP_N, len, len, len, ONE, w.X, len, w.Y, len, ZERO, w.LU, len, s));  // X^3
      hipLaunchKernelGGL(axpby_kernel, dim3(nblk(ll)), dim3(256), 0, s, w.X, w.LU, len, len, 1.5, -0.5);
      RSRR_LAUNCH_CHECK();
      std::swap(w.X, w.LU);
      continue;
    }
    lw.A = w.LU;
    RSRR_TRY((convert<double, double>(w.X, len, 0, w.LU, len, 0, len, len, 1, s)));
    RSRR_TRY(set_identity(w.Y, len, len, s));
    RSRR_TRY(lu_factor<double>(lw, s));
    int info = 0;
    RSRR_HIP(hipMemcpyAsync(&info, w.info, sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    if (info) { *iters = it; return -1; }
    RSRR_TRY(lu_solve<double>(lw, w.Y, len, ll, len, s));
    double fx = 0, fy = 0;
    RSRR_TRY(fro_sums(w.X, nullptr, len, len, w, s, &fx, nullptr));
    RSRR_TRY(fro_sums(w.Y, nullptr, len, len, w, s, &fy, nullptr));
    const double mu = scaling ? sqrt(sqrt(fy) / sqrt(fx)) : 1.0;
    // Y <- (mu X + Y / mu) / 2
    hipLaunchKernelGGL(axpby_kernel, dim3(nblk(ll)), dim3(256), 0, s, w.X, w.Y, len, len, 0.5 * mu, 0.5 / mu);
    RSRR_LAUNCH_CHECK();
    double fn = 0, fd = 0;
    RSRR_TRY(fro_sums(w.Y, w.X, len, len, w, s, &fn, &fd));
    std::swap(w.X, w.Y);
    const double rel = sqrt(fd / std::max(fn, 1e-300));
    if (!(rel == rel)) { *iters = it; return -1; }
    if (rel < 1e-2) { scaling = false; schulz = true; }
  }
  *iters = 100;
  return -1;
}

// ---------------------------------------------------------------- batched
// The blocks of one level of the split tree are iterated together: block b is
// stored at X + b * Lmax^2 with leading dimension Lmax (the largest block of
// the batch) and padded with the identity, which every update keeps exact
// (the padding is reset after each step), so the blocks never interact.
__global__ __launch_bounds__(256) void pad_identity_kernel(c128* X, int Lmax, const int* lens) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)Lmax * Lmax) return;
  const int b = blockIdx.y, len = lens[b];
  const int r = (int)(e % Lmax), c = (int)(e / Lmax);
  if (r < len && c < len) return;
  X[(long)b * Lmax * Lmax + e] = mk<double>(r == c ? 1.0 : 0.0, 0);
}

// out[2*(b*nch + x)] = sum |X_b|^2 over FCOLS columns of block b (minus I if
// sub_identity), out[... + 1] = sum |Y_b - X_b|^2 (when Y given)
__global__ __launch_bounds__(256) void fro_partial_batched_kernel(const c128* X, const c128* Y, int Lmax,
                                                                  const int* lens, int nch, double* out,
                                                                  int sub_identity) {
  __shared__ double r0[256], r1[256];
  const int b = blockIdx.y, len = lens[b];
  const long base = (long)b * Lmax * Lmax;
  const int c0 = blockIdx.x * FCOLS;
  double a = 0, d = 0;
  for (int c = c0; c < min(len, c0 + FCOLS); ++c)
    for (int r = threadIdx.x; r < len; r += 256) {
      c128 x = X[base + r + (long)c * Lmax];
      if (sub_identity && r == c) x.re -= 1.0;
      a += abs2(x);
      if (Y) d += abs2(Y[base + r + (long)c * Lmax] - x);
    }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = d;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) { r0[threadIdx.x] += r0[threadIdx.x + o]; r1[threadIdx.x] += r1[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * ((long)b * nch + blockIdx.x)] = r0[0];
    out[2 * ((long)b * nch + blockIdx.x) + 1] = r1[0];
  }
}

// Y_b <- coef[2b] X_b + coef[2b+1] Y_b
__global__ __launch_bounds__(256) void axpby_batched_kernel(const c128* X, c128* Y, int Lmax, const double* coef) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)Lmax * Lmax) return;
  const int b = blockIdx.y;
  const double a = coef[2 * b], c = coef[2 * b + 1];
  const long i = (long)b * Lmax * Lmax + e;
  const c128 x = X[i], y = Y[i];
  Y[i] = mk<double>(a * x.re + c * y.re, a * x.im + c * y.im);
}

struct DcBatch {
  int nbk = 0, Lmax = 0;
  std::vector<int> lens;
  int* lens_dev = nullptr;
  c128 *X = nullptr, *Y = nullptr, *LU = nullptr, *dinv = nullptr;
  int *ipiv = nullptr, *info = nullptr;
  double *part = nullptr, *coef = nullptr;
  c128* diag = nullptr;
};

static int fro_batched(const c128* X, const c128* Y, DcBatch& bt, hipStream_t s, std::vector<double>* fx,
                       std::vector<double>* fd, int sub_identity = 0) {
  const int nch = (bt.Lmax + FCOLS - 1) / FCOLS;
  hipLaunchKernelGGL(fro_partial_batched_kernel, dim3(nch, bt.nbk), dim3(256), 0, s, X, Y, bt.Lmax, bt.lens_dev,
                     nch, bt.part, sub_identity);
  RSRR_LAUNCH_CHECK();
  std::vector<double> h(2 * (size_t)nch * bt.nbk);
  RSRR_HIP(hipMemcpyAsync(h.data(), bt.part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  fx->assign(bt.nbk, 0.0);
  if (fd) fd->assign(bt.nbk, 0.0);
  for (int b = 0; b < bt.nbk; ++b)
    for (int x = 0; x < nch; ++x) {
      (*fx)[b] += h[2 * ((size_t)b * nch + x)];
      if (fd) (*fd)[b] += h[2 * ((size_t)b * nch + x) + 1];
    }
  return ST_OK;
}

static int axpby_batched(const c128* X, c128* Y, DcBatch& bt, const std::vector<double>& coef, hipStream_t s) {
  RSRR_HIP(hipMemcpyAsync(bt.coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const long ll = (long)bt.Lmax * bt.Lmax;
  hipLaunchKernelGGL(axpby_batched_kernel, dim3(nblk(ll), bt.nbk), dim3(256), 0, s, X, Y, bt.Lmax, bt.coef);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

static int pad_identity(c128* X, DcBatch& bt, hipStream_t s) {
  const long ll = (long)bt.Lmax * bt.Lmax;
  hipLaunchKernelGGL(pad_identity_kernel, dim3(nblk(ll), bt.nbk), dim3(256), 0, s, X, bt.Lmax, bt.lens_dev);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// Principal Pade iteration of order 2m for the sign function in partial
// fractions: r_m(x) = tanh(2m artanh x) = sum_j w_j x / (x^2 + beta_j^2),
// beta_j = tan(pi (2j-1) / (4m)), w_j from the residues at x = i beta_j.  One
// step X <- sum_j w_j Z_j with (X^2 + beta_j^2 I) Z_j = X needs m independent
// LU solves (one batch) and gains a factor 2m per step near the split line,
// where Newton gains 2.
constexpr int PADE_M = 4;
struct PadeCoef { double b2[PADE_M]; double w[PADE_M]; };

static PadeCoef pade_coefficients() {
  PadeCoef pc;
  const int p = 2 * PADE_M;
  for (int j = 0; j < PADE_M; ++j) {
    const double beta = tan(M_PI * (2 * j + 1) / (2.0 * p));
    const cd x(0.0, beta);
    const cd num = std::pow(1.0 + x, p) - std::pow(1.0 - x, p);
    const cd dden = (double)p * (std::pow(1.0 + x, p - 1) - std::pow(1.0 - x, p - 1));
    pc.b2[j] = beta * beta;
    pc.w[j] = (2.0 * num / dden).real();
  }
  return pc;
}

// slot q = j * nbk + b:  LU_q = X2_b + beta_j^2 I,  Z_q = X_b
__global__ __launch_bounds__(256) void pade_setup_kernel(const c128* X2, const c128* X, int nbk, int L,
                                                         PadeCoef pc, c128* LU, c128* Z) {
  const long ll = (long)L * L;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ll) return;
  const int q = blockIdx.y, j = q / nbk, b = q % nbk;
  c128 v = X2[(long)b * ll + e];
  if (e % L == e / L) v.re += pc.b2[j];
  LU[(long)q * ll + e] = v;
  Z[(long)q * ll + e] = X[(long)b * ll + e];
}

// Y_b = sum_j w_j Z_{j * nbk + b}
__global__ __launch_bounds__(256) void pade_combine_kernel(const c128* Z, int nbk, int L, PadeCoef pc, c128* Y) {
  const long ll = (long)L * L;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ll) return;
  const int b = blockIdx.y;
  c128 acc = mk<double>(0, 0);
#pragma unroll
  for (int j = 0; j < PADE_M; ++j) acc = acc + pc.w[j] * Z[((long)j * nbk + b) * ll + e];
  Y[(long)b * ll + e] = acc;
}

// Sign functions of the nbk matrices in bt.X (destroyed; results in bt.X),
// run on all of them in lock step: DC_NEWTON_STEPS Newton steps with a scaling
// factor per matrix, then Pade steps of order 2*PADE_M until ||X^2 - I||_F / sqrt(len) <
// 0.3 for every block (or the relative change is below 1e-2), then
// Newton-Schulz to convergence.  ok[b] = 0 if matrix b became
// singular or did not converge (its slot is reset to the identity so it stays
// inert).
// scaled Newton steps before the Pade steps (each is one LU and inverse per
// block; they move the spectrum towards +-1 faster per unit of work than a
// Pade step while it is far from converged)
constexpr int DC_NEWTON_STEPS = 2;

static int newton_sign_batched(DcBatch& bt, Arena& ws, hipStream_t s, std::vector<int>* ok, int* iters) {
  const int nbk = bt.nbk, L = bt.Lmax;
  const long ll = (long)L * L;
  LUWork<double> lw;
  lw.n = L; lw.nb = 32; lw.batch = nbk; lw.lda = L; lw.sA = ll;
  lw.ipiv = bt.ipiv; lw.dinv = bt.dinv; lw.info = bt.info;
  lw.tag = "dc_lu";
  lw.gauss3m = true;
  lw.pair = true;
  RSRR_TRY(ws.aux_stream(&lw.aux, &lw.ev_main, &lw.ev_aux));
  GemmBatch<double> g;
  g.tag = "dc_gemm";
  g.gauss3m = true;
  g.M = g.N = g.K = L;
  g.lda = g.ldb = g.ldc = L;
  g.sA = g.sB = g.sC = ll;
  g.batch = nbk;
  ok->assign(nbk, 1);
  std::vector<int> done(nbk, 0);
  std::vector<double> prev(nbk, 1e300), coef(2 * nbk), fx, fy, fn, fd;
  bool scaling = true, schulz = false;
  int n_newton = 0, n_schulz = 0, n_pade = 0;
  const PadeCoef pc = pade_coefficients();
  const int nq = PADE_M * nbk;
  c128 *LUp = nullptr, *Zp = nullptr, *dinvp = nullptr;
  int *ipivp = nullptr, *infop = nullptr;
  RSRR_TRY(ws.get<c128>("dcp_LU", (size_t)nq * ll, &LUp));
  RSRR_TRY(ws.get<c128>("dcp_Z", (size_t)nq * ll, &Zp));
  RSRR_TRY(ws.get<c128>("dcp_dinv", LUWork<double>::dinv_elems(L, 32, nq), &dinvp));
  RSRR_TRY(ws.get<int>("dcp_ipiv", (size_t)nq * L, &ipivp));
  RSRR_TRY(ws.get<int>("dcp_info", nq, &infop));
  LUWork<double> lwp = lw;
  lw.full_swap = true;           // the Newton steps invert (lu_inverse)
  int* nperm = nullptr;
  RSRR_TRY(ws.get<int>("dcp_perm", (size_t)nbk * L, &nperm));
  RSRR_TRY(ws.get<int>("dcn_lperm", (size_t)nbk * lw.npanel() * L, &lw.lperm));
  lwp.batch = nq; lwp.A = LUp; lwp.ipiv = ipivp; lwp.dinv = dinvp; lwp.info = infop;
  auto reset = [&](int b) -> int {
    (*ok)[b] = 0;
    done[b] = 1;
    return set_identity(bt.X + (long)b * ll, L, L, s);
  };
  for (int it = 0; it < 100; ++it) {
    if (schulz) {
      g.alpha = ONE; g.beta = ZERO;
      g.A = bt.X; g.B = bt.X; g.C = bt.Y;
      RSRR_TRY(gemm_batched<double>(g, s));                         // X^2
      std::vector<double> r2;
      RSRR_TRY(fro_batched(bt.Y, nullptr, bt, s, &r2, nullptr, 1));
      bool back = false, all = true;
      for (int b = 0; b < nbk; ++b) {
        if (done[b]) continue;
        const double r = sqrt(r2[b] / bt.lens[b]);
        // converged, or stagnating at the rounding level of a non-normal S
        if (r < 1e-13 || (r < 1e-8 && r > 0.5 * prev[b])) { done[b] = 1; continue; }
        prev[b] = r;
        all = false;
        if (!(r < 0.5)) back = true;
      }
      if (all) {
        *iters = it;
        vlog("dc sign batch of %d (len %d): %d newton + %d pade + %d schulz steps", nbk, L, n_newton, n_pade, n_schulz);
        return ST_OK;
      }
      if (back) {
        schulz = false;
        std::fill(prev.begin(), prev.end(), 1e300);
        continue;
      }
      g.A = bt.X; g.B = bt.Y; g.C = bt.LU;
      ++n_schulz;
      RSRR_TRY(gemm_batched<double>(g, s));                         // X^3
      for (int b = 0; b < nbk; ++b) { coef[2 * b] = -0.5; coef[2 * b + 1] = 1.5; }
      RSRR_TRY(axpby_batched(bt.LU, bt.X, bt, coef, s));           // X <- 1.5 X - 0.5 X^3
      RSRR_TRY(pad_identity(bt.X, bt, s));
      continue;
    }
    if (it >= DC_NEWTON_STEPS) {  // Pade step
      g.alpha = ONE; g.beta = ZERO;
      g.A = bt.X; g.B = bt.X; g.C = bt.Y;
      RSRR_TRY(gemm_batched<double>(g, s));                         // X^2
      {
        // once every block is close to an involution, Newton-Schulz (two
        // products per step, quadratic) finishes faster than another Pade step
        std::vector<double> r2;
        RSRR_TRY(fro_batched(bt.Y, nullptr, bt, s, &r2, nullptr, 1));
        bool close = true;
        for (int b = 0; b < nbk && close; ++b)
          if (!done[b] && !(sqrt(r2[b] / bt.lens[b]) < 0.3)) close = false;
        if (close) {
          schulz = true;
          std::fill(prev.begin(), prev.end(), 1e300);
          continue;
        }
      }
      hipLaunchKernelGGL(pade_setup_kernel, dim3(nblk(ll), nq), dim3(256), 0, s, bt.Y, bt.X, nbk, L, pc, LUp, Zp);
      RSRR_LAUNCH_CHECK();
      RSRR_TRY(lu_factor<double>(lwp, s));
      std::vector<int> infq(nq);
      RSRR_HIP(hipMemcpyAsync(infq.data(), infop, nq * sizeof(int), hipMemcpyDeviceToHost, s));
      RSRR_TRY(lu_solve<double>(lwp, Zp, L, ll, L, s));
      hipLaunchKernelGGL(pade_combine_kernel, dim3(nblk(ll), nbk), dim3(256), 0, s, Zp, nbk, L, pc, bt.Y);
      RSRR_LAUNCH_CHECK();
      RSRR_TRY(pad_identity(bt.Y, bt, s));
      RSRR_TRY(fro_batched(bt.Y, bt.X, bt, s, &fn, &fd));
      std::swap(bt.X, bt.Y);
      ++n_pade;
      bool all = true, any = false;
      for (int b = 0; b < nbk; ++b) {
        if (done[b]) continue;
        int sing = 0;
        for (int j = 0; j < PADE_M; ++j) sing |= infq[j * nbk + b];
        const double rel = sqrt(fd[b] / std::max(fn[b], 1e-300));
        if (sing || !(rel == rel)) { RSRR_TRY(reset(b)); continue; }
        if (!(rel < 1e-2)) all = false;
      }
      if (all) { schulz = true; std::fill(prev.begin(), prev.end(), 1e300); }
      for (int b = 0; b < nbk; ++b) any = any || !done[b];
      if (!any) { *iters = it; return ST_OK; }
      continue;
    }
    RSRR_HIP(hipMemcpyAsync(bt.LU, bt.X, (size_t)nbk * ll * sizeof(c128), hipMemcpyDeviceToDevice, s));
    ++n_newton;
    lw.A = bt.LU;
    RSRR_TRY(lu_factor<double>(lw, s));
    std::vector<int> info(nbk);
    RSRR_HIP(hipMemcpyAsync(info.data(), bt.info, nbk * sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    RSRR_TRY(lu_inverse<double>(lw, Zp, bt.Y, L, ll, nperm, s));   // Y = X^{-1}; Zp is work space
    RSRR_TRY(fro_batched(bt.X, nullptr, bt, s, &fx, nullptr));
    RSRR_TRY(fro_batched(bt.Y, nullptr, bt, s, &fy, nullptr));
    for (int b = 0; b < nbk; ++b) {
      const double mu = (scaling && fx[b] > 0 && fy[b] > 0) ? sqrt(sqrt(fy[b]) / sqrt(fx[b])) : 1.0;
      coef[2 * b] = 0.5 * mu;
      coef[2 * b + 1] = 0.5 / mu;
    }
    RSRR_TRY(axpby_batched(bt.X, bt.Y, bt, coef, s));               // Y <- (mu X + Y/mu)/2
    RSRR_TRY(pad_identity(bt.Y, bt, s));
    RSRR_TRY(fro_batched(bt.Y, bt.X, bt, s, &fn, &fd));
    std::swap(bt.X, bt.Y);
    bool all = true;
    for (int b = 0; b < nbk; ++b) {
      if (done[b]) continue;
      const double rel = sqrt(fd[b] / std::max(fn[b], 1e-300));
      if (info[b] || !(rel == rel)) { RSRR_TRY(reset(b)); continue; }
      if (!(rel < 1e-2)) all = false;
    }
    if (all) { scaling = false; schulz = true; std::fill(prev.begin(), prev.end(), 1e300); }
    bool any = false;
    for (int b = 0; b < nbk; ++b) any = any || !done[b];
    if (!any) { *iters = it; return ST_OK; }
  }
  for (int b = 0; b < nbk; ++b)
    if (!done[b]) (*ok)[b] = 0;
  *iters = 100;
  return ST_OK;
}

// Deterministic complex Gaussian entries (x + iy)/sqrt(2): splitmix64 of the
// element index and the seed, two uniforms per entry, Box-Muller.
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void gauss_fill_kernel(c128* X, long ldx, int rows, int cols, uint64_t seed) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const uint64_t a = mix64(seed ^ (2 * (uint64_t)e)), b = mix64(seed ^ (2 * (uint64_t)e + 1));
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
  const double r = sqrt(-2.0 * log(u1)) * 0.7071067811865476;
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  X[(e % rows) + (long)(e / rows) * ldx] = mk<double>(r * cs, r * sn);
}

// Q2 (len x (len-k)): an orthonormal basis of the orthogonal complement of
// range(Q1) from a seeded Gaussian block, projected against Q1 twice and
// orthonormalised by Cholesky-QR, then projected and orthonormalised once
// more.  A Gaussian block restricted to the complement is well conditioned
// with high probability; *ok = false if a Cholesky factorisation breaks down.
static int complement_basis(const c128* Q1, int len, int k, c128* Q2, DcWork& w, Arena& ws, hipStream_t s,
                            bool* ok) {
  const int r = len - k;
  *ok = false;
  hipLaunchKernelGGL(gauss_fill_kernel, dim3(nblk((long)len * r)), dim3(256), 0, s, Q2, (long)len, len, r,
                     0x5DEECE66Dull * (uint64_t)len + (uint64_t)k);
  RSRR_LAUNCH_CHECK();
  for (int pass = 0; pass < 3; ++pass) {
    RSRR_TRY(zg(OP_C, OP_N, k, r, len, ONE, Q1, len, Q2, len, ZERO, w.tmp, k, s));
    RSRR_TRY(zg(OP_N, OP_N, len, r, k, MONE, Q1, len, w.tmp, k, ONE, Q2, len, s));
    if (pass >= 1) {
      bool good = false;
      RSRR_TRY(cholqr(Q2, len, len, r, ws, s, &good));
      if (!good) return ST_OK;
    }
  }
  *ok = true;
  return ST_OK;
}

// Q1 (len x k): an orthonormal basis of range(P) (P a projector of rank k)
// from P times a seeded Gaussian block, orthonormalised by two Cholesky-QR
// passes; *ok = false if a factorisation breaks down (P Omega too ill
// conditioned for Cholesky-QR).
static int range_basis(const c128* P, long ldp, int len, int k, c128* Q1, DcWork& w, Arena& ws, hipStream_t s,
                       bool* ok) {
  *ok = false;
  hipLaunchKernelGGL(gauss_fill_kernel, dim3(nblk((long)len * k)), dim3(256), 0, s, w.tmp, (long)len, len, k,
                     0x2545F4914F6CDD1Dull * (uint64_t)len + (uint64_t)k);
  RSRR_LAUNCH_CHECK();
  RSRR_TRY(zg(OP_N, OP_N, len, k, len, ONE, P, ldp, w.tmp, len, ZERO, Q1, len, s));
  for (int pass = 0; pass < 2; ++pass) {
    bool good = false;
    RSRR_TRY(cholqr(Q1, len, len, k, ws, s, &good));
    if (!good) return ST_OK;
  }
  *ok = true;
  return ST_OK;
}

// Q = [Q1 Q2] (len x len, ld len): Q1 an orthonormal basis of range(P) (rank
// k, P len x len with leading dimension ldp), Q2 of its orthogonal complement.
// scratch: len x len, distinct from P and w.Q.
static int bases_from_projector(const c128* P, long ldp, int len, int k, c128* Q, c128* scratch, DcWork& w,
                                Arena& ws, hipStream_t s) {
  c128* Q1 = Q;
  c128* Q2 = Q + (long)k * len;
  bool ok = false;
  RSRR_TRY(range_basis(P, ldp, len, k, Q1, w, ws, s, &ok));
  if (!ok) RSRR_TRY(basis_of_columns(P, ldp, len, len, k, Q1, len, ws, s));
  RSRR_TRY(complement_basis(Q1, len, k, Q2, w, ws, s, &ok));
  if (ok) return ST_OK;
  // fallback: pivoted basis of range(I - Q1 Q1^H)
  RSRR_TRY(set_identity(scratch, len, len, s));
  RSRR_TRY(zg(OP_N, OP_C, len, len, k, MONE, Q1, len, Q1, len, ONE, scratch, len, s));
  RSRR_TRY(basis_of_columns(scratch, len, len, len, len - k, Q2, len, ws, s));
  // one more orthogonalisation of Q2 against Q1 (classical Gram-Schmidt, then Cholesky-QR)
  RSRR_TRY(zg(OP_C, OP_N, k, len - k, len, ONE, Q1, len, Q2, len, ZERO, w.tmp, k, s));
  RSRR_TRY(zg(OP_N, OP_N, len, len - k, k, MONE, Q1, len, w.tmp, k, ONE, Q2, len, s));
  RSRR_TRY((convert<double, double>(Q2, len, 0, scratch, len, 0, len, len - k, 1, s)));
  RSRR_TRY(basis_of_columns(scratch, len, len, len - k, len - k, Q2, len, ws, s));
  return ST_OK;
}

// Splits the diagonal block B = T[off.., off..] (len x len).  On success Q
// (len x len, ld len) holds [Q1 Q2] and *k the size of the leading block.
static int split_block(const c128* B, long ldb, int len, DcWork& w, Arena& ws, hipStream_t s, int* k_out,
                       int first_attempt = 0) {
  *k_out = 0;
  std::vector<c128> d;
  RSRR_TRY(host_diag(B, ldb, len, w, s, &d));
  double sr = 0, si = 0;
  for (int i = 0; i < len; ++i) { sr += d[i].re; si += d[i].im; }
  sr /= len;
  si /= len;
  const long ll = (long)len * len;
  int k = 0;
  for (int attempt = first_attempt; attempt < 4 && (k <= 0 || k >= len); ++attempt) {
    // attempts: vertical line through the mean, horizontal line, then nudged lines
    const bool vert = (attempt % 2 == 0);
    const double nudge = (attempt >= 2) ? 1e-3 * (1 + sqrt(sr * sr + si * si)) : 0.0;
    const c128 shift = vert ? mk<double>(sr + nudge, 0) : mk<double>(0, si + nudge);
    const c128 rot = vert ? mk<double>(1, 0) : mk<double>(0, -1);
    hipLaunchKernelGGL(shift_copy_kernel, dim3(nblk(ll)), dim3(256), 0, s, B, ldb, w.X, len, len, shift, rot);
    RSRR_LAUNCH_CHECK();
    int its = 0;
    const int st = newton_sign(len, w, ws, s, &its);
    if (st < 0) { vlog("dc split len=%d attempt %d: no convergence (%d its)", len, attempt, its); continue; }
    hipLaunchKernelGGL(projector_kernel, dim3(nblk(ll)), dim3(256), 0, s, w.X, len, len, w.diag);
    RSRR_LAUNCH_CHECK();
    std::vector<c128> pd(len);
    RSRR_HIP(hipMemcpyAsync(pd.data(), w.diag, len * sizeof(c128), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    double tr = 0;
    for (int i = 0; i < len; ++i) tr += pd[i].re;
    k = (int)std::lround(tr);
    vlog("dc split len=%d attempt %d: %d newton its, k=%d (trace %.6f)", len, attempt, its, k, tr);
  }
  if (k <= 0 || k >= len) return ST_OK;
  RSRR_TRY(bases_from_projector(w.X, len, len, k, w.Q, w.Y, w, ws, s));
  *k_out = k;
  return ST_OK;
}

// T <- diag(I, Q, I)^H T diag(I, Q, I) on block [off, off+len); Z <- Z diag(I, Q, I).
static int apply_block(c128* T, long ldt, int m, c128* Z, long ldz, int off, int len, const c128* Q,
                       long ldq, DcWork& w, hipStream_t s, bool diag_too) {
  const int right = m - off - len;
  if (right > 0) {          // rows of the block, columns right of it
    c128* R = T + off + (long)(off + len) * ldt;
    RSRR_TRY(zg(OP_C, OP_N, len, right, len, ONE, Q, ldq, R, ldt, ZERO, w.tmp, len, s));
    RSRR_TRY((convert<double, double>(w.tmp, len, 0, R, ldt, 0, len, right, 1, s)));
  }
  if (off > 0) {            // columns of the block, rows above it
    c128* Ab = T + (long)off * ldt;
    RSRR_TRY(zg(OP_N, OP_N, off, len, len, ONE, Ab, ldt, Q, ldq, ZERO, w.tmp, off, s));
    RSRR_TRY((convert<double, double>(w.tmp, off, 0, Ab, ldt, 0, off, len, 1, s)));
  }
  if (diag_too) {
    c128* D = T + off + (long)off * ldt;
    RSRR_TRY(zg(OP_N, OP_N, len, len, len, ONE, D, ldt, Q, ldq, ZERO, w.tmp, len, s));
    RSRR_TRY(zg(OP_C, OP_N, len, len, len, ONE, Q, ldq, w.tmp, len, ZERO, w.tmp2, len, s));
    RSRR_TRY((convert<double, double>(w.tmp2, len, 0, D, ldt, 0, len, len, 1, s)));
  }
  c128* Zb = Z + (long)off * ldz;
  RSRR_TRY(zg(OP_N, OP_N, m, len, len, ONE, Zb, ldz, Q, ldq, ZERO, w.tmp, m, s));
  RSRR_TRY((convert<double, double>(w.tmp, m, 0, Zb, ldz, 0, m, len, 1, s)));
  return ST_OK;
}

int eig_dc(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
           hipStream_t s, double refine_above) {
  const long mm = (long)m * m;
  DcWork w;
  c128* Z = nullptr;
  RSRR_TRY(ws.get<c128>("dc_Z", mm, &Z));
  RSRR_TRY(ws.get<c128>("dc_X", mm, &w.X));
  RSRR_TRY(ws.get<c128>("dc_Y", mm, &w.Y));
  RSRR_TRY(ws.get<c128>("dc_LU", mm, &w.LU));
  RSRR_TRY(ws.get<c128>("dc_dinv", LUWork<double>::dinv_elems(m, 64, 1), &w.dinv));
  RSRR_TRY(ws.get<c128>("dc_Q", mm, &w.Q));
  RSRR_TRY(ws.get<c128>("dc_tmp", mm, &w.tmp));
  RSRR_TRY(ws.get<c128>("dc_tmp2", mm, &w.tmp2));
  RSRR_TRY(ws.get<c128>("dc_diag", m, &w.diag));
  RSRR_TRY(ws.get<int>("dc_ipiv", m, &w.ipiv));
  RSRR_TRY(ws.get<int>("dc_info", 1, &w.info));
  RSRR_TRY(ws.get<double>("dc_part", 2 * (size_t)(m / FCOLS + 2), &w.part));
  c128 *A0 = nullptr, *Dc = nullptr, *mu = nullptr;
  RSRR_TRY(ws.get<c128>("dc_A0", mm, &A0));
  RSRR_TRY(ws.get<c128>("dc_D", mm, &Dc));
  RSRR_TRY(ws.get<c128>("dc_mu", m, &mu));
  RSRR_TRY((convert<double, double>(A, lda, 0, A0, m, 0, m, m, 1, s)));
  RSRR_TRY(set_identity(Z, m, m, s));
  struct Blk { int off, len; };
  std::vector<Blk> level{{0, m}}, leaves;
  const double t_dc = now_s();
  double dropped = 0;         // largest ||B21|| / ||B|| over the splits
  // block b of T split into k + (len - k) with the bases in w.Q
  auto finish_split = [&](const Blk& b, int k, std::vector<Blk>& next) -> int {
    c128* B = A + b.off + (long)b.off * lda;
    RSRR_TRY(apply_block(A, lda, m, Z, m, b.off, b.len, w.Q, b.len, w, s, true));
    double f_all = 0, f_low = 0;
    RSRR_TRY(fro_sums(B, nullptr, lda, b.len, w, s, &f_all, nullptr));
    {   // norm of the block below the split (should be at rounding level), then zero it
      std::vector<double> h;
      const int rows = b.len - k;
      c128* Lo = B + k;
      RSRR_TRY((convert<double, double>(Lo, lda, 0, w.tmp, rows, 0, rows, k, 1, s)));
      double part = 0;
      const int nb = (k + FCOLS - 1) / FCOLS;
      hipLaunchKernelGGL(fro_partial_kernel, dim3(nb), dim3(256), 0, s, w.tmp, (const c128*)nullptr, (long)rows, rows, k, w.part);
      RSRR_LAUNCH_CHECK();
      h.resize(2 * nb);
      RSRR_HIP(hipMemcpyAsync(h.data(), w.part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      RSRR_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < nb; ++i) part += h[2 * i];
      f_low = part;
      hipLaunchKernelGGL(zero_block_kernel, dim3(nblk((long)rows * k)), dim3(256), 0, s, Lo, lda, rows, k);
      RSRR_LAUNCH_CHECK();
    }
    const double ratio = sqrt(f_low / std::max(f_all, 1e-300));
    dropped = std::max(dropped, ratio);
    vlog("dc block off=%d len=%d -> %d + %d, ||B21||/||B|| = %.2e", b.off, b.len, k, b.len - k, ratio);
    next.push_back({b.off, k});
    next.push_back({b.off + k, b.len - k});
    return ST_OK;
  };
  // the split tree level by level; the blocks of a level (largest first, as
  // many as fit the m x m work buffers) share one batched sign iteration
  while (!level.empty()) {
    std::vector<Blk> big, next;
    for (const Blk& b : level) (b.len <= DC_LEAF ? leaves : big).push_back(b);
    std::sort(big.begin(), big.end(), [](const Blk& x, const Blk& y) { return x.len > y.len; });
    for (size_t g0 = 0; g0 < big.size();) {
      const int L = big[g0].len;
      const long ll = (long)L * L;
      const size_t cnt = std::min(std::max<size_t>(1, (size_t)(mm / ll)), big.size() - g0);
      DcBatch bt;
      bt.nbk = (int)cnt;
      bt.Lmax = L;
      bt.X = w.X; bt.Y = w.Y; bt.LU = w.LU;
      const int nch = (L + FCOLS - 1) / FCOLS;
      RSRR_TRY(ws.get<int>("dcb_lens", cnt, &bt.lens_dev));
      RSRR_TRY(ws.get<c128>("dcb_dinv", LUWork<double>::dinv_elems(L, 32, (int)cnt), &bt.dinv));
      RSRR_TRY(ws.get<int>("dcb_ipiv", cnt * (size_t)L, &bt.ipiv));
      RSRR_TRY(ws.get<int>("dcb_info", cnt, &bt.info));
      RSRR_TRY(ws.get<double>("dcb_part", 2 * cnt * (size_t)nch, &bt.part));
      RSRR_TRY(ws.get<double>("dcb_coef", 2 * cnt, &bt.coef));
      RSRR_TRY(ws.get<c128>("dcb_diag", cnt * (size_t)L, &bt.diag));
      for (size_t i = 0; i < cnt; ++i) {
        const Blk& b = big[g0 + i];
        bt.lens.push_back(b.len);
        // vertical line through the mean of the block's diagonal
        std::vector<c128> d;
        const c128* B = A + b.off + (long)b.off * lda;
        RSRR_TRY(host_diag(B, lda, b.len, w, s, &d));
        double sr = 0;
        for (int q = 0; q < b.len; ++q) sr += d[q].re;
        sr /= b.len;
        hipLaunchKernelGGL(shift_copy_kernel, dim3(nblk((long)b.len * b.len)), dim3(256), 0, s, B, lda,
                           bt.X + (long)i * ll, (long)L, b.len, mk<double>(sr, 0), mk<double>(1, 0));
        RSRR_LAUNCH_CHECK();
      }
      RSRR_HIP(hipMemcpyAsync(bt.lens_dev, bt.lens.data(), cnt * sizeof(int), hipMemcpyHostToDevice, s));
      RSRR_TRY(pad_identity(bt.X, bt, s));
      std::vector<int> ok;
      int its = 0;
      RSRR_TRY(newton_sign_batched(bt, ws, s, &ok, &its));
      std::vector<int> ks(cnt, 0);
      for (size_t i = 0; i < cnt; ++i)
        if (ok[i]) {
          hipLaunchKernelGGL(projector_kernel, dim3(nblk((long)bt.lens[i] * bt.lens[i])), dim3(256), 0, s,
                             bt.X + (long)i * ll, (long)L, bt.lens[i], bt.diag + (long)i * L);
          RSRR_LAUNCH_CHECK();
        }
      std::vector<c128> pd(cnt * (size_t)L);
      RSRR_HIP(hipMemcpyAsync(pd.data(), bt.diag, pd.size() * sizeof(c128), hipMemcpyDeviceToHost, s));
      RSRR_HIP(hipStreamSynchronize(s));
      for (size_t i = 0; i < cnt; ++i) {
        if (!ok[i]) continue;
        double tr = 0;
        for (int q = 0; q < bt.lens[i]; ++q) tr += pd[i * (size_t)L + q].re;
        ks[i] = (int)std::lround(tr);
      }
      vlog("dc level batch: %d blocks up to %d, %d iterations, sign done at %.3fs", (int)cnt, L, its, now_s() - t_dc);
      // successful splits first: their projectors live in bt.X
      for (size_t i = 0; i < cnt; ++i) {
        const Blk& b = big[g0 + i];
        if (ks[i] <= 0 || ks[i] >= b.len) continue;
        RSRR_TRY(bases_from_projector(bt.X + (long)i * ll, L, b.len, ks[i], w.Q, w.LU, w, ws, s));
        RSRR_TRY(finish_split(b, ks[i], next));
      }
      // the others: one block at a time, from the horizontal line on
      for (size_t i = 0; i < cnt; ++i) {
        const Blk& b = big[g0 + i];
        if (ks[i] > 0 && ks[i] < b.len) continue;
        int k = 0;
        RSRR_TRY(split_block(A + b.off + (long)b.off * lda, lda, b.len, w, ws, s, &k, 1));
        if (k <= 0 || k >= b.len) {
          if (b.len > 512) return set_error(ST_ENOTCONV, "divide and conquer: no split of a %d block", b.len);
          leaves.push_back(b);
          continue;
        }
        RSRR_TRY(finish_split(b, k, next));
      }
      g0 += cnt;
      RSRR_HIP(hipStreamSynchronize(s));
      vlog("dc level batch done at %.3fs", now_s() - t_dc);
    }
    level.swap(next);
  }
  // ---- leaves: Schur forms of the diagonal blocks, all at once
  const int nl = (int)leaves.size();
  std::vector<c128*> hH(nl), hZ(nl);
  std::vector<int> hlen(nl);
  size_t total = 0;
  for (auto& b : leaves) total += (size_t)b.len * b.len;
  c128 *Lbuf = nullptr, *Zbuf = nullptr;
  c128** pdev = nullptr;
  int* idev = nullptr;
  RSRR_TRY(ws.get<c128>("dc_leafH", total, &Lbuf));
  RSRR_TRY(ws.get<c128>("dc_leafZ", total, &Zbuf));
  RSRR_TRY(ws.get<c128*>("dc_leafP", 2 * (size_t)nl, &pdev));
  RSRR_TRY(ws.get<int>("dc_leafI", 2 * (size_t)nl, &idev));
  size_t o = 0;
  for (int i = 0; i < nl; ++i) {
    hH[i] = Lbuf + o;
    hZ[i] = Zbuf + o;
    hlen[i] = leaves[i].len;
    RSRR_TRY((convert<double, double>(A + leaves[i].off + (long)leaves[i].off * lda, lda, 0, hH[i],
                                      leaves[i].len, 0, leaves[i].len, leaves[i].len, 1, s)));
    o += (size_t)leaves[i].len * leaves[i].len;
  }
  RSRR_HIP(hipMemcpyAsync(pdev, hH.data(), nl * sizeof(c128*), hipMemcpyHostToDevice, s));
  RSRR_HIP(hipMemcpyAsync(pdev + nl, hZ.data(), nl * sizeof(c128*), hipMemcpyHostToDevice, s));
  RSRR_HIP(hipMemcpyAsync(idev, hlen.data(), nl * sizeof(int), hipMemcpyHostToDevice, s));
  int maxlen = 0;
  for (int i = 0; i < nl; ++i) maxlen = std::max(maxlen, hlen[i]);
  RSRR_TRY(leaf_schur_batched(pdev, pdev + nl, idev, nl, idev + nl, s, maxlen));
  std::vector<int> st(nl);
  RSRR_HIP(hipMemcpyAsync(st.data(), idev + nl, nl * sizeof(int), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < nl; ++i)
    if (st[i] < 0) return set_error(ST_ENOTCONV, "leaf QR did not converge (len %d)", hlen[i]);
  for (int i = 0; i < nl; ++i) {
    const Blk& b = leaves[i];
    RSRR_TRY(apply_block(A, lda, m, Z, m, b.off, b.len, hZ[i], b.len, w, s, false));
    RSRR_TRY((convert<double, double>(hH[i], b.len, 0, A + b.off + (long)b.off * lda, lda, 0, b.len,
                                      b.len, 1, s)));
  }
  vlog("dc: %d leaves, at %.3fs", nl, now_s() - t_dc);
  // ---- eigenvalues and eigenvectors of the Schur form
  c128* X = nullptr;
  RSRR_TRY(ws.get<c128>("dc_Xv", mm, &X));
  RSRR_TRY(tri_eigvecs(A, lda, m, X, m, s));
  // the splits leave T' = Z^H A0 Z = T + E with E at the level of the sign
  // function's error (well above rounding for eigenvalues near a split
  // line); the residual of an eigenpair of T is about ||E|| ||x||, so when a
  // dropped block exceeds refine_above the eigenvectors and eigenvalues are
  // corrected to first order in E
  std::vector<c128> d, dmu(m, mk<double>(0, 0));
  const bool refine = dropped > refine_above;
  vlog("dc: largest dropped block %.2e, eigenpair correction %s", dropped, refine ? "on" : "off");
  if (refine) {
    RSRR_TRY(zg(OP_N, OP_N, m, m, m, ONE, A0, m, Z, m, ZERO, w.tmp, m, s));
    RSRR_TRY(zg(OP_C, OP_N, m, m, m, ONE, Z, m, w.tmp, m, ZERO, w.tmp2, m, s));
    RSRR_TRY(zg(OP_N, OP_N, m, m, m, ONE, w.tmp2, m, X, m, ZERO, w.tmp, m, s));
    RSRR_TRY(tri_eigvecs_correct(A, lda, m, w.tmp, m, X, m, Dc, mu, s));
    RSRR_HIP(hipMemcpyAsync(dmu.data(), mu, m * sizeof(c128), hipMemcpyDeviceToHost, s));
  }
  RSRR_TRY(zg(OP_N, OP_N, m, m, m, ONE, Z, m, X, m, ZERO, V, ldv, s));
  RSRR_TRY(host_diag(A, lda, m, w, s, &d));
  RSRR_HIP(hipStreamSynchronize(s));
  lam->resize(m);
  for (int j = 0; j < m; ++j) (*lam)[j] = cd(d[j].re + dmu[j].re, d[j].im + dmu[j].im);
  return ST_OK;
}

}  // namespace rsrr
