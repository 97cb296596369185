// C ABI of the RSRR library: handles, parameters, errors and dispatch.
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>

#include "driver.h"

namespace rsrr {

static thread_local char g_err[1024] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void vlog(const char* fmt, ...) {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("RSRR_VERBOSE");
    on = (e && e[0] == '1') ? 1 : 0;
  }
  if (!on) return;
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "[rsrr] ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  fflush(stderr);
  va_end(ap);
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int Arena::get(const char* name, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  auto it = bufs.find(name);
  if (it != bufs.end() && it->second.second >= bytes) {
    *out = it->second.first;
    return ST_OK;
  }
  if (it != bufs.end()) {
    (void)hipFree(it->second.first);
    bufs.erase(it);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(ST_ENOMEM, "device allocation of %zu bytes for '%s' failed", bytes, name);
  }
  bufs[name] = std::make_pair(p, bytes);
  *out = p;
  return ST_OK;
}

int Arena::aux_stream(hipStream_t* s, hipEvent_t* ev_main, hipEvent_t* ev_aux) {
  if (no_aux) {
    *s = nullptr;
    *ev_main = *ev_aux = nullptr;
    return ST_OK;
  }
  if (!aux) {
    if (hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) {
      aux = nullptr;
      return set_error(ST_EHIP, "cannot create the look-ahead stream");
    }
    for (auto& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        e = nullptr;
        return set_error(ST_EHIP, "cannot create the look-ahead events");
      }
  }
  *s = aux;
  *ev_main = ev[0];
  *ev_aux = ev[1];
  return ST_OK;
}

void Arena::release() {
  if (aux) (void)hipStreamSynchronize(aux);
  for (auto& kv : bufs) (void)hipFree(kv.second.first);
  bufs.clear();
  for (auto& e : ev)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
  if (aux) { (void)hipStreamDestroy(aux); aux = nullptr; }
}

void eval_fn(const rsrr_fn& f, cd z, cd* val, cd* der) {
  const cd c(f.c.re, f.c.im), t(f.t.re, f.t.im);
  const int p = f.p;
  // integer powers by repeated multiplication (exact for small p, no log/exp)
  cd zpm1(1, 0);
  for (int q = 1; q < p; ++q) zpm1 *= z;
  const cd zp = (p == 0) ? cd(1, 0) : zpm1 * z;
  const cd dzp = (p == 0) ? cd(0, 0) : (double)p * zpm1;
  switch (f.kind) {
    case RSRR_F_EXP: {
      const cd e = std::exp(t * z);
      *val = c * zp * e;
      if (der) *der = c * e * (dzp + t * zp);
      break;
    }
    case RSRR_F_RAT: {
      const cd d = z - t;
      *val = c * zp / d;
      if (der) *der = c * (dzp * d - zp) / (d * d);
      break;
    }
    default:
      *val = c * zp;
      if (der) *der = c * dzp;
  }
}

int eval_scalars(const rsrr_problem* p, const cd* z, size_t m, cd* f, cd* df) {
  const int J = p->J;
  if (!p->cb) {
    for (size_t q = 0; q < m; ++q)
      for (int k = 0; k < J; ++k) eval_fn(p->fns[k], z[q], f + q * J + k, df ? df + q * J + k : nullptr);
    return ST_OK;
  }
  // std::complex<double> has the layout of rsrr_complex (two doubles)
  static_assert(sizeof(cd) == sizeof(rsrr_complex), "complex layout");
  int r = p->cb(p->cb_ctx, (const rsrr_complex*)z, m, (rsrr_complex*)f, (rsrr_complex*)df);
  if (r == 1 && df) {
    r = p->cb(p->cb_ctx, (const rsrr_complex*)z, m, (rsrr_complex*)f, nullptr);
    if (r == 0) return 1;
  }
  if (r != 0) return set_error(ST_EINVAL, "scalar-function callback returned %d", r);
  return ST_OK;
}

void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  // roots of P_n by Newton's method from Tricomi's initial guesses; P_n and
  // P_{n-1} by the three-term recurrence k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2};
  // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1); w = 2 / ((1 - x^2) P_n'(x)^2)
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  // P_n(t) and P_n'(t)
  auto legendre = [n](double t, double* pn, double* dpn) {
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    *pn = p1;
    *dpn = n * (t * p1 - p0) / (t * t - 1.0);
  };
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5)), pn, dp;
    for (int it = 0; it < 50; ++it) {           // quadratic convergence: a few steps
      legendre(t, &pn, &dp);
      const double dt = pn / dp;
      t -= dt;
      if (fabs(dt) < 1e-15) break;
    }
    legendre(t, &pn, &dp);
    t -= pn / dp;                                // one more step at full accuracy
    legendre(t, &pn, &dp);
    const double wi = 2.0 / ((1.0 - t * t) * dp * dp);
    // t is the i-th largest root; store ascending with exact symmetry
    (*x)[n - 1 - i] = t;
    (*x)[i] = -t;
    (*w)[n - 1 - i] = wi;
    (*w)[i] = wi;
  }
  if (n % 2 == 1) (*x)[n / 2] = 0.0;
}

bool rect_split(const rsrr_contour* c, int N, bool sampling, int* nh, int* nv) {
  if (sampling && (c->n_h > 0 || c->n_v > 0)) {
    *nh = c->n_h;
    *nv = c->n_v;
    return c->n_h > 0 && c->n_v > 0 && N == 2 * (c->n_h + c->n_v);
  }
  if (N < 4 || N % 2) return false;
  const int half = N / 2;
  int h = (int)std::lround(half * c->a / (c->a + c->b));
  h = std::min(std::max(h, 1), half - 1);
  *nh = h;
  *nv = half - h;
  return true;
}

void contour_nodes(const rsrr_contour* c, int N, bool sampling, std::vector<cd>* z, std::vector<cd>* dz) {
  z->resize(N);
  if (dz) dz->resize(N);
  const cd g(c->center.re, c->center.im);
  if (c->kind == RSRR_CONTOUR_RECT) {
    int nh = 0, nv = 0;
    if (!rect_split(c, N, sampling, &nh, &nv)) return;   // rejected by the parameter check
    const double a = c->a, b = c->b;
    // side j: z = p0 + h x, x in [-1, 1], dz = h dx; counter-clockwise
    const cd p0[4] = {g + cd(0, -b), g + cd(a, 0), g + cd(0, b), g + cd(-a, 0)};
    const cd hv[4] = {cd(a, 0), cd(0, b), cd(-a, 0), cd(0, -b)};
    const int cnt[4] = {nh, nv, nh, nv};
    std::vector<double> x, w;
    int j = 0;
    for (int side = 0; side < 4; ++side) {
      gauss_legendre(cnt[side], &x, &w);
      for (int k = 0; k < cnt[side]; ++k, ++j) {
        (*z)[j] = p0[side] + hv[side] * x[k];
        if (dz) (*dz)[j] = hv[side] * w[k];
      }
    }
    return;
  }
  for (int j = 0; j < N; ++j) {
    const double th = 2.0 * M_PI * (j + 0.5) / N;
    (*z)[j] = g + cd(c->a * cos(th), c->b * sin(th));
    if (dz) (*dz)[j] = (2.0 * M_PI / N) * cd(-c->a * sin(th), c->b * cos(th));
  }
}

bool bem_circle_interp(const rsrr_contour* c, const rsrr_params* prm, double* R) {
  *R = c->kind == RSRR_CONTOUR_RECT ? std::hypot(c->a, c->b) : std::max(c->a, c->b);
  if (prm->interp == RSRR_INTERP_CHEB) return false;
  if (prm->interp == RSRR_INTERP_CIRCLE) return true;
  return c->b > 0.25 * c->a;
}

bool contour_inside(const rsrr_contour* c, cd lam) {
  const double xr = (lam.real() - c->center.re) / c->a, xi = (lam.imag() - c->center.im) / c->b;
  if (c->kind == RSRR_CONTOUR_RECT) return fabs(xr) < 1.0 && fabs(xi) < 1.0;
  return xr * xr + xi * xi < 1.0;
}

int check_params(const rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm) {
  if (!p || !c || !prm) return set_error(ST_EINVAL, "null argument");
  if (prm->N < 1 || prm->L < 1) return set_error(ST_EINVAL, "N and L must be >= 1");
  if (!(c->a > 0) || !(c->b > 0)) return set_error(ST_EINVAL, "contour semi-axes must be > 0");
  if (c->kind != RSRR_CONTOUR_ELLIPSE && c->kind != RSRR_CONTOUR_RECT)
    return set_error(ST_EINVAL, "unknown contour kind %d", c->kind);
  if (c->kind == RSRR_CONTOUR_RECT) {
    int nh, nv;
    if (!rect_split(c, prm->N, true, &nh, &nv))
      return set_error(ST_EINVAL, "rectangle: N=%d does not match n_h=%d, n_v=%d (N = 2(n_h+n_v), or "
                       "n_h = n_v = 0 and N even >= 4)", prm->N, c->n_h, c->n_v);
    if (!rect_split(c, prm->NS, false, &nh, &nv))
      return set_error(ST_EINVAL, "rectangle: NS=%d must be even and >= 4", prm->NS);
  }
  if (prm->nb < 0 || prm->nb > 64) return set_error(ST_EINVAL, "nb must be in [0, 64] (0: tuned)");
  if (prm->nb_reduced < 0 || prm->nb_reduced > 64)
    return set_error(ST_EINVAL, "nb_reduced must be in [0, 64] (0: 64)");
  if (prm->precision != RSRR_PREC_C128 && prm->precision != RSRR_PREC_C64_IR)
    return set_error(ST_EINVAL, "unknown precision %d", prm->precision);
  if (prm->precision == RSRR_PREC_C128 && p->n > LU_MAX_N_C128)
    return set_error(ST_EINVAL, "n=%d: complex128 factorisations go up to order %d (use c64_ir)", p->n,
                     LU_MAX_N_C128);
  if (prm->NS < 2 || prm->K < 1) return set_error(ST_EINVAL, "NS >= 2 and K >= 1 required");
  if ((long)prm->N * prm->L > (1L << 20)) return set_error(ST_EINVAL, "N*L too large");
  if (prm->scheme != RSRR_SCHEME_SAMPLING && prm->scheme != RSRR_SCHEME_MOMENT)
    return set_error(ST_EINVAL, "unknown scheme %d", prm->scheme);
  if (!(prm->chunk_gib >= 0.0625) || prm->chunk_gib > 256.0)
    return set_error(ST_EINVAL, "chunk_gib=%g outside [1/16, 256]", prm->chunk_gib);
  if (prm->graph != 0 && prm->graph != 1) return set_error(ST_EINVAL, "graph must be 0 or 1");
  if (prm->interp < RSRR_INTERP_AUTO || prm->interp > RSRR_INTERP_CIRCLE)
    return set_error(ST_EINVAL, "unknown interpolation %d", prm->interp);
  if (prm->Kp < 0 || (long)prm->Kp * prm->L > (1L << 20))
    return set_error(ST_EINVAL, "Kp=%d outside [0, 2^20/L]", prm->Kp);
  return ST_OK;
}

rsrr_params resolve_params(const rsrr_problem* p, const rsrr_params* prm) {
  rsrr_params q = *prm;
  if (q.nb == 0) q.nb = tuned_nb(q.precision, p->n, q.N);
  return q;
}

}  // namespace rsrr

using namespace rsrr;

extern "C" {

const char* rsrr_last_error(void) { return rsrr::g_err; }

void rsrr_default_params(rsrr_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->N = 32;
  p->L = 16;
  p->NS = 512;
  p->K = 2;
  p->delta = 1e-14;
  p->tol_gap = 1e3;
  p->tol_res = 1e-10;
  p->hankel_tol = 1e-13;
  p->precision = RSRR_PREC_C64_IR;
  p->ir_max_iter = 5;
  p->ir_tol = 1e-14;
  p->cheb_degree = 40;
  p->nb = 64;
  p->seed = 1;
  p->chunk_gib = 24.0;
}

// Coefficient-form problem: validates and uploads the A_k and forms their
// Gram matrix; the scalar functions are set by the caller.
static int create_coeff(rsrr_problem** out, int n, int J, const int* kinds, const void* const* A,
                        void* stream) {
  if (!out || !kinds || !A) return set_error(ST_EINVAL, "rsrr_create: null argument");
  *out = nullptr;
  if (n < 1 || n > LU_MAX_N_C64)
    return set_error(ST_EINVAL, "rsrr_create: n=%d outside [1, %d]", n, LU_MAX_N_C64);
  if (J < 1 || J > 16) return set_error(ST_EINVAL, "rsrr_create: J=%d outside [1, 16]", J);
  for (int k = 0; k < J; ++k) {
    if (kinds[k] < 0 || kinds[k] > 3) return set_error(ST_EINVAL, "rsrr_create: kind[%d]=%d", k, kinds[k]);
    if (kinds[k] != RSRR_MAT_IDENTITY && !A[k]) return set_error(ST_EINVAL, "rsrr_create: A[%d] is NULL", k);
  }
  rsrr_problem* p = new rsrr_problem();
  p->n = n;
  p->J = J;
  p->stream = (hipStream_t)stream;
  p->kinds.assign(kinds, kinds + J);
  p->mats.assign(J, nullptr);
  const size_t nn = (size_t)n * n;
  for (int k = 0; k < J; ++k) {
    size_t bytes = 0;
    if (kinds[k] == RSRR_MAT_DIAG) bytes = n * sizeof(c128);
    else if (kinds[k] == RSRR_MAT_REAL) bytes = nn * sizeof(double);
    else if (kinds[k] == RSRR_MAT_DENSE) bytes = nn * sizeof(c128);
    if (!bytes) continue;
    hipError_t e = hipMalloc(&p->mats[k], bytes);
    if (e == hipSuccess) e = hipMemcpy(p->mats[k], A[k], bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rsrr_destroy(p);
      return set_error(ST_ENOMEM, "rsrr_create: cannot upload coefficient %d (%zu bytes): %s", k, bytes,
                       hipGetErrorString(e));
    }
  }
  // Gram of the coefficients, gram[k,l] = sum_ij conj(A_k)_ij (A_l)_ij, so that
  // ||T(z)||_F^2 = sum_kl conj(f_k) f_l gram[k,l] exactly.
  p->gram.assign(2 * J * J, 0.0);
  auto entry = [&](int k, size_t e, size_t i, size_t j) -> cd {
    switch (kinds[k]) {
      case RSRR_MAT_IDENTITY: return i == j ? cd(1, 0) : cd(0, 0);
      case RSRR_MAT_DIAG: { const rsrr_complex* d = (const rsrr_complex*)A[k];
                            return i == j ? cd(d[i].re, d[i].im) : cd(0, 0); }
      case RSRR_MAT_REAL: return cd(((const double*)A[k])[e], 0);
      default: { const rsrr_complex* d = (const rsrr_complex*)A[k]; return cd(d[e].re, d[e].im); }
    }
  };
  for (int k = 0; k < J; ++k)
    for (int l = 0; l < J; ++l) {
      cd s(0, 0);
      const bool dk = kinds[k] >= RSRR_MAT_REAL, dl = kinds[l] >= RSRR_MAT_REAL;
      if (dk && dl) {
        for (size_t e = 0; e < nn; ++e) s += std::conj(entry(k, e, e % n, e / n)) * entry(l, e, e % n, e / n);
      } else {
        for (size_t i = 0; i < (size_t)n; ++i) {
          const size_t e = i + i * n;
          s += std::conj(entry(k, e, i, i)) * entry(l, e, i, i);
        }
      }
      p->gram[2 * (k * J + l)] = s.real();
      p->gram[2 * (k * J + l) + 1] = s.imag();
    }
  *out = p;
  return ST_OK;
}

int rsrr_create(rsrr_problem** out, int n, int J, const int* kinds, const void* const* A,
                const rsrr_fn* f, void* stream) {
  if (!out || !f) return set_error(ST_EINVAL, "rsrr_create: null argument");
  *out = nullptr;
  for (int k = 0; k < J && k < 16; ++k)
    if (f[k].kind < 0 || f[k].kind > 2 || f[k].p < 0)
      return set_error(ST_EINVAL, "rsrr_create: bad scalar function %d", k);
  RSRR_TRY(create_coeff(out, n, J, kinds, A, stream));
  (*out)->fns.assign(f, f + J);
  return ST_OK;
}

int rsrr_create_fn(rsrr_problem** out, int n, int J, const int* kinds, const void* const* A,
                   rsrr_scalar_fn f, void* f_ctx, void* stream) {
  if (!out || !f) return set_error(ST_EINVAL, "rsrr_create_fn: null argument");
  *out = nullptr;
  RSRR_TRY(create_coeff(out, n, J, kinds, A, stream));
  (*out)->cb = f;
  (*out)->cb_ctx = f_ctx;
  return ST_OK;
}

int rsrr_create_bem(rsrr_problem** out, int n, const double* xyz, double h, void* stream) {
  if (!out || !xyz) return set_error(ST_EINVAL, "rsrr_create_bem: null argument");
  *out = nullptr;
  if (n < 2 || n > LU_MAX_N_C64)
    return set_error(ST_EINVAL, "rsrr_create_bem: n=%d outside [2, %d]", n, LU_MAX_N_C64);
  if (!(h > 0)) return set_error(ST_EINVAL, "rsrr_create_bem: h must be positive");
  rsrr_problem* p = new rsrr_problem();
  p->n = n;
  p->bem = true;
  p->h = h;
  p->stream = (hipStream_t)stream;
  hipError_t e = hipMalloc(&p->xyz, (size_t)n * 3 * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(p->xyz, xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    rsrr_destroy(p);
    return set_error(ST_ENOMEM, "rsrr_create_bem: cannot upload points: %s", hipGetErrorString(e));
  }
  *out = p;
  return ST_OK;
}

void rsrr_destroy(rsrr_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (void* m : p->mats) if (m) (void)hipFree(m);
  if (p->xyz) (void)hipFree(p->xyz);
  p->ws.release();
  if (p->batch_view) {
    unbind_view(p->batch_view);
    delete p->batch_view;
  }
  delete p;
}


int rsrr_sample(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                const rsrr_complex* U, int ldu, rsrr_complex* S, int lds, rsrr_info* info) {
  RSRR_TRY(check_params(p, c, prm));
  if (!U || !S || ldu < p->n || lds < p->n) return set_error(ST_EINVAL, "rsrr_sample: bad buffers");
  const rsrr_params q = resolve_params(p, prm);
  return sample_impl(p, c, &q, (const c128*)U, ldu, (c128*)S, lds, info);
}

int rsrr_workspace_bound(const rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                         size_t* bytes) {
  if (!bytes) return set_error(ST_EINVAL, "rsrr_workspace_bound: null output");
  RSRR_TRY(check_params(p, c, prm));
  const rsrr_params q = resolve_params(p, prm);
  *bytes = solve_workspace_bound(p, &q);
  return ST_OK;
}

int rsrr_moment_matrix(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                       const rsrr_complex* S, int lds, rsrr_complex* M, int ldm) {
  RSRR_TRY(check_params(p, c, prm));
  if (!S || !M || lds < p->n || ldm < p->n) return set_error(ST_EINVAL, "rsrr_moment_matrix: bad buffers");
  return moment_impl(p, c, prm, (const c128*)S, lds, (c128*)M, ldm);
}

int rsrr_orthonormalize(int rows, int cols, const rsrr_complex* S, int lds, double delta,
                        rsrr_complex* Q, int ldq, int* k_S, void* stream) {
  if (!S || !Q || !k_S || rows < 1 || cols < 1 || lds < rows || ldq < rows || !(delta > 0))
    return set_error(ST_EINVAL, "rsrr_orthonormalize: bad arguments");
  Arena ws;
  int st = ortho_impl(rows, cols, (const c128*)S, lds, delta, (c128*)Q, ldq, k_S, ws,
                      (hipStream_t)stream, 3);
  (void)hipStreamSynchronize((hipStream_t)stream);
  return st;
}

int rsrr_project(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                 const rsrr_complex* Q, int ldq, int k_S, rsrr_complex* B, int* J_out) {
  RSRR_TRY(check_params(p, c, prm));
  if (!Q || !B || k_S < 1 || ldq < p->n || k_S > p->n) return set_error(ST_EINVAL, "rsrr_project: bad arguments");
  return project_impl(p, c, prm, (const c128*)Q, ldq, k_S, (c128*)B, J_out);
}

int rsrr_solve(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
               const rsrr_complex* U, rsrr_result** out) {
  if (!out) return set_error(ST_EINVAL, "rsrr_solve: null result pointer");
  *out = nullptr;
  RSRR_TRY(check_params(p, c, prm));
  rsrr_result* r = new rsrr_result();
  memset(&r->info, 0, sizeof(r->info));
  const rsrr_params q = resolve_params(p, prm);
  int st = solve_impl(p, c, &q, (const c128*)U, r);
  if (st < 0) {
    delete r;
    return st;
  }
  r->info.status = st;
  *out = r;
  return st;
}

int rsrr_solve_batched(int count, rsrr_problem* const* probs, const rsrr_contour* contours,
                       const rsrr_params* prms, const rsrr_complex* const* U, rsrr_result** out) {
  if (count < 1 || !probs || !contours || !prms || !out)
    return set_error(ST_EINVAL, "rsrr_solve_batched: bad arguments");
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  // one panel width for the whole batch: the tuned one for the largest order
  // and the total number of matrices when the parameters leave it open
  std::vector<rsrr_params> q(prms, prms + count);
  {
    int nmax = 0, tot = 0;
    for (int i = 0; i < count; ++i) {
      if (!probs[i]) return set_error(ST_EINVAL, "rsrr_solve_batched: null problem %d", i);
      nmax = std::max(nmax, probs[i]->n);
      tot += prms[i].N;
    }
    for (int i = 0; i < count; ++i)
      if (q[i].nb == 0) q[i].nb = tuned_nb(q[i].precision, nmax, tot);
  }
  prms = q.data();
  for (int i = 0; i < count; ++i) {
    RSRR_TRY(check_params(probs[i], &contours[i], &prms[i]));
    if (probs[i]->stream != probs[0]->stream)
      return set_error(ST_EINVAL, "rsrr_solve_batched: problems %d and 0 use different streams", i);
    if (prms[i].precision != prms[0].precision || prms[i].nb != prms[0].nb)
      return set_error(ST_EINVAL, "rsrr_solve_batched: problems must share the precision and nb");
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return set_error(ST_EINVAL, "rsrr_solve_batched: problem %d given twice", i);
  }
  std::vector<rsrr_result*> res(count, nullptr);
  std::vector<SamplePlan> sp(count);
  auto fail = [&](int st) {
    for (rsrr_result* r : res) delete r;
    return st;
  };
  for (int i = 0; i < count; ++i) {
    res[i] = new rsrr_result();
    memset(&res[i]->info, 0, sizeof(res[i]->info));
    const int st = solve_begin(probs[i], &contours[i], &prms[i], U ? (const c128*)U[i] : nullptr, res[i], &sp[i]);
    if (st < 0) return fail(st);
  }
  // the sampling LUs of all problems, each panel step one set of launches
  hipStream_t s = probs[0]->stream;
  int st = ST_OK;
  for (int i = 0; i < count; ++i) {
    st = sample_assemble(&sp[i], s);
    if (st < 0) return fail(st);
  }
  if (sp[0].c64) {
    std::vector<LUWork<float>> w;
    for (const SamplePlan& q : sp) w.push_back(q.w64);
    st = lu_factor_segments<float>(w, s, w[0].aux, w[0].ev_main, w[0].ev_aux);
  } else {
    std::vector<LUWork<double>> w;
    for (const SamplePlan& q : sp) w.push_back(q.w128);
    st = lu_factor_segments<double>(w, s, w[0].aux, w[0].ev_main, w[0].ev_aux);
  }
  if (st < 0) return fail(st);
  // the later stages problem by problem, in one workspace kept by the first
  // handle (the sampled matrices stay in each problem's own workspace)
  rsrr_problem* v = probs[0]->batch_view;
  if (!v) {
    v = probs[0]->batch_view = new rsrr_problem();
    v->ws.no_aux = probs[0]->ws.no_aux;
  }
  int warn = 0;
  for (int i = 0; i < count; ++i) {
    bind_view(v, probs[i], s);
    st = solve_end(v, &contours[i], &prms[i], res[i], &sp[i]);
    unbind_view(v);
    if (st < 0) return fail(st);
    res[i]->info.status = st;
    res[i]->info.ws_bytes += (double)probs[i]->ws.bytes();
    warn |= st;
  }
  for (int i = 0; i < count; ++i) out[i] = res[i];
  return warn;
}

int rsrr_result_info(const rsrr_result* r, rsrr_info* info) {
  if (!r || !info) return set_error(ST_EINVAL, "rsrr_result_info: null argument");
  *info = r->info;
  return ST_OK;
}

int rsrr_result_copy(const rsrr_result* r, rsrr_complex* lambda, rsrr_complex* V, double* resid,
                     double* resid_paper, double* hankel_sigma) {
  if (!r) return set_error(ST_EINVAL, "rsrr_result_copy: null result");
  if (lambda && !r->lambda.empty()) memcpy(lambda, r->lambda.data(), r->lambda.size() * sizeof(rsrr_complex));
  if (V && !r->V.empty()) memcpy(V, r->V.data(), r->V.size() * sizeof(rsrr_complex));
  if (resid && !r->resid.empty()) memcpy(resid, r->resid.data(), r->resid.size() * sizeof(double));
  if (resid_paper && !r->resid_paper.empty())
    memcpy(resid_paper, r->resid_paper.data(), r->resid_paper.size() * sizeof(double));
  if (hankel_sigma && !r->hankel_sigma.empty())
    memcpy(hankel_sigma, r->hankel_sigma.data(), r->hankel_sigma.size() * sizeof(double));
  return ST_OK;
}

void rsrr_result_free(rsrr_result* r) { delete r; }

}  // extern "C"
