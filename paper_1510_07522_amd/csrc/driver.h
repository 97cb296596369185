// Host-side driver structures shared by the C-ABI implementation files.
#pragma once
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/rsrr.h"
#include "common.h"
#include "kernels.h"

namespace rsrr {

typedef std::complex<double> cd;

// Named, grow-only device buffers owned by one handle.  Calls on a handle do
// not overlap, so a buffer is reused across calls without re-allocation.
struct Arena {
  std::map<std::string, std::pair<void*, size_t>> bufs;
  // second stream (default priority) and two events for the look-ahead of
  // the LU factorisations, created on first use
  hipStream_t aux = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // no look-ahead stream: aux_stream() hands out none, and the LU
  // factorisations run on the caller's stream alone
  bool no_aux = false;
  int get(const char* name, size_t bytes, void** out);
  template <typename T> int get(const char* name, size_t count, T** out) {
    return get(name, count * sizeof(T), (void**)out);
  }
  int aux_stream(hipStream_t* s, hipEvent_t* ev_main, hipEvent_t* ev_aux);
  size_t bytes() const;   // device memory held
  void release();
  ~Arena() { release(); }
};

// Evaluates f(z) and f'(z) of a scalar-function spec.
void eval_fn(const rsrr_fn& f, cd z, cd* val, cd* der);

}  // namespace rsrr

struct rsrr_problem {
  int n = 0, J = 0;
  bool bem = false;
  hipStream_t stream = nullptr;
  std::vector<int> kinds;
  std::vector<rsrr_fn> fns;           // menu entries (empty when cb is set)
  rsrr_scalar_fn cb = nullptr;        // caller's scalar functions (rsrr_create_fn)
  void* cb_ctx = nullptr;
  std::vector<void*> mats;            // device data per coefficient (nullptr for identity)
  std::vector<double> gram;           // J x J complex (re, im): gram[k,l] = sum conj(A_k) A_l
  double* xyz = nullptr;              // BEM points (device, n*3)
  double h = 0.0;
  rsrr::Arena ws;
};

struct rsrr_result {
  rsrr_info info;
  std::vector<rsrr_complex> lambda, V;
  std::vector<double> resid, resid_paper, hankel_sigma;
};

namespace rsrr {

// Stage implementations (driver_*.hip).
int sample_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                const c128* U, long ldu, c128* S, long lds, rsrr_info* info);
// Moment matrix M_hat of the SSRR moment scheme from S_hat (eq. eq-hatMS).
int moment_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* S, long lds,
                c128* M, long ldm);
// Orthonormal basis Q (rows x k_S) of the columns of S above delta * sigma_1:
// pivoted Cholesky of the Gram matrix and Cholesky-QR, then up to levels - 1
// deflation levels for the directions one Gram matrix cannot resolve.
int ortho_impl(int rows, int cols, const c128* S, long lds, double delta, c128* Q, long ldq,
               int* k_S, Arena& ws, hipStream_t s, int levels = 2);
// One Cholesky-QR pass, X <- X chol(X^H X)^{-H} in place (ok = false if the
// Cholesky factorisation breaks down).
int cholqr(c128* X, long ldx, int rows, int k, Arena& ws, hipStream_t s, bool* ok);
int basis_of_columns(const c128* X, long ldx, int rows, int cols, int rank, c128* Q, long ldq,
                     Arena& ws, hipStream_t s);
int project_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* Q,
                 long ldq, int kS, c128* B, int* J_out);
int solve_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* U,
               rsrr_result* res);
// Upper bound of the device workspace one solve of p with prm allocates.
size_t solve_workspace_bound(const rsrr_problem* p, const rsrr_params* prm);
int check_params(const rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm);
// f_k(z_q) into f[q*J + k] for the m nodes z, and f_k'(z_q) into df when df is
// not null: the problem's menu entries or the caller's callback.  Returns
// ST_OK, 1 when the callback has no derivatives (f is then filled), or an error.
int eval_scalars(const rsrr_problem* p, const cd* z, size_t m, cd* f, cd* df);
// Gauss-Legendre nodes x (ascending) and weights w of the n-point rule on [-1, 1].
void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w);
// Per-side node counts of a rectangular contour for N nodes in total: the
// contour's own (n_h, n_v) when `sampling` and they are set, else the split
// in proportion to the side lengths.  Returns false if N cannot be split.
bool rect_split(const rsrr_contour* c, int N, bool sampling, int* nh, int* nv);
// Quadrature of the contour integral with N nodes: integral of g(z) dz ~=
// sum_j dz[j] g(z[j]).  Sampling nodes when `sampling` (rectangles then use
// the contour's own per-side counts), moment nodes otherwise.
void contour_nodes(const rsrr_contour* c, int N, bool sampling, std::vector<cd>* z, std::vector<cd>* dz);
// Interpolation of a BEM matrix for the reduced problem: true for the circle
// basis ((z - center)/R)^j (radius in *R), false for the Chebyshev
// interpolant on [Re(center) - a, Re(center) + a].
bool bem_circle_interp(const rsrr_contour* c, const rsrr_params* prm, double* R);
// lambda strictly inside the contour.
bool contour_inside(const rsrr_contour* c, cd lam);
double now_s();
// Progress line on stderr when RSRR_VERBOSE=1 (stage boundaries of long solves).
void vlog(const char* fmt, ...);

}  // namespace rsrr
