// Host-side driver structures shared by the C-ABI implementation files.
#pragma once
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/rsrr.h"
#include "common.h"
#include "kernels.h"
#include "timers.h"

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

// The sampling launches (assembly and factorisation of all nodes) captured
// in a HIP graph, with the key of everything they depend on.
struct SampleGraph {
  std::vector<long long> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;     // capture stream (a capture needs a stream of its own)
  void reset();
  ~SampleGraph();
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
  rsrr::SampleGraph sgraph;           // captured sampling launches (rsrr_params.graph)
  // workspace of the stages after sampling when this handle is the first of
  // a batched solve (shared by the problems of the batch, created on use)
  rsrr_problem* batch_view = nullptr;
};

namespace rsrr {
// A problem that shares another's data (coefficients, BEM points, scalar
// functions) but has its own stream and workspace: a serving slot, or the
// later stages of a batched solve.  Never frees the shared data.
inline void bind_view(rsrr_problem* v, const rsrr_problem* p, hipStream_t s) {
  v->n = p->n;
  v->J = p->J;
  v->bem = p->bem;
  v->kinds = p->kinds;
  v->fns = p->fns;
  v->cb = p->cb;
  v->cb_ctx = p->cb_ctx;
  v->mats = p->mats;
  v->gram = p->gram;
  v->xyz = p->xyz;
  v->h = p->h;
  v->stream = s;
}
inline void unbind_view(rsrr_problem* v) {
  v->mats.clear();
  v->xyz = nullptr;
}
}  // namespace rsrr

struct rsrr_result {
  rsrr_info info;
  std::vector<rsrr_complex> lambda, V;
  std::vector<double> resid, resid_paper, hankel_sigma;
};

namespace rsrr {

// Stage implementations (driver_*.hip).
int sample_impl(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                const c128* U, long ldu, c128* S, long lds, rsrr_info* info);
// Alg. 2 Steps 1-2 split at the factorisation (sample_impl = begin, factor,
// end), so that the factorisations of several problems can be one set of
// launches: begin computes the nodes and coefficients and assembles T(z_j)
// into the handle's workspace; the factorisation descriptor is w128 or w64;
// end checks the pivots and runs the solves, the refinement and the
// complex128 fallback.
struct SamplePlan {
  rsrr_problem* p = nullptr;
  const rsrr_contour* c = nullptr;
  const rsrr_params* prm = nullptr;
  const c128* U = nullptr;
  long ldu = 0, lds = 0;
  c128* S = nullptr;
  rsrr_info* info = nullptr;
  double t0 = 0;
  std::vector<cd> z;
  std::vector<c128> f, zc;
  c128 *f_dev = nullptr, *z_dev = nullptr;
  int *ipiv = nullptr, *infod = nullptr;
  bool c64 = true;
  LUWork<double> w128;
  LUWork<float> w64;
};
int sample_begin(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* U, long ldu,
                 c128* S, long lds, rsrr_info* info, SamplePlan* sp);
int sample_factor(SamplePlan* sp);
// Assembly of the sampled matrices T(z_j) on stream s (part of sample_factor;
// the batched solve calls it for each problem before their joint factorisation).
int sample_assemble(SamplePlan* sp, hipStream_t s);
int sample_end(SamplePlan* sp);
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
// solve_impl split at the sampling factorisations (solve_impl = begin,
// sample_factor, end): begin draws or takes U and prepares the sampling;
// end finishes the sampling and runs Steps 3-5 and the residual filter.
int solve_begin(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, const c128* U,
                rsrr_result* res, SamplePlan* sp);
int solve_end(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm, rsrr_result* res,
              SamplePlan* sp);
// Upper bound of the device workspace one solve of p with prm allocates.
size_t solve_workspace_bound(const rsrr_problem* p, const rsrr_params* prm);
int check_params(const rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm);
// A copy of prm with the panel width resolved (nb = 0: the autotuned width
// for this precision, order and node count, tune.hip).
rsrr_params resolve_params(const rsrr_problem* p, const rsrr_params* prm);
int tuned_nb(int precision, int n, int batch);
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
