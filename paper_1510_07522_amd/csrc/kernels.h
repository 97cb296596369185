// Internal (C++) interfaces between the RSRR host driver and its kernels.
#pragma once
#include <vector>

#include "common.h"

namespace rsrr {

enum { OP_N = 0, OP_T = 1, OP_C = 2 };

// Strided batched complex GEMM descriptor (column-major operands).
template <typename R> struct GemmBatch {
  int opA = OP_N, opB = OP_N;
  int M = 0, N = 0, K = 0;
  cplx<R> alpha = {1, 0}, beta = {0, 0};
  const void* A = nullptr; long lda = 0, sA = 0;   // complex or (a_real) real R
  const cplx<R>* B = nullptr; long ldb = 0, sB = 0;
  cplx<R>* C = nullptr; long ldc = 0, sC = 0;
  int batch = 1;
  bool a_real = false;
  bool gauss3m = false;   // 3-multiplication complex product (normwise stable)
  const int* active = nullptr;   // optional: batch entries with active[b] == 0 are skipped
  // Gram matrix C = alpha A^H A (opA OP_C, opB OP_N, B == A, M == N, real
  // alpha, beta 0): only the tiles on and below the diagonal are formed; each
  // one below it also stores its conjugate transpose above
  bool herm = false;
  const char* tag = "gemm";   // kernel-timer class
};
template <typename R> int gemm_batched(const GemmBatch<R>& g, hipStream_t s);
// The triangular solves inside one group of panels p0 .. p1-1 of a batched LU
// (lu_solve): each panel's diagonal block by its inverse from dinv, then the
// group's rows below it (lower) or above it (upper) updated, panel after panel,
// for all nrhs right-hand sides of B in one launch.  Every 64x64 product is
// computed as gemm_batched computes it.
template <typename R> struct LUGroupSolve {
  const cplx<R>* A = nullptr; long lda = 0, sA = 0;      // the factors
  const cplx<R>* dinv = nullptr; long sD = 0;             // per panel: L then U block inverses
  cplx<R>* B = nullptr; long ldb = 0, sB = 0;
  int n = 0, nb = 0, nrhs = 0, batch = 0, p0 = 0, p1 = 0;
  bool lower = true, gauss3m = false;
  const int* active = nullptr;
  const char* tag = "solve";
};
template <typename R> int lu_group_solve(const LUGroupSolve<R>& q, hipStream_t s);
// Up to GSEG strided batches of different shapes in one launch (the LU
// updates of instances of different orders): a persistent grid of workgroups
// walks the 64x64 tiles of all segments in a fixed order, with no atomics,
// each workgroup ending after its last tile.  Both operands untransposed and
// complex; segment q is g[q] (M, N, K, pointers, leading dims, strides,
// batch); alpha, beta, gauss3m and the timer tag are those of g[0].  Every
// element is computed exactly as gemm_batched computes it.
constexpr int GSEG = 16;
template <typename R> struct GemmSegs {
  int count = 0;
  GemmBatch<R> g[GSEG];
};
template <typename R> int gemm_segments(const GemmSegs<R>& sg, hipStream_t s);
// C_b = alpha T(z_b) B_b + beta C_b (fp64, 4M on the matrix cores) with T(z_b)
// the BEM single-layer matrix (n = g.M = g.K points xyz, spacing h) generated
// tile by tile where the GEMM stages its A operand; g.A is ignored.
int bem_gemm(const GemmBatch<double>& g, const double* xyz, double h, const c128* z_dev, hipStream_t s);

// ---------------------------------------------------------------- batched LU
// Factors `batch` n x n matrices stored with leading dimension lda and batch
// stride sA (elements).  Partial pivoting with row interchanges recorded in
// ipiv[b*n + i] (0-based, LAPACK order).  Row interchanges are applied only
// to the columns right of each panel: the L columns of panel p keep the row
// order they had when panel p was factored, and the solver applies the
// interchanges panel by panel.  The inverses of the unit-lower and upper
// diagonal blocks of every panel are kept in dinv (batch x npanel x 2 x nb x nb).
// info[b] = 0 or the 1-based index of the first exactly-zero pivot.
// Orders up to lu_max_order<R>(): a panel's rows live in the registers of one
// 1024-thread workgroup, 16 complex64 or 8 complex128 values per thread.
constexpr int LU_MAX_N_C64 = 16384, LU_MAX_N_C128 = 8192;
template <typename R> constexpr int lu_max_order() { return sizeof(R) == 4 ? LU_MAX_N_C64 : LU_MAX_N_C128; }
template <typename R> struct LUWork {
  int n = 0, nb = 64, batch = 0;
  long lda = 0, sA = 0;
  cplx<R>* A = nullptr;
  int* ipiv = nullptr;       // batch * n
  cplx<R>* dinv = nullptr;   // batch * npanel * 2 * nb * nb
  int* info = nullptr;       // batch
  const char* tag = "lu";    // kernel-timer class prefix (<tag>_panel, <tag>_update, ...)
  bool gauss3m = false;      // update and solve products with 3 real multiplications
  // every panel's interchanges also applied to all earlier L columns, so that
  // P A = L U with one row order (needed by lu_inverse); otherwise only within
  // the groups of panels the solver uses
  bool full_swap = false;
  // full_swap only, optional: batch * npanel * n ints of work space; each
  // panel's L columns are then moved once, by the composition of the later
  // panels' interchanges, instead of once per later panel
  int* lperm = nullptr;
  // panels in blocks of lu_group(nb): inside a block each panel updates the
  // block's later columns; the columns beyond a block take all its panels'
  // updates as one product with K = 256 (nb <= 128).  With full_swap the
  // later blocks' interchanges reach a block's L columns at the end.
  bool pair = false;
  // look-ahead (optional): the trailing update beyond the next panel runs on
  // `aux`, in column pieces, while the next panel is factored; ev_main /
  // ev_aux order the two
  hipStream_t aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_aux = nullptr;
  int npanel() const { return (n + nb - 1) / nb; }
  static size_t dinv_elems(int n, int nb, int batch) {
    return (size_t)batch * ((n + nb - 1) / nb) * 2 * nb * nb;
  }
};
template <typename R> int lu_factor(const LUWork<R>& w, hipStream_t s);
// Several strided batches of matrices of different orders (same nb and product
// form; blocks of panels as lu_factor's pair mode are always used) factored as one set of
// launches per panel step: every panel, interchange and update launch covers
// all batches whose order reaches that step (updates through gemm_segments,
// a persistent grid over the tiles of all batches).  Look-ahead on aux when
// aux and both events are given.  Each matrix is factored bit for bit as
// lu_factor (with pairs) factors it alone.
template <typename R> int lu_factor_segments(const std::vector<LUWork<R>>& ws, hipStream_t s, hipStream_t aux,
                                             hipEvent_t ev_main, hipEvent_t ev_aux);
// Solves A_b X_b = B_b in place for nrhs columns (B leading dim ldb, stride sB).
// active (optional, device): systems b with active[b] == 0 are left untouched.
template <typename R> int lu_solve(const LUWork<R>& w, cplx<R>* B, long ldb, long sB,
                                   int nrhs, hipStream_t s, const int* active = nullptr);
// Inverses of factors computed with full_swap: out_b = A_b^{-1} (n x n,
// leading dim ldo, stride sO).  X (n x n per matrix, ld n, stride n*n) is
// work space: U^{-1} L^{-1} is formed there (the forward solve on the identity
// skips the zero upper part of L^{-1}) and its columns are scattered to out by
// the row permutation of the factorisation (A^{-1} = U^{-1} L^{-1} P).
// perm: batch * n ints of work space.  out must not overlap X or the factors.
template <typename R> int lu_inverse(const LUWork<R>& w, cplx<R>* X, cplx<R>* out, long ldo, long sO,
                                     int* perm, hipStream_t s);

// ----------------------------------------------------------------- assembly
// Coefficient form: T_j = sum_k f[j*J + k] * A_k for j < nz, written to
// T + j*sT (leading dim ldt).  Coefficient k has kind kinds[k]:
//   0 identity, 1 diagonal (complex128 vector), 2 dense real (float64),
//   3 dense complex (complex128).
struct CoeffSet {
  int n = 0, J = 0;
  const int* kinds_host = nullptr;     // J kinds (host)
  const void* const* mats = nullptr;   // J device pointers (host array)
};
template <typename R> int assemble_coeff(const CoeffSet& cs, int nz, const c128* f_dev,
                                         cplx<R>* T, long ldt, long sT, hipStream_t s);
// BEM single layer: T_ij = exp(i z r_ij)/(4 pi r_ij), T_ii = i z/(4 pi) + 1/(2h).
template <typename R> int assemble_bem(int n, const double* xyz, double h, int nz,
                                       const c128* z_dev, cplx<R>* T, long ldt, long sT,
                                       hipStream_t s);
// Frobenius norms of the BEM matrices at nz nodes (fp64), fro2[j] = ||T(z_j)||_F^2;
// partial holds nz * ceil(n / 2) doubles.
int bem_fro2(int n, const double* xyz, double h, int nz, const c128* z_dev,
             double* partial, double* fro2, hipStream_t s);
// R_j = U - T(z_j) Y_j for the BEM matrix, assembled on the fly in fp64.
int bem_residual(int n, const double* xyz, double h, int nz, const c128* z_dev,
                 const c128* U, long ldu, const c128* Y, long ldy, long sY, int L,
                 c128* Rout, long ldr, long sR, hipStream_t s);

// ------------------------------------------------------------- elementwise
template <typename D, typename S>
int convert(const cplx<S>* src, long lds, long ss, cplx<D>* dst, long ldd, long sd,
            int rows, int cols, int batch, hipStream_t s);
// dst_b = src (same block replicated batch times)
template <typename R>
int replicate(const cplx<R>* src, long lds, cplx<R>* dst, long ldd, long sd, int rows,
              int cols, int batch, hipStream_t s);
// Y_b += D_b (fp64 += fp32) for the batches with active[b] != 0
int add_correction(c128* Y, long ldy, long sY, const c64* D, long ldd, long sD, int rows,
                   int cols, int batch, const int* active, hipStream_t s);
// R_b = U - sum_k coef[b*J+k] * P_k[:, b*L:(b+1)*L]  (P_k = A_k Y, n x (batch*L))
int combine_residual(const c128* U, long ldu, const c128* const* P_dev, int J,
                     const c128* coef, int n, int L, int batch, c128* R, long ldr,
                     hipStream_t s);
// Per-batch Frobenius norm squared of an n x cols block: out[b] (deterministic).
// part holds batch * min(cols, 32) partial sums (unused, and may be null, when
// cols == 1).
constexpr int BLOCK_FRO2_PARTS = 32;
int block_fro2(const c128* X, long ldx, long sX, int rows, int cols, int batch,
               double* out, double* part, hipStream_t s);

// Y = diag(d) X  (n x cols)
int diag_scale(const c128* d, const c128* X, long ldx, c128* Y, long ldy, int n, int cols,
               hipStream_t s);

}  // namespace rsrr
