// Dense fp64 eigen/SVD building blocks of the projected problem.
#pragma once
#include <vector>

#include "driver.h"

namespace rsrr {

// Singular value decomposition of the rows x cols matrix X (destroyed) by
// one-sided block Jacobi: X = U diag(sigma) W^H, sigma descending (cols
// values).  U: rows x cols, W: cols x cols.  Columns whose norm falls below
// trunc * (largest column norm) are not orthogonalised (0 = full accuracy
// for every singular value).
int jacobi_svd(c128* X, long ldx, int rows, int cols, c128* U, long ldu, c128* W, long ldw,
               std::vector<double>* sigma, Arena& ws, hipStream_t s, double trunc = 0.0);

// SVD of the M x M matrix H restricted to its numerical range: a pivoted
// orthonormal basis Q1 (r columns, directions above basis_tol * sigma_1) and
// one-sided Jacobi on H^H Q1.  H ~= Vh diag(sigma) Wh^H with Vh, Wh: M x r,
// sigma: r values, descending.  H is not modified.
int hankel_svd(const c128* H, int M, double basis_tol, double trunc, c128* Vh, long ldv, c128* Wh, long ldw,
               std::vector<double>* sigma, int* r_out, Arena& ws, hipStream_t s);

// Eigenvalues lam and eigenvectors V (columns, not normalised) of the general
// m x m matrix A (destroyed: it ends in Schur form).  When spectral splits
// drop a block larger than refine_above relative to its diagonal block, the
// eigenpairs are corrected to first order in the dropped coupling.
int eig_general(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
                hipStream_t s, double refine_above = 0.0);

int set_identity(c128* X, long ldx, int m, hipStream_t s);

// Matrices up to this size are put in Schur form by one workgroup (Householder
// + single-shift QR); larger ones by spectral divide and conquer first.
constexpr int DC_LEAF = 128;
int eig_dc(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
           hipStream_t s, double refine_above = 0.0);
// Schur forms of `count` independent small matrices (len <= DC_LEAF, the
// largest max_len), in place, with their unitary factors Z_b (status_b = QR
// iterations, or -1 on failure).  One workgroup each, in LDS when it fits.
int leaf_schur_batched(c128* const* H_dev, c128* const* Z_dev, const int* len_dev, int count,
                       int* status_dev, hipStream_t s, int max_len);
// Eigenvectors X (columns) of the m x m upper-triangular T.
int tri_eigvecs(const c128* T, long ldt, int m, c128* X, long ldx, hipStream_t s);
// First-order correction of the eigenvectors X of T (from tri_eigvecs) for
// T' = T + E, given P = T' X: X is updated in place, mu (device, m) receives
// the eigenvalue corrections (0 where a correction was not applied).  D: m x m
// work space.
int tri_eigvecs_correct(const c128* T, long ldt, int m, const c128* P, long ldp, c128* X, long ldx,
                        c128* D, c128* mu, hipStream_t s);

}  // namespace rsrr
