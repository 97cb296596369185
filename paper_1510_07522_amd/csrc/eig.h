// Dense fp64 eigen/SVD building blocks of the projected problem.
#pragma once
#include <vector>

#include "driver.h"

namespace rsrr {

// Singular value decomposition of the M x M matrix H (destroyed) by one-sided
// Jacobi: H = U diag(sigma) W^H, sigma descending.  U, W: M x M outputs.
// Columns whose norm falls below trunc * (largest column norm) are not
// orthogonalised (0 = full accuracy for every singular value).
int jacobi_svd(c128* H, long ldh, int M, c128* U, long ldu, c128* W, long ldw,
               std::vector<double>* sigma, Arena& ws, hipStream_t s, double trunc = 0.0);

// Eigenvalues lam and eigenvectors V (columns, not normalised) of the general
// m x m matrix A (destroyed: it ends in Schur form).
int eig_general(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
                hipStream_t s);

int set_identity(c128* X, long ldx, int m, hipStream_t s);

// Matrices up to this size are put in Schur form by one workgroup (Householder
// + single-shift QR); larger ones by spectral divide and conquer first.
constexpr int DC_LEAF = 128;
int eig_dc(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
           hipStream_t s);
// Schur forms of `count` independent small matrices (len <= 512), in place, with
// their unitary factors Z_b (status_b = QR iterations, or -1 on failure).
int leaf_schur_batched(c128* const* H_dev, c128* const* Z_dev, const int* len_dev, int count,
                       int* status_dev, hipStream_t s);
// Eigenvectors X (columns) of the m x m upper-triangular T.
int tri_eigvecs(const c128* T, long ldt, int m, c128* X, long ldx, hipStream_t s);

}  // namespace rsrr
