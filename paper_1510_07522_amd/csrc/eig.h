// Dense fp64 eigen/SVD building blocks of the projected problem.
#pragma once
#include <vector>

#include "driver.h"

namespace rsrr {

// Singular value decomposition of the M x M matrix H (destroyed) by one-sided
// Jacobi: H = U diag(sigma) W^H, sigma descending.  U, W: M x M outputs.
int jacobi_svd(c128* H, long ldh, int M, c128* U, long ldu, c128* W, long ldw,
               std::vector<double>* sigma, Arena& ws, hipStream_t s);

// Eigenvalues lam and eigenvectors V (columns, not normalised) of the general
// m x m matrix A (destroyed: it ends in Schur form).
int eig_general(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
                hipStream_t s);

int set_identity(c128* X, long ldx, int m, hipStream_t s);

}  // namespace rsrr
