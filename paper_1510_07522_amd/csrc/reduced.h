// Small kernels of the reduced problem and the final eigenpairs.
#pragma once
#include "driver.h"

namespace rsrr {
int transpose_blocks(const c128* in, c128* out, int k, int batch, hipStream_t s);
// H (K k square) from the moments Amom (block a at Amom + a*k*k): block (i, j) = A_{i+j+shift}
int build_hankel(const c128* Amom, int k, int K, int shift, c128* H, long ldh, hipStream_t s);
// partial[b*nchunk + c] = sum_{e in chunk c} X_b[e] Y_b[e]   (X_b = X + b*len)
int dot_partials(const c128* X, const c128* Y, long len, int batch, int nchunk, c128* partial,
                 hipStream_t s);
int gather_scale_cols(const c128* in, long ldi, const int* perm, const double* scale, int rows,
                      int ncol, c128* out, long ldo, hipStream_t s);
int normalize_cols(c128* V, long ldv, int rows, int ncol, hipStream_t s);
int fill_c128(c128* x, long n, c128 v, hipStream_t s);
}  // namespace rsrr
