// Small kernels of the reduced problem and the final eigenpairs.
#pragma once
#include "bounds.h"
#include "driver.h"

namespace rsrr {
int transpose_blocks(const c128* in, c128* out, int k, int batch, hipStream_t s);
// H (K k square) from the moments Amom (block a at Amom + a*k*k): block (i, j) = A_{i+j+shift}
int build_hankel(const c128* Amom, int k, int K, int shift, c128* H, long ldh, hipStream_t s);
// partial[b*nchunk + c] = sum_{e in chunk c} X_b[e] Y_b[e]   (X_b = X + b*len)
int dot_partials(const c128* X, const c128* Y, long len, int batch, int nchunk, c128* partial,
                 hipStream_t s);
// One pass over the inverses X_m (m < cnt, kk elements each, stride kk) of a
// batch of reduced nodes (Alg. 1, Step 2, and the winding number):
//   A[e + p kk] = (accumulate ? A[e + p kk] : 0) + sum_m X_m[e] cw[m + p cnt]   (p < P)
//   D[m J + k]  = sum_e X_m[e] BT[e + k kk]                                       (k < J)
// Deterministic (fixed summation orders).  Dpart: moments_wind_parts(kk, cnt,
// J) elements of work space.  Returns ST_EINVAL unless P <= 8 and J <= 4.
int moments_wind(const c128* X, long kk, int cnt, const c128* cw, int P, const c128* BT, int J,
                 c128* A, bool accumulate, c128* Dpart, c128* D, hipStream_t s);
int gather_scale_cols(const c128* in, long ldi, const int* perm, const double* scale, int rows,
                      int ncol, c128* out, long ldo, hipStream_t s);
int normalize_cols(c128* V, long ldv, int rows, int ncol, hipStream_t s);
int fill_c128(c128* x, long n, c128 v, hipStream_t s);
}  // namespace rsrr
