// Entries of the Helmholtz single-layer matrix on a point set (cf. eq.
// eq-nyes): T_ij(z) = exp(i z r_ij)/(4 pi r_ij) for i != j and the regularised
// diagonal T_ii(z) = i z/(4 pi) + 1/(2h), generated on the fly by the kernels
// that need them (assembly, Frobenius norms, the fp64 refinement residual).
#pragma once
#include "common.h"

namespace rsrr {

#define RSRR_INV4PI 0.07957747154594767

__device__ inline void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline double exp_r(double x) { return exp(x); }
__device__ inline float exp_r(float x) { return expf(x); }

// exp(i z r)/(4 pi r) = exp(-zi r) (cos(zr r) + i sin(zr r)) / (4 pi r)
template <typename R>
__device__ inline cplx<R> bem_entry(R r, R zr, R zi) {
  R sn, cs;
  sincos_r(zr * r, &sn, &cs);
  const R m = exp_r(-zi * r) * (R(RSRR_INV4PI) / r);
  return mk<R>(m * cs, m * sn);
}

// i z/(4 pi) + 1/(2h)
__device__ inline c128 bem_diag(c128 z, double h) {
  return mk<double>(-z.im * RSRR_INV4PI + 0.5 / h, z.re * RSRR_INV4PI);
}

}  // namespace rsrr
