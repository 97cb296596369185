// Host-only workspace arithmetic: the device memory one solve allocates at
// most (the admission figure of the serving loop) and the batching of the
// reduced-problem nodes.  No HIP dependency, so host-only tests compute the
// same figures as the library.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <utility>

#include "../../include/rsrr.h"

namespace rsrr {

// elements per workgroup of the fused moments / winding-trace kernel
constexpr long MOMENTS_BLOCK = 1024;

// work space (complex128 elements) of the fused moments / winding kernel for
// kk elements per inverse, cnt inverses and J coefficient blocks
inline long moments_wind_parts(long kk, int cnt, int J) {
  return (kk + MOMENTS_BLOCK - 1) / MOMENTS_BLOCK * (long)cnt * J;
}

// (number of batches, nodes per batch) for NS nodes of `per` bytes each in
// chunk_gib GiB: the fewest batches that fit, with the nodes spread evenly.
inline std::pair<int, int> chunk_count(int NS, size_t per, double chunk_gib) {
  const size_t cap = (size_t)(chunk_gib * 1073741824.0);
  const int fit = (int)std::max<size_t>(1, std::min<size_t>(NS, cap / std::max<size_t>(per, 1)));
  const int nb = (NS + fit - 1) / fit;
  return {nb, (NS + nb - 1) / nb};
}

// Panel width of the reduced-problem LUs.
inline int reduced_nb(const rsrr_params* prm) { return prm->nb_reduced > 0 ? prm->nb_reduced : 64; }

// Upper bound of the device workspace of one solve of an order-n problem with
// J coefficients (BEM: the Chebyshev degree decides J) and parameters prm.
inline size_t workspace_bound(int n_, int J_, bool bem, const rsrr_params* prm) {
  const double z = 16.0;   // bytes of a complex128
  const double cap = prm->chunk_gib * 1073741824.0;
  const double n = n_, N = prm->N, L = prm->L, K = prm->K, nb = prm->nb, nbr = reduced_nb(prm);
  const double NL = N * L;
  const double cols = prm->scheme == RSRR_SCHEME_MOMENT ? (double)(prm->Kp > 0 ? prm->Kp : prm->N) * L : NL;
  const double kS = std::min(n, cols), kk = kS * kS, M = K * kS;   // m <= M
  const double J = bem ? (prm->cheb_degree > 0 ? prm->cheb_degree : 40) + 1 : J_;
  // sampling: complex128 factors and diagonal-block inverses (the precision,
  // the fallback of every node, or the fp64 BEM matrices of the refinement),
  // complex64 factors, solutions and residuals
  double samp = N * n * n * z + 2 * N * n * nb * z + (J + 10) * n * NL * z;
  if (prm->precision == RSRR_PREC_C64_IR) samp += N * n * n * 8 + 2 * N * n * nb * 8;
  if (bem) samp += N * n * 8;
  // basis: S_hat or M_hat, Q and the Gram matrices of the levels
  const double basis = (cols + kS) * n * z + 8 * cols * cols * z;
  // projection (BEM: Chebyshev samples T(x_k) and T(x_k) Q in chunks)
  double proj = 2 * J * kk * z + n * kS * z;
  if (bem) {
    // the interpolation samples T(x_k) in batches within chunk_gib (the fp64
    // T(z_j) of the refinement use the complex128 factor buffer above)
    const double fit = std::max(1.0, std::floor(cap / (n * n * z)));
    const double chb = std::min(J, fit);
    proj += chb * n * n * z + chb * n * kS * z + J * J * z + J * kk * z;
  }
  // moments: a batch of T_S(zeta) and inverses within chunk_gib
  const double ch = chunk_count(prm->NS, (size_t)(kk * z * 2), prm->chunk_gib).second;
  const double red = 2 * ch * kk * z + (2 * K + 1) * kk * z + 2 * ch * kS * nbr * z + ch * (kS + 64) * z +
                     ch * std::ceil(kS / nbr) * kS * 4 +
                     (double)moments_wind_parts((long)kk, (int)ch, (int)std::min(J, 4.0)) * z;
  // Hankel matrices, SVD (basis, Jacobi copies), extraction, eigen-solve
  const double hank = 18 * M * M * z + (kS + n) * M * z;
  const double eig = 26 * M * M * z;
  // residual filter
  const double resid = (J + 4) * n * M * z;
  return (size_t)(1.1 * (samp + basis + proj + red + hank + eig + resid)) + ((size_t)64 << 20);
}

}  // namespace rsrr
