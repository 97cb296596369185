// Dense fp64 kernels of the projected problem (Alg. 1, Steps 3-4):
//   * one-sided (Hestenes) Jacobi SVD of the block Hankel matrix H, and
//   * the standard eigenproblem of A = V0^H H^< W0 S0^{-1}: Householder
//     reduction to Hessenberg form, single-shift complex QR to Schur form
//     T = Z^H A Z, and eigenvectors of T by back substitution.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "driver.h"
#include "eig.h"
#include "timers.h"

namespace rsrr {

// ------------------------------------------------------------------- SVD
// One-sided block Jacobi.  A round pairs the column blocks (width JB) by the
// circle method.  For every block pair the Gram matrix G of its 2*JB columns
// is formed (partial sums over row slices, added in a fixed order), G is
// diagonalised by cyclic two-sided Jacobi in LDS (accumulated in V), and V is
// applied to the pair's columns of H and W, again by row slices, so a round
// spreads over (pairs x slices) workgroups.  A column pair (p, q) with inner
// product g and squared norms al, be is rotated only if |g| > tol sqrt(al be)
// (relative criterion), |g| > gfloor (absolute noise floor: such rotations
// cannot move a singular value by more than ~sqrt(gfloor)) and al, be > nfloor
// (columns below the caller's truncation level are dropped afterwards and are
// not orthogonalised).  For |g| > 0 the rotation is: column q times
// conj(g)/|g|, then the real rotation t = sign(z)/(|z| + sqrt(1+z^2)),
// z = (be - al)/(2|g|).  `counter` counts the block pairs that were rotated.
constexpr int JB = 16, J2 = 2 * JB, JCH = 32;
constexpr int KSL = 16;   // row slices per block pair in the Gram and apply kernels

// Global column of local column j (0 <= j < 2*JB) of block pair i in `round`
// of the circle method over nbk blocks.
__device__ inline int pair_col(int round, int nbk, int i, int j) {
  const int a = (round + i) % (nbk - 1);
  const int cb = (i == 0) ? nbk - 1 : (round - i + nbk - 1) % (nbk - 1);
  return (j < JB) ? a * JB + j : cb * JB + (j - JB);
}

typedef double jd4 __attribute__((ext_vector_type(4)));
__device__ inline jd4 jmfma(double a, double b, jd4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial Gram X^H X of block pair i = blockIdx.x over row slice ks = blockIdx.y
// on the matrix cores.  A chunk of JCH rows of the pair's 32 columns is staged
// in LDS (real and imaginary parts apart); each wave takes two of the chunk's
// eight 4-row steps and accumulates the blocks (0,0), (0,1), (1,1) of the
// 32x32 Gram (16x16 MFMA blocks, four real products per complex block and
// step; the A and B operands of a lane are the same LDS values).  The wave
// partials are added in LDS in wave order and block (1,0) is the conjugate
// transpose of block (0,1).  MFMA f64 16x16x4 lane layout: A[m][k] and
// B[k][n] with m, n = lane % 16, k = lane / 16; accumulator element r holds
// row lane / 16 + 4 r, column lane % 16.
__global__ __launch_bounds__(256) void bj_gram_kernel(const c128* H, long ldh, int rows, int cols, int nbk,
                                                      int round, int rows_per, c128* part) {
  __shared__ double Xr[JCH][J2 + 1], Xi[JCH][J2 + 1];
  __shared__ c128 R[J2][J2 + 1];
  const int i = blockIdx.x, ks = blockIdx.y, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int r_begin = ks * rows_per, r_end = min(rows, r_begin + rows_per);
  jd4 are[3], aim[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) { are[b] = jd4{0, 0, 0, 0}; aim[b] = jd4{0, 0, 0, 0}; }
  // element e = tid + 256 t of a chunk: row e % JCH, local column e / JCH;
  // the next chunk is loaded into registers while this one is multiplied
  constexpr int PER = JCH * J2 / 256;
  int gcol[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) gcol[t] = pair_col(round, nbk, i, (tid + 256 * t) / JCH);
  c128 pf[PER];
  auto load = [&](int r0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int r = r0 + (tid + 256 * t) % JCH, c = gcol[t];
      pf[t] = (r < r_end && c < cols) ? H[r + (long)c * ldh] : mk<double>(0, 0);
    }
  };
  if (r_begin < r_end) load(r_begin);
  for (int r0 = r_begin; r0 < r_end; r0 += JCH) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + 256 * t;
      Xr[e % JCH][e / JCH] = pf[t].re;
      Xi[e % JCH][e / JCH] = pf[t].im;
    }
    __syncthreads();
    if (r0 + JCH < r_end) load(r0 + JCH);
    for (int q = wave; q < JCH / 4; q += 4) {
      const int kk = q * 4 + (lane >> 4), n = lane & 15;
      const double x0r = Xr[kk][n], x0i = Xi[kk][n], x1r = Xr[kk][16 + n], x1i = Xi[kk][16 + n];
      // conj(x_a) x_b: re = xr_a xr_b + xi_a xi_b, im = xr_a xi_b - xi_a xr_b
      are[0] = jmfma(x0r, x0r, are[0]); are[0] = jmfma(x0i, x0i, are[0]);
      aim[0] = jmfma(x0r, x0i, aim[0]); aim[0] = jmfma(-x0i, x0r, aim[0]);
      are[1] = jmfma(x0r, x1r, are[1]); are[1] = jmfma(x0i, x1i, are[1]);
      aim[1] = jmfma(x0r, x1i, aim[1]); aim[1] = jmfma(-x0i, x1r, aim[1]);
      are[2] = jmfma(x1r, x1r, are[2]); are[2] = jmfma(x1i, x1i, are[2]);
      aim[2] = jmfma(x1r, x1i, aim[2]); aim[2] = jmfma(-x1i, x1r, aim[2]);
    }
    __syncthreads();
  }
  // wave partials added in the order 0, 1, 2, 3
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = (lane >> 4) + 4 * r, n = lane & 15;
        const c128 g0 = mk<double>(are[0][r], aim[0][r]), g1 = mk<double>(are[1][r], aim[1][r]),
                   g2 = mk<double>(are[2][r], aim[2][r]);
        if (w == 0) {
          R[m][n] = g0; R[m][16 + n] = g1; R[16 + m][16 + n] = g2;
        } else {
          R[m][n] = R[m][n] + g0; R[m][16 + n] = R[m][16 + n] + g1; R[16 + m][16 + n] = R[16 + m][16 + n] + g2;
        }
      }
    }
    __syncthreads();
  }
  {
    const int m = tid % 16, n = tid / 16;          // 256 threads: the 16x16 block (1,0)
    R[16 + m][n] = conj(R[n][16 + m]);
  }
  __syncthreads();
  c128* out = part + ((long)i * gridDim.y + ks) * (J2 * J2);
  for (int e = tid; e < J2 * J2; e += 256) out[e] = R[e % J2][e / J2];
}

// Gram of block pair i (slices added in a fixed order), convergence test and
// one sweep of cyclic two-sided Jacobi (circle method over the 2*JB indices)
// per visit: the outer sweeps finish the job, and more inner sweeps do not
// save outer ones (13 outer sweeps with one inner sweep or three on the
// benchmark's Hankel matrix).
// Writes V (2*JB x 2*JB, column-major) and flag[i] = 1 if V is to be applied.
__global__ __launch_bounds__(256) void bj_rotate_kernel(const c128* part, int nks, double tol, double gfloor,
                                                        double nfloor, c128* Vout, int* flag, int* counter) {
  __shared__ c128 G[J2][J2 + 1];
  __shared__ c128 V[J2][J2 + 1];
  __shared__ double s_rc[J2 / 2], s_rs[J2 / 2];
  __shared__ c128 s_ph[J2 / 2];
  __shared__ int s_pp[J2 / 2], s_qq[J2 / 2];
  __shared__ int s_flag;
  const int i = blockIdx.x, tid = threadIdx.x;
  for (int e = tid; e < J2 * J2; e += 256) {
    c128 g = mk<double>(0, 0);
    for (int ks = 0; ks < nks; ++ks) g = g + part[((long)i * nks + ks) * (J2 * J2) + e];
    G[e % J2][e / J2] = g;
    V[e % J2][e / J2] = mk<double>((e % J2) == (e / J2) ? 1.0 : 0.0, 0);
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  for (int e = tid; e < J2 * J2; e += 256) {
    const int p = e % J2, q = e / J2;
    if (p < q) {
      const double al = G[p][p].re, be = G[q][q].re, g = sqrt(abs2(G[p][q]));
      if (al > nfloor && be > nfloor && g > tol * sqrt(al * be) && g > gfloor) s_flag = 1;
    }
  }
  __syncthreads();
  const int need = s_flag;
  if (tid == 0) {
    flag[i] = need;
    if (need) atomicAdd(counter, 1);
  }
  if (!need) return;
  for (int sweep = 0; sweep < 1; ++sweep) {
    __syncthreads();
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int step = 0; step < J2 - 1; ++step) {
      if (tid < J2 / 2) {
        const int x = (step + tid) % (J2 - 1);
        const int y = (tid == 0) ? J2 - 1 : (step - tid + J2 - 1) % (J2 - 1);
        const int p = min(x, y), q = max(x, y);
        const double al = G[p][p].re, be = G[q][q].re;
        const c128 gpq = G[p][q];
        const double g = sqrt(abs2(gpq));
        double c = 1, sn = 0;
        c128 phc = mk<double>(1, 0);
        if (al > nfloor && be > nfloor && g > tol * sqrt(al * be) && g > gfloor) {
          s_flag = 1;
          phc = mk<double>(gpq.re / g, -gpq.im / g);
          const double zeta = (be - al) / (2.0 * g);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = c * t;
        }
        s_pp[tid] = p; s_qq[tid] = q; s_rc[tid] = c; s_rs[tid] = sn; s_ph[tid] = phc;
      }
      __syncthreads();
      // The step's pairs are disjoint and cover every index, so G <- J^H G J
      // acts on each 2x2 block (rows of pair k, columns of pair l) on its own:
      // with M = [[c, s], [-s phc, c phc]] per pair, block <- M_k^H block M_l;
      // V <- V J acts on each row's 2-vector of pair l.  One phase, no thread
      // reads what another writes.
      for (int e = tid; e < (J2 / 2) * (J2 / 2) + J2 * (J2 / 2); e += 256) {
        if (e < (J2 / 2) * (J2 / 2)) {
          const int k = e % (J2 / 2), l = e / (J2 / 2);
          if (s_rs[k] == 0.0 && s_rs[l] == 0.0) continue;
          const int pk = s_pp[k], qk = s_qq[k], pl = s_pp[l], ql = s_qq[l];
          // columns of the block: [x, y] <- [c x - s ph y, s x + c ph y] with pair l
          const double cl = s_rc[l], sl = s_rs[l];
          const c128 phl = s_ph[l];
          c128 a0 = G[pk][pl], a1 = G[pk][ql] * phl, b0 = G[qk][pl], b1 = G[qk][ql] * phl;
          c128 u0 = cl * a0 - sl * a1, u1 = sl * a0 + cl * a1;    // row pk
          c128 w0 = cl * b0 - sl * b1, w1 = sl * b0 + cl * b1;    // row qk
          // rows: [x; y] <- [c x - s conj(ph) y; s x + c conj(ph) y] with pair k
          const double ck = s_rc[k], sk = s_rs[k];
          const c128 phb = conj(s_ph[k]);
          w0 = w0 * phb;
          w1 = w1 * phb;
          G[pk][pl] = ck * u0 - sk * w0;
          G[pk][ql] = ck * u1 - sk * w1;
          G[qk][pl] = sk * u0 + ck * w0;
          G[qk][ql] = sk * u1 + ck * w1;
        } else {
          const int f = e - (J2 / 2) * (J2 / 2);
          const int l = f / J2, r = f % J2;
          if (s_rs[l] == 0.0) continue;
          const int p = s_pp[l], q = s_qq[l];
          const double c = s_rc[l], sn = s_rs[l];
          const c128 x = V[r][p], y = V[r][q] * s_ph[l];
          V[r][p] = c * x - sn * y;
          V[r][q] = sn * x + c * y;
        }
      }
      __syncthreads();
    }
    if (!s_flag) break;   // every thread reads s_flag before the reset above (barrier first)
  }
  c128* vo = Vout + (long)i * (J2 * J2);
  for (int e = tid; e < J2 * J2; e += 256) vo[e] = V[e % J2][e / J2];
}

// Columns of block pair i = blockIdx.x times its V (32x32) over row slice
// ks = blockIdx.y, for H (blockIdx.z == 0, rowsH rows) or W (blockIdx.z == 1,
// rowsW rows); both have `cols` columns.  On the matrix cores: a chunk of JAR
// rows of the pair's columns is staged in LDS column by column (real and
// imaginary parts apart), each wave computes 16 rows x 32 columns (two 16x16
// MFMA blocks, four real products per complex block and 4-column step), and
// the result goes back through LDS so that the global stores run along rows.
constexpr int JAR = 64;
__global__ __launch_bounds__(256) void bj_apply_kernel(c128* H, long ldh, int rowsH, c128* W, long ldw,
                                                       int rowsW, int cols, int nbk, int round, int rows_per,
                                                       const c128* Vin, const int* flag) {
  __shared__ double Xr[J2][JAR + 1], Xi[J2][JAR + 1];
  __shared__ double Vr[J2][J2 + 1], Vi[J2][J2 + 1];
  __shared__ int s_gc[J2];
  const int i = blockIdx.x, ks = blockIdx.y, tid = threadIdx.x;
  if (!flag[i]) return;
  c128* Mx = blockIdx.z == 0 ? H : W;
  const long ld = blockIdx.z == 0 ? ldh : ldw;
  const int rows = blockIdx.z == 0 ? rowsH : rowsW;
  const int wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < J2 * J2; e += 256) {
    const c128 v = Vin[(long)i * (J2 * J2) + e];
    Vr[e % J2][e / J2] = v.re;
    Vi[e % J2][e / J2] = v.im;
  }
  if (tid < J2) s_gc[tid] = pair_col(round, nbk, i, tid);
  const int r_begin = ks * rows_per, r_end = min(rows, r_begin + rows_per);
  // element e = tid + 256 t of a chunk: row e % JAR, local column e / JAR; the
  // next chunk is loaded into registers while this one is multiplied
  constexpr int PER = JAR * J2 / 256;
  int gcol[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) gcol[t] = pair_col(round, nbk, i, (tid + 256 * t) / JAR);
  c128 pf[PER];
  auto load = [&](int r0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int r = r0 + (tid + 256 * t) % JAR, c = gcol[t];
      pf[t] = (r < r_end && c < cols) ? Mx[r + (long)c * ld] : mk<double>(0, 0);
    }
  };
  if (r_begin < r_end) load(r_begin);
  for (int r0 = r_begin; r0 < r_end; r0 += JAR) {
    __syncthreads();                     // V, s_gc ready; the previous chunk's stores done
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + 256 * t;
      Xr[e / JAR][e % JAR] = pf[t].re;
      Xi[e / JAR][e % JAR] = pf[t].im;
    }
    __syncthreads();
    if (r0 + JAR < r_end) load(r0 + JAR);
    jd4 yr[2], yi[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) { yr[b] = jd4{0, 0, 0, 0}; yi[b] = jd4{0, 0, 0, 0}; }
    const int m = 16 * wave + (lane & 15);
#pragma unroll 4
    for (int kq = 0; kq < J2 / 4; ++kq) {
      const int kk = kq * 4 + (lane >> 4);
      const double ar = Xr[kk][m], ai = Xi[kk][m];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double br = Vr[kk][16 * b + (lane & 15)], bi = Vi[kk][16 * b + (lane & 15)];
        // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
        yr[b] = jmfma(ar, br, yr[b]); yr[b] = jmfma(-ai, bi, yr[b]);
        yi[b] = jmfma(ar, bi, yi[b]); yi[b] = jmfma(ai, br, yi[b]);
      }
    }
    __syncthreads();                     // every wave has read the chunk
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * wave + (lane >> 4) + 4 * r, col = 16 * b + (lane & 15);
        Xr[col][row] = yr[b][r];
        Xi[col][row] = yi[b][r];
      }
    __syncthreads();
    for (int e = tid; e < JAR * J2; e += 256) {
      const int rr = e % JAR, j = e / JAR;
      const int r = r0 + rr, c = s_gc[j];
      if (r < r_end && c < cols) Mx[r + (long)c * ld] = mk<double>(Xr[j][rr], Xi[j][rr]);
    }
  }
}

__global__ __launch_bounds__(256) void col_norms_kernel(const c128* H, long ldh, int M, int ncol,
                                                        double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  if (j >= ncol) return;
  double acc = 0;
  for (int r = threadIdx.x; r < M; r += 256) acc += abs2(H[r + (long)j * ldh]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sqrt(red[0]);
}

// out[:, j] = in[:, perm[j]] * scale[j]  (scale may be null)
__global__ __launch_bounds__(256) void permute_cols_kernel(const c128* in, long ldi, const int* perm,
                                                           const double* scale, int rows, int ncol,
                                                           c128* out, long ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * ncol) return;
  const int r = (int)(e % rows), j = (int)(e / rows);
  const int src = perm[j];
  c128 v = in[r + (long)src * ldi];
  if (scale) v = scale[j] * v;
  out[r + (long)j * ldo] = v;
}

__global__ void identity_kernel(c128* X, long ldx, int m) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)m * m) return;
  const int r = (int)(e % m), c = (int)(e / m);
  X[r + (long)c * ldx] = mk<double>(r == c ? 1.0 : 0.0, 0);
}

int set_identity(c128* X, long ldx, int m, hipStream_t s) {
  if (m <= 0) return ST_OK;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)cdivl((long)m * m, 256)), dim3(256), 0, s, X, ldx, m);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

int jacobi_svd(c128* X, long ldx, int rows, int cols, c128* U, long ldu, c128* W, long ldw,
               std::vector<double>* sigma, Arena& ws, hipStream_t s, double trunc) {
  sigma->clear();
  if (rows <= 0 || cols <= 0) return ST_OK;
  int* cnt = nullptr;
  double* sg = nullptr;
  int* perm = nullptr;
  c128 *Wa = nullptr, *Wb = nullptr, *Xb = nullptr;
  RSRR_TRY(ws.get<int>("sv_cnt", 64, &cnt));
  RSRR_TRY(ws.get<double>("sv_sig", cols, &sg));
  RSRR_TRY(ws.get<int>("sv_perm", cols, &perm));
  // X and the accumulated W ping-pong with Xb, Wb (columns re-sorted by
  // decreasing norm at the start of every sweep)
  RSRR_TRY(ws.get<c128>("sv_Wa", (size_t)cols * cols, &Wa));
  RSRR_TRY(ws.get<c128>("sv_Wb", (size_t)cols * cols, &Wb));
  RSRR_TRY(ws.get<c128>("sv_Xb", (size_t)rows * cols, &Xb));
  RSRR_TRY(set_identity(Wa, cols, cols, s));
  RSRR_HIP(hipMemsetAsync(cnt, 0, 64 * sizeof(int), s));
  const double u = 1.1102230246251565e-16;
  const double tol = 16.0 * u * sqrt((double)rows);
  const int maxsweep = 40;
  // absolute floors from the largest column norm
  std::vector<double> h0(cols);
  hipLaunchKernelGGL(col_norms_kernel, dim3(cols), dim3(256), 0, s, X, ldx, rows, cols, sg);
  RSRR_LAUNCH_CHECK();
  RSRR_HIP(hipMemcpyAsync(h0.data(), sg, cols * sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  double smax = 0;
  for (double v : h0) smax = std::max(smax, v);
  const double fl = sqrt((double)rows) * 2.0 * u * smax;
  const double gfloor = fl * fl;
  const double nfloor = (trunc * smax) * (trunc * smax);
  // nbk blocks of JB columns (padded to an even count), paired by the circle method
  int nbk = (cols + JB - 1) / JB;
  nbk += (nbk & 1);
  const int np = nbk / 2;
  // row slices of the Gram / apply kernels (multiples of JCH rows)
  const int rows_per = (int)(cdivl(cdivl(std::max(rows, cols), KSL), JCH) * JCH);
  const int nks = (int)cdivl(std::max(rows, cols), rows_per);
  c128 *part = nullptr, *Vr = nullptr;
  int* flg = nullptr;
  RSRR_TRY(ws.get<c128>("sv_part", (size_t)np * nks * J2 * J2, &part));
  RSRR_TRY(ws.get<c128>("sv_V", (size_t)np * J2 * J2, &Vr));
  RSRR_TRY(ws.get<int>("sv_flag", (size_t)np, &flg));
  c128* Xc = X;
  long ldc = ldx;
  c128* Wc = Wa;
  std::vector<int> ord(cols);
  bool converged = false;
  int sweep = 0;
  for (; sweep < maxsweep && !converged; ++sweep) {
    hipLaunchKernelGGL(col_norms_kernel, dim3(cols), dim3(256), 0, s, Xc, ldc, rows, cols, sg);
    RSRR_LAUNCH_CHECK();
    RSRR_HIP(hipMemcpyAsync(h0.data(), sg, cols * sizeof(double), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return h0[x] > h0[y]; });
    RSRR_HIP(hipMemcpyAsync(perm, ord.data(), cols * sizeof(int), hipMemcpyHostToDevice, s));
    c128* Xn = (Xc == Xb) ? X : Xb;
    const long ldn = (Xc == Xb) ? ldx : rows;
    c128* Wn = (Wc == Wb) ? Wa : Wb;
    hipLaunchKernelGGL(permute_cols_kernel, dim3((unsigned)cdivl((long)rows * cols, 256)), dim3(256), 0, s, Xc,
                       ldc, perm, nullptr, rows, cols, Xn, ldn);
    RSRR_LAUNCH_CHECK();
    hipLaunchKernelGGL(permute_cols_kernel, dim3((unsigned)cdivl((long)cols * cols, 256)), dim3(256), 0, s, Wc,
                       (long)cols, perm, nullptr, cols, cols, Wn, (long)cols);
    RSRR_LAUNCH_CHECK();
    Xc = Xn;
    ldc = ldn;
    Wc = Wn;
    if (cols >= 2) {
      // per round: np block pairs; each reads its 2*JB columns of X twice
      // (Gram, apply) and of W once, and writes both once
      for (int r = 0; r < nbk - 1; ++r) {
        {
          KernelTimer kt("jacobi_gram", s, 8.0 * np * J2 * J2 * (double)rows, np * J2 * (double)rows * sizeof(c128),
                         "bj_gram_kernel");
          hipLaunchKernelGGL(bj_gram_kernel, dim3(np, nks), dim3(256), 0, s, Xc, ldc, rows, cols, nbk, r, rows_per,
                             part);
          RSRR_LAUNCH_CHECK();
        }
        {
          KernelTimer kt("jacobi_rotate", s, 0.0, 0.0, "bj_rotate_kernel");
          hipLaunchKernelGGL(bj_rotate_kernel, dim3(np), dim3(256), 0, s, part, nks, tol, gfloor, nfloor, Vr, flg,
                             cnt + (sweep % 64));
          RSRR_LAUNCH_CHECK();
        }
        {
          // upper bound: every pair rotated (skipped pairs cost nothing)
          KernelTimer kt("jacobi_apply", s, 8.0 * np * J2 * J2 * (double)(rows + cols),
                         2.0 * np * J2 * (double)(rows + cols) * sizeof(c128), "bj_apply_kernel");
          hipLaunchKernelGGL(bj_apply_kernel, dim3(np, nks, 2), dim3(256), 0, s, Xc, ldc, rows, Wc, (long)cols,
                             cols, cols, nbk, r, rows_per, Vr, flg);
          RSRR_LAUNCH_CHECK();
        }
      }
    }
    int c = 0;
    RSRR_HIP(hipMemcpyAsync(&c, cnt + (sweep % 64), sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    if (c == 0) converged = true;
    vlog("jacobi sweep %d: %d block pairs rotated", sweep, c);
  }
  if (!converged) return set_error(ST_ENOTCONV, "Jacobi SVD did not converge in %d sweeps", maxsweep);
  hipLaunchKernelGGL(col_norms_kernel, dim3(cols), dim3(256), 0, s, Xc, ldc, rows, cols, sg);
  RSRR_LAUNCH_CHECK();
  std::vector<double> hs(cols);
  RSRR_HIP(hipMemcpyAsync(hs.data(), sg, cols * sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  std::vector<int> order(cols);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return hs[x] > hs[y]; });
  sigma->resize(cols);
  std::vector<double> inv(cols);
  for (int j = 0; j < cols; ++j) {
    (*sigma)[j] = hs[order[j]];
    inv[j] = hs[order[j]] > 0 ? 1.0 / hs[order[j]] : 0.0;
  }
  double* invd = nullptr;
  RSRR_TRY(ws.get<double>("sv_inv", cols, &invd));
  RSRR_HIP(hipMemcpyAsync(perm, order.data(), cols * sizeof(int), hipMemcpyHostToDevice, s));
  RSRR_HIP(hipMemcpyAsync(invd, inv.data(), cols * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(permute_cols_kernel, dim3((unsigned)cdivl((long)rows * cols, 256)), dim3(256), 0, s, Xc, ldc,
                     perm, invd, rows, cols, U, ldu);
  RSRR_LAUNCH_CHECK();
  hipLaunchKernelGGL(permute_cols_kernel, dim3((unsigned)cdivl((long)cols * cols, 256)), dim3(256), 0, s, Wc,
                     (long)cols, perm, nullptr, cols, cols, W, ldw);
  RSRR_LAUNCH_CHECK();
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

// SVD of the M x M Hankel matrix H by one-sided Jacobi preconditioned with a
// column-pivoted orthonormal basis Q1 of range(H) (H P = Q1 R; pivoted
// Cholesky of H^H H with deflation levels (three at most), the same basis routine as
// Alg. 2 Step 3):  Jacobi runs on X = H^H Q1 = P R^H, whose columns are far
// closer to orthogonal than those of H, so far fewer sweeps are needed.
// X J = Wh diag(sigma)  =>  H = (Q1 J) diag(sigma) Wh^H.
static int svd_gemm(int opA, int opB, int M, int N, int K, const c128* A, long lda, const c128* B, long ldb,
                    c128* C, long ldc, hipStream_t s) {
  GemmBatch<double> g;
  g.tag = "svd_gemm";
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = mk<double>(1, 0); g.beta = mk<double>(0, 0);
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  return gemm_batched<double>(g, s);
}

int hankel_svd(const c128* H, int M, double basis_tol, double trunc, c128* Vh, long ldv, c128* Wh, long ldw,
               std::vector<double>* sigma, int* r_out, Arena& ws, hipStream_t s) {
  *r_out = 0;
  sigma->clear();
  if (M <= 0) return ST_OK;
  c128 *Q1 = nullptr, *Xh = nullptr, *J = nullptr;
  RSRR_TRY(ws.get<c128>("hs_Q1", (size_t)M * M, &Q1));
  int r = 0;
  RSRR_TRY(ortho_impl(M, M, H, M, basis_tol, Q1, M, &r, ws, s, 3));
  if (r == 0) return ST_OK;
  RSRR_TRY(ws.get<c128>("hs_X", (size_t)M * r, &Xh));
  RSRR_TRY(ws.get<c128>("hs_J", (size_t)r * r, &J));
  RSRR_TRY(svd_gemm(OP_C, OP_N, M, r, M, H, M, Q1, M, Xh, M, s));
  RSRR_TRY(jacobi_svd(Xh, M, M, r, Wh, ldw, J, r, sigma, ws, s, trunc));
  RSRR_TRY(svd_gemm(OP_N, OP_N, M, r, r, Q1, M, J, r, Vh, ldv, s));
  *r_out = r;
  return ST_OK;
}

// ------------------------------------------------------------- Schur QR
// Single-shift complex QR on the Hessenberg matrix (one workgroup), with the
// full Schur form (rotations applied to all columns right / rows above) and
// the accumulated unitary Z.
constexpr int QT = 1024;
__device__ inline c128 csqrt_d(c128 z) {
  const double r = sqrt(sqrt(abs2(z)));
  const double th = 0.5 * atan2(z.im, z.re);
  return mk<double>(r * cos(th), r * sin(th));
}

__device__ __forceinline__ void hqr_body(c128* H, long ldh, c128* Z, long ldz, int m, int maxit, int* status) {
  __shared__ int s_l, s_i, s_its, s_total;
  __shared__ c128 s_rot[2];     // (c, s) with c real in rot[0].re
  __shared__ int s_red[QT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double ulp = 2.220446049250313e-16;
  if (tid == 0) { s_i = m - 1; s_its = 0; s_total = 0; }
  __syncthreads();
  while (true) {
    const int i = s_i;
    if (i < 0) break;
    // deflation: largest k in [1, i] with a negligible subdiagonal (else 0)
    int best = 0;
    for (int k = 1 + tid; k <= i; k += QT) {
      const double sub = cabs1(H[k + (long)(k - 1) * ldh]);
      const double dsum = cabs1(H[k - 1 + (long)(k - 1) * ldh]) + cabs1(H[k + (long)k * ldh]);
      if (sub <= ulp * dsum) best = max(best, k);
    }
    for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off));
    if (lane == 0) s_red[wave] = best;
    __syncthreads();
    if (tid == 0) {
      int b = 0;
      for (int q = 0; q < QT / 64; ++q) b = max(b, s_red[q]);
      if (b > 0) H[b + (long)(b - 1) * ldh] = mk<double>(0, 0);
      s_l = b;
    }
    __syncthreads();
    const int l = s_l;
    if (l == i) {                        // 1x1 block converged
      if (tid == 0) { s_i = i - 1; s_its = 0; }
      __syncthreads();
      continue;
    }
    if (tid == 0) {
      s_its += 1;
      s_total += 1;
    }
    __syncthreads();
    if (s_total > maxit) {
      if (tid == 0) *status = -1;
      return;
    }
    // shift and first rotation (thread 0)
    for (int k = l; k < i; ++k) {
      if (tid == 0) {
        c128 x, y;
        if (k == l) {
          c128 mu;
          const int its = s_its;
          if (its == 10 || its == 20) {
            const c128 hii = H[i + (long)i * ldh];
            mu = mk<double>(hii.re + 0.75 * fabs(H[i + (long)(i - 1) * ldh].re), hii.im);
          } else {
            const c128 a = H[i - 1 + (long)(i - 1) * ldh], b = H[i - 1 + (long)i * ldh];
            const c128 c = H[i + (long)(i - 1) * ldh], d = H[i + (long)i * ldh];
            const c128 tr = 0.5 * (a + d);
            const c128 disc = csqrt_d(tr * tr - (a * d - b * c));
            const c128 e1 = tr + disc, e2 = tr - disc;
            mu = (abs2(e1 - d) < abs2(e2 - d)) ? e1 : e2;
          }
          x = H[l + (long)l * ldh] - mu;
          y = H[l + 1 + (long)l * ldh];
        } else {
          x = H[k + (long)(k - 1) * ldh];
          y = H[k + 1 + (long)(k - 1) * ldh];
        }
        const double ax = sqrt(abs2(x)), ay = sqrt(abs2(y));
        const double rho = hypot(ax, ay);
        c128 cc = mk<double>(1, 0), ss = mk<double>(0, 0);
        if (rho > 0) {
          if (ax == 0) { cc = mk<double>(0, 0); ss = mk<double>(y.re / ay, -y.im / ay); }
          else {
            cc = mk<double>(ax / rho, 0);
            const c128 ph = mk<double>(x.re / ax, x.im / ax);
            ss = (1.0 / rho) * mulc(ph, y);     // ph * conj(y) / rho
          }
        }
        s_rot[0] = cc;
        s_rot[1] = ss;
      }
      __syncthreads();
      const double c = s_rot[0].re;
      const c128 sn = s_rot[1];
      // rows k, k+1:  [r_k; r_k1] = [c, s; -conj(s), c] [r_k; r_k1]
      const int c0 = (k == l) ? l : k - 1;
      for (int col = c0 + tid; col < m; col += QT) {
        const c128 a = H[k + (long)col * ldh], b = H[k + 1 + (long)col * ldh];
        H[k + (long)col * ldh] = c * a + sn * b;
        H[k + 1 + (long)col * ldh] = c * b - conj(sn) * a;
      }
      __syncthreads();
      // columns k, k+1:  [c_k, c_k1] = [c_k, c_k1] G^H, G^H = [c, -s; conj(s), c]
      const int r1 = min(k + 2, i);
      for (int row = tid; row <= r1; row += QT) {
        const c128 a = H[row + (long)k * ldh], b = H[row + (long)(k + 1) * ldh];
        H[row + (long)k * ldh] = c * a + conj(sn) * b;
        H[row + (long)(k + 1) * ldh] = c * b - sn * a;
      }
      for (int row = tid; row < m; row += QT) {
        const c128 a = Z[row + (long)k * ldz], b = Z[row + (long)(k + 1) * ldz];
        Z[row + (long)k * ldz] = c * a + conj(sn) * b;
        Z[row + (long)(k + 1) * ldz] = c * b - sn * a;
      }
      __syncthreads();
      if (k > l && tid == 0) H[k + 1 + (long)(k - 1) * ldh] = mk<double>(0, 0);
      __syncthreads();
    }
  }
  if (tid == 0) *status = s_total;
}

// Schur form of many small independent matrices, one workgroup each:
// Householder reduction to Hessenberg form (accumulated into Z = I ...), then
// the single-shift QR of hqr_body.  H_b and Z_b are len_b x len_b, ld len_b.
struct LeafArgs {
  c128* const* H;
  c128* const* Z;
  const int* len;
  int* status;
  int lds_len;      // matrices up to this order are worked on in LDS
};
// dynamic LDS for H (m x m complex128) beside the kernel's static arrays
constexpr int LEAF_LDS_BYTES = 144 * 1024;
inline int leaf_lds_len() {
  int m = 0;
  while ((long)(m + 1) * (m + 1) * (long)sizeof(c128) <= LEAF_LDS_BYTES) ++m;
  return m;
}

__global__ __launch_bounds__(QT) void leaf_schur_kernel(LeafArgs a) {
  __shared__ c128 s_v[DC_LEAF];
  __shared__ double s_red[QT / 64];
  extern __shared__ c128 s_H[];
  const int b = blockIdx.x;
  c128* const Hg = a.H[b];
  c128* Z = a.Z[b];
  const int m = a.len[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // small enough: the reduction and the QR iteration run on a copy in LDS,
  // where every step's reads and writes take a fraction of a global round trip
  const bool lds = m <= a.lds_len;
  c128* H = lds ? s_H : Hg;
  for (int e = tid; e < m * m; e += QT) Z[e] = mk<double>((e % m) == (e / m) ? 1.0 : 0.0, 0);
  if (lds)
    for (int e = tid; e < m * m; e += QT) s_H[e] = Hg[e];
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    double acc = 0;
    for (int r = k + 1 + tid; r < m; r += QT) acc += abs2(H[r + (long)k * m]);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s_red[wave] = acc;
    __syncthreads();
    double nx2 = 0;
    for (int q = 0; q < QT / 64; ++q) nx2 += s_red[q];
    const c128 x0 = H[k + 1 + (long)k * m];
    const double ax0 = sqrt(abs2(x0));
    if (!(nx2 - abs2(x0) > 0.0)) { __syncthreads(); continue; }
    const double nx = sqrt(nx2);
    const c128 ph = ax0 > 0 ? mk<double>(x0.re / ax0, x0.im / ax0) : mk<double>(1, 0);
    const c128 alpha = mk<double>(-ph.re * nx, -ph.im * nx);
    const double vn = sqrt(2.0 * nx * (nx + ax0));
    for (int r = tid; r < m; r += QT) {
      c128 v = mk<double>(0, 0);
      if (r > k) {
        v = H[r + (long)k * m];
        if (r == k + 1) v = v - alpha;
        v = (1.0 / vn) * v;
      }
      s_v[r] = v;
    }
    __syncthreads();
    for (int r = k + 1 + tid; r < m; r += QT) H[r + (long)k * m] = (r == k + 1) ? alpha : mk<double>(0, 0);
    // left: columns c > k, one thread per column
    for (int c = k + 1 + tid; c < m; c += QT) {
      c128 w = mk<double>(0, 0);
      for (int r = k + 1; r < m; ++r) w = w + cmul(s_v[r], H[r + (long)c * m]);
      for (int r = k + 1; r < m; ++r) {
        const c128 t = s_v[r] * w;
        H[r + (long)c * m] = mk<double>(H[r + (long)c * m].re - 2 * t.re, H[r + (long)c * m].im - 2 * t.im);
      }
    }
    __syncthreads();
    // right: rows of H and of Z, one thread per row
    for (int r = tid; r < m; r += QT) {
      c128 u = mk<double>(0, 0), uz = mk<double>(0, 0);
      for (int c = k + 1; c < m; ++c) {
        u = u + H[r + (long)c * m] * s_v[c];
        uz = uz + Z[r + (long)c * m] * s_v[c];
      }
      for (int c = k + 1; c < m; ++c) {
        const c128 t = mulc(u, s_v[c]), tz = mulc(uz, s_v[c]);
        H[r + (long)c * m] = mk<double>(H[r + (long)c * m].re - 2 * t.re, H[r + (long)c * m].im - 2 * t.im);
        Z[r + (long)c * m] = mk<double>(Z[r + (long)c * m].re - 2 * tz.re, Z[r + (long)c * m].im - 2 * tz.im);
      }
    }
    __syncthreads();
  }
  hqr_body(H, m, Z, m, m, 60 * m + 100, a.status + b);
  if (lds) {
    __syncthreads();
    for (int e = tid; e < m * m; e += QT) Hg[e] = s_H[e];
  }
}

int leaf_schur_batched(c128* const* H_dev, c128* const* Z_dev, const int* len_dev, int count,
                       int* status_dev, hipStream_t s, int max_len) {
  if (count <= 0) return ST_OK;
  if (max_len > DC_LEAF) return set_error(ST_EINVAL, "leaf_schur: order %d above %d", max_len, DC_LEAF);
  LeafArgs a;
  a.H = H_dev; a.Z = Z_dev; a.len = len_dev; a.status = status_dev;
  a.lds_len = leaf_lds_len();
  const size_t shm = (size_t)std::min(max_len, a.lds_len) * std::min(max_len, a.lds_len) * sizeof(c128);
  KernelTimer kt("leaf_schur", s, 0.0, 0.0);
  hipLaunchKernelGGL(leaf_schur_kernel, dim3(count), dim3(QT), shm, s, a);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// Eigenvector i of the upper-triangular T (one workgroup per eigenvalue):
// x_i = 1, x_j = -(sum_{l>j} T[j][l] x_l) / (T[j][j] - T[i][i]) for j < i.
__global__ __launch_bounds__(256) void trevc_kernel(const c128* T, long ldt, int m, double small,
                                                    c128* X, long ldx) {
  extern __shared__ c128 r_acc[];      // m partial sums
  const int i = blockIdx.x;
  const c128 lam = T[i + (long)i * ldt];
  c128* x = X + (long)i * ldx;
  for (int j = threadIdx.x; j < m; j += 256) {
    r_acc[j] = mk<double>(0, 0);
    x[j] = mk<double>(j == i ? 1.0 : 0.0, 0);
  }
  __syncthreads();
  c128 xl = mk<double>(1, 0);
  for (int l = i; l >= 1; --l) {
    // column l of T contributes to rows j < l
    for (int j = threadIdx.x; j < l; j += 256) r_acc[j] = r_acc[j] + T[j + (long)l * ldt] * xl;
    __syncthreads();
    c128 d = T[l - 1 + (long)(l - 1) * ldt] - lam;
    if (abs2(d) < small * small) d = mk<double>(small, 0);
    const c128 r = r_acc[l - 1];
    xl = cdiv(mk<double>(-r.re, -r.im), d);
    if (threadIdx.x == 0) x[l - 1] = xl;
    __syncthreads();
  }
}

static __global__ __launch_bounds__(256) void diag_gather_kernel(const c128* A, long lda, int m, c128* d) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < m) d[j] = A[j + (long)j * lda];
}

// Diagonal of A (device) to the host: gathered into tmp (m device elements)
// by a kernel, then one contiguous copy.  (A strided 2-D copy of the diagonal
// straight to pageable host memory returned zeros in runs under the kernel
// profiler.)
static int diag_to_host(const c128* A, long lda, int m, c128* tmp, std::vector<c128>* out, hipStream_t s) {
  out->resize(m);
  hipLaunchKernelGGL(diag_gather_kernel, dim3((unsigned)cdivl(m, 256)), dim3(256), 0, s, A, lda, m, tmp);
  RSRR_LAUNCH_CHECK();
  RSRR_HIP(hipMemcpyAsync(out->data(), tmp, (size_t)m * sizeof(c128), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

int tri_eigvecs(const c128* T, long ldt, int m, c128* X, long ldx, hipStream_t s) {
  std::vector<c128> diag;
  RSRR_TRY(diag_to_host(T, ldt, m, X, &diag, s));    // X is written by the kernel below
  double tnorm = 0;
  for (int j = 0; j < m; ++j) tnorm = std::max(tnorm, sqrt(abs2(diag[j])));
  const double small = std::max(tnorm, 1e-300) * 2.220446049250313e-16;
  const size_t shm = (size_t)m * sizeof(c128);
  if (shm > 150 * 1024) return set_error(ST_EINVAL, "eigenvectors: m=%d too large", m);
  KernelTimer kt("trevc", s, 8.0 * (double)m * m * m / 6, 16.0 * (double)m * m * m / 2);
  hipLaunchKernelGGL(trevc_kernel, dim3(m), dim3(256), shm, s, T, ldt, m, small, X, ldx);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// First-order correction of eigenvector i of the upper-triangular T when the
// Schur form it came from is inexact: T' = T + E (E the coupling a spectral
// split dropped), x = X[:, i] with T x = t x (x_i = 1), P[:, i] = T' x and
// R = P - t x.  Solves (T - t I) d = mu x - R with d_i = 0 by one
// back-substitution from the last row up (row i gives mu); then x + d and
// t + mu satisfy T' (x + d) = (t + mu)(x + d) up to second-order terms.  The
// correction is applied only if ||d|| <= ||x|| / 10 (else mu_out[i] = 0 and
// x is kept), and only to eigenvectors with ||R|| > tau ||x|| (the others are
// already backward stable).  D: m x m work space (column i holds d).  One
// workgroup per eigenvector; r_acc[j] = sum_{k > j} T[j][k] d_k.
__device__ inline void block_sum2(double& a, double& b, double (*s_red)[4]) {
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { s_red[0][threadIdx.x >> 6] = a; s_red[1][threadIdx.x >> 6] = b; }
  __syncthreads();
  a = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
  b = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
}

__global__ __launch_bounds__(256) void evec_correct_kernel(const c128* T, long ldt, const c128* P, long ldp,
                                                           int m, double small, double tau, c128* X, long ldx,
                                                           c128* D, c128* mu_out) {
  extern __shared__ c128 r_acc[];
  __shared__ double s_red[2][4];
  const int i = blockIdx.x, tid = threadIdx.x;
  const c128 lam = T[i + (long)i * ldt];
  c128* x = X + (long)i * ldx;
  const c128* p = P + (long)i * ldp;
  c128* d = D + (long)i * m;
  {
    double nr = 0, nx = 0;
    for (int j = tid; j < m; j += 256) {
      const c128 xj = (j <= i) ? x[j] : mk<double>(0, 0);
      nr += abs2(p[j] - lam * xj);
      nx += abs2(xj);
    }
    block_sum2(nr, nx, s_red);
    if (nr <= tau * tau * nx) {                 // uniform
      if (tid == 0) mu_out[i] = mk<double>(0, 0);
      return;
    }
  }
  for (int j = tid; j < m; j += 256) r_acc[j] = mk<double>(0, 0);
  __syncthreads();
  c128 mu = mk<double>(0, 0);
  for (int l = m - 1; l >= 0; --l) {
    // every thread forms d_l (the same value) from r_acc[l], final since the last barrier
    const c128 xl = (l <= i) ? x[l] : mk<double>(0, 0);
    const c128 rl = p[l] - lam * xl;
    c128 dl = mk<double>(0, 0);
    if (l == i) {
      mu = cdiv(rl + r_acc[l], xl);
    } else {
      c128 dd = T[l + (long)l * ldt] - lam;
      if (abs2(dd) < small * small) dd = mk<double>(small, 0);
      c128 rhs = mk<double>(0, 0) - (rl + r_acc[l]);
      if (l < i) rhs = rhs + mu * xl;
      dl = cdiv(rhs, dd);
    }
    if (tid == 0) d[l] = dl;
    for (int j = tid; j < l; j += 256) r_acc[j] = r_acc[j] + T[j + (long)l * ldt] * dl;
    __syncthreads();
  }
  // apply if small against x
  double nd = 0, nx = 0;
  for (int j = tid; j < m; j += 256) {
    nd += abs2(d[j]);
    if (j <= i) nx += abs2(x[j]);
  }
  block_sum2(nd, nx, s_red);
  const bool ok = (nd <= 0.01 * nx) && (nd == nd);
  if (ok)
    for (int j = tid; j < m; j += 256) x[j] = x[j] + d[j];
  if (tid == 0) mu_out[i] = ok ? mu : mk<double>(0, 0);
}

int tri_eigvecs_correct(const c128* T, long ldt, int m, const c128* P, long ldp, c128* X, long ldx,
                        c128* D, c128* mu, hipStream_t s) {
  if (m <= 0) return ST_OK;
  std::vector<c128> diag;
  RSRR_TRY(diag_to_host(T, ldt, m, mu, &diag, s));   // mu is written by the kernel below
  double tnorm = 0;
  for (int j = 0; j < m; ++j) tnorm = std::max(tnorm, sqrt(abs2(diag[j])));
  const double small = std::max(tnorm, 1e-300) * 2.220446049250313e-16;
  const size_t shm = (size_t)m * sizeof(c128);
  if (shm > 150 * 1024) return set_error(ST_EINVAL, "eigenvector correction: m=%d too large", m);
  // residuals within 64 u ||T|| are at the rounding level of the Schur form
  const double tau = 64 * 1.1102230246251565e-16 * std::max(tnorm, 1e-300);
  KernelTimer kt("evec_correct", s, 8.0 * (double)m * m * m / 2, 16.0 * (double)m * m * m / 2);
  hipLaunchKernelGGL(evec_correct_kernel, dim3(m), dim3(256), shm, s, T, ldt, P, ldp, m, small, tau, X, ldx,
                     D, mu);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

int eig_general(c128* A, long lda, int m, std::vector<cd>* lam, c128* V, long ldv, Arena& ws,
                hipStream_t s, double refine_above) {
  lam->clear();
  if (m <= 0) return ST_OK;
  if (m > DC_LEAF) return eig_dc(A, lda, m, lam, V, ldv, ws, s, refine_above);
  // ---- Schur form A = Z T Z^H: Householder reduction to Hessenberg form and
  // the QR iteration in one workgroup (in LDS when the matrix fits), on a
  // contiguous copy H of A
  c128 *H = nullptr, *Z = nullptr, *w = nullptr, *X = nullptr;
  c128** pdev = nullptr;
  int* idev = nullptr;
  RSRR_TRY(ws.get<c128>("eg_H", (size_t)m * m, &H));
  RSRR_TRY(ws.get<c128>("eg_Z", (size_t)m * m, &Z));
  RSRR_TRY(ws.get<c128>("eg_w", m, &w));
  RSRR_TRY(ws.get<c128>("eg_X", (size_t)m * m, &X));
  RSRR_TRY(ws.get<c128*>("eg_P", 2, &pdev));
  RSRR_TRY(ws.get<int>("eg_I", 2, &idev));
  RSRR_TRY((convert<double, double>(A, lda, 0, H, m, 0, m, m, 1, s)));
  c128* hp[2] = {H, Z};
  RSRR_HIP(hipMemcpyAsync(pdev, hp, sizeof(hp), hipMemcpyHostToDevice, s));
  RSRR_HIP(hipMemcpyAsync(idev, &m, sizeof(int), hipMemcpyHostToDevice, s));
  RSRR_TRY(leaf_schur_batched(pdev, pdev + 1, idev, 1, idev + 1, s, m));
  int st = 0;
  RSRR_HIP(hipMemcpyAsync(&st, idev + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  if (st < 0) return set_error(ST_ENOTCONV, "Hessenberg QR did not converge (m=%d)", m);
  // ---- eigenvalues and eigenvectors
  std::vector<c128> diag;
  RSRR_TRY(diag_to_host(H, m, m, w, &diag, s));
  double tnorm = 0;
  for (int j = 0; j < m; ++j) tnorm = std::max(tnorm, sqrt(abs2(diag[j])));
  const double small = std::max(tnorm, 1e-300) * 2.220446049250313e-16;
  const size_t shm = (size_t)m * sizeof(c128);
  if (shm > 150 * 1024) return set_error(ST_EINVAL, "eigenvectors: m=%d too large", m);
  KernelTimer kt("trevc", s, 8.0 * (double)m * m * m / 6, 16.0 * (double)m * m * m / 2);
  hipLaunchKernelGGL(trevc_kernel, dim3(m), dim3(256), shm, s, H, (long)m, m, small, X, m);
  RSRR_LAUNCH_CHECK();
  GemmBatch<double> g;                    // V = Z X
  g.M = m; g.N = m; g.K = m;
  g.A = Z; g.lda = m; g.B = X; g.ldb = m; g.C = V; g.ldc = ldv;
  RSRR_TRY(gemm_batched<double>(g, s));
  lam->resize(m);
  for (int j = 0; j < m; ++j) (*lam)[j] = cd(diag[j].re, diag[j].im);
  return ST_OK;
}

}  // namespace rsrr
