// Alg. 2, Step 3: an orthonormal basis of the sampling matrix S_hat keeping its
// singular directions above delta * sigma_1.
//
// A Gram matrix squares singular values, so one Gram pass resolves sigma_i /
// sigma_1 only down to its own rounding floor (about sqrt(rows u) sigma_1).
// Up to three levels are used (the caller passes the number):
//   level 1: G = S^H S, pivoted (rank-revealing) Cholesky G = P L L^H P^T
//            stopped when the largest remaining pivot drops below
//            1e-14 sigma_1^2 (singular-value ratio 1e-7, above the floor),
//            S1 = S P(:, 1:k1) L11^{-H}, then one more Cholesky-QR pass
//            (CholeskyQR2).
//   level l > 1: R = (I - Q Q^H)^2 S restricted to the columns the previous
//            level left, the same on R^H R stopped at the larger of
//            (delta sigma_1)^2 and its own floor, orthogonalised against the basis so far and
//            CholeskyQR2'd; appended to the basis.
// A level runs only while the basis is below min(rows, cols) and the previous
// level stopped at its floor rather than at delta sigma_1.  sigma_1^2 is the
// largest eigenvalue of G (power iteration).
#include <algorithm>
#include <cmath>

#include "driver.h"
#include "timers.h"

namespace rsrr {

constexpr int PCT = 1024;     // threads of the pivoted-Cholesky panel kernel
constexpr int PBS = 64;       // block size of the triangular solves
constexpr int PCB = 16;       // columns per pivoted-Cholesky panel
constexpr int PMAX = 8192;    // largest Gram matrix (the Schur-complement diagonal lives in LDS)

// One block of the right-looking pivoted Cholesky, in place on G (m x m, both
// triangles stored).  Columns j0 .. j0+jb-1 of L are written to the lower part
// of G.  d holds the diagonal of the current Schur complement (kept in LDS
// while the block is factored), perm the symmetric permutation.  Stops at the
// first pivot <= tol (rank -> *rank).  The pivot is the largest remaining
// diagonal entry (compared through the high word of the double, so within a
// relative 2^-20 of the maximum), found with DPP wave maxima.
__global__ __launch_bounds__(PCT) void pchol_panel_kernel(c128* G, long ldg, int m, int j0, int jb,
                                                          int* perm, double* d, double tol,
                                                          int pivot, int* rank) {
  __shared__ double s_d[PMAX];
  __shared__ unsigned s_val[16];
  __shared__ int s_row[16];
  __shared__ c128 s_lj[PCB];
  __shared__ int s_stop;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (j0 == 0) {
    for (int i = tid; i < m; i += PCT) {
      s_d[i] = G[i + (long)i * ldg].re;
      perm[i] = i;
    }
  } else {
    for (int i = j0 + tid; i < m; i += PCT) s_d[i] = d[i];
  }
  if (tid == 0) s_stop = 0;
  __syncthreads();
  int jdone = jb;
  for (int jj = 0; jj < jb; ++jj) {
    const int j = j0 + jj;
    int p = j;
    double best = s_d[j];
    if (pivot) {
      unsigned bv = 0;
      int brow = -1;
      for (int i = j + tid; i < m; i += PCT) {
        const unsigned v = mag_bits(fmax(s_d[i], 0.0));
        if (brow < 0 || v > bv) { bv = v; brow = i; }
      }
      const unsigned wm = wave_umax(bv);
      const unsigned long long hw = __ballot(brow >= 0 && bv == wm);
      const int wrow = hw ? __builtin_amdgcn_readlane(brow, __ffsll((long long)hw) - 1) : -1;
      if (lane == 0) { s_val[wave] = wm; s_row[wave] = wrow; }
      __syncthreads();
      const unsigned vq = (lane < 16) ? s_val[lane] : 0u;
      const int rq = (lane < 16) ? s_row[lane] : -1;
      const unsigned gm = (unsigned)__builtin_amdgcn_readlane((int)row16_umax_all(vq), 0);
      const unsigned long long hq = __ballot(rq >= 0 && vq == gm);
      p = __builtin_amdgcn_readlane(rq, __ffsll((long long)hq) - 1);
      best = s_d[p];
    }
    if (!(best > tol)) {                       // rank found (uniform decision)
      if (tid == 0) { *rank = j; s_stop = 1; }
      jdone = jj;
      break;
    }
    if (p != j) {
      for (int c = tid; c < m; c += PCT) {     // rows
        const c128 a = G[j + (long)c * ldg];
        G[j + (long)c * ldg] = G[p + (long)c * ldg];
        G[p + (long)c * ldg] = a;
      }
      __syncthreads();
      for (int r = tid; r < m; r += PCT) {     // columns
        const c128 a = G[r + (long)j * ldg];
        G[r + (long)j * ldg] = G[r + (long)p * ldg];
        G[r + (long)p * ldg] = a;
      }
      if (tid == 0) {
        const double t = s_d[j]; s_d[j] = s_d[p]; s_d[p] = t;
        const int q = perm[j]; perm[j] = perm[p]; perm[p] = q;
      }
      __syncthreads();
    }
    const double ljj = sqrt(s_d[j]);
    if (tid < jj) s_lj[tid] = G[j + (long)(j0 + tid) * ldg];
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += PCT) {
      c128 v = G[i + (long)j * ldg];
      for (int l = 0; l < jj; ++l) v = v - mulc(G[i + (long)(j0 + l) * ldg], s_lj[l]);
      v = (1.0 / ljj) * v;
      G[i + (long)j * ldg] = v;
      s_d[i] -= abs2(v);
    }
    if (tid == 0) {
      G[j + (long)j * ldg] = mk<double>(ljj, 0);
      s_d[j] = 0.0;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int i = j0 + tid; i < m; i += PCT) d[i] = s_d[i];
  if (tid == 0 && !s_stop) *rank = j0 + jdone;
}

// Inverses of the diagonal blocks (bs <= 64) of a lower-triangular L, one
// 256-thread workgroup per block, right-looking: step i finishes row i of
// X = L^{-1} (X[i][j] = (delta_ij - acc[i][j]) / L[i][i]) and every later row
// r adds L[r][i] X[i][j] to its accumulators.  Thread t keeps row t / 4,
// columns t % 4 + 4q, in registers; one barrier per step.
__global__ __launch_bounds__(256) void tri_inv_lower_blocks(const c128* L, long ldl, int k, int bs,
                                                            c128* out) {
  __shared__ c128 s[PBS][PBS + 1];     // the block of L; row i becomes row i of X at step i
  __shared__ c128 rd[PBS];
  __shared__ c128 xrow[2][PBS];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int b0 = blk * bs, be = min(bs, k - b0);
  for (int e = tid; e < be * be; e += 256) {
    const int r = e % be, c = e / be;
    s[r][c] = (r >= c) ? L[b0 + r + (long)(b0 + c) * ldl] : mk<double>(0, 0);
  }
  __syncthreads();
  if (tid < be) rd[tid] = crecip(s[tid][tid]);
  const int r = tid >> 2, j0 = tid & 3;
  c128 acc[PBS / 4];
#pragma unroll
  for (int q = 0; q < PBS / 4; ++q) acc[q] = mk<double>(0, 0);
  __syncthreads();
  for (int i = 0; i < be; ++i) {
    const int par = i & 1;
    if (r == i) {
      const c128 d = rd[i];
#pragma unroll
      for (int q = 0; q < PBS / 4; ++q) {
        const int j = j0 + 4 * q;
        if (j <= i) {
          const c128 x = (mk<double>(j == i ? 1.0 : 0.0, 0) - acc[q]) * d;
          xrow[par][j] = x;
          s[i][j] = x;
        }
      }
    }
    __syncthreads();
    if (r > i && r < be) {
      const c128 lri = s[r][i];
#pragma unroll
      for (int q = 0; q < PBS / 4; ++q) {
        if (4 * q > i) break;                   // columns right of i (uniform)
        const int j = j0 + 4 * q;
        if (j <= i) acc[q] = acc[q] + lri * xrow[par][j];
      }
    }
  }
  __syncthreads();
  c128* o = out + (long)blk * bs * bs;
  for (int e = tid; e < bs * bs; e += 256) {
    const int rr = e % bs, c = e / bs;
    o[e] = (rr < be && c < be && rr >= c) ? s[rr][c] : mk<double>(0, 0);
  }
}

// Cholesky of the jb x jb diagonal block at (j0, j0) of G (Hermitian, the
// lower triangle is used), right-looking; L11 overwrites the lower triangle.
// *bad is set to 1 if a pivot is not positive.  Thread t keeps row t / 4,
// columns t % 4 + 4q, in registers; per column k the owners post column k
// (not yet scaled) to LDS, and after one barrier every thread scales by
// 1 / sqrt(a_kk) itself and updates its entries.
__global__ __launch_bounds__(256) void chol_diag_kernel(c128* G, long ldg, int j0, int jb, int* bad) {
  __shared__ c128 lo[PBS][PBS + 1];   // staging of the block, then L
  __shared__ c128 col[2][PBS];
  const int tid = threadIdx.x, r = tid >> 2, c0 = tid & 3;
  c128* B = G + j0 + (long)j0 * ldg;
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e % jb, c = e / jb;
    lo[i][c] = (i >= c) ? B[i + (long)c * ldg] : mk<double>(0, 0);
  }
  __syncthreads();
  c128 a[PBS / 4];
#pragma unroll
  for (int q = 0; q < PBS / 4; ++q) {
    const int j = c0 + 4 * q;
    a[q] = (r < jb && j < jb && r >= j) ? lo[r][j] : mk<double>(0, 0);
  }
  __syncthreads();
  int done = jb;
  for (int k = 0; k < jb; ++k) {
    const int par = k & 1;
    const bool owner = c0 == (k & 3) && r >= k && r < jb;
    if (owner) {
      c128 v = a[0];
#pragma unroll
      for (int q = 1; q < PBS / 4; ++q)
        if (q == (k >> 2)) v = a[q];
      col[par][r] = v;
    }
    __syncthreads();
    const double d = col[par][k].re;
    if (!(d > 0.0)) { done = k; break; }      // same value in every thread: uniform
    const double lkk = sqrt(d), rl = 1.0 / lkk;
    if (owner) lo[r][k] = (r == k) ? mk<double>(lkk, 0) : rl * col[par][r];
    if (r > k && r < jb) {
      const c128 lr = rl * col[par][r];
#pragma unroll
      for (int q = 0; q < PBS / 4; ++q) {
        if (4 * q + 3 <= k) continue;           // columns left of k (uniform)
        const int j = c0 + 4 * q;
        if (j > k && j <= r) a[q] = a[q] - lr * conj(rl * col[par][j]);
      }
    }
  }
  if (done < jb) {
    if (tid == 0) *bad = 1;
    return;
  }
  __syncthreads();
  for (int e = tid; e < jb * jb; e += 256) {
    const int i = e % jb, c = e / jb;
    if (i >= c) B[i + (long)c * ldg] = lo[i][c];
  }
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

__global__ __launch_bounds__(256) void gather_cols_kernel(const c128* S, long lds, const int* perm,
                                                          int rows, int k, c128* out, long ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * k) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  out[i + (long)c * ldo] = S[i + (long)perm[c] * lds];
}

// x <- y / ||y|| (one workgroup), lam[0] <- ||y||
__global__ __launch_bounds__(1024) void normalize_kernel(const c128* y, c128* x, int m, double* lam) {
  __shared__ double red[1024];
  double acc = 0;
  for (int i = threadIdx.x; i < m; i += 1024) acc += abs2(y[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < m; i += 1024) x[i] = inv * y[i];
  if (threadIdx.x == 0) *lam = nrm;
}

__global__ void fill_kernel(c128* x, int m, c128 v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = v;
}

static int gemm_z(int opA, int opB, int M, int N, int K, c128 alpha, const c128* A, long lda,
                  const c128* B, long ldb, c128 beta, c128* C, long ldc, hipStream_t s) {
  GemmBatch<double> g;
  g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.tag = "ortho_gemm";
  return gemm_batched<double>(g, s);
}

__global__ __launch_bounds__(256) void sum_slices_kernel(const c128* W, int S, int M, int N, c128 alpha,
                                                          c128* C, long ldc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  c128 acc = W[e];
  for (int q = 1; q < S; ++q) acc = acc + W[(long)q * M * N + e];
  C[e % M + (e / M) * ldc] = alpha * acc;
}

// C = alpha A^H B (beta 0, one product) with K = the rows of the sample
// matrix.  With few 64x64 output tiles each workgroup would walk the whole K
// while most CUs idle, so the K range is cut into S slices that run as one
// batched product into work space, summed afterwards in slice order.
static int gemm_hk(GemmBatch<double> g, Arena& ws, hipStream_t s) {
  const long tiles = cdivl(g.M, 64) * cdivl(g.N, 64);
  const int S = (int)std::min<long>(256 / std::max<long>(1, tiles), g.K / 1024);
  if (S < 2) return gemm_batched<double>(g, s);
  c128* W = nullptr;
  RSRR_TRY(ws.get<c128>("or_kslices", (size_t)S * g.M * g.N, &W));
  const int K = g.K, Ks = K / S;
  const c128 alpha = g.alpha;
  c128* const C = g.C;
  const long ldc = g.ldc, mn = (long)g.M * g.N;
  const c128* A = (const c128*)g.A;
  const c128* B = g.B;
  g.alpha = mk<double>(1, 0);
  g.C = W; g.ldc = g.M; g.sC = mn;
  g.K = Ks; g.sA = Ks; g.sB = Ks; g.batch = S - 1;     // rows [q Ks, (q+1) Ks) of A and B
  RSRR_TRY(gemm_batched<double>(g, s));
  g.A = A + (long)(S - 1) * Ks; g.B = B + (long)(S - 1) * Ks; g.C = W + (S - 1) * mn;
  g.K = K - (S - 1) * Ks; g.batch = 1;
  RSRR_TRY(gemm_batched<double>(g, s));
  hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)cdivl(mn, 256)), dim3(256), 0, s, W, S, g.M, g.N, alpha, C,
                     ldc);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// C = A^H B (M x N, K = rows)
static int gemm_ct(int M, int N, int rows, const c128* A, long lda, const c128* B, long ldb, c128* C, long ldc,
                   Arena& ws, hipStream_t s) {
  GemmBatch<double> g;
  g.opA = OP_C; g.opB = OP_N; g.M = M; g.N = N; g.K = rows;
  g.alpha = mk<double>(1, 0); g.beta = mk<double>(0, 0);
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.tag = "ortho_gemm";
  return gemm_hk(g, ws, s);
}

// G = X^H X (cols x cols, leading dim ldg): the tiles on and below the
// diagonal, mirrored above it
static int gram_z(int cols, int rows, const c128* X, long ldx, c128* G, long ldg, Arena& ws, hipStream_t s) {
  GemmBatch<double> g;
  g.opA = OP_C; g.opB = OP_N; g.M = cols; g.N = cols; g.K = rows;
  g.alpha = mk<double>(1, 0); g.beta = mk<double>(0, 0);
  g.A = X; g.lda = ldx; g.B = X; g.ldb = ldx; g.C = G; g.ldc = ldg;
  g.herm = true;
  g.tag = "ortho_gemm";
  return gemm_hk(g, ws, s);
}

static const c128 ONE = {1, 0}, ZERO = {0, 0}, MONE = {-1, 0};

// Largest eigenvalue of the Hermitian PSD m x m matrix G (power iteration).
static int power_lambda(const c128* G, long ldg, int m, Arena& ws, hipStream_t s, double* lam) {
  c128 *x = nullptr, *y = nullptr;
  double* l = nullptr;
  RSRR_TRY(ws.get<c128>("pw_x", m, &x));
  RSRR_TRY(ws.get<c128>("pw_y", m, &y));
  RSRR_TRY(ws.get<double>("pw_l", 1, &l));
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)cdivl(m, 256)), dim3(256), 0, s, x, m,
                     mk<double>(1.0 / sqrt((double)m), 0));
  RSRR_LAUNCH_CHECK();
  for (int it = 0; it < 12; ++it) {
    RSRR_TRY(gemm_z(OP_N, OP_N, m, 1, m, ONE, G, ldg, x, m, ZERO, y, m, s));
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, y, x, m, l);
    RSRR_LAUNCH_CHECK();
  }
  RSRR_HIP(hipMemcpyAsync(lam, l, sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

__global__ __launch_bounds__(1024) void max_diag_kernel(const c128* G, long ldg, int m, double* out) {
  __shared__ double red[1024];
  double b = 0;
  for (int i = threadIdx.x; i < m; i += 1024) b = fmax(b, G[i + (long)i * ldg].re);
  red[threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

static int max_real_diag(const c128* G, long ldg, int m, Arena& ws, hipStream_t s, double* out) {
  double* d = nullptr;
  RSRR_TRY(ws.get<double>("md_out", 1, &d));
  hipLaunchKernelGGL(max_diag_kernel, dim3(1), dim3(1024), 0, s, G, ldg, m, d);
  RSRR_LAUNCH_CHECK();
  RSRR_HIP(hipMemcpyAsync(out, d, sizeof(double), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  return ST_OK;
}

// Blocked pivoted Cholesky of G (m x m, overwritten; L in the lower part).
static int pchol(c128* G, long ldg, int m, int maxrank, double tol, bool pivot, int* perm,
                 Arena& ws, hipStream_t s, int* rank_out) {
  double* d = nullptr;
  int* rk = nullptr;
  RSRR_TRY(ws.get<double>("pc_d", m, &d));
  RSRR_TRY(ws.get<int>("pc_rank", 1, &rk));
  if (m > PMAX) return set_error(ST_EINVAL, "pivoted Cholesky: Gram matrix of order %d > %d", m, PMAX);
  int rank = 0;
  for (int j0 = 0; j0 < maxrank; j0 += PCB) {
    const int jb = std::min(PCB, maxrank - j0);
    KernelTimer kt("pchol_panel", s, 8.0 * (double)m * jb * jb / 2, 16.0 * 4 * (double)m * jb,
                   "pchol_panel_kernel");
    hipLaunchKernelGGL(pchol_panel_kernel, dim3(1), dim3(PCT), 0, s, G, ldg, m, j0, jb, perm, d,
                       tol, pivot ? 1 : 0, rk);
    RSRR_LAUNCH_CHECK();
    RSRR_HIP(hipMemcpyAsync(&rank, rk, sizeof(int), hipMemcpyDeviceToHost, s));
    RSRR_HIP(hipStreamSynchronize(s));
    if (rank < j0 + jb) break;
    const int t = j0 + jb, rest = m - t;
    if (rest > 0 && t < maxrank)
      RSRR_TRY(gemm_z(OP_N, OP_C, rest, rest, jb, MONE, G + t + (long)j0 * ldg, ldg,
                      G + t + (long)j0 * ldg, ldg, ONE, G + t + (long)t * ldg, ldg, s));
  }
  *rank_out = rank;
  return ST_OK;
}

// X (rows x k) <- X L^{-H} with L (k x k) lower triangular (the Cholesky factor).
static int trsm_right_lh(const c128* L, long ldl, int k, c128* X, long ldx, int rows, Arena& ws,
                         hipStream_t s) {
  const int nblk = (k + PBS - 1) / PBS;
  c128* inv = nullptr;
  c128* tmp = nullptr;
  RSRR_TRY(ws.get<c128>("tr_inv", (size_t)nblk * PBS * PBS, &inv));
  RSRR_TRY(ws.get<c128>("tr_tmp", (size_t)rows * PBS, &tmp));
  hipLaunchKernelGGL(tri_inv_lower_blocks, dim3(nblk), dim3(256), 0, s, L, ldl, k, PBS, inv);
  RSRR_LAUNCH_CHECK();
  // right-looking over groups of TRSM_G column blocks: inside a group each
  // block is solved after the group's earlier blocks are subtracted, then the
  // columns right of the group are updated with one product (K = group width)
  constexpr int TRSM_G = 4;
  for (int g0 = 0; g0 < nblk; g0 += TRSM_G) {
    const int g1 = std::min(nblk, g0 + TRSM_G);
    const int c0 = g0 * PBS, c1 = std::min(k, g1 * PBS);
    for (int b = g0; b < g1; ++b) {
      const int j = b * PBS, be = std::min(PBS, k - j);
      if (j > c0)   // X_b -= X[:, c0:j] (L[b, c0:j])^H
        RSRR_TRY(gemm_z(OP_N, OP_C, rows, be, j - c0, MONE, X + (long)c0 * ldx, ldx, L + j + (long)c0 * ldl, ldl,
                        ONE, X + (long)j * ldx, ldx, s));
      // X_b <- X_b inv(L_bb)^H
      RSRR_TRY(gemm_z(OP_N, OP_C, rows, be, be, ONE, X + (long)j * ldx, ldx, inv + (long)b * PBS * PBS,
                      PBS, ZERO, tmp, rows, s));
      RSRR_TRY((convert<double, double>(tmp, rows, 0, X + (long)j * ldx, ldx, 0, rows, be, 1, s)));
    }
    if (c1 < k)     // X[:, c1:] -= X[:, c0:c1] (L[c1:, c0:c1])^H
      RSRR_TRY(gemm_z(OP_N, OP_C, rows, k - c1, c1 - c0, MONE, X + (long)c0 * ldx, ldx, L + c1 + (long)c0 * ldl,
                      ldl, ONE, X + (long)c1 * ldx, ldx, s));
  }
  return ST_OK;
}

// Unpivoted blocked Cholesky of the Hermitian positive definite G (m x m, L
// in the lower triangle): per block of PBS columns the diagonal block in LDS,
// L21 = G21 L11^{-H} and G22 -= L21 L21^H as matrix-core GEMMs.
static int chol_blocked(c128* G, long ldg, int m, Arena& ws, hipStream_t s, bool* ok) {
  int* bad = nullptr;
  c128 *inv = nullptr, *tmp = nullptr;
  RSRR_TRY(ws.get<int>("ch_bad", 1, &bad));
  RSRR_TRY(ws.get<c128>("ch_inv", (size_t)PBS * PBS, &inv));
  RSRR_TRY(ws.get<c128>("ch_tmp", (size_t)std::max(1, m) * PBS, &tmp));
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, bad, 0);
  RSRR_LAUNCH_CHECK();
  for (int j0 = 0; j0 < m; j0 += PBS) {
    const int jb = std::min(PBS, m - j0);
    {
      KernelTimer kt("chol_diag", s, 8.0 * (double)jb * jb * jb / 6, 32.0 * (double)jb * jb, "chol_diag_kernel");
      hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, G, ldg, j0, jb, bad);
      RSRR_LAUNCH_CHECK();
    }
    const int rest = m - j0 - jb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(tri_inv_lower_blocks, dim3(1), dim3(256), 0, s, G + j0 + (long)j0 * ldg, ldg, jb, PBS, inv);
    RSRR_LAUNCH_CHECK();
    c128* L21 = G + (j0 + jb) + (long)j0 * ldg;
    RSRR_TRY(gemm_z(OP_N, OP_C, rest, jb, jb, ONE, L21, ldg, inv, PBS, ZERO, tmp, rest, s));
    RSRR_TRY((convert<double, double>(tmp, rest, 0, L21, ldg, 0, rest, jb, 1, s)));
    RSRR_TRY(gemm_z(OP_N, OP_C, rest, rest, jb, MONE, L21, ldg, L21, ldg, ONE, G + (j0 + jb) + (long)(j0 + jb) * ldg,
                    ldg, s));
  }
  int hb = 0;
  RSRR_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  RSRR_HIP(hipStreamSynchronize(s));
  *ok = (hb == 0);
  return ST_OK;
}

// One Cholesky-QR pass on X (rows x k, in place): X <- X chol(X^H X)^{-H}.
static int cholqr_pass(c128* X, long ldx, int rows, int k, Arena& ws, hipStream_t s, bool* ok) {
  c128* G = nullptr;
  int* perm = nullptr;
  RSRR_TRY(ws.get<c128>("cq_G", (size_t)k * k, &G));
  RSRR_TRY(ws.get<int>("cq_perm", k, &perm));
  (void)perm;
  RSRR_TRY(gram_z(k, rows, X, ldx, G, k, ws, s));
  RSRR_TRY(chol_blocked(G, k, k, ws, s, ok));
  if (!*ok) return ST_OK;
  return trsm_right_lh(G, k, k, X, ldx, rows, ws, s);
}

int cholqr(c128* X, long ldx, int rows, int k, Arena& ws, hipStream_t s, bool* ok) {
  return cholqr_pass(X, ldx, rows, k, ws, s, ok);
}

// Orthonormal basis (rows x rank, into Q) of the span of the columns of X
// (rows x cols) whose rank is known: pivoted Cholesky of X^H X stopped at
// `rank`, the selected columns times L11^{-H}, then one more Cholesky-QR pass.
int basis_of_columns(const c128* X, long ldx, int rows, int cols, int rank, c128* Q, long ldq,
                     Arena& ws, hipStream_t s) {
  if (rank <= 0) return ST_OK;
  c128* G = nullptr;
  int* perm = nullptr;
  RSRR_TRY(ws.get<c128>("bc_G", (size_t)cols * cols, &G));
  RSRR_TRY(ws.get<int>("bc_perm", cols, &perm));
  RSRR_TRY(gram_z(cols, rows, X, ldx, G, cols, ws, s));
  int r = 0;
  RSRR_TRY(pchol(G, cols, cols, rank, 0.0, true, perm, ws, s, &r));
  if (r < rank) return set_error(ST_ENOTCONV, "basis_of_columns: rank %d < %d", r, rank);
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)cdivl((long)rows * rank, 256)), dim3(256), 0,
                     s, X, ldx, perm, rows, rank, Q, ldq);
  RSRR_LAUNCH_CHECK();
  RSRR_TRY(trsm_right_lh(G, cols, rank, Q, ldq, rows, ws, s));
  bool ok = true;
  RSRR_TRY(cholqr_pass(Q, ldq, rows, rank, ws, s, &ok));
  if (!ok) return set_error(ST_ENOTCONV, "basis_of_columns: Cholesky-QR pass broke down");
  return ST_OK;
}

int ortho_impl(int rows, int cols, const c128* S, long lds, double delta, c128* Q, long ldq,
               int* k_S, Arena& ws, hipStream_t s, int levels) {
  const int m = cols, kmax = std::min(rows, cols);
  c128* G = nullptr;
  int* perm = nullptr;
  RSRR_TRY(ws.get<c128>("or_G", (size_t)m * m, &G));
  RSRR_TRY(ws.get<int>("or_perm", m, &perm));
  // ---- level 1
  RSRR_TRY(gram_z(m, rows, S, lds, G, m, ws, s));
  double lam1 = 0;
  RSRR_TRY(power_lambda(G, m, m, ws, s, &lam1));
  if (!(lam1 > 0)) { *k_S = 0; return ST_OK; }
  const double tau1 = 1e-14;           // level-1 pivots: sigma ratio >= ~1e-7
  int k1 = 0;
  RSRR_TRY(pchol(G, m, m, kmax, tau1 * lam1, true, perm, ws, s, &k1));
  if (k1 == 0) { *k_S = 0; return ST_OK; }
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)cdivl((long)rows * k1, 256)), dim3(256), 0,
                     s, S, lds, perm, rows, k1, Q, ldq);
  RSRR_LAUNCH_CHECK();
  RSRR_TRY(trsm_right_lh(G, m, k1, Q, ldq, rows, ws, s));
  bool ok = true;
  RSRR_TRY(cholqr_pass(Q, ldq, rows, k1, ws, s, &ok));
  if (!ok) return set_error(ST_ENOTCONV, "orthonormalize: second Cholesky-QR pass broke down");
  int kS = k1;
  // ---- levels 2, 3, ...: directions of S outside the span found so far,
  // above delta * sigma_1.  Each level's Gram matrix resolves singular values
  // down to its own rounding floor (rows * u times its largest column norm
  // squared).  A level whose floor lies above delta sigma_1 leaves directions
  // for the next one, which starts from that floor; a level whose threshold
  // was delta sigma_1 itself is the last.
  if (kS < kmax && levels > 1) {
    c128 *Rm = nullptr, *Cc = nullptr;
    RSRR_TRY(ws.get<c128>("or_R", (size_t)rows * m, &Rm));
    RSRR_TRY(ws.get<c128>("or_C", (size_t)kmax * m, &Cc));
    // R = S - Q Q^H S (two passes); later levels remove only the columns
    // they add, since R is already orthogonal to the earlier ones
    RSRR_TRY((convert<double, double>(S, lds, 0, Rm, rows, 0, rows, m, 1, s)));
    int k0 = 0, kn = kS;
    for (int level = 2; level <= levels && kS < kmax; ++level) {
      for (int pass = 0; pass < 2; ++pass) {
        RSRR_TRY(gemm_ct(kn, m, rows, Q + (long)k0 * ldq, ldq, Rm, rows, Cc, kn, ws, s));
        RSRR_TRY(gemm_z(OP_N, OP_N, rows, m, kn, MONE, Q + (long)k0 * ldq, ldq, Cc, kn, ONE, Rm, rows, s));
      }
      RSRR_TRY(gram_z(m, rows, Rm, rows, G, m, ws, s));
      // stop at (delta sigma_1)^2, but not below the rounding floor of the Gram
      // matrix of R: pivots under rows * u * max_i ||R_i||^2 are noise
      double dmax = 0;
      RSRR_TRY(max_real_diag(G, m, m, ws, s, &dmax));
      const double floor2 = rows * 1.1102230246251565e-16 * dmax;
      const double tau2 = std::max(delta * delta * lam1, floor2);
      int k2 = 0;
      RSRR_TRY(pchol(G, m, m, kmax - kS, tau2, true, perm, ws, s, &k2));
      if (k2 == 0) break;
      c128* Q2 = Q + (long)kS * ldq;
      hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)cdivl((long)rows * k2, 256)), dim3(256),
                         0, s, Rm, rows, perm, rows, k2, Q2, ldq);
      RSRR_LAUNCH_CHECK();
      RSRR_TRY(trsm_right_lh(G, m, k2, Q2, ldq, rows, ws, s));
      for (int pass = 0; pass < 2; ++pass) {
        RSRR_TRY(gemm_ct(kS, k2, rows, Q, ldq, Q2, ldq, Cc, kS, ws, s));
        RSRR_TRY(gemm_z(OP_N, OP_N, rows, k2, kS, MONE, Q, ldq, Cc, kS, ONE, Q2, ldq, s));
        bool ok2 = true;
        RSRR_TRY(cholqr_pass(Q2, ldq, rows, k2, ws, s, &ok2));
        if (!ok2) { k2 = 0; break; }
      }
      if (k2 == 0) break;
      k0 = kS;
      kn = k2;
      kS += k2;
      if (floor2 <= delta * delta * lam1) break;
    }
  }
  RSRR_HIP(hipStreamSynchronize(s));
  *k_S = kS;
  return ST_OK;
}

}  // namespace rsrr
