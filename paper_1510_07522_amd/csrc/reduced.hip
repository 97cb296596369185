// Small kernels of the reduced problem (Alg. 1) and of the final eigenpairs.
#include "driver.h"
#include "reduced.h"
#include "timers.h"

namespace rsrr {

// out_b = in_b^T for batch square blocks (k x k, ld k, stride k*k)
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const c128* in, c128* out, int k) {
  __shared__ c128 t[32][33];
  const int b = blockIdx.z;
  const long kk = (long)k * k;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = x0 + tx, j = y0 + r;
    if (i < k && j < k) t[r][tx] = in[b * kk + i + (long)j * k];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = y0 + tx, j = x0 + r;      // out[i][j] = in[j][i]
    if (i < k && j < k) out[b * kk + i + (long)j * k] = t[tx][r];
  }
}

int transpose_blocks(const c128* in, c128* out, int k, int batch, hipStream_t s) {
  if (k <= 0 || batch <= 0) return ST_OK;
  dim3 grid((unsigned)cdivl(k, 32), (unsigned)cdivl(k, 32), (unsigned)batch);
  hipLaunchKernelGGL(transpose_blocks_kernel, grid, dim3(256), 0, s, in, out, k);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// H[bi*k + i][bj*k + j] = A_{bi+bj+shift}[i][j]   (H is (K k) x (K k))
__global__ __launch_bounds__(256) void hankel_kernel(const c128* Amom, int k, int K, int shift,
                                                     c128* H, long ldh) {
  const long M = (long)K * k;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int r = (int)(e % M), c = (int)(e / M);
  const int bi = r / k, i = r % k, bj = c / k, j = c % k;
  H[r + (long)c * ldh] = Amom[(long)(bi + bj + shift) * k * k + i + (long)j * k];
}

int build_hankel(const c128* Amom, int k, int K, int shift, c128* H, long ldh, hipStream_t s) {
  const long M = (long)K * k;
  hipLaunchKernelGGL(hankel_kernel, dim3((unsigned)cdivl(M * M, 256)), dim3(256), 0, s, Amom, k, K,
                     shift, H, ldh);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// partial[b * nchunk + ch] = sum over the chunk of X_b[e] * Y_b[e]
__global__ __launch_bounds__(256) void dot_partial_kernel(const c128* X, const c128* Y, long len,
                                                          long chunk, int nchunk, c128* partial) {
  __shared__ double re_[256], im_[256];
  const int b = blockIdx.y, ch = blockIdx.x;
  const long e0 = (long)ch * chunk, e1 = min(len, e0 + chunk);
  double ar = 0, ai = 0;
  for (long e = e0 + threadIdx.x; e < e1; e += 256) {
    const c128 t = X[(long)b * len + e] * Y[(long)b * len + e];
    ar += t.re;
    ai += t.im;
  }
  re_[threadIdx.x] = ar;
  im_[threadIdx.x] = ai;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) { re_[threadIdx.x] += re_[threadIdx.x + o]; im_[threadIdx.x] += im_[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)b * nchunk + ch] = mk<double>(re_[0], im_[0]);
}

int dot_partials(const c128* X, const c128* Y, long len, int batch, int nchunk, c128* partial,
                 hipStream_t s) {
  const long chunk = cdivl(len, nchunk);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nchunk, batch), dim3(256), 0, s, X, Y, len, chunk,
                     nchunk, partial);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// Moments and winding partials in one pass over the inverses.  Each thread
// takes MWE elements (consecutive threads on consecutive elements) and runs
// over the nodes in order: the P moment sums of its elements stay in
// registers; the J products X_m[e] BT_k[e] are summed over the wave by a
// fixed butterfly and the four wave sums of node m are added in wave order at
// the end.  Block partials go to Dpart[blk][m][k].
constexpr int MWE = 4, MWB = 256 * MWE;

template <int P, int JJ>
__global__ __launch_bounds__(256) void moments_wind_kernel(const c128* X, long kk, int cnt, const c128* cw,
                                                           const c128* BT, c128* A, int accumulate,
                                                           c128* Dpart, int cmax) {
  extern __shared__ c128 s_w[];          // [4][cmax][JJ] wave sums
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long e0 = (long)blockIdx.x * MWB + tid;
  c128 acc[MWE][P], bt[MWE][JJ];
#pragma unroll
  for (int i = 0; i < MWE; ++i) {
    const long e = e0 + 256L * i;
#pragma unroll
    for (int p = 0; p < P; ++p) acc[i][p] = mk<double>(0, 0);
#pragma unroll
    for (int k = 0; k < JJ; ++k) bt[i][k] = e < kk ? BT[e + (long)k * kk] : mk<double>(0, 0);
  }
  for (int m = 0; m < cnt; ++m) {
    c128 x[MWE];
#pragma unroll
    for (int i = 0; i < MWE; ++i) {
      const long e = e0 + 256L * i;
      x[i] = e < kk ? X[(long)m * kk + e] : mk<double>(0, 0);
    }
    c128 w[P];
#pragma unroll
    for (int p = 0; p < P; ++p) w[p] = cw[m + (long)p * cnt];
    c128 d[JJ];
#pragma unroll
    for (int k = 0; k < JJ; ++k) d[k] = mk<double>(0, 0);
#pragma unroll
    for (int i = 0; i < MWE; ++i) {
#pragma unroll
      for (int p = 0; p < P; ++p) acc[i][p] = acc[i][p] + x[i] * w[p];
#pragma unroll
      for (int k = 0; k < JJ; ++k) d[k] = d[k] + x[i] * bt[i][k];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int k = 0; k < JJ; ++k) {
        d[k].re += __shfl_xor(d[k].re, off);
        d[k].im += __shfl_xor(d[k].im, off);
      }
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < JJ; ++k) s_w[((long)wave * cmax + m) * JJ + k] = d[k];
  }
#pragma unroll
  for (int i = 0; i < MWE; ++i) {
    const long e = e0 + 256L * i;
    if (e < kk)
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const long o = e + (long)p * kk;
        A[o] = accumulate ? A[o] + acc[i][p] : acc[i][p];
      }
  }
  __syncthreads();
  c128* out = Dpart + (long)blockIdx.x * cnt * JJ;
  for (int o = tid; o < cnt * JJ; o += 256) {
    const int m = o / JJ, k = o % JJ;
    c128 v = s_w[((long)0 * cmax + m) * JJ + k];
#pragma unroll
    for (int q = 1; q < 4; ++q) v = v + s_w[((long)q * cmax + m) * JJ + k];
    out[o] = v;
  }
}

// D[o] = sum over blocks b (in order, per thread then a fixed tree) of Dpart[b][o]
__global__ __launch_bounds__(256) void sum_parts_kernel(const c128* Dpart, int nblk, int ncol, c128* D) {
  __shared__ double re_[256], im_[256];
  const int o = blockIdx.x;
  double ar = 0, ai = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    const c128 v = Dpart[(long)b * ncol + o];
    ar += v.re;
    ai += v.im;
  }
  re_[threadIdx.x] = ar;
  im_[threadIdx.x] = ai;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { re_[threadIdx.x] += re_[threadIdx.x + h]; im_[threadIdx.x] += im_[threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) D[o] = mk<double>(re_[0], im_[0]);
}

static_assert(MWB == MOMENTS_BLOCK, "moments block of the workspace arithmetic");

template <int P, int JJ>
static int launch_mw(const c128* X, long kk, int cnt, const c128* cw, const c128* BT, c128* A, bool accumulate,
                     c128* Dpart, hipStream_t s) {
  const long nblk = cdivl(kk, MWB);
  const size_t lds = (size_t)4 * cnt * JJ * sizeof(c128);
  if (lds > 60 * 1024) return set_error(ST_EINVAL, "moments: %d nodes per batch exceed the LDS of one pass", cnt);
  KernelTimer kt("reduced_moments", s, 8.0 * (double)kk * cnt * (P + JJ), 16.0 * (double)kk * (cnt + JJ + P),
                 "moments_wind_kernel");
  hipLaunchKernelGGL((moments_wind_kernel<P, JJ>), dim3((unsigned)nblk), dim3(256), lds, s, X, kk, cnt, cw, BT, A,
                     accumulate ? 1 : 0, Dpart, cnt);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

int moments_wind(const c128* X, long kk, int cnt, const c128* cw, int P, const c128* BT, int J, c128* A,
                 bool accumulate, c128* Dpart, c128* D, hipStream_t s) {
  if (kk <= 0 || cnt <= 0) return ST_OK;
  int st = ST_OK;
  // instantiations: P in {2, 4, 6, 8}, J in 1..4
#define RSRR_MW(PP, JV) \
  if (P == PP && J == JV) st = launch_mw<PP, JV>(X, kk, cnt, cw, BT, A, accumulate, Dpart, s); else
#define RSRR_MW_J(PP) RSRR_MW(PP, 1) RSRR_MW(PP, 2) RSRR_MW(PP, 3) RSRR_MW(PP, 4)
  RSRR_MW_J(2) RSRR_MW_J(4) RSRR_MW_J(6) RSRR_MW_J(8)
  return set_error(ST_EINVAL, "moments: P=%d, J=%d outside the one-pass kernel", P, J);
#undef RSRR_MW_J
#undef RSRR_MW
  if (st < 0) return st;
  const long nblk = cdivl(kk, MWB);
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)(cnt * J)), dim3(256), 0, s, Dpart, (int)nblk, cnt * J, D);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// out[:, j] = in[:, perm ? perm[j] : j] * (scale ? scale[j] : 1)
__global__ __launch_bounds__(256) void gather_scale_kernel(const c128* in, long ldi, const int* perm,
                                                           const double* scale, int rows, int ncol,
                                                           c128* out, long ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * ncol) return;
  const int r = (int)(e % rows), j = (int)(e / rows);
  c128 v = in[r + (long)(perm ? perm[j] : j) * ldi];
  if (scale) v = scale[j] * v;
  out[r + (long)j * ldo] = v;
}

int gather_scale_cols(const c128* in, long ldi, const int* perm, const double* scale, int rows,
                      int ncol, c128* out, long ldo, hipStream_t s) {
  const long cnt = (long)rows * ncol;
  if (cnt <= 0) return ST_OK;
  hipLaunchKernelGGL(gather_scale_kernel, dim3((unsigned)cdivl(cnt, 256)), dim3(256), 0, s, in, ldi,
                     perm, scale, rows, ncol, out, ldo);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// Unit 2-norm, entry of largest modulus (first on ties) real and positive.
__global__ __launch_bounds__(256) void normalize_cols_kernel(c128* V, long ldv, int rows) {
  __shared__ double s_n[256], s_m[256];
  __shared__ int s_i[256];
  const int j = blockIdx.x;
  c128* v = V + (long)j * ldv;
  double nrm = 0, best = -1;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < rows; r += 256) {
    const double a = abs2(v[r]);
    nrm += a;
    if (a > best) { best = a; bi = r; }
  }
  s_n[threadIdx.x] = nrm;
  s_m[threadIdx.x] = best;
  s_i[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s_n[threadIdx.x] += s_n[threadIdx.x + o];
      const double ob = s_m[threadIdx.x + o];
      const int oi = s_i[threadIdx.x + o];
      if (ob > s_m[threadIdx.x] || (ob == s_m[threadIdx.x] && oi < s_i[threadIdx.x])) {
        s_m[threadIdx.x] = ob;
        s_i[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double n = sqrt(s_n[0]);
  const c128 big = v[s_i[0]];
  const double ab = sqrt(abs2(big));
  if (!(n > 0) || !(ab > 0)) return;
  // multiply by conj(big)/|big| / n
  const c128 f = mk<double>(big.re / (ab * n), -big.im / (ab * n));
  __syncthreads();
  for (int r = threadIdx.x; r < rows; r += 256) v[r] = v[r] * f;
}

int normalize_cols(c128* V, long ldv, int rows, int ncol, hipStream_t s) {
  if (ncol <= 0) return ST_OK;
  hipLaunchKernelGGL(normalize_cols_kernel, dim3(ncol), dim3(256), 0, s, V, ldv, rows);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

__global__ void fill_c128_kernel(c128* x, long n, c128 v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

int fill_c128(c128* x, long n, c128 v, hipStream_t s) {
  if (n <= 0) return ST_OK;
  hipLaunchKernelGGL(fill_c128_kernel, dim3((unsigned)cdivl(n, 256)), dim3(256), 0, s, x, n, v);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

}  // namespace rsrr
