// Small kernels of the reduced problem (Alg. 1) and of the final eigenpairs.
#include "driver.h"
#include "reduced.h"

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
