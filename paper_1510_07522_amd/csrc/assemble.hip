// Assembly of T(z_j) at many nodes, BEM kernels, and small elementwise kernels.
#include <algorithm>

#include "bem.h"
#include "common.h"
#include "kernels.h"
#include "timers.h"

namespace rsrr {

constexpr int MAXJ = 16;
struct CoeffArgs {
  int n, J, nz;
  int kinds[MAXJ];
  const void* mats[MAXJ];
};

// One thread per matrix entry; every node j reuses the J coefficient values.
// Sums are formed in fp64 and rounded once to the output precision.
template <typename R>
__global__ __launch_bounds__(256) void assemble_coeff_kernel(CoeffArgs ca, const c128* f,
                                                             cplx<R>* T, long ldt, long sT) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)ca.n * ca.n;
  if (e >= nn) return;
  const int i = (int)(e % ca.n), c = (int)(e / ca.n);
  c128 v[MAXJ];
  bool nz[MAXJ];
#pragma unroll
  for (int k = 0; k < MAXJ; ++k) {
    v[k] = mk<double>(0, 0);
    nz[k] = false;
    if (k < ca.J) {
      switch (ca.kinds[k]) {
        case 0: if (i == c) { v[k] = mk<double>(1, 0); nz[k] = true; } break;
        case 1: if (i == c) { v[k] = ((const c128*)ca.mats[k])[i]; nz[k] = true; } break;
        case 2: v[k] = mk<double>(((const double*)ca.mats[k])[e], 0); nz[k] = true; break;
        default: v[k] = ((const c128*)ca.mats[k])[e]; nz[k] = true; break;
      }
    }
  }
  const long out = (long)i + (long)c * ldt;
  for (int j = 0; j < ca.nz; ++j) {
    c128 s = mk<double>(0, 0);
#pragma unroll
    for (int k = 0; k < MAXJ; ++k)
      if (k < ca.J && nz[k]) s = s + f[(long)j * ca.J + k] * v[k];
    T[out + (long)j * sT] = ccast<R>(s);
  }
}

template <typename R>
int assemble_coeff(const CoeffSet& cs, int nz, const c128* f_dev, cplx<R>* T, long ldt, long sT,
                   hipStream_t s) {
  if (cs.J > MAXJ) return set_error(ST_EINVAL, "assemble: J=%d > %d", cs.J, MAXJ);
  if (nz <= 0 || cs.n <= 0) return ST_OK;
  CoeffArgs ca;
  ca.n = cs.n; ca.J = cs.J; ca.nz = nz;
  for (int k = 0; k < MAXJ; ++k) {
    ca.kinds[k] = k < cs.J ? cs.kinds_host[k] : 0;
    ca.mats[k] = k < cs.J ? cs.mats[k] : nullptr;
  }
  const long nn = (long)cs.n * cs.n;
  KernelTimer kt("assemble_coeff", s, 8.0 * nn * nz * cs.J, (double)nn * nz * sizeof(cplx<R>));
  hipLaunchKernelGGL((assemble_coeff_kernel<R>), dim3((unsigned)cdivl(nn, 256)), dim3(256), 0, s,
                     ca, f_dev, T, ldt, sT);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}
template int assemble_coeff<double>(const CoeffSet&, int, const c128*, c128*, long, long, hipStream_t);
template int assemble_coeff<float>(const CoeffSet&, int, const c128*, c64*, long, long, hipStream_t);

// ------------------------------------------------------------------- BEM
template <typename R>
__global__ __launch_bounds__(256) void assemble_bem_kernel(int n, const double* xyz, double h,
                                                           int nz, const c128* z, cplx<R>* T,
                                                           long ldt, long sT) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), c = (int)(e / n);
  const long out = (long)i + (long)c * ldt;
  if (i == c) {
    for (int j = 0; j < nz; ++j) {
      const c128 zj = z[j];
      T[out + (long)j * sT] = ccast<R>(mk<double>(-zj.im * RSRR_INV4PI + 0.5 / h, zj.re * RSRR_INV4PI));
    }
    return;
  }
  const double dx = xyz[3 * i] - xyz[3 * c], dy = xyz[3 * i + 1] - xyz[3 * c + 1],
               dz = xyz[3 * i + 2] - xyz[3 * c + 2];
  const R r = (R)sqrt(dx * dx + dy * dy + dz * dz);
  for (int j = 0; j < nz; ++j) {
    const c128 zj = z[j];
    T[out + (long)j * sT] = bem_entry<R>(r, (R)zj.re, (R)zj.im);
  }
}

template <typename R>
int assemble_bem(int n, const double* xyz, double h, int nz, const c128* z_dev, cplx<R>* T,
                 long ldt, long sT, hipStream_t s) {
  if (nz <= 0 || n <= 0) return ST_OK;
  const long nn = (long)n * n;
  KernelTimer kt("assemble_bem", s, 0.0, (double)nn * nz * sizeof(cplx<R>));
  hipLaunchKernelGGL((assemble_bem_kernel<R>), dim3((unsigned)cdivl(nn, 256)), dim3(256), 0, s, n,
                     xyz, h, nz, z_dev, T, ldt, sT);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}
template int assemble_bem<double>(int, const double*, double, int, const c128*, c128*, long, long, hipStream_t);
template int assemble_bem<float>(int, const double*, double, int, const c128*, c64*, long, long, hipStream_t);

// ||T(z_j)||_F^2 of the BEM matrix.  |T_ic| depends on the distance of points i
// and c alone, so each workgroup sums the entries right of the diagonal in rows
// x and n-1-x (n-1 entries together), doubled, plus their diagonal entries
// (the same value in every row); the pairs' partial sums are then added in a
// fixed order per node (no float atomics: results are bit-reproducible).
__global__ __launch_bounds__(256) void bem_fro2_partial(int n, const double* xyz, double h, int nz,
                                                        const c128* z, double* partial) {
  __shared__ double red[4];
  const int x = blockIdx.x, j = blockIdx.y, tid = threadIdx.x;
  const int np = (n + 1) / 2, i1 = x, i2 = n - 1 - x;
  const int len1 = n - 1 - i1, len = i2 != i1 ? len1 + (n - 1 - i2) : len1;
  const c128 zj = z[j];
  double acc = 0.0;
  for (int t = tid; t < len; t += 256) {
    const int i = t < len1 ? i1 : i2;
    const int c = t < len1 ? i1 + 1 + t : i2 + 1 + (t - len1);
    const double dx = xyz[3 * i] - xyz[3 * c], dy = xyz[3 * i + 1] - xyz[3 * c + 1],
                 dz = xyz[3 * i + 2] - xyz[3 * c + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double m = exp(-zj.im * r) * (RSRR_INV4PI / r);
    acc += m * m;
  }
  acc *= 2.0;
  if (tid == 0) {
    const double re = -zj.im * RSRR_INV4PI + 0.5 / h, im = zj.re * RSRR_INV4PI;
    acc += (i2 != i1 ? 2.0 : 1.0) * (re * re + im * im);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) partial[(long)j * np + x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sum_rows_kernel(const double* partial, int len, int count,
                                                       double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int t = threadIdx.x; t < len; t += 256) acc += partial[(long)j * len + t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

int bem_fro2(int n, const double* xyz, double h, int nz, const c128* z_dev, double* partial,
             double* fro2, hipStream_t s) {
  if (nz <= 0) return ST_OK;
  const int np = (n + 1) / 2;
  hipLaunchKernelGGL(bem_fro2_partial, dim3(np, nz), dim3(256), 0, s, n, xyz, h, nz, z_dev, partial);
  RSRR_LAUNCH_CHECK();
  hipLaunchKernelGGL(sum_rows_kernel, dim3(nz), dim3(256), 0, s, partial, np, nz, fro2);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// R_j = U - T(z_j) Y_j with T generated on the fly in fp64: U copied into R,
// then the fp64 matrix-core GEMM whose A tiles are BEM entries computed where
// they are staged (gemm.hip: bem_gemm).
int bem_residual(int n, const double* xyz, double h, int nz, const c128* z_dev, const c128* U, long ldu,
                 const c128* Y, long ldy, long sY, int L, c128* Rout, long ldr, long sR, hipStream_t s) {
  if (nz <= 0) return ST_OK;
  RSRR_TRY((convert<double, double>(U, ldu, 0, Rout, ldr, sR, n, L, nz, s)));
  GemmBatch<double> g;
  g.M = n; g.N = L; g.K = n;
  g.alpha = mk<double>(-1, 0); g.beta = mk<double>(1, 0);
  g.B = Y; g.ldb = ldy; g.sB = sY;
  g.C = Rout; g.ldc = ldr; g.sC = sR;
  g.batch = nz;
  g.tag = "bem_residual";
  return bem_gemm(g, xyz, h, z_dev, s);
}

// ------------------------------------------------------------ elementwise
template <typename D, typename S>
__global__ __launch_bounds__(256) void convert_kernel(const cplx<S>* src, long lds, long ss,
                                                      cplx<D>* dst, long ldd, long sd, int rows,
                                                      int cols) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (e >= (long)rows * cols) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[(long)b * sd + i + (long)c * ldd] = ccast<D>(src[(long)b * ss + i + (long)c * lds]);
}

template <typename D, typename S>
int convert(const cplx<S>* src, long lds, long ss, cplx<D>* dst, long ldd, long sd, int rows,
            int cols, int batch, hipStream_t s) {
  const long cnt = (long)rows * cols;
  if (cnt <= 0 || batch <= 0) return ST_OK;
  hipLaunchKernelGGL((convert_kernel<D, S>), dim3((unsigned)cdivl(cnt, 256), (unsigned)batch),
                     dim3(256), 0, s, src, lds, ss, dst, ldd, sd, rows, cols);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}
template int convert<double, float>(const c64*, long, long, c128*, long, long, int, int, int, hipStream_t);
template int convert<float, double>(const c128*, long, long, c64*, long, long, int, int, int, hipStream_t);
template int convert<double, double>(const c128*, long, long, c128*, long, long, int, int, int, hipStream_t);
template int convert<float, float>(const c64*, long, long, c64*, long, long, int, int, int, hipStream_t);

template <typename R>
int replicate(const cplx<R>* src, long lds, cplx<R>* dst, long ldd, long sd, int rows, int cols,
              int batch, hipStream_t s) {
  return convert<R, R>(src, lds, 0, dst, ldd, sd, rows, cols, batch, s);
}
template int replicate<double>(const c128*, long, c128*, long, long, int, int, int, hipStream_t);
template int replicate<float>(const c64*, long, c64*, long, long, int, int, int, hipStream_t);

__global__ __launch_bounds__(256) void add_correction_kernel(c128* Y, long ldy, long sY,
                                                             const c64* D, long ldd, long sD,
                                                             int rows, int cols,
                                                             const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  c128& y = Y[(long)b * sY + i + (long)c * ldy];
  const c64 d = D[(long)b * sD + i + (long)c * ldd];
  y = y + ccast<double>(d);
}

int add_correction(c128* Y, long ldy, long sY, const c64* D, long ldd, long sD, int rows, int cols,
                   int batch, const int* active, hipStream_t s) {
  const long cnt = (long)rows * cols;
  if (cnt <= 0 || batch <= 0) return ST_OK;
  hipLaunchKernelGGL(add_correction_kernel, dim3((unsigned)cdivl(cnt, 256), (unsigned)batch),
                     dim3(256), 0, s, Y, ldy, sY, D, ldd, sD, rows, cols, active);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

struct PtrArgs { const c128* p[MAXJ]; };
__global__ __launch_bounds__(256) void combine_residual_kernel(const c128* U, long ldu, PtrArgs P,
                                                               int J, const c128* coef, int n,
                                                               int L, c128* R, long ldr) {
  const int b = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * L) return;
  const int i = (int)(e % n), l = (int)(e / n);
  c128 acc = U[i + (long)l * ldu];
  const long col = (long)b * L + l;
#pragma unroll
  for (int k = 0; k < MAXJ; ++k)
    if (k < J) acc = acc - coef[(long)b * J + k] * P.p[k][i + col * n];
  R[i + col * ldr] = acc;
}

int combine_residual(const c128* U, long ldu, const c128* const* P_host, int J, const c128* coef,
                     int n, int L, int batch, c128* R, long ldr, hipStream_t s) {
  if (J > MAXJ) return set_error(ST_EINVAL, "combine_residual: J too large");
  PtrArgs pa;
  for (int k = 0; k < MAXJ; ++k) pa.p[k] = k < J ? P_host[k] : nullptr;
  const long cnt = (long)n * L;
  hipLaunchKernelGGL(combine_residual_kernel, dim3((unsigned)cdivl(cnt, 256), (unsigned)batch),
                     dim3(256), 0, s, U, ldu, pa, J, coef, n, L, R, ldr);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// Column slices of each batch entry, one workgroup each (lanes along the rows,
// so a wave reads a contiguous piece of a column); the slices' sums are added
// in a fixed order afterwards.
__global__ __launch_bounds__(256) void block_fro2_kernel(const c128* X, long ldx, long sX, int rows,
                                                         int cols, int P, double* part) {
  __shared__ double red[4];
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const c128* Xb = X + (long)b * sX;
  double acc = 0.0;
  for (int c = x; c < cols; c += P)
    for (int i = tid; i < rows; i += 256) acc += abs2(Xb[i + (long)c * ldx]);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) part[(long)b * P + x] = (red[0] + red[1]) + (red[2] + red[3]);
}

int block_fro2(const c128* X, long ldx, long sX, int rows, int cols, int batch, double* out,
               double* part, hipStream_t s) {
  if (batch <= 0) return ST_OK;
  const int P = std::max(1, std::min(cols, BLOCK_FRO2_PARTS));
  if (P > 1 && !part) return set_error(ST_EINVAL, "block_fro2: no buffer for the partial sums");
  hipLaunchKernelGGL(block_fro2_kernel, dim3(P, batch), dim3(256), 0, s, X, ldx, sX, rows, cols, P,
                     P > 1 ? part : out);
  RSRR_LAUNCH_CHECK();
  if (P > 1) {
    hipLaunchKernelGGL(sum_rows_kernel, dim3(batch), dim3(256), 0, s, part, P, batch, out);
    RSRR_LAUNCH_CHECK();
  }
  return ST_OK;
}

__global__ __launch_bounds__(256) void diag_scale_kernel(const c128* d, const c128* X, long ldx,
                                                         c128* Y, long ldy, int n, int cols) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * cols) return;
  const int i = (int)(e % n), c = (int)(e / n);
  Y[i + (long)c * ldy] = d[i] * X[i + (long)c * ldx];
}

int diag_scale(const c128* d, const c128* X, long ldx, c128* Y, long ldy, int n, int cols,
               hipStream_t s) {
  const long cnt = (long)n * cols;
  if (cnt <= 0) return ST_OK;
  hipLaunchKernelGGL(diag_scale_kernel, dim3((unsigned)cdivl(cnt, 256)), dim3(256), 0, s, d, X, ldx,
                     Y, ldy, n, cols);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

}  // namespace rsrr
