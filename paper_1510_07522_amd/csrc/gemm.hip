// Batched complex GEMM on CDNA4 matrix cores.
//
//   C_b = alpha * op(A_b) * op(B_b) + beta * C_b,   b = 0 .. batch-1
//
// Complex products are split into real MFMA products on interleaved data:
//   4M:  Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br          (4 MFMA / k-quad)
//   3M:  P1 += Ar Br, P2 += Ai Bi, P3 += (Ar+Ai)(Br+Bi);    (3 MFMA / k-quad)
//        Cr = P1 - P2, Ci = P3 - P1 - P2 (normwise stable; used where the
//        result is refined or self-correcting)
// A may be real (fp64/fp32 values), which halves the products.
//
// Tiling: 64x64 C tile per workgroup; complex128 uses 8 waves of 32x16,
// complex64 4 waves of 32x32 (blocks of the 16x16x4 MFMA).  K is staged
// through LDS 16 at a time with one register-prefetched tile in flight.  The
// LDS tiles are stored [k][m ^ (k & 15)]: a store with k running across lanes
// (column-major B, or A^T / A^H) then hits 16 different banks instead of one,
// and the MFMA operand reads stay conflict-free.  The epilogue stages the
// products through the same LDS bytes so that C is read and written one
// contiguous column per wave instruction.
#include <algorithm>

#include "bem.h"
#include "common.h"
#include "kernels.h"
#include "timers.h"

namespace rsrr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R> struct V4;
template <> struct V4<double> { typedef d4 T; };
template <> struct V4<float> { typedef f4 T; };

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int BM = 64, BN = 64, BK = 16, PAD = 16;
// threads per workgroup: 512 for complex128 (8 waves of 32x16, so that the
// accumulators and the register staging of one wave fit 4 waves per SIMD),
// 256 for complex64 (4 waves of 32x32)
template <typename R> constexpr int gemm_threads() { return sizeof(R) == 8 ? 512 : 256; }

// Where the A operand of the BEM residual comes from: the points, the
// spacing and one node z per batch entry (A_b = T(z_b) generated in place).
struct BemGen {
  const double* xyz;
  double h;
  const c128* z;
};

// One 64x64 tile of C (rows m0.., columns n0.. of batch entry bz).  Every
// thread of the workgroup calls it with the same arguments; it ends with a
// barrier, so a workgroup may run several tiles in turn.
template <typename R, int OPA, int OPB, bool AREAL, bool G3M, bool ABEM>
__device__ __forceinline__ void gemm_body(const GemmBatch<R>& g, const BemGen& bg, int m0, int n0, int bz) {
  typedef typename V4<R>::T acc_t;
  constexpr int NT = gemm_threads<R>();
  constexpr int WJ = NT == 512 ? 1 : 2;          // 16-column blocks per wave
  constexpr int LP = BM * BK / NT;               // tile elements per thread and operand
  // operand tiles during the K loop; the epilogue reuses the same bytes to
  // stage half of the C tile (32 columns x 64 rows of complex values)
  constexpr int OPND = (3 * BK + (AREAL ? 1 : BK)) * (BM + PAD) * (int)sizeof(R);
  constexpr int SLD = BM + 1;                    // staged column stride (odd: fewer bank conflicts)
  constexpr int STAGE = (BN / 2) * SLD * 2 * (int)sizeof(R);
  __shared__ __align__(16) unsigned char smem[OPND > STAGE ? OPND : STAGE];
  typedef R Tile[BM + PAD];
  Tile* As_re = (Tile*)smem;
  Tile* Bs_re = As_re + BK;
  Tile* Bs_im = Bs_re + BK;
  Tile* As_im = Bs_im + BK;

  const int M = g.M, N = g.N, K = g.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;       // 32-row half, 16*WJ-column slice

  const R* Ar = AREAL ? (const R*)g.A + (long)bz * g.sA : nullptr;
  const cplx<R>* Ac = AREAL ? nullptr : (const cplx<R>*)g.A + (long)bz * g.sA;
  const cplx<R>* Bp = g.B + (long)bz * g.sB;
  cplx<R>* Cp = g.C + (long)bz * g.sC;

  acc_t acc0[2][WJ], acc1[2][WJ], acc2[2][WJ];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      acc0[i][j] = acc_t{0, 0, 0, 0};
      acc1[i][j] = acc_t{0, 0, 0, 0};
      acc2[i][j] = acc_t{0, 0, 0, 0};
    }

  // register staging of one A and one B tile (LP elements per thread each)
  cplx<R> ra[LP], rb[LP];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      int m, k;
      if (OPA == OP_N) { m = tid & 63; k = (tid >> 6) + (NT / 64) * p; }
      else             { k = tid & 15; m = (tid >> 4) + (NT / 16) * p; }
      int gm = m0 + m, gk = k0 + k;
      cplx<R> v = mk<R>(0, 0);
      if constexpr (ABEM) {
        // A = T(z_bz): row gm, column gk of the single-layer matrix
        if (gm < M && gk < K) {
          const c128 zb = bg.z[bz];
          if (gm == gk) {
            v = bem_diag(zb, bg.h);
          } else {
            const double dx = bg.xyz[3 * gm] - bg.xyz[3 * gk], dy = bg.xyz[3 * gm + 1] - bg.xyz[3 * gk + 1],
                         dz = bg.xyz[3 * gm + 2] - bg.xyz[3 * gk + 2];
            v = bem_entry<double>(sqrt(dx * dx + dy * dy + dz * dz), zb.re, zb.im);
          }
        }
      } else if (gm < M && gk < K) {
        long idx = (OPA == OP_N) ? (long)gm + (long)gk * g.lda : (long)gk + (long)gm * g.lda;
        if (AREAL) v.re = Ar[idx];
        else {
          v = Ac[idx];
          if (OPA == OP_C) v.im = -v.im;
        }
      }
      ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      int n, k;
      if (OPB == OP_N) { k = tid & 15; n = (tid >> 4) + (NT / 16) * p; }
      else             { n = tid & 63; k = (tid >> 6) + (NT / 64) * p; }
      int gn = n0 + n, gk = k0 + k;
      cplx<R> v = mk<R>(0, 0);
      if (gn < N && gk < K) {
        long idx = (OPB == OP_N) ? (long)gk + (long)gn * g.ldb : (long)gn + (long)gk * g.ldb;
        v = Bp[idx];
        if (OPB == OP_C) v.im = -v.im;
      }
      rb[p] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      int m, k;
      if (OPA == OP_N) { m = tid & 63; k = (tid >> 6) + (NT / 64) * p; }
      else             { k = tid & 15; m = (tid >> 4) + (NT / 16) * p; }
      As_re[k][m ^ (k & 15)] = ra[p].re;
      if (!AREAL) As_im[k][m ^ (k & 15)] = ra[p].im;
    }
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      int n, k;
      if (OPB == OP_N) { k = tid & 15; n = (tid >> 4) + (NT / 16) * p; }
      else             { n = tid & 63; k = (tid >> 6) + (NT / 64) * p; }
      Bs_re[k][n ^ (k & 15)] = rb[p].re;
      Bs_im[k][n ^ (k & 15)] = rb[p].im;
    }
  };

  const int ntiles = (K + BK - 1) / BK;
  if (ntiles > 0) load_tiles(0);
  for (int t = 0; t < ntiles; ++t) {
    store_tiles();
    __syncthreads();
    if (t + 1 < ntiles) load_tiles((t + 1) * BK);
#pragma unroll
    for (int kq = 0; kq < BK / 4; ++kq) {
      const int kk = kq * 4 + (lane >> 4);
      const int sw = (lane & 15) ^ (kk & 15);      // swizzled column within a 16-block
      R ar[2], ai[2], br[WJ], bi[WJ];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        int mm = wm * 32 + i * 16 + sw;
        ar[i] = As_re[kk][mm];
        ai[i] = AREAL ? R(0) : As_im[kk][mm];
      }
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
        int nn = wn * 16 * WJ + j * 16 + sw;
        br[j] = Bs_re[kk][nn];
        bi[j] = Bs_im[kk][nn];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          if (AREAL) {
            acc0[i][j] = mfma16(ar[i], br[j], acc0[i][j]);
            acc1[i][j] = mfma16(ar[i], bi[j], acc1[i][j]);
          } else if (G3M) {
            acc0[i][j] = mfma16(ar[i], br[j], acc0[i][j]);
            acc1[i][j] = mfma16(ai[i], bi[j], acc1[i][j]);
            acc2[i][j] = mfma16(ar[i] + ai[i], br[j] + bi[j], acc2[i][j]);
          } else {
            acc0[i][j] = mfma16(ar[i], br[j], acc0[i][j]);
            acc0[i][j] = mfma16(-ai[i], bi[j], acc0[i][j]);
            acc1[i][j] = mfma16(ar[i], bi[j], acc1[i][j]);
            acc1[i][j] = mfma16(ai[i], br[j], acc1[i][j]);
          }
        }
    }
    __syncthreads();
  }

  // epilogue.  Accumulator lane layout (column lane%16 of each 16x16 block):
  //   f32 16x16x4: element r holds row 4*(lane/16) + r
  //   f64 16x16x4: element r holds row lane/16 + 4*r
  // The combined complex products go through LDS, half a tile (32 columns) at
  // a time, so that the read-modify-write of C runs one column of 64 rows per
  // wave instruction (contiguous) instead of 16 columns by 4 rows.
  const bool beta0 = (g.beta.re == R(0) && g.beta.im == R(0));
  R* st_re = (R*)smem;                       // [32 columns][SLD] real parts
  R* st_im = st_re + (BN / 2) * SLD;         // imaginary parts
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // waves whose columns lie in this half write their values
    const int wcol0 = wn * 16 * WJ;          // first column of this wave in the tile
    if (wcol0 / (BN / 2) == h) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          const int cl = wcol0 - h * (BN / 2) + j * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rr = (sizeof(R) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
            const int rl = wm * 32 + i * 16 + rr;
            R vr, vi;
            if (AREAL) { vr = acc0[i][j][r]; vi = acc1[i][j][r]; }
            else if (G3M) {
              vr = acc0[i][j][r] - acc1[i][j][r];
              vi = acc2[i][j][r] - acc0[i][j][r] - acc1[i][j][r];
            } else { vr = acc0[i][j][r]; vi = acc1[i][j][r]; }
            st_re[cl * SLD + rl] = vr;
            st_im[cl * SLD + rl] = vi;
          }
        }
    }
    __syncthreads();
    // one column of 64 rows per wave instruction
#pragma unroll
    for (int e = 0; e < (BN / 2) * BM / NT; ++e) {
      const int q = e * NT + tid;
      const int cl = q / BM, rl = q % BM;
      const int row = m0 + rl, col = n0 + h * (BN / 2) + cl;
      if (row < M && col < N) {
        cplx<R> v;
        v.re = st_re[cl * SLD + rl];
        v.im = st_im[cl * SLD + rl];
        cplx<R> out = g.alpha * v;
        const long idx = (long)row + (long)col * g.ldc;
        if (!beta0) out = out + g.beta * Cp[idx];
        Cp[idx] = out;
      }
    }
    if (g.herm && m0 > n0) {
      // the conjugate transpose of this tile below the diagonal, above it:
      // consecutive threads take consecutive columns of the staged half,
      // which are consecutive rows of the mirrored tile
#pragma unroll
      for (int e = 0; e < (BN / 2) * BM / NT; ++e) {
        const int q = e * NT + tid;
        const int cl = q % (BN / 2), rl = q / (BN / 2);
        const int row = m0 + rl, col = n0 + h * (BN / 2) + cl;
        if (row < M && col < N) {
          const cplx<R> v = mk<R>(st_re[cl * SLD + rl], -st_im[cl * SLD + rl]);
          Cp[(long)col + (long)row * g.ldc] = g.alpha.re * v;
        }
      }
    }
    __syncthreads();
  }
}

template <typename R, int OPA, int OPB, bool AREAL, bool G3M>
__global__ __launch_bounds__(sizeof(R) == 8 ? 512 : 256) void gemm_kernel(GemmBatch<R> g) {
  if (g.active && !g.active[blockIdx.z]) return;
  if (g.herm && blockIdx.x < blockIdx.y) return;   // above the diagonal: written by its mirror
  gemm_body<R, OPA, OPB, AREAL, G3M, false>(g, BemGen{nullptr, 0.0, nullptr}, blockIdx.x * BM, blockIdx.y * BN,
                                            blockIdx.z);
}

// Workgroup (x, b) takes columns 64x .. 64x+63 of B_b through the group's
// panels in order, one 64x64 tile product at a time: the columns are
// independent, so no other workgroup reads or writes them, and the barrier
// that ends each product makes its stores visible to the next one.  The
// diagonal block's product is in place: its single row tile reads all of B_k
// before writing it.
template <typename R, bool G3M>
__global__ __launch_bounds__(sizeof(R) == 8 ? 512 : 256) void lu_group_solve_kernel(LUGroupSolve<R> q) {
  const int b = blockIdx.y, n0 = blockIdx.x * BN;
  if (q.active && !q.active[b]) return;
  const BemGen none{nullptr, 0.0, nullptr};
  GemmBatch<R> g;
  g.N = q.nrhs;
  g.ldb = q.ldb; g.sB = q.sB;
  g.ldc = q.ldb; g.sC = q.sB;
  for (int t = 0; t < q.p1 - q.p0; ++t) {
    const int p = q.lower ? q.p0 + t : q.p1 - 1 - t;
    const int k = p * q.nb, nbe = min(q.nb, q.n - k);
    g.M = nbe; g.K = nbe;
    g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
    g.A = q.dinv + (long)p * 2 * q.nb * q.nb + (q.lower ? 0 : (long)q.nb * q.nb);
    g.lda = q.nb; g.sA = q.sD;
    g.B = q.B + k; g.C = q.B + k;
    gemm_body<R, OP_N, OP_N, false, G3M, false>(g, none, 0, n0, b);
    const int k0 = q.p0 * q.nb, k1 = min(q.n, q.p1 * q.nb);
    const int r0 = q.lower ? k + nbe : k0, rows = q.lower ? k1 - k - nbe : k - k0;
    if (rows <= 0) continue;
    g.M = rows; g.K = nbe;
    g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
    g.A = q.A + r0 + (long)k * q.lda; g.lda = q.lda; g.sA = q.sA;
    g.B = q.B + k; g.C = q.B + r0;
    for (int m0 = 0; m0 < rows; m0 += BM) gemm_body<R, OP_N, OP_N, false, G3M, false>(g, none, m0, n0, b);
  }
}

template <typename R>
int lu_group_solve(const LUGroupSolve<R>& q, hipStream_t s) {
  if (q.nrhs <= 0 || q.batch <= 0 || q.p1 <= q.p0) return ST_OK;
  if (q.nb < 1 || q.nb > BM || q.p0 < 0 || (long)q.p1 * q.nb > (long)q.n + q.nb - 1)
    return set_error(ST_EINVAL, "lu_group_solve: bad group %d..%d (nb %d, n %d)", q.p0, q.p1, q.nb, q.n);
  const dim3 grid((unsigned)cdivl(q.nrhs, BN), (unsigned)q.batch);
  const int k0 = q.p0 * q.nb, k1 = std::min(q.n, q.p1 * q.nb), w = k1 - k0;
  // the group's triangle (w^2 / 2 entries) applied to nrhs columns
  const double fl = 8.0 * 0.5 * w * (double)w * q.nrhs * q.batch;
  KernelTimer kt(q.tag, s, fl, 2.0 * sizeof(cplx<R>) * (0.5 * w * (double)w + 2.0 * w * q.nrhs) * q.batch,
                 timers_on() ? std::string("lu_group_solve_kernel<") + (sizeof(R) == 8 ? "double" : "float") +
                                   (q.gauss3m ? ", true>" : ", false>")
                             : std::string());
  if (q.gauss3m)
    hipLaunchKernelGGL((lu_group_solve_kernel<R, true>), grid, dim3(gemm_threads<R>()), 0, s, q);
  else
    hipLaunchKernelGGL((lu_group_solve_kernel<R, false>), grid, dim3(gemm_threads<R>()), 0, s, q);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

template int lu_group_solve<double>(const LUGroupSolve<double>&, hipStream_t);
template int lu_group_solve<float>(const LUGroupSolve<float>&, hipStream_t);

__global__ __launch_bounds__(512) void bem_gemm_kernel(GemmBatch<double> g, BemGen bg) {
  gemm_body<double, OP_N, OP_N, false, false, true>(g, bg, blockIdx.x * BM, blockIdx.y * BN, blockIdx.z);
}

int bem_gemm(const GemmBatch<double>& g, const double* xyz, double h, const c128* z_dev, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return ST_OK;
  if (g.M != g.K || g.opA != OP_N || g.opB != OP_N || g.a_real || g.gauss3m)
    return set_error(ST_EINVAL, "bem_gemm: needs a square generated A, no transposes, 4M products");
  dim3 grid((unsigned)cdivl(g.M, BM), (unsigned)cdivl(g.N, BN), (unsigned)g.batch);
  KernelTimer kt(g.tag, s, 8.0 * g.M * (double)g.N * g.K * g.batch,
                 16.0 * g.batch * ((double)g.K * g.N + 2.0 * g.M * g.N),
                 timers_on() ? std::string("bem_gemm_kernel") : std::string());
  hipLaunchKernelGGL(bem_gemm_kernel, grid, dim3(gemm_threads<double>()), 0, s, g, BemGen{xyz, h, z_dev});
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

template <typename R> struct GSegDev {
  const cplx<R>* A;
  const cplx<R>* B;
  cplx<R>* C;
  long lda, sA, ldb, sB, ldc, sC;
  int M, N, K, tm, tn;      // shape, tiles along M and N
  long tile0;               // first tile of the segment in the launch
};
template <typename R> struct GSegArgs {
  int count;
  long total;
  cplx<R> alpha, beta;
  GSegDev<R> s[GSEG];
};

template <typename R, bool G3M>
__global__ __launch_bounds__(sizeof(R) == 8 ? 512 : 256) void gemm_seg_kernel(GSegArgs<R> a) {
  for (long t = blockIdx.x; t < a.total; t += gridDim.x) {
    int q = 0;
    while (q + 1 < a.count && t >= a.s[q + 1].tile0) ++q;
    const GSegDev<R>& d = a.s[q];
    const long u = t - d.tile0, per = (long)d.tm * d.tn;
    const int bz = (int)(u / per);
    const int r = (int)(u - (long)bz * per);
    GemmBatch<R> g;
    g.M = d.M; g.N = d.N; g.K = d.K;
    g.alpha = a.alpha; g.beta = a.beta;
    g.A = d.A; g.lda = d.lda; g.sA = d.sA;
    g.B = d.B; g.ldb = d.ldb; g.sB = d.sB;
    g.C = d.C; g.ldc = d.ldc; g.sC = d.sC;
    gemm_body<R, OP_N, OP_N, false, G3M, false>(g, BemGen{nullptr, 0.0, nullptr}, (r % d.tm) * BM,
                                                (r / d.tm) * BN, bz);
  }
}

template <typename R>
int gemm_segments(const GemmSegs<R>& sg, hipStream_t s) {
  if (sg.count < 0 || sg.count > GSEG) return set_error(ST_EINVAL, "gemm_segments: %d segments", sg.count);
  GSegArgs<R> a;
  a.count = 0;
  a.total = 0;
  double flops = 0, bytes = 0;
  const double es = (double)sizeof(cplx<R>);
  for (int q = 0; q < sg.count; ++q) {
    const GemmBatch<R>& g = sg.g[q];
    if (g.opA != OP_N || g.opB != OP_N || g.a_real || g.active)
      return set_error(ST_EINVAL, "gemm_segments: untransposed complex operands only");
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) continue;
    GSegDev<R>& d = a.s[a.count++];
    d.A = (const cplx<R>*)g.A; d.B = g.B; d.C = g.C;
    d.lda = g.lda; d.sA = g.sA; d.ldb = g.ldb; d.sB = g.sB; d.ldc = g.ldc; d.sC = g.sC;
    d.M = g.M; d.N = g.N; d.K = g.K;
    d.tm = (int)cdivl(g.M, BM);
    d.tn = (int)cdivl(g.N, BN);
    d.tile0 = a.total;
    a.total += (long)d.tm * d.tn * g.batch;
    flops += 8.0 * g.M * (double)g.N * g.K * g.batch;
    bytes += g.batch * (es * ((double)g.M * g.K + (double)g.K * g.N) + 2.0 * es * (double)g.M * g.N);
  }
  if (a.total == 0) return ST_OK;
  a.alpha = sg.g[0].alpha;
  a.beta = sg.g[0].beta;
  const long cap = (sizeof(R) == 8 ? 4 : 8) * 256;      // resident workgroups on 256 CUs
  const unsigned grid = (unsigned)std::min<long>(a.total, cap);
  const bool g3m = sg.g[0].gauss3m;
  KernelTimer kt(sg.g[0].tag, s, flops, bytes,
                 timers_on() ? std::string("gemm_seg_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                   (g3m ? "true" : "false") + ">"
                             : std::string());
  if (g3m) hipLaunchKernelGGL((gemm_seg_kernel<R, true>), dim3(grid), dim3(gemm_threads<R>()), 0, s, a);
  else hipLaunchKernelGGL((gemm_seg_kernel<R, false>), dim3(grid), dim3(gemm_threads<R>()), 0, s, a);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}
template int gemm_segments<double>(const GemmSegs<double>&, hipStream_t);
template int gemm_segments<float>(const GemmSegs<float>&, hipStream_t);

template <typename R, int OPA, int OPB, bool AREAL, bool G3M>
static int launch_one(const GemmBatch<R>& g, hipStream_t s) {
  dim3 grid((unsigned)cdivl(g.M, BM), (unsigned)cdivl(g.N, BN), (unsigned)g.batch);
  const double es = (double)sizeof(cplx<R>);
  const double tiles = (double)cdivl(g.M, BM);
  const double flops = (AREAL ? 4.0 : 8.0) * g.M * (double)g.N * g.K * g.batch *
                       (g.herm ? (tiles + 1) / (2 * tiles) : 1.0);
  const double bytes = g.batch * ((AREAL ? es / 2 : es) * (double)g.M * g.K + es * (double)g.K * g.N +
                                  es * (double)g.M * g.N *
                                      ((g.beta.re != R(0) || g.beta.im != R(0)) ? 2.0 : 1.0));
  KernelTimer kt(g.tag, s, flops, bytes,
                 timers_on() ? std::string("gemm_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                   std::to_string(OPA) + ", " + std::to_string(OPB) + ", " +
                                   (AREAL ? "true" : "false") + ", " + (G3M ? "true" : "false") + ">"
                             : std::string());
  hipLaunchKernelGGL((gemm_kernel<R, OPA, OPB, AREAL, G3M>), grid, dim3(gemm_threads<R>()), 0, s, g);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

template <typename R, bool AREAL, bool G3M>
static int launch_ops(const GemmBatch<R>& g, hipStream_t s) {
#define RSRR_CASE(a, b) if (g.opA == a && g.opB == b) return launch_one<R, a, b, AREAL, G3M>(g, s);
  RSRR_CASE(OP_N, OP_N) RSRR_CASE(OP_N, OP_T) RSRR_CASE(OP_N, OP_C)
  RSRR_CASE(OP_T, OP_N) RSRR_CASE(OP_T, OP_T) RSRR_CASE(OP_T, OP_C)
  RSRR_CASE(OP_C, OP_N) RSRR_CASE(OP_C, OP_T) RSRR_CASE(OP_C, OP_C)
#undef RSRR_CASE
  return set_error(ST_EINVAL, "gemm: bad op pair %d,%d", g.opA, g.opB);
}

template <typename R>
int gemm_batched(const GemmBatch<R>& g, hipStream_t s) {
  if (g.M < 0 || g.N < 0 || g.K < 0 || g.batch < 0)
    return set_error(ST_EINVAL, "gemm: negative size");
  if (g.M == 0 || g.N == 0 || g.batch == 0) return ST_OK;
  if (g.a_real && g.opA == OP_C) return set_error(ST_EINVAL, "gemm: real A with conj op");
  if (g.herm && (g.opA != OP_C || g.opB != OP_N || (const void*)g.B != g.A || g.M != g.N || g.a_real ||
                 g.alpha.im != R(0) || g.beta.re != R(0) || g.beta.im != R(0) || g.active))
    return set_error(ST_EINVAL, "gemm: the Gram form needs C = alpha A^H A with real alpha and beta 0");
  if (g.a_real) return launch_ops<R, true, false>(g, s);
  if (g.gauss3m) return launch_ops<R, false, true>(g, s);
  return launch_ops<R, false, false>(g, s);
}

template int gemm_batched<double>(const GemmBatch<double>&, hipStream_t);
template int gemm_batched<float>(const GemmBatch<float>&, hipStream_t);

}  // namespace rsrr
