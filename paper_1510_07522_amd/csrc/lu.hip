// Batched blocked right-looking complex LU with partial pivoting, and the
// matching solve, for the probed-resolvent solves T(z_j) Y_j = U.
//
// Per panel of width nb (default 64):
//   1. lu_panel_kernel (one 1024-thread workgroup per matrix): the panel is
//      factored in register-resident micro-panels of W columns; pivot search
//      is a workgroup arg-max of |re|+|im| (first index on ties, as LAPACK);
//      the rest of the panel is updated in place; finally the unit-lower and
//      upper diagonal blocks are inverted in LDS (kept for the solves).
//   2. lu_permute_kernel: the panel's interchanges, applied as one gather to
//      the columns right of the panel.
//   3. U12 = inv(L11) A12 and A22 -= L21 U12 as matrix-core GEMMs.
// Panels come in blocks of lu_group(nb) (K = 256 products for the columns
// beyond a block); with look-ahead, the far columns' product runs on a second
// stream in column pieces while the next panels are factored.
#include "common.h"
#include "kernels.h"
#include "timers.h"
#include <algorithm>
#include <string>
#include <vector>

namespace rsrr {

constexpr int PNT = 1024;           // panel workgroup size (16 waves)
// flops per launch of the look-ahead stream's trailing-update pieces
constexpr double WINDOW_FLOP = 1.6e11;
constexpr int MAXNB = 64;
// panels per group of the triangular solves (and of the row order lu_factor
// gives the L columns): groups of 256 columns
__host__ __device__ constexpr int lu_group(int nb) { return nb >= 256 ? 1 : 256 / nb; }

// Several strided batches of matrices of different orders, for launches that
// cover them all (segment q: matrices first[q] .. first[q+1]-1 of the launch).
constexpr int MAXSEG = 16;
template <typename R> struct LUSegDev {
  cplx<R>* A;        // first matrix, leading dim lda, batch stride sA
  long lda, sA;
  int n;             // order
  int* ipiv;         // n per matrix
  cplx<R>* dinv;     // sD per matrix
  long sD;
  int* info;         // one per matrix
  int c0, ncols;     // row interchanges: the columns they apply to
  int k, nbe;        // row interchanges: the panel whose pivots are applied
};
template <typename R> struct LUSegArgs {
  int count;
  int first[MAXSEG + 1];
  LUSegDev<R> seg[MAXSEG];
};

template <typename R> __device__ inline cplx<R> shfl_c(cplx<R> v, int src) {
  return mk<R>(__shfl(v.re, src), __shfl(v.im, src));
}

// Panel of one matrix: columns [k, k + nbe) of Ab (order n, leading dim lda),
// pivots into pv, the diagonal-block inverses into dl (2 nb^2 elements), the
// status word *info_b.
template <typename R, int ROWS, int W>
__device__ __forceinline__ void lu_panel_body(cplx<R>* Ab, long lda, int n, int k, int nbe, int nb, int* pv,
                                              cplx<R>* dl, int* info_b) {
  // Thread tid owns rows c + tid + PNT*i (i < ROWS) of the current micro-panel
  // of W columns, kept in registers.  Per pivot: wave arg-max -> every wave
  // leader publishes its value and index, the lane owning the wave's best row
  // publishes that row (one barrier); all threads then pick the winner.  The
  // pivot loop is unrolled over the W columns so that every register access
  // is static.
  __shared__ unsigned s_val[2][16];
  __shared__ int s_row[2][16];
  __shared__ cplx<R> s_cand[2][16][W];
  __shared__ cplx<R> s_crow[2][W];
  __shared__ cplx<R> s_L[W][W];
  __shared__ cplx<R> s_U[W][MAXNB];       // U rows of the micro-panel, one column per thread
  // rows k .. k+nbe-1 of the panel as far as they are final (U rows and the
  // micro-panels' L rows), then the diagonal block for its inverses
  __shared__ cplx<R> s_D[MAXNB][MAXNB + 1];
  __shared__ int s_piv[W];
  __shared__ int t_row[2 * W], t_src[2 * W];
  __shared__ int s_cnt;
  __shared__ cplx<R> s_mv[2 * W][MAXNB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cplx<R> a[ROWS][W];
  int parity = 0;

  // Left-looking (Crout) order inside the panel: a micro-panel receives the
  // updates of the panel's earlier columns when it is loaded, and the U rows
  // of each micro-panel are formed for the later columns of the panel right
  // after it is factored, so the later columns are read and written once
  // instead of after every micro-panel.
  for (int c = k; c < k + nbe; c += W) {
    const int w = min(W, k + nbe - c);
    const int done = c - k;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = c + tid + PNT * i;
#pragma unroll
      for (int j = 0; j < W; ++j)
        a[i][j] = (r < n && j < w) ? Ab[r + (long)(c + j) * lda] : mk<R>(0, 0);
    }
    if (done > 0) {
      // a -= L[rows, k..c) U[k..c, c..c+w), the U rows from s_D; the L
      // entries of CH columns are loaded together (one memory round trip per
      // CH columns; 8 complex128 or 16 complex64 values per thread)
      constexpr int CHV = sizeof(R) == 8 ? 8 : 16;
      constexpr int CH = CHV / ROWS > 8 ? 8 : (CHV / ROWS < 1 ? 1 : CHV / ROWS);
      for (int l0 = 0; l0 < done; l0 += CH) {
        cplx<R> lv[CH][ROWS];
#pragma unroll
        for (int t = 0; t < CH; ++t)
#pragma unroll
          for (int i = 0; i < ROWS; ++i) {
            const int r = c + tid + PNT * i, l = l0 + t;
            lv[t][i] = (r < n && l < done) ? Ab[r + (long)(k + l) * lda] : mk<R>(0, 0);
          }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
          const int l = l0 + t;
          if (l < done) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
              const cplx<R> u = (j < w) ? s_D[l][done + j] : mk<R>(0, 0);
#pragma unroll
              for (int i = 0; i < ROWS; ++i) a[i][j] = a[i][j] - lv[t][i] * u;
            }
          }
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
      if (jj < w) {
        const int col = c + jj;
        unsigned bv = 0;
        int brow = -1;
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
          const int r = c + tid + PNT * i;
          if (r >= col && r < n) {
            const unsigned v = mag_bits(cabs1(a[i][jj]));
            if (brow < 0 || v > bv) { bv = v; brow = r; }
          }
        }
        const unsigned wm = wave_umax(bv);
        const unsigned long long hw = __ballot(brow >= 0 && bv == wm);
        int wrow = -1;
        if (hw) {
          const int wl = __ffsll((long long)hw) - 1;
          wrow = __builtin_amdgcn_readlane(brow, wl);
          if (lane == wl) {
#pragma unroll
            for (int i = 0; i < ROWS; ++i)
              if (c + tid + PNT * i == wrow) {
#pragma unroll
                for (int j = 0; j < W; ++j) s_cand[parity][wave][j] = a[i][j];
              }
          }
        }
        if (lane == 0) { s_val[parity][wave] = wm; s_row[parity][wave] = wrow; }
        // row col itself is row jj of the micro-panel: thread jj, register row 0
        if (tid == jj) {
#pragma unroll
          for (int j = 0; j < W; ++j) s_crow[parity][j] = a[0][j];
        }
        __syncthreads();
        // workgroup maximum over the 16 wave results (row col is a candidate,
        // so at least one wave has a row)
        const unsigned vq = (lane < 16) ? s_val[parity][lane] : 0u;
        const int rq = (lane < 16) ? s_row[parity][lane] : -1;
        const unsigned gm = (unsigned)__builtin_amdgcn_readlane((int)row16_umax_all(vq), 0);
        const unsigned long long hq = __ballot(rq >= 0 && vq == gm);
        const int wb = __ffsll((long long)hq) - 1;
        const bool zero = (gm == 0u);
        const int p = zero ? col : __builtin_amdgcn_readlane(rq, wb);
        if (tid == 0) {
          pv[col] = p;
          s_piv[jj] = p;
          if (zero && *info_b == 0) *info_b = col + 1;
        }
        const cplx<R>* prow = zero ? s_crow[parity] : s_cand[parity][wb];
        if (p != col) {
          const int tp = (p - c) % PNT, ip = (p - c) / PNT;
          if (tid == jj) {
#pragma unroll
            for (int j = 0; j < W; ++j) a[0][j] = prow[j];
          }
          if (tid == tp) {
#pragma unroll
            for (int i = 0; i < ROWS; ++i)
              if (i == ip) {
#pragma unroll
                for (int j = 0; j < W; ++j) a[i][j] = s_crow[parity][j];
              }
          }
        }
        const cplx<R> inv = zero ? mk<R>(1, 0) : crecip(prow[jj]);
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
          const int r = c + tid + PNT * i;
          if (r > col && r < n) {
            const cplx<R> l = a[i][jj] * inv;
            a[i][jj] = l;
#pragma unroll
            for (int j = jj + 1; j < W; ++j) a[i][j] = a[i][j] - l * prow[j];
          }
        }
        parity ^= 1;
      }
    }
    // ---- write the micro-panel back
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = c + tid + PNT * i;
      if (r < n)
#pragma unroll
        for (int j = 0; j < W; ++j)
          if (j < w) Ab[r + (long)(c + j) * lda] = a[i][j];
    }
    // ---- this micro-panel's interchanges on the other columns of the panel,
    // as one gather.  Wave 0 composes the w swaps: lane e holds touched row
    // t_row and its final source row t_src (registers, ballot to locate rows).
    if (wave == 0) {
      int my_row = (lane < w) ? c + lane : -1;
      int my_src = my_row;
      int cnt = w;
      for (int j = 0; j < w; ++j) {
        const int p = s_piv[j];
        if (p == c + j) continue;
        int pos;
        if (p < c + w) {
          pos = p - c;
        } else {
          const unsigned long long m = __ballot(my_row == p);
          if (m) {
            pos = __ffsll((long long)m) - 1;
          } else {
            pos = cnt;
            if (lane == cnt) { my_row = p; my_src = p; }
            ++cnt;
          }
        }
        const int sj = __shfl(my_src, j), sp = __shfl(my_src, pos);
        if (lane == j) my_src = sp;
        if (lane == pos) my_src = sj;
      }
      if (lane < cnt) { t_row[lane] = my_row; t_src[lane] = my_src; }
      if (lane == 0) s_cnt = cnt;
    }
    __syncthreads();
    {
      const int cnt = s_cnt;
      for (int e = tid; e < cnt * nbe; e += PNT) {
        const int q = e % cnt, cc = k + e / cnt;
        if (cc < c || cc >= c + w) s_mv[q][cc - k] = Ab[t_src[q] + (long)cc * lda];
      }
      __syncthreads();
      for (int e = tid; e < cnt * nbe; e += PNT) {
        const int q = e % cnt, cc = k + e / cnt;
        if (cc < c || cc >= c + w) Ab[t_row[q] + (long)cc * lda] = s_mv[q][cc - k];
      }
    }
    // U rows of this micro-panel for the later columns of the panel: the
    // earlier columns' terms, then the unit-lower solve with the micro-panel's
    // diagonal block; one column per thread
    const int rc0 = c + w, ncols = k + nbe - rc0;
    if (ncols > 0) {
      if (tid < w) {
#pragma unroll
        for (int j = 0; j < W; ++j) s_L[tid][j] = a[0][j];
      }
      __syncthreads();                   // the interchanges above are written
      // the micro-panel's rows are final in columns k..c-1 (L) from here on
      for (int e = tid; e < W * done; e += PNT) {
        const int jj = e % W, l = e / W;
        if (jj < w) s_D[done + jj][l] = Ab[c + jj + (long)(k + l) * lda];
      }
      __syncthreads();
      if (tid < ncols) {
        const int cc = rc0 + tid, cl = cc - k;
        cplx<R> v[W];
#pragma unroll
        for (int j = 0; j < W; ++j) v[j] = (j < w) ? Ab[c + j + (long)cc * lda] : mk<R>(0, 0);
        for (int l = 0; l < done; ++l) {
          const cplx<R> u = s_D[l][cl];
#pragma unroll
          for (int j = 0; j < W; ++j)
            if (j < w) v[j] = v[j] - s_D[done + j][l] * u;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) s_U[j][tid] = v[j];
        for (int j = 1; j < w; ++j) {
          cplx<R> x = s_U[j][tid];
          for (int l = 0; l < j; ++l) x = x - s_L[j][l] * s_U[l][tid];
          s_U[j][tid] = x;
        }
        for (int j = 0; j < w; ++j) {
          const cplx<R> x = s_U[j][tid];
          s_D[done + j][cl] = x;
          Ab[c + j + (long)cc * lda] = x;
        }
      }
    }
    __syncthreads();
  }

  // ---- inverses of the unit-lower and upper diagonal blocks (kept for the
  // solves): waves 0-7 take the columns of L^{-1}, waves 8-15 those of U^{-1};
  // lane i holds row i of the column, the substitution broadcasts by shuffle.
  for (int e = tid; e < nbe * nbe; e += PNT) {
    const int i = e % nbe, j = e / nbe;
    s_D[i][j] = Ab[k + i + (long)(k + j) * lda];
  }
  __syncthreads();
  cplx<R>* DL = dl;
  cplx<R>* DU = DL + (long)nb * nb;
  const int i = lane;
  if (wave < 8) {
    for (int j = wave; j < nb; j += 8) {
      cplx<R> x = mk<R>(i == j ? 1 : 0, 0);
      if (j < nbe) {
        for (int l = j; l < nbe - 1; ++l) {
          const cplx<R> xl = shfl_c(x, l);
          if (i > l && i < nbe) x = x - s_D[i][l] * xl;
        }
      }
      if (i < nb) DL[i + (long)j * nb] = (i >= j && i < nbe && j < nbe) ? x : mk<R>(0, 0);
    }
  } else {
    for (int j = wave - 8; j < nb; j += 8) {
      cplx<R> x = mk<R>(i == j ? 1 : 0, 0);
      if (j < nbe) {
        for (int l = j; l >= 0; --l) {
          if (i == l) x = x * crecip(s_D[l][l]);
          const cplx<R> xl = shfl_c(x, l);
          if (i < l) x = x - s_D[i][l] * xl;
        }
      }
      if (i < nb) DU[i + (long)j * nb] = (i <= j && j < nbe) ? x : mk<R>(0, 0);
    }
  }
}

template <typename R, int ROWS, int W>
__global__ __launch_bounds__(PNT) void lu_panel_kernel(cplx<R>* A, long lda, long sA, int n,
                                                        int k, int nbe, int nb, int* ipiv,
                                                        cplx<R>* dinv, long sD, int* info) {
  const int b = blockIdx.x;
  lu_panel_body<R, ROWS, W>(A + (long)b * sA, lda, n, k, nbe, nb, ipiv + (long)b * n, dinv + (long)b * sD,
                            info + b);
}

// The panels at column k of several strided batches of different orders in
// one launch: workgroup g factors matrix g - first[q] of segment q.
template <typename R, int ROWS, int W>
__global__ __launch_bounds__(PNT) void lu_panel_seg_kernel(LUSegArgs<R> a, int k, int nb) {
  int q = 0;
  while (q + 1 < a.count && (int)blockIdx.x >= a.first[q + 1]) ++q;
  const LUSegDev<R>& sg = a.seg[q];
  const int b = blockIdx.x - a.first[q];
  const int nbe = min(nb, sg.n - k);
  lu_panel_body<R, ROWS, W>(sg.A + (long)b * sg.sA, sg.lda, sg.n, k, nbe, nb, sg.ipiv + (long)b * sg.n,
                            sg.dinv + (long)b * sg.sD + (long)(k / nb) * 2 * nb * nb, sg.info + b);
}

// Applies the interchanges ipiv[k .. k+nbe) (each row i swapped with
// ipiv[i] >= i, in order) to columns [0, ncols) of X as one gather: every
// touched row gets its final source row.
template <typename R> struct SwCols { static constexpr int v = 8 * 16 / (int)sizeof(cplx<R>) * 2; };  // 32 (fp32) / 16 (fp64) columns per workgroup
template <typename R>
__device__ __forceinline__ void lu_permute_body(cplx<R>* Xb, long ldx, int ncols, const int* pv, int k, int nbe,
                                                int c0) {
  __shared__ int t_row[2 * MAXNB], t_src[2 * MAXNB];
  __shared__ int s_cnt;
  constexpr int SWC = SwCols<R>::v;
  __shared__ cplx<R> vals[SWC][2 * MAXNB];
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int lane = tid;
    for (int e = lane; e < nbe; e += 64) { t_row[e] = k + e; t_src[e] = k + e; }
    int cnt = nbe;
    wave_sync();
    for (int c = 0; c < nbe; c += 64) {
      // the chunk's pivots in one load; only the rows that move are visited
      const int mp = c + lane < nbe ? pv[k + c + lane] : k + c + lane;
      unsigned long long moved = __ballot(mp != k + c + lane);
      while (moved) {
        const int j = __ffsll((long long)moved) - 1;
        moved &= moved - 1;
        const int i = c + j;
        const int p = __shfl(mp, j);
        // locate p among the touched rows (rows k..k+nbe-1 sit at index row-k)
        int pos = -1;
        if (p < k + nbe) pos = p - k;
        else {
          for (int base = nbe; base < cnt; base += 64) {
            const int e = base + lane;
            const bool hit = (e < cnt) && (t_row[e] == p);
            const unsigned long long m = __ballot(hit);
            if (m) { pos = base + __ffsll((long long)m) - 1; break; }
          }
          if (pos < 0) {
            pos = cnt;
            if (lane == 0) { t_row[cnt] = p; t_src[cnt] = p; }
            cnt += 1;
            wave_sync();
          }
        }
        if (lane == 0) {
          const int s = t_src[i];
          t_src[i] = t_src[pos];
          t_src[pos] = s;
        }
        wave_sync();
      }
    }
    // keep only the rows whose source differs (a panel that pivots on its
    // diagonal moves nothing); a chunk's entries are read before any is
    // written, and land at or below their own index
    int kept = 0;
    for (int base = 0; base < cnt; base += 64) {
      const int e = base + lane;
      const int r = e < cnt ? t_row[e] : 0, sr = e < cnt ? t_src[e] : 0;
      const bool keep = e < cnt && sr != r;
      const unsigned long long m = __ballot(keep);
      const int at = kept + __popcll(m & ((1ull << lane) - 1ull));
      wave_sync();
      if (keep) { t_row[at] = r; t_src[at] = sr; }
      kept += __popcll(m);
      wave_sync();
    }
    if (lane == 0) s_cnt = kept;
  }
  __syncthreads();
  const int cnt = s_cnt;
  // a wave moves whole columns, its lanes along the touched rows (the panel's
  // rows are contiguous in a column, so those accesses coalesce)
  const int lane = tid & 63, wv = tid >> 6;
  for (int jc = wv; jc < SWC && c0 + jc < ncols; jc += 4) {
    const cplx<R>* xc = Xb + (long)(c0 + jc) * ldx;
    for (int e = lane; e < cnt; e += 64) vals[jc][e] = xc[t_src[e]];
  }
  __syncthreads();
  for (int jc = wv; jc < SWC && c0 + jc < ncols; jc += 4) {
    cplx<R>* xc = Xb + (long)(c0 + jc) * ldx;
    for (int e = lane; e < cnt; e += 64) xc[t_row[e]] = vals[jc][e];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void lu_permute_kernel(cplx<R>* X, long ldx, long sX, int ncols,
                                                         const int* ipiv, int ipiv_stride, int k,
                                                         int nbe, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  lu_permute_body<R>(X + (long)b * sX, ldx, ncols, ipiv + (long)b * ipiv_stride, k, nbe,
                     blockIdx.x * SwCols<R>::v);
}

// The same over segments: workgroup row y is matrix y - first[q] of segment q,
// whose columns [c0, c0 + ncols) take the interchanges of its panel at k.
template <typename R>
__global__ __launch_bounds__(256) void lu_permute_seg_kernel(LUSegArgs<R> a) {
  int q = 0;
  while (q + 1 < a.count && (int)blockIdx.y >= a.first[q + 1]) ++q;
  const LUSegDev<R>& sg = a.seg[q];
  const int c0 = blockIdx.x * SwCols<R>::v;
  if (c0 >= sg.ncols) return;
  const int b = blockIdx.y - a.first[q];
  lu_permute_body<R>(sg.A + (long)b * sg.sA + (long)sg.c0 * sg.lda, sg.lda, sg.ncols, sg.ipiv + (long)b * sg.n,
                     sg.k, sg.nbe, c0);
}

// The interchanges of panels p0 .. p1-1 in order, on columns [0, ncols) of
// every active matrix: one launch for a group of panels of the solves.
template <typename R>
__global__ __launch_bounds__(256) void lu_permute_group_kernel(cplx<R>* X, long ldx, long sX, int ncols,
                                                               const int* ipiv, int n, int nb, int p0, int p1,
                                                               const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  for (int p = p0; p < p1; ++p) {
    lu_permute_body<R>(X + (long)b * sX, ldx, ncols, ipiv + (long)b * n, p * nb, min(nb, n - p * nb),
                       blockIdx.x * SwCols<R>::v);
    __syncthreads();
  }
}

template <typename R>
static int launch_permute_group(cplx<R>* X, long ldx, long sX, int ncols, const int* ipiv, int n, int nb,
                                int p0, int p1, int batch, hipStream_t s, const int* active) {
  if (ncols <= 0 || p1 <= p0) return ST_OK;
  dim3 grid((unsigned)cdivl(ncols, SwCols<R>::v), (unsigned)batch);
  KernelTimer kt("lu_permute", s, 0.0, 4.0 * sizeof(cplx<R>) * nb * (double)(p1 - p0) * ncols * batch,
                 timers_on() ? std::string("lu_permute_group_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ">"
                             : std::string());
  hipLaunchKernelGGL((lu_permute_group_kernel<R>), grid, dim3(256), 0, s, X, ldx, sX, ncols, ipiv, n, nb, p0, p1,
                     active);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

template <typename R>
static int launch_permute(cplx<R>* X, long ldx, long sX, int ncols, const int* ipiv,
                          int ipiv_stride, int k, int nbe, int batch, hipStream_t s,
                          const int* active = nullptr) {
  if (ncols <= 0) return ST_OK;
  dim3 grid((unsigned)cdivl(ncols, SwCols<R>::v), (unsigned)batch);
  KernelTimer kt("lu_permute", s, 0.0, 4.0 * sizeof(cplx<R>) * nbe * (double)ncols * batch,
                 timers_on() ? std::string("lu_permute_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ">"
                             : std::string());
  hipLaunchKernelGGL((lu_permute_kernel<R>), grid, dim3(256), 0, s, X, ldx, sX, ncols, ipiv,
                     ipiv_stride, k, nbe, active);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// full_swap: the row order that the interchanges of panels p+1 .. np-1 give
// the L columns of panel p, as a gather G[b][p][r] (r in [k_{p+1}, n)): the
// entry that ends in row r comes from row G[b][p][r].  Built from the last
// panel backwards, g_p = sigma_{p+1} o g_{p+1}, where sigma_q(x) is the row
// found at x after panel q's swaps (ipiv[i] >= i, applied in order).  One
// workgroup per matrix; LDS holds g and sigma (2 n ints) and the panel's pivots.
__global__ __launch_bounds__(256) void lu_left_perm_kernel(const int* ipiv, int n, int nb, int* G) {
  extern __shared__ int sh[];
  __shared__ int s_pv[MAXNB];
  int* g = sh;
  int* sig = sh + n;
  const int b = blockIdx.x, tid = threadIdx.x, np = (n + nb - 1) / nb;
  const int* pv = ipiv + (long)b * n;
  int* Gb = G + (long)b * np * n;
  for (int r = tid; r < n; r += 256) g[r] = r;
  for (int p = np - 2; p >= 0; --p) {
    const int k = (p + 1) * nb, nbe = min(nb, n - k);
    for (int x = k + tid; x < n; x += 256) sig[x] = x;
    if (tid < nbe) s_pv[tid] = pv[k + tid];
    __syncthreads();
    if (tid == 0)
      for (int e = 0; e < nbe; ++e) {
        const int a = k + e, c = s_pv[e];
        if (c != a) { const int t = sig[a]; sig[a] = sig[c]; sig[c] = t; }
      }
    __syncthreads();
    for (int r = k + tid; r < n; r += 256) {
      const int v = sig[g[r]];
      g[r] = v;
      Gb[(long)p * n + r] = v;
    }
    __syncthreads();
  }
}

// Applies G to the L columns: column c of panel p = c / nb < np - 1, rows
// [k_{p+1}, n), gathered through registers (every read before any write);
// rows that keep their place are not touched.  With blocks of grp panels, p
// is the last panel of c's block.
constexpr int LGT = 1024;               // threads per column
constexpr int LGR = 4;                  // rows per thread: n - nb <= LGT * LGR
template <typename R>
__global__ __launch_bounds__(LGT) void lu_left_gather_kernel(cplx<R>* A, long lda, long sA, int n, int nb,
                                                             const int* G, int grp) {
  const int c = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, np = (n + nb - 1) / nb;
  // factored in blocks of grp panels, a panel's L columns already carry the
  // interchanges of its block's later panels: they take those of the panels
  // after the block, the composition stored for the block's last panel
  const int p = min(np - 1, (c / nb / grp + 1) * grp - 1);
  if (p >= np - 1) return;
  const int k1 = (p + 1) * nb;
  cplx<R>* col = A + (long)b * sA + (long)c * lda;
  const int* g = G + ((long)b * np + p) * n;
  cplx<R> v[LGR];
  int src[LGR];
#pragma unroll
  for (int i = 0; i < LGR; ++i) {
    const int r = k1 + tid + LGT * i;
    src[i] = (r < n) ? g[r] : r;
    if (src[i] != r) v[i] = col[src[i]];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < LGR; ++i) {
    const int r = k1 + tid + LGT * i;
    if (src[i] != r) col[r] = v[i];
  }
}

__global__ void zero_int_kernel(int* p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

template <typename R, int ROWS>
static int launch_panel_rows(const LUWork<R>& w, int k, int nbe, hipStream_t s) {
  // micro-panel width: the ROWS x W register block must fit the 128 VGPRs a
  // 1024-thread workgroup allows
  constexpr int W = (sizeof(R) == 8) ? (ROWS == 1 ? 8 : 8 / ROWS)
                                     : (ROWS == 1 ? 16 : 16 / ROWS);
  const long sD = (long)w.npanel() * 2 * w.nb * w.nb;
  cplx<R>* dslot = w.dinv + (long)(k / w.nb) * 2 * w.nb * w.nb;
  const std::string tn = std::string(w.tag) + "_panel";
  KernelTimer kt(tn.c_str(), s, 8.0 * nbe * nbe * (w.n - k) * w.batch / 2.0,
                 2.0 * sizeof(cplx<R>) * (double)(w.n - k) * nbe * w.batch,
                 timers_on() ? std::string("lu_panel_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                   std::to_string(ROWS) + ", " + std::to_string(W) + ">"
                             : std::string());
  hipLaunchKernelGGL((lu_panel_kernel<R, ROWS, W>), dim3(w.batch), dim3(PNT), 0, s, w.A, w.lda,
                     w.sA, w.n, k, nbe, w.nb, w.ipiv, dslot, sD, w.info);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

template <typename R>
static int launch_panel(const LUWork<R>& w, int k, int nbe, hipStream_t s) {
  const int m = w.n - k;
  if (m <= PNT) return launch_panel_rows<R, 1>(w, k, nbe, s);
  if (m <= 2 * PNT) return launch_panel_rows<R, 2>(w, k, nbe, s);
  if (m <= 4 * PNT) return launch_panel_rows<R, 4>(w, k, nbe, s);
  if constexpr (sizeof(R) == 4) {
    if (m > 8 * PNT) return launch_panel_rows<R, 16>(w, k, nbe, s);
  }
  return launch_panel_rows<R, 8>(w, k, nbe, s);
}

template <typename R>
int lu_factor(const LUWork<R>& w, hipStream_t s) {
  if (w.n <= 0 || w.batch <= 0) return ST_OK;
  if (w.n > lu_max_order<R>()) return set_error(ST_EINVAL, "lu_factor: n=%d exceeds %d", w.n, lu_max_order<R>());
  if (w.nb < 1 || w.nb > MAXNB) return set_error(ST_EINVAL, "lu_factor: nb=%d", w.nb);
  hipLaunchKernelGGL(zero_int_kernel, dim3((unsigned)cdivl(w.batch, 256)), dim3(256), 0, s,
                     w.info, w.batch);
  RSRR_LAUNCH_CHECK();
  const int n = w.n, nb = w.nb;
  const long sD = (long)w.npanel() * 2 * nb * nb;
  const std::string t_trsm = std::string(w.tag) + "_trsm", t_upd = std::string(w.tag) + "_update";
  // U12 = inv(L11) A12 on columns [c0, c0 + nc) (in place)
  auto trsm = [&](int k, int nbe, int c0, int nc, hipStream_t st) -> int {
    GemmBatch<R> g;
    g.M = nbe; g.N = nc; g.K = nbe;
    g.A = w.dinv + (long)(k / nb) * 2 * nb * nb; g.lda = nb; g.sA = sD;
    g.B = w.A + k + (long)c0 * w.lda; g.ldb = w.lda; g.sB = w.sA;
    g.C = w.A + k + (long)c0 * w.lda; g.ldc = w.lda; g.sC = w.sA;
    g.batch = w.batch;
    g.tag = t_trsm.c_str();
    g.gauss3m = w.gauss3m;
    return gemm_batched<R>(g, st);
  };
  // A22 -= L21 U12 on columns [c0, c0 + nc): rows [k + nbe, k + nbe + M) (M < 0:
  // to the last row), L21 = columns [k, k + nbe)
  auto update = [&](int k, int nbe, int c0, int nc, hipStream_t st, int M = -1) -> int {
    GemmBatch<R> u;
    u.M = M < 0 ? n - k - nbe : M; u.N = nc; u.K = nbe;
    u.alpha = mk<R>(-1, 0); u.beta = mk<R>(1, 0);
    u.A = w.A + (k + nbe) + (long)k * w.lda; u.lda = w.lda; u.sA = w.sA;
    u.B = w.A + k + (long)c0 * w.lda; u.ldb = w.lda; u.sB = w.sA;
    u.C = w.A + (k + nbe) + (long)c0 * w.lda; u.ldc = w.lda; u.sC = w.sA;
    u.batch = w.batch;
    u.tag = t_upd.c_str();
    u.gauss3m = w.gauss3m;
    return gemm_batched<R>(u, st);
  };
  // The trailing update on the look-ahead stream goes in column pieces of
  // about WINDOW_FLOP each: a panel queued on the other stream needs a whole
  // CU, which it finds only where one launch has drained and the next has
  // not begun.
  auto far_update = [&](int k, int K, int c0, int nc, hipStream_t st) -> int {
    int pw = nc;
    if (w.aux && st == w.aux) {
      const double fl = 8.0 * (double)(n - k - K) * nc * K * w.batch;
      const int np = (int)std::max(1.0, std::min(64.0, std::floor(fl / WINDOW_FLOP)));
      pw = std::max(256, (nc + np - 1) / np + 63) / 64 * 64;
    }
    for (int off = 0; off < nc; off += pw) RSRR_TRY(update(k, K, c0 + off, std::min(pw, nc - off), st));
    return ST_OK;
  };
  // With look-ahead, step k updates the next panel's columns on s and starts
  // the next panel at once, while the columns beyond it are updated on aux:
  //   s:   [wait aux(k-1)] next-panel permute/trsm/update, panel k+1, record main
  //   aux: wait main(panel k), far permute/trsm/update, record aux
  const bool la = (w.aux != nullptr && w.ev_main != nullptr && w.ev_aux != nullptr);
  bool aux_busy = false;
  const int SB0 = lu_group(nb);
  // full_swap: every panel's interchanges on all earlier L columns, after the
  // factorisation, as one gather per L column (lperm) or one permute per panel;
  // grp = panels per block, whose interchanges the L columns of a block
  // already took inside the block
  auto left_swaps = [&](int grp) -> int {
    const int np = w.npanel();
    if (w.lperm && np > 1 && n - nb <= LGT * LGR && 2 * (size_t)n * sizeof(int) <= 64 * 1024) {
      {
        KernelTimer kt("lu_permute", s, 0.0, 4.0 * (double)np * n * w.batch, "lu_left_perm_kernel");
        hipLaunchKernelGGL(lu_left_perm_kernel, dim3(w.batch), dim3(256), 2 * (size_t)n * sizeof(int), s, w.ipiv,
                           n, nb, w.lperm);
        RSRR_LAUNCH_CHECK();
      }
      const int lcols = (np - 1) * nb;
      KernelTimer kt("lu_permute", s, 0.0, 2.0 * sizeof(cplx<R>) * 0.5 * (double)n * lcols * w.batch,
                     timers_on() ? std::string("lu_left_gather_kernel<") + (sizeof(R) == 8 ? "double" : "float") +
                                       ">"
                                 : std::string());
      hipLaunchKernelGGL((lu_left_gather_kernel<R>), dim3(lcols, w.batch), dim3(LGT), 0, s, w.A, w.lda, w.sA, n,
                         nb, w.lperm, grp);
      RSRR_LAUNCH_CHECK();
      return ST_OK;
    }
    for (int q = 1; q < np; ++q) {
      const int cols = (q / grp) * grp * nb;      // the L columns of the earlier blocks
      if (cols > 0)
        RSRR_TRY(launch_permute<R>(w.A, w.lda, w.sA, cols, w.ipiv, n, q * nb, min(nb, n - q * nb), w.batch, s));
    }
    return ST_OK;
  };
  if (w.pair && SB0 >= 2) {
    // Blocks of P = SB0 panels (the solver's groups of 256 columns).  Inside
    // a block, each panel once factored updates the block's later columns
    // (right-looking: interchanges, U rows, the rows below), and its
    // interchanges are applied to the block's earlier L columns, so that all
    // L columns of the block share one row order.  Every column beyond the
    // block then takes the block's interchanges, its U rows (panel by panel:
    // U_q = inv(L_qq) A_q, then the rows of the later panels of the block
    // take panel q's update) and one product with K = P nb for all rows
    // below the block: the trailing matrix is read and written once per 256
    // columns, by products four times as deep as single panels (for
    // nb = 64).  Look-ahead at the level of blocks: the next block's columns
    // on s, the columns beyond them on aux.
    const int P = SB0, BW = P * nb;
    auto tail = [&](int k, int c0, int nc, hipStream_t st) -> int {
      if (nc <= 0) return ST_OK;
      const int kend = min(n, k + BW);
      for (int kq = k; kq < kend; kq += nb)
        RSRR_TRY(launch_permute<R>(w.A + (long)c0 * w.lda, w.lda, w.sA, nc, w.ipiv, n, kq, min(nb, n - kq),
                                   w.batch, st));
      for (int kq = k; kq < kend; kq += nb) {
        const int nq = min(nb, n - kq);
        RSRR_TRY(trsm(kq, nq, c0, nc, st));
        if (kq + nq < kend) RSRR_TRY(update(kq, nq, c0, nc, st, kend - kq - nq));
      }
      if (kend < n) RSRR_TRY(far_update(k, kend - k, c0, nc, st));
      return ST_OK;
    };
    RSRR_TRY(launch_panel<R>(w, 0, min(nb, n), s));
    for (int k = 0; k < n; k += BW) {
      const int kend = min(n, k + BW);
      for (int kq = k + nb; kq < kend; kq += nb) {
        // the previous panel's update on the block's remaining columns,
        // then this panel, then its interchanges on the block's earlier L columns
        const int kp = kq - nb, rem = kend - kq;
        RSRR_TRY(launch_permute<R>(w.A + (long)kq * w.lda, w.lda, w.sA, rem, w.ipiv, n, kp, nb, w.batch, s));
        RSRR_TRY(trsm(kp, nb, kq, rem, s));
        RSRR_TRY(update(kp, nb, kq, rem, s));
        RSRR_TRY(launch_panel<R>(w, kq, min(nb, n - kq), s));
        RSRR_TRY(launch_permute<R>(w.A + (long)k * w.lda, w.lda, w.sA, kq - k, w.ipiv, n, kq, min(nb, n - kq),
                                   w.batch, s));
      }
      const int rest = n - kend;
      if (rest <= 0) break;
      const int nxt = la ? min(BW, rest) : rest;
      const int far = rest - nxt;
      if (aux_busy) {              // the next block's columns had the previous block's far update
        RSRR_HIP(hipStreamWaitEvent(s, w.ev_aux, 0));
        aux_busy = false;
      }
      if (far > 0) {
        RSRR_HIP(hipEventRecord(w.ev_main, s));
        RSRR_HIP(hipStreamWaitEvent(w.aux, w.ev_main, 0));
        RSRR_TRY(tail(k, kend + nxt, far, w.aux));
        RSRR_HIP(hipEventRecord(w.ev_aux, w.aux));
        aux_busy = true;
      }
      RSRR_TRY(tail(k, kend, nxt, s));
      RSRR_TRY(launch_panel<R>(w, kend, min(nb, n - kend), s));
    }
    if (aux_busy) RSRR_HIP(hipStreamWaitEvent(s, w.ev_aux, 0));
    return w.full_swap ? left_swaps(P) : ST_OK;
  }
  RSRR_TRY(launch_panel<R>(w, 0, min(nb, n), s));
  if (la) RSRR_HIP(hipEventRecord(w.ev_main, s));
  for (int k = 0; k < n; k += nb) {
    const int nbe = min(nb, n - k);
    const int rest = n - k - nbe;
    if (rest <= 0) break;
    const int c1 = k + nbe;
    const int nxt = la ? min(nb, rest) : rest;
    const int far = rest - nxt;
    if (aux_busy) {              // the next panel's columns had step k-1's far update
      RSRR_HIP(hipStreamWaitEvent(s, w.ev_aux, 0));
      aux_busy = false;
    }
    if (far > 0) {
      RSRR_HIP(hipStreamWaitEvent(w.aux, w.ev_main, 0));
      RSRR_TRY(launch_permute<R>(w.A + (long)(c1 + nxt) * w.lda, w.lda, w.sA, far, w.ipiv, n, k, nbe,
                                 w.batch, w.aux));
      RSRR_TRY(trsm(k, nbe, c1 + nxt, far, w.aux));
      RSRR_TRY(far_update(k, nbe, c1 + nxt, far, w.aux));
      RSRR_HIP(hipEventRecord(w.ev_aux, w.aux));
      aux_busy = true;
    }
    RSRR_TRY(launch_permute<R>(w.A + (long)c1 * w.lda, w.lda, w.sA, nxt, w.ipiv, n, k, nbe, w.batch, s));
    RSRR_TRY(trsm(k, nbe, c1, nxt, s));
    RSRR_TRY(update(k, nbe, c1, nxt, s));
    if (c1 < n) {
      RSRR_TRY(launch_panel<R>(w, c1, min(nb, n - c1), s));
      if (la) RSRR_HIP(hipEventRecord(w.ev_main, s));
    }
  }
  if (aux_busy) RSRR_HIP(hipStreamWaitEvent(s, w.ev_aux, 0));
  // Within every group of lu_group(nb) panels, the interchanges of a panel are also
  // applied to the L columns of the group's earlier panels, so that all L
  // columns of a group share one row order (that after its last panel) and
  // the solver can update the rows below a group with one product.  Rows of a
  // panel's own diagonal block are never touched, so L stays unit lower
  // triangular and dinv is unchanged.
  if (w.full_swap) return left_swaps(1);
  const int np = w.npanel(), SB = lu_group(nb);
  for (int q = 1; q < np; ++q) {
    if (q % SB == 0) continue;
    const int k = q * nb, c0 = (q / SB) * SB * nb;
    RSRR_TRY(launch_permute<R>(w.A + (long)c0 * w.lda, w.lda, w.sA, k - c0, w.ipiv, n, k, min(nb, n - k),
                               w.batch, s));
  }
  return ST_OK;
}

template <typename R>
int lu_solve(const LUWork<R>& w, cplx<R>* B, long ldb, long sB, int nrhs, hipStream_t s, const int* active) {
  if (w.n <= 0 || w.batch <= 0 || nrhs <= 0) return ST_OK;
  const int n = w.n, nb = w.nb, np = w.npanel(), SB = lu_group(nb);
  const std::string t_solve = std::string(w.tag) + "_solve";
  const long sD = (long)np * 2 * nb * nb;
  // C[rows] = alpha A B + beta C on the batch (A from the factors or dinv)
  auto mm = [&](int M, int K, const cplx<R>* A, long lda, long sA, const cplx<R>* Bp, cplx<R>* Cp, bool acc) {
    GemmBatch<R> g;
    g.M = M; g.N = nrhs; g.K = K;
    if (acc) { g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0); }
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = Bp; g.ldb = ldb; g.sB = sB;
    g.C = Cp; g.ldc = ldb; g.sC = sB;
    g.batch = w.batch;
    g.tag = t_solve.c_str();
    g.gauss3m = w.gauss3m;
    g.active = active;
    return gemm_batched<R>(g, s);
  };
  // the triangular solves and updates inside a group, one launch
  LUGroupSolve<R> gq;
  gq.A = w.A; gq.lda = w.lda; gq.sA = w.sA;
  gq.dinv = w.dinv; gq.sD = sD;
  gq.B = B; gq.ldb = ldb; gq.sB = sB;
  gq.n = n; gq.nb = nb; gq.nrhs = nrhs; gq.batch = w.batch;
  gq.gauss3m = w.gauss3m; gq.active = active; gq.tag = t_solve.c_str();
  // forward, L: per group of lu_group(nb) panels (the row order lu_factor gives its L
  // columns): the group's interchanges on B, the triangular solves with the
  // diagonal-block inverses and updates inside the group, then the rows below
  // the group in one product with K = the group's width
  for (int p0 = 0; p0 < np; p0 += SB) {
    const int p1 = min(np, p0 + SB);
    const int k0 = p0 * nb, k1 = min(n, p1 * nb);
    RSRR_TRY(launch_permute_group<R>(B, ldb, sB, nrhs, w.ipiv, n, nb, p0, p1, w.batch, s, active));
    gq.p0 = p0; gq.p1 = p1; gq.lower = true;
    RSRR_TRY(lu_group_solve<R>(gq, s));
    if (k1 < n) RSRR_TRY(mm(n - k1, k1 - k0, w.A + k1 + (long)k0 * w.lda, w.lda, w.sA, B + k0, B + k1, true));
  }
  // backward, U: per group from the last, solves and updates inside the
  // group, then the rows above it in one product
  for (int p0 = ((np - 1) / SB) * SB; p0 >= 0; p0 -= SB) {
    const int p1 = min(np, p0 + SB);
    const int k0 = p0 * nb, k1 = min(n, p1 * nb);
    gq.p0 = p0; gq.p1 = p1; gq.lower = false;
    RSRR_TRY(lu_group_solve<R>(gq, s));
    if (k0 > 0) RSRR_TRY(mm(k0, k1 - k0, w.A + (long)k0 * w.lda, w.lda, w.sA, B + k0, B, true));
  }
  return ST_OK;
}

// perm_b: the row order of P A = L U, composed from the interchanges
// (row i of P A is row perm[i] of A); one thread per matrix.
__global__ void lu_perm_kernel(const int* ipiv, int n, int batch, int* perm) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int* pv = ipiv + (long)b * n;
  int* pm = perm + (long)b * n;
  for (int i = 0; i < n; ++i) pm[i] = i;
  for (int i = 0; i < n; ++i) {
    const int p = pv[i];
    if (p != i) { const int t = pm[i]; pm[i] = pm[p]; pm[p] = t; }
  }
}

// out_b[:, perm_b[k]] = X_b[:, k]: column k of U^{-1} L^{-1} is column perm[k]
// of A^{-1}.  One workgroup per (column, matrix).
template <typename R>
__global__ __launch_bounds__(256) void scatter_cols_kernel(const cplx<R>* X, int n, const int* perm, cplx<R>* out,
                                                           long ldo, long sO) {
  const int k = blockIdx.x, b = blockIdx.y;
  const cplx<R>* src = X + (long)b * n * n + (long)k * n;
  cplx<R>* dst = out + (long)b * sO + (long)perm[(long)b * n + k] * ldo;
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void identity_batch_kernel(double* X, int n, long total_re) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;   // over batch * n * n complex
  if (e >= total_re) return;
  const long nn = (long)n * n, q = e % nn;
  X[2 * e] = (q % n == q / n) ? 1.0 : 0.0;
  X[2 * e + 1] = 0.0;
}

template <typename R>
int lu_inverse(const LUWork<R>& w, cplx<R>* X, cplx<R>* out, long ldo, long sO, int* perm, hipStream_t s) {
  static_assert(sizeof(R) == 8, "complex128 only");
  if (w.n <= 0 || w.batch <= 0) return ST_OK;
  if (!w.full_swap) return set_error(ST_EINVAL, "lu_inverse needs factors computed with full_swap");
  const int n = w.n, nb = w.nb, np = w.npanel(), SB = lu_group(nb);
  const long nn = (long)n * n;
  const std::string t_solve = std::string(w.tag) + "_solve";
  const long sD = (long)np * 2 * nb * nb;
  {
    const long tot = nn * w.batch;
    hipLaunchKernelGGL(identity_batch_kernel, dim3((unsigned)cdivl(tot, 256)), dim3(256), 0, s, (double*)X, n, tot);
    RSRR_LAUNCH_CHECK();
  }
  // C[rows, 0:N) = alpha A B + beta C on the batch, X with ld n
  auto mm = [&](int M, int N, int K, const cplx<R>* A, long lda, long sA, const cplx<R>* Bp, cplx<R>* Cp,
                bool acc) {
    GemmBatch<R> g;
    g.M = M; g.N = N; g.K = K;
    if (acc) { g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0); }
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = Bp; g.ldb = n; g.sB = nn;
    g.C = Cp; g.ldc = n; g.sC = nn;
    g.batch = w.batch;
    g.tag = t_solve.c_str();
    g.gauss3m = w.gauss3m;
    return gemm_batched<R>(g, s);
  };
  // forward, L Y = I: rows of panel p of Y vanish beyond column p*nb + nbe
  // (L^{-1} is lower triangular), so every product stops at that column
  for (int p0 = 0; p0 < np; p0 += SB) {
    const int p1 = min(np, p0 + SB);
    const int k0 = p0 * nb, k1 = min(n, p1 * nb);
    for (int p = p0; p < p1; ++p) {
      const int k = p * nb, nbe = min(nb, n - k);
      RSRR_TRY(mm(nbe, k + nbe, nbe, w.dinv + (long)p * 2 * nb * nb, nb, sD, X + k, X + k, false));
      if (k + nbe < k1)
        RSRR_TRY(mm(k1 - k - nbe, k + nbe, nbe, w.A + (k + nbe) + (long)k * w.lda, w.lda, w.sA, X + k,
                    X + k + nbe, true));
    }
    if (k1 < n) RSRR_TRY(mm(n - k1, k1, k1 - k0, w.A + k1 + (long)k0 * w.lda, w.lda, w.sA, X + k0, X + k1, true));
  }
  // backward, U Z = Y (dense)
  for (int p0 = ((np - 1) / SB) * SB; p0 >= 0; p0 -= SB) {
    const int p1 = min(np, p0 + SB);
    const int k0 = p0 * nb, k1 = min(n, p1 * nb);
    for (int p = p1 - 1; p >= p0; --p) {
      const int k = p * nb, nbe = min(nb, n - k);
      RSRR_TRY(mm(nbe, n, nbe, w.dinv + (long)p * 2 * nb * nb + (long)nb * nb, nb, sD, X + k, X + k, false));
      if (k > k0) RSRR_TRY(mm(k - k0, n, nbe, w.A + k0 + (long)k * w.lda, w.lda, w.sA, X + k, X + k0, true));
    }
    if (k0 > 0) RSRR_TRY(mm(k0, n, k1 - k0, w.A + (long)k0 * w.lda, w.lda, w.sA, X + k0, X, true));
  }
  hipLaunchKernelGGL(lu_perm_kernel, dim3((unsigned)cdivl(w.batch, 64)), dim3(64), 0, s, w.ipiv, n, w.batch, perm);
  RSRR_LAUNCH_CHECK();
  hipLaunchKernelGGL((scatter_cols_kernel<R>), dim3(n, w.batch), dim3(256), 0, s, X, n, perm, out, ldo, sO);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

// ---------------------------------------------------------------------------
// Several strided batches of different orders factored as one set of launches
// per panel step (see kernels.h).  The operations and their order per matrix
// are those of lu_factor with blocks of panels and look-ahead, so each matrix
// is factored bit for bit as lu_factor factors it alone.
namespace {

template <typename R> LUSegDev<R> seg_of(const LUWork<R>& w) {
  LUSegDev<R> d;
  d.A = w.A; d.lda = w.lda; d.sA = w.sA; d.n = w.n; d.ipiv = w.ipiv; d.dinv = w.dinv;
  d.sD = (long)w.npanel() * 2 * w.nb * w.nb; d.info = w.info;
  d.c0 = d.ncols = d.k = d.nbe = 0;
  return d;
}

// one launch per MAXSEG entries of `list`; grid rows are the matrices
template <typename R, typename F>
int seg_chunks(const std::vector<LUSegDev<R>>& list, const std::vector<int>& batch, F launch) {
  for (size_t i0 = 0; i0 < list.size(); i0 += MAXSEG) {
    LUSegArgs<R> a;
    a.count = 0;
    int tot = 0, maxc = 0;
    for (size_t i = i0; i < list.size() && i < i0 + MAXSEG; ++i) {
      a.first[a.count] = tot;
      a.seg[a.count] = list[i];
      tot += batch[i];
      maxc = std::max(maxc, list[i].ncols);
      ++a.count;
    }
    a.first[a.count] = tot;
    RSRR_TRY(launch(a, tot, maxc));
  }
  return ST_OK;
}

template <typename R, int ROWS>
int launch_panel_seg_rows(const LUSegArgs<R>& a, int tot, int k, int nb, const char* tag, double flops,
                          double bytes, hipStream_t s) {
  constexpr int W = (sizeof(R) == 8) ? (ROWS == 1 ? 8 : 8 / ROWS) : (ROWS == 1 ? 16 : 16 / ROWS);
  const std::string tn = std::string(tag) + "_panel";
  KernelTimer kt(tn.c_str(), s, flops, bytes,
                 timers_on() ? std::string("lu_panel_seg_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                   std::to_string(ROWS) + ", " + std::to_string(W) + ">"
                             : std::string());
  hipLaunchKernelGGL((lu_panel_seg_kernel<R, ROWS, W>), dim3(tot), dim3(PNT), 0, s, a, k, nb);
  RSRR_LAUNCH_CHECK();
  return ST_OK;
}

}  // namespace

template <typename R>
int lu_factor_segments(const std::vector<LUWork<R>>& ws, hipStream_t s, hipStream_t aux, hipEvent_t ev_main,
                       hipEvent_t ev_aux) {
  if (ws.empty()) return ST_OK;
  const int nb = ws[0].nb;
  const bool g3m = ws[0].gauss3m;
  int nmax = 0;
  for (const LUWork<R>& w : ws) {
    if (w.nb != nb || w.gauss3m != g3m || w.full_swap)
      return set_error(ST_EINVAL, "lu_factor_segments: batches must share nb and the product form");
    if (w.n > lu_max_order<R>() || w.n < 1 || w.batch < 1) return set_error(ST_EINVAL, "lu_factor_segments: n=%d", w.n);
    nmax = std::max(nmax, w.n);
  }
  if (nb < 1 || nb > MAXNB || lu_group(nb) < 2) return set_error(ST_EINVAL, "lu_factor_segments: nb=%d", nb);
  const int P = lu_group(nb), BW = P * nb;      // blocks of panels, as lu_factor
  for (const LUWork<R>& w : ws) {
    hipLaunchKernelGGL(zero_int_kernel, dim3((unsigned)cdivl(w.batch, 256)), dim3(256), 0, s, w.info, w.batch);
    RSRR_LAUNCH_CHECK();
  }
  const int Q = (int)ws.size();
  const std::string t_trsm = std::string(ws[0].tag) + "_trsm", t_upd = std::string(ws[0].tag) + "_update";
  const bool la = aux && ev_main && ev_aux;
  bool aux_busy = false;
  // panels at column k of every batch whose order exceeds k, one launch per
  // register class (rows per thread) and MAXSEG batches
  auto panels = [&](int k, hipStream_t st) -> int {
    for (int rows : {1, 2, 4, 8, 16}) {
      std::vector<LUSegDev<R>> list;
      std::vector<int> bt;
      double fl = 0, by = 0;
      for (const LUWork<R>& w : ws) {
        const int m = w.n - k;
        if (m <= 0) continue;
        const int cls = m <= PNT ? 1 : m <= 2 * PNT ? 2 : m <= 4 * PNT ? 4 : m <= 8 * PNT ? 8 : 16;
        if (cls != rows) continue;
        list.push_back(seg_of(w));
        bt.push_back(w.batch);
        const int nbe = std::min(nb, m);
        fl += 8.0 * nbe * nbe * m * w.batch / 2.0;
        by += 2.0 * sizeof(cplx<R>) * (double)m * nbe * w.batch;
      }
      RSRR_TRY(seg_chunks<R>(list, bt, [&](const LUSegArgs<R>& a, int tot, int) -> int {
        switch (rows) {
          case 1: return launch_panel_seg_rows<R, 1>(a, tot, k, nb, ws[0].tag, fl, by, st);
          case 2: return launch_panel_seg_rows<R, 2>(a, tot, k, nb, ws[0].tag, fl, by, st);
          case 4: return launch_panel_seg_rows<R, 4>(a, tot, k, nb, ws[0].tag, fl, by, st);
          case 8: return launch_panel_seg_rows<R, 8>(a, tot, k, nb, ws[0].tag, fl, by, st);
          default:
            if constexpr (sizeof(R) == 4) return launch_panel_seg_rows<R, 16>(a, tot, k, nb, ws[0].tag, fl, by, st);
            return set_error(ST_EINVAL, "lu_factor_segments: order above %d", lu_max_order<R>());
        }
      }));
    }
    return ST_OK;
  };
  // row interchanges: (batch q, first column, columns, panel k, its width)
  struct PJob { int q, c0, ncols, k, nbe; };
  auto permutes = [&](const std::vector<PJob>& jobs, hipStream_t st) -> int {
    std::vector<LUSegDev<R>> list;
    std::vector<int> bt;
    double by = 0;
    for (const PJob& j : jobs) {
      if (j.ncols <= 0 || j.nbe <= 0) continue;
      LUSegDev<R> d = seg_of(ws[j.q]);
      d.c0 = j.c0; d.ncols = j.ncols; d.k = j.k; d.nbe = j.nbe;
      list.push_back(d);
      bt.push_back(ws[j.q].batch);
      by += 4.0 * sizeof(cplx<R>) * j.nbe * (double)j.ncols * ws[j.q].batch;
    }
    return seg_chunks<R>(list, bt, [&](const LUSegArgs<R>& a, int tot, int maxc) -> int {
      KernelTimer kt("lu_permute", st, 0.0, by,
                     timers_on() ? std::string("lu_permute_seg_kernel<") + (sizeof(R) == 8 ? "double" : "float") + ">"
                                 : std::string());
      hipLaunchKernelGGL((lu_permute_seg_kernel<R>), dim3((unsigned)cdivl(maxc, SwCols<R>::v), (unsigned)tot),
                         dim3(256), 0, st, a);
      RSRR_LAUNCH_CHECK();
      return ST_OK;
    });
  };
  // products, GSEG batches per launch
  auto gemms = [&](const std::vector<GemmBatch<R>>& list, hipStream_t st) -> int {
    for (size_t i0 = 0; i0 < list.size(); i0 += GSEG) {
      GemmSegs<R> sg;
      for (size_t i = i0; i < list.size() && i < i0 + GSEG; ++i) sg.g[sg.count++] = list[i];
      RSRR_TRY(gemm_segments<R>(sg, st));
    }
    return ST_OK;
  };
  // U rows = inv(L_diag) A rows (in place) for batch q, panel at k of width nbe, columns [c0, c0 + nc)
  auto trsm_g = [&](int q, int k, int nbe, int c0, int nc) {
    const LUWork<R>& w = ws[q];
    GemmBatch<R> g;
    g.M = nbe; g.N = nc; g.K = nbe;
    g.A = w.dinv + (long)(k / nb) * 2 * nb * nb; g.lda = nb; g.sA = (long)w.npanel() * 2 * nb * nb;
    g.B = w.A + k + (long)c0 * w.lda; g.ldb = w.lda; g.sB = w.sA;
    g.C = w.A + k + (long)c0 * w.lda; g.ldc = w.lda; g.sC = w.sA;
    g.batch = w.batch;
    g.tag = t_trsm.c_str();
    g.gauss3m = g3m;
    return g;
  };
  // rows [k + nbe, k + nbe + M) -= L(:, k .. k+nbe) U(k .. k+nbe, columns)
  auto upd_g = [&](int q, int k, int nbe, int c0, int nc, int M) {
    const LUWork<R>& w = ws[q];
    GemmBatch<R> u;
    u.M = M; u.N = nc; u.K = nbe;
    u.alpha = mk<R>(-1, 0); u.beta = mk<R>(1, 0);
    u.A = w.A + (k + nbe) + (long)k * w.lda; u.lda = w.lda; u.sA = w.sA;
    u.B = w.A + k + (long)c0 * w.lda; u.ldb = w.lda; u.sB = w.sA;
    u.C = w.A + (k + nbe) + (long)c0 * w.lda; u.ldc = w.lda; u.sC = w.sA;
    u.batch = w.batch;
    u.tag = t_upd.c_str();
    u.gauss3m = g3m;
    return u;
  };
  // the block at k applied to columns [c0[q], c0[q] + nc[q]) of every batch
  // with nc > 0: its interchanges panel by panel, the U rows of its panels
  // (each followed by its update of the later panels' rows), one product below
  auto tail = [&](int k, const std::vector<int>& c0, const std::vector<int>& nc, hipStream_t st) -> int {
    for (int kq = k; kq < k + BW; kq += nb) {
      std::vector<PJob> pj;
      for (int q = 0; q < Q; ++q)
        if (nc[q] > 0 && kq < ws[q].n) pj.push_back(PJob{q, c0[q], nc[q], kq, std::min(nb, ws[q].n - kq)});
      RSRR_TRY(permutes(pj, st));
    }
    for (int kq = k; kq < k + BW; kq += nb) {
      std::vector<GemmBatch<R>> tq, uq;
      for (int q = 0; q < Q; ++q) {
        const int n = ws[q].n;
        if (nc[q] <= 0 || kq >= n) continue;
        const int nq = std::min(nb, n - kq), kend = std::min(n, k + BW);
        tq.push_back(trsm_g(q, kq, nq, c0[q], nc[q]));
        if (kq + nq < kend) uq.push_back(upd_g(q, kq, nq, c0[q], nc[q], kend - kq - nq));
      }
      RSRR_TRY(gemms(tq, st));
      RSRR_TRY(gemms(uq, st));
    }
    // the product below the block; on the look-ahead stream in column
    // pieces of about WINDOW_FLOP together, as lu_factor does
    double fl = 0;
    for (int q = 0; q < Q; ++q) {
      const int n = ws[q].n, kend = std::min(n, k + BW);
      if (nc[q] > 0 && kend < n) fl += 8.0 * (double)(n - kend) * nc[q] * (kend - k) * ws[q].batch;
    }
    const int np = (la && st == aux) ? (int)std::max(1.0, std::min(64.0, std::floor(fl / WINDOW_FLOP))) : 1;
    for (int p = 0; p < np; ++p) {
      std::vector<GemmBatch<R>> big;
      for (int q = 0; q < Q; ++q) {
        const int n = ws[q].n, kend = std::min(n, k + BW);
        if (nc[q] <= 0 || kend >= n) continue;
        const int pw = std::max(256, (nc[q] + np - 1) / np + 63) / 64 * 64;
        const int off = p * pw;
        if (off < nc[q]) big.push_back(upd_g(q, k, kend - k, c0[q] + off, std::min(pw, nc[q] - off), n - kend));
      }
      RSRR_TRY(gemms(big, st));
    }
    return ST_OK;
  };

  RSRR_TRY(panels(0, s));
  for (int k = 0; k < nmax; k += BW) {
    // the block's later panels: the previous panel's update on the block's
    // remaining columns, the panel, its interchanges on the block's earlier L columns
    for (int kq = k + nb; kq < k + BW && kq < nmax; kq += nb) {
      std::vector<PJob> pb, fix;
      std::vector<GemmBatch<R>> tr, up;
      for (int q = 0; q < Q; ++q) {
        const int n = ws[q].n;
        if (kq >= n) continue;
        const int kp = kq - nb, rem = std::min(n, k + BW) - kq;
        pb.push_back(PJob{q, kq, rem, kp, nb});
        tr.push_back(trsm_g(q, kp, nb, kq, rem));
        up.push_back(upd_g(q, kp, nb, kq, rem, n - kp - nb));
        fix.push_back(PJob{q, k, kq - k, kq, std::min(nb, n - kq)});
      }
      if (pb.empty()) continue;
      RSRR_TRY(permutes(pb, s));
      RSRR_TRY(gemms(tr, s));
      RSRR_TRY(gemms(up, s));
      RSRR_TRY(panels(kq, s));
      RSRR_TRY(permutes(fix, s));
    }
    std::vector<int> nx0(Q, 0), nxc(Q, 0), fr0(Q, 0), frc(Q, 0);
    bool anyrest = false, anyfar = false;
    for (int q = 0; q < Q; ++q) {
      const int n = ws[q].n;
      if (k >= n) continue;
      const int kend = std::min(n, k + BW), rest = n - kend;
      if (rest <= 0) continue;
      const int nxt = la ? std::min(BW, rest) : rest;
      nx0[q] = kend; nxc[q] = nxt;
      fr0[q] = kend + nxt; frc[q] = rest - nxt;
      anyrest = true;
      anyfar |= frc[q] > 0;
    }
    if (!anyrest) continue;
    if (aux_busy) {
      RSRR_HIP(hipStreamWaitEvent(s, ev_aux, 0));
      aux_busy = false;
    }
    if (anyfar) {
      RSRR_HIP(hipEventRecord(ev_main, s));
      RSRR_HIP(hipStreamWaitEvent(aux, ev_main, 0));
      RSRR_TRY(tail(k, fr0, frc, aux));
      RSRR_HIP(hipEventRecord(ev_aux, aux));
      aux_busy = true;
    }
    RSRR_TRY(tail(k, nx0, nxc, s));
    RSRR_TRY(panels(k + BW, s));
  }
  if (aux_busy) RSRR_HIP(hipStreamWaitEvent(s, ev_aux, 0));
  return ST_OK;
}
template int lu_factor_segments<double>(const std::vector<LUWork<double>>&, hipStream_t, hipStream_t, hipEvent_t,
                                        hipEvent_t);
template int lu_factor_segments<float>(const std::vector<LUWork<float>>&, hipStream_t, hipStream_t, hipEvent_t,
                                       hipEvent_t);

template int lu_factor<double>(const LUWork<double>&, hipStream_t);
template int lu_factor<float>(const LUWork<float>&, hipStream_t);
template int lu_solve<double>(const LUWork<double>&, c128*, long, long, int, hipStream_t, const int*);
template int lu_solve<float>(const LUWork<float>&, c64*, long, long, int, hipStream_t, const int*);
template int lu_inverse<double>(const LUWork<double>&, c128*, c128*, long, long, int*, hipStream_t);

}  // namespace rsrr
