// Shared device/host helpers for the RSRR library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace rsrr {

// ------------------------------------------------------------ complex types
// Interleaved (re, im) storage, the same bytes as std::complex / torch complex.
template <typename R> struct cplx { R re, im; };
typedef cplx<double> c128;
typedef cplx<float> c64;

template <typename R> __host__ __device__ inline cplx<R> mk(R a, R b) { cplx<R> z; z.re = a; z.im = b; return z; }
template <typename R> __host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename R> __host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename R> __host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R> __host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return mk(s * a.re, s * a.im); }
template <typename R> __host__ __device__ inline cplx<R> conj(cplx<R> a) { return mk(a.re, -a.im); }
template <typename R> __host__ __device__ inline R abs2(cplx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R> __host__ __device__ inline R cabs1(cplx<R> a) { return fabs(a.re) + fabs(a.im); }
// a * conj(b) and conj(a) * b
template <typename R> __host__ __device__ inline cplx<R> mulc(cplx<R> a, cplx<R> b) {
  return mk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename R> __host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {  // conj(a)*b
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// Smith's algorithm for a / b.
template <typename R> __host__ __device__ inline cplx<R> cdiv(cplx<R> a, cplx<R> b) {
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, d = b.re + b.im * r;
    return mk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  } else {
    R r = b.re / b.im, d = b.re * r + b.im;
    return mk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
  }
}
template <typename R> __host__ __device__ inline cplx<R> crecip(cplx<R> b) { return cdiv(mk<R>(1, 0), b); }

template <typename D, typename S> __host__ __device__ inline cplx<D> ccast(cplx<S> a) {
  return mk<D>((D)a.re, (D)a.im);
}

// ------------------------------------------------------------- status codes
enum {
  ST_OK = 0, ST_EINVAL = -1, ST_ENOMEM = -2, ST_EHIP = -3, ST_ESINGULAR = -4,
  ST_EBUSY = -5, ST_ENOTCONV = -6, ST_ETIMEDOUT = -7
};

// Records an error message in thread-local storage; returns code.
int set_error(int code, const char* fmt, ...);

#define RSRR_HIP(call)                                                         \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::rsrr::set_error(::rsrr::ST_EHIP, "%s:%d %s: %s", __FILE__,      \
                               __LINE__, #call, hipGetErrorString(e_));        \
  } while (0)

#define RSRR_TRY(call)                                                         \
  do {                                                                         \
    int s_ = (call);                                                           \
    if (s_ < 0) return s_;                                                     \
  } while (0)

#define RSRR_LAUNCH_CHECK()                                                    \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess)                                                      \
      return ::rsrr::set_error(::rsrr::ST_EHIP, "%s:%d launch: %s", __FILE__,  \
                               __LINE__, hipGetErrorString(e_));               \
  } while (0)

inline long cdivl(long a, long b) { return (a + b - 1) / b; }

// Orders LDS accesses between the lanes of one wavefront (64 lanes run in
// lock step; this keeps the compiler and the memory pipeline from reordering).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pivot searches.  A non-negative magnitude is compared through the bits of a
// non-negative float (exact) or the high word of a non-negative double (a
// pivot within a relative 2^-20 of the column maximum, which keeps the growth
// bound of partial pivoting).  Maxima over a wave use DPP moves inside rows of
// 16 lanes (quad xor 1, quad xor 2, half-row mirror, row mirror) and the four
// row results by readlane: no LDS round trips.
__device__ inline unsigned mag_bits(float v) { return __float_as_uint(v); }
__device__ inline unsigned mag_bits(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
}
__device__ inline unsigned row16_umax_all(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  return v;
}
__device__ inline unsigned wave_umax(unsigned v) {
  v = row16_umax_all(v);
  const unsigned a = __builtin_amdgcn_readlane((int)v, 0), b = __builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = __builtin_amdgcn_readlane((int)v, 32), d = __builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

}  // namespace rsrr
