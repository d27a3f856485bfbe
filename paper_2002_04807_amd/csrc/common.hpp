// Shared device/host helpers for the FEAST contour-integration library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

namespace mf {

// ---------------------------------------------------------------------------
// small complex type (interleaved re, im) usable in device and host code
// ---------------------------------------------------------------------------
template <typename R>
struct cplx {
  R re, im;
  cplx() = default;
  __host__ __device__ cplx(R r, R i = R(0)) : re(r), im(i) {}
};

template <typename R> __host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __host__ __device__ inline cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
template <typename R> __host__ __device__ inline R abs1(cplx<R> a) { return fabs(a.re) + fabs(a.im); }
template <typename R> __host__ __device__ inline R norm2(cplx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R> __host__ __device__ inline cplx<R> cdiv(cplx<R> a, cplx<R> b) {
  // Smith's algorithm (scaled division) for a / b
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    R r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}

// scalar traits: "real" overloads so templated code can treat double and cplx alike
__host__ __device__ inline double conj(double a) { return a; }
__host__ __device__ inline float conj(float a) { return a; }
__host__ __device__ inline double norm2(double a) { return a * a; }
__host__ __device__ inline double abs1(double a) { return fabs(a); }
__host__ __device__ inline double real_part(double a) { return a; }
__host__ __device__ inline float norm2(float a) { return a * a; }
__host__ __device__ inline float abs1(float a) { return fabsf(a); }
__host__ __device__ inline float real_part(float a) { return a; }
__host__ __device__ inline double cdiv(double a, double b) { return a / b; }
__host__ __device__ inline float cdiv(float a, float b) { return a / b; }
template <typename R> __host__ __device__ inline R real_part(cplx<R> a) { return a.re; }

using c32 = cplx<float>;
using c64 = cplx<double>;

template <typename T> struct is_cplx { static constexpr bool value = false; };
template <typename R> struct is_cplx<cplx<R>> { static constexpr bool value = true; };
template <typename T> struct real_of { using type = T; };
template <typename R> struct real_of<cplx<R>> { using type = R; };

// conversions between precisions
template <typename To, typename From> __host__ __device__ inline To convert(From a);
template <> __host__ __device__ inline c32 convert<c32, c64>(c64 a) { return {(float)a.re, (float)a.im}; }
template <> __host__ __device__ inline c64 convert<c64, c64>(c64 a) { return a; }
template <> __host__ __device__ inline c64 convert<c64, c32>(c32 a) { return {(double)a.re, (double)a.im}; }
template <> __host__ __device__ inline c32 convert<c32, double>(double a) { return {(float)a, 0.f}; }
template <> __host__ __device__ inline c64 convert<c64, double>(double a) { return {a, 0.0}; }
// real solve types (real shifted matrices): the real part
template <> __host__ __device__ inline float convert<float, c64>(c64 a) { return (float)a.re; }
template <> __host__ __device__ inline double convert<double, c64>(c64 a) { return a.re; }
template <> __host__ __device__ inline c64 convert<c64, float>(float a) { return {(double)a, 0.0}; }

}  // namespace mf

#define MF_HIP_CHECK(expr)                                                                  \
  do {                                                                                      \
    hipError_t mf_err_ = (expr);                                                            \
    if (mf_err_ != hipSuccess) {                                                            \
      fprintf(stderr, "mfeast: HIP error %s at %s:%d (%s)\n", hipGetErrorString(mf_err_), \
              __FILE__, __LINE__, #expr);                                                   \
      return -2;                                                                            \
    }                                                                                       \
  } while (0)
