// Shared device/host helpers of the two-grid library: complex arithmetic on
// interleaved (re, im) pairs, launch checking and small integer helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <cstdio>
#include <string>

namespace th {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

using c64 = cx<double>;   // complex128 element
using c32 = cx<float>;    // complex64 element

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T re, T im) { return cx<T>{re, im}; }

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }

// acc += a * b (complex multiply-accumulate with explicit FMAs)
template <typename T>
__host__ __device__ __forceinline__ void cmac(cx<T> &acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += s * b for real s
template <typename T>
__host__ __device__ __forceinline__ void rmac(cx<T> &acc, T s, cx<T> b) {
  acc.re = fma(s, b.re, acc.re);
  acc.im = fma(s, b.im, acc.im);
}

template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> ccast(cx<Ti> a) { return {(To)a.re, (To)a.im}; }

// Vector load of data that is read exactly once per launch (non-temporal hint).
__device__ __forceinline__ cx<double> ld_stream(const cx<double> *p) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 v = __builtin_nontemporal_load((const d2 *)p);
  return {v.x, v.y};
}
__device__ __forceinline__ cx<float> ld_stream(const cx<float> *p) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 v = __builtin_nontemporal_load((const f2 *)p);
  return {v.x, v.y};
}

__host__ __device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ __forceinline__ long long ceil_div_ll(long long a, long long b) { return (a + b - 1) / b; }

// Maximum polynomial order supported by the fixed-size reference tables.
constexpr int kMaxP = 8;

// 1-D reference data passed by value to kernels.
struct Ref1D {
  double K[(kMaxP + 1) * (kMaxP + 1)];   // int phi_a' phi_b' on [0,1]
  double M[(kMaxP + 1) * (kMaxP + 1)];   // int phi_a phi_b on [0,1]
  double L[(kMaxP + 1) * (kMaxP / 2 + 1)]; // interpolation: fine GLL node a <- coarse point b
};

}  // namespace th

#define TH_HIP_CHECK_RET(expr)                                                     \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) return ::th::hip_fail(_e, #expr, __FILE__, __LINE__);    \
  } while (0)

namespace th {
// Records a HIP failure in the thread-local error slot; returns TH_EHIP (-4).
int hip_fail(hipError_t e, const char *expr, const char *file, int line);
}  // namespace th
