// Shared device/host helpers: complex arithmetic over double and float.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Host-side counts, per host thread, of kernel launches and of host waits on the device
// (the factorisation reports both per call).  Every launch goes through PMX_LAUNCH.
void pmx_count_launch();
void pmx_count_sync();
#define PMX_LAUNCH(...)              \
  do {                               \
    pmx_count_launch();              \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)

// complex number over a real type R (double or float)
template <class R>
struct cx {
  R re, im;
};
typedef cx<double> zd;
typedef cx<float> zf;

// The same pointer in the global address space.  Pointers read from descriptors in memory
// are generic to the compiler, which then emits flat loads and stores: those also count
// against the LDS wait counter, so every wait for an LDS read waits for the outstanding
// global loads as well, and at most 15 can be in flight.  Accesses through the returned
// pointer compile to global_load / global_store.  Only for device memory.
template <class T>
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
#else
// the host pass only checks kernel bodies; it keeps the pointer as it is
__host__ __device__ inline T* gbl(T* p) {
  return p;
}
#endif

template <class R>
__host__ __device__ inline cx<R> cmk(R r, R i) {
  cx<R> z;
  z.re = r;
  z.im = i;
  return z;
}
__host__ __device__ inline zd zmk(double r, double i) { return cmk<double>(r, i); }
template <class R>
__host__ __device__ inline cx<R> zadd(cx<R> a, cx<R> b) { return cmk<R>(a.re + b.re, a.im + b.im); }
template <class R>
__host__ __device__ inline cx<R> zsub(cx<R> a, cx<R> b) { return cmk<R>(a.re - b.re, a.im - b.im); }
template <class R>
__host__ __device__ inline cx<R> zmul(cx<R> a, cx<R> b) {
  return cmk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R>
__host__ __device__ inline cx<R> zconj(cx<R> a) { return cmk<R>(a.re, -a.im); }
// the scale factor does not take part in deducing R (it may be given in double)
template <class T>
struct nodeduce {
  typedef T type;
};
template <class R>
__host__ __device__ inline cx<R> zscale(cx<R> a, typename nodeduce<R>::type s) {
  return cmk<R>(a.re * s, a.im * s);
}
template <class R>
__host__ __device__ inline R zabs2(cx<R> a) { return a.re * a.re + a.im * a.im; }
// a * conj(b)
template <class R>
__host__ __device__ inline cx<R> zmulc(cx<R> a, cx<R> b) {
  return cmk<R>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
// conj(a) * b
template <class R>
__host__ __device__ inline cx<R> zcmul(cx<R> a, cx<R> b) {
  return cmk<R>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class R>
__host__ __device__ inline cx<R> zdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, d = b.re + b.im * r;
    return cmk<R>((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  } else {
    R r = b.re / b.im, d = b.re * r + b.im;
    return cmk<R>((a.re * r + a.im) / d, (a.im * r - a.re) / d);
  }
}
// 1 / b by Smith's algorithm (the quotients of zdiv with a = 1, one division for both)
template <class R>
__host__ __device__ inline cx<R> zrecip(cx<R> b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const R r = b.im / b.re, t = R(1) / (b.re + b.im * r);
    return cmk<R>(t, -r * t);
  }
  const R r = b.re / b.im, t = R(1) / (b.re * r + b.im);
  return cmk<R>(r * t, -t);
}
template <class R>
__host__ __device__ inline cx<R> zfma(cx<R> a, cx<R> b, cx<R> c) {  // a*b + c
  return cmk<R>(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}
template <class R>
__host__ __device__ inline cx<R> zfms(cx<R> c, cx<R> a, cx<R> b) {  // c - a*b in four fused operations
  return cmk<R>(fma(-a.re, b.re, fma(a.im, b.im, c.re)), fma(-a.re, b.im, fma(-a.im, b.re, c.im)));
}

#define PMX_PI 3.14159265358979323846264338327950288
#define PMX_EULER 0.57721566490153286060651209008240243
