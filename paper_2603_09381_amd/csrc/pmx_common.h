// Shared device/host helpers: complex double arithmetic, error plumbing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct zd {
  double re, im;
};

__host__ __device__ inline zd zmk(double r, double i) { zd z; z.re = r; z.im = i; return z; }
__host__ __device__ inline zd zadd(zd a, zd b) { return zmk(a.re + b.re, a.im + b.im); }
__host__ __device__ inline zd zsub(zd a, zd b) { return zmk(a.re - b.re, a.im - b.im); }
__host__ __device__ inline zd zmul(zd a, zd b) {
  return zmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__host__ __device__ inline zd zconj(zd a) { return zmk(a.re, -a.im); }
__host__ __device__ inline zd zscale(zd a, double s) { return zmk(a.re * s, a.im * s); }
__host__ __device__ inline double zabs2(zd a) { return a.re * a.re + a.im * a.im; }
// a * conj(b)
__host__ __device__ inline zd zmulc(zd a, zd b) {
  return zmk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
// conj(a) * b
__host__ __device__ inline zd zcmul(zd a, zd b) {
  return zmk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
__host__ __device__ inline zd zdiv(zd a, zd b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return zmk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  } else {
    double r = b.re / b.im, d = b.re * r + b.im;
    return zmk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
  }
}
__host__ __device__ inline zd zfma(zd a, zd b, zd c) {  // a*b + c
  return zmk(fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im)));
}

#define PMX_PI 3.14159265358979323846264338327950288
#define PMX_EULER 0.57721566490153286060651209008240243
