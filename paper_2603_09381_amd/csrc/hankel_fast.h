// H0 and H1 of the first kind at large argument, for the dense operator apply: the
// large-argument expansion (the coefficients of bessel01) with fewer terms where the
// argument allows it, the phase sin / cos of z - pi/4 by additive reduction and Taylor
// polynomials (trig_table.h), and the amplitude and 1/z from the hardware reciprocal
// square root refined by Newton steps.
#pragma once
#include "bessel.h"
#include "trig_table.h"

// 1/sqrt(x), x > 0: the hardware estimate and two Newton steps y <- y + y (1 - x y^2) / 2
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// s = sin(z - pi/4), c = cos(z - pi/4) for 0 <= z < 8e5: z - pi/4 = r + n pi/2 with
// n = floor(2 z / pi) and r = z - (2n+1) pi/4 in [-pi/4, pi/4]
__device__ inline void sincos_shift(double z, double& s, double& c) {
  const double n = floor(z * (0.5 * PMX_FOUR_OVER_PI));
  const double m = 2.0 * n + 1.0;
  double r = fma(-m, PMX_PIO4_1, z);
  r = fma(-m, PMX_PIO4_2, r);
  r = fma(-m, PMX_PIO4_3, r);
  const double r2 = r * r;
  double ps = pmx_sin_c[PMX_SIN_NC - 1], pc = pmx_cos_c[PMX_COS_NC - 1];
#pragma unroll
  for (int k = PMX_SIN_NC - 2; k >= 0; --k) ps = fma(ps, r2, pmx_sin_c[k]);
#pragma unroll
  for (int k = PMX_COS_NC - 2; k >= 0; --k) pc = fma(pc, r2, pmx_cos_c[k]);
  ps *= r;
  const int q = (int)(n - 4.0 * floor(0.25 * n));
  const double sa = (q & 1) ? pc : ps, ca = (q & 1) ? ps : pc;
  s = (q & 2) ? -sa : sa;
  c = ((q + 1) & 2) ? -ca : ca;
}

// K-term expansion (K <= PMX_ASYM_TERMS; 12 terms hold 2e-17 for z >= 50, 16 for z >= 30,
// 20 for z >= 24); iz = 1/z
template <int K>
__device__ inline void hankel_far(double z, double iz, double& J0, double& J1, double& Y0, double& Y1) {
  const double iz2 = iz * iz;
  double p0 = 0, q0 = 0, p1 = 0, q1 = 0;
#pragma unroll
  for (int k = ((K - 1) / 2) * 2; k >= 0; k -= 2) {
    const double sg = ((k / 2) & 1) ? -1.0 : 1.0;
    p0 = fma(p0, iz2, sg * pmx_asym0[k]);
    p1 = fma(p1, iz2, sg * pmx_asym1[k]);
  }
#pragma unroll
  for (int k = ((K - 2) / 2) * 2 + 1; k >= 1; k -= 2) {
    const double sg = (((k - 1) / 2) & 1) ? -1.0 : 1.0;
    q0 = fma(q0, iz2, sg * pmx_asym0[k]);
    q1 = fma(q1, iz2, sg * pmx_asym1[k]);
  }
  q0 *= iz;
  q1 *= iz;
  double s0, c0;
  sincos_shift(z, s0, c0);   // cos, sin of z - pi/4; those of z - 3 pi/4 are s0, -c0
  const double amp = 0.79788456080286535588 * rsqrt_nr(z);   // sqrt(2 / (pi z))
  J0 = amp * (p0 * c0 - q0 * s0);
  Y0 = amp * (p0 * s0 + q0 * c0);
  J1 = amp * (p1 * s0 + q1 * c0);
  Y1 = amp * (q1 * s0 - p1 * c0);
}

// The same evaluation with every coefficient read from a table in constant memory
// (pmx_far_table below) through a pointer t: in a loop whose pointer the compiler cannot
// hoist, the coefficients are scalar loads per use instead of ~120 registers held across
// the loop.  Layout: [0, 10) P0, [10, 20) Q0, [20, 30) P1, [30, 40) Q1 (signed terms of
// the expansion in 1/z^2, lowest first), [40, 49) sin, [49, 59) cos coefficients.
#define PMX_FAR_TABLE_SIZE 59
typedef const __attribute__((address_space(4))) double* pmx_ctab;

// a b + c with c wave-uniform, taken as a scalar operand (no copy to vector registers)
__device__ inline double fma_su(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

template <int K>
__device__ inline void hankel_far_t(double z, double iz, pmx_ctab t, double& J0, double& J1, double& Y0, double& Y1) {
  constexpr int NP = (K - 1) / 2 + 1, NQ = (K - 2) / 2 + 1;
  const double iz2 = iz * iz;
  double p0 = t[NP - 1], p1 = t[20 + NP - 1];
#pragma unroll
  for (int i = NP - 2; i >= 0; --i) {
    p0 = fma_su(p0, iz2, t[i]);
    p1 = fma_su(p1, iz2, t[20 + i]);
  }
  double q0 = t[10 + NQ - 1], q1 = t[30 + NQ - 1];
#pragma unroll
  for (int i = NQ - 2; i >= 0; --i) {
    q0 = fma_su(q0, iz2, t[10 + i]);
    q1 = fma_su(q1, iz2, t[30 + i]);
  }
  q0 *= iz;
  q1 *= iz;
  // sin, cos of z - pi/4 as in sincos_shift
  const double n = floor(z * (0.5 * PMX_FOUR_OVER_PI));
  const double m = 2.0 * n + 1.0;
  double r = fma(-m, PMX_PIO4_1, z);
  r = fma(-m, PMX_PIO4_2, r);
  r = fma(-m, PMX_PIO4_3, r);
  const double r2 = r * r;
  double ps = t[40 + PMX_SIN_NC - 1], pc = t[49 + PMX_COS_NC - 1];
#pragma unroll
  for (int k = PMX_SIN_NC - 2; k >= 0; --k) ps = fma_su(ps, r2, t[40 + k]);
#pragma unroll
  for (int k = PMX_COS_NC - 2; k >= 0; --k) pc = fma_su(pc, r2, t[49 + k]);
  ps *= r;
  const int q = (int)(n - 4.0 * floor(0.25 * n));
  const double sa = (q & 1) ? pc : ps, ca = (q & 1) ? ps : pc;
  const double s0 = (q & 2) ? -sa : sa;
  const double c0 = ((q + 1) & 2) ? -ca : ca;
  const double amp = 0.79788456080286535588 * rsqrt_nr(z);   // sqrt(2 / (pi z))
  J0 = amp * (p0 * c0 - q0 * s0);
  Y0 = amp * (p0 * s0 + q0 * c0);
  J1 = amp * (p1 * s0 + q1 * c0);
  Y1 = amp * (q1 * s0 - p1 * c0);
}

// J0, J1, Y0, Y1 at any z > 0 for the near pairs of the apply, with bessel01's small- and
// mid-argument evaluations and hankel_far_t<20> above 24; the power-series coefficients
// come from a table s in constant memory ([f * PMX_SERIES_TERMS + k] for the series of J0,
// J1, Y0's and Y1's remainder), read as scalar operands like those of hankel_far_t.
__device__ inline bes4 bessel01_t(double z, pmx_ctab t, pmx_ctab s) {
  bes4 r;
  if (z < PMX_CHEB_A) {
    const double u = 0.25 * z * z;
    constexpr int T = PMX_SERIES_TERMS;
    double s0 = s[T - 1], s1 = s[2 * T - 1], h0 = s[3 * T - 1], h1 = s[4 * T - 1];
#pragma unroll
    for (int k = T - 2; k >= 0; --k) {
      s0 = fma_su(s0, u, s[k]);
      s1 = fma_su(s1, u, s[T + k]);
      h0 = fma_su(h0, u, s[2 * T + k]);
      h1 = fma_su(h1, u, s[3 * T + k]);
    }
    const double J0 = s0, J1 = 0.5 * z * s1;
    const double lg = log(0.5 * z) + PMX_EULER;
    const double tpi = 2.0 / PMX_PI;
    r.j0 = J0;
    r.j1 = J1;
    r.y0 = tpi * (lg * J0 - h0);
    r.y1 = -tpi / z + tpi * lg * J1 - (0.5 / PMX_PI) * z * h1;
  } else if (z < PMX_CHEB_B) {
    r = bessel01_cheb(z);
  } else {
    hankel_far_t<20>(z, 1.0 / z, t, r.j0, r.j1, r.y0, r.y1);
  }
  return r;
}

// Coefficients of hankel_far_t in constant memory (signed expansion terms, then the
// sine and cosine polynomials)
struct FarTable {
  double v[PMX_FAR_TABLE_SIZE];
};
constexpr FarTable make_far_table() {
  FarTable t{};
  for (int i = 0; i < 10; ++i) {
    const double sg = (i & 1) ? -1.0 : 1.0;
    t.v[i] = sg * pmx_asym0[2 * i];
    t.v[10 + i] = sg * pmx_asym0[2 * i + 1];
    t.v[20 + i] = sg * pmx_asym1[2 * i];
    t.v[30 + i] = sg * pmx_asym1[2 * i + 1];
  }
  for (int k = 0; k < PMX_SIN_NC; ++k) t.v[40 + k] = pmx_sin_c[k];
  for (int k = 0; k < PMX_COS_NC; ++k) t.v[49 + k] = pmx_cos_c[k];
  return t;
}

// power-series coefficients of bessel01_t: J0, J1, then Y0's and Y1's remainders
struct SeriesTable {
  double v[4 * PMX_SERIES_TERMS];
};
constexpr SeriesTable make_series_table() {
  SeriesTable t{};
  for (int k = 0; k < PMX_SERIES_TERMS; ++k) {
    t.v[k] = pmx_ser_j0[k];
    t.v[PMX_SERIES_TERMS + k] = pmx_ser_j1[k];
    t.v[2 * PMX_SERIES_TERMS + k] = pmx_ser_y0h[k];
    t.v[3 * PMX_SERIES_TERMS + k] = pmx_ser_y1h[k];
  }
  return t;
}
