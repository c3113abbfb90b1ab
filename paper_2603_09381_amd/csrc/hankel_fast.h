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
