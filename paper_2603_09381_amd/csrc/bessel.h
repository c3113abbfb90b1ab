// FP64 Bessel functions J0, J1, Y0, Y1 of real positive argument, for the Hankel
// kernels H0^(1) = J0 + i Y0 and H1^(1) = J1 + i Y1 of the 2-D Helmholtz equation.
//
// Three regimes, all with coefficients from gen_bessel_table.py:
//   z < 4        power series in t = z^2/4 (DLMF 10.2.2, 10.8.1);
//   4 <= z < 24  Chebyshev expansions on intervals of width 2 (Clenshaw);
//   z >= 24      Hankel asymptotic expansion (DLMF 10.17.3) with 20 terms.
#pragma once
#include "pmx_common.h"
#include "bessel_table.h"

struct bes4 {
  double j0, j1, y0, y1;
};

// power series, z < PMX_CHEB_A
__device__ inline bes4 bessel01_series(double z) {
  bes4 r;
  double t = 0.25 * z * z;
  double s0 = pmx_ser_j0[PMX_SERIES_TERMS - 1], s1 = pmx_ser_j1[PMX_SERIES_TERMS - 1];
  double h0 = pmx_ser_y0h[PMX_SERIES_TERMS - 1], h1 = pmx_ser_y1h[PMX_SERIES_TERMS - 1];
#pragma unroll
  for (int k = PMX_SERIES_TERMS - 2; k >= 0; --k) {
    s0 = fma(s0, t, pmx_ser_j0[k]);
    s1 = fma(s1, t, pmx_ser_j1[k]);
    h0 = fma(h0, t, pmx_ser_y0h[k]);
    h1 = fma(h1, t, pmx_ser_y1h[k]);
  }
  double J0 = s0, J1 = 0.5 * z * s1;
  double lg = log(0.5 * z) + PMX_EULER;
  const double tpi = 2.0 / PMX_PI;
  r.j0 = J0;
  r.j1 = J1;
  r.y0 = tpi * (lg * J0 - h0);
  r.y1 = -tpi / z + tpi * lg * J1 - (0.5 / PMX_PI) * z * h1;
  return r;
}

// Chebyshev expansions, PMX_CHEB_A <= z < PMX_CHEB_B
__device__ inline bes4 bessel01_cheb(double z) {
  bes4 r;
  int iv = (int)((z - PMX_CHEB_A) * (1.0 / PMX_CHEB_W));
  iv = iv < 0 ? 0 : (iv >= PMX_CHEB_NINT ? PMX_CHEB_NINT - 1 : iv);
  double a = PMX_CHEB_A + PMX_CHEB_W * iv;
  double x = (2.0 * (z - a) - PMX_CHEB_W) * (1.0 / PMX_CHEB_W);
  double x2 = 2.0 * x;
  double b1[4] = {0, 0, 0, 0}, b2[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = PMX_CHEB_NC - 1; k >= 1; --k) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double b0 = fma(x2, b1[f], pmx_cheb[iv][f][k] - b2[f]);
      b2[f] = b1[f];
      b1[f] = b0;
    }
  }
  double v[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) v[f] = fma(x, b1[f], pmx_cheb[iv][f][0] - b2[f]);
  r.j0 = v[0];
  r.j1 = v[1];
  r.y0 = v[2];
  r.y1 = v[3];
  return r;
}

// large-argument expansion, z >= PMX_CHEB_B
__device__ inline bes4 bessel01_asym(double z) {
  bes4 r;
  // H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} sum_k i^k a_k(nu) / z^k
  double iz = 1.0 / z;
  // Horner in 1/z separately on the even and odd subsequences.
  double iz2 = iz * iz;
  double p0 = 0, q0 = 0, p1 = 0, q1 = 0;
#pragma unroll
  for (int k = ((PMX_ASYM_TERMS - 1) / 2) * 2; k >= 0; k -= 2) {
    double sg = ((k / 2) & 1) ? -1.0 : 1.0;
    p0 = fma(p0, iz2, sg * pmx_asym0[k]);
    p1 = fma(p1, iz2, sg * pmx_asym1[k]);
  }
#pragma unroll
  for (int k = ((PMX_ASYM_TERMS - 2) / 2) * 2 + 1; k >= 1; k -= 2) {
    double sg = (((k - 1) / 2) & 1) ? -1.0 : 1.0;
    q0 = fma(q0, iz2, sg * pmx_asym0[k]);
    q1 = fma(q1, iz2, sg * pmx_asym1[k]);
  }
  q0 *= iz;
  q1 *= iz;
  // sum = P + i Q; H = amp e^{i w}(P + i Q): J = amp (P cos w - Q sin w), Y = amp (P sin w + Q cos w)
  double s, c;
  sincos(z, &s, &c);
  const double r2 = 0.70710678118654752440;
  // w0 = z - pi/4, w1 = z - 3pi/4
  double c0 = r2 * (c + s), s0 = r2 * (s - c);
  double c1 = r2 * (s - c), s1 = -r2 * (c + s);
  double amp = sqrt((2.0 / PMX_PI) * iz);
  r.j0 = amp * (p0 * c0 - q0 * s0);
  r.y0 = amp * (p0 * s0 + q0 * c0);
  r.j1 = amp * (p1 * c1 - q1 * s1);
  r.y1 = amp * (p1 * s1 + q1 * c1);
  return r;
}

__device__ inline bes4 bessel01(double z) {
  if (z < PMX_CHEB_A) return bessel01_series(z);
  if (z < PMX_CHEB_B) return bessel01_cheb(z);
  return bessel01_asym(z);
}
