// Dense FP64 application of the PMCHWT (Omit) Nystrom operator for the residual
// r = f - A x of iterative refinement (arXiv 2603.09381, Sec. 2.2 system).
//
// The self blocks A_ii are applied as a batched FP64 MFMA product with the stored Kress
// blocks.  The blocks between different inclusions use only k+ and the source's trapezoid
// weight; with x~ = w x at the source and H_n = J_n + i Y_n of k+ r, the value and
// normal-derivative rows of a target node receive
//   val += (i/4) [ -e+ H0 q~ + k (n_s.d/r) H1 u~ ],
//   der += (i/4) [ k (n_t.d/r) H1 q~ + (k/e+) (k a H0 + b H1) u~ ],
// a = (n_t.d)(n_s.d)/r^2, b = (n_t.n_s - 2 a)/r, d = x_t - x_s: the four operators S, D,
// D*, N of Sec. 2.1 written out.  One thread owns one target node and NR right-hand
// sides.
//
// Near inclusions (see ApplyArgs) are summed pair by pair with those formulas.  Every other
// inclusion j acts through Graf's addition theorem about its centre c: for |y - c| <
// |x - c|, H0(k|x - y|) = sum_n H_n(k rho_x) e^{i n th_x} J_n(k rho_y) e^{-i n th_y}, so
// with R_n(y) = J_n(k rho_y) e^{-i n th_y}, O_n(x) = H_n(k rho_x) e^{i n th_x} and the
// normal derivative d_nu R_n = (k/2)(-nu R_{n+1} + conj(nu) R_{n-1}) (nu = n_x + i n_y),
//   val = (i/4) sum_n O_n A_n,  der = (i/4)(k/2) sum_n O_n (nu_t B_{n+1} - conj(nu_t) B_{n-1}),
//   A_n = -e+ Mq_n + Mu_n,  B_n = -Mq_n + Mu_n / e+,
//   Mq_n = sum_y R_n q~,  Mu_n = (k/2) sum_y (-nu R_{n+1} + conj(nu) R_{n-1}) u~.
// The truncation order of a (wave, inclusion) pair is the larger of the order the sources'
// J_n decay needs and ceil(PMX_APPLY_TRUNC / ln(rho_min / r_j)) (rho_min: the centre's distance
// to the wave's bounding circle), so that dropped terms stay below about 1e-17 of the kept ones.
#include "assemble.h"
#include "bessel.h"
#include "hankel_fast.h"
#include "ktimer.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

// Source data of a group of NR right-hand sides, packed per source node so that every
// lane of a wave reads the same address (scalar loads): x, y, normal, owning inclusion,
// then per right-hand side the weighted densities w q and w u.
#define APPLY_SRC(NR) (5 + 4 * (NR))

template <int NR>
__global__ void k_apply_pack(ApplyArgs A, int r0, double* pk) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.n_nodes) return;
  const int own = A.owner[b];
  const int64_t o = A.node_off[own];
  const int64_t n = A.node_off[own + 1] - o;
  const double w = A.w[b];
  double* p = pk + (int64_t)b * APPLY_SRC(NR);
  p[0] = A.x[b];
  p[1] = A.y[b];
  p[2] = A.nx[b];
  p[3] = A.ny[b];
  p[4] = (double)own;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    zd q = zmk(0, 0), u = zmk(0, 0);
    if (r0 + r < A.nrhs) {
      const zd* col = A.xin + (int64_t)(r0 + r) * A.ld + 2 * o + (b - o);
      q = col[0];
      u = col[n];
    }
    p[5 + 4 * r] = w * q.re;
    p[6 + 4 * r] = w * q.im;
    p[7 + 4 * r] = w * u.re;
    p[8 + 4 * r] = w * u.im;
  }
}

// constant-memory copies of the coefficient tables (one per translation unit)
static __constant__ FarTable pmx_far_table = make_far_table();
static __constant__ SeriesTable pmx_series_table = make_series_table();

// Value and derivative rows of one target from one source (the four kernels of the
// header comment), accumulated for NR right-hand sides
template <int NR>
__device__ inline void apply_pair(double J0, double J1, double Y0, double Y1, double ir, double d1, double d2,
                                  double anx, double any, const double* p, double k, double eps, double ke,
                                  double wgt, double* vr, double* vi, double* dr, double* di) {
  const double nsd = (p[2] * d1 + p[3] * d2) * ir;
  const double ntd = (anx * d1 + any * d2) * ir;
  const double aa = ntd * nsd;
  const double bc = (anx * p[2] + any * p[3] - 2.0 * aa) * ir;
  // c1 = -e+ H0, c2 = k nsd H1, c3 = k ntd H1, c4 = (k/e+)(k aa H0 + bc H1), times wgt
  const double e0 = -eps * wgt, k1 = k * wgt, k4 = ke * wgt;
  const double c1r = e0 * J0, c1i = e0 * Y0;
  const double c2r = k1 * nsd * J1, c2i = k1 * nsd * Y1;
  const double c3r = k1 * ntd * J1, c3i = k1 * ntd * Y1;
  const double c4r = k4 * (k * aa * J0 + bc * J1), c4i = k4 * (k * aa * Y0 + bc * Y1);
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    const double qr = p[5 + 4 * rr], qi = p[6 + 4 * rr], ur = p[7 + 4 * rr], ui = p[8 + 4 * rr];
    vr[rr] = fma(c1r, qr, fma(-c1i, qi, fma(c2r, ur, fma(-c2i, ui, vr[rr]))));
    vi[rr] = fma(c1r, qi, fma(c1i, qr, fma(c2r, ui, fma(c2i, ur, vi[rr]))));
    dr[rr] = fma(c3r, qr, fma(-c3i, qi, fma(c4r, ur, fma(-c4i, ui, dr[rr]))));
    di[rr] = fma(c3r, qi, fma(c3i, qr, fma(c4r, ui, fma(c4i, ur, di[rr]))));
  }
}

// partial sums of one target times i/4 into its value and derivative rows of slot `out`
template <int NR>
__device__ inline void apply_store(const ApplyArgs& A, zd* out, int r0, int nr, int a, const double* vr,
                                   const double* vi, const double* dr, const double* di) {
  const int aown = A.owner[a];
  const int64_t o = A.node_off[aown];
  const int64_t n = A.node_off[aown + 1] - o;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      zd* col = out + (int64_t)(r0 + r) * A.ld + 2 * o + (a - o);
      col[0] = zmk(-0.25 * vi[r], 0.25 * vr[r]);
      col[n] = zmk(-0.25 * di[r], 0.25 * dr[r]);
    }
  }
}

__device__ inline double wave_sum_a(double v) {
  auto mv = [](double x, auto ctrl, auto rowmask) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), decltype(ctrl)::value, decltype(rowmask)::value, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), decltype(ctrl)::value, decltype(rowmask)::value, 0xf, false);
    return __hiloint2double(hi, lo);
  };
  using I = std::integral_constant<int, 0xf>;
  v += mv(v, std::integral_constant<int, 0xB1>{}, I{});     // quad_perm [1,0,3,2]
  v += mv(v, std::integral_constant<int, 0x4E>{}, I{});     // quad_perm [2,3,0,1]
  v += mv(v, std::integral_constant<int, 0x141>{}, I{});    // row_half_mirror
  v += mv(v, std::integral_constant<int, 0x140>{}, I{});    // row_mirror
  v += mv(v, std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});   // row_bcast15
  v += mv(v, std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});   // row_bcast31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// The general evaluation for waves with an argument below 24 (expansions of nearby
// inclusions): out of line, so that its constants do not take registers in the far loop.
__device__ __noinline__ bes4 bessel01_mid(double z) {
  pmx_ctab tab = (pmx_ctab)pmx_far_table.v, ser = (pmx_ctab)pmx_series_table.v;
  return bessel01_t(z, tab, ser);
}

// Expansion coefficients of every inclusion (one workgroup of four waves per inclusion, its
// nodes 64 at a time; every wave runs the recurrences, wave w reduces the orders m = w mod 4,
// so that four reduction chains proceed at once).  J_0 .. J_{PMAX+3} of k rho_y by Miller's backward recurrence from order
// PMAX + 27 + k r_j (normalised by J_0 + 2 sum J_2k = 1, a first pass finding the norm),
// R_{+-m} = J_m e^{-+i m th} (R_{-m} = (-1)^m J_m e^{+i m th}), and the three sums
// Mq_n = sum R_n q~, U+_n = sum R_n nu u~, U-_n = sum R_n conj(nu) u~ reduced over the wave
// and accumulated in LDS; then Mu_n = (k/2)(-U+_{n+1} + U-_{n-1}) and the records.
constexpr int P2M_MO = PMX_APPLY_PMAX + 3;   // orders -P2M_MO .. P2M_MO accumulated

template <int NR>
__global__ __launch_bounds__(256) void k_apply_p2m(ApplyArgs A, const double* __restrict__ pk, int r0) {
  constexpr int S = APPLY_SRC(NR);
  constexpr int NM = 2 * P2M_MO + 1;
  __shared__ double acc[NM][NR][6];           // per order: Mq, U+, U- (re, im)
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < NM * NR * 6; e += 256) (&acc[0][0][0])[e] = 0.0;
  __syncthreads();
  const double cx = A.incl_geo[4 * j], cy = A.incl_geo[4 * j + 1], rj = A.incl_geo[4 * j + 2];
  const double k = A.k;
  const int nstart = P2M_MO + 24 + (int)ceil(k * rj);
  const int64_t b0 = A.node_off[j], b1 = A.node_off[j + 1];
  for (int64_t c0 = b0; c0 < b1; c0 += 64) {
    const int64_t bn = c0 + lane;
    const bool valid = bn < b1;
    const double* p = pk + (valid ? bn : b1 - 1) * S;
    const double dx = p[0] - cx, dy = p[1] - cy;
    const double rho = fmax(sqrt(dx * dx + dy * dy), 1e-30 * (1.0 + rj));   // a node at the centre stays finite
    const double z = k * rho;
    const double er = dx / rho, ei = -dy / rho;     // e^{-i th}
    const double nur = p[2], nui = p[3];
    double qr[NR], qi[NR], ur[NR], ui[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      const double f = valid ? 1.0 : 0.0;
      qr[rr] = f * p[5 + 4 * rr];
      qi[rr] = f * p[6 + 4 * rr];
      ur[rr] = f * p[7 + 4 * rr];
      ui[rr] = f * p[8 + 4 * rr];
    }
    // pass 1: the norm of the backward recurrence
    const double iz2 = 2.0 / z;
    double jp = 0.0, jc = 1e-280, nrm = (nstart % 2 == 0) ? 2.0 * jc : 0.0;
    for (int m = nstart; m >= 1; --m) {
      const double jm = m * iz2 * jc - jp;
      jp = jc;
      jc = jm;
      if (((m - 1) & 1) == 0) nrm += (m - 1 == 0) ? jm : 2.0 * jm;
    }
    const double inv = 1.0 / nrm;
    // e^{-i P2M_MO th} by repeated squaring
    double Er = 1.0, Ei = 0.0, br = er, bi = ei;
    for (int e = P2M_MO; e > 0; e >>= 1) {
      if (e & 1) {
        const double t = Er * br - Ei * bi;
        Ei = Er * bi + Ei * br;
        Er = t;
      }
      const double t = br * br - bi * bi;
      bi = 2.0 * br * bi;
      br = t;
    }
    // pass 2: the same recurrence, accumulating orders P2M_MO .. 0
    jp = 0.0;
    jc = 1e-280;
    for (int m = nstart; m >= 0; --m) {
      if (m <= P2M_MO) {
        const double Jm = jc * inv;
        const double sg = (m & 1) ? -1.0 : 1.0;
        // R_m = Jm (Er + i Ei), R_-m = sg Jm (Er - i Ei)
        const double Rpr = Jm * Er, Rpi = Jm * Ei, Rmr = sg * Jm * Er, Rmi = -sg * Jm * Ei;
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          if ((m & 3) != wave) break;   // another wave reduces this order
          const double vur = nur * ur[rr] - nui * ui[rr], vui = nur * ui[rr] + nui * ur[rr];      // nu u
          const double wur = nur * ur[rr] + nui * ui[rr], wui = nur * ui[rr] - nui * ur[rr];      // conj(nu) u
          double t[12];
          t[0] = Rpr * qr[rr] - Rpi * qi[rr];
          t[1] = Rpr * qi[rr] + Rpi * qr[rr];
          t[2] = Rpr * vur - Rpi * vui;
          t[3] = Rpr * vui + Rpi * vur;
          t[4] = Rpr * wur - Rpi * wui;
          t[5] = Rpr * wui + Rpi * wur;
          t[6] = Rmr * qr[rr] - Rmi * qi[rr];
          t[7] = Rmr * qi[rr] + Rmi * qr[rr];
          t[8] = Rmr * vur - Rmi * vui;
          t[9] = Rmr * vui + Rmi * vur;
          t[10] = Rmr * wur - Rmi * wui;
          t[11] = Rmr * wui + Rmi * wur;
#pragma unroll
          for (int q = 0; q < 12; ++q) t[q] = wave_sum_a(t[q]);
          if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q) acc[P2M_MO + m][rr][q] += t[q];
            if (m > 0) {
#pragma unroll
              for (int q = 0; q < 6; ++q) acc[P2M_MO - m][rr][q] += t[6 + q];
            }
          }
        }
        // e^{-i (m-1) th} = e^{-i m th} e^{+i th}
        const double t = Er * er + Ei * ei;
        Ei = Ei * er - Er * ei;
        Er = t;
      }
      if (m == 0) break;
      const double jm = m * iz2 * jc - jp;
      jp = jc;
      jc = jm;
    }
  }
  __syncthreads();
  // records: A_n = -e Mq_n + Mu_n, B_n = -Mq_n + Mu_n / e, Mu_n = (k/2)(-U+_{n+1} + U-_{n-1})
  const double eps = A.eps, hk = 0.5 * k;
  auto coefAB = [&](int n, int rr, int ab, double& re, double& im) {
    if (n < -(P2M_MO - 1) || n > P2M_MO - 1) {
      re = im = 0.0;
      return;
    }
    const double* a0 = acc[P2M_MO + n][rr];
    const double* ap = acc[P2M_MO + n + 1][rr];
    const double* am = acc[P2M_MO + n - 1][rr];
    const double mur = hk * (-ap[2] + am[4]), mui = hk * (-ap[3] + am[5]);
    if (ab == 0) {
      re = -eps * a0[0] + mur;
      im = -eps * a0[1] + mui;
    } else {
      re = -a0[0] + mur / eps;
      im = -a0[1] + mui / eps;
    }
  };
  zd* rec = A.coef + (int64_t)j * PMX_APPLY_NRECA * NR * 6;
  for (int e = threadIdx.x; e < PMX_APPLY_NREC * NR; e += 256) {
    const int m = e / NR, rr = e % NR;
    double re, im;
    zd* o = rec + ((int64_t)m * NR + rr) * 6;
    coefAB(m, rr, 0, re, im);
    o[0] = zmk(re, im);
    coefAB(-m, rr, 0, re, im);
    o[1] = m ? zmk(re, im) : zmk(0, 0);
    coefAB(m + 1, rr, 1, re, im);
    o[2] = zmk(re, im);
    coefAB(-m + 1, rr, 1, re, im);
    o[3] = m ? zmk(re, im) : zmk(0, 0);
    coefAB(m - 1, rr, 1, re, im);
    o[4] = zmk(re, im);
    coefAB(-m - 1, rr, 1, re, im);
    o[5] = m ? zmk(re, im) : zmk(0, 0);
  }
}

// Cluster expansions from their children's, by the regular translation: with
// R_n(v) = J_n(k|v|) e^{-i n arg v}, R_m(u + d) = sum_n R_{m-n}(d) R_n(u) for all u, d, so for
// a child whose centre is d from the cluster's, A^_m = sum_n R_{m-n}(d) A_n and the same for
// B.  One workgroup per cluster of the level (at most four children, the quadtree's).  Lane
// c of the first wave computes child c's J_nu(k|d|), nu = 0 .. M2M_NU, by Miller's backward
// recurrence (rescaled against overflow, normalised by J_0 + 2 sum J_2k = 1); the table of
// R_nu(d), nu = -M2M_NU .. M2M_NU, follows.  Per child the workgroup stages the child's A_n
// and B_n in LDS, and each thread accumulates its (order, right-hand side) outputs.  The
// records are then written as p2m writes them, orders up to PMX_APPLY_PMAXC + 1.
constexpr int M2M_MO = PMX_APPLY_PMAXC + 2;                // outputs for orders -M2M_MO .. M2M_MO
constexpr int M2M_NM = 2 * M2M_MO + 1;
constexpr int M2M_NU = M2M_MO + PMX_APPLY_NRECA + 1;       // translation orders |m - n| <= M2M_NU
constexpr int M2M_NI = 2 * PMX_APPLY_NRECA + 1;            // child orders -NRECA .. NRECA
constexpr int M2M_KIDS = 4;

template <int NR>
__global__ __launch_bounds__(512) void k_apply_m2m(ApplyArgs A, int c0) {
  const int c = c0 + blockIdx.x;
  const int sc = A.n_incl + c;
  const double Cx = A.incl_geo[4 * sc], Cy = A.incl_geo[4 * sc + 1];
  const double k = A.k;
  const int q0 = A.kid_off[c], nk = min(A.kid_off[c + 1] - q0, M2M_KIDS);
  __shared__ double jt[M2M_KIDS][M2M_NU + 1];
  __shared__ zd Rt[M2M_KIDS][2 * M2M_NU + 1];
  __shared__ zd An[NR][M2M_NI], Bn[NR][M2M_NI];
  __shared__ zd accA[M2M_NM][NR], accB[M2M_NM][NR];
  const int tid = threadIdx.x;
  for (int e = tid; e < M2M_NM * NR; e += 512) {
    accA[e / NR][e % NR] = zmk(0, 0);
    accB[e / NR][e % NR] = zmk(0, 0);
  }
  if (tid < nk) {
    const int ch = A.kid_idx[q0 + tid];
    const double dx = A.incl_geo[4 * ch] - Cx, dy = A.incl_geo[4 * ch + 1] - Cy;
    const double z = k * sqrt(dx * dx + dy * dy);
    double* J = jt[tid];
    if (!(z > 0.0)) {
      J[0] = 1.0;
      for (int nu = 1; nu <= M2M_NU; ++nu) J[nu] = 0.0;
    } else {
      const int nstart = M2M_NU + 30 + (int)ceil(z);
      const double iz2 = 2.0 / z;
      double jp = 0.0, jc = 1e-280, nrm = 0.0;
      for (int m = nstart; m >= 1; --m) {
        const double jm = m * iz2 * jc - jp;   // J_{m-1}, unnormalised
        jp = jc;
        jc = jm;
        if (m - 1 <= M2M_NU) J[m - 1] = jc;
        if (((m - 1) & 1) == 0) nrm += (m - 1 == 0) ? jc : 2.0 * jc;
        if (fabs(jc) > 1e200) {   // rescale everything kept so far
          jp *= 1e-200;
          jc *= 1e-200;
          nrm *= 1e-200;
          for (int nu = m - 1; nu <= M2M_NU; ++nu) J[nu] *= 1e-200;
        }
      }
      const double inv = 1.0 / nrm;
      for (int nu = 0; nu <= M2M_NU; ++nu) J[nu] *= inv;
    }
  }
  __syncthreads();
  for (int e = tid; e < nk * (2 * M2M_NU + 1); e += 512) {
    const int kc = e / (2 * M2M_NU + 1), nu = e % (2 * M2M_NU + 1) - M2M_NU;
    const int ch = A.kid_idx[q0 + kc];
    const double dx = A.incl_geo[4 * ch] - Cx, dy = A.incl_geo[4 * ch + 1] - Cy;
    const int anu = nu < 0 ? -nu : nu;
    // R_nu(d) = J_nu e^{-i nu th}, J_{-nu} = (-1)^nu J_nu
    const double Jv = ((nu < 0) && (anu & 1)) ? -jt[kc][anu] : jt[kc][anu];
    double sn, cs;
    sincos(nu * atan2(dy, dx), &sn, &cs);
    Rt[kc][nu + M2M_NU] = zmk(Jv * cs, -Jv * sn);
  }
  for (int kc = 0; kc < nk; ++kc) {
    const int ch = A.kid_idx[q0 + kc];
    const int nrc = (ch < A.n_incl) ? PMX_APPLY_NREC : PMX_APPLY_NRECA;   // record rows of the child
    const zd* rec = A.coef + (int64_t)ch * PMX_APPLY_NRECA * NR * 6;
    __syncthreads();   // the previous child's A, B are read no more; the R table is complete
    // stored: A_n for |n| <= nrc - 1, B_n for 2 - nrc <= n <= nrc; the rest is zero
    for (int e = tid; e < NR * M2M_NI; e += 512) {
      const int rr = e / M2M_NI, n = e % M2M_NI - PMX_APPLY_NRECA;
      zd a = zmk(0, 0), b = zmk(0, 0);
      if (n >= 1 - nrc && n <= nrc - 1) a = n >= 0 ? rec[((int64_t)n * NR + rr) * 6] : rec[((int64_t)(-n) * NR + rr) * 6 + 1];
      if (n >= 2 - nrc && n <= nrc)
        b = n >= 1 ? rec[((int64_t)(n - 1) * NR + rr) * 6 + 2] : rec[((int64_t)(1 - n) * NR + rr) * 6 + 3];
      An[rr][n + PMX_APPLY_NRECA] = a;
      Bn[rr][n + PMX_APPLY_NRECA] = b;
    }
    __syncthreads();
    for (int e = tid; e < M2M_NM * NR; e += 512) {
      const int m = e / NR - M2M_MO, rr = e % NR;
      double ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll 4
      for (int n = 1 - nrc; n <= nrc; ++n) {
        const zd R = Rt[kc][m - n + M2M_NU];
        const zd a = An[rr][n + PMX_APPLY_NRECA], b = Bn[rr][n + PMX_APPLY_NRECA];
        ar = fma(-R.im, a.im, fma(R.re, a.re, ar));
        ai = fma(R.im, a.re, fma(R.re, a.im, ai));
        br = fma(-R.im, b.im, fma(R.re, b.re, br));
        bi = fma(R.im, b.re, fma(R.re, b.im, bi));
      }
      accA[m + M2M_MO][rr] = zadd(accA[m + M2M_MO][rr], zmk(ar, ai));
      accB[m + M2M_MO][rr] = zadd(accB[m + M2M_MO][rr], zmk(br, bi));
    }
  }
  __syncthreads();
  zd* out = A.coef + (int64_t)sc * PMX_APPLY_NRECA * NR * 6;
  for (int e = tid; e < PMX_APPLY_NRECA * NR; e += 512) {
    const int m = e / NR, rr = e % NR;
    zd* o = out + ((int64_t)m * NR + rr) * 6;
    const zd z0 = zmk(0, 0);
    o[0] = accA[M2M_MO + m][rr];
    o[1] = m ? accA[M2M_MO - m][rr] : z0;
    o[2] = accB[M2M_MO + m + 1][rr];
    o[3] = m ? accB[M2M_MO - m + 1][rr] : z0;
    o[4] = accB[M2M_MO + m - 1][rr];
    o[5] = m ? accB[M2M_MO - m - 1][rr] : z0;
  }
}

// Far part: part blockIdx.y of the wave's list of far sources (inclusions and clusters),
// each through its expansion: per lane rho, th of the target about the source's centre, H0
// and H1 (large-argument expansion when the whole wave allows it), then orders m = 0 .. p+1
// by the upward recurrence H_{m+1} = (2m/z) H_m - H_{m-1} (stable for the Hankel function)
// and e^{i(m+1)th} = e^{i m th} e^{i th}; O_{-m} = (-1)^m H_m e^{-i m th}.  The sums
// S1 = sum O_m B_{m+1}, S2 = sum O_m B_{m-1} are kept over all sources and turned into
// derivative rows once at the end.
template <int NR>
__global__ __launch_bounds__(256) void k_apply_far(ApplyArgs A, const double* __restrict__ cf, int r0) {
  const int N = A.n_nodes;
  const int a_raw = blockIdx.x * 256 + threadIdx.x;
  const bool active = a_raw < N;
  const int a = active ? a_raw : N - 1;   // idle lanes follow the last node and write nothing
  const int wv = __builtin_amdgcn_readfirstlane(a_raw >> 6);
  if (wv >= (N + 63) / 64) return;        // a wave past the last target (no barrier follows)
  const int nr = min(NR, A.nrhs - r0);
  const double ax = A.x[a], ay = A.y[a], anx = A.nx[a], any = A.ny[a];
  const double k = A.k, ik = 1.0 / k;
  const double wcx = A.wave_geo[4 * wv], wcy = A.wave_geo[4 * wv + 1], wr = A.wave_geo[4 * wv + 2];
  double vr[NR], vi[NR], s1r[NR], s1i[NR], s2r[NR], s2i[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) vr[r] = vi[r] = s1r[r] = s1i[r] = s2r[r] = s2i[r] = 0.0;
  const int fq0 = A.far_off[wv], flen = A.far_off[wv + 1] - fq0;
  const int ns = gridDim.y, ys = blockIdx.y;
  const int q0 = fq0 + (int)((int64_t)flen * ys / ns), q1 = fq0 + (int)((int64_t)flen * (ys + 1) / ns);
  for (int q = q0; q < q1; ++q) {
    const int j = A.far_idx[q];
    const double cx = A.incl_geo[4 * j], cy = A.incl_geo[4 * j + 1], rj = A.incl_geo[4 * j + 2];
    const double pj = A.incl_geo[4 * j + 3];
    // truncation order of the pair (uniform)
    const double rmin = sqrt((wcx - cx) * (wcx - cx) + (wcy - cy) * (wcy - cy)) - wr;
    const double pr = fmax(pj, ceil(PMX_APPLY_TRUNC / log(rmin / rj)));
    const int p = __builtin_amdgcn_readfirstlane((int)fmin(pr, (double)PMX_APPLY_PMAXC));
    const double dx = ax - cx, dy = ay - cy;
    const double irho = rsqrt_nr(dx * dx + dy * dy);
    const double z = k * ((dx * dx + dy * dy) * irho);
    const double er = dx * irho, ei = dy * irho;   // e^{i th}
    double H0r, H1r, H0i, H1i;
    if (__all(z >= 24.0)) {
      pmx_ctab tab = (pmx_ctab)pmx_far_table.v;
      asm volatile("" : "+s"(tab));
      if (__all(z >= 60.0))
        hankel_far_t<12>(z, irho * ik, tab, H0r, H1r, H0i, H1i);
      else if (__all(z >= 35.0))
        hankel_far_t<16>(z, irho * ik, tab, H0r, H1r, H0i, H1i);
      else
        hankel_far_t<20>(z, irho * ik, tab, H0r, H1r, H0i, H1i);
    } else {
      const bes4 h = bessel01_mid(z);
      H0r = h.j0;
      H0i = h.y0;
      H1r = h.j1;
      H1i = h.y1;
    }
    const double iz2 = 2.0 / z;
    // m = 0 .. p + 1: Hc = H_m, Hp = H_{m-1}, (Emr, Emi) = e^{i m th}
    double Hcr = H0r, Hci = H0i, Hpr = -H1r, Hpi = -H1i;   // H_{-1} = -H_1
    double Emr = 1.0, Emi = 0.0;
    const double* rec = cf + (int64_t)j * PMX_APPLY_NRECA * NR * 12;
    for (int m = 0; m <= p + 1; ++m) {
      const double sg = (m & 1) ? -1.0 : 1.0;
      const double Opr = Hcr * Emr - Hci * Emi, Opi = Hcr * Emi + Hci * Emr;               // O_m
      const double Omr = sg * (Hcr * Emr + Hci * Emi), Omi = sg * (Hci * Emr - Hcr * Emi);  // O_-m
      const double* o = rec + (int64_t)m * NR * 12;
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) {
        // A_m, A_-m, B_m+1, B_-m+1, B_m-1, B_-m-1 (wave-uniform addresses: scalar loads)
        const double* c = o + rr * 12;
        // four fused operations into each accumulator
        vr[rr] = fma(-Omi, c[3], fma(Omr, c[2], fma(-Opi, c[1], fma(Opr, c[0], vr[rr]))));
        vi[rr] = fma(Omi, c[2], fma(Omr, c[3], fma(Opi, c[0], fma(Opr, c[1], vi[rr]))));
        s1r[rr] = fma(-Omi, c[7], fma(Omr, c[6], fma(-Opi, c[5], fma(Opr, c[4], s1r[rr]))));
        s1i[rr] = fma(Omi, c[6], fma(Omr, c[7], fma(Opi, c[4], fma(Opr, c[5], s1i[rr]))));
        s2r[rr] = fma(-Omi, c[11], fma(Omr, c[10], fma(-Opi, c[9], fma(Opr, c[8], s2r[rr]))));
        s2i[rr] = fma(Omi, c[10], fma(Omr, c[11], fma(Opi, c[8], fma(Opr, c[9], s2i[rr]))));
      }
      // H_{m+1} = (2m/z) H_m - H_{m-1}; e^{i(m+1)th}
      const double f = m * iz2;
      double Hnr = f * Hcr - Hpr, Hni = f * Hci - Hpi;
      if (m == 0) {
        Hnr = H1r;
        Hni = H1i;
      }
      Hpr = Hcr;
      Hpi = Hci;
      Hcr = Hnr;
      Hci = Hni;
      const double t = Emr * er - Emi * ei;
      Emi = Emr * ei + Emi * er;
      Emr = t;
    }
  }
  if (!active) return;
  // der = (k/2)(nu S1 - conj(nu) S2)
  const double hk = 0.5 * k;
  double dr[NR], di[NR];
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    dr[rr] = hk * (anx * s1r[rr] - any * s1i[rr] - (anx * s2r[rr] + any * s2i[rr]));
    di[rr] = hk * (anx * s1i[rr] + any * s1r[rr] - (anx * s2i[rr] - any * s2r[rr]));
  }
  apply_store<NR>(A, A.part + (int64_t)blockIdx.y * A.nrhs * A.ld, r0, nr, a, vr, vi, dr, di);
}

// Near part: one wave per workgroup; part blockIdx.y of the wave's near list, every
// argument through the general Bessel evaluation; pairs on the target's own inclusion
// (the self block, applied separately) are left out.
template <int NR>
__global__ __launch_bounds__(64) void k_apply_near(ApplyArgs A, const double* __restrict__ pk, int r0, int slot0) {
  constexpr int S = APPLY_SRC(NR);
  const int N = A.n_nodes;
  const int wv = blockIdx.x;
  const int a_raw = wv * 64 + threadIdx.x;
  const bool active = a_raw < N;
  const int a = active ? a_raw : N - 1;
  const int nr = min(NR, A.nrhs - r0);
  const double ax = A.x[a], ay = A.y[a], anx = A.nx[a], any = A.ny[a];
  const int aown = A.owner[a];
  const double k = A.k, eps = A.eps;
  const double ke = k / eps;
  double vr[NR], vi[NR], dr[NR], di[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) vr[r] = vi[r] = dr[r] = di[r] = 0.0;
  const int qs = A.near_off[wv], len = A.near_off[wv + 1] - qs;
  const int ns = A.nsplit_near, y = blockIdx.y;
  const int q0 = qs + (int)((int64_t)len * y / ns), q1 = qs + (int)((int64_t)len * (y + 1) / ns);
  for (int q = q0; q < q1; ++q) {
    const int j = A.near_idx[q];
    const bool self = (j == aown);
    if (__all(self)) continue;   // the whole wave lies on inclusion j: its self block, applied separately
    const int b1 = (int)A.node_off[j + 1];
    for (int b = (int)A.node_off[j]; b < b1; ++b) {
      pmx_ctab tab = (pmx_ctab)pmx_far_table.v, ser = (pmx_ctab)pmx_series_table.v;
      asm volatile("" : "+s"(tab), "+s"(ser));   // re-read the coefficients in every iteration
      const double* p = pk + (int64_t)b * S;
      const double d1 = ax - p[0], d2 = ay - p[1];
      const double dd = self ? 1.0 : d1 * d1 + d2 * d2;
      const double ir = rsqrt_nr(dd);
      const bes4 h = bessel01_t(k * (dd * ir), tab, ser);
      apply_pair<NR>(h.j0, h.j1, h.y0, h.y1, ir, d1, d2, anx, any, p, k, eps, ke, self ? 0.0 : 1.0, vr, vi, dr, di);
    }
  }
  if (active) apply_store<NR>(A, A.part + (int64_t)(slot0 + y) * A.nrhs * A.ld, r0, nr, a, vr, vi, dr, di);
}

// out = sf f + sa (ydiag + sum of the partial sums); f may be NULL
__global__ void k_apply_finish(const zd* f, const zd* ydiag, const zd* part, int nsplit, int64_t total, double sf,
                               double sa, zd* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  zd s = ydiag[i];
  for (int p = 0; p < nsplit; ++p) s = zadd(s, part[(int64_t)p * total + i]);
  zd v = zscale(s, sa);
  if (f) v = zfma(zmk(sf, 0), f[i], v);
  out[i] = v;
}

// source splits so that one launch has about wg_target workgroups, with at least 128
// sources per split
int apply_splits(int n_nodes, int wg_target) {
  const int nwg = (n_nodes + 255) / 256;
  int ns = (wg_target + nwg - 1) / nwg;
  ns = std::max(1, std::min(ns, 64));
  ns = std::min(ns, std::max(1, n_nodes / 128));
  return ns;
}

int apply_near_splits(int n_nodes, int wg_target) {
  const int nw = (n_nodes + 63) / 64;
  return std::max(1, std::min(8, (wg_target + nw - 1) / nw));
}

int64_t apply_pack_size(int n_nodes, int nr_max) { return (int64_t)n_nodes * APPLY_SRC(nr_max); }

int64_t apply_coef_size(int n_src, int nr_max) { return (int64_t)n_src * PMX_APPLY_NRECA * nr_max * 6; }

int apply_source_order(double kr) {
  for (int p = 1; p < 1000; ++p)
    if (p > 0.5 * M_E * kr + 2 && std::pow(0.5 * M_E * kr / p, p) <= 1e-17) return p;
  return 1000;
}

template <int NR>
static void apply_group(const ApplyArgs& A, double* pk, int r0, int nsplit, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_pack<NR>, dim3((A.n_nodes + 255) / 256), dim3(256), 0, s, A, r0, pk);
  const int m = (int)A.n_incl;
  hipLaunchKernelGGL(k_apply_p2m<NR>, dim3(m), dim3(256), 0, s, A, (const double*)pk, r0);
  for (int l = 0; l < A.n_lev; ++l)
    if (A.lev_off[l + 1] > A.lev_off[l])
      hipLaunchKernelGGL(k_apply_m2m<NR>, dim3(A.lev_off[l + 1] - A.lev_off[l]), dim3(512), 0, s, A, A.lev_off[l]);
  hipLaunchKernelGGL(k_apply_far<NR>, dim3((A.n_nodes + 255) / 256, nsplit), dim3(256), 0, s, A,
                     (const double*)A.coef, r0);
  hipLaunchKernelGGL(k_apply_near<NR>, dim3((A.n_nodes + 63) / 64, A.nsplit_near), dim3(64), 0, s, A,
                     (const double*)pk, r0, nsplit);
}

// right-hand sides in groups of nr_max (1, 2, 4 or 8); a last smaller group takes the
// smallest of those sizes that holds it
void asm_apply_off(const ApplyArgs& A, int nsplit, int nr_max, hipStream_t s) {
  if (A.n_nodes <= 0 || A.nrhs <= 0) return;
  for (int r0 = 0; r0 < A.nrhs;) {
    const int left = A.nrhs - r0;
    const int g = left >= nr_max ? nr_max : (left <= 1 ? 1 : left <= 2 ? 2 : left <= 4 ? 4 : 8);
    switch (g) {
      case 1: apply_group<1>(A, A.pack, r0, nsplit, s); break;
      case 2: apply_group<2>(A, A.pack, r0, nsplit, s); break;
      case 4: apply_group<4>(A, A.pack, r0, nsplit, s); break;
      default: apply_group<8>(A, A.pack, r0, nsplit, s); break;
    }
    r0 += g;
  }
}

void asm_apply_finish(const zd* f, const zd* ydiag, const zd* part, int nsplit, int64_t total, double sf, double sa,
                      zd* out, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_apply_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f, ydiag, part, nsplit,
                     total, sf, sa, out);
}

// squared 2-norms of the ncol columns of a (n x ncol, leading dimension ld): partial sums
// part[c * nblk + b] of nblk workgroups per column
__global__ __launch_bounds__(256) void k_colnorm2(const zd* a, int64_t n, int64_t ld, double* part) {
  const int c = blockIdx.y;
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const zd v = a[(int64_t)c * ld + i];
    s += v.re * v.re + v.im * v.im;
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = red[0];
}

void asm_colnorm2(const zd* a, int64_t n, int ncol, int64_t ld, int nblk, double* part, hipStream_t s) {
  if (n <= 0 || ncol <= 0) return;
  hipLaunchKernelGGL(k_colnorm2, dim3(nblk, ncol), dim3(256), 0, s, a, n, ld, part);
}
