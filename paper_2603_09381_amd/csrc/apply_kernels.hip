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
// to the wave's bounding circle), so that dropped terms stay below about e^-PMX_APPLY_TRUNC of the
// kept ones.
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

// Expansion coefficients of every inclusion (one workgroup per inclusion, its nodes 32 at a
// time).  R_{+-m} = J_m e^{-+i m th} (R_{-m} = (-1)^m conj R_m), with J_0 .. J_{P2M_MO} of
// k rho_y by Miller's backward recurrence from order PMAX + 27 + k r_j (normalised by
// J_0 + 2 sum J_2k = 1, a first pass finding the norm), and the three sums
// Mq_n = sum R_n q~, U+_n = sum R_n nu u~, U-_n = sum R_n conj(nu) u~ over the nodes; then
// Mu_n = (k/2)(-U+_{n+1} + U-_{n-1}) and the records.  Per chunk of 32 nodes the eight
// threads of a node each run its recurrence and store every eighth order of R_m in LDS
// (node-major, so that the threads of consecutive orders read consecutive words), and the
// node's three density products; then thread (|m|, kind) accumulates, over the chunk's
// nodes, R_m and R_-m times its kind's products for every right-hand side in registers: no
// reduction across lanes.  The sums go to LDS (the chunk buffers' space) at the end.
constexpr int P2M_MO = PMX_APPLY_PMAX + 3;   // orders -P2M_MO .. P2M_MO accumulated
constexpr int P2M_NC = 32;                   // nodes per chunk
constexpr int P2M_OM = P2M_MO + 1;           // orders 0 .. P2M_MO in the table

template <int NR>
__global__ __launch_bounds__(256) void k_apply_p2m(ApplyArgs A, const double* __restrict__ pk, int r0) {
  constexpr int S = APPLY_SRC(NR);
  constexpr int NM = 2 * P2M_MO + 1;
  constexpr int TAB = P2M_NC * P2M_OM * 2 + P2M_NC * 3 * NR * 2;   // doubles of the chunk buffers
  constexpr int ACC = NM * NR * 6;
  __shared__ double sm[TAB > ACC ? TAB : ACC];
  double* Rt = sm;                                  // [node][order] (re, im)
  double* Vt = sm + P2M_NC * P2M_OM * 2;            // [node][kind][rhs] (re, im)
  double(*acc)[NR][6] = reinterpret_cast<double(*)[NR][6]>(sm);   // after the chunks: [order][rhs][6]
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const double cx = A.incl_geo[4 * j], cy = A.incl_geo[4 * j + 1], rj = A.incl_geo[4 * j + 2];
  const double k = A.k;
  const int nstart = P2M_MO + 24 + (int)ceil(k * rj);
  const int64_t b0 = A.node_off[j], b1 = A.node_off[j + 1];
  // phase B roles: thread (|m|, kind) for |m| <= P2M_MO, kind 0 q, 1 nu u, 2 conj(nu) u
  const bool acc_thread = tid < 3 * P2M_OM;
  const int om = tid % P2M_OM, kind = tid / P2M_OM;
  double pr[NR], pi[NR], mr[NR], mi[NR];     // sums for +|m| and -|m|
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) pr[rr] = pi[rr] = mr[rr] = mi[rr] = 0.0;
  for (int64_t c0 = b0; c0 < b1; c0 += P2M_NC) {
    {
      // phase A: node nd of the chunk, part pt of its orders (m = pt mod 8)
      const int nd = tid & (P2M_NC - 1), pt = tid / P2M_NC;
      const int64_t bn = c0 + nd;
      const bool valid = bn < b1;
      const double* p = pk + (valid ? bn : b1 - 1) * S;
      const double dx = p[0] - cx, dy = p[1] - cy;
      const double rho = fmax(sqrt(dx * dx + dy * dy), 1e-30 * (1.0 + rj));   // a node at the centre stays finite
      const double z = k * rho;
      const double er = dx / rho, ei = -dy / rho;     // e^{-i th}
      const double iz2 = 2.0 / z;
      double jp = 0.0, jc = 1e-280, nrm = (nstart % 2 == 0) ? 2.0 * jc : 0.0;
      for (int m = nstart; m >= 1; --m) {
        const double jm = m * iz2 * jc - jp;
        jp = jc;
        jc = jm;
        if (((m - 1) & 1) == 0) nrm += (m - 1 == 0) ? jm : 2.0 * jm;
      }
      const double inv = valid ? 1.0 / nrm : 0.0;   // a missing node contributes nothing
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
      jp = 0.0;
      jc = 1e-280;
      for (int m = nstart; m >= 0; --m) {
        if (m <= P2M_MO) {
          if ((m & 7) == pt) {
            const double Jm = jc * inv;
            Rt[(nd * P2M_OM + m) * 2] = Jm * Er;
            Rt[(nd * P2M_OM + m) * 2 + 1] = Jm * Ei;
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
      // the node's density products, right-hand sides split over the node's eight threads
      const double nur = p[2], nui = p[3];
      for (int rr = pt; rr < NR; rr += 8) {
        const double qr = p[5 + 4 * rr], qi = p[6 + 4 * rr], ur = p[7 + 4 * rr], ui = p[8 + 4 * rr];
        double* v = Vt + (nd * 3 * NR) * 2;
        v[(0 * NR + rr) * 2] = qr;
        v[(0 * NR + rr) * 2 + 1] = qi;
        v[(1 * NR + rr) * 2] = nur * ur - nui * ui;     // nu u
        v[(1 * NR + rr) * 2 + 1] = nur * ui + nui * ur;
        v[(2 * NR + rr) * 2] = nur * ur + nui * ui;     // conj(nu) u
        v[(2 * NR + rr) * 2 + 1] = nur * ui - nui * ur;
      }
    }
    __syncthreads();
    if (acc_thread) {
      // phase B: R_m v and R_-m v = (-1)^m conj(R_m) v over the chunk's nodes
      const int nn = (int)min<int64_t>(P2M_NC, b1 - c0);
      for (int nd = 0; nd < nn; ++nd) {
        const double rr_ = Rt[(nd * P2M_OM + om) * 2], ri_ = Rt[(nd * P2M_OM + om) * 2 + 1];
        const double* v = Vt + (nd * 3 * NR + kind * NR) * 2;
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          const double vr = v[2 * rr], vi = v[2 * rr + 1];
          pr[rr] = fma(rr_, vr, fma(-ri_, vi, pr[rr]));
          pi[rr] = fma(rr_, vi, fma(ri_, vr, pi[rr]));
          mr[rr] = fma(rr_, vr, fma(ri_, vi, mr[rr]));
          mi[rr] = fma(rr_, vi, fma(-ri_, vr, mi[rr]));
        }
      }
    }
    __syncthreads();
  }
  // the sums into acc[P2M_MO +- m][rr][2 kind ..]: the chunk buffers are free
  if (acc_thread) {
    const double sg = (om & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) {
      acc[P2M_MO + om][rr][2 * kind] = pr[rr];
      acc[P2M_MO + om][rr][2 * kind + 1] = pi[rr];
      if (om > 0) {
        acc[P2M_MO - om][rr][2 * kind] = sg * mr[rr];
        acc[P2M_MO - om][rr][2 * kind + 1] = sg * mi[rr];
      }
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
// and B_n in LDS, and each thread accumulates its (order, right-hand side) outputs in
// registers: orders up to the cluster's own order + 2 (its sources' J_n decay; beyond,
// the coefficients are below e^-PMX_APPLY_TRUNC of the leading ones and are written as zeros), child
// orders up to the child's order + 2.  The records are then written as p2m writes them,
// orders up to PMX_APPLY_PMAXC + 1.
constexpr int M2M_MO = PMX_APPLY_PMAXC + 2;                // outputs for orders -M2M_MO .. M2M_MO
constexpr int M2M_NM = 2 * M2M_MO + 1;
constexpr int M2M_NU = M2M_MO + PMX_APPLY_NRECA + 1;       // translation orders |m - n| <= M2M_NU
constexpr int M2M_NI = 2 * PMX_APPLY_NRECA + 1;            // child orders -NRECA .. NRECA
constexpr int M2M_KIDS = 4;
constexpr int M2M_THREADS = 512;
static_assert(M2M_NI >= M2M_NM, "the child stage holds the outputs at the end");

template <int NR>
__global__ __launch_bounds__(M2M_THREADS) void k_apply_m2m(ApplyArgs A, int c0) {
  constexpr int NOUT = (M2M_NM * NR + M2M_THREADS - 1) / M2M_THREADS;   // outputs per thread
  const int c = c0 + blockIdx.x;
  const int sc = A.n_incl + c;
  const double Cx = A.incl_geo[4 * sc], Cy = A.incl_geo[4 * sc + 1];
  const int mo = min((int)A.incl_geo[4 * sc + 3], PMX_APPLY_PMAXC) + 2;   // orders kept
  const double k = A.k;
  const int q0 = A.kid_off[c], nk = min(A.kid_off[c + 1] - q0, M2M_KIDS);
  __shared__ double jt[M2M_KIDS][M2M_NU + 1];
  __shared__ zd Rt[M2M_KIDS][2 * M2M_NU + 1];
  __shared__ zd An[NR][M2M_NI], Bn[NR][M2M_NI];
  const int tid = threadIdx.x;
  double aar[NOUT], aai[NOUT], abr[NOUT], abi[NOUT];
#pragma unroll
  for (int i = 0; i < NOUT; ++i) aar[i] = aai[i] = abr[i] = abi[i] = 0.0;
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
  for (int e = tid; e < nk * (2 * M2M_NU + 1); e += M2M_THREADS) {
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
    const int pch = min((int)A.incl_geo[4 * ch + 3], nrc - 1) + 2;        // child orders kept
    const int nlo = max(1 - nrc, -pch), nhi = min(nrc, pch);
    const zd* rec = A.coef + (int64_t)ch * PMX_APPLY_NRECA * NR * 6;
    __syncthreads();   // the previous child's A, B are read no more; the R table is complete
    // stored: A_n for |n| <= nrc - 1, B_n for 2 - nrc <= n <= nrc; the rest is zero
    for (int e = tid; e < NR * M2M_NI; e += M2M_THREADS) {
      const int rr = e / M2M_NI, n = e % M2M_NI - PMX_APPLY_NRECA;
      zd a = zmk(0, 0), b = zmk(0, 0);
      if (n >= 1 - nrc && n <= nrc - 1) a = n >= 0 ? rec[((int64_t)n * NR + rr) * 6] : rec[((int64_t)(-n) * NR + rr) * 6 + 1];
      if (n >= 2 - nrc && n <= nrc)
        b = n >= 1 ? rec[((int64_t)(n - 1) * NR + rr) * 6 + 2] : rec[((int64_t)(1 - n) * NR + rr) * 6 + 3];
      An[rr][n + PMX_APPLY_NRECA] = a;
      Bn[rr][n + PMX_APPLY_NRECA] = b;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
      const int e = tid + M2M_THREADS * i;
      const int m = e / NR - M2M_MO, rr = e % NR;
      if (e >= M2M_NM * NR || m < -mo || m > mo) continue;
      double ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll 4
      for (int n = nlo; n <= nhi; ++n) {
        const zd R = Rt[kc][m - n + M2M_NU];
        const zd a = An[rr][n + PMX_APPLY_NRECA], b = Bn[rr][n + PMX_APPLY_NRECA];
        ar = fma(-R.im, a.im, fma(R.re, a.re, ar));
        ai = fma(R.im, a.re, fma(R.re, a.im, ai));
        br = fma(-R.im, b.im, fma(R.re, b.re, br));
        bi = fma(R.im, b.re, fma(R.re, b.im, bi));
      }
      aar[i] += ar;
      aai[i] += ai;
      abr[i] += br;
      abi[i] += bi;
    }
  }
  // the outputs, orders -M2M_MO .. M2M_MO, into the child stage (An: A, Bn: B)
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NOUT; ++i) {
    const int e = tid + M2M_THREADS * i;
    if (e >= M2M_NM * NR) continue;
    const int mi = e / NR, rr = e % NR;
    An[rr][mi] = zmk(aar[i], aai[i]);
    Bn[rr][mi] = zmk(abr[i], abi[i]);
  }
  __syncthreads();
  zd* out = A.coef + (int64_t)sc * PMX_APPLY_NRECA * NR * 6;
  for (int e = tid; e < PMX_APPLY_NRECA * NR; e += M2M_THREADS) {
    const int m = e / NR, rr = e % NR;
    zd* o = out + ((int64_t)m * NR + rr) * 6;
    const zd z0 = zmk(0, 0);
    o[0] = An[rr][M2M_MO + m];
    o[1] = m ? An[rr][M2M_MO - m] : z0;
    o[2] = Bn[rr][M2M_MO + m + 1];
    o[3] = m ? Bn[rr][M2M_MO - m + 1] : z0;
    o[4] = Bn[rr][M2M_MO + m - 1];
    o[5] = m ? Bn[rr][M2M_MO - m - 1] : z0;
  }
}

// ---------------------------------------------------------------------------------
// Fast multipole part.  With O_n(v) = H_n(k|v|) e^{i n arg v} and I_m(v) = J_m(k|v|)
// e^{i m arg v}, Graf's addition theorem gives, for |u| < |D|,
//   O_n(u + D) = sum_m O_{n-m}(D) I_m(u)                         (M2L)
// and, for all u, d,  I_m(u + d) = sum_l I_{m-l}(d) I_l(u)         (L2L).
// A source's field sum_n X_n O_n(x - c_S) (X = A for value rows, B for derivative rows)
// is therefore sum_m L_m I_m(x - c_T) near c_T with L_m = sum_n O_{n-m}(c_T - c_S) X_n,
// a local expansion passes to a child as L'_l = sum_m I_{m-l}(c_C - c_P) L_m, and at a
// target  val = (i/4) sum_m L^A_m I_m,  der = (i/4)(k/2) sum_m I_m (nu L^B_{m+1} -
// conj(nu) L^B_{m-1})  (the normal derivative of I_m is (k/2)(nu I_{m-1} - conj(nu) I_{m+1})).

// X_n (X = 0: A, 1: B) of source record rec for right-hand side rr (layout of the records
// written by p2m and m2m: per order row m, A_m, A_-m, B_m+1, B_-m+1, B_m-1, B_-m-1, where
// row 0 holds zeros in its -m entries); |n| <= the source's record order - 1 for A, and
// 1 - n <= that order - 1 for B with n <= 0.
template <int NR>
__device__ inline zd rec_coef(const double* __restrict__ rec, int X, int n, int rr) {
  int row, slot;
  if (X == 0) {
    row = n >= 0 ? n : -n;
    slot = n >= 0 ? 0 : 1;
  } else {   // B_n: the B_{m+1} entry of row n - 1, or for n <= 0 the B_{-m+1} entry of row 1 - n
    row = n >= 1 ? n - 1 : 1 - n;
    slot = n >= 1 ? 2 : 3;
  }
  const double* c = rec + ((int64_t)row * NR + rr) * 12 + 2 * slot;
  return zmk(c[0], c[1]);
}

// O_nu(D), nu = -V .. V, of every M2L pair (one thread per pair): H0, H1 of k|D|, the
// upward recurrence H_{nu+1} = (2 nu / z) H_nu - H_{nu-1} (stable for the Hankel function),
// O_-nu = (-1)^nu H_nu e^{-i nu phi}.
__global__ __launch_bounds__(256) void k_apply_m2l_tab(ApplyArgs A, int n_pairs) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_pairs) return;
  const int t = A.m2l_slot[q], S = A.m2l_src[q];
  const int V = A.m2l_mmax[q] + 1 + A.m2l_nmax[q];
  const double dx = A.loc_geo[2 * t] - A.incl_geo[4 * S], dy = A.loc_geo[2 * t + 1] - A.incl_geo[4 * S + 1];
  const double z = A.k * sqrt(dx * dx + dy * dy), phi = atan2(dy, dx);
  const bes4 h = bessel01_mid(z);
  zd* out = A.m2l_tab + A.m2l_toff[q] + V;
  double hcr = h.j0, hci = h.y0, hpr = -h.j1, hpi = -h.y1;   // H_0, H_{-1} = -H_1
  const double iz2 = 2.0 / z;
  for (int nu = 0; nu <= V; ++nu) {
    double sn, cs;
    sincos(nu * phi, &sn, &cs);
    out[nu] = zmk(hcr * cs - hci * sn, hcr * sn + hci * cs);
    if (nu > 0) {
      const double sg = (nu & 1) ? -1.0 : 1.0;
      out[-nu] = zmk(sg * (hcr * cs + hci * sn), sg * (hci * cs - hcr * sn));
    }
    double hnr = nu * iz2 * hcr - hpr, hni = nu * iz2 * hci - hpi;
    if (nu == 0) {
      hnr = h.j1;
      hni = h.y1;
    }
    hpr = hcr;
    hpi = hci;
    hcr = hnr;
    hci = hni;
  }
}

// I_nu(d), nu = -W .. W, of every L2L pair (one thread per pair): J_nu(k|d|) by Miller's
// backward recurrence (rescaled against overflow, normalised by J_0 + 2 sum J_2k = 1).
__global__ __launch_bounds__(256) void k_apply_l2l_tab(ApplyArgs A, int n_pairs) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_pairs) return;
  const int c = A.l2l_child[q], P = A.l2l_parent[q];
  const int W = A.loc_p[P] + A.loc_p[c] + 2;
  const double dx = A.loc_geo[2 * c] - A.loc_geo[2 * P], dy = A.loc_geo[2 * c + 1] - A.loc_geo[2 * P + 1];
  const double z = A.k * sqrt(dx * dx + dy * dy), phi = atan2(dy, dx);
  zd* out = A.l2l_tab + A.l2l_toff[q] + W;
  if (!(z > 1e-300)) {   // coincident centres (a cluster with one child): the identity
    for (int nu = -W; nu <= W; ++nu) out[nu] = zmk(nu == 0 ? 1.0 : 0.0, 0.0);
    return;
  }
  const int nstart = W + 30 + (int)ceil(z);
  const double iz2 = 2.0 / z;
  double jp = 0.0, jc = 1e-280, nrm = 0.0;
  for (int m = nstart; m >= 1; --m) {
    const double jm = m * iz2 * jc - jp;   // J_{m-1}, unnormalised
    jp = jc;
    jc = jm;
    if (m - 1 <= W) out[m - 1] = zmk(jc, 0.0);
    if (((m - 1) & 1) == 0) nrm += (m - 1 == 0) ? jc : 2.0 * jc;
    if (fabs(jc) > 1e200) {   // rescale everything kept so far
      jp *= 1e-200;
      jc *= 1e-200;
      nrm *= 1e-200;
      for (int nu = m - 1; nu <= W; ++nu) out[nu].re *= 1e-200;
    }
  }
  const double inv = 1.0 / nrm;
  for (int nu = 0; nu <= W; ++nu) {
    const double J = out[nu].re * inv;
    double sn, cs;
    sincos(nu * phi, &sn, &cs);
    out[nu] = zmk(J * cs, J * sn);
    if (nu > 0) {
      const double sg = (nu & 1) ? -J : J;
      out[-nu] = zmk(sg * cs, -sg * sn);
    }
  }
}

void asm_apply_tables(const ApplyArgs& a, int n_m2l, int n_l2l, hipStream_t s) {
  if (n_m2l > 0)
    PMX_LAUNCH(k_apply_m2l_tab, dim3((n_m2l + 255) / 256), dim3(256), 0, s, a, n_m2l);
  if (n_l2l > 0)
    PMX_LAUNCH(k_apply_l2l_tab, dim3((n_l2l + 255) / 256), dim3(256), 0, s, a, n_l2l);
}

// The translated sources' coefficients in the layout the m2l kernel reads: per source,
// X (A, B), order n = -PMX_FMM_NMAX .. PMX_FMM_NMAX and right-hand side, contiguous in the
// right-hand side (one thread per entry; sources with expansion records only).
constexpr int M2L_NX = 2 * PMX_FMM_NMAX + 1;                        // orders of a source

template <int NR>
__global__ __launch_bounds__(256) void k_apply_m2l_coef(ApplyArgs A, const double* __restrict__ cf, int nsrc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nsrc * 2 * M2L_NX * NR) return;
  const int rr = (int)(e % NR);
  const int n = (int)((e / NR) % M2L_NX) - PMX_FMM_NMAX;
  const int X = (int)((e / (NR * M2L_NX)) % 2);
  const int S = (int)(e / (2 * NR * M2L_NX));
  const double* rec = cf + (int64_t)S * PMX_APPLY_NRECA * NR * 12;
  A.cm[e] = rec_coef<NR>(rec, X, n, rr);
}

// Part of a local expansion: the translated sources of work item blockIdx.x (a run of at
// most PMX_FMM_CHUNK pairs of one slot), one wave, into the item's partial sums.  Lane l
// holds the orders m = l - 32 (pass 0), and 32 j + l or l - 32 (j + 2) for l < 32 or
// l >= 32 (pass j = 1, 2), for every right-hand side; a pair with orders |m| <= mmax + 1
// runs the passes that hold them.  A and B are summed one after the other.  Per pair the
// wave stages its table O_nu in LDS (read per lane); the source's coefficients A_n, B_n
// (|n| <= nmax) are wave-uniform (scalar loads).
constexpr int M2L_TAB = 2 * (PMX_FMM_PL + 1 + PMX_FMM_NMAX) + 1;   // largest table
constexpr int M2L_PASS = 3;                                         // |m| <= 95
static_assert(PMX_FMM_PL + 1 <= 32 * M2L_PASS - 1, "local orders beyond the passes");

template <int NR>
__global__ __launch_bounds__(64) void k_apply_m2l(ApplyArgs A) {
  __shared__ zd tab_s[M2L_TAB];
  const int it = blockIdx.x;
  const int t = A.m2l_item[3 * it];
  const int lane = threadIdx.x;
  const int p = A.loc_p[t];
  const int q0 = A.m2l_item[3 * it + 1], q1 = A.m2l_item[3 * it + 2];
  int mj[M2L_PASS];
  mj[0] = lane - 32;
#pragma unroll
  for (int j = 1; j < M2L_PASS; ++j) mj[j] = lane < 32 ? 32 * j + lane : lane - 32 * (j + 2);
  zd* loc = A.m2l_part + (int64_t)it * 2 * PMX_FMM_NL * NR;
  for (int X = 0; X < 2; ++X) {
    double ar[M2L_PASS][NR], ai[M2L_PASS][NR];
#pragma unroll
    for (int j = 0; j < M2L_PASS; ++j)
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) ar[j][rr] = ai[j][rr] = 0.0;
    for (int q = q0; q < q1; ++q) {
      const int S = A.m2l_src[q], nmax = A.m2l_nmax[q], mm = A.m2l_mmax[q] + 1;
      const int V = mm + nmax;
      const zd* tab = A.m2l_tab + A.m2l_toff[q];
      const zd* xs = A.cm + (((int64_t)S * 2 + X) * M2L_NX + PMX_FMM_NMAX) * NR;   // X_n at xs[n NR + rr]
      __syncthreads();   // the previous pair's table is read no more
      for (int e = lane; e < 2 * V + 1; e += 64) tab_s[e] = tab[e];
      __syncthreads();
      const int npass = mm <= 31 ? 1 : (mm <= 63 ? 2 : 3);
      bool ok[M2L_PASS];
      int mc[M2L_PASS];
#pragma unroll
      for (int j = 0; j < M2L_PASS; ++j) {
        ok[j] = mj[j] >= -mm && mj[j] <= mm;
        mc[j] = min(max(mj[j], -mm), mm);   // lanes outside the pair's orders read a valid entry and add 0
      }
#pragma unroll(NR <= 4 ? 2 : 1)
      for (int n = -nmax; n <= nmax; ++n) {
        zd x[NR];
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) x[rr] = xs[n * NR + rr];
#pragma unroll
        for (int j = 0; j < M2L_PASS; ++j) {
          if (j < npass) {
            zd o = tab_s[n - mc[j] + V];
            if (!ok[j]) o = zmk(0.0, 0.0);
#pragma unroll
            for (int rr = 0; rr < NR; ++rr) {
              ar[j][rr] = fma(o.re, x[rr].re, fma(-o.im, x[rr].im, ar[j][rr]));
              ai[j][rr] = fma(o.re, x[rr].im, fma(o.im, x[rr].re, ai[j][rr]));
            }
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < M2L_PASS; ++j) {
      const int m = mj[j];
      if (m >= -(p + 1) && m <= p + 1) {
#pragma unroll
        for (int rr = 0; rr < NR; ++rr)
          loc[((int64_t)X * PMX_FMM_NL + (m + PMX_FMM_PL + 1)) * NR + rr] = zmk(ar[j][rr], ai[j][rr]);
      }
    }
  }
}

// Local expansions from their items' partial sums, added in item order (one thread per
// slot, X, order |m| <= p + 1 and right-hand side).
template <int NR>
__global__ __launch_bounds__(256) void k_apply_m2l_sum(ApplyArgs A) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)A.n_loc * 2 * PMX_FMM_NL * NR) return;
  const int rr = (int)(e % NR);
  const int mi = (int)((e / NR) % PMX_FMM_NL);
  const int X = (int)((e / (NR * PMX_FMM_NL)) % 2);
  const int t = (int)(e / (2 * NR * PMX_FMM_NL));
  const int p = A.loc_p[t];
  const int m = mi - (PMX_FMM_PL + 1);
  if (m < -(p + 1) || m > p + 1) return;
  const int i0 = A.m2l_item_off[t], i1 = A.m2l_item_off[t + 1];
  const int64_t o = ((int64_t)X * PMX_FMM_NL + mi) * NR + rr;
  zd acc = zmk(0.0, 0.0);
  for (int it = i0; it < i1; ++it) acc = zadd(acc, A.m2l_part[(int64_t)it * 2 * PMX_FMM_NL * NR + o]);
  A.loc[(int64_t)t * 2 * PMX_FMM_NL * NR + o] = acc;
}

// Parent-to-child translations of one tree level (one wave per child): L^C_l += sum_m
// I_{m-l}(c_C - c_P) L^P_m for |l| <= p_C + 1, |m| <= p_P + 1.
template <int NR>
__global__ __launch_bounds__(64) void k_apply_l2l(ApplyArgs A, int q0) {
  const int q = q0 + blockIdx.x;
  const int c = A.l2l_child[q], P = A.l2l_parent[q];
  const int lane = threadIdx.x;
  const int pc = A.loc_p[c], pp = A.loc_p[P];
  const int W = pp + pc + 2;
  const int npass = (2 * pc + 3 + 63) / 64;
  const zd* tab = A.l2l_tab + A.l2l_toff[q] + W;
  zd* lc = A.loc + (int64_t)c * 2 * PMX_FMM_NL * NR;
  const zd* lp = A.loc + (int64_t)P * 2 * PMX_FMM_NL * NR;
  for (int X = 0; X < 2; ++X) {
    double ar[3][NR], ai[3][NR];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) ar[j][rr] = ai[j][rr] = 0.0;
    for (int m = -(pp + 1); m <= pp + 1; ++m) {
      zd x[NR];
#pragma unroll
      for (int rr = 0; rr < NR; ++rr) x[rr] = lp[((int64_t)X * PMX_FMM_NL + (m + PMX_FMM_PL + 1)) * NR + rr];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (j < npass) {
          const int l = min(-(pc + 1) + lane + 64 * j, pc + 1);
          const zd o = tab[m - l];
#pragma unroll
          for (int rr = 0; rr < NR; ++rr) {
            ar[j][rr] = fma(o.re, x[rr].re, fma(-o.im, x[rr].im, ar[j][rr]));
            ai[j][rr] = fma(o.re, x[rr].im, fma(o.im, x[rr].re, ai[j][rr]));
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int l = -(pc + 1) + lane + 64 * j;
      if (j < npass && l <= pc + 1) {
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          zd* o = lc + ((int64_t)X * PMX_FMM_NL + (l + PMX_FMM_PL + 1)) * NR + rr;
          *o = zadd(*o, zmk(ar[j][rr], ai[j][rr]));
        }
      }
    }
  }
}

// Far part: part blockIdx.y of the wave's list of far sources (inclusions and clusters),
// each through its expansion: per lane rho, th of the target about the source's centre, H0
// and H1 (large-argument expansion when the whole wave allows it), then orders m = 0 .. p+1
// by the upward recurrence H_{m+1} = (2m/z) H_m - H_{m-1} (stable for the Hankel function)
// and e^{i(m+1)th} = e^{i m th} e^{i th}; O_{-m} = (-1)^m H_m e^{-i m th}.  The sums
// S1 = sum O_m B_{m+1}, S2 = sum O_m B_{m-1} are kept over all sources and turned into
// derivative rows once at the end.  Slice blockIdx.z takes right-hand sides NH z .. NH z +
// NH - 1 of the group of NR (the records keep the group's layout): fewer accumulators, so
// more waves per SIMD, for one Hankel evaluation and recurrence per slice.
template <int NR, int NH>
__global__ __launch_bounds__(256) void k_apply_far(ApplyArgs A, const double* __restrict__ cf, int r0) {
  const int wv = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * 256 + threadIdx.x) >> 6));
  if (wv >= A.n_waves) return;            // a wave past the last target (no barrier follows)
  const int lane = threadIdx.x & 63;
  const int w0 = A.wave_node[2 * wv], wn = A.wave_node[2 * wv + 1];
  const bool active = lane < wn;
  const int a = w0 + (active ? lane : wn - 1);   // idle lanes follow the wave's last node and write nothing
  const int h0 = (int)blockIdx.z * NH;   // this slice: right-hand sides h0 .. h0 + NH - 1 of the group
  const int nr = min(NH, A.nrhs - r0 - h0);
  if (nr <= 0) return;
  const double ax = A.x[a], ay = A.y[a], anx = A.nx[a], any = A.ny[a];
  const double k = A.k, ik = 1.0 / k;
  const double wcx = A.wave_geo[4 * wv], wcy = A.wave_geo[4 * wv + 1], wr = A.wave_geo[4 * wv + 2];
  double vr[NH], vi[NH], s1r[NH], s1i[NH], s2r[NH], s2i[NH];
#pragma unroll
  for (int r = 0; r < NH; ++r) vr[r] = vi[r] = s1r[r] = s1i[r] = s2r[r] = s2i[r] = 0.0;
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
    // this slice's part of the next source's record rows (12 NH doubles a row), one double
    // per 128-byte line, is read into L2 while this source is summed, so that the scalar
    // loads of the next source find it there
    double pf = 0.0;
    if (q + 1 < q1) {
      const int j1 = A.far_idx[q + 1];
      const int rows = min((int)A.incl_geo[4 * j1 + 3] + 2, PMX_APPLY_NRECA);
      const double* r1 = cf + (int64_t)j1 * PMX_APPLY_NRECA * NR * 12 + h0 * 12;
      constexpr int LPR = (12 * NH + 15) / 16;   // lines of a row's slice
      for (int c = lane; c < rows * LPR; c += 64) pf += r1[(c / LPR) * NR * 12 + (c % LPR) * 16];
    }
    for (int m = 0; m <= p + 1; ++m) {
      const double sg = (m & 1) ? -1.0 : 1.0;
      const double Opr = Hcr * Emr - Hci * Emi, Opi = Hcr * Emi + Hci * Emr;               // O_m
      const double Omr = sg * (Hcr * Emr + Hci * Emi), Omi = sg * (Hci * Emr - Hcr * Emi);  // O_-m
      const double* o = rec + (int64_t)m * NR * 12;
#pragma unroll
      for (int rr = 0; rr < NH; ++rr) {
        // A_m, A_-m, B_m+1, B_-m+1, B_m-1, B_-m-1 (wave-uniform addresses: scalar loads)
        const double* c = o + (h0 + rr) * 12;
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
    vr[0] = fma(fmin(fabs(pf), 1.0), 0.0, vr[0]);   // keeps the prefetch; adds zero
  }
  // the local expansion of the wave's inclusion (part 0 only): I_m(x - c_T) = J_m e^{i m th}
  // with J_m by Miller's backward recurrence (a first pass for the norm J_0 + 2 sum J_2k),
  // accumulated from the top order down, as S1 and S2 above with I_m in place of O_m
  const int own = A.owner[w0];
  const int slot = A.loc_id[own];
  if (blockIdx.y == 0 && slot >= 0) {
    const int p = A.loc_p[slot];
    const zd* L = A.loc + (int64_t)slot * 2 * PMX_FMM_NL * NR;
    const double ux = ax - A.loc_geo[2 * slot], uy = ay - A.loc_geo[2 * slot + 1];
    const double rho = fmax(sqrt(ux * ux + uy * uy), 1e-300);
    const double z = k * rho;
    const double er = ux / rho, ei = uy / rho;   // e^{i th}
    const int nstart = __builtin_amdgcn_readfirstlane(p + 26 + (int)ceil(k * wr + k * sqrt((wcx - A.loc_geo[2 * slot]) *
                                                                                   (wcx - A.loc_geo[2 * slot]) +
                                                                               (wcy - A.loc_geo[2 * slot + 1]) *
                                                                                   (wcy - A.loc_geo[2 * slot + 1]))));
    const double iz2 = 2.0 / fmax(z, 1e-300);
    double jp = 0.0, jc = 1e-280, nrm = (nstart % 2 == 0) ? 2.0 * jc : 0.0;
    for (int m = nstart; m >= 1; --m) {
      const double jm = m * iz2 * jc - jp;
      jp = jc;
      jc = jm;
      if (((m - 1) & 1) == 0) nrm += (m - 1 == 0) ? jm : 2.0 * jm;
    }
    const double inv = (z > 1e-12) ? 1.0 / nrm : 0.0;
    // e^{i p th} by repeated squaring, then stepped down
    double Er = 1.0, Ei = 0.0, br = er, bi = ei;
    for (int e = p; e > 0; e >>= 1) {
      if (e & 1) {
        const double t = Er * br - Ei * bi;
        Ei = Er * bi + Ei * br;
        Er = t;
      }
      const double t = br * br - bi * bi;
      bi = 2.0 * br * bi;
      br = t;
    }
    jp = 0.0;
    jc = 1e-280;
    for (int m = nstart; m >= 0; --m) {
      if (m <= p) {
        // J_m; at the centre itself only J_0 = 1 survives
        const double Jm = (z > 1e-12) ? jc * inv : (m == 0 ? 1.0 : 0.0);
        const double sg = (m & 1) ? -1.0 : 1.0;
        const double Ipr = Jm * Er, Ipi = Jm * Ei;                 // I_m
        const double Imr = sg * Jm * Er, Imi = -sg * Jm * Ei;      // I_-m
        const zd* la = L + (int64_t)(m + PMX_FMM_PL + 1) * NR + h0;                // L^A_m
        const zd* lna = L + (int64_t)(-m + PMX_FMM_PL + 1) * NR + h0;              // L^A_-m
        const zd* lb = L + (int64_t)(PMX_FMM_NL + m + PMX_FMM_PL + 1) * NR + h0;   // L^B_m
        const zd* lnb = L + (int64_t)(PMX_FMM_NL - m + PMX_FMM_PL + 1) * NR + h0;  // L^B_-m
#pragma unroll
        for (int rr = 0; rr < NH; ++rr) {
          zd c = la[rr];
          vr[rr] = fma(Ipr, c.re, fma(-Ipi, c.im, vr[rr]));
          vi[rr] = fma(Ipr, c.im, fma(Ipi, c.re, vi[rr]));
          c = lb[NR + rr];   // L^B_{m+1}
          s1r[rr] = fma(Ipr, c.re, fma(-Ipi, c.im, s1r[rr]));
          s1i[rr] = fma(Ipr, c.im, fma(Ipi, c.re, s1i[rr]));
          c = lb[-NR + rr];  // L^B_{m-1}
          s2r[rr] = fma(Ipr, c.re, fma(-Ipi, c.im, s2r[rr]));
          s2i[rr] = fma(Ipr, c.im, fma(Ipi, c.re, s2i[rr]));
          if (m > 0) {
            c = lna[rr];
            vr[rr] = fma(Imr, c.re, fma(-Imi, c.im, vr[rr]));
            vi[rr] = fma(Imr, c.im, fma(Imi, c.re, vi[rr]));
            c = lnb[NR + rr];   // L^B_{-m+1}
            s1r[rr] = fma(Imr, c.re, fma(-Imi, c.im, s1r[rr]));
            s1i[rr] = fma(Imr, c.im, fma(Imi, c.re, s1i[rr]));
            c = lnb[-NR + rr];  // L^B_{-m-1}
            s2r[rr] = fma(Imr, c.re, fma(-Imi, c.im, s2r[rr]));
            s2i[rr] = fma(Imr, c.im, fma(Imi, c.re, s2i[rr]));
          }
        }
        // e^{i (m-1) th} = e^{i m th} e^{-i th}
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
  if (!active) return;
  // der = (k/2)(nu S1 - conj(nu) S2)
  const double hk = 0.5 * k;
  double dr[NH], di[NH];
#pragma unroll
  for (int rr = 0; rr < NH; ++rr) {
    dr[rr] = hk * (anx * s1r[rr] - any * s1i[rr] - (anx * s2r[rr] + any * s2i[rr]));
    di[rr] = hk * (anx * s1i[rr] + any * s1r[rr] - (anx * s2i[rr] - any * s2r[rr]));
  }
  apply_store<NH>(A, A.part + (int64_t)blockIdx.y * A.nrhs * A.ld, r0 + h0, nr, a, vr, vi, dr, di);
}

// Near part: one wave per workgroup; part blockIdx.y of the wave's near list, every
// argument through the general Bessel evaluation; pairs on the target's own inclusion
// (the self block, applied separately) are left out.
template <int NR>
__global__ __launch_bounds__(64) void k_apply_near(ApplyArgs A, const double* __restrict__ pk, int r0, int slot0) {
  constexpr int S = APPLY_SRC(NR);
  const int wv = blockIdx.x;
  const int w0 = A.wave_node[2 * wv], wn = A.wave_node[2 * wv + 1];
  const bool active = (int)threadIdx.x < wn;
  const int a = w0 + (active ? (int)threadIdx.x : wn - 1);
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

// Near pairs through stored Bessel values.  Every (wave, near inclusion) pair has a block of
// the pair's J0 + i Y0 and J1 + i Y1 at k+ |x_t - x_s| for each source node and target lane,
// made once per solve state: entry (b, c, lane) of block q at near_blk[near_blk_off[q] +
// (2 b + c) 64 + lane].  The apply streams them (coalesced) and forms the four coefficients
// of apply_pair from the pair's geometry, so that it reads 32 B a pair instead of 64 B.
__global__ __launch_bounds__(64) void k_apply_near_build(ApplyArgs A) {
  const int wv = blockIdx.x;
  const int w0 = A.wave_node[2 * wv], wn = A.wave_node[2 * wv + 1];
  const int lane = threadIdx.x;
  const int a = w0 + (lane < wn ? lane : wn - 1);
  const double ax = A.x[a], ay = A.y[a];
  const double k = A.k;
  for (int q = A.near_off[wv]; q < A.near_off[wv + 1]; ++q) {
    const int j = A.near_idx[q];
    const int bb0 = (int)A.node_off[j], b1 = (int)A.node_off[j + 1];
    zd* blk = A.near_blk + A.near_blk_off[q];
    for (int b = bb0; b < b1; ++b) {
      pmx_ctab tab = (pmx_ctab)pmx_far_table.v, ser = (pmx_ctab)pmx_series_table.v;
      asm volatile("" : "+s"(tab), "+s"(ser));
      const double d1 = ax - A.x[b], d2 = ay - A.y[b];
      const double dd = d1 * d1 + d2 * d2;
      const double ir = rsqrt_nr(dd);
      const bes4 h = bessel01_t(k * (dd * ir), tab, ser);
      zd* e = blk + (int64_t)(b - bb0) * 2 * 64 + lane;
      e[0] = zmk(h.j0, h.y0);
      e[64] = zmk(h.j1, h.y1);
    }
  }
}

void asm_apply_near_build(const ApplyArgs& a, hipStream_t s) {
  if (a.near_blk && a.n_waves > 0) PMX_LAUNCH(k_apply_near_build, dim3(a.n_waves), dim3(64), 0, s, a);
}

template <int NR>
__global__ __launch_bounds__(64) void k_apply_near_blk(ApplyArgs A, const double* __restrict__ pk, int r0, int slot0) {
  constexpr int S = APPLY_SRC(NR);
  const int wv = blockIdx.x;
  const int w0 = A.wave_node[2 * wv], wn = A.wave_node[2 * wv + 1];
  const int lane = threadIdx.x;
  const bool active = lane < wn;
  const int a = w0 + (active ? lane : wn - 1);
  const int nr = min(NR, A.nrhs - r0);
  double vr[NR], vi[NR], dr[NR], di[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) vr[r] = vi[r] = dr[r] = di[r] = 0.0;
  const double ax = A.x[a], ay = A.y[a], anx = A.nx[a], any = A.ny[a];
  const double k = A.k, eps = A.eps, ke = k / eps;
  const int qs = A.near_off[wv], len = A.near_off[wv + 1] - qs;
  const int ns = A.nsplit_near, y = blockIdx.y;
  const int q0 = qs + (int)((int64_t)len * y / ns), q1 = qs + (int)((int64_t)len * (y + 1) / ns);
  for (int q = q0; q < q1; ++q) {
    const int j = A.near_idx[q];
    const int bb0 = (int)A.node_off[j], b1 = (int)A.node_off[j + 1];
    const zd* blk = A.near_blk + A.near_blk_off[q] + lane;
    for (int b = bb0; b < b1; ++b) {
      const zd* e = blk + (int64_t)(b - bb0) * 2 * 64;
      const zd h0 = e[0], h1 = e[64];
      const double* p = pk + (int64_t)b * S;
      const double d1 = ax - p[0], d2 = ay - p[1];
      const double ir = rsqrt_nr(d1 * d1 + d2 * d2);
      apply_pair<NR>(h0.re, h1.re, h0.im, h1.im, ir, d1, d2, anx, any, p, k, eps, ke, 1.0, vr, vi, dr, di);
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

int64_t apply_m2l_coef_size(int n_src, int nr_max) { return (int64_t)n_src * 2 * M2L_NX * nr_max; }

int apply_source_order(double kr) {
  for (int p = 1; p < 1000; ++p)
    if (p > 0.5 * M_E * kr + 2 && std::pow(0.5 * M_E * kr / p, p) <= std::exp(-PMX_APPLY_TRUNC)) return p;
  return 1000;
}

template <int NR>
static void apply_group(const ApplyArgs& A, double* pk, int r0, int nsplit, hipStream_t s) {
  PMX_LAUNCH(k_apply_pack<NR>, dim3((A.n_nodes + 255) / 256), dim3(256), 0, s, A, r0, pk);
  const int m = (int)A.n_incl;
  PMX_LAUNCH(k_apply_p2m<NR>, dim3(m), dim3(256), 0, s, A, (const double*)pk, r0);
  for (int l = 0; l < A.n_lev; ++l)
    if (A.lev_off[l + 1] > A.lev_off[l])
      PMX_LAUNCH(k_apply_m2m<NR>, dim3(A.lev_off[l + 1] - A.lev_off[l]), dim3(M2M_THREADS), 0, s, A,
                         A.lev_off[l]);
  if (A.n_loc > 0) {
    const int nsrc = A.n_incl + A.lev_off[A.n_lev];   // sources with expansion records
    const int64_t ncm = (int64_t)nsrc * 2 * M2L_NX * NR;
    PMX_LAUNCH(k_apply_m2l_coef<NR>, dim3((unsigned)((ncm + 255) / 256)), dim3(256), 0, s, A,
                       (const double*)A.coef, nsrc);
    if (A.n_m2l_items > 0) PMX_LAUNCH(k_apply_m2l<NR>, dim3(A.n_m2l_items), dim3(64), 0, s, A);
    const int64_t nl = (int64_t)A.n_loc * 2 * PMX_FMM_NL * NR;
    PMX_LAUNCH(k_apply_m2l_sum<NR>, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s, A);
    for (int l = 0; l < A.n_l2l_lev; ++l)
      if (A.l2l_lev[l + 1] > A.l2l_lev[l])
        PMX_LAUNCH(k_apply_l2l<NR>, dim3(A.l2l_lev[l + 1] - A.l2l_lev[l]), dim3(64), 0, s, A, A.l2l_lev[l]);
  }
  // groups of 8 right-hand sides run as two workgroup slices of 4 (half the accumulators)
  constexpr int NH = NR > 4 ? NR / 2 : NR;
  PMX_LAUNCH((k_apply_far<NR, NH>), dim3((A.n_waves + 3) / 4, nsplit, NR / NH), dim3(256), 0, s, A,
                     (const double*)A.coef, r0);
}

// near pairs of a group of right-hand sides (the Bessel functions of a pair are evaluated
// once per group, so the near part takes the largest groups)
template <int NR>
static void near_group(const ApplyArgs& A, double* pk, int r0, int nsplit, hipStream_t s) {
  PMX_LAUNCH(k_apply_pack<NR>, dim3((A.n_nodes + 255) / 256), dim3(256), 0, s, A, r0, pk);
  if (A.near_blk)
    PMX_LAUNCH(k_apply_near_blk<NR>, dim3(A.n_waves, A.nsplit_near), dim3(64), 0, s, A, (const double*)pk,
                       r0, nsplit);
  else
    PMX_LAUNCH(k_apply_near<NR>, dim3(A.n_waves, A.nsplit_near), dim3(64), 0, s, A, (const double*)pk, r0,
                       nsplit);
}

// groups of g right-hand sides: g = nr_max while enough remain; a last smaller group takes
// the smallest size of 1, 2, 4, 8 (16 for the near part) that holds it
static int group_size(int left, int nr_max) {
  return left >= nr_max ? nr_max : (left <= 1 ? 1 : left <= 2 ? 2 : left <= 4 ? 4 : left <= 8 ? 8 : 16);
}

// expansions, translations and far parts in groups of nr_max (1, 2, 4 or 8) right-hand
// sides, then the near parts in groups of up to PMX_APPLY_NR_NEAR
void asm_apply_off(const ApplyArgs& A, int nsplit, int nr_max, hipStream_t s) {
  if (A.n_nodes <= 0 || A.nrhs <= 0) return;
  for (int r0 = 0; r0 < A.nrhs;) {
    const int g = group_size(A.nrhs - r0, nr_max);
    switch (g) {
      case 1: apply_group<1>(A, A.pack, r0, nsplit, s); break;
      case 2: apply_group<2>(A, A.pack, r0, nsplit, s); break;
      case 4: apply_group<4>(A, A.pack, r0, nsplit, s); break;
      default: apply_group<8>(A, A.pack, r0, nsplit, s); break;
    }
    r0 += g;
  }
  // stored coefficients: the largest groups (the coefficients are read once per group)
  const int nr_near = A.near_blk ? 16 : PMX_APPLY_NR_NEAR;
  for (int r0 = 0; r0 < A.nrhs;) {
    const int g = group_size(A.nrhs - r0, nr_near);
    switch (g) {
      case 1: near_group<1>(A, A.pack, r0, nsplit, s); break;
      case 2: near_group<2>(A, A.pack, r0, nsplit, s); break;
      case 4: near_group<4>(A, A.pack, r0, nsplit, s); break;
      case 8: near_group<8>(A, A.pack, r0, nsplit, s); break;
      default: near_group<16>(A, A.pack, r0, nsplit, s); break;
    }
    r0 += g;
  }
}

void asm_apply_finish(const zd* f, const zd* ydiag, const zd* part, int nsplit, int64_t total, double sf, double sa,
                      zd* out, hipStream_t s) {
  if (total <= 0) return;
  PMX_LAUNCH(k_apply_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f, ydiag, part, nsplit,
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
  PMX_LAUNCH(k_colnorm2, dim3(nblk, ncol), dim3(256), 0, s, a, n, ld, part);
}
