// Dense FP64 application of the PMCHWT (Omit) Nystrom operator, evaluated on the fly, for
// the residual r = f - A x of iterative refinement (arXiv 2603.09381, Sec. 2.2 system).
//
// The self blocks A_ii are applied as a batched FP64 MFMA product with the stored Kress
// blocks.  The blocks between different inclusions use only k+ and the source's trapezoid
// weight; with x~ = w x at the source and H_n = J_n + i Y_n of k+ r, the value and
// normal-derivative rows of a target node receive
//   val += (i/4) [ -e+ H0 q~ + k (n_s.d/r) H1 u~ ],
//   der += (i/4) [ k (n_t.d/r) H1 q~ + (k/e+) (k a H0 + b H1) u~ ],
// a = (n_t.d)(n_s.d)/r^2, b = (n_t.n_s - 2 a)/r, d = x_t - x_s: the four operators S, D,
// D*, N of Sec. 2.1 written out.  One thread owns one target node and NR right-hand
// sides; sources are read with wave-uniform (scalar) loads, in a far kernel (pairs with
// k+ r >= 24, large-argument expansion only) over source ranges and a near kernel over
// each wave's near inclusions; partial sums are reduced by a third kernel in a fixed
// order.
#include "assemble.h"
#include "bessel.h"
#include "hankel_fast.h"
#include "ktimer.h"

#include <algorithm>

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
__constant__ FarTable pmx_far_table = make_far_table();

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
__constant__ SeriesTable pmx_series_table = make_series_table();

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

// Far part: every source inclusion of range blockIdx.y outside the wave's near list.  All
// arguments are >= PMX_APPLY_FAR_Z, so the large-argument expansion alone serves, with as
// many terms as the wave's smallest argument needs.  No per-lane branch in the loop.
template <int NR>
__global__ __launch_bounds__(256) void k_apply_far(ApplyArgs A, const double* __restrict__ pk, int r0) {
  constexpr int S = APPLY_SRC(NR);
  const int N = A.n_nodes;
  const int a_raw = blockIdx.x * 256 + threadIdx.x;
  const bool active = a_raw < N;
  const int a = active ? a_raw : N - 1;   // idle lanes follow the last node and write nothing
  const int wv = __builtin_amdgcn_readfirstlane(a_raw >> 6);
  if (wv >= (N + 63) / 64) return;        // a wave past the last target (no barrier follows)
  const int nr = min(NR, A.nrhs - r0);
  const double ax = A.x[a], ay = A.y[a], anx = A.nx[a], any = A.ny[a];
  const double k = A.k, eps = A.eps;
  const double ik = 1.0 / k, ke = k / eps;
  double vr[NR], vi[NR], dr[NR], di[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) vr[r] = vi[r] = dr[r] = di[r] = 0.0;
  int q = A.near_off[wv];
  const int qe = A.near_off[wv + 1];
  const int j0 = A.split_incl[blockIdx.y], j1 = A.split_incl[blockIdx.y + 1];
  int nxt = q < qe ? A.near_idx[q] : 0x7fffffff;
  while (nxt < j0) {
    ++q;
    nxt = q < qe ? A.near_idx[q] : 0x7fffffff;
  }
  for (int j = j0; j < j1; ++j) {
    if (j == nxt) {
      ++q;
      nxt = q < qe ? A.near_idx[q] : 0x7fffffff;
      continue;
    }
    const int b1 = (int)A.node_off[j + 1];
    for (int b = (int)A.node_off[j]; b < b1; ++b) {
      pmx_ctab tab = (pmx_ctab)pmx_far_table.v;
      asm volatile("" : "+s"(tab));   // re-read the coefficients in every iteration
      const double* p = pk + (int64_t)b * S;
      const double d1 = ax - p[0], d2 = ay - p[1];
      const double ir = rsqrt_nr(d1 * d1 + d2 * d2);
      const double z = k * ((d1 * d1 + d2 * d2) * ir);
      double J0, J1, Y0, Y1;
      if (__all(z >= 60.0))
        hankel_far_t<12>(z, ir * ik, tab, J0, J1, Y0, Y1);
      else if (__all(z >= 35.0))
        hankel_far_t<16>(z, ir * ik, tab, J0, J1, Y0, Y1);
      else
        hankel_far_t<20>(z, ir * ik, tab, J0, J1, Y0, Y1);
      apply_pair<NR>(J0, J1, Y0, Y1, ir, d1, d2, anx, any, p, k, eps, ke, 1.0, vr, vi, dr, di);
    }
  }
  if (active) apply_store<NR>(A, A.part + (int64_t)blockIdx.y * A.nrhs * A.ld, r0, nr, a, vr, vi, dr, di);
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

template <int NR>
static void apply_group(const ApplyArgs& A, double* pk, int r0, int nsplit, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_pack<NR>, dim3((A.n_nodes + 255) / 256), dim3(256), 0, s, A, r0, pk);
  KScope ks(PK_APPLY, s);
  hipLaunchKernelGGL(k_apply_far<NR>, dim3((A.n_nodes + 255) / 256, nsplit), dim3(256), 0, s, A, (const double*)pk,
                     r0);
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
