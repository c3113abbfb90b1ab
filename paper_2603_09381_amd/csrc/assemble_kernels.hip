// Kernel-matrix assembly for the PMCHWT (Omit) system (arXiv 2603.09381, Sec. 2),
// FP64 on gfx950 vector ALUs.
//
// Kernels: G = (i/4) H0(k r) with d = x - y, r = |d|; the four operators of Sec. 2.1
// (eqs. slp, dlp, d_slp, d_dlp):
//   S  = (i/4) H0,  D = (ik/4) H1 (n_y.d)/r,  D* = -(ik/4) H1 (n_x.d)/r,
//   N  = (ik/4) [k H0 (n_x.d)(n_y.d)/r^2 - 2 H1 (n_x.d)(n_y.d)/r^3 + H1 (n_x.n_y)/r].
// Off-diagonal blocks of the Omit form use only k+ and the trapezoid weight of the
// source node (Sec. 2.2):  [[-e+ S, D], [-D*, N/e+]].  Self blocks use both k+ and
// the inclusion's k- with Kress' logarithmic product quadrature, or the paper's
// zeta-corrected trapezoid rule with 41 local correction points (Sec. 2.2), and N written by
// Maue's identity N = |x'|^-1 D_t S |x'|^-1 D_t + k^2 S_nn (trigonometric
// differentiation D_t), then combined as
//   [[-(e+ S+ + e- S-), D+ + D-], [-(D*+ + D*-), N+/e+ + N-/e-]].
#include <algorithm>
#include <cmath>
#include <mutex>

#include "assemble.h"
#include "bessel.h"
#include "hankel_fast.h"
#include "ktimer.h"
#include "zeta_table.h"

struct Pt {
  double x, y, nx, ny, w;
  int type;
};

__device__ inline Pt fetch_pt(const DevGeom& g, const DevProxy& p, int code) {
  Pt q;
  if (code >= 0) {
    int n = code >> 1;
    q.type = code & 1;
    q.x = g.x[n];
    q.y = g.y[n];
    q.nx = g.nx[n];
    q.ny = g.ny[n];
    q.w = g.w[n];
  } else {
    int c = -code - 1;
    int i = c >> 1;
    q.type = c & 1;
    q.x = p.x[i];
    q.y = p.y[i];
    q.nx = p.nx[i];
    q.ny = p.ny[i];
    q.w = p.w[i];
  }
  return q;
}

// One entry of the exterior (Omit off-diagonal) operator between target t (row type)
// and source s (column type, carrying its quadrature weight).
// constant-memory copies of the coefficient tables (one per translation unit)
static __constant__ FarTable pmx_far_table = make_far_table();
static __constant__ SeriesTable pmx_series_table = make_series_table();

// The entry from its geometry (d = x_t - x_s, 1/|d|) and the Bessel values at k+ |d|.
__device__ inline zd omit_entry_from(const Pt& t, const Pt& s, double d1, double d2, double ir, const bes4& b,
                                     const ExtParams& e) {
  if (t.type == 0) {
    if (s.type == 0) {  // -e+ (i/4) H0 w
      const double f = 0.25 * e.eps * s.w;
      return zmk(f * b.y0, -f * b.j0);
    }
    const double f = 0.25 * e.k * (s.nx * d1 + s.ny * d2) * ir * s.w;  // (ik/4) H1 (n_s.d)/r w
    return zmk(-f * b.y1, f * b.j1);
  }
  const double ntd = (t.nx * d1 + t.ny * d2) * ir;
  if (s.type == 0) {  // -D* w = (ik/4) H1 (n_t.d)/r w
    const double f = 0.25 * e.k * ntd * s.w;
    return zmk(-f * b.y1, f * b.j1);
  }
  const double nsd = (s.nx * d1 + s.ny * d2) * ir;
  const double a = ntd * nsd;
  const double bc = (t.nx * s.nx + t.ny * s.ny - 2.0 * a) * ir;
  const double X = e.k * b.j0 * a + b.j1 * bc;
  const double Y = e.k * b.y0 * a + b.y1 * bc;
  const double f = 0.25 * e.k * s.w / e.eps;
  return zmk(-f * Y, f * X);
}

__device__ inline bes4 omit_bessel(double kr) {
  // coefficient tables read through scalar loads at each use (kept out of vector registers)
  pmx_ctab tab = (pmx_ctab)pmx_far_table.v, ser = (pmx_ctab)pmx_series_table.v;
  asm volatile("" : "+s"(tab), "+s"(ser));
  return bessel01_t(kr, tab, ser);
}

__device__ inline zd omit_entry(const Pt& t, const Pt& s, const ExtParams& e) {
  const double d1 = t.x - s.x, d2 = t.y - s.y;
  const double r = sqrt(d1 * d1 + d2 * d2);
  const double ir = 1.0 / r;
  return omit_entry_from(t, s, d1, d2, ir, omit_bessel(e.k * r), e);
}

// ---------------------------------------------------------------------------------
__global__ void k_geometry(const double* dx, const double* dy, const double* ddx, const double* ddy,
                           const int* owner, const int64_t* node_off, double* nx, double* ny,
                           double* w, double* speed, double* kappa, int n_nodes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  const double a = dx[i], b = dy[i];
  const double sp = sqrt(a * a + b * b);
  const int j = owner[i];
  const double n = (double)(node_off[j + 1] - node_off[j]);
  speed[i] = sp;
  nx[i] = b / sp;
  ny[i] = -a / sp;
  w[i] = (2.0 * PMX_PI / n) * sp;
  kappa[i] = (a * ddy[i] - b * ddx[i]) / (sp * sp * sp);
}

void asm_geometry(const double* dx, const double* dy, const double* ddx, const double* ddy,
                  const int* owner, const int64_t* node_off, double* nx, double* ny, double* w,
                  double* speed, double* kappa, int n_nodes, hipStream_t s) {
  if (n_nodes <= 0) return;
  PMX_LAUNCH(k_geometry, dim3((n_nodes + 255) / 256), dim3(256), 0, s, dx, dy, ddx, ddy,
                     owner, node_off, nx, ny, w, speed, kappa, n_nodes);
}

// Kress weights R_d = -(2pi/h) sum_{m<h} cos(m t_d)/m - (pi/h^2) cos(h t_d), n = 2h, and the
// trigonometric differentiation stencil dt_d = (1/2)(-1)^d cot(t_d/2), t_d = 2 pi d / n.
// With quad = 1 R holds the zeta-corrected trapezoid rule instead (Sec. 2.2): the self-block
// entry R_d K1 + q (K - K1 L_d) (L_d = ln 4 sin^2(t_d/2), q = 2 pi / n) then equals q K plus
// the correction q w_|d| (2 K1) on the 2 P + 1 nearest nodes, and q (K2 + 2 K1 (ln(q/2pi) + w_0))
// on the diagonal: R_0 = 2 q (ln(q / 2 pi) + w_0), R_d = q L_d + 2 q w_min(d, n-d) (0 beyond P).
__global__ void k_tables(const int* ns, const int* tbl_off, double* R, double* dt, int quad) {
  const int t = blockIdx.y;
  const int n = ns[t];
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const int h = n / 2;
  double s = 0;
  for (int m = h - 1; m >= 1; --m) {
    const int ph = (int)(((int64_t)m * d) % n);
    s += cos(2.0 * PMX_PI * ph / n) / m;
  }
  const double sign = (d & 1) ? -1.0 : 1.0;
  if (quad == 1) {
    const double q = 2.0 * PMX_PI / n;
    const int dm = min(d, n - d);
    const double wz = dm <= PMX_ZETA_P ? pmx_zeta_w[dm] : 0.0;
    if (d == 0) {
      R[tbl_off[t]] = 2.0 * q * (log(q / (2.0 * PMX_PI)) + wz);
    } else {
      const double sn = sin(PMX_PI * d / n);
      R[tbl_off[t] + d] = q * log(4.0 * sn * sn) + 2.0 * q * wz;
    }
  } else {
    R[tbl_off[t] + d] = -(2.0 * PMX_PI / h) * s - (PMX_PI / ((double)h * h)) * sign;
  }
  dt[tbl_off[t] + d] = d == 0 ? 0.0 : 0.5 * sign / tan(PMX_PI * d / n);
}

void asm_tables(const int* ns, const int* tbl_off, int ntbl, int max_n, double* R, double* dt, int quad,
                hipStream_t s) {
  if (ntbl <= 0) return;
  PMX_LAUNCH(k_tables, dim3((max_n + 127) / 128, ntbl), dim3(128), 0, s, ns, tbl_off, R, dt, quad);
}

// ---------------------------------------------------------------------------------
// self block, pair stage: everything except the D_t products of Maue's identity
struct KressOps {
  zd S, D, Ds, Snn;
};

__device__ inline KressOps kress_pair(double k, double r, double d1, double d2, double nxa, double nya,
                                      double nxb, double nyb, double spb, double Rw, double L, double q) {
  const bes4 b = bessel01(k * r);
  const double ir = 1.0 / r;
  const double ndy = (nxb * d1 + nyb * d2) * ir;
  const double ndx = (nxa * d1 + nya * d2) * ir;
  const double nn = nxa * nxb + nya * nyb;
  const double i4p = 1.0 / (4.0 * PMX_PI);
  KressOps o;
  // S: K = (-y0/4 + i j0/4) sp, K1 = -j0 sp/(4 pi)
  {
    const double K1 = -b.j0 * spb * i4p;
    o.S = zmk(Rw * K1 + q * (-0.25 * b.y0 * spb - K1 * L), q * 0.25 * b.j0 * spb);
    o.Snn = zscale(o.S, nn);
  }
  // D: K = (ik/4) H1 ndy sp = (-k y1/4 + i k j1/4) ndy sp, K1 = -(k/4pi) j1 ndy sp
  {
    const double f = ndy * spb;
    const double K1 = -k * i4p * b.j1 * f;
    o.D = zmk(Rw * K1 + q * (-0.25 * k * b.y1 * f - K1 * L), q * 0.25 * k * b.j1 * f);
  }
  // D*: K = -(ik/4) H1 ndx sp = (k y1/4 - i k j1/4) ndx sp, K1 = (k/4pi) j1 ndx sp
  {
    const double f = ndx * spb;
    const double K1 = k * i4p * b.j1 * f;
    o.Ds = zmk(Rw * K1 + q * (0.25 * k * b.y1 * f - K1 * L), -q * 0.25 * k * b.j1 * f);
  }
  return o;
}

__device__ inline KressOps kress_self(double k, double sp, double kap, double R0, double q) {
  KressOps o;
  const double i4p = 1.0 / (4.0 * PMX_PI);
  const double K1 = -sp * i4p;
  const zd K2 = zmk((-PMX_EULER / (2.0 * PMX_PI) - log(0.5 * k * sp) / (2.0 * PMX_PI)) * sp, 0.25 * sp);
  o.S = zmk(R0 * K1 + q * K2.re, q * K2.im);
  o.Snn = o.S;
  o.D = zmk(-q * kap * sp * i4p, 0.0);
  o.Ds = o.D;
  return o;
}

__global__ __launch_bounds__(256) void k_diag_pairs(DevGeom g, ExtParams e, const DiagDesc* ds,
                                                     const double* R) {
  const DiagDesc d = ds[blockIdx.y];
  const int n = d.n;
  const int e_idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (e_idx >= n * n) return;
  const int a = e_idx % n, b = e_idx / n;
  const int ia = d.node0 + a, ib = d.node0 + b;
  const double q = 2.0 * PMX_PI / n;
  const int dd = ((a - b) % n + n) % n;
  const double Rw = R[d.tbl + dd];
  KressOps P, M;
  if (a == b) {
    P = kress_self(e.k, g.speed[ia], g.kappa[ia], Rw, q);
    M = kress_self(d.k_int, g.speed[ia], g.kappa[ia], Rw, q);
  } else {
    const double d1 = g.x[ia] - g.x[ib], d2 = g.y[ia] - g.y[ib];
    const double r = sqrt(d1 * d1 + d2 * d2);
    const double sn = sin(PMX_PI * dd / n);
    const double L = log(4.0 * sn * sn);
    P = kress_pair(e.k, r, d1, d2, g.nx[ia], g.ny[ia], g.nx[ib], g.ny[ib], g.speed[ib], Rw, L, q);
    M = kress_pair(d.k_int, r, d1, d2, g.nx[ia], g.ny[ia], g.nx[ib], g.ny[ib], g.speed[ib], Rw, L, q);
  }
  const double ep = e.eps, em = d.eps_int;
  const int64_t ld = 2 * n;
  zd* out = d.out;
  out[a + (int64_t)b * ld] = zadd(zscale(P.S, -ep), zscale(M.S, -em));
  out[a + (int64_t)(n + b) * ld] = zadd(P.D, M.D);
  out[(n + a) + (int64_t)b * ld] = zscale(zadd(P.Ds, M.Ds), -1.0);
  out[(n + a) + (int64_t)(n + b) * ld] =
      zadd(zscale(P.Snn, e.k * e.k / ep), zscale(M.Snn, d.k_int * d.k_int / em));
  d.scratch[a + (int64_t)b * n] = zadd(zscale(P.S, 1.0 / ep), zscale(M.S, 1.0 / em));
}

// W = X |x'|^-1 D_t   (X in scratch, W to scratch2).  The block's stencil and 1/|x'| go to
// LDS first; the circulant index advances by one per term, so the loop has no division and
// no modulo.
__global__ __launch_bounds__(256) void k_diag_maue1(DevGeom g, const DiagDesc* ds, const double* dt) {
  extern __shared__ double dm_lds[];   // [n] stencil, [n] 1/|x'|
  const DiagDesc d = ds[blockIdx.y];
  const int n = d.n;
  if ((int)(blockIdx.x * blockDim.x) >= n * n) return;   // the whole workgroup
  double* tbs = dm_lds;
  double* isp = dm_lds + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    tbs[i] = dt[d.tbl + i];
    isp[i] = 1.0 / g.speed[d.node0 + i];
  }
  __syncthreads();
  const int e_idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (e_idx >= n * n) return;
  const int c = e_idx % n, b = e_idx / n;
  double sr = 0, si = 0;
  int dd = (b == 0) ? 0 : n - b;   // (k - b) mod n at k = 0
  for (int k = 0; k < n; ++k) {
    const double f = tbs[dd] * isp[k];
    const zd x = d.scratch[c + (int64_t)k * n];
    sr = fma(x.re, f, sr);
    si = fma(x.im, f, si);
    dd = (dd + 1 == n) ? 0 : dd + 1;
  }
  d.scratch2[c + (int64_t)b * n] = zmk(sr, si);
}

// A22 += |x'|^-1 D_t W, the stencil in LDS as above
__global__ __launch_bounds__(256) void k_diag_maue2(DevGeom g, const DiagDesc* ds, const double* dt) {
  extern __shared__ double dm_lds[];   // [n] stencil
  const DiagDesc d = ds[blockIdx.y];
  const int n = d.n;
  if ((int)(blockIdx.x * blockDim.x) >= n * n) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dm_lds[i] = dt[d.tbl + i];
  __syncthreads();
  const int e_idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (e_idx >= n * n) return;
  const int a = e_idx % n, b = e_idx / n;
  double sr = 0, si = 0;
  int dd = a;   // (a - c) mod n at c = 0
  for (int c = 0; c < n; ++c) {
    const zd w = d.scratch2[c + (int64_t)b * n];
    const double t = dm_lds[dd];
    sr = fma(t, w.re, sr);
    si = fma(t, w.im, si);
    dd = (dd == 0) ? n - 1 : dd - 1;
  }
  const double f = 1.0 / g.speed[d.node0 + a];
  const int64_t ld = 2 * n;
  zd* o = d.out + (n + a) + (int64_t)(n + b) * ld;
  *o = zadd(*o, zmk(sr * f, si * f));
}

void asm_diag(DevGeom g, ExtParams e, const DiagDesc* d, int batch, int max_n, const double* R,
              const double* dt, hipStream_t s) {
  if (batch <= 0 || max_n <= 0) return;
  dim3 grid((max_n * max_n + 255) / 256, batch);
  KScope ks(PK_DIAG, s);
  PMX_LAUNCH(k_diag_pairs, grid, dim3(256), 0, s, g, e, d, R);
  const size_t shm = 2 * (size_t)max_n * sizeof(double);
  if (shm > 64 * 1024) {
    (void)hipFuncSetAttribute((const void*)k_diag_maue1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipFuncSetAttribute((const void*)k_diag_maue2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  }
  PMX_LAUNCH(k_diag_maue1, grid, dim3(256), shm, s, g, d, dt);
  PMX_LAUNCH(k_diag_maue2, grid, dim3(256), shm / 2, s, g, d, dt);
}

// ---------------------------------------------------------------------------------
#define ENT_ROWS 64
#define ENT_COLS 16
template <class R>
__global__ __launch_bounds__(256) void k_entries(DevGeom g, DevProxy p, ExtParams e, const EntryMatT<R>* ms) {
  const EntryMatT<R> m = ms[blockIdx.z];
  const int i = blockIdx.x * ENT_ROWS + (threadIdx.x & 63);
  const int j0 = blockIdx.y * ENT_COLS + (threadIdx.x >> 6);
  if (blockIdx.x * ENT_ROWS >= m.na || blockIdx.y * ENT_COLS >= m.nb) return;
  if (i >= m.na) return;
  const Pt pa = fetch_pt(g, p, m.a[i]);
  for (int j = j0; j < min(m.nb, (int)(blockIdx.y + 1) * ENT_COLS); j += 4) {
    const Pt pb = fetch_pt(g, p, m.b[j]);
    const zd v = m.a_is_target ? omit_entry(pa, pb, e) : omit_entry(pb, pa, e);
    m.out[i + (int64_t)j * m.ld] = cmk<R>(v.re, v.im);
  }
}

template <class R>
void asm_entries(DevGeom g, DevProxy p, ExtParams e, const EntryMatT<R>* d, int batch, int max_a, int max_b,
                 hipStream_t s) {
  if (batch <= 0 || max_a <= 0 || max_b <= 0) return;
  dim3 grid((max_a + ENT_ROWS - 1) / ENT_ROWS, (max_b + ENT_COLS - 1) / ENT_COLS, batch);
  KScope ks(PK_ENTRIES, s);
  PMX_LAUNCH(k_entries<R>, grid, dim3(256), 0, s, g, p, e, d);
}

// The node-node part of the four ID matrices of a one-inclusion cell against one near
// one-inclusion cell: for the pair (near node i, own node j) the Bessel values at k+ |x_i -
// x_j| serve all eight entries: rows (i, value) and (i, derivative) of the q- and u-column
// IDs (target i, source j), and rows (i, q) and (i, u) of the value- and derivative-row IDs
// (target j, source i).  Each entry equals what omit_entry gives for it.
template <class R>
__global__ __launch_bounds__(256) void k_leaf_pairs(DevGeom g, ExtParams e, const LeafPairDescT<R>* ds) {
  const LeafPairDescT<R> d = ds[blockIdx.x];
  const int64_t np = (int64_t)d.n_near * d.n_own;
  for (int64_t q = threadIdx.x; q < np; q += blockDim.x) {
    const int li = (int)(q % d.n_near), lj = (int)(q / d.n_near);
    const int ni = d.near0 + li, nj = d.own0 + lj;
    Pt pi, pj;
    pi.x = g.x[ni];
    pi.y = g.y[ni];
    pi.nx = g.nx[ni];
    pi.ny = g.ny[ni];
    pi.w = g.w[ni];
    pj.x = g.x[nj];
    pj.y = g.y[nj];
    pj.nx = g.nx[nj];
    pj.ny = g.ny[nj];
    pj.w = g.w[nj];
    const double d1 = pi.x - pj.x, d2 = pi.y - pj.y;
    const double r = sqrt(d1 * d1 + d2 * d2);
    const double ir = 1.0 / r;
    const bes4 b = omit_bessel(e.k * r);
    const double d1r = pj.x - pi.x, d2r = pj.y - pi.y;   // reversed pair, same |d| and Bessel values
    const int64_t o0 = li + (int64_t)lj * d.ld, o1 = o0 + d.n_near;
#pragma unroll
    for (int kd = 0; kd < 4; ++kd) {
      zd v0, v1;
      if (kd < 2) {   // column IDs: target i (value, derivative row), source j (q or u column)
        pj.type = kd;
        pi.type = 0;
        v0 = omit_entry_from(pi, pj, d1, d2, ir, b, e);
        pi.type = 1;
        v1 = omit_entry_from(pi, pj, d1, d2, ir, b, e);
      } else {        // row IDs: target j (value or derivative row), source i (q, u column)
        pj.type = kd - 2;
        pi.type = 0;
        v0 = omit_entry_from(pj, pi, d1r, d2r, ir, b, e);
        pi.type = 1;
        v1 = omit_entry_from(pj, pi, d1r, d2r, ir, b, e);
      }
      d.out[kd][o0] = cmk<R>(v0.re, v0.im);
      d.out[kd][o1] = cmk<R>(v1.re, v1.im);
    }
  }
}

template <class R>
void asm_leaf_pairs(DevGeom g, ExtParams e, const LeafPairDescT<R>* d, int n, hipStream_t s) {
  if (n <= 0) return;
  KScope ks(PK_ENTRIES, s);
  PMX_LAUNCH(k_leaf_pairs<R>, dim3(n), dim3(256), 0, s, g, e, d);
}

template <class R>
__global__ __launch_bounds__(256) void k_parent(DevGeom g, ExtParams e, const ParentDescT<R>* ds) {
  const ParentDescT<R> d = ds[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d.s * d.s) return;
  const int a = (int)(idx % d.s), b = (int)(idx / d.s);
  const int ra = d.rloc[a], cb = d.cloc[b];
  const int sa = ra >> 24, sb = cb >> 24;
  cx<R> v;
  if (sa == sb) {
    const int la = ra & 0xFFFFFF, lb = cb & 0xFFFFFF;
    v = d.at[sa][la + (int64_t)lb * d.kc[sa]];
  } else {
    DevProxy none{nullptr, nullptr, nullptr, nullptr, nullptr};
    const zd w = omit_entry(fetch_pt(g, none, d.rcode[a]), fetch_pt(g, none, d.ccode[b]), e);
    v = cmk<R>(w.re, w.im);
  }
  d.out[idx] = v;
}

template <class R>
void asm_parent(DevGeom g, ExtParams e, const ParentDescT<R>* d, int batch, int max_s, hipStream_t s) {
  if (batch <= 0 || max_s <= 0) return;
  int64_t tot = (int64_t)max_s * max_s;
  PMX_LAUNCH(k_parent<R>, dim3((unsigned)((tot + 255) / 256), batch), dim3(256), 0, s, g, e, d);
}

// ---------------------------------------------------------------------------------
__global__ void k_incident(DevGeom g, ExtParams e, const int* cell_node0, const int* cell_n,
                           const int64_t* cell_off, const double* angles, int nrhs, zd* f) {
  const int c = blockIdx.z;
  const int n = cell_n[c];
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (row >= 2 * n || r >= nrhs) return;
  const int node = cell_node0[c] + (row < n ? row : row - n);
  double sa, ca;
  sincos(angles[r], &sa, &ca);
  const double ph = e.k * (ca * g.x[node] + sa * g.y[node]);
  double s, co;
  sincos(ph, &s, &co);
  zd u = zmk(co, s);
  zd v;
  if (row < n) {
    v = zmk(-u.re, -u.im);
  } else {
    const double dn = e.k * (ca * g.nx[node] + sa * g.ny[node]) / e.eps;  // q = i k (d.n)/e u
    v = zmk(dn * u.im, -dn * u.re);                                        // -(i dn) u
  }
  f[cell_off[c] + row + (int64_t)r * 2 * n] = v;
}

void asm_incident(DevGeom g, ExtParams e, const int* cell_node0, const int* cell_n,
                  const int64_t* cell_off, int ncell, int max_n, const double* angles, int nrhs,
                  zd* f, hipStream_t s) {
  if (ncell <= 0 || nrhs <= 0) return;
  dim3 grid((2 * max_n + 127) / 128, nrhs, ncell);
  PMX_LAUNCH(k_incident, grid, dim3(128), 0, s, g, e, cell_node0, cell_n, cell_off,
                     angles, nrhs, f);
}

template <class RS, class RD, bool ACC>
__global__ void k_gather(const cx<RS>* src, const GatherDescT<RD>* ds) {
  const GatherDescT<RD> d = ds[blockIdx.z];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= d.nrows || c >= d.ncols) return;
  const RowSrc rs = d.src[i];
  const cx<RS> v = src[rs.off + (int64_t)c * rs.ld];
  cx<RD>* o = d.dst + i + (int64_t)c * d.ld;
  if (ACC)
    *o = cmk<RD>(o->re + (RD)v.re, o->im + (RD)v.im);
  else
    *o = cmk<RD>((RD)v.re, (RD)v.im);
}

template <class RS, class RD>
void asm_gather(const cx<RS>* src, const GatherDescT<RD>* d, int batch, int max_rows, int max_cols, hipStream_t s,
                int acc) {
  if (batch <= 0 || max_rows <= 0 || max_cols <= 0) return;
  dim3 grid((max_rows + 63) / 64, (max_cols + 3) / 4, batch);
  if (acc)
    PMX_LAUNCH((k_gather<RS, RD, true>), grid, dim3(256), 0, s, src, d);
  else
    PMX_LAUNCH((k_gather<RS, RD, false>), grid, dim3(256), 0, s, src, d);
}

template <class R>
__global__ void k_identity(const Mat2T<R>* ds) {
  const Mat2T<R> d = ds[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)d.n * d.n) return;
  const int i = (int)(e % d.n), j = (int)(e / d.n);
  d.p[i + j * d.ld] = cmk<R>(i == j ? 1 : 0, 0);
}

template <class R>
void asm_identity(const Mat2T<R>* d, int batch, int max_n, hipStream_t s) {
  if (batch <= 0 || max_n <= 0) return;
  int64_t tot = (int64_t)max_n * max_n;
  PMX_LAUNCH(k_identity<R>, dim3((unsigned)((tot + 255) / 256), batch), dim3(256), 0, s, d);
}

template <class R>
__global__ void k_zero(cx<R>* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = cmk<R>(0, 0);
}

template <class R>
void asm_zero(cx<R>* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH(k_zero<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

// Near row and column code lists of every cell of a level (one workgroup per cell): the
// active codes of its near cells in list order, then its proxy points, value type first.
__global__ __launch_bounds__(256) void k_near_lists(const int* rows, const int* cols, const int64_t* offS,
                                                     const int* noff, const int* nidx, const int64_t* nro,
                                                     const int* poff, const int* np, int* nr, int* ncl) {
  const int t = blockIdx.x;
  int64_t o = nro[t];
  for (int q = noff[t]; q < noff[t + 1]; ++q) {
    const int sg = nidx[q];
    const int64_t b = offS[sg];
    const int len = (int)(offS[sg + 1] - b);
    for (int i = threadIdx.x; i < len; i += 256) {
      nr[o + i] = rows[b + i];
      ncl[o + i] = cols[b + i];
    }
    o += len;
  }
  const int P = np[t], p0 = poff[t];
  for (int i = threadIdx.x; i < 2 * P; i += 256) {
    const int ty = i / P, k = i - ty * P;
    const int c = pmx_code_proxy(p0 + k, ty);
    nr[o + i] = c;
    ncl[o + i] = c;
  }
}

void asm_near_lists(const int* rows, const int* cols, const int64_t* offS, const int* noff, const int* nidx,
                    const int64_t* nro, const int* poff, const int* np, int ncell, int* nr, int* ncl, hipStream_t s) {
  if (ncell <= 0) return;
  PMX_LAUNCH(k_near_lists, dim3(ncell), dim3(256), 0, s, rows, cols, offS, noff, nidx, nro, poff, np, nr, ncl);
}

__global__ void k_zero_i32(int* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void asm_zero_i32(int* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

template <class RS, class RD>
__global__ void k_convert(const cx<RS>* src, cx<RD>* dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = cmk<RD>((RD)src[i].re, (RD)src[i].im);
}

template <class RS, class RD>
void asm_convert(const cx<RS>* src, cx<RD>* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH((k_convert<RS, RD>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
}

// block t of dst = block of src at soff[t], rounded to RD (len[t] entries each)
template <class RD>
__global__ void k_convert_blocks(const zd* src, cx<RD>* dst, const int64_t* soff, const int64_t* doff,
                                 const int64_t* len) {
  const int t = blockIdx.y;
  const int64_t n = len[t], so = soff[t], dof = doff[t];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[dof + i] = cmk<RD>((RD)src[so + i].re, (RD)src[so + i].im);
}

template <class RD>
void asm_convert_blocks(const zd* src, cx<RD>* dst, const int64_t* d_soff, const int64_t* d_doff,
                        const int64_t* d_len, int nblocks, int64_t max_len, hipStream_t s) {
  if (nblocks <= 0 || max_len <= 0) return;
  const unsigned gx = (unsigned)std::min<int64_t>(64, (max_len + 255) / 256);
  PMX_LAUNCH(k_convert_blocks<RD>, dim3(gx, nblocks), dim3(256), 0, s, src, dst, d_soff, d_doff, d_len);
}

__global__ void k_axpy(zd* y, const zd* x, zd a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = zfma(a, x[i], y[i]);
}

void asm_axpy(zd* y, const zd* x, zd a, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, a, n);
}

// ---------------------------------------------------------------------------------
// u_inf(xh) = e^{i pi/4}/sqrt(8 pi k) sum_b w_b [-i k (xh.n_b) u_b - e+ q_b] e^{-i k xh.y_b}
// (Colton-Kress normalisation of the exterior representation of Sec. 2.1).
//
// The node sum is split into `nsplit` contiguous node ranges so that the grid fills the
// chip also for few directions and right-hand sides; each workgroup sums PMX_FF_GROUP
// directions of one right-hand side over one range (node data read once for the group)
// and writes its partial sums, which a second kernel adds in split order (deterministic)
// and scales by the normalisation.  Directions travel as kernel arguments, so the pair
// needs no device copy of them.
constexpr int PMX_FF_GROUP = 4;

__global__ __launch_bounds__(256) void k_far_field_part(DevGeom g, ExtParams e, const int* owner,
                                                         const int64_t* node_off, const zd* dens, int nrhs,
                                                         FarDirs D, int ndir, int64_t chunk, zd* part) {
  const int t0 = blockIdx.x * PMX_FF_GROUP, r = blockIdx.y, sp = blockIdx.z;
  const int nt = min(PMX_FF_GROUP, D.nt - t0);
  const int64_t lo = (int64_t)sp * chunk, hi = min((int64_t)g.n_nodes, lo + chunk);
  const int64_t ld = 2 * (int64_t)g.n_nodes;
  double cx[PMX_FF_GROUP], sx[PMX_FF_GROUP], ar[PMX_FF_GROUP], ai[PMX_FF_GROUP];
#pragma unroll
  for (int a = 0; a < PMX_FF_GROUP; ++a) {
    const int t = t0 + min(a, nt - 1);
    cx[a] = D.c[t];
    sx[a] = D.s[t];
    ar[a] = 0;
    ai[a] = 0;
  }
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const int j = owner[i];
    const int64_t o = node_off[j];
    const int64_t n = node_off[j + 1] - o;
    const int64_t l = i - o;
    const zd q = dens[r * ld + 2 * o + l];
    const zd u = dens[r * ld + 2 * o + n + l];
    const double px = g.x[i], py = g.y[i], nx = g.nx[i], ny = g.ny[i], wi = g.w[i];
#pragma unroll
    for (int a = 0; a < PMX_FF_GROUP; ++a) {
      const double xn = cx[a] * nx + sx[a] * ny;
      // -i k xn u - e q
      const zd v = zmk(e.k * xn * u.im - e.eps * q.re, -e.k * xn * u.re - e.eps * q.im);
      double s, c;
      sincos(-e.k * (cx[a] * px + sx[a] * py), &s, &c);
      const zd p = zmul(v, zmk(c, s));
      ar[a] = fma(wi, p.re, ar[a]);
      ai[a] = fma(wi, p.im, ai[a]);
    }
  }
  __shared__ double red[2 * PMX_FF_GROUP][4];
#pragma unroll
  for (int a = 0; a < PMX_FF_GROUP; ++a) {
    for (int o = 32; o >= 1; o >>= 1) {
      ar[a] += __shfl_xor(ar[a], o, 64);
      ai[a] += __shfl_xor(ai[a], o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[2 * a][threadIdx.x >> 6] = ar[a];
      red[2 * a + 1][threadIdx.x >> 6] = ai[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < nt) {
    const int a = threadIdx.x;
    const double sr = red[2 * a][0] + red[2 * a][1] + red[2 * a][2] + red[2 * a][3];
    const double si = red[2 * a + 1][0] + red[2 * a + 1][1] + red[2 * a + 1][2] + red[2 * a + 1][3];
    part[((int64_t)sp * nrhs + r) * ndir + D.t0 + t0 + a] = zmk(sr, si);
  }
}

__global__ __launch_bounds__(256) void k_far_field_finish(const zd* part, int nsplit, int nrhs, int ndir, double k,
                                                           zd* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)nrhs * ndir;
  if (i >= n) return;
  double sr = 0, si = 0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const zd v = part[(int64_t)sp * n + i];
    sr += v.re;
    si += v.im;
  }
  const double amp = 1.0 / sqrt(8.0 * PMX_PI * k);
  const double c4 = 0.70710678118654752440;
  out[i] = zmul(zmk(c4 * amp, c4 * amp), zmk(sr, si));
}

int far_field_splits(int64_t n_nodes, int nrhs, int ndir) {
  // about 2048 workgroups in all, ranges of at least 2048 nodes, at most 256 ranges
  const int64_t per = (int64_t)nrhs * ((ndir + PMX_FF_GROUP - 1) / PMX_FF_GROUP);
  int64_t ns = std::max<int64_t>(1, (2048 + per - 1) / per);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, (n_nodes + 2047) / 2048));
  return (int)std::min<int64_t>(ns, 256);
}

size_t far_field_part_bytes(int64_t n_nodes, int nrhs, int ndir) {
  return sizeof(zd) * (size_t)far_field_splits(n_nodes, nrhs, ndir) * (size_t)nrhs * (size_t)ndir;
}

void asm_far_field(DevGeom g, ExtParams e, const int* owner, const int64_t* node_off, const zd* dens, int nrhs,
                   const double* dirs, int ndir, zd* part, zd* out, hipStream_t s) {
  if (nrhs <= 0 || ndir <= 0) return;
  const int nsplit = far_field_splits(g.n_nodes, nrhs, ndir);
  const int64_t chunk = ((int64_t)g.n_nodes + nsplit - 1) / nsplit;
  for (int t0 = 0; t0 < ndir; t0 += PMX_FF_DIRS) {
    FarDirs D;
    D.t0 = t0;
    D.nt = std::min(PMX_FF_DIRS, ndir - t0);
    for (int a = 0; a < PMX_FF_DIRS; ++a) {
      const double th = dirs[t0 + std::min(a, D.nt - 1)];
      D.c[a] = std::cos(th);
      D.s[a] = std::sin(th);
    }
    const dim3 grid((D.nt + PMX_FF_GROUP - 1) / PMX_FF_GROUP, nrhs, nsplit);
    PMX_LAUNCH(k_far_field_part, grid, dim3(256), 0, s, g, e, owner, node_off, dens, nrhs, D, ndir,
                       chunk, part);
  }
  const int64_t n = (int64_t)nrhs * ndir;
  PMX_LAUNCH(k_far_field_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nsplit, nrhs,
                     ndir, e.k, out);
}

// The partial sums of the allocation-free far field live in this file-scope array, one
// copy per GPU, for the life of the process.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and is kept per device.
static __device__ __align__(256) double scratch[PMX_FF_SCRATCH_BYTES / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[PMX_MAX_DEVICES] = {};
}  // namespace

hipError_t far_field_scratch(zd** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= PMX_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = (zd*)g_scratch_ptr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------------
template <class R>
__global__ void k_build_l(const LDescT<R>* ds) {
  const LDescT<R> d = ds[blockIdx.z];
  const int type = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int sb = type ? d.s1 : d.s0;
  if (j >= sb) return;
  const int kb = type ? d.k1 : d.k0;
  const int* piv = type ? d.piv1 : d.piv0;
  const cx<R>* t = type ? d.t1 : d.t0;
  const int ldt = type ? d.ldt1 : d.ldt0;
  const int off_r = type ? d.s0 : 0;
  const int off_c = type ? d.k0 : 0;
  const int64_t s = d.s0 + d.s1;
  const int row = off_r + piv[j];
  if (j < kb) {
    d.out[row + (int64_t)(off_c + j) * s] = cmk<R>(1, 0);
  } else {
    for (int i = 0; i < kb; ++i) d.out[row + (int64_t)(off_c + i) * s] = t[i + (int64_t)(j - kb) * ldt];
  }
}

template <class R>
void asm_build_l(const LDescT<R>* d, int batch, int max_s, int max_k, hipStream_t s) {
  (void)max_k;
  if (batch <= 0 || max_s <= 0) return;
  dim3 grid((max_s + 127) / 128, 2, batch);
  PMX_LAUNCH(k_build_l<R>, grid, dim3(128), 0, s, d);
}

__global__ void k_probe_bessel(const double* z, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bes4 b = bessel01(z[i]);
  out[i] = b.j0;
  out[n + i] = b.j1;
  out[2 * n + i] = b.y0;
  out[3 * n + i] = b.y1;
}

void asm_probe_bessel(const double* z, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH(k_probe_bessel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, n, out);
}

// explicit instantiations: storage in complex FP64 and complex FP32
#define PMX_ASM_INST(R)                                                                                    \
  template void asm_entries<R>(DevGeom, DevProxy, ExtParams, const EntryMatT<R>*, int, int, int, hipStream_t); \
  template void asm_leaf_pairs<R>(DevGeom, ExtParams, const LeafPairDescT<R>*, int, hipStream_t);             \
  template void asm_parent<R>(DevGeom, ExtParams, const ParentDescT<R>*, int, int, hipStream_t);          \
  template void asm_identity<R>(const Mat2T<R>*, int, int, hipStream_t);                                  \
  template void asm_zero<R>(cx<R>*, int64_t, hipStream_t);                                                \
  template void asm_build_l<R>(const LDescT<R>*, int, int, int, hipStream_t);
PMX_ASM_INST(double)
PMX_ASM_INST(float)
#undef PMX_ASM_INST
template void asm_gather<double, double>(const zd*, const GatherDescT<double>*, int, int, int, hipStream_t, int);
template void asm_gather<float, float>(const zf*, const GatherDescT<float>*, int, int, int, hipStream_t, int);
template void asm_gather<double, float>(const zd*, const GatherDescT<float>*, int, int, int, hipStream_t, int);
template void asm_gather<float, double>(const zf*, const GatherDescT<double>*, int, int, int, hipStream_t, int);
template void asm_convert_blocks<float>(const zd*, zf*, const int64_t*, const int64_t*, const int64_t*, int, int64_t,
                                        hipStream_t);
template void asm_convert_blocks<double>(const zd*, zd*, const int64_t*, const int64_t*, const int64_t*, int, int64_t,
                                         hipStream_t);
template void asm_convert<double, float>(const zd*, zf*, int64_t, hipStream_t);
template void asm_convert<float, double>(const zf*, zd*, int64_t, hipStream_t);
template void asm_convert<double, double>(const zd*, zd*, int64_t, hipStream_t);
template void asm_convert<float, float>(const zf*, zf*, int64_t, hipStream_t);
