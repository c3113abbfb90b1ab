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
// sides; sources are staged through LDS in tiles and split over workgroups (partial sums
// reduced by a second kernel, in a fixed order).
#include "assemble.h"
#include "bessel.h"
#include "ktimer.h"

#include <algorithm>

#define APPLY_TS 128

template <int NR>
__global__ __launch_bounds__(256) void k_apply_off(ApplyArgs A, int r0, int per_split) {
  __shared__ double sx[APPLY_TS], sy[APPLY_TS], snx[APPLY_TS], sny[APPLY_TS];
  __shared__ int sown[APPLY_TS];
  __shared__ zd sq[NR][APPLY_TS], su[NR][APPLY_TS];
  const int tid = threadIdx.x;
  const int N = A.n_nodes;
  const int a = blockIdx.x * 256 + tid;
  const bool active = a < N;
  const int b0 = blockIdx.y * per_split;
  const int b1 = min(b0 + per_split, N);
  const int nr = min(NR, A.nrhs - r0);
  double ax = 0, ay = 0, anx = 0, any = 0;
  int aown = -1;
  if (active) {
    ax = A.x[a];
    ay = A.y[a];
    anx = A.nx[a];
    any = A.ny[a];
    aown = A.owner[a];
  }
  const double k = A.k, eps = A.eps;
  const double ke = k / eps;
  zd val[NR], der[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    val[r] = zmk(0, 0);
    der[r] = zmk(0, 0);
  }
  for (int t0 = b0; t0 < b1; t0 += APPLY_TS) {
    const int nt = min(APPLY_TS, b1 - t0);
    if (tid < APPLY_TS) {
      const int b = t0 + tid;
      if (tid < nt) {
        const int own = A.owner[b];
        const int64_t o = A.node_off[own];
        const int64_t n = A.node_off[own + 1] - o;
        const double w = A.w[b];
        sx[tid] = A.x[b];
        sy[tid] = A.y[b];
        snx[tid] = A.nx[b];
        sny[tid] = A.ny[b];
        sown[tid] = own;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          zd q = zmk(0, 0), u = zmk(0, 0);
          if (r < nr) {
            const zd* col = A.xin + (int64_t)(r0 + r) * A.ld + 2 * o + (b - o);
            q = col[0];
            u = col[n];
          }
          sq[r][tid] = zscale(q, w);
          su[r][tid] = zscale(u, w);
        }
      }
    }
    __syncthreads();
    if (active) {
      for (int j = 0; j < nt; ++j) {
        if (sown[j] == aown) continue;
        const double d1 = ax - sx[j], d2 = ay - sy[j];
        const double r = sqrt(d1 * d1 + d2 * d2);
        const double ir = 1.0 / r;
        const bes4 h = bessel01(k * r);
        const double nsd = (snx[j] * d1 + sny[j] * d2) * ir;
        const double ntd = (anx * d1 + any * d2) * ir;
        const double aa = ntd * nsd;
        const double bc = (anx * snx[j] + any * sny[j] - 2.0 * aa) * ir;
        const zd c1 = zmk(-eps * h.j0, -eps * h.y0);
        const zd c2 = zmk(k * nsd * h.j1, k * nsd * h.y1);
        const zd c3 = zmk(k * ntd * h.j1, k * ntd * h.y1);
        const zd c4 = zmk(ke * (k * aa * h.j0 + bc * h.j1), ke * (k * aa * h.y0 + bc * h.y1));
#pragma unroll
        for (int rr = 0; rr < NR; ++rr) {
          const zd q = sq[rr][j], u = su[rr][j];
          val[rr] = zfma(c1, q, zfma(c2, u, val[rr]));
          der[rr] = zfma(c3, q, zfma(c4, u, der[rr]));
        }
      }
    }
    __syncthreads();
  }
  if (!active) return;
  const int64_t o = A.node_off[aown];
  const int64_t n = A.node_off[aown + 1] - o;
  zd* out = A.part + (int64_t)blockIdx.y * A.nrhs * A.ld;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      zd* col = out + (int64_t)(r0 + r) * A.ld + 2 * o + (a - o);
      // times i/4
      col[0] = zmk(-0.25 * val[r].im, 0.25 * val[r].re);
      col[n] = zmk(-0.25 * der[r].im, 0.25 * der[r].re);
    }
  }
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

int apply_splits(int n_nodes, int nrhs) {
  const int nwg = (n_nodes + 255) / 256;
  const int chunks = (nrhs + 7) / 8;
  int ns = (2048 + nwg * chunks - 1) / (nwg * chunks);
  ns = std::max(1, std::min(ns, 64));
  // at least one full source tile per split
  ns = std::min(ns, std::max(1, n_nodes / APPLY_TS));
  return ns;
}

void asm_apply_off(const ApplyArgs& A, int nsplit, hipStream_t s) {
  if (A.n_nodes <= 0 || A.nrhs <= 0) return;
  const int per = (A.n_nodes + nsplit - 1) / nsplit;
  dim3 grid((A.n_nodes + 255) / 256, nsplit);
  KScope ks(PK_APPLY, s);
  for (int r0 = 0; r0 < A.nrhs;) {
    const int left = A.nrhs - r0;
    if (left == 1) {
      hipLaunchKernelGGL(k_apply_off<1>, grid, dim3(256), 0, s, A, r0, per);
      r0 += 1;
    } else if (left == 2) {
      hipLaunchKernelGGL(k_apply_off<2>, grid, dim3(256), 0, s, A, r0, per);
      r0 += 2;
    } else if (left <= 4) {
      hipLaunchKernelGGL(k_apply_off<4>, grid, dim3(256), 0, s, A, r0, per);
      r0 += 4;
    } else {
      hipLaunchKernelGGL(k_apply_off<8>, grid, dim3(256), 0, s, A, r0, per);
      r0 += 8;
    }
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
