// Batched complex FP64 dense linear algebra kernels for gfx950.
//
//  * zgemm: 64x64 tiles per 256-thread workgroup, each wave a 32x32 sub-tile built
//    from 16x16x4 FP64 MFMA blocks; a complex product is four real MFMAs.
//  * getrf: right-looking blocked LU with partial pivoting (panel of 32 columns in
//    one workgroup per matrix, row swaps, unit-lower triangular solve, MFMA update).
//  * getrs: blocked forward and backward substitution (small triangular solves on
//    32x32 diagonal blocks in LDS, MFMA updates of the rest).
//  * geqrf: blocked Householder QR (16-column panels, compact WY form I - V T V^H,
//    trailing update as two MFMA products); only R is kept.
//  * cpqr: column pivoted Householder QR with norm downdating, one workgroup per
//    matrix, one wave per trailing column, stopping at a relative threshold.
// Reflectors are Hermitian: H = I - tau v v^H with real tau, so |R_jj| equals the
// norm of the trailing part of the pivot column, which is what the threshold tests.
#include "la.h"

typedef double d4 __attribute__((ext_vector_type(4)));

#define PMX_CHECK_LAUNCH() (void)hipGetLastError()

// ---------------------------------------------------------------------------------
// wave / block reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// argmax of (val, idx): larger val wins, ties go to the smaller index
__device__ inline void argmax_pair(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 >= 0 && (i < 0 || i2 < i))) {
    v = v2;
    i = i2;
  }
}

template <int NT>
__device__ inline int block_argmax(double v, int i, double* redv, int* redi, double* outv) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    double v2 = __shfl_xor(v, o, 64);
    int i2 = __shfl_xor(i, o, 64);
    argmax_pair(v, i, v2, i2);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    redv[wave] = v;
    redi[wave] = i;
  }
  __syncthreads();
  double bv = redv[0];
  int bi = redi[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) argmax_pair(bv, bi, redv[w], redi[w]);
  if (outv) *outv = bv;
  return bi;
}

// ---------------------------------------------------------------------------------
// ZGEMM
template <int OPA, int OPB, class F>
__global__ __launch_bounds__(256) void k_zgemm(F f, zd alpha, zd beta) {
  GemmArgs g;
  if (!f(blockIdx.z, g)) return;
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= g.m || tn >= g.n) return;
  __shared__ zd As[8][64 + 1];
  __shared__ zd Bs[8][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accR[a][b] = (d4){0, 0, 0, 0};
      accI[a][b] = (d4){0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < g.k; k0 += 8) {
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      int i, kk;
      if (OPA == OP_N) {
        i = tid & 63;
        kk = (tid >> 6) + 4 * pass;
      } else {
        kk = tid & 7;
        i = (tid >> 3) + 32 * pass;
      }
      const int gi = tm + i, gk = k0 + kk;
      zd v = zmk(0, 0);
      if (gi < g.m && gk < g.k) {
        if (OPA == OP_N) {
          v = g.A[gi + (int64_t)gk * g.lda];
        } else {
          v = g.A[gk + (int64_t)gi * g.lda];
          if (OPA == OP_C) v.im = -v.im;
        }
      }
      As[kk][i] = v;
    }
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      int j, kk;
      if (OPB == OP_N) {
        kk = tid & 7;
        j = (tid >> 3) + 32 * pass;
      } else {
        j = tid & 63;
        kk = (tid >> 6) + 4 * pass;
      }
      const int gj = tn + j, gk = k0 + kk;
      zd v = zmk(0, 0);
      if (gj < g.n && gk < g.k) {
        if (OPB == OP_N) {
          v = g.B[gk + (int64_t)gj * g.ldb];
        } else {
          v = g.B[gj + (int64_t)gk * g.ldb];
          if (OPB == OP_C) v.im = -v.im;
        }
      }
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 8; ks += 4) {
      zd a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[ks + (lane >> 4)][wm + t * 16 + (lane & 15)];
        b[t] = Bs[ks + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          accR[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].re, b[bj].re, accR[bi][bj], 0, 0, 0);
          accR[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[bi].im, b[bj].im, accR[bi][bj], 0, 0, 0);
          accI[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].re, b[bj].im, accI[bi][bj], 0, 0, 0);
          accI[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi].im, b[bj].re, accI[bi][bj], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const bool use_beta = (beta.re != 0.0 || beta.im != 0.0);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm + wm + bi * 16 + (lane >> 4) + 4 * r;  // accumulator r of lane: row lane/16 + 4r
        const int col = tn + wn + bj * 16 + (lane & 15);
        if (row < g.m && col < g.n) {
          zd v = zmul(alpha, zmk(accR[bi][bj][r], accI[bi][bj][r]));
          zd* cp = g.C + row + (int64_t)col * g.ldc;
          if (use_beta) v = zfma(beta, *cp, v);
          *cp = v;
        }
      }
}

template <int OPA, int OPB, class F>
static void launch_zgemm(F f, int batch, int max_m, int max_n, zd alpha, zd beta, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  dim3 grid((max_m + 63) / 64, (max_n + 63) / 64, batch);
  hipLaunchKernelGGL((k_zgemm<OPA, OPB, F>), grid, dim3(256), 0, s, f, alpha, beta);
}

struct FList {
  const GemmArgs* l;
  __device__ bool operator()(int b, GemmArgs& g) const {
    g = l[b];
    return g.m > 0 && g.n > 0;
  }
};

void la_zgemm_list(int opa, int opb, const GemmArgs* d_list, int batch, int max_m, int max_n,
                   zd alpha, zd beta, hipStream_t s) {
  FList f{d_list};
#define PMX_G(A, B)                                                   \
  if (opa == A && opb == B) {                                         \
    launch_zgemm<A, B>(f, batch, max_m, max_n, alpha, beta, s);       \
    return;                                                           \
  }
  PMX_G(OP_N, OP_N) PMX_G(OP_N, OP_T) PMX_G(OP_N, OP_C)
  PMX_G(OP_T, OP_N) PMX_G(OP_T, OP_T) PMX_G(OP_T, OP_C)
  PMX_G(OP_C, OP_N) PMX_G(OP_C, OP_T) PMX_G(OP_C, OP_C)
#undef PMX_G
}

// ---------------------------------------------------------------------------------
// small triangular solve on a <=32 x <=32 diagonal block, one thread per right-hand side
struct TrsmArgs {
  const zd* T;
  int64_t ldt;
  zd* B;
  int64_t ldb;
  int nb, nrhs;
};

template <bool UPPER, bool UNIT, class F>
__global__ __launch_bounds__(64) void k_trsm_small(F f) {
  TrsmArgs a;
  if (!f(blockIdx.y, a)) return;
  __shared__ zd Ts[32][33];
  __shared__ zd xs[32][64];
  const int tid = threadIdx.x;
  const int col = blockIdx.x * 64 + tid;
  if (blockIdx.x * 64 >= a.nrhs) return;
  for (int e = tid; e < a.nb * a.nb; e += 64) {
    int r = e % a.nb, c = e / a.nb;
    Ts[r][c] = a.T[r + (int64_t)c * a.ldt];
  }
  const bool active = col < a.nrhs;
  if (active)
    for (int i = 0; i < a.nb; ++i) xs[i][tid] = a.B[i + (int64_t)col * a.ldb];
  __syncthreads();
  if (active) {
    if (!UPPER) {
      for (int i = 0; i < a.nb; ++i) {
        zd xi = xs[i][tid];
        if (!UNIT) {
          xi = zdiv(xi, Ts[i][i]);
          xs[i][tid] = xi;
        }
        for (int r = i + 1; r < a.nb; ++r) xs[r][tid] = zsub(xs[r][tid], zmul(Ts[r][i], xi));
      }
    } else {
      for (int i = a.nb - 1; i >= 0; --i) {
        zd xi = xs[i][tid];
        if (!UNIT) {
          xi = zdiv(xi, Ts[i][i]);
          xs[i][tid] = xi;
        }
        for (int r = 0; r < i; ++r) xs[r][tid] = zsub(xs[r][tid], zmul(Ts[r][i], xi));
      }
    }
    for (int i = 0; i < a.nb; ++i) a.B[i + (int64_t)col * a.ldb] = xs[i][tid];
  }
}

template <bool UPPER, bool UNIT, class F>
static void launch_trsm_small(F f, int batch, int max_nrhs, hipStream_t s) {
  if (batch <= 0 || max_nrhs <= 0) return;
  dim3 grid((max_nrhs + 63) / 64, batch);
  hipLaunchKernelGGL((k_trsm_small<UPPER, UNIT, F>), grid, dim3(64), 0, s, f);
}

// ---------------------------------------------------------------------------------
// LU
__global__ __launch_bounds__(256) void k_getrf_panel(const LuDesc* lus, int j0, int* info) {
  const LuDesc L = lus[blockIdx.x];
  const int jb = min(PMX_LU_NB, L.n - j0);
  if (jb <= 0) return;
  __shared__ double redv[4];
  __shared__ int redi[4];
  const int tid = threadIdx.x;
  zd* A = L.a;
  const int64_t ld = L.ld;
  for (int c = j0; c < j0 + jb; ++c) {
    double best = -1.0;
    int bi = -1;
    for (int r = c + tid; r < L.n; r += 256) {
      zd v = A[r + c * ld];
      double av = fabs(v.re) + fabs(v.im);
      argmax_pair(best, bi, av, r);
    }
    double bestv;
    const int p = block_argmax<256>(best, bi, redv, redi, &bestv);
    if (tid == 0) {
      L.ipiv[c] = p;
      if (bestv == 0.0 && info && info[blockIdx.x] == 0) info[blockIdx.x] = c + 1;
    }
    if (p != c) {
      for (int cc = j0 + tid; cc < j0 + jb; cc += 256) {
        zd t = A[c + cc * ld];
        A[c + cc * ld] = A[p + cc * ld];
        A[p + cc * ld] = t;
      }
    }
    __syncthreads();
    zd piv = A[c + c * ld];
    if (piv.re != 0.0 || piv.im != 0.0) {
      zd inv = zdiv(zmk(1, 0), piv);
      for (int r = c + 1 + tid; r < L.n; r += 256) {
        zd l = zmul(A[r + c * ld], inv);
        A[r + c * ld] = l;
        for (int cc = c + 1; cc < j0 + jb; ++cc)
          A[r + cc * ld] = zsub(A[r + cc * ld], zmul(l, A[c + cc * ld]));
      }
    }
    __syncthreads();
  }
}

// apply the swaps of panel [j0, j0+jb) to the columns outside the panel
__global__ void k_laswp_panel(const LuDesc* lus, int j0) {
  const LuDesc L = lus[blockIdx.y];
  const int jb = min(PMX_LU_NB, L.n - j0);
  if (jb <= 0) return;
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= L.n - jb) return;
  if (col >= j0) col += jb;
  zd* A = L.a + col * L.ld;
  for (int c = j0; c < j0 + jb; ++c) {
    int p = L.ipiv[c];
    if (p != c) {
      zd t = A[c];
      A[c] = A[p];
      A[p] = t;
    }
  }
}

struct FLuTrsm {
  const LuDesc* d;
  int j0;
  __device__ bool operator()(int b, TrsmArgs& a) const {
    LuDesc L = d[b];
    int jb = min(PMX_LU_NB, L.n - j0);
    if (jb <= 0 || L.n - j0 - jb <= 0) return false;
    a.T = L.a + j0 + j0 * L.ld;
    a.ldt = L.ld;
    a.B = L.a + j0 + (j0 + jb) * L.ld;
    a.ldb = L.ld;
    a.nb = jb;
    a.nrhs = L.n - j0 - jb;
    return true;
  }
};

struct FLuUpd {
  const LuDesc* d;
  int j0;
  __device__ bool operator()(int b, GemmArgs& g) const {
    LuDesc L = d[b];
    int jb = min(PMX_LU_NB, L.n - j0);
    int r = L.n - j0 - jb;
    if (jb <= 0 || r <= 0) return false;
    g.m = r;
    g.n = r;
    g.k = jb;
    g.A = L.a + (j0 + jb) + j0 * L.ld;
    g.lda = L.ld;
    g.B = L.a + j0 + (j0 + jb) * L.ld;
    g.ldb = L.ld;
    g.C = L.a + (j0 + jb) + (j0 + jb) * L.ld;
    g.ldc = L.ld;
    return true;
  }
};

void la_getrf(const LuDesc* d_lu, int batch, int max_n, int* d_info, hipStream_t s) {
  if (batch <= 0 || max_n <= 0) return;
  for (int j0 = 0; j0 < max_n; j0 += PMX_LU_NB) {
    hipLaunchKernelGGL(k_getrf_panel, dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
    hipLaunchKernelGGL(k_laswp_panel, dim3((max_n + 255) / 256, batch), dim3(256), 0, s, d_lu, j0);
    int rem = max_n - j0 - PMX_LU_NB;
    if (rem > 0) {
      launch_trsm_small<false, true>(FLuTrsm{d_lu, j0}, batch, rem, s);
      launch_zgemm<OP_N, OP_N>(FLuUpd{d_lu, j0}, batch, rem, rem, zmk(-1, 0), zmk(1, 0), s);
    }
  }
}

// ---------------------------------------------------------------------------------
// getrs
__global__ void k_laswp_rhs(const LuDesc* lus, const Mat* bs) {
  const LuDesc L = lus[blockIdx.y];
  const Mat B = bs[blockIdx.y];
  int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= B.n) return;
  zd* x = B.p + col * B.ld;
  for (int c = 0; c < L.n; ++c) {
    int p = L.ipiv[c];
    if (p != c) {
      zd t = x[c];
      x[c] = x[p];
      x[p] = t;
    }
  }
}

struct FRsTrsm {
  const LuDesc* d;
  const Mat* b;
  int j0;
  __device__ bool operator()(int i, TrsmArgs& a) const {
    LuDesc L = d[i];
    Mat B = b[i];
    int jb = min(PMX_LU_NB, L.n - j0);
    if (jb <= 0 || B.n <= 0) return false;
    a.T = L.a + j0 + j0 * L.ld;
    a.ldt = L.ld;
    a.B = B.p + j0;
    a.ldb = B.ld;
    a.nb = jb;
    a.nrhs = B.n;
    return true;
  }
};

struct FRsFwd {
  const LuDesc* d;
  const Mat* b;
  int j0;
  __device__ bool operator()(int i, GemmArgs& g) const {
    LuDesc L = d[i];
    Mat B = b[i];
    int jb = min(PMX_LU_NB, L.n - j0);
    int r = L.n - j0 - jb;
    if (jb <= 0 || r <= 0 || B.n <= 0) return false;
    g.m = r;
    g.n = B.n;
    g.k = jb;
    g.A = L.a + (j0 + jb) + j0 * L.ld;
    g.lda = L.ld;
    g.B = B.p + j0;
    g.ldb = B.ld;
    g.C = B.p + j0 + jb;
    g.ldc = B.ld;
    return true;
  }
};

struct FRsBwd {
  const LuDesc* d;
  const Mat* b;
  int j0;
  __device__ bool operator()(int i, GemmArgs& g) const {
    LuDesc L = d[i];
    Mat B = b[i];
    int jb = min(PMX_LU_NB, L.n - j0);
    if (jb <= 0 || j0 <= 0 || B.n <= 0) return false;
    g.m = j0;
    g.n = B.n;
    g.k = jb;
    g.A = L.a + j0 * L.ld;
    g.lda = L.ld;
    g.B = B.p + j0;
    g.ldb = B.ld;
    g.C = B.p;
    g.ldc = B.ld;
    return true;
  }
};

void la_getrs(const LuDesc* d_lu, const Mat* d_b, int batch, int max_n, int max_nrhs, hipStream_t s) {
  if (batch <= 0 || max_n <= 0 || max_nrhs <= 0) return;
  hipLaunchKernelGGL(k_laswp_rhs, dim3((max_nrhs + 63) / 64, batch), dim3(64), 0, s, d_lu, d_b);
  const int nblk = (max_n + PMX_LU_NB - 1) / PMX_LU_NB;
  for (int bk = 0; bk < nblk; ++bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<false, true>(FRsTrsm{d_lu, d_b, j0}, batch, max_nrhs, s);
    int rem = max_n - j0 - PMX_LU_NB;
    if (rem > 0) launch_zgemm<OP_N, OP_N>(FRsFwd{d_lu, d_b, j0}, batch, rem, max_nrhs, zmk(-1, 0), zmk(1, 0), s);
  }
  for (int bk = nblk - 1; bk >= 0; --bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<true, false>(FRsTrsm{d_lu, d_b, j0}, batch, max_nrhs, s);
    if (j0 > 0) launch_zgemm<OP_N, OP_N>(FRsBwd{d_lu, d_b, j0}, batch, j0, max_nrhs, zmk(-1, 0), zmk(1, 0), s);
  }
}

// ---------------------------------------------------------------------------------
// Householder QR (only R is kept)
#define QR_NT 256
__global__ __launch_bounds__(QR_NT) void k_geqrf_panel(const QrDesc* qrs, int j0) {
  const QrDesc Q = qrs[blockIdx.x];
  const int kmax = min(Q.m, Q.c);
  const int jb = min(PMX_QR_NB, kmax - j0);
  if (jb <= 0) return;
  __shared__ double red[QR_NT / 64][2 * PMX_QR_NB];
  __shared__ zd Ts[PMX_QR_NB][PMX_QR_NB];
  __shared__ zd sh_beta_scale[2];
  __shared__ double sh_tau;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  zd* A = Q.a;
  const int64_t ld = Q.ld;
  const int64_t ldv = Q.m;
  for (int i = 0; i < jb; ++i) {
    const int col = j0 + i;
    double p = 0;
    for (int r = col + tid; r < Q.m; r += QR_NT) p += zabs2(A[r + col * ld]);
    p = wave_sum(p);
    __syncthreads();
    if (lane == 0) red[wave][0] = p;
    __syncthreads();
    if (tid == 0) {
      double s2 = 0;
      for (int w = 0; w < QR_NT / 64; ++w) s2 += red[w][0];
      double xn = sqrt(s2);
      zd alpha = A[col + col * ld];
      double aa = sqrt(zabs2(alpha));
      if (xn == 0.0) {
        sh_tau = 0.0;
        sh_beta_scale[0] = zmk(0, 0);
        sh_beta_scale[1] = zmk(0, 0);
      } else {
        zd sg = aa > 0 ? zscale(alpha, 1.0 / aa) : zmk(1, 0);
        zd beta = zscale(sg, -xn);
        sh_tau = 1.0 + aa / xn;
        sh_beta_scale[0] = beta;
        sh_beta_scale[1] = zdiv(zmk(1, 0), zsub(alpha, beta));
      }
    }
    __syncthreads();
    const double tau = sh_tau;
    const zd beta = sh_beta_scale[0], scale = sh_beta_scale[1];
    // reflector into the column and the explicit V buffer (rows j0..m-1)
    for (int r = j0 + tid; r < Q.m; r += QR_NT) {
      zd v;
      if (r < col) {
        v = zmk(0, 0);
      } else if (r == col) {
        v = zmk(1, 0);
      } else {
        v = zmul(A[r + col * ld], scale);
        A[r + col * ld] = v;
      }
      Q.v[(r - j0) + i * ldv] = v;
    }
    __syncthreads();
    if (tid == 0) A[col + col * ld] = beta;
    // dot products: w_cc = v^H A[:, cc] for the remaining panel columns, z_j = V_j^H v
    const int nrem = jb - 1 - i;
    double acc[2 * PMX_QR_NB];
#pragma unroll
    for (int t = 0; t < 2 * PMX_QR_NB; ++t) acc[t] = 0;
    for (int r = col + tid; r < Q.m; r += QR_NT) {
      zd v = Q.v[(r - j0) + i * ldv];
#pragma unroll
      for (int t = 0; t < PMX_QR_NB; ++t) {
        if (t < nrem) {
          zd a = (r == col) ? A[col + (col + 1 + t) * ld] : A[r + (col + 1 + t) * ld];
          zd w = zcmul(v, a);
          acc[2 * t] += w.re;
          acc[2 * t + 1] += w.im;
        } else if (t - nrem < i) {
          int j = t - nrem;
          zd vj = Q.v[(r - j0) + j * ldv];
          zd z = zcmul(vj, v);
          acc[2 * t] += z.re;
          acc[2 * t + 1] += z.im;
        }
      }
    }
    const int nred = nrem + i;
#pragma unroll
    for (int t = 0; t < 2 * PMX_QR_NB; ++t)
      if (t < 2 * nred) acc[t] = wave_sum(acc[t]);
    __syncthreads();
    if (lane == 0)
      for (int t = 0; t < 2 * nred; ++t) red[wave][t] = acc[t];
    __syncthreads();
    if (tid < 2 * nred) {
      double s = 0;
      for (int w = 0; w < QR_NT / 64; ++w) s += red[w][tid];
      red[0][tid] = s;
    }
    __syncthreads();
    // A[:, cc] -= tau v w_cc ; the pivot row of the panel uses the value before beta was
    // written, but row col of column col is excluded from the update (cc > col).
    for (int r = col + tid; r < Q.m; r += QR_NT) {
      zd v = Q.v[(r - j0) + i * ldv];
      for (int t = 0; t < nrem; ++t) {
        zd w = zmk(red[0][2 * t], red[0][2 * t + 1]);
        int cc = col + 1 + t;
        A[r + cc * ld] = zsub(A[r + cc * ld], zscale(zmul(v, w), tau));
      }
    }
    // T column i: T[i,i] = tau, T[0:i, i] = -tau T[0:i,0:i] z
    if (tid == 0) {
      Ts[i][i] = zmk(tau, 0);
      for (int r = 0; r < i; ++r) {
        zd s = zmk(0, 0);
        for (int j = r; j < i; ++j) s = zadd(s, zmul(Ts[r][j], zmk(red[0][2 * (nrem + j)], red[0][2 * (nrem + j) + 1])));
        Ts[r][i] = zscale(s, -tau);
      }
      for (int r = i + 1; r < PMX_QR_NB; ++r) Ts[r][i] = zmk(0, 0);
    }
    __syncthreads();
  }
  // VT = V T^H for the trailing update, stored in the T workspace area after V
  // (Q.t holds m x NB entries): VT[r, j] = sum_{i >= j} V[r, i] conj(T[j, i])
  for (int r = j0 + tid; r < Q.m; r += QR_NT) {
    zd vr[PMX_QR_NB];
#pragma unroll
    for (int i = 0; i < PMX_QR_NB; ++i) vr[i] = (i < jb) ? Q.v[(r - j0) + i * ldv] : zmk(0, 0);
#pragma unroll
    for (int j = 0; j < PMX_QR_NB; ++j) {
      if (j >= jb) break;
      zd s = zmk(0, 0);
#pragma unroll
      for (int i = 0; i < PMX_QR_NB; ++i)
        if (i >= j && i < jb) s = zadd(s, zmul(vr[i], zconj(Ts[j][i])));
      Q.t[(r - j0) + j * ldv] = s;
    }
  }
}

struct FQrW {  // W = V^H A[j0:m, j0+jb:c]
  const QrDesc* d;
  int j0;
  __device__ bool operator()(int b, GemmArgs& g) const {
    QrDesc Q = d[b];
    int jb = min(PMX_QR_NB, min(Q.m, Q.c) - j0);
    int nc = Q.c - j0 - jb;
    if (jb <= 0 || nc <= 0) return false;
    g.m = jb;
    g.n = nc;
    g.k = Q.m - j0;
    g.A = Q.v;
    g.lda = Q.m;
    g.B = Q.a + j0 + (j0 + jb) * Q.ld;
    g.ldb = Q.ld;
    g.C = Q.w;
    g.ldc = PMX_QR_NB;
    return true;
  }
};

struct FQrUpd {  // A[j0:m, j0+jb:c] -= VT W
  const QrDesc* d;
  int j0;
  __device__ bool operator()(int b, GemmArgs& g) const {
    QrDesc Q = d[b];
    int jb = min(PMX_QR_NB, min(Q.m, Q.c) - j0);
    int nc = Q.c - j0 - jb;
    if (jb <= 0 || nc <= 0) return false;
    g.m = Q.m - j0;
    g.n = nc;
    g.k = jb;
    g.A = Q.t;
    g.lda = Q.m;
    g.B = Q.w;
    g.ldb = PMX_QR_NB;
    g.C = Q.a + j0 + (j0 + jb) * Q.ld;
    g.ldc = Q.ld;
    return true;
  }
};

__global__ void k_copy_r(const QrDesc* qrs) {
  const QrDesc Q = qrs[blockIdx.y];
  const int mb = min(Q.m, Q.c);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mb * Q.c) return;
  const int r = (int)(e % mb), c = (int)(e / mb);
  Q.r[e] = (r <= c) ? Q.a[r + c * Q.ld] : zmk(0, 0);
}

void la_geqrf_r(const QrDesc* d_qr, int batch, int max_m, int max_c, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_c <= 0) return;
  const int kmax = min(max_m, max_c);
  for (int j0 = 0; j0 < kmax; j0 += PMX_QR_NB) {
    hipLaunchKernelGGL(k_geqrf_panel, dim3(batch), dim3(QR_NT), 0, s, d_qr, j0);
    int nc = max_c - j0 - PMX_QR_NB;
    if (nc > 0) {
      launch_zgemm<OP_C, OP_N>(FQrW{d_qr, j0}, batch, PMX_QR_NB, nc, zmk(1, 0), zmk(0, 0), s);
      launch_zgemm<OP_N, OP_N>(FQrUpd{d_qr, j0}, batch, max_m - j0, nc, zmk(-1, 0), zmk(1, 0), s);
    }
  }
  int64_t tot = (int64_t)kmax * max_c;
  hipLaunchKernelGGL(k_copy_r, dim3((unsigned)((tot + 255) / 256), batch), dim3(256), 0, s, d_qr);
}

// ---------------------------------------------------------------------------------
// column pivoted QR with threshold rank
#define CP_NT 512
__global__ __launch_bounds__(CP_NT) void k_cpqr(const CpqrDesc* cps, double tol, const int* kmin, int init) {
  const CpqrDesc C = cps[blockIdx.x];
  if (C.c <= 0) return;
  extern __shared__ zd vs[];  // [mb]
  __shared__ double redv[CP_NT / 64];
  __shared__ int redi[CP_NT / 64];
  __shared__ double sh_tau;
  __shared__ int sh_stop;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = CP_NT / 64;
  zd* B = C.b;
  const int mb = C.mb, c = C.c;
  const int64_t ld = mb;
  const int kmax = min(mb, c);
  double* nrm = C.nrm;
  if (init) {
    for (int l = wave; l < c; l += nw) {
      double p = 0;
      for (int r = lane; r < mb; r += 64) p += zabs2(B[r + l * ld]);
      p = wave_sum(p);
      if (lane == 0) {
        nrm[l] = p;
        nrm[c + l] = p;
        C.piv[l] = l;
      }
    }
    if (tid == 0) {
      C.state[0] = 0;
      C.state[1] = -1;
      C.state[2] = 0;
      *C.r11 = 0.0;
    }
    __syncthreads();
    __threadfence_block();
  }
  int j = C.state[0];
  const int target = (tol > 0.0) ? kmax : min(kmax, kmin ? kmin[blockIdx.x] : kmax);
  double r11 = *C.r11;
  while (j < target) {
    double best = -1.0;
    int bi = -1;
    for (int l = j + tid; l < c; l += CP_NT) argmax_pair(best, bi, nrm[l], l);
    const int p = block_argmax<CP_NT>(best, bi, redv, redi, nullptr);
    if (p != j) {
      for (int r = tid; r < mb; r += CP_NT) {
        zd t = B[r + j * ld];
        B[r + j * ld] = B[r + p * ld];
        B[r + p * ld] = t;
      }
    }
    __syncthreads();
    if (tid == 0 && p != j) {
      int ti = C.piv[j];
      C.piv[j] = C.piv[p];
      C.piv[p] = ti;
      double t0 = nrm[j];
      nrm[j] = nrm[p];
      nrm[p] = t0;
      t0 = nrm[c + j];
      nrm[c + j] = nrm[c + p];
      nrm[c + p] = t0;
    }
    double part = 0;
    for (int r = j + tid; r < mb; r += CP_NT) part += zabs2(B[r + j * ld]);
    const double xn = sqrt(block_sum<CP_NT>(part, redv));
    if (tid == 0) {
      if (j == 0) r11 = xn;
      int stop = 0;
      if (xn == 0.0) stop = 1;
      else if (tol > 0.0 && xn <= tol * r11) stop = 1;
      sh_stop = stop;
      zd alpha = B[j + j * ld];
      double aa = sqrt(zabs2(alpha));
      if (!stop) {
        zd sg = aa > 0 ? zscale(alpha, 1.0 / aa) : zmk(1, 0);
        zd beta = zscale(sg, -xn);
        sh_tau = 1.0 + aa / xn;
        vs[0] = zdiv(zmk(1, 0), zsub(alpha, beta));   // scale, replaced by 1 below
        B[j + j * ld] = beta;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const zd scale = vs[0];
    __syncthreads();
    for (int r = j + tid; r < mb; r += CP_NT) {
      zd v = (r == j) ? zmk(1, 0) : zmul(B[r + j * ld], scale);
      vs[r - j] = v;
      if (r > j) B[r + j * ld] = zmk(0, 0);
    }
    __syncthreads();
    const double tau = sh_tau;
    for (int l = j + 1 + wave; l < c; l += nw) {
      zd* col = B + l * ld;
      double wr = 0, wi = 0;
      for (int r = j + lane; r < mb; r += 64) {
        zd t = zcmul(vs[r - j], col[r]);
        wr += t.re;
        wi += t.im;
      }
      wr = wave_sum(wr);
      wi = wave_sum(wi);
      const zd w = zscale(zmk(wr, wi), tau);
      double tail = 0;
      zd first = zmk(0, 0);
      for (int r = j + lane; r < mb; r += 64) {
        zd nv = zsub(col[r], zmul(vs[r - j], w));
        col[r] = nv;
        if (r > j) tail += zabs2(nv);
        else first = nv;
      }
      // norm downdating with recomputation on cancellation; lane 0 holds row j
      zd rjl = zmk(__shfl(first.re, 0, 64), __shfl(first.im, 0, 64));
      double nw2 = nrm[l] - zabs2(rjl);
      if (nw2 <= 1e-8 * nrm[c + l]) {
        tail = wave_sum(tail);
        if (lane == 0) {
          nrm[l] = tail;
          nrm[c + l] = tail;
        }
      } else if (lane == 0) {
        nrm[l] = nw2;
      }
    }
    __syncthreads();
    ++j;
  }
  if (tid == 0) {
    C.state[0] = j;
    if (tol > 0.0) C.state[1] = j;
    *C.r11 = r11;
  }
}

void la_cpqr(const CpqrDesc* d_cp, int batch, int max_c, double tol, const int* d_kmin, int init,
             hipStream_t s) {
  if (batch <= 0 || max_c <= 0) return;
  size_t shm = (size_t)max_c * sizeof(zd) + 16;
  if (shm > 64 * 1024) (void)hipFuncSetAttribute((const void*)k_cpqr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL(k_cpqr, dim3(batch), dim3(CP_NT), shm, s, d_cp, tol, d_kmin, init);
}

// T = R11^-1 R12 in place
struct FTTrsm {
  const CpqrDesc* d;
  const int* ks;
  int j0;
  __device__ bool operator()(int b, TrsmArgs& a) const {
    CpqrDesc C = d[b];
    int k = ks[b];
    int jb = min(PMX_LU_NB, k - j0);
    if (jb <= 0 || C.c - k <= 0) return false;
    a.T = C.b + j0 + (int64_t)j0 * C.mb;
    a.ldt = C.mb;
    a.B = C.b + j0 + (int64_t)k * C.mb;
    a.ldb = C.mb;
    a.nb = jb;
    a.nrhs = C.c - k;
    return true;
  }
};

struct FTUpd {
  const CpqrDesc* d;
  const int* ks;
  int j0;
  __device__ bool operator()(int b, GemmArgs& g) const {
    CpqrDesc C = d[b];
    int k = ks[b];
    int jb = min(PMX_LU_NB, k - j0);
    if (jb <= 0 || j0 <= 0 || C.c - k <= 0) return false;
    g.m = j0;
    g.n = C.c - k;
    g.k = jb;
    g.A = C.b + (int64_t)j0 * C.mb;
    g.lda = C.mb;
    g.B = C.b + j0 + (int64_t)k * C.mb;
    g.ldb = C.mb;
    g.C = C.b + (int64_t)k * C.mb;
    g.ldc = C.mb;
    return true;
  }
};

void la_cpqr_tsolve(const CpqrDesc* d_cp, const int* d_k, int batch, int max_k, int max_c,
                    hipStream_t s) {
  if (batch <= 0 || max_k <= 0 || max_c <= 0) return;
  const int nblk = (max_k + PMX_LU_NB - 1) / PMX_LU_NB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<true, false>(FTTrsm{d_cp, d_k, j0}, batch, max_c, s);
    if (j0 > 0) launch_zgemm<OP_N, OP_N>(FTUpd{d_cp, d_k, j0}, batch, j0, max_c, zmk(-1, 0), zmk(1, 0), s);
  }
}
