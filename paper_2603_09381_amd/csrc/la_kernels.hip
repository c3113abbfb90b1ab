// Batched complex dense linear algebra kernels for gfx950, templated on the real type R
// (double: FP64 MFMA 16x16x4; float: FP32 MFMA 16x16x4).
//
//  * zgemm: 64x64 tiles per 256-thread workgroup, each wave a 32x32 sub-tile built
//    from 16x16x4 MFMA blocks; a complex product is four real MFMAs.
//  * getrf: right-looking blocked LU with partial pivoting (panel of 32 columns in
//    one workgroup per matrix, row swaps, unit-lower triangular solve, MFMA update).
//  * getrs: blocked forward and backward substitution (small triangular solves on
//    32x32 diagonal blocks in LDS, MFMA updates of the rest).
//  * geqrf: Householder QR as a tree of in-LDS block factorisations (TSQR panels of 32
//    columns), trailing update in compact WY form on MFMA; only R is kept.
//  * cpqr: column pivoted Householder QR with norm downdating, stopping at a relative
//    threshold; one workgroup per matrix, or a pivot and an update launch per step for
//    large matrices.  Norms and pivot decisions are FP64 for both real types.
// Reflectors are Hermitian: H = I - tau v v^H with real tau, so |R_jj| equals the
// norm of the trailing part of the pivot column, which is what the threshold tests.
#include "la.h"
#include "ktimer.h"
#include "tune.h"

#include <hip/hip_cooperative_groups.h>

#include <algorithm>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class R>
struct AccT;
template <>
struct AccT<double> {
  typedef d4 type;
};
template <>
struct AccT<float> {
  typedef f4 type;
};

// D += A B on a 16x16x4 block.  Operand lanes: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k.  The accumulator layouts differ: FP64 keeps element (i, j) in register i / 4 of
// lane j + 16 (i % 4), FP32 in register i % 4 of lane j + 16 (i / 4).
__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class R>
__device__ inline int mfma_row(int lane, int r);
template <>
__device__ inline int mfma_row<double>(int lane, int r) {
  return (lane >> 4) + 4 * r;
}
template <>
__device__ inline int mfma_row<float>(int lane, int r) {
  return 4 * (lane >> 4) + r;
}

// ---------------------------------------------------------------------------------
// wave / block reductions
// DPP moves of a 32-bit value; lanes outside row_mask receive 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ inline int dpp_move_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK = 0xf>
__device__ inline double dpp_move(double v) {
  const int lo = dpp_move_i<CTRL, ROWMASK>(__double2loint(v));
  const int hi = dpp_move_i<CTRL, ROWMASK>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK = 0xf>
__device__ inline float dpp_move(float v) {
  return __int_as_float(dpp_move_i<CTRL, ROWMASK>(__float_as_int(v)));
}

// Sum over the 64 lanes of a wave, returned to every lane: quad permutations, half-row and
// row mirrors give each row of 16 its sum, row broadcasts 15 and 31 carry the row sums up
// to lane 63, which is read back as a scalar.
template <class T>
__device__ inline T wave_sum_dpp(T v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);        // row_half_mirror
  v += dpp_move<0x140>(v);        // row_mirror
  v += dpp_move<0x142, 0xA>(v);   // row_bcast15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);   // row_bcast31 into rows 2 and 3
  return v;
}
__device__ inline double wave_sum(double v) {
  v = wave_sum_dpp(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
__device__ inline float wave_sum(float v) {
  v = wave_sum_dpp(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
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

// argmax of (val, idx): larger val wins, ties go to the smaller index (evaluated without
// branches).  A NaN candidate counts as +infinity, so that a search over any real or NaN
// values ends with a valid index (the pivot checks then report such a pivot as unusable).
__device__ inline void argmax_pair(double& v, int& i, double v2, int i2) {
  v2 = (v2 == v2) ? v2 : __builtin_huge_val();
  const bool take = (v2 > v) | ((v2 == v) & (i2 >= 0) & ((i < 0) | (i2 < i)));
  v = take ? v2 : v;
  i = take ? i2 : i;
}

// Argmax of (value, index) over the 64 lanes of a wave with DPP moves (larger value wins,
// ties go to the smaller index, a total order, so the result does not depend on the
// combination order); lanes a move does not reach keep their own pair.  Returned to
// every lane through lane 63.
template <int CTRL, int ROWMASK = 0xf>
__device__ inline void dpp_argmax_step(double& v, int& i) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
  const int i2 = __builtin_amdgcn_update_dpp(i, i, CTRL, ROWMASK, 0xf, false);
  argmax_pair(v, i, __hiloint2double(hi2, lo2), i2);
}

__device__ inline void wave_argmax(double& v, int& i) {
  dpp_argmax_step<0xB1>(v, i);        // quad_perm [1,0,3,2]
  dpp_argmax_step<0x4E>(v, i);        // quad_perm [2,3,0,1]
  dpp_argmax_step<0x141>(v, i);       // row_half_mirror
  dpp_argmax_step<0x140>(v, i);       // row_mirror
  dpp_argmax_step<0x142, 0xA>(v, i);  // row_bcast15 into rows 1 and 3
  dpp_argmax_step<0x143, 0xC>(v, i);  // row_bcast31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  v = __hiloint2double(hi, lo);
  i = __builtin_amdgcn_readlane(i, 63);
}

// value of lane l (uniform l) of every lane's v, as a scalar
__device__ inline double readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ inline float readlane(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
template <class R>
__device__ inline cx<R> readlane(cx<R> v, int l) {
  return cmk<R>(readlane(v.re, l), readlane(v.im, l));
}

template <int NT>
__device__ inline int block_argmax(double v, int i, double* redv, int* redi, double* outv) {
  wave_argmax(v, i);
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
// C = alpha op(A) op(B) + beta C on 64 x 64 tiles, four waves of 32 x 32 (2 x 2 blocks of
// 16 x 16 MFMA).  The k loop moves 16 at a time through LDS; the next slice's global loads
// are issued into registers before the current slice is multiplied, so they are in flight
// during the MFMAs.  In FP64 complex products as three real ones (Gauss): p1 = sum ar br,
// p2 = sum ai bi, p3 = sum (ar + ai)(br + bi), C = (p1 - p2) + i (p3 - p1 - p2); in FP32
// as four.
#define ZG_KS 16
template <class R, int OPA, int OPB, class F>
__global__ __launch_bounds__(256, 2) void k_zgemm(F f, cx<R> alpha, cx<R> beta) {
  typedef cx<R> C;
  typedef typename AccT<R>::type V4;
  GemmArgsT<R> g;
  if (!f(blockIdx.z, g)) return;
  const auto gA = gbl(g.A);
  const auto gB = gbl(g.B);
  const auto gC = gbl(g.C);
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= g.m || tn >= g.n) return;
  __shared__ C As[ZG_KS][64 + 1];
  __shared__ C Bs[ZG_KS][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  // three real products per complex one in FP64 only: in the FP32 factor the larger
  // rounding of the Gauss form's imaginary part (p3 - p1 - p2 cancels) weakened the
  // refinement's contraction enough to cost a whole extra step at 1M unknowns
  constexpr bool ZG_GAUSS = sizeof(R) == 8;
  V4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      p1[a][b] = V4{0, 0, 0, 0};
      p2[a][b] = V4{0, 0, 0, 0};
      p3[a][b] = V4{0, 0, 0, 0};
    }
  // slice loads: 64 x 16 of A and 16 x 64 of B, four entries each per thread
  constexpr int NP = 64 * ZG_KS / 256;
  C ra[NP], rb[NP];
  auto a_pos = [&](int pass, int& i, int& kk) {
    if (OPA == OP_N) {
      i = tid & 63;
      kk = (tid >> 6) + 4 * pass;
    } else {
      kk = tid & (ZG_KS - 1);
      i = (tid / ZG_KS) + (256 / ZG_KS) * pass;
    }
  };
  auto b_pos = [&](int pass, int& j, int& kk) {
    if (OPB == OP_N) {
      kk = tid & (ZG_KS - 1);
      j = (tid / ZG_KS) + (256 / ZG_KS) * pass;
    } else {
      j = tid & 63;
      kk = (tid >> 6) + 4 * pass;
    }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      int i, kk;
      a_pos(pass, i, kk);
      const int gi = tm + i, gk = k0 + kk;
      const int ci = min(gi, g.m - 1), ck = min(gk, g.k - 1);
      C v = (OPA == OP_N) ? gA[ci + (int64_t)ck * g.lda] : gA[ck + (int64_t)ci * g.lda];
      if (OPA == OP_C) v.im = -v.im;
      ra[pass] = (gi < g.m && gk < g.k) ? v : cmk<R>(0, 0);
    }
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      int j, kk;
      b_pos(pass, j, kk);
      const int gj = tn + j, gk = k0 + kk;
      const int cj = min(gj, g.n - 1), ck = min(gk, g.k - 1);
      C v = (OPB == OP_N) ? gB[ck + (int64_t)cj * g.ldb] : gB[cj + (int64_t)ck * g.ldb];
      if (OPB == OP_C) v.im = -v.im;
      rb[pass] = (gj < g.n && gk < g.k) ? v : cmk<R>(0, 0);
    }
  };
  load(0);
  for (int k0 = 0; k0 < g.k; k0 += ZG_KS) {
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      int i, kk;
      a_pos(pass, i, kk);
      As[kk][i] = ra[pass];
      int j, kb;
      b_pos(pass, j, kb);
      Bs[kb][j] = rb[pass];
    }
    __syncthreads();
    if (k0 + ZG_KS < g.k) load(k0 + ZG_KS);
#pragma unroll
    for (int ks = 0; ks < ZG_KS; ks += 4) {
      C a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[ks + (lane >> 4)][wm + t * 16 + (lane & 15)];
        b[t] = Bs[ks + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
      if constexpr (ZG_GAUSS) {
        R as[2], bs[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          as[t] = a[t].re + a[t].im;
          bs[t] = b[t].re + b[t].im;
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            p1[bi][bj] = mfma16(a[bi].re, b[bj].re, p1[bi][bj]);
            p2[bi][bj] = mfma16(a[bi].im, b[bj].im, p2[bi][bj]);
            p3[bi][bj] = mfma16(as[bi], bs[bj], p3[bi][bj]);
          }
      } else {
        // real part in p1, imaginary part in p2
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            p1[bi][bj] = mfma16(a[bi].re, b[bj].re, p1[bi][bj]);
            p1[bi][bj] = mfma16(-a[bi].im, b[bj].im, p1[bi][bj]);
            p2[bi][bj] = mfma16(a[bi].re, b[bj].im, p2[bi][bj]);
            p2[bi][bj] = mfma16(a[bi].im, b[bj].re, p2[bi][bj]);
          }
      }
    }
    __syncthreads();
  }
  const bool use_beta = (beta.re != R(0) || beta.im != R(0));
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm + wm + bi * 16 + mfma_row<R>(lane, r);
        const int col = tn + wn + bj * 16 + (lane & 15);
        if (row < g.m && col < g.n) {
          const R x1 = p1[bi][bj][r], x2 = p2[bi][bj][r], x3 = p3[bi][bj][r];
          C v = zmul(alpha, ZG_GAUSS ? cmk<R>(x1 - x2, x3 - x1 - x2) : cmk<R>(x1, x2));
          auto cp = gC + row + (int64_t)col * g.ldc;
          if (use_beta) v = zfma(beta, *cp, v);
          *cp = v;
        }
      }
}

// C = alpha A B + beta C (both untransposed) for n <= 16: 64 x 16 tiles, wave w the 16 x 16
// MFMA block of rows 16 w.  Same k slices, prefetch and complex product forms as k_zgemm,
// so every entry is the same sum in the same order; k_zgemm's 64-column tiles would spend
// three quarters of their MFMA work on absent columns.
template <class R, class F>
__global__ __launch_bounds__(256) void k_zgemm_n16(F f, cx<R> alpha, cx<R> beta) {
  typedef cx<R> C;
  typedef typename AccT<R>::type V4;
  GemmArgsT<R> g;
  if (!f(blockIdx.z, g)) return;
  const auto gA = gbl(g.A);
  const auto gB = gbl(g.B);
  const auto gC = gbl(g.C);
  const int tm = blockIdx.x * 64;
  if (tm >= g.m) return;
  __shared__ C As[ZG_KS][64 + 1];
  __shared__ C Bs[ZG_KS][16 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave * 16;
  constexpr bool ZG_GAUSS = sizeof(R) == 8;
  V4 p1 = V4{0, 0, 0, 0}, p2 = V4{0, 0, 0, 0}, p3 = V4{0, 0, 0, 0};
  // slice loads: 64 x 16 of A (four entries per thread), 16 x 16 of B (one)
  constexpr int NP = 64 * ZG_KS / 256;
  C ra[NP], rb = cmk<R>(0, 0);
#pragma unroll
  for (int pass = 0; pass < NP; ++pass) ra[pass] = cmk<R>(0, 0);
  const int bk = tid & (ZG_KS - 1), bj = tid / ZG_KS;
  auto load = [&](int k0) {
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int i = tid & 63, kk = (tid >> 6) + 4 * pass;
      const int gi = tm + i, gk = k0 + kk;
      const C v = gA[min(gi, g.m - 1) + (int64_t)min(gk, g.k - 1) * g.lda];
      ra[pass] = (gi < g.m && gk < g.k) ? v : cmk<R>(0, 0);
    }
    const int gk = k0 + bk;
    const C v = gB[min(gk, g.k - 1) + (int64_t)min(bj, g.n - 1) * g.ldb];
    rb = (bj < g.n && gk < g.k) ? v : cmk<R>(0, 0);
  };
  if (g.k > 0) load(0);   // k = 0: no loads, C = beta C
  for (int k0 = 0; k0 < g.k; k0 += ZG_KS) {
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) As[(tid >> 6) + 4 * pass][tid & 63] = ra[pass];
    Bs[bk][bj] = rb;
    __syncthreads();
    if (k0 + ZG_KS < g.k) load(k0 + ZG_KS);
#pragma unroll
    for (int ks = 0; ks < ZG_KS; ks += 4) {
      const C a = As[ks + (lane >> 4)][wm + (lane & 15)];
      const C b = Bs[ks + (lane >> 4)][lane & 15];
      if constexpr (ZG_GAUSS) {
        p1 = mfma16(a.re, b.re, p1);
        p2 = mfma16(a.im, b.im, p2);
        p3 = mfma16(a.re + a.im, b.re + b.im, p3);
      } else {
        p1 = mfma16(a.re, b.re, p1);
        p1 = mfma16(-a.im, b.im, p1);
        p2 = mfma16(a.re, b.im, p2);
        p2 = mfma16(a.im, b.re, p2);
      }
    }
    __syncthreads();
  }
  const bool use_beta = (beta.re != R(0) || beta.im != R(0));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = tm + wm + mfma_row<R>(lane, r);
    const int col = lane & 15;
    if (row < g.m && col < g.n) {
      const R x1 = p1[r], x2 = p2[r], x3 = p3[r];
      C v = zmul(alpha, ZG_GAUSS ? cmk<R>(x1 - x2, x3 - x1 - x2) : cmk<R>(x1, x2));
      auto cp = gC + row + (int64_t)col * g.ldc;
      if (use_beta) v = zfma(beta, *cp, v);
      *cp = v;
    }
  }
}

template <class R, int OPA, int OPB, class F>
static void launch_zgemm(F f, int batch, int max_m, int max_n, cx<R> alpha, cx<R> beta, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  KScope ks(PK_ZGEMM, s);
  if constexpr (OPA == OP_N && OPB == OP_N) {
    if (max_n <= 16) {   // same sums in the same order on 64 x 16 tiles
      PMX_LAUNCH((k_zgemm_n16<R, F>), dim3((max_m + 63) / 64, 1, batch), dim3(256), 0, s, f, alpha, beta);
      return;
    }
  }
  dim3 grid((max_m + 63) / 64, (max_n + 63) / 64, batch);
  PMX_LAUNCH((k_zgemm<R, OPA, OPB, F>), grid, dim3(256), 0, s, f, alpha, beta);
}

// C = alpha A B + beta C for few columns of B (n <= NB, both operands untransposed): the
// product is bound by reading A, which MFMA tiles of 64 columns would mostly waste.  A
// workgroup of NW waves takes 64 rows of one matrix; wave w accumulates the k range
// [w kc, (w + 1) kc) with one row per lane (the column-major A is read 64 consecutive
// rows at a time, coalesced, eight loads in flight) and the row of B of each k read at a
// wave-uniform address; the NW partial sums are added through LDS.
template <class R, int NB, int NW, class F>
__global__ __launch_bounds__(NW * 64) void k_zgemm_skinny(F f, cx<R> alpha, cx<R> beta) {
  typedef cx<R> C;
  GemmArgsT<R> g;
  if (!f(blockIdx.z, g)) return;
  const auto gB = gbl(g.B);
  const int tm = blockIdx.x * 64;
  if (tm >= g.m) return;
  __shared__ C red[NW - 1][NB][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = min(tm + lane, g.m - 1);
  const int kc = (g.k + NW - 1) / NW;
  const int k0 = min(wave * kc, g.k), k1 = min(k0 + kc, g.k);
  const int n = min(g.n, NB);
  R ar[NB], ai[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) ar[j] = ai[j] = R(0);
  const auto Ap = gbl(g.A) + row;
#pragma unroll 8
  for (int kk = k0; kk < k1; ++kk) {
    const C a = Ap[(int64_t)kk * g.lda];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < n) {
        const C b = gB[kk + (int64_t)j * g.ldb];
        ar[j] = fma(a.re, b.re, ar[j]);
        ar[j] = fma(-a.im, b.im, ar[j]);
        ai[j] = fma(a.re, b.im, ai[j]);
        ai[j] = fma(a.im, b.re, ai[j]);
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j) red[wave - 1][j][lane] = cmk<R>(ar[j], ai[j]);
  }
  __syncthreads();
  if (wave > 0 || tm + lane >= g.m) return;
  const bool use_beta = (beta.re != R(0) || beta.im != R(0));
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < n) {
      C v = cmk<R>(ar[j], ai[j]);
#pragma unroll
      for (int w = 0; w < NW - 1; ++w) v = zadd(v, red[w][j][lane]);
      v = zmul(alpha, v);
      auto cp = gbl(g.C) + (tm + lane) + (int64_t)j * g.ldc;
      if (use_beta) v = zfma(beta, *cp, v);
      *cp = v;
    }
  }
}

template <class R, class F>
static bool launch_zgemm_skinny(F f, int batch, int max_m, int max_n, cx<R> alpha, cx<R> beta, hipStream_t s) {
  if (max_n > 8) return false;
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return true;
  dim3 grid((max_m + 63) / 64, 1, batch);
  KScope ks(PK_ZGEMM, s);
  if (max_n <= 4)
    PMX_LAUNCH((k_zgemm_skinny<R, 4, 8, F>), grid, dim3(512), 0, s, f, alpha, beta);
  else
    PMX_LAUNCH((k_zgemm_skinny<R, 8, 8, F>), grid, dim3(512), 0, s, f, alpha, beta);
  return true;
}

template <class R>
struct FList {
  const GemmArgsT<R>* l;
  __device__ bool operator()(int b, GemmArgsT<R>& g) const {
    g = l[b];
    return g.m > 0 && g.n > 0;
  }
};

template <class R>
void la_zgemm_list(int opa, int opb, const GemmArgsT<R>* d_list, int batch, int max_m, int max_n, cx<R> alpha,
                   cx<R> beta, hipStream_t s) {
  FList<R> f{d_list};
  if (opa == OP_N && opb == OP_N && launch_zgemm_skinny<R>(f, batch, max_m, max_n, alpha, beta, s)) return;
#define PMX_G(A, B)                                                \
  if (opa == A && opb == B) {                                      \
    launch_zgemm<R, A, B>(f, batch, max_m, max_n, alpha, beta, s); \
    return;                                                        \
  }
  PMX_G(OP_N, OP_N) PMX_G(OP_N, OP_T) PMX_G(OP_N, OP_C)
  PMX_G(OP_T, OP_N) PMX_G(OP_T, OP_T) PMX_G(OP_T, OP_C)
  PMX_G(OP_C, OP_N) PMX_G(OP_C, OP_T) PMX_G(OP_C, OP_C)
#undef PMX_G
}

template <class R>
struct FApplyList : FList<R> {};

void la_zgemm_apply_list(const GemmArgsT<double>* d_list, int batch, int max_m, int max_n, hipStream_t s) {
  FApplyList<double> f{{d_list}};
  const zd one = zmk(1.0, 0.0), zero = zmk(0.0, 0.0);
  if (launch_zgemm_skinny<double>(f, batch, max_m, max_n, one, zero, s)) return;
  launch_zgemm<double, OP_N, OP_N>(f, batch, max_m, max_n, one, zero, s);
}

// ---------------------------------------------------------------------------------
// small triangular solve on a <=32 x <=32 diagonal block, one thread per right-hand side
template <class R>
struct TrsmArgs {
  const cx<R>* T;
  int64_t ldt;
  cx<R>* B;
  int64_t ldb;
  int nb, nrhs;
};

// X = T^-1 B for a triangle T (nb <= 32, lower or upper, unit or not) and the columns of
// B: one thread per column, held in registers with the loops over the triangle unrolled
// (compile-time register indices).  The triangle goes to LDS padded to 32 x 32 with the
// identity, so the unrolled substitution runs the same 32 steps for every nb with no
// branch; column i of T is stored as a row of LDS and read at wave-uniform addresses.  The
// 64 columns of B pass through LDS so that global loads and stores run down columns
// (32 consecutive rows per half wave) rather than one column per lane.
template <class R, bool UPPER, bool UNIT, class F>
__global__ __launch_bounds__(64) void k_trsm_small(F f) {
  typedef cx<R> C;
  TrsmArgs<R> a;
  if (!f(blockIdx.y, a)) return;
  if (blockIdx.x * 64 >= a.nrhs) return;
  const auto gT = gbl(a.T);
  const auto gB = gbl(a.B);
  __shared__ C Tt[32][32];        // Tt[c][r] = T[r][c]; identity outside nb x nb
  __shared__ C dinv[32];
  __shared__ C Bs[64][33];        // Bs[column][row]
  const int tid = threadIdx.x;
  const int nb = a.nb;
  const int rr = tid & 31, ch = tid >> 5;
  const int rc = min(rr, nb - 1);
  const int cbase = blockIdx.x * 64;
  const int nrhs = a.nrhs;
  {
    C tv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = min(ch + 2 * q, nb - 1);
      tv[q] = gT[rc + (int64_t)c * a.ldt];
    }
    C bv[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int c = min(cbase + ch + 2 * q, nrhs - 1);
      bv[q] = gB[rc + (int64_t)c * a.ldb];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = ch + 2 * q;
      const bool in = rr < nb && c < nb;
      const bool keep = UPPER ? (rr < c) : (rr > c);
      Tt[c][rr] = (in && keep) ? tv[q] : cmk<R>(0, 0);
      if (!UNIT && rr == c) dinv[c] = in ? zrecip(tv[q]) : cmk<R>(1, 0);
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) Bs[ch + 2 * q][rr] = (rr < nb) ? bv[q] : cmk<R>(0, 0);
  }
  __syncthreads();
  C x[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) x[i] = Bs[tid][i];
  if (!UPPER) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      if (!UNIT) x[i] = zmul(x[i], dinv[i]);
#pragma unroll
      for (int r = i + 1; r < 32; ++r) x[r] = zfms(x[r], Tt[i][r], x[i]);
    }
  } else {
#pragma unroll
    for (int i = 31; i >= 0; --i) {
      if (!UNIT) x[i] = zmul(x[i], dinv[i]);
#pragma unroll
      for (int r = 0; r < i; ++r) x[r] = zfms(x[r], Tt[i][r], x[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) Bs[tid][i] = x[i];
  __syncthreads();
  if (rr < nb) {
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int c = cbase + ch + 2 * q;
      if (c < nrhs) gB[rr + (int64_t)c * a.ldb] = Bs[ch + 2 * q][rr];
    }
  }
}

template <class R, bool UPPER, bool UNIT, class F>
static void launch_trsm_small(F f, int batch, int max_nrhs, hipStream_t s) {
  if (batch <= 0 || max_nrhs <= 0) return;
  dim3 grid((max_nrhs + 63) / 64, batch);
  KScope ks(PK_TRSM, s);
  PMX_LAUNCH((k_trsm_small<R, UPPER, UNIT, F>), grid, dim3(64), 0, s, f);
}

// ---------------------------------------------------------------------------------
// LU
template <class R>
__global__ __launch_bounds__(256) void k_getrf_panel(const LuDescT<R>* lus, int j0, int* info) {
  typedef cx<R> C;
  const LuDescT<R> L = lus[blockIdx.x];
  const int jb = min(PMX_LU_NB, L.n - j0);
  if (jb <= 0) return;
  __shared__ double redv[4];
  __shared__ int redi[4];
  const int tid = threadIdx.x;
  const auto A = gbl(L.a);
  const int64_t ld = L.ld;
  for (int c = j0; c < j0 + jb; ++c) {
    double best = -1.0;
    int bi = -1;
    for (int r = c + tid; r < L.n; r += 256) {
      C v = A[r + c * ld];
      double av = fabs((double)v.re) + fabs((double)v.im);
      argmax_pair(best, bi, av, r);
    }
    double bestv;
    const int p = block_argmax<256>(best, bi, redv, redi, &bestv);
    if (tid == 0) {
      gbl(L.ipiv)[c] = p;
      if ((bestv == 0.0 || bestv == __builtin_huge_val()) && info && info[blockIdx.x] == 0) info[blockIdx.x] = c + 1;
    }
    if (p != c) {
      for (int cc = j0 + tid; cc < j0 + jb; cc += 256) {
        C t = A[c + cc * ld];
        A[c + cc * ld] = A[p + cc * ld];
        A[p + cc * ld] = t;
      }
    }
    __syncthreads();
    C piv = A[c + c * ld];
    if (piv.re != R(0) || piv.im != R(0)) {
      C inv = zdiv(cmk<R>(1, 0), piv);
      for (int r = c + 1 + tid; r < L.n; r += 256) {
        C l = zmul(A[r + c * ld], inv);
        A[r + c * ld] = l;
        for (int cc = c + 1; cc < j0 + jb; ++cc)
          A[r + cc * ld] = zfms(A[r + cc * ld], l, A[c + cc * ld]);
      }
    }
    __syncthreads();
  }
}

// The same panel step with the panel held in registers: thread t owns rows j0 + t + NT q
// (q < RPT) of the panel's columns, so a column step costs a block argmax, one exchange
// of two rows through LDS and register updates, instead of global read-modify-writes.
// Pivots, tie-breaks and the order of the updates are those of k_getrf_panel.
template <class R, int NT, int RPT>
__global__ __launch_bounds__(NT) void k_getrf_panel_reg(const LuDescT<R>* lus, int j0, int* info) {
  typedef cx<R> C;
  const LuDescT<R> L = lus[blockIdx.x];
  const int jb = min(PMX_LU_NB, L.n - j0);
  if (jb <= 0) return;
  __shared__ double redv[NT / 64];
  __shared__ int redi[NT / 64];
  __shared__ C prow[PMX_LU_NB], crow[PMX_LU_NB];
  const int tid = threadIdx.x;
  const auto A = gbl(L.a);
  const int64_t ld = L.ld;
  C P[RPT][PMX_LU_NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + NT * q;
    const int ci = min(i, L.n - 1);
#pragma unroll
    for (int c = 0; c < PMX_LU_NB; ++c) P[q][c] = A[ci + (int64_t)(j0 + min(c, jb - 1)) * ld];
  }
#pragma unroll 1
  for (int c = 0; c < jb; ++c) {
    const int col = j0 + c;
    double best = -1.0;
    int bi = -1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = j0 + tid + NT * q;
      C v = P[q][0];
#pragma unroll
      for (int cc = 1; cc < PMX_LU_NB; ++cc)
        if (cc == c) v = P[q][cc];
      if (i >= col && i < L.n) argmax_pair(best, bi, fabs((double)v.re) + fabs((double)v.im), i);
    }
    double bestv;
    const int p = block_argmax<NT>(best, bi, redv, redi, &bestv);
    if (tid == 0) {
      gbl(L.ipiv)[col] = p;
      if ((bestv == 0.0 || bestv == __builtin_huge_val()) && info && info[blockIdx.x] == 0) info[blockIdx.x] = col + 1;
    }
    // exchange rows col and p through LDS
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = j0 + tid + NT * q;
      if (i == p) {
#pragma unroll
        for (int cc = 0; cc < PMX_LU_NB; ++cc) prow[cc] = P[q][cc];
      }
      if (i == col) {
#pragma unroll
        for (int cc = 0; cc < PMX_LU_NB; ++cc) crow[cc] = P[q][cc];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = j0 + tid + NT * q;
      if (i == p && p != col) {
#pragma unroll
        for (int cc = 0; cc < PMX_LU_NB; ++cc) P[q][cc] = crow[cc];
      }
      if (i == col) {
#pragma unroll
        for (int cc = 0; cc < PMX_LU_NB; ++cc) P[q][cc] = prow[cc];
      }
    }
    const C piv = prow[c];
    if (piv.re != R(0) || piv.im != R(0)) {
      const C inv = zdiv(cmk<R>(1, 0), piv);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int i = j0 + tid + NT * q;
        if (i > col && i < L.n) {
          C l = P[q][0];
#pragma unroll
          for (int cc = 1; cc < PMX_LU_NB; ++cc)
            if (cc == c) l = P[q][cc];
          l = zmul(l, inv);
#pragma unroll
          for (int cc = 0; cc < PMX_LU_NB; ++cc) {
            if (cc == c) P[q][cc] = l;
            else if (cc > c) P[q][cc] = zfms(P[q][cc], l, prow[cc]);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + NT * q;
    if (i < L.n) {
#pragma unroll
      for (int cc = 0; cc < PMX_LU_NB; ++cc)
        if (cc < jb) A[i + (int64_t)(j0 + cc) * ld] = P[q][cc];
    }
  }
}

// The panel step with the rows held in registers and the column loop unrolled, so that
// every column index is a compile-time register index, and row exchanges made virtual:
// each thread keeps its rows in place and tracks the row position pos they hold in the
// exchanged order (the exchange of rows col and p swaps two positions, no data moves).
// Per column: local candidates among positions >= col, a DPP wave argmax (ties to the
// smaller position, as k_getrf_panel), wave maxima through LDS and a barrier; the pivot's
// owner writes the pivot row's columns c.. to LDS, a barrier; every row at a position
// below col is eliminated with it.  Each LDS buffer is rewritten only after the next
// barrier, which every thread reaches after its reads.  At the end every row is written
// at its position, which leaves the panel as after the explicit exchanges.
template <class R, int NT, int RPT>
__global__ __launch_bounds__(NT) void k_getrf_panel_u(const LuDescT<R>* lus, int j0, int* info) {
  typedef cx<R> C;
  constexpr int NB = PMX_LU_NB, NW = NT / 64;
  const LuDescT<R> L = lus[blockIdx.x];
  const int jb = min(NB, L.n - j0);
  if (jb <= 0) return;
  __shared__ double sv[NW];
  __shared__ int si[NW];
  __shared__ C prow[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const auto A = gbl(L.a);
  const int64_t ld = L.ld;
  C P[RPT][NB];
  int pos[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = j0 + tid + NT * q;
    pos[q] = i < L.n ? i : -1;   // -1: no row
    const int ci = min(i, L.n - 1);
#pragma unroll
    for (int c = 0; c < NB; ++c) P[q][c] = A[ci + (int64_t)(j0 + min(c, jb - 1)) * ld];
  }
#pragma clang loop unroll(full)
  for (int c = 0; c < NB; ++c) {
    if (c >= jb) continue;   // uniform: the panel's last columns (no barrier is skipped by part of the block)
    const int col = j0 + c;
    double best = -1.0;
    int bi = -1;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (pos[q] >= col) argmax_pair(best, bi, fabs((double)P[q][c].re) + fabs((double)P[q][c].im), pos[q]);
    wave_argmax(best, bi);
    if (lane == 0) {
      sv[wave] = best;
      si[wave] = bi;
    }
    __syncthreads();
    double bv = sv[0];
    int p = si[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) argmax_pair(bv, p, sv[w], si[w]);
    if (tid == 0) {
      gbl(L.ipiv)[col] = p;
      if ((bv == 0.0 || bv == __builtin_huge_val()) && info && info[blockIdx.x] == 0) info[blockIdx.x] = col + 1;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (pos[q] == p) {
#pragma unroll
        for (int cc = c; cc < NB; ++cc) prow[cc] = P[q][cc];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {   // exchange of positions col and p
      const int pq = pos[q];
      pos[q] = (pq == p) ? col : (pq == col ? p : pq);
    }
    const C piv = prow[c];
    if (piv.re != R(0) || piv.im != R(0)) {
      const C inv = zrecip(piv);
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (pos[q] > col) {
          const C l = zmul(P[q][c], inv);
          P[q][c] = l;
#pragma unroll
          for (int cc = c + 1; cc < NB; ++cc) P[q][cc] = zfms(P[q][cc], l, prow[cc]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    if (pos[q] >= 0) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc)
        if (cc < jb) A[pos[q] + (int64_t)(j0 + cc) * ld] = P[q][cc];
    }
  }
}

// Panels taller than the register kernels hold (a few thousand rows by PMX_LU_NB columns,
// cache-resident): the rows stay in memory, thread t taking rows j0 + t + NT q.  Per
// column: a block argmax of the candidates found in the previous column's pass; the
// explicit exchange of the pivot row with row col by the panel's jb threads, which also
// stage in LDS the pivot and the pivot row's entries right of it (zeros elsewhere, so the
// elimination needs no per-column mask); one pass over the rows below col that issues all
// loads of a row's remaining columns at once, eliminates, stores, and takes the next
// column's candidate.  Matrices of a batch may be smaller than the one that chose this
// kernel, so a panel may be narrower than PMX_LU_NB (jb columns).  Pivots, ties (to the
// smaller row) and the update order are those of k_getrf_panel.
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_getrf_panel_t(const LuDescT<R>* lus, int j0, int* info) {
  typedef cx<R> C;
  constexpr int NB = PMX_LU_NB, NW = NT / 64;
  const LuDescT<R> L = lus[blockIdx.x];
  const int jb = min(NB, L.n - j0);
  if (jb <= 0) return;
  __shared__ double sv[NW];
  __shared__ int si[NW];
  __shared__ C prow[NB];
  __shared__ C spiv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = L.n;
  const int ld = (int)L.ld;
  const auto P = gbl(L.a) + (int64_t)j0 * L.ld;   // the panel's first column
  double best = -1.0;
  int bi = -1;
  for (int r = j0 + tid; r < n; r += NT) {
    const C v = P[r];
    argmax_pair(best, bi, fabs((double)v.re) + fabs((double)v.im), r);
  }
#pragma unroll 1
  for (int c = 0; c < jb; ++c) {
    const int col = j0 + c;
    wave_argmax(best, bi);
    if (lane == 0) {
      sv[wave] = best;
      si[wave] = bi;
    }
    __syncthreads();
    double bv = sv[0];
    int p = si[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) argmax_pair(bv, p, sv[w], si[w]);
    if (tid == 0) {
      gbl(L.ipiv)[col] = p;
      if ((bv == 0.0 || bv == __builtin_huge_val()) && info && info[blockIdx.x] == 0) info[blockIdx.x] = col + 1;
    }
    if (tid < NB) {
      C b = cmk<R>(0, 0);
      if (tid < jb) {
        const auto pc = P + (int64_t)tid * ld;
        const C a = pc[col];
        b = pc[p];
        if (p != col) {
          pc[col] = b;
          pc[p] = a;
        }
        if (tid == c) spiv = b;
      }
      prow[tid] = tid > c ? b : cmk<R>(0, 0);
    }
    __syncthreads();
    const C piv = spiv;
    const bool nz = piv.re != R(0) || piv.im != R(0);
    const C inv = nz ? zrecip(piv) : cmk<R>(0, 0);
    const C pn = prow[min(c + 1, NB - 1)];
    best = -1.0;
    bi = -1;
    for (int r = j0 + tid; r < n; r += NT) {
      if (r <= col) continue;
      // c, jb and the LDS index base pass through an empty asm statement once per row:
      // the per-column predicates and the pivot-row reads are then formed inside the loop
      // instead of being hoisted out of it into registers that would not fit
      int cr = c, jr = jb, zr = 0;
      asm volatile("" : "+s"(cr));
      asm volatile("" : "+s"(jr));
      asm volatile("" : "+v"(zr));
      const int o0 = r + c * ld;
      const C l = zmul(P[o0], inv);
      C nxt = P[o0 + (c + 1 < jb ? ld : 0)];
      // the row's columns right of col in two halves of NB / 2, each with all its loads
      // issued at once
      constexpr int HB = NB / 2;
      int o = o0;   // element offset of (r, cc), advanced one column at a time
      if (nz) P[o0] = l;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        C v[HB];
        int os = o;
#pragma unroll
        for (int t = 0; t < HB; ++t) {
          v[t] = cmk<R>(0, 0);
          if (hh * HB + t > cr && hh * HB + t < jr) {
            o += ld;
            v[t] = P[o];
          }
        }
        if (nz) {
#pragma unroll
          for (int t = 0; t < HB; ++t) v[t] = zfms(v[t], l, prow[hh * HB + t + zr]);
#pragma unroll
          for (int t = 0; t < HB; ++t)
            if (hh * HB + t > cr && hh * HB + t < jr) {
              os += ld;
              P[os] = v[t];
            }
        }
      }
      if (nz) nxt = zfms(nxt, l, pn);
      if (c + 1 < jb) argmax_pair(best, bi, fabs((double)nxt.re) + fabs((double)nxt.im), r);
    }
  }
}

// apply the swaps of panel [j0, j0+jb) to the columns outside the panel.  The swaps are
// composed first (one lane, in LDS: cont[r] = the row whose entry ends in row r), so that
// each thread (one column) loads every affected entry at once and stores them after: the
// rows j0 .. j0+jb-1 and the pivot rows, at most 2 PMX_LU_NB entries, with no chain of
// dependent loads.
template <class R>
__global__ __launch_bounds__(64) void k_laswp_panel(const LuDescT<R>* lus, int j0) {
  typedef cx<R> C;
  extern __shared__ int cont[];   // [n]
  const LuDescT<R> L = lus[blockIdx.y];
  const int n = L.n;
  const int jb = min(PMX_LU_NB, n - j0);
  if (jb <= 0) return;
  if ((int)(blockIdx.x * 64) >= n - jb) return;
  __shared__ int ipl[PMX_LU_NB];   // the panel's pivots, read from memory once, by jb lanes at once
  for (int r = threadIdx.x; r < n; r += 64) cont[r] = r;
  if ((int)threadIdx.x < jb) ipl[threadIdx.x] = gbl(L.ipiv)[j0 + threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    int pv[PMX_LU_NB];
#pragma unroll
    for (int c = 0; c < PMX_LU_NB; ++c) pv[c] = ipl[min(c, jb - 1)];
#pragma unroll
    for (int c = 0; c < PMX_LU_NB; ++c) {
      if (c < jb) {
        const int p = pv[c];
        const int t = cont[j0 + c];
        cont[j0 + c] = cont[p];
        cont[p] = t;
      }
    }
  }
  __syncthreads();
  int col = blockIdx.x * 64 + threadIdx.x;
  if (col >= n - jb) return;
  if (col >= j0) col += jb;
  const auto A = gbl(L.a) + (int64_t)col * L.ld;
  C v[2 * PMX_LU_NB];
#pragma unroll
  for (int c = 0; c < PMX_LU_NB; ++c) {
    if (c < jb) {
      v[c] = A[cont[j0 + c]];
      v[PMX_LU_NB + c] = A[cont[ipl[c]]];
    }
  }
#pragma unroll
  for (int c = 0; c < PMX_LU_NB; ++c) {
    if (c < jb) {
      A[j0 + c] = v[c];
      A[ipl[c]] = v[PMX_LU_NB + c];
    }
  }
}

template <class R>
struct FLuTrsm {
  const LuDescT<R>* d;
  int j0;
  __device__ bool operator()(int b, TrsmArgs<R>& a) const {
    LuDescT<R> L = d[b];
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

template <class R>
struct FLuUpd {
  const LuDescT<R>* d;
  int j0;
  __device__ bool operator()(int b, GemmArgsT<R>& g) const {
    LuDescT<R> L = d[b];
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

// the row permutation P of the swaps ipiv: perm[i] = original row of row i of P b
template <class R>
__global__ __launch_bounds__(256) void k_lu_perm(const LuDescT<R>* lus) {
  const LuDescT<R> L = lus[blockIdx.x];
  if (!L.perm || L.n <= 0) return;
  extern __shared__ int pl[];
  for (int i = threadIdx.x; i < L.n; i += 256) pl[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 0; i < L.n; ++i) {
      const int p = gbl(L.ipiv)[i];
      const int t = pl[i];
      pl[i] = pl[p];
      pl[p] = t;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < L.n; i += 256) gbl(L.perm)[i] = pl[i];
}

// whether panel variant v holds `rows` panel rows (registers: 256, 512, 1024 rows; the
// 1024-row variant spills in FP64)
template <class R>
static bool lu_panel_fits(int v, int rows) {
  switch (v) {
    case 0: return rows <= 256;
    case 1: return rows <= 512;
    case 2: return sizeof(R) == 4 && rows <= 1024;
    case 3: return true;
    case 4: return rows <= 256;
    case 6: return rows <= 512;
    case 8: return sizeof(R) == 4 && rows <= 1024;
    case 10: return true;
    default: return false;
  }
}

template <class R>
void la_lu_panel(int variant, const LuDescT<R>* d_lu, int batch, int j0, int* d_info, hipStream_t s) {
  KScope ks(PK_GETRF_PANEL, s);
  switch (variant) {
    case 0:
      PMX_LAUNCH((k_getrf_panel_reg<R, 256, 1>), dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
      break;
    case 1:
      PMX_LAUNCH((k_getrf_panel_reg<R, 256, 2>), dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
      break;
    case 2:
      if (sizeof(R) == 4) {
        PMX_LAUNCH((k_getrf_panel_reg<R, 512, 2>), dim3(batch), dim3(512), 0, s, d_lu, j0, d_info);
        break;
      }
      PMX_LAUNCH(k_getrf_panel<R>, dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
      break;
    case 4:
      PMX_LAUNCH((k_getrf_panel_u<R, 256, 1>), dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
      break;
    case 6:
      PMX_LAUNCH((k_getrf_panel_u<R, 512, 1>), dim3(batch), dim3(512), 0, s, d_lu, j0, d_info);
      break;
    case 8:
      if (sizeof(R) == 4) {
        PMX_LAUNCH((k_getrf_panel_u<float, 1024, 1>), dim3(batch), dim3(1024), 0, s,
                           (const LuDescT<float>*)d_lu, j0, d_info);
        break;
      }
      [[fallthrough]];
    case 10:
      if (sizeof(R) == 4)
        PMX_LAUNCH((k_getrf_panel_t<float, 1024>), dim3(batch), dim3(1024), 0, s,
                           (const LuDescT<float>*)d_lu, j0, d_info);
      else
        PMX_LAUNCH((k_getrf_panel_t<double, 512>), dim3(batch), dim3(512), 0, s,
                           (const LuDescT<double>*)d_lu, j0, d_info);
      break;
    default:
      PMX_LAUNCH(k_getrf_panel<R>, dim3(batch), dim3(256), 0, s, d_lu, j0, d_info);
      break;
  }
}

template <class R>
void la_getrf(const LuDescT<R>* d_lu, int batch, int max_n, int* d_info, hipStream_t s) {
  if (batch <= 0 || max_n <= 0) return;
  for (int j0 = 0; j0 < max_n; j0 += PMX_LU_NB) {
    {
      // panel rows max_n - j0: by default the unrolled register kernels when the rows fit
      // one per thread (512 rows, 1024 in FP32), else the tall-panel kernel; a
      // launch-parameter table may choose another variant that holds the rows
      const int rows = max_n - j0;
      const int dflt = rows <= 256 ? 4 : rows <= 512 ? 6 : (rows <= 1024 && sizeof(R) == 4) ? 8 : 10;
      int v = tune_choice(TK_LU_PANEL, (int)sizeof(R), tune_bucket_size(rows), tune_bucket_batch(batch), 0, dflt,
                          rows, batch, 0);
      if (!lu_panel_fits<R>(v, rows)) v = dflt;
      la_lu_panel<R>(v, d_lu, batch, j0, d_info, s);
    }
    const size_t shm = (size_t)max_n * sizeof(int);
    if (shm > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)k_laswp_panel<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    PMX_LAUNCH(k_laswp_panel<R>, dim3((max_n + 63) / 64, batch), dim3(64), shm, s, d_lu, j0);
    int rem = max_n - j0 - PMX_LU_NB;
    if (rem > 0) {
      launch_trsm_small<R, false, true>(FLuTrsm<R>{d_lu, j0}, batch, rem, s);
      launch_zgemm<R, OP_N, OP_N>(FLuUpd<R>{d_lu, j0}, batch, rem, rem, cmk<R>(-1, 0), cmk<R>(1, 0), s);
    }
  }
  const size_t shm = (size_t)max_n * sizeof(int);
  if (shm > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_lu_perm<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  PMX_LAUNCH(k_lu_perm<R>, dim3(batch), dim3(256), shm, s, d_lu);
}

// ---------------------------------------------------------------------------------
// getrs
// B <- P B: row i of the result is row perm[i] of B (from getrf, or composed here from
// ipiv by one lane when the factor has none).  Each workgroup stages ncol columns in LDS
// and writes them back permuted: two coalesced passes instead of a chain of swaps.
template <class R>
__global__ __launch_bounds__(256) void k_laswp_rhs(const LuDescT<R>* lus, const MatT<R>* bs, int ncol) {
  typedef cx<R> C;
  extern __shared__ char ls_smem[];
  const LuDescT<R> L = lus[blockIdx.y];
  const MatT<R> B = bs[blockIdx.y];
  const int n = L.n;
  const int c0 = blockIdx.x * ncol;
  if (n <= 0 || c0 >= B.n) return;
  const int nc = min(ncol, B.n - c0);
  int* cont = reinterpret_cast<int*>(ls_smem);                       // [n]
  C* col = reinterpret_cast<C*>(ls_smem + ((n * sizeof(int) + 15) / 16) * 16);   // [ncol][n]
  const auto Bp = gbl(B.p);
  if (L.perm) {
    const auto perm = gbl(L.perm);
    for (int r = threadIdx.x; r < n; r += 256) cont[r] = perm[r];
  } else {
    for (int r = threadIdx.x; r < n; r += 256) cont[r] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
      const auto ipiv = gbl(L.ipiv);
      for (int c = 0; c < n; ++c) {
        const int p = ipiv[c];
        const int t = cont[c];
        cont[c] = cont[p];
        cont[p] = t;
      }
    }
  }
  // eight loads in flight per thread before their LDS stores
  for (int e0 = threadIdx.x; e0 < n * nc; e0 += 256 * 8) {
    C t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + 256 * u, n * nc - 1);
      t[u] = Bp[e % n + (int64_t)(c0 + e / n) * B.ld];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 256 * u;
      if (e < n * nc) col[(e / n) * n + e % n] = t[u];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * nc; e += 256) {
    const int i = e % n, c = e / n;
    Bp[i + (int64_t)(c0 + c) * B.ld] = col[c * n + cont[i]];
  }
}

template <class R>
struct FRsTrsm {
  const LuDescT<R>* d;
  const MatT<R>* b;
  int j0;
  __device__ bool operator()(int i, TrsmArgs<R>& a) const {
    LuDescT<R> L = d[i];
    MatT<R> B = b[i];
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

template <class R>
struct FRsFwd {
  const LuDescT<R>* d;
  const MatT<R>* b;
  int j0;
  __device__ bool operator()(int i, GemmArgsT<R>& g) const {
    LuDescT<R> L = d[i];
    MatT<R> B = b[i];
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

template <class R>
struct FRsBwd {
  const LuDescT<R>* d;
  const MatT<R>* b;
  int j0;
  __device__ bool operator()(int i, GemmArgsT<R>& g) const {
    LuDescT<R> L = d[i];
    MatT<R> B = b[i];
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

template <class R>
void la_getrs(const LuDescT<R>* d_lu, const MatT<R>* d_b, int batch, int max_n, int max_nrhs, hipStream_t s) {
  if (batch <= 0 || max_n <= 0 || max_nrhs <= 0) return;
  const cx<R> one = cmk<R>(1, 0), mone = cmk<R>(-1, 0);
  {
    // columns staged per workgroup: about 32 KiB of LDS, at least one
    const size_t cb = (size_t)max_n * sizeof(cx<R>);
    const int ncol = (int)std::max<size_t>(1, std::min<size_t>(16, (32 * 1024) / cb));
    const size_t shm = ((size_t)max_n * sizeof(int) + 15) / 16 * 16 + (size_t)ncol * cb;
    if (shm > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)k_laswp_rhs<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    PMX_LAUNCH(k_laswp_rhs<R>, dim3((max_nrhs + ncol - 1) / ncol, batch), dim3(256), shm, s, d_lu, d_b, ncol);
  }
  const int nblk = (max_n + PMX_LU_NB - 1) / PMX_LU_NB;
  for (int bk = 0; bk < nblk; ++bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<R, false, true>(FRsTrsm<R>{d_lu, d_b, j0}, batch, max_nrhs, s);
    int rem = max_n - j0 - PMX_LU_NB;
    if (rem > 0) launch_zgemm<R, OP_N, OP_N>(FRsFwd<R>{d_lu, d_b, j0}, batch, rem, max_nrhs, mone, one, s);
  }
  for (int bk = nblk - 1; bk >= 0; --bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<R, true, false>(FRsTrsm<R>{d_lu, d_b, j0}, batch, max_nrhs, s);
    if (j0 > 0) launch_zgemm<R, OP_N, OP_N>(FRsBwd<R>{d_lu, d_b, j0}, batch, j0, max_nrhs, mone, one, s);
  }
}

// Fused solve for few right-hand sides.  Workgroup (entry b, group of NRC columns): the
// permuted right-hand side goes to the workspace, then blocks of 32 rows are finished in
// turn.  Inside a block each wave solves the 32x32 triangle for its columns with the block
// of the factor held in registers (one row per lane, broadcasts by lane shuffles, no
// barrier); then the whole workgroup subtracts the block's contribution from the rows
// still to come, each thread issuing the 32 loads of a row of the factor at once (coalesced
// across threads) so that the sweep is bound by bandwidth rather than load latency.  The
// backward sweep writes each finished block to B.
#define GS_NT 256

// rows [i0, i1) of x (workspace columns c0..c0+nc-1) -= A[rows, j0:j0+jb] xb
template <class R, int NRC>
__device__ inline void getrs_update(const cx<R>* A, int64_t ld, cx<R>* W, int64_t ldw, int c0, int nc, int i0, int i1,
                                    int j0, int jb, const cx<R> (*xb)[NRC]) {
  typedef cx<R> C;
  const auto Ag = gbl(A);
  const auto Wg = gbl(W);
  for (int i = i0 + (int)threadIdx.x; i < i1; i += GS_NT) {
    C acc[NRC];
#pragma unroll
    for (int c = 0; c < NRC; ++c) acc[c] = (c < nc) ? Wg[i + (int64_t)(c0 + c) * ldw] : cmk<R>(0, 0);
#pragma unroll
    for (int h = 0; h < 32; h += 16) {
      C l[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) l[k] = Ag[i + (int64_t)(j0 + min(h + k, jb - 1)) * ld];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (h + k < jb) {
#pragma unroll
          for (int c = 0; c < NRC; ++c) acc[c] = zfms(acc[c], l[k], xb[h + k][c]);
        }
    }
#pragma unroll
    for (int c = 0; c < NRC; ++c)
      if (c < nc) Wg[i + (int64_t)(c0 + c) * ldw] = acc[c];
  }
}

template <class R, int NRC>
__global__ __launch_bounds__(GS_NT) void k_getrs_small(const LuDescT<R>* lus, const MatT<R>* bs, const MatT<R>* ws) {
  typedef cx<R> C;
  const LuDescT<R> L = lus[blockIdx.x];
  const MatT<R> B = bs[blockIdx.x];
  const MatT<R> W = ws[blockIdx.x];
  const int n = L.n;
  const int c0 = blockIdx.y * NRC;
  const int nc = min(NRC, B.n - c0);
  if (n <= 0 || nc <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const auto A = gbl(L.a);
  const int64_t ld = L.ld;
  __shared__ C xb[32][NRC];
  for (int e = tid; e < n * nc; e += GS_NT) {
    const int i = e % n, c = e / n;
    gbl(W.p)[i + (int64_t)(c0 + c) * W.ld] = gbl(B.p)[gbl(L.perm)[i] + (int64_t)(c0 + c) * B.ld];
  }
  __syncthreads();
  // forward: L unit lower
  for (int j0 = 0; j0 < n; j0 += 32) {
    const int jb = min(32, n - j0);
    if (wave < nc) {
      const int r = j0 + min(lane, jb - 1);
      C lrow[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) lrow[k] = A[r + (int64_t)(j0 + min(k, jb - 1)) * ld];
      for (int c = wave; c < nc; c += GS_NT / 64) {
        C x = (lane < jb) ? W.p[j0 + lane + (int64_t)(c0 + c) * W.ld] : cmk<R>(0, 0);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
          const C xk = readlane(x, k);
          if (lane > k && k < jb) x = zfms(x, lrow[k], xk);
        }
        if (lane < jb) {
          xb[lane][c] = x;
          W.p[j0 + lane + (int64_t)(c0 + c) * W.ld] = x;
        }
      }
    }
    __syncthreads();
    getrs_update<R, NRC>(A, ld, W.p, W.ld, c0, nc, j0 + jb, n, j0, jb, xb);
    __syncthreads();
  }
  // backward: U upper with its diagonal
  for (int j0 = ((n - 1) / 32) * 32; j0 >= 0; j0 -= 32) {
    const int jb = min(32, n - j0);
    if (wave < nc) {
      const int r = j0 + min(lane, jb - 1);
      C urow[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) urow[k] = A[r + (int64_t)(j0 + min(k, jb - 1)) * ld];
      for (int c = wave; c < nc; c += GS_NT / 64) {
        C x = (lane < jb) ? W.p[j0 + lane + (int64_t)(c0 + c) * W.ld] : cmk<R>(0, 0);
#pragma unroll
        for (int k = 31; k >= 0; --k) {
          if (k < jb) {
            if (lane == k) x = zdiv(x, urow[k]);
            const C xk = readlane(x, k);
            if (lane < k) x = zfms(x, urow[k], xk);
          }
        }
        if (lane < jb) {
          xb[lane][c] = x;
          B.p[j0 + lane + (int64_t)(c0 + c) * B.ld] = x;
        }
      }
    }
    __syncthreads();
    getrs_update<R, NRC>(A, ld, W.p, W.ld, c0, nc, 0, j0, j0, jb, xb);
    __syncthreads();
  }
}

// The same solve with the whole solution block x (n x NRC) held in LDS: no global round
// trips for x between the steps, diagonal blocks of BS rows (one lane per row, solved
// values broadcast by readlane), and NT threads so that every thread has about one row
// of each trailing update, whose BS factors it loads in two halves.  Rows beyond n and
// right-hand sides beyond the matrix's count are padded with zeros and not stored.
template <class R, int NRC, int NT, int BS>
__global__ __launch_bounds__(NT) void k_getrs_lds_wide(const LuDescT<R>* lus, const MatT<R>* bs) {
  typedef cx<R> C;
  constexpr int HB = BS / 2;
  const LuDescT<R> L = lus[blockIdx.x];
  const MatT<R> B = bs[blockIdx.x];
  const int n = L.n;
  const int c0 = blockIdx.y * NRC;
  const int nc = min(NRC, B.n - c0);
  if (n <= 0 || nc <= 0) return;
  extern __shared__ char gs_smem[];
  C* xs = reinterpret_cast<C*>(gs_smem);   // xs[c * n + i]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const auto A = gbl(L.a);
  const auto Bp = gbl(B.p);
  const auto perm = gbl(L.perm);
  const int64_t ld = L.ld;
  for (int e = tid; e < n * NRC; e += NT) {
    const int i = e % n, c = e / n;
    xs[e] = (c < nc) ? Bp[perm[i] + (int64_t)(c0 + c) * B.ld] : cmk<R>(0, 0);
  }
  __syncthreads();
  // forward: L unit lower
  for (int j0 = 0; j0 < n; j0 += BS) {
    const int jb = min(BS, n - j0);
    if (wave < NRC) {
      const int r = j0 + min(lane, jb - 1);
      C lrow[BS];
#pragma unroll
      for (int k = 0; k < BS; ++k) lrow[k] = A[r + (int64_t)(j0 + min(k, jb - 1)) * ld];
      C x = (lane < jb) ? xs[wave * n + j0 + lane] : cmk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < BS; ++k) {
        const C xk = readlane(x, k);
        if (lane > k && k < jb) x = zfms(x, lrow[k], xk);
      }
      if (lane < jb) xs[wave * n + j0 + lane] = x;
    }
    __syncthreads();
    for (int i = j0 + jb + tid; i < n; i += NT) {
      C acc[NRC];
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[c] = xs[c * n + i];
#pragma unroll
      for (int h = 0; h < BS; h += HB) {
        C l[HB];
#pragma unroll
        for (int k = 0; k < HB; ++k) l[k] = A[i + (int64_t)(j0 + min(h + k, jb - 1)) * ld];
#pragma unroll
        for (int k = 0; k < HB; ++k)
          if (h + k < jb) {
#pragma unroll
            for (int c = 0; c < NRC; ++c) acc[c] = zfms(acc[c], l[k], xs[c * n + j0 + h + k]);
          }
      }
#pragma unroll
      for (int c = 0; c < NRC; ++c) xs[c * n + i] = acc[c];
    }
    __syncthreads();
  }
  // backward: U upper with its diagonal
  for (int j0 = ((n - 1) / BS) * BS; j0 >= 0; j0 -= BS) {
    const int jb = min(BS, n - j0);
    if (wave < NRC) {
      const int r = j0 + min(lane, jb - 1);
      C urow[BS];
#pragma unroll
      for (int k = 0; k < BS; ++k) urow[k] = A[r + (int64_t)(j0 + min(k, jb - 1)) * ld];
      C dinv = urow[0];
#pragma unroll
      for (int k = 1; k < BS; ++k)
        if (k == lane) dinv = urow[k];
      dinv = zrecip(dinv);
      C x = (lane < jb) ? xs[wave * n + j0 + lane] : cmk<R>(0, 0);
#pragma unroll
      for (int k = BS - 1; k >= 0; --k) {
        if (k < jb) {
          if (lane == k) x = zmul(x, dinv);
          const C xk = readlane(x, k);
          if (lane < k) x = zfms(x, urow[k], xk);
        }
      }
      if (lane < jb) xs[wave * n + j0 + lane] = x;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += NT) {
      C acc[NRC];
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[c] = xs[c * n + i];
#pragma unroll
      for (int h = 0; h < BS; h += HB) {
        C l[HB];
#pragma unroll
        for (int k = 0; k < HB; ++k) l[k] = A[i + (int64_t)(j0 + min(h + k, jb - 1)) * ld];
#pragma unroll
        for (int k = 0; k < HB; ++k)
          if (h + k < jb) {
#pragma unroll
            for (int c = 0; c < NRC; ++c) acc[c] = zfms(acc[c], l[k], xs[c * n + j0 + h + k]);
          }
      }
#pragma unroll
      for (int c = 0; c < NRC; ++c) xs[c * n + i] = acc[c];
    }
    __syncthreads();
  }
  for (int e = tid; e < n * nc; e += NT) {
    const int i = e % n, c = e / n;
    Bp[i + (int64_t)(c0 + c) * B.ld] = xs[c * n + i];
  }
}

// The LDS-resident solve with its waves in two roles and the loads of the factor issued one
// block ahead.  Wave 0 solves the diagonal blocks (one lane per row of the block, the four
// right-hand sides at once, solved values broadcast by readlane).  The other NTT threads own
// fixed rows (thread t: rows t + q NTT, q < RPT) and keep their rows of the solution block
// in registers across the whole sweep; per block they subtract the block's contribution,
// with the block's factor columns of their first row already in registers, and store a row
// to LDS only when it enters the next diagonal block.  Right after its use, each role issues
// the loads of the next block (wave 0: the next diagonal block's row; the others: the next
// block's columns of their first row), so that the loads overlap the other role's work
// instead of following it.  Two barriers per block.  Rows beyond n and right-hand sides
// beyond the matrix's count are padded with zeros and not stored; the block of a lane
// beyond the block's rows is clamped to its last row.
template <class R, int NTT, int RPT, int BS, int NRC>
__global__ __launch_bounds__(64 + NTT) void k_getrs_lds(const LuDescT<R>* lus, const MatT<R>* bs) {
  typedef cx<R> C;
  constexpr int NT = 64 + NTT;
  const LuDescT<R> L = lus[blockIdx.x];
  const MatT<R> B = bs[blockIdx.x];
  const int n = L.n;
  const int c0 = blockIdx.y * NRC;
  const int nc = min(NRC, B.n - c0);
  if (n <= 0 || nc <= 0) return;
  extern __shared__ char gs_smem[];
  C* xs = reinterpret_cast<C*>(gs_smem);   // xs[c * n + i]
  const int tid = threadIdx.x, lane = tid & 63;
  const bool dw = tid < 64;
  const int t = tid - 64;
  const auto A = gbl(L.a);
  const auto Bp = gbl(B.p);
  const auto perm = gbl(L.perm);
  const int64_t ld = L.ld;
  for (int e = tid; e < n * NRC; e += NT) {
    const int i = e % n, c = e / n;
    xs[e] = (c < nc) ? Bp[perm[i] + (int64_t)(c0 + c) * B.ld] : cmk<R>(0, 0);
  }
  C buf[BS];             // wave 0: its row of the diagonal block; others: the block of their first row
  C acc[RPT][NRC];       // others: their rows of the solution block (wave 0: the block's values)
#define PMX_GS_LOAD(r, j, jb)                                                    \
  _Pragma("unroll") for (int k = 0; k < BS; ++k) buf[k] = A[(r) + (int64_t)((j) + min(k, (jb) - 1)) * ld]
  // a row's update by the solved block: without per-column branches for full blocks, so
  // that the LDS reads of the solved values can be issued ahead of their use
#define PMX_GS_UPDATE(q)                                                                   \
  if (jb == BS) {                                                                          \
    _Pragma("unroll") for (int k = 0; k < BS; ++k)                                         \
      _Pragma("unroll") for (int c = 0; c < NRC; ++c)                                      \
        acc[q][c] = zfms(acc[q][c], buf[k], xs[c * n + j0 + k]);                    \
  } else {                                                                                 \
    _Pragma("unroll") for (int k = 0; k < BS; ++k) {                                       \
      if (k < jb) {                                                                        \
        _Pragma("unroll") for (int c = 0; c < NRC; ++c)                                    \
          acc[q][c] = zfms(acc[q][c], buf[k], xs[c * n + j0 + k]);                  \
      }                                                                                    \
    }                                                                                      \
  }
  // ---- forward: L unit lower
  {
    const int jb = min(BS, n);
    if (dw) {
      PMX_GS_LOAD(min(lane, jb - 1), 0, jb);
    } else if (t >= jb && t < n) {
      PMX_GS_LOAD(t, 0, jb);
    }
  }
  __syncthreads();
  if (!dw) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + q * NTT;
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[q][c] = (r < n) ? xs[c * n + r] : cmk<R>(0, 0);
    }
  }
  for (int j0 = 0; j0 < n; j0 += BS) {
    const int jb = min(BS, n - j0);
    const int j1 = j0 + BS;
    const int jb1 = min(BS, n - j1);
    if (dw) {
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[0][c] = (lane < jb) ? xs[c * n + j0 + lane] : cmk<R>(0, 0);
#pragma unroll
      for (int k = 0; k < BS; ++k) {
        if (k < jb) {
#pragma unroll
          for (int c = 0; c < NRC; ++c) {
            const C xk = readlane(acc[0][c], k);
            if (lane > k) acc[0][c] = zfms(acc[0][c], buf[k], xk);
          }
        }
      }
      if (lane < jb) {
#pragma unroll
        for (int c = 0; c < NRC; ++c) xs[c * n + j0 + lane] = acc[0][c];
      }
      if (j1 < n) PMX_GS_LOAD(j1 + min(lane, jb1 - 1), j1, jb1);
    }
    __syncthreads();
    if (!dw) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * NTT;
        if (r >= j0 + jb && r < n) {
          if (q > 0) PMX_GS_LOAD(r, j0, jb);
          PMX_GS_UPDATE(q);
          if (r < j1 + jb1) {
#pragma unroll
            for (int c = 0; c < NRC; ++c) xs[c * n + r] = acc[q][c];
          }
        }
      }
      if (j1 < n && t >= j1 + jb1 && t < n) PMX_GS_LOAD(t, j1, jb1);
    }
    __syncthreads();
  }
  // ---- backward: U upper with its diagonal
  const int jl = ((n - 1) / BS) * BS;
  {
    const int jb = n - jl;
    if (dw) {
      PMX_GS_LOAD(jl + min(lane, jb - 1), jl, jb);
    } else if (t < jl) {
      PMX_GS_LOAD(t, jl, jb);
    }
  }
  if (!dw) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + q * NTT;
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[q][c] = (r < n) ? xs[c * n + r] : cmk<R>(0, 0);
    }
  }
  for (int j0 = jl; j0 >= 0; j0 -= BS) {
    const int jb = min(BS, n - j0);
    const int j1 = j0 - BS;
    if (dw) {
      C dinv = buf[0];
#pragma unroll
      for (int k = 1; k < BS; ++k)
        if (k == lane) dinv = buf[k];
      dinv = zrecip(dinv);
#pragma unroll
      for (int c = 0; c < NRC; ++c) acc[0][c] = (lane < jb) ? xs[c * n + j0 + lane] : cmk<R>(0, 0);
#pragma unroll
      for (int k = BS - 1; k >= 0; --k) {
        if (k < jb) {
#pragma unroll
          for (int c = 0; c < NRC; ++c) {
            if (lane == k) acc[0][c] = zmul(acc[0][c], dinv);
            const C xk = readlane(acc[0][c], k);
            if (lane < k) acc[0][c] = zfms(acc[0][c], buf[k], xk);
          }
        }
      }
      if (lane < jb) {
#pragma unroll
        for (int c = 0; c < NRC; ++c) xs[c * n + j0 + lane] = acc[0][c];
      }
      if (j1 >= 0) PMX_GS_LOAD(j1 + min(lane, BS - 1), j1, BS);
    }
    __syncthreads();
    if (!dw) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = t + q * NTT;
        if (r < j0) {
          if (q > 0) PMX_GS_LOAD(r, j0, jb);
          PMX_GS_UPDATE(q);
          if (r >= j1) {
#pragma unroll
            for (int c = 0; c < NRC; ++c) xs[c * n + r] = acc[q][c];
          }
        }
      }
      if (j1 >= 0 && t < j1) PMX_GS_LOAD(t, j1, BS);
    }
    __syncthreads();
  }
#undef PMX_GS_LOAD
#undef PMX_GS_UPDATE
  for (int e = tid; e < n * nc; e += NT) {
    const int i = e % n, c = e / n;
    Bp[i + (int64_t)(c0 + c) * B.ld] = xs[c * n + i];
  }
}

// LDS-resident level solve for up to 4 right-hand sides per workgroup; false when the
// solution block does not fit (the caller then uses another variant)
template <class R>
bool la_getrs_lds(const LuDescT<R>* d_lu, const MatT<R>* d_b, int batch, int max_n, int max_nrhs, hipStream_t s) {
  const size_t shm4 = (size_t)max_n * 4 * sizeof(cx<R>);
  if (shm4 > 128 * 1024 || max_n <= 0) return false;
  // few matrices: one workgroup per right-hand side, so that more compute units share the
  // sequential sweeps (each reads the factor once more); more: two, then four right-hand
  // sides each
  const int nrc = (batch * max_nrhs <= 256 && max_n <= 1792) ? 1 : (batch * max_nrhs <= 1024 && max_n <= 1920) ? 2 : 4;
  const size_t shm = (size_t)max_n * nrc * sizeof(cx<R>);
  const dim3 grid(batch, (max_nrhs + nrc - 1) / nrc);
  KScope ks(PK_GETRS, s);
  auto go = [&](auto kern, int nt) {
    if (shm > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    PMX_LAUNCH(kern, grid, dim3(nt), shm, s, d_lu, d_b);
  };
  // blocks of 32 rows (FP32) or 16 (FP64): the row held in registers stays at 64 of them
  constexpr int BS = sizeof(R) == 4 ? 32 : 16;
  // one right-hand side per workgroup: 512 threads and diagonal blocks of 64 rows (FP32) or
  // 32 (FP64), half the sequential steps; the row-owning threads take up to four rows each
  constexpr int BS1 = sizeof(R) == 4 ? 64 : 32;
  if (nrc == 1) {
    if constexpr (sizeof(R) == 4) {
      // FP32 above 448 rows: 1024 threads with blocks of 32 rows, so that each row-owning
      // thread has at most two rows (the first one's loads issued a block ahead)
      if (max_n > 448) {
        if (max_n <= 960)
          go(k_getrs_lds<R, 960, 1, 32, 1>, 1024);
        else
          go(k_getrs_lds<R, 960, 2, 32, 1>, 1024);
        return true;
      }
    }
    if (max_n <= 448)
      go(k_getrs_lds<R, 448, 1, BS1, 1>, 512);
    else if (max_n <= 896)
      go(k_getrs_lds<R, 448, 2, BS1, 1>, 512);
    else if (max_n <= 1344)
      go(k_getrs_lds<R, 448, 3, BS1, 1>, 512);
    else
      go(k_getrs_lds<R, 448, 4, BS1, 1>, 512);
  } else if (nrc == 2) {
    if (max_n <= 256)
      go(k_getrs_lds<R, 256, 1, BS, 2>, 320);
    else if (max_n <= 448)
      go(k_getrs_lds<R, 448, 1, BS, 2>, 512);
    else if (max_n <= 960)
      go(k_getrs_lds<R, 960, 1, BS, 2>, 1024);
    else
      go(k_getrs_lds<R, 960, 2, BS, 2>, 1024);
  } else if (max_n <= 256) {
    go(k_getrs_lds<R, 256, 1, BS, 4>, 320);
  } else if (max_n <= 448) {
    go(k_getrs_lds<R, 448, 1, BS, 4>, 512);
  } else if (max_n <= 960) {
    go(k_getrs_lds<R, 960, 1, BS, 4>, 1024);
  } else if (max_n <= 1920) {
    go(k_getrs_lds<R, 960, 2, BS, 4>, 1024);
  } else {
    // 1024 threads leave 128 registers each: diagonal blocks of 32 (FP32) or 16 rows
    go(k_getrs_lds_wide<R, 4, 1024, sizeof(R) == 4 ? 32 : 16>, 1024);
  }
  return true;
}

template <class R>
void la_getrs_small(const LuDescT<R>* d_lu, const MatT<R>* d_b, const MatT<R>* d_w, int batch, int max_n,
                    int max_nrhs, hipStream_t s) {
  if (batch <= 0 || max_n <= 0 || max_nrhs <= 0) return;
  KScope ks(PK_GETRS, s);
  if (max_nrhs <= 1) {
    PMX_LAUNCH((k_getrs_small<R, 1>), dim3(batch, 1), dim3(GS_NT), 0, s, d_lu, d_b, d_w);
  } else if (max_nrhs <= 2) {
    PMX_LAUNCH((k_getrs_small<R, 2>), dim3(batch, 1), dim3(GS_NT), 0, s, d_lu, d_b, d_w);
  } else {
    PMX_LAUNCH((k_getrs_small<R, 4>), dim3(batch, (max_nrhs + 3) / 4), dim3(GS_NT), 0, s, d_lu, d_b, d_w);
  }
}

// ---------------------------------------------------------------------------------
// Householder QR as a tree of in-LDS block factorisations (TSQR panels); only R is kept.
//
// Panel [j0, j0+jb) of rows [j0, m): the rows are cut into blocks of PMX_TS_BR rows; each
// block is factored in LDS by one workgroup, leaving its R in the block's first jb rows.
// The stacked R factors form the rows of the next tree level (block b, row r < jb of
// level L-1 becomes row b*jb + r of level L), factored the same way until a single block
// remains, whose R is the panel's R in rows j0 .. j0+jb-1.  After each tree level the
// trailing columns of the same rows receive the block reflectors
// Q_b^H = I - V_b T_b^H V_b^H (one fused kernel: W = V^H A, A -= V (T^H W)).  Only R is
// kept, so the order of the untouched remaining rows is free.
#define PMX_TS_BR 256

struct TsGeom {
  int mr0, mr1, mr2, mr3;        // rows of tree levels 0..3
  int nb0, nb1, nb2, nb3;        // blocks of tree levels 0..3
  int64_t wo0, wo1, wo2, wo3;    // workspace offsets of the levels' V and T blocks
  int nlev;
};

__device__ inline int ts_sel(int L, int a0, int a1, int a2, int a3) {
  return L == 0 ? a0 : (L == 1 ? a1 : (L == 2 ? a2 : a3));
}
__device__ inline int64_t ts_sel64(int L, int64_t a0, int64_t a1, int64_t a2, int64_t a3) {
  return L == 0 ? a0 : (L == 1 ? a1 : (L == 2 ? a2 : a3));
}

__device__ inline void ts_geom(int m, int j0, int jb, TsGeom& g) {
  const int64_t blk = (int64_t)PMX_TS_BR * PMX_QR_NB;
  g.mr0 = m - j0;
  g.nb0 = (g.mr0 + PMX_TS_BR - 1) / PMX_TS_BR;
  g.wo0 = 0;
  g.mr1 = g.nb0 * jb;
  g.nb1 = g.nb0 > 1 ? (g.mr1 + PMX_TS_BR - 1) / PMX_TS_BR : 0;
  g.wo1 = g.wo0 + g.nb0 * blk;
  g.mr2 = g.nb1 * jb;
  g.nb2 = g.nb1 > 1 ? (g.mr2 + PMX_TS_BR - 1) / PMX_TS_BR : 0;
  g.wo2 = g.wo1 + g.nb1 * blk;
  g.mr3 = g.nb2 * jb;
  g.nb3 = g.nb2 > 1 ? (g.mr3 + PMX_TS_BR - 1) / PMX_TS_BR : 0;
  g.wo3 = g.wo2 + g.nb2 * blk;
  g.nlev = g.nb0 <= 1 ? 1 : (g.nb1 <= 1 ? 2 : (g.nb2 <= 1 ? 3 : 4));
}

// physical row of local row lr at tree level L, or -1 if the row does not exist
__device__ inline int ts_phys(int lr, int L, int jb, int j0, const TsGeom& g) {
  if (lr >= ts_sel(L, g.mr0, g.mr1, g.mr2, g.mr3)) return -1;
#pragma unroll
  for (int l = 3; l >= 1; --l) {
    if (l <= L) {
      const int b = lr / jb, r = lr - b * jb;
      lr = b * PMX_TS_BR + r;
      if (lr >= ts_sel(l - 1, g.mr0, g.mr1, g.mr2, g.mr3)) return -1;
    }
  }
  return j0 + lr;
}

// One block of one tree level: Householder QR of its rows of the panel, in registers.
// Columns are owned cyclically by the NT / 64 waves (column q by wave q % (NT / 64)), each
// lane holding rows lane + 64 k of them.  Step i: the owner of column i forms the
// reflector (norm accumulated in FP64 for both real types) and publishes it in LDS; after
// one barrier every wave applies it to its later columns and forms the compact-WY inner
// products z_q = V_q^H v of its earlier ones, the partial sums of all its columns reduced
// together.  Reflectors and inner products are double-buffered, so that a step needs one
// barrier; the column i - 1 of T (T[0:i-1, i-1] = -tau T z) is formed at step i, each
// thread on its own row of T.  Written back: R in the block's first rows, V and T to the
// workspace (V column-major, BR rows; T row-major, PMX_QR_NB x PMX_QR_NB, upper triangular).
template <class R, int NT>
__global__ __launch_bounds__(NT) void k_ts_leaf(const QrDescT<R>* qrs, int j0, int L) {
  typedef cx<R> C;
  constexpr int NW = NT / 64;                  // waves
  constexpr int RPL = PMX_TS_BR / 64;          // rows per lane
  constexpr int CPW = PMX_QR_NB / NW;          // columns per wave
  const QrDescT<R> Q = qrs[blockIdx.y];
  const int kmax = Q.kc;
  const int jb = min(PMX_QR_NB, kmax - j0);
  if (jb <= 0) return;
  TsGeom g;
  ts_geom(Q.m, j0, jb, g);
  if (L >= g.nlev) return;
  const int b = blockIdx.x;
  if (b >= ts_sel(L, g.nb0, g.nb1, g.nb2, g.nb3)) return;
  const int nrb = min(PMX_TS_BR, ts_sel(L, g.mr0, g.mr1, g.mr2, g.mr3) - b * PMX_TS_BR);
  __shared__ C vs[2][PMX_TS_BR];               // reflectors of even and odd steps
  __shared__ C zs[2][PMX_QR_NB];               // inner products of even and odd steps
  __shared__ C Ts[PMX_QR_NB][PMX_QR_NB + 1];
  __shared__ double taus[2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const auto A = gbl(Q.a);
  const int64_t ld = Q.ld;
  int phys[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int r = lane + 64 * k;
    phys[k] = (r < nrb) ? ts_phys(b * PMX_TS_BR + r, L, jb, j0, g) : -1;
  }
  C P[CPW][RPL];
#pragma unroll
  for (int m = 0; m < CPW; ++m) {
    const int q = wave + NW * m;
    const int64_t co = (int64_t)min(j0 + q, Q.c - 1) * ld;
#pragma unroll
    for (int k = 0; k < RPL; ++k) P[m][k] = (phys[k] >= 0 && q < jb) ? A[phys[k] + co] : cmk<R>(0, 0);
  }
  const int nref = min(jb, nrb);
  for (int i = 0; i < nref; ++i) {
    const int bi = i & 1;
    if (wave == i % NW) {
      const int om = i / NW;
      C x[RPL];
#pragma unroll
      for (int m = 0; m < CPW; ++m)
        if (m == om) {
#pragma unroll
          for (int k = 0; k < RPL; ++k) x[k] = P[m][k];
        }
      double p = 0;
      C a = x[0];
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        if (r >= i) p += (double)x[k].re * x[k].re + (double)x[k].im * x[k].im;
        if (k == (i >> 6)) a = x[k];
      }
      const double xn = sqrt(wave_sum(p));
      const C alpha = readlane(a, i & 63);
      const double aa = sqrt((double)alpha.re * alpha.re + (double)alpha.im * alpha.im);
      double tau;
      C beta, scale;
      if (xn == 0.0) {
        tau = 0.0;
        beta = cmk<R>(0, 0);
        scale = cmk<R>(0, 0);
      } else if (aa == 0.0) {
        tau = 1.0;
        beta = cmk<R>(-xn, 0);
        scale = cmk<R>(1.0 / xn, 0);
      } else {
        // beta = -alpha |x|/|alpha|, tau = 1 + |alpha|/|x|, scale = conj(alpha)/(|alpha|(|alpha|+|x|))
        const double ip = 1.0 / (aa * xn * (aa + xn));
        tau = (aa + xn) * aa * (aa + xn) * ip;
        beta = zscale(alpha, -xn * xn * (aa + xn) * ip);
        scale = zscale(zconj(alpha), xn * ip);
      }
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        const C v = (r == i) ? cmk<R>(1, 0) : ((r > i) ? zmul(x[k], scale) : cmk<R>(0, 0));
        vs[bi][r] = v;
        x[k] = (r == i) ? beta : ((r > i) ? v : x[k]);
      }
#pragma unroll
      for (int m = 0; m < CPW; ++m)
        if (m == om) {
#pragma unroll
          for (int k = 0; k < RPL; ++k) P[m][k] = x[k];
        }
      if (lane == 0) {
        taus[bi] = tau;
        Ts[i][i] = cmk<R>(tau, 0);
      }
    }
    __syncthreads();
    if (i >= 1 && t < i - 1) {   // T[0:i-1, i-1] = -tau_{i-1} T[0:i-1, 0:i-1] z_{i-1}, one row per thread
      const int c = i - 1;
      C s2 = cmk<R>(0, 0);
      for (int jj = t; jj < c; ++jj) s2 = zfma(Ts[t][jj], zs[c & 1][jj], s2);
      Ts[t][c] = zscale(s2, -Ts[c][c].re);
    }
    const R tau = (R)taus[bi];
    C vr[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) vr[k] = vs[bi][lane + 64 * k];
    R dr[CPW], di[CPW];
#pragma unroll
    for (int m = 0; m < CPW; ++m) {
      const int q = wave + NW * m;
      R sr = 0, si = 0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        // column q's reflector for q < i (unit diagonal, zero above), the column itself for q > i
        const C cq = (q > i) ? P[m][k] : ((r == q) ? cmk<R>(1, 0) : ((r > q) ? P[m][k] : cmk<R>(0, 0)));
        const C pr = zcmul(vr[k], cq);   // conj(v) c_q
        sr += pr.re;
        si += pr.im;
      }
      dr[m] = sr;
      di[m] = si;
    }
#pragma unroll
    for (int m = 0; m < CPW; ++m) {
      dr[m] = wave_sum(dr[m]);
      di[m] = wave_sum(di[m]);
    }
#pragma unroll
    for (int m = 0; m < CPW; ++m) {
      const int q = wave + NW * m;
      if (q > i && q < jb) {
        const C w = zscale(cmk<R>(dr[m], di[m]), tau);
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int r = lane + 64 * k;
          if (r >= i) P[m][k] = zfms(P[m][k], vr[k], w);
        }
      } else if (q < i && lane == 0) {
        zs[bi][q] = cmk<R>(dr[m], -di[m]);   // V_q^H v = conj(v^H V_q)
      }
    }
  }
  __syncthreads();
  if (nref >= 1 && t < nref - 1) {
    const int c = nref - 1;
    C s2 = cmk<R>(0, 0);
    for (int jj = t; jj < c; ++jj) s2 = zfma(Ts[t][jj], zs[c & 1][jj], s2);
    Ts[t][c] = zscale(s2, -Ts[c][c].re);
  }
  __syncthreads();
  // write back: R in the block's first rows, the reflectors V and T to the workspace
  if (phys[0] >= 0 && lane < jb) {
#pragma unroll
    for (int m = 0; m < CPW; ++m) {
      const int q = wave + NW * m;
      if (q < jb) A[phys[0] + (int64_t)(j0 + q) * ld] = (q >= lane) ? P[m][0] : cmk<R>(0, 0);
    }
  }
  const int64_t wo = ts_sel64(L, g.wo0, g.wo1, g.wo2, g.wo3) + (int64_t)b * PMX_TS_BR * PMX_QR_NB;
  const auto V = gbl(Q.v) + wo;
  const auto Tw = gbl(Q.t) + wo;
#pragma unroll
  for (int m = 0; m < CPW; ++m) {
    const int q = wave + NW * m;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      C v = cmk<R>(0, 0);
      if (q < nref && r < nrb) v = (r == q) ? cmk<R>(1, 0) : ((r > q) ? P[m][k] : cmk<R>(0, 0));
      V[r + (int64_t)q * PMX_TS_BR] = v;
    }
  }
  for (int e = t; e < PMX_QR_NB * PMX_QR_NB; e += NT) {
    const int r = e / PMX_QR_NB, c = e % PMX_QR_NB;
    Tw[e] = (r <= c && c < nref) ? Ts[r][c] : cmk<R>(0, 0);
  }
}

// The chip's eight XCDs each have their own L2, and consecutive workgroups of a dispatch go
// to them in turn (workgroup b to XCD b mod 8).  The column tiles of one block of a QR
// trailing update all read that block's V, so the update kernels map their linear workgroup
// index through this bijection, which hands each XCD runs of TS_XCD_RUN consecutive indices
// (run c of XCD x: indices (8 c + x) TS_XCD_RUN + i); indices past the last whole group of
// runs map to themselves.
#ifndef TS_XCD_RUN
#define TS_XCD_RUN 64
#endif
__device__ inline int ts_xcd_run(int b, int n) {
  constexpr int G = 8 * TS_XCD_RUN;
  if (b >= (n / G) * G) return b;
  const int x = b % 8, j = b / 8;
  return (j / TS_XCD_RUN) * G + x * TS_XCD_RUN + j % TS_XCD_RUN;
}

// trailing update of one block of one tree level in FP64: A_b -= V (T^H (V^H A_b)) on 32
// columns per workgroup.  Wave w owns columns 16 (w & 1) .. +15 and half w >> 1 of the
// block's rows; each lane keeps its entries of A_b in registers for the whole update, in
// the B-operand layout of the 16x16x4 FP64 MFMA of W = V^H A_b (lane j + 16 k holds rows
// 4 s + k of every 16-row block), which is also the accumulator layout of the product V W,
// so that A_b is read once and written once with no staging.  V comes from the workspace
// (shared through the cache by the block's column tiles); the two halves' partial W are
// summed in LDS, multiplied by T^H there, and read back as the B operand of V W.
// CB column blocks of 16 per workgroup (2 CB waves), so that one read of V from the cache
// serves 16 CB columns.  The launcher takes CB = 2: with CB = 4 (one read of V for 64
// columns, one workgroup of 512 threads per compute unit) a launch took 5.30 ms against
// 4.89 at 1M unknowns.
template <int CB>
__global__ __launch_bounds__(128 * CB, 2) void k_ts_update_f64(const QrDescT<double>* qrs, int j0, int L) {
  typedef double R;
  typedef cx<R> C;
  constexpr int NT = 128 * CB, TSU64_COLS = 16 * CB;
  constexpr int NRB = PMX_TS_BR / 32;   // 16-row blocks per half
  const int gx = (int)gridDim.x, gy = (int)gridDim.y;
  const int lb = ts_xcd_run((int)(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z)), gx * gy * (int)gridDim.z);
  const int bx = lb % gx, by = (lb / gx) % gy, bz = lb / (gx * gy);
  const QrDescT<R> Q = qrs[bz];
  const int kmax = Q.kc;
  const int jb = min(PMX_QR_NB, kmax - j0);
  const int nc = Q.c - j0 - jb;
  if (jb <= 0 || nc <= 0) return;
  const int c0 = bx * TSU64_COLS;
  if (c0 >= nc) return;
  TsGeom g;
  ts_geom(Q.m, j0, jb, g);
  if (L >= g.nlev) return;
  const int b = by;
  if (b >= ts_sel(L, g.nb0, g.nb1, g.nb2, g.nb3)) return;
  const int nrb = min(PMX_TS_BR, ts_sel(L, g.mr0, g.mr1, g.mr2, g.mr3) - b * PMX_TS_BR);
  const int64_t wo = ts_sel64(L, g.wo0, g.wo1, g.wo2, g.wo3) + (int64_t)b * PMX_TS_BR * PMX_QR_NB;
  const auto V = gbl(Q.v) + wo;
  const auto Tw = gbl(Q.t) + wo;
  __shared__ C Ws[PMX_QR_NB][TSU64_COLS + 1];
  __shared__ C Tl[PMX_QR_NB][PMX_QR_NB + 1];
  __shared__ int rows[PMX_TS_BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cb = wave % CB, h = wave / CB;
  const int j = lane & 15, k = lane >> 4;
  const auto A = gbl(Q.a);
  const int64_t ld = Q.ld;
  for (int i = tid; i < PMX_TS_BR; i += NT) rows[i] = (i < nrb) ? ts_phys(b * PMX_TS_BR + i, L, jb, j0, g) : -1;
  for (int e = tid; e < PMX_QR_NB * PMX_QR_NB; e += NT) Tl[e / PMX_QR_NB][e % PMX_QR_NB] = Tw[e];
  __syncthreads();
  const int cl = cb * 16 + j;                    // column within the tile
  const bool cok = c0 + cl < nc;
  const int64_t coff = (int64_t)(j0 + jb + c0 + min(cl, nc - 1 - c0)) * ld;
  const int rbase = h * (PMX_TS_BR / 2);
  C ar[NRB][4];
  // complex products as three real ones (Gauss): for W = V^H A, p1 = sum vr ar,
  // p2 = sum vi ai, p3 = sum (vr - vi)(ar + ai), so W = (p1 + p2) + i (p3 - p1 + p2)
  d4 p1[2], p2[2], p3[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    p1[q] = d4{0, 0, 0, 0};
    p2[q] = d4{0, 0, 0, 0};
    p3[q] = d4{0, 0, 0, 0};
  }
  // W = V^H A_b over this half's rows: step s of row block rb takes rows rb * 16 + 4 s + k
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int r0 = rbase + rb * 16;
#pragma unroll
    for (int t = 0; t < 4; ++t) ar[rb][t] = cmk<R>(0, 0);
    if (r0 < nrb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int lr = r0 + 4 * t + k;
        const int pr = rows[lr];
        if (pr >= 0 && cok) ar[rb][t] = A[pr + coff];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int lr = r0 + 4 * t + k;
        const bool rok = lr < nrb;
        const R as = ar[rb][t].re + ar[rb][t].im;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const C a = rok ? V[lr + (int64_t)(q * 16 + j) * PMX_TS_BR] : cmk<R>(0, 0);
          p1[q] = mfma16(a.re, ar[rb][t].re, p1[q]);
          p2[q] = mfma16(a.im, ar[rb][t].im, p2[q]);
          p3[q] = mfma16(a.re - a.im, as, p3[q]);
        }
      }
    }
  }
  // sum the halves: accumulator element (q * 16 + k + 4 r, cl) in register r
  if (h == 1) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Ws[q * 16 + k + 4 * r][cl] = cmk<R>(p1[q][r] + p2[q][r], p3[q][r] - p1[q][r] + p2[q][r]);
  }
  __syncthreads();
  if (h == 0) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const C o = Ws[q * 16 + k + 4 * r][cl];
        Ws[q * 16 + k + 4 * r][cl] =
            cmk<R>(o.re + (p1[q][r] + p2[q][r]), o.im + (p3[q][r] - p1[q][r] + p2[q][r]));
      }
  }
  __syncthreads();
  // W <- T^H W, T upper triangular
  {
    constexpr int PER = PMX_QR_NB * TSU64_COLS / NT;
    const int col = tid % TSU64_COLS, i0 = (tid / TSU64_COLS) * PER;
    C w2[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = i0 + u;
      C acc = cmk<R>(0, 0);
      for (int jj = 0; jj <= i; ++jj) acc = zfma(zconj(Tl[jj][i]), Ws[jj][col], acc);
      w2[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) Ws[i0 + u][col] = w2[u];
  }
  __syncthreads();
  // A_b -= V W, row block by row block (Gauss: q1 = sum vr wr, q2 = sum vi wi,
  // q3 = sum (vr + vi)(wr + wi), V W = (q1 - q2) + i (q3 - q1 - q2)); accumulator register
  // t of lane (j, k) is row r0 + k + 4 t, the row whose entry the lane holds in ar[rb][t]
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int r0 = rbase + rb * 16;
    if (r0 < nrb) {
      d4 q1 = d4{0, 0, 0, 0}, q2 = d4{0, 0, 0, 0}, q3 = d4{0, 0, 0, 0};
      const bool rok = r0 + j < nrb;
#pragma unroll
      for (int kk = 0; kk < PMX_QR_NB; kk += 4) {
        const C a = rok ? V[r0 + j + (int64_t)(kk + k) * PMX_TS_BR] : cmk<R>(0, 0);
        const C bb = Ws[kk + k][cl];
        q1 = mfma16(a.re, bb.re, q1);
        q2 = mfma16(a.im, bb.im, q2);
        q3 = mfma16(a.re + a.im, bb.re + bb.im, q3);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int pr = rows[r0 + 4 * t + k];
        if (pr >= 0 && cok) A[pr + coff] = zsub(ar[rb][t], cmk<R>(q1[t] - q2[t], q3[t] - q1[t] - q2[t]));
      }
    }
  }
}

#define TSU_ROWS 32
// FP32 form of the trailing update: the block's rows of A (up to PMX_TS_BR x 64, 64 complex
// values per thread) stay in registers between the two products, so A is read from memory
// once instead of twice; the product V W goes through LDS, and the updated slice is written
// down columns (32 consecutive rows per half wave) instead of one column per lane.
__global__ __launch_bounds__(256) void k_ts_update_f32(const QrDescT<float>* qrs, int j0, int L) {
  typedef float R;
  typedef cx<R> C;
  typedef typename AccT<R>::type V4;
  constexpr int NS = PMX_TS_BR / TSU_ROWS;
  const int gx = (int)gridDim.x, gy = (int)gridDim.y;
  const int lb = ts_xcd_run((int)(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z)), gx * gy * (int)gridDim.z);
  const int bx = lb % gx, by = (lb / gx) % gy, bz = lb / (gx * gy);
  const QrDescT<R> Q = qrs[bz];
  const int kmax = Q.kc;
  const int jb = min(PMX_QR_NB, kmax - j0);
  const int nc = Q.c - j0 - jb;
  if (jb <= 0 || nc <= 0) return;
  const int c0 = bx * 64;
  if (c0 >= nc) return;
  TsGeom g;
  ts_geom(Q.m, j0, jb, g);
  if (L >= g.nlev) return;
  const int b = by;
  if (b >= ts_sel(L, g.nb0, g.nb1, g.nb2, g.nb3)) return;
  const int nrb = min(PMX_TS_BR, ts_sel(L, g.mr0, g.mr1, g.mr2, g.mr3) - b * PMX_TS_BR);
  const int64_t wo = ts_sel64(L, g.wo0, g.wo1, g.wo2, g.wo3) + (int64_t)b * PMX_TS_BR * PMX_QR_NB;
  const auto V = gbl(Q.v) + wo;
  const auto Tw = gbl(Q.t) + wo;
  __shared__ C Vs[TSU_ROWS][PMX_QR_NB + 1];
  __shared__ C As[TSU_ROWS][64 + 1];
  __shared__ C Ws[PMX_QR_NB][64 + 1];
  __shared__ int rows[PMX_TS_BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const auto A = gbl(Q.a);
  const int64_t ld = Q.ld;
  const int ccol0 = j0 + jb + c0;
  for (int i = tid; i < PMX_TS_BR; i += 256) rows[i] = (i < nrb) ? ts_phys(b * PMX_TS_BR + i, L, jb, j0, g) : -1;
  const int rr = tid & (TSU_ROWS - 1);
  const int cc = tid >> 5;
  constexpr int RB = PMX_QR_NB / 16;
  V4 accR[RB], accI[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    accR[q] = V4{0, 0, 0, 0};
    accI[q] = V4{0, 0, 0, 0};
  }
  C ar[NS][8];   // thread's entries of A: slice sl, row rr, columns cc + 8 p
  __syncthreads();
  // W = V^H A_b
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int rb = sl * TSU_ROWS;
    if (rb < nrb) {
      const int pr = rows[rb + rr];
      const int prc = pr >= 0 ? pr : j0;
      C tv[PMX_QR_NB / 8];
#pragma unroll
      for (int pass = 0; pass < PMX_QR_NB / 8; ++pass)
        tv[pass] = V[rb + rr + (int64_t)(cc + 8 * pass) * PMX_TS_BR];
#pragma unroll
      for (int pass = 0; pass < 8; ++pass)
        ar[sl][pass] = A[prc + (int64_t)(ccol0 + min(cc + 8 * pass, nc - 1 - c0)) * ld];
#pragma unroll
      for (int pass = 0; pass < PMX_QR_NB / 8; ++pass)
        Vs[rr][cc + 8 * pass] = (rb + rr < nrb) ? tv[pass] : cmk<R>(0, 0);
#pragma unroll
      for (int pass = 0; pass < 8; ++pass)
        As[rr][cc + 8 * pass] = (pr >= 0 && c0 + cc + 8 * pass < nc) ? ar[sl][pass] : cmk<R>(0, 0);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TSU_ROWS; kk += 4) {
        const C bb = As[kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const C a = Vs[kk + (lane >> 4)][q * 16 + (lane & 15)];
          accR[q] = mfma16(a.re, bb.re, accR[q]);
          accR[q] = mfma16(a.im, bb.im, accR[q]);
          accI[q] = mfma16(a.re, bb.im, accI[q]);
          accI[q] = mfma16(-a.im, bb.re, accI[q]);
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < RB; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Ws[q * 16 + mfma_row<R>(lane, r)][wave * 16 + (lane & 15)] = cmk<R>(accR[q][r], accI[q][r]);
  // W <- T^H W, T upper triangular (row-major in the workspace), staged in the A slice's space
  C(*Tl)[PMX_QR_NB + 1] = reinterpret_cast<C(*)[PMX_QR_NB + 1]>(&As[0][0]);
  for (int e = tid; e < PMX_QR_NB * PMX_QR_NB; e += 256) Tl[e / PMX_QR_NB][e % PMX_QR_NB] = Tw[e];
  __syncthreads();
  {
    constexpr int PER = PMX_QR_NB * 64 / 256;
    const int col = tid & 63, i0 = (tid >> 6) * PER;
    C w2[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = i0 + u;
      C acc = cmk<R>(0, 0);
      for (int j = 0; j <= i; ++j) acc = zfma(zconj(Tl[j][i]), Ws[j][col], acc);
      w2[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) Ws[i0 + u][col] = w2[u];
  }
  __syncthreads();
  // A_b -= V W, slice by slice: the 32 x 64 product on MFMA (2 x 4 blocks of 16x16, two per
  // wave) into LDS, then subtracted from the registers and stored
  const int rbk = wave & 1;
  const int cbk0 = (wave >> 1) * 2;
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int rb = sl * TSU_ROWS;
    if (rb < nrb) {
      {
        C tv[PMX_QR_NB / 8];
#pragma unroll
        for (int pass = 0; pass < PMX_QR_NB / 8; ++pass)
          tv[pass] = V[rb + rr + (int64_t)(cc + 8 * pass) * PMX_TS_BR];
#pragma unroll
        for (int pass = 0; pass < PMX_QR_NB / 8; ++pass)
          Vs[rr][cc + 8 * pass] = (rb + rr < nrb) ? tv[pass] : cmk<R>(0, 0);
      }
      __syncthreads();
      V4 dR[2] = {V4{0, 0, 0, 0}, V4{0, 0, 0, 0}}, dI[2] = {V4{0, 0, 0, 0}, V4{0, 0, 0, 0}};
#pragma unroll
      for (int kk = 0; kk < PMX_QR_NB; kk += 4) {
        const C a = Vs[rbk * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const C bb = Ws[kk + (lane >> 4)][(cbk0 + q) * 16 + (lane & 15)];
          dR[q] = mfma16(a.re, bb.re, dR[q]);
          dR[q] = mfma16(-a.im, bb.im, dR[q]);
          dI[q] = mfma16(a.re, bb.im, dI[q]);
          dI[q] = mfma16(a.im, bb.re, dI[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          As[rbk * 16 + mfma_row<R>(lane, r)][(cbk0 + q) * 16 + (lane & 15)] = cmk<R>(dR[q][r], dI[q][r]);
      __syncthreads();
      const int pr = rows[rb + rr];
      if (pr >= 0) {
#pragma unroll
        for (int pass = 0; pass < 8; ++pass) {
          const int col = cc + 8 * pass;
          if (c0 + col < nc) A[pr + (int64_t)(ccol0 + col) * ld] = zsub(ar[sl][pass], As[rr][col]);
        }
      }
      __syncthreads();
    }
  }
}

template <class R>
__global__ void k_copy_r(const QrDescT<R>* qrs) {
  const QrDescT<R> Q = qrs[blockIdx.y];
  const int mb = Q.kc;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mb * Q.c) return;
  const int r = (int)(e % mb), c = (int)(e / mb);
  Q.r[e] = (r <= c) ? Q.a[r + c * Q.ld] : cmk<R>(0, 0);
}

int64_t la_geqrf_workspace(int m) {
  // V blocks (and, in the second workspace, T blocks) of every tree level for m rows
  int64_t tot = 0;
  int mr = m;
  for (int L = 0; L < PMX_TS_MAXLEV; ++L) {
    int nb = (mr + PMX_TS_BR - 1) / PMX_TS_BR;
    tot += (int64_t)std::max(nb, 1) * PMX_TS_BR * PMX_QR_NB;
    if (nb <= 1) break;
    mr = nb * PMX_QR_NB;
  }
  return tot;
}

template <class R>
void la_geqrf_r(const QrDescT<R>* d_qr, int batch, int max_m, int max_c, hipStream_t s) {
  if (batch <= 0 || max_m <= 0 || max_c <= 0) return;
  // four tree levels cover PMX_TS_BR * (PMX_TS_BR / PMX_QR_NB)^3 rows
  const int64_t cap = (int64_t)PMX_TS_BR * (PMX_TS_BR / PMX_QR_NB) * (PMX_TS_BR / PMX_QR_NB) * (PMX_TS_BR / PMX_QR_NB);
  if (max_m > cap) return;
  const int kmax = min(max_m, max_c);
  // threads per leaf block: built-in 512, or the launch-parameter table's choice for the
  // shape of this call
  const int v = tune_choice(TK_TS_LEAF, (int)sizeof(R), tune_bucket_size(max_m), tune_bucket_batch(batch),
                            tune_bucket_size(max_c), 512, max_m, batch, max_c);
  for (int j0 = 0; j0 < kmax; j0 += PMX_QR_NB) {
    int mr = max_m - j0;
    const int nc = max_c - j0 - 1;
    for (int L = 0; L < PMX_TS_MAXLEV; ++L) {
      const int nb = (mr + PMX_TS_BR - 1) / PMX_TS_BR;
      {
        KScope ks(PK_TS_LEAF, s);
        if (v == 1024 && sizeof(R) == 4)   // FP64 spills at 1024 threads
          PMX_LAUNCH((k_ts_leaf<float, 1024>), dim3(nb, batch), dim3(1024), 0, s,
                             (const QrDescT<float>*)d_qr, j0, L);
        else if (v == 256)
          PMX_LAUNCH((k_ts_leaf<R, 256>), dim3(nb, batch), dim3(256), 0, s, d_qr, j0, L);
        else
          PMX_LAUNCH((k_ts_leaf<R, 512>), dim3(nb, batch), dim3(512), 0, s, d_qr, j0, L);
      }
      if (nc > 0) {
        KScope ks(PK_TS_UPDATE, s);
        if constexpr (sizeof(R) == 4)
          PMX_LAUNCH(k_ts_update_f32, dim3((nc + 63) / 64, nb, batch), dim3(256), 0, s,
                             reinterpret_cast<const QrDescT<float>*>(d_qr), j0, L);
        else
          PMX_LAUNCH(k_ts_update_f64<2>, dim3((nc + 31) / 32, nb, batch), dim3(256), 0, s,
                     reinterpret_cast<const QrDescT<double>*>(d_qr), j0, L);
      }
      if (nb <= 1) break;
      mr = nb * PMX_QR_NB;
    }
  }
  int64_t tot = (int64_t)kmax * max_c;
  PMX_LAUNCH(k_copy_r<R>, dim3((unsigned)((tot + 255) / 256), batch), dim3(256), 0, s, d_qr);
}

// ---------------------------------------------------------------------------------
// column pivoted QR with threshold rank
#define CP_NT 512
// the reflector in dynamic LDS (declared once as double for every real type)
extern __shared__ double cp_lds[];

// Householder vector of the pivot column: beta = -sign(alpha) |x|, tau = 1 + |alpha|/|x|,
// entries below the diagonal scaled by 1/(alpha - beta).
template <class R>
__device__ inline void cp_reflector(cx<R> alpha, double xn, cx<R>& beta, double& tau, cx<R>& scale) {
  const double aa = sqrt((double)alpha.re * alpha.re + (double)alpha.im * alpha.im);
  const cx<R> sg = aa > 0 ? zscale(alpha, 1.0 / aa) : cmk<R>(1, 0);
  beta = zscale(sg, -xn);
  tau = 1.0 + aa / xn;
  // 1/(alpha - beta) = conj(sg) / (aa + xn)
  scale = zscale(zconj(sg), 1.0 / (aa + xn));
}

// Relative squared norm below which a downdated column norm is recomputed: the downdate
// loses the digits of the ratio, so at a squared ratio under the square root of the unit
// roundoff of the data it no longer carries any (the criterion of LAPACK's xGEQP3).
template <class R>
__device__ constexpr double cp_recompute_ratio();
template <>
__device__ constexpr double cp_recompute_ratio<double>() {
  return 1.5e-8;
}
template <>
__device__ constexpr double cp_recompute_ratio<float>() {
  return 2.5e-4;
}

// apply the current reflector (vs, rows j..mb-1) to column l and downdate its norm;
// one wave per column, lane 0 ends with row j
template <class R>
__device__ inline void cp_apply_column(cx<R>* col_, const cx<R>* vs, int j, int mb, double tau, double* nrm_,
                                       int c, int l, int lane, const double* extra_) {
  typedef cx<R> C;
  const auto col = gbl(col_);
  const auto nrm = gbl(nrm_);
  const auto extra = gbl(extra_);
  R wr = 0, wi = 0;
  for (int r = j + lane; r < mb; r += 64) {
    const C t = zcmul(vs[r - j], col[r]);
    wr += t.re;
    wi += t.im;
  }
  wr = wave_sum(wr);
  wi = wave_sum(wi);
  const C w = zscale(cmk<R>(wr, wi), tau);
  double tail = 0;
  C first = cmk<R>(0, 0);
  for (int r = j + lane; r < mb; r += 64) {
    const C nv = zfms(col[r], vs[r - j], w);
    col[r] = nv;
    if (r > j) tail += (double)nv.re * nv.re + (double)nv.im * nv.im;
    else first = nv;
  }
  // norm downdating with recomputation on cancellation
  const double fr = readlane((double)first.re, 0), fi = readlane((double)first.im, 0);
  const double nw2 = nrm[l] - (fr * fr + fi * fi);
  if (nw2 <= cp_recompute_ratio<R>() * nrm[c + l]) {
    tail = wave_sum(tail);
    if (extra) tail += extra[l];
    if (lane == 0) {
      nrm[l] = tail;
      nrm[c + l] = tail;
    }
  } else if (lane == 0) {
    nrm[l] = nw2;
  }
}

template <class R>
__global__ __launch_bounds__(CP_NT) void k_cpqr(const CpqrDescT<R>* cps, double tol, const int* kmin, int init) {
  typedef cx<R> C;
  const CpqrDescT<R> Cd = cps[blockIdx.x];
  if (Cd.c <= 0) return;
  C* vs = reinterpret_cast<C*>(cp_lds);  // [mb]
  __shared__ double redv[CP_NT / 64];
  __shared__ int redi[CP_NT / 64];
  __shared__ double sh_tau;
  __shared__ int sh_stop;
  __shared__ C sh_scale;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = CP_NT / 64;
  const auto B = gbl(Cd.b);
  const int mb = Cd.mb, c = Cd.c;
  const int64_t ld = mb;
  const int cpiv = Cd.cpiv;
  const int kmax = min(min(mb, c), cpiv);
  const auto nrm = gbl(Cd.nrm);
  if (init) {
    for (int l = wave; l < c; l += nw) {
      double p = 0;
      for (int r = lane; r < mb; r += 64) {
        const C x = B[r + l * ld];
        p += (double)x.re * x.re + (double)x.im * x.im;
      }
      p = wave_sum(p);
      if (lane == 0) {
        if (Cd.extra) p += Cd.extra[l];
        nrm[l] = p;
        nrm[c + l] = p;
        Cd.piv[l] = l;
      }
    }
    __syncthreads();
    __threadfence_block();
    // restricted pivoting: the threshold refers to the largest column of the whole matrix
    double big = 0;
    if (cpiv < c) {
      int bi = -1;
      for (int l = tid; l < c; l += CP_NT) argmax_pair(big, bi, nrm[l], l);
      block_argmax<CP_NT>(big, bi, redv, redi, &big);
    }
    if (tid == 0) {
      Cd.state[0] = 0;
      Cd.state[1] = -1;
      Cd.state[2] = 0;
      *Cd.r11 = sqrt(big);
    }
    __syncthreads();
    __threadfence_block();
  }
  int j = Cd.state[0];
  const int target = (tol > 0.0) ? kmax : min(kmax, kmin ? kmin[blockIdx.x] : kmax);
  double r11 = *Cd.r11;
  while (j < target) {
    double best = -1.0;
    int bi = -1;
    for (int l = j + tid; l < cpiv; l += CP_NT) argmax_pair(best, bi, nrm[l], l);
    const int p = block_argmax<CP_NT>(best, bi, redv, redi, nullptr);
    if (p != j) {
      for (int r = tid; r < mb; r += CP_NT) {
        C t = B[r + j * ld];
        B[r + j * ld] = B[r + p * ld];
        B[r + p * ld] = t;
      }
    }
    __syncthreads();
    if (tid == 0 && p != j) {
      int ti = Cd.piv[j];
      Cd.piv[j] = Cd.piv[p];
      Cd.piv[p] = ti;
      double t0 = nrm[j];
      nrm[j] = nrm[p];
      nrm[p] = t0;
      t0 = nrm[c + j];
      nrm[c + j] = nrm[c + p];
      nrm[c + p] = t0;
    }
    double part = 0;
    for (int r = j + tid; r < mb; r += CP_NT) {
      const C x = B[r + j * ld];
      part += (double)x.re * x.re + (double)x.im * x.im;
    }
    const double xn = sqrt(block_sum<CP_NT>(part, redv));
    if (tid == 0) {
      if (j == 0 && cpiv >= c) r11 = xn;
      int stop = 0;
      if (!(xn > 0.0)) stop = 1;   // zero or NaN
      else if (tol > 0.0 && xn <= tol * r11) stop = 1;
      sh_stop = stop;
      if (!stop) {
        C beta, scale;
        double tau;
        cp_reflector<R>(B[j + j * ld], xn, beta, tau, scale);
        sh_tau = tau;
        sh_scale = scale;
        B[j + j * ld] = beta;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    const C scale = sh_scale;
    for (int r = j + tid; r < mb; r += CP_NT) {
      C v = (r == j) ? cmk<R>(1, 0) : zmul(B[r + j * ld], scale);
      vs[r - j] = v;
      if (r > j) B[r + j * ld] = cmk<R>(0, 0);
    }
    __syncthreads();
    const double tau = sh_tau;
    for (int l = j + 1 + wave; l < c; l += nw)
      cp_apply_column<R>(B + l * ld, vs, j, mb, tau, nrm, c, l, lane, Cd.extra);
    __syncthreads();
    ++j;
  }
  if (tid == 0) {
    Cd.state[0] = j;
    if (tol > 0.0) Cd.state[1] = j;
    *Cd.r11 = r11;
  }
}

// Multi-workgroup variant for large matrices: per step one launch selects the pivot,
// swaps it in and forms the reflector (one workgroup per matrix), a second applies the
// reflector to the trailing columns (16 columns per workgroup, one wave per column) and
// downdates their norms.  state[2] marks a finished matrix; finished matrices bump *ndone.
template <class R>
__global__ __launch_bounds__(256) void k_cpqr_init(const CpqrDescT<R>* cps, int init) {
  const CpqrDescT<R> Cd = cps[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l = blockIdx.x * 4 + wave;
  if (blockIdx.x == 0 && threadIdx.x == 0 && Cd.c > 0) {
    if (init) {
      Cd.state[0] = 0;
      Cd.state[1] = -1;
      *Cd.r11 = 0.0;
    }
    Cd.state[2] = 0;
  }
  if (!init || l >= Cd.c) return;
  double p = 0;
  for (int r = lane; r < Cd.mb; r += 64) {
    const cx<R> x = Cd.b[r + (int64_t)l * Cd.mb];
    p += (double)x.re * x.re + (double)x.im * x.im;
  }
  p = wave_sum(p);
  if (lane == 0) {
    if (Cd.extra) p += Cd.extra[l];
    Cd.nrm[l] = p;
    Cd.nrm[Cd.c + l] = p;
    Cd.piv[l] = l;
  }
}

// One column step of matrix b's CPQR (one workgroup of 256 threads): pivot, exchange,
// reflector.  Every exit is taken by the whole workgroup.
template <class R>
__device__ void cpqr_pivot_step(const CpqrDescT<R>& Cd, int b, double tol, const int* kmin, int* ndone) {
  typedef cx<R> C;
  if (Cd.c <= 0 || Cd.state[2]) return;
  __shared__ double redv[4];
  __shared__ int redi[4];
  __shared__ int sh_stop;
  __shared__ C sh_scale;
  const int tid = threadIdx.x;
  const auto B = gbl(Cd.b);
  const int mb = Cd.mb, c = Cd.c;
  const int64_t ld = mb;
  const int cpiv = Cd.cpiv;
  const int kmax = min(min(mb, c), cpiv);
  const int target = (tol > 0.0) ? kmax : min(kmax, kmin ? kmin[b] : kmax);
  const int j = Cd.state[0];
  if (j >= target) {
    __syncthreads();   // every thread has read the state before it changes
    if (tid == 0) {
      Cd.state[2] = 1;
      if (tol > 0.0) Cd.state[1] = j;
      atomicAdd(ndone, 1);
    }
    return;
  }
  const auto nrm = gbl(Cd.nrm);
  double big = 0;
  if (j == 0 && cpiv < c) {
    // restricted pivoting: the threshold refers to the largest column of the whole matrix
    int bb = -1;
    for (int l = tid; l < c; l += 256) argmax_pair(big, bb, nrm[l], l);
    block_argmax<256>(big, bb, redv, redi, &big);
  }
  double best = -1.0;
  int bi = -1;
  for (int l = j + tid; l < cpiv; l += 256) argmax_pair(best, bi, nrm[l], l);
  const int p = block_argmax<256>(best, bi, redv, redi, nullptr);
  if (p != j) {
    for (int r = tid; r < mb; r += 256) {
      C t = B[r + j * ld];
      B[r + j * ld] = B[r + p * ld];
      B[r + p * ld] = t;
    }
  }
  __syncthreads();
  if (tid == 0 && p != j) {
    int ti = Cd.piv[j];
    Cd.piv[j] = Cd.piv[p];
    Cd.piv[p] = ti;
    double t0 = nrm[j];
    nrm[j] = nrm[p];
    nrm[p] = t0;
    t0 = nrm[c + j];
    nrm[c + j] = nrm[c + p];
    nrm[c + p] = t0;
  }
  double part = 0;
  for (int r = j + tid; r < mb; r += 256) {
    const C x = B[r + j * ld];
    part += (double)x.re * x.re + (double)x.im * x.im;
  }
  const double xn = sqrt(block_sum<256>(part, redv));
  if (tid == 0) {
    const double first = (cpiv < c) ? sqrt(big) : xn;
    double r11 = (j == 0) ? first : *Cd.r11;
    if (j == 0) *Cd.r11 = first;
    int stop = 0;
    if (!(xn > 0.0)) stop = 1;   // zero or NaN
    else if (tol > 0.0 && xn <= tol * r11) stop = 1;
    sh_stop = stop;
    if (stop) {
      Cd.state[2] = 1;
      if (tol > 0.0) Cd.state[1] = j;
      atomicAdd(ndone, 1);
    } else {
      C beta, scale;
      double tau;
      cp_reflector<R>(B[j + j * ld], xn, beta, tau, scale);
      *Cd.tau = tau;
      sh_scale = scale;
      B[j + j * ld] = beta;
    }
  }
  __syncthreads();
  if (sh_stop) return;
  const C scale = sh_scale;
  for (int r = j + tid; r < mb; r += 256) {
    if (r == j) {
      Cd.v[0] = cmk<R>(1, 0);
    } else {
      Cd.v[r - j] = zmul(B[r + j * ld], scale);
      B[r + j * ld] = cmk<R>(0, 0);
    }
  }
  if (tid == 0) {
    Cd.state[3] = j;
    Cd.state[0] = j + 1;
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_cpqr_pivot(const CpqrDescT<R>* cps, double tol, const int* kmin,
                                                    int* ndone) {
  const CpqrDescT<R> Cd = cps[blockIdx.x];
  cpqr_pivot_step<R>(Cd, blockIdx.x, tol, kmin, ndone);
}

// columns per workgroup of the update: one per wave, so that a column's dot product, update
// and norm are the whole chain of a wave
#define CPU_COLS 4
// The update of column group g of one matrix after its pivot step.
template <class R>
__device__ void cpqr_update_step(const CpqrDescT<R>& Cd, int g) {
  typedef cx<R> C;
  if (Cd.c <= 0 || Cd.state[2]) return;
  const int j = Cd.state[3];
  const int l0 = g * CPU_COLS;
  if (l0 + CPU_COLS <= j + 1 || l0 >= Cd.c) return;
  C* vs = reinterpret_cast<C*>(cp_lds);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mb = Cd.mb, c = Cd.c;
  const int64_t ld = mb;
  for (int r = j + tid; r < mb; r += 256) vs[r - j] = gbl(Cd.v)[r - j];
  __syncthreads();
  const double tau = *Cd.tau;
  const int l = l0 + wave;   // one column per wave
  if (l > j && l < c) cp_apply_column<R>(Cd.b + (int64_t)l * ld, vs, j, mb, tau, Cd.nrm, c, l, lane, Cd.extra);
}

template <class R>
__global__ __launch_bounds__(256) void k_cpqr_update(const CpqrDescT<R>* cps) {
  const CpqrDescT<R> Cd = cps[blockIdx.y];
  cpqr_update_step<R>(Cd, blockIdx.x);
}

// The whole column loop in one cooperative launch: every workgroup of the grid (sized to
// be resident at once) takes the pivot steps of the matrices b = its index + grid * i, a
// grid barrier, the update groups u = its index + grid * i of all matrices, a grid barrier,
// and so on until every matrix is done or max_c + 1 steps have run (the bound of the
// host-driven loop), so every workgroup leaves after the same number of barriers.  The
// stop test reads the done count after a barrier and before any later increment, so all
// workgroups see one value.  Device-scope fences order the steps' writes across XCDs.
// A choice of the launch tables (variant 2), not the built-in rule: each grid barrier
// across the resident grid costs about 100 us against about 15 us for the two launches
// of a host-driven step, so the tuned 1M-unknown factorisation took 1.29 s instead of
// 0.55 s with it.
template <class R>
__global__ __launch_bounds__(256) void k_cpqr_persist(const CpqrDescT<R>* cps, int batch, int ucols, int steps,
                                                      double tol, const int* kmin, int* ndone) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int G = gridDim.x;
  for (int it = 0; it < steps; ++it) {
    for (int b = blockIdx.x; b < batch; b += G) {
      const CpqrDescT<R> Cd = cps[b];
      cpqr_pivot_step<R>(Cd, b, tol, kmin, ndone);
      __syncthreads();
    }
    __threadfence();
    grid.sync();
    if (__hip_atomic_load(ndone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= batch) break;
    for (int u = blockIdx.x; u < batch * ucols; u += G) {
      const CpqrDescT<R> Cd = cps[u / ucols];
      cpqr_update_step<R>(Cd, u % ucols);
      __syncthreads();
    }
    __threadfence();
    grid.sync();
  }
}

template <class R>
hipError_t la_cpqr(const CpqrDescT<R>* d_cp, int batch, int max_c, double tol, const int* d_kmin, int init,
                   int* d_work, hipStream_t s) {
  if (batch <= 0 || max_c <= 0) return hipSuccess;
  size_t shm = (size_t)max_c * sizeof(cx<R>) + 16;
  if (shm > 64 * 1024) {
    (void)hipFuncSetAttribute((const void*)k_cpqr<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipFuncSetAttribute((const void*)k_cpqr_update<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  }
  const int mode = tune_choice(TK_CPQR, (int)sizeof(R), tune_bucket_size(max_c), tune_bucket_batch(batch), 0,
                               max_c < PMX_CPQR_MULTI_MIN ? 0 : 1, max_c, batch, 0);
  if (mode == 0) {
    KScope ks(PK_CPQR, s);
    PMX_LAUNCH(k_cpqr<R>, dim3(batch), dim3(CP_NT), shm, s, d_cp, tol, d_kmin, init);
    return hipSuccess;
  }
  (void)hipMemsetAsync(d_work, 0, sizeof(int), s);
  PMX_LAUNCH(k_cpqr_init<R>, dim3((max_c + 3) / 4, batch), dim3(256), 0, s, d_cp, init);
  const int ucols = (max_c + CPU_COLS - 1) / CPU_COLS;
  if (mode == 2) {
    // one cooperative launch: as many workgroups as can be resident at once (at most one
    // per unit of work)
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (shm > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)k_cpqr_persist<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_cpqr_persist<R>, 256, shm);
    const int grid = std::max(1, std::min(per * ncu, batch * ucols));
    int steps = max_c + 1, bt = batch, uc = ucols;
    const int* km = d_kmin;
    int* nd = d_work;
    void* args[] = {(void*)&d_cp, (void*)&bt, (void*)&uc, (void*)&steps, (void*)&tol, (void*)&km, (void*)&nd};
    KScope ks(PK_CPQR_UPDATE, s);
    pmx_count_launch();
    const hipError_t e = hipLaunchCooperativeKernel((const void*)k_cpqr_persist<R>, dim3(grid), dim3(256), args,
                                                    (unsigned)shm, s);
    if (e == hipSuccess) return hipSuccess;
    (void)hipGetLastError();   // not launchable as one resident grid: the step-by-step loop below
  }
  // Progress polls, one chunk behind: after every 16 columns the done count is copied to
  // pinned host memory behind an event, and the host waits for the previous chunk's copy
  // only, so that the stream always holds the current chunk while the host checks (a
  // matrix that is done makes the later steps return at once).
  static thread_local int* h_nd = nullptr;
  if (!h_nd) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) return hipErrorOutOfMemory;
    h_nd = (int*)p;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t err = hipSuccess;
  for (int k = 0; k < 2 && err == hipSuccess; ++k) err = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
  int pending = -1, chunk = 0;
  for (int it = 0; it <= max_c && err == hipSuccess; ++it) {
    PMX_LAUNCH(k_cpqr_pivot<R>, dim3(batch), dim3(256), 0, s, d_cp, tol, d_kmin, d_work);
    {
      KScope ks(PK_CPQR_UPDATE, s);
      PMX_LAUNCH(k_cpqr_update<R>, dim3(ucols, batch), dim3(256), shm, s, d_cp);
    }
    if ((it & 15) == 15) {
      const int slot = chunk & 1;
      err = hipMemcpyAsync(&h_nd[slot], d_work, sizeof(int), hipMemcpyDeviceToHost, s);
      if (err == hipSuccess) err = hipEventRecord(ev[slot], s);
      if (err == hipSuccess && pending >= 0) {
        pmx_count_sync();
        err = hipEventSynchronize(ev[pending]);
        if (err == hipSuccess && h_nd[pending] >= batch) break;
      }
      pending = slot;
      ++chunk;
    }
  }
  // no copy into the host buffer may still be in flight when the call returns
  if (chunk > 0) {
    const hipError_t e = hipEventSynchronize(ev[(chunk - 1) & 1]);
    if (err == hipSuccess) err = e;
  }
  for (int k = 0; k < 2; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  return err;
}

// T = R11^-1 R12 in place
template <class R>
struct FTTrsm {
  const CpqrDescT<R>* d;
  const int* ks;
  int j0;
  __device__ bool operator()(int b, TrsmArgs<R>& a) const {
    CpqrDescT<R> C = d[b];
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

template <class R>
struct FTUpd {
  const CpqrDescT<R>* d;
  const int* ks;
  int j0;
  __device__ bool operator()(int b, GemmArgsT<R>& g) const {
    CpqrDescT<R> C = d[b];
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

template <class R>
void la_cpqr_tsolve(const CpqrDescT<R>* d_cp, const int* d_k, int batch, int max_k, int max_c, hipStream_t s) {
  if (batch <= 0 || max_k <= 0 || max_c <= 0) return;
  const int nblk = (max_k + PMX_LU_NB - 1) / PMX_LU_NB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    int j0 = bk * PMX_LU_NB;
    launch_trsm_small<R, true, false>(FTTrsm<R>{d_cp, d_k, j0}, batch, max_c, s);
    if (j0 > 0)
      launch_zgemm<R, OP_N, OP_N>(FTUpd<R>{d_cp, d_k, j0}, batch, j0, max_c, cmk<R>(-1, 0), cmk<R>(1, 0), s);
  }
}

// squared norms of rows kc.. of each column of a truncated QR
template <class R>
__global__ __launch_bounds__(256) void k_qr_tail_norms(const QrDescT<R>* qrs, double* const* outs) {
  const QrDescT<R> Q = qrs[blockIdx.y];
  double* out = outs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l = blockIdx.x * 4 + wave;
  if (l >= Q.c || !out) return;
  double p = 0;
  if (l >= Q.kc)
    for (int r = Q.kc + lane; r < Q.m; r += 64) {
      const cx<R> x = Q.a[r + (int64_t)l * Q.ld];
      p += (double)x.re * x.re + (double)x.im * x.im;
    }
  p = wave_sum(p);
  if (lane == 0) out[l] = p;
}

template <class R>
void la_qr_tail_norms(const QrDescT<R>* d_qr, double* const* d_out, int batch, int max_c, hipStream_t s) {
  if (batch <= 0 || max_c <= 0) return;
  PMX_LAUNCH(k_qr_tail_norms<R>, dim3((max_c + 3) / 4, batch), dim3(256), 0, s, d_qr, d_out);
}

template <class R>
__global__ __launch_bounds__(256) void k_cpqr_judge(const CpqrDescT<R>* cps, const int* ks, double tol, int* accept) {
  const CpqrDescT<R> Cd = cps[blockIdx.x];
  __shared__ double redv[4];
  __shared__ int redi[4];
  const int k = ks[blockIdx.x];
  double big = 0;
  int bi = -1;
  for (int l = k + (int)threadIdx.x; l < Cd.c; l += 256) argmax_pair(big, bi, Cd.nrm[l], l);
  block_argmax<256>(big, bi, redv, redi, &big);
  if (threadIdx.x == 0) {
    const double r11 = *Cd.r11;
    accept[blockIdx.x] = (Cd.c > 0 && Cd.state[0] >= k && big <= tol * tol * r11 * r11) ? 1 : 0;
  }
}

template <class R>
void la_cpqr_judge(const CpqrDescT<R>* d_cp, const int* d_k, double tol, int* d_accept, int batch, hipStream_t s) {
  if (batch <= 0) return;
  PMX_LAUNCH(k_cpqr_judge<R>, dim3(batch), dim3(256), 0, s, d_cp, d_k, tol, d_accept);
}

// Algorithmic work of the QR kernels for one m x c matrix, mirroring the launch sequence,
// with z = 2 real_bytes bytes per complex entry.  Trailing update of an nrb x nc block by
// jb reflectors: bytes z (2 nrb nc + nrb jb + jb^2) (the block read and written once, V and
// T read once), flops 16 nrb nc jb + 4 jb^2 nc (the products with V and with T^H).  Leaf
// factorisation of an nrb x jb block: bytes z (2 nrb jb + nrb PMX_QR_NB + PMX_QR_NB^2)
// (panel read and written, V and T written), flops 8 nrb jb^2.
void la_geqrf_work(int m, int c, int kc, int real_bytes, double* upd_bytes, double* upd_flops, double* leaf_bytes,
                   double* leaf_flops) {
  const double z = 2.0 * real_bytes;
  const int kmax = std::min(kc, std::min(m, c));
  for (int j0 = 0; j0 < kmax; j0 += PMX_QR_NB) {
    const int jb = std::min(PMX_QR_NB, kmax - j0);
    const int nc = c - j0 - jb;
    int mr = m - j0;
    for (int L = 0; L < PMX_TS_MAXLEV; ++L) {
      const int nb = (mr + PMX_TS_BR - 1) / PMX_TS_BR;
      for (int b = 0; b < nb; ++b) {
        const double nrb = std::min(PMX_TS_BR, mr - b * PMX_TS_BR);
        *leaf_bytes += z * (2 * nrb * jb + nrb * PMX_QR_NB + PMX_QR_NB * PMX_QR_NB);
        *leaf_flops += 8.0 * nrb * jb * jb;
        if (nc > 0) {
          *upd_bytes += z * (2 * nrb * nc + nrb * jb + (double)jb * jb);
          *upd_flops += 16.0 * nrb * nc * jb + 4.0 * jb * jb * nc;
        }
      }
      if (nb <= 1) break;
      mr = nb * jb;
    }
  }
}

// Algorithmic work of the LU panels of one n x n factorisation: each panel of jb columns
// is read and written once (bytes 2 z (n - j0) jb, z = 2 real_bytes) and its column steps
// cost 8 (n - c - 1) (j0 + jb - c - 1) flops for the rank-one updates.
void la_getrf_work(int n, int real_bytes, double* bytes, double* flops) {
  const double z = 2.0 * real_bytes;
  for (int j0 = 0; j0 < n; j0 += PMX_LU_NB) {
    const int jb = std::min(PMX_LU_NB, n - j0);
    *bytes += 2.0 * z * (double)(n - j0) * jb;
    for (int c = j0; c < j0 + jb; ++c) *flops += 8.0 * (double)(n - c - 1) * (j0 + jb - c - 1);
  }
}

// explicit instantiations: complex FP64 and complex FP32
#define PMX_LA_INST(R)                                                                                       \
  template void la_zgemm_list<R>(int, int, const GemmArgsT<R>*, int, int, int, cx<R>, cx<R>, hipStream_t);  \
  template void la_getrf<R>(const LuDescT<R>*, int, int, int*, hipStream_t);                                 \
  template void la_lu_panel<R>(int, const LuDescT<R>*, int, int, int*, hipStream_t);                         \
  template void la_getrs<R>(const LuDescT<R>*, const MatT<R>*, int, int, int, hipStream_t);                  \
  template void la_getrs_small<R>(const LuDescT<R>*, const MatT<R>*, const MatT<R>*, int, int, int, hipStream_t); \
  template bool la_getrs_lds<R>(const LuDescT<R>*, const MatT<R>*, int, int, int, hipStream_t);                \
  template void la_geqrf_r<R>(const QrDescT<R>*, int, int, int, hipStream_t);                                \
  template hipError_t la_cpqr<R>(const CpqrDescT<R>*, int, int, double, const int*, int, int*, hipStream_t);       \
  template void la_cpqr_tsolve<R>(const CpqrDescT<R>*, const int*, int, int, int, hipStream_t);             \
  template void la_qr_tail_norms<R>(const QrDescT<R>*, double* const*, int, int, hipStream_t);              \
  template void la_cpqr_judge<R>(const CpqrDescT<R>*, const int*, double, int*, int, hipStream_t);
PMX_LA_INST(double)
PMX_LA_INST(float)
#undef PMX_LA_INST
