// Batched complex FP64 dense linear algebra on gfx950: descriptors and launchers.
// Every matrix is column major; a batch entry may be empty (size 0) and sizes may
// differ between entries.  All launchers are stream ordered and allocate nothing.
#pragma once
#include "pmx_common.h"

struct Mat {         // one column-major matrix view
  zd* p;
  int64_t ld;
  int m, n;
};

struct LuDesc {      // square matrix factored in place, P A = L U
  zd* a;
  int64_t ld;
  int n;
  int* ipiv;         // [n], 0-based row swapped with row i at step i
};

struct GemmArgs {
  int m, n, k;
  const zd* A;
  int64_t lda;
  const zd* B;
  int64_t ldb;
  zd* C;
  int64_t ldc;
};

struct QrDesc {      // tall matrix M (m x c), factored by Householder, R written to r (c x c)
  zd* a;
  int64_t ld;
  int m, c;
  zd* r;             // [min(m,c) x c], leading dimension min(m,c)
  zd* v;             // workspace: m x PMX_QR_NB explicit reflectors
  zd* t;             // workspace: m x PMX_QR_NB, the reflectors times T^H (compact WY)
  zd* w;             // workspace: PMX_QR_NB x c
};

struct CpqrDesc {    // column pivoted QR of b (mb x c, ld mb) in place
  zd* b;
  int mb, c;
  int* piv;          // [c] column permutation
  double* nrm;       // [2c] running squared norms and the reference squared norms
  int* state;        // [4]: next step, threshold rank (-1 while running), status, pad
  double* r11;       // |R_11|
};

#define PMX_LU_NB 32
#define PMX_QR_NB 16

enum { OP_N = 0, OP_T = 1, OP_C = 2 };

// C = alpha op(A) op(B) + beta C for a device list of GemmArgs.
void la_zgemm_list(int opa, int opb, const GemmArgs* d_list, int batch, int max_m, int max_n,
                   zd alpha, zd beta, hipStream_t s);
// In-place LU with partial pivoting. info[b] = first zero pivot (1-based) or 0.
void la_getrf(const LuDesc* d_lu, int batch, int max_n, int* d_info, hipStream_t s);
// Solve A X = B in place in B (n x nrhs per entry) using the LU of getrf.
void la_getrs(const LuDesc* d_lu, const Mat* d_b, int batch, int max_n, int max_nrhs, hipStream_t s);
// Householder QR of each M; writes R (upper, zero below) to QrDesc::r.
void la_geqrf_r(const QrDesc* d_qr, int batch, int max_m, int max_c, hipStream_t s);
// Column pivoted QR with threshold rank on each CpqrDesc (in place).
// Runs steps until |R_jj| <= tol |R_11| (phase 1, tol > 0) or until the step count
// reaches kmin[b] (continuation, tol <= 0; kmin may be NULL).  A zero column stops both.
void la_cpqr(const CpqrDesc* d_cp, int batch, int max_c, double tol, const int* d_kmin,
             int init, hipStream_t s);
// T = R11^-1 R12 in place: R11 = b[0:k,0:k] upper, R12 = b[0:k,k:c]; k from d_k.
void la_cpqr_tsolve(const CpqrDesc* d_cp, const int* d_k, int batch, int max_k, int max_c,
                    hipStream_t s);
