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

struct QrDesc {      // tall matrix M (m x c), factored by Householder, R written to r
  zd* a;
  int64_t ld;
  int m, c;
  zd* r;             // [min(m,c) x c], leading dimension min(m,c)
  zd* v;             // workspace: la_geqrf_workspace(m) reflector entries
  zd* t;             // workspace: as v, the reflectors times T^H (compact WY)
};

struct CpqrDesc {    // column pivoted QR of b (mb x c, ld mb) in place
  zd* b;
  int mb, c;
  int* piv;          // [c] column permutation
  double* nrm;       // [2c] running squared norms and the reference squared norms
  int* state;        // [4]: next step, threshold rank (-1 while running), done flag, current step
  double* r11;       // |R_11|
  zd* v;             // [mb] current reflector (multi-workgroup variant)
  double* tau;       // current reflector coefficient (multi-workgroup variant)
};

#define PMX_LU_NB 32
#define PMX_QR_NB 32
#define PMX_TS_MAXLEV 4

enum { OP_N = 0, OP_T = 1, OP_C = 2 };

// C = alpha op(A) op(B) + beta C for a device list of GemmArgs.
void la_zgemm_list(int opa, int opb, const GemmArgs* d_list, int batch, int max_m, int max_n,
                   zd alpha, zd beta, hipStream_t s);
// algorithmic bytes and flops of the LU panels of one n x n factorisation
void la_getrf_work(int n, double* bytes, double* flops);
// In-place LU with partial pivoting. info[b] = first zero pivot (1-based) or 0.
void la_getrf(const LuDesc* d_lu, int batch, int max_n, int* d_info, hipStream_t s);
// Solve A X = B in place in B (n x nrhs per entry) using the LU of getrf.
void la_getrs(const LuDesc* d_lu, const Mat* d_b, int batch, int max_n, int max_nrhs, hipStream_t s);
// Householder QR of each M (destroyed); writes R (upper, zero below) to QrDesc::r.
int64_t la_geqrf_workspace(int m);
// algorithmic bytes and flops of the trailing updates and the leaf factorisations
void la_geqrf_work(int m, int c, double* upd_bytes, double* upd_flops, double* leaf_bytes, double* leaf_flops);
void la_geqrf_r(const QrDesc* d_qr, int batch, int max_m, int max_c, hipStream_t s);
// Matrices with max_c >= PMX_CPQR_MULTI_MIN columns use the multi-workgroup variant, which
// needs d_work (one device int) and synchronises the stream every 16 steps.
#define PMX_CPQR_MULTI_MIN 256
void la_cpqr(const CpqrDesc* d_cp, int batch, int max_c, double tol, const int* d_kmin,
             int init, int* d_work, hipStream_t s);
// T = R11^-1 R12 in place: R11 = b[0:k,0:k] upper, R12 = b[0:k,k:c]; k from d_k.
void la_cpqr_tsolve(const CpqrDesc* d_cp, const int* d_k, int batch, int max_k, int max_c,
                    hipStream_t s);
