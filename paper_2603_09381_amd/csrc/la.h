// Batched complex dense linear algebra on gfx950, templated on the real type R: double
// (complex FP64 on FP64 MFMA) and float (complex FP32 on FP32 MFMA).  Every matrix is
// column major; a batch entry may be empty (size 0) and sizes may differ between
// entries.  All launchers are stream ordered and allocate nothing.
#pragma once
#include "pmx_common.h"

template <class R>
struct MatT {        // one column-major matrix view
  cx<R>* p;
  int64_t ld;
  int m, n;
};

template <class R>
struct LuDescT {     // square matrix factored in place, P A = L U
  cx<R>* a;
  int64_t ld;
  int n;
  int* ipiv;         // [n], 0-based row swapped with row i at step i
  int* perm;         // [n] or NULL: row i of P b is row perm[i] of b (filled by getrf)
};

template <class R>
struct GemmArgsT {
  int m, n, k;
  const cx<R>* A;
  int64_t lda;
  const cx<R>* B;
  int64_t ldb;
  cx<R>* C;
  int64_t ldc;
};

template <class R>
struct QrDescT {     // tall matrix M (m x c), factored by Householder, R written to r
  cx<R>* a;
  int64_t ld;
  int m, c;
  cx<R>* r;          // [kc x c], leading dimension kc
  cx<R>* v;          // workspace: la_geqrf_workspace(m) reflector entries
  cx<R>* t;          // workspace: as v, the triangular factors T of the blocks (compact WY)
  int kc;            // columns triangularised (min(m, c) for a full QR; fewer: the reflectors
                     // of the first kc columns are applied to all others, rows kc.. of
                     // the remaining columns keep their component orthogonal to the first kc)
};

// Column pivoted QR of b (mb x c, ld mb) in place.  Column norms, |R_11| and the pivot
// decisions are FP64 for both real types.
template <class R>
struct CpqrDescT {
  cx<R>* b;
  int mb, c;
  int* piv;          // [c] column permutation
  double* nrm;       // [2c] running squared norms and the reference squared norms
  int* state;        // [4]: next step, threshold rank (-1 while running), done flag, current step
  double* r11;       // |R_11|
  cx<R>* v;          // [mb] current reflector (multi-workgroup variant)
  double* tau;       // current reflector coefficient (multi-workgroup variant)
  int cpiv;          // pivots are chosen among the first cpiv columns only (c: all)
  const double* extra;  // [c] or NULL: squared norm each column has outside b (added to its
                        // norms; with cpiv < c, |R_11| is the largest initial column norm)
};

typedef MatT<double> Mat;
typedef LuDescT<double> LuDesc;
typedef GemmArgsT<double> GemmArgs;
typedef QrDescT<double> QrDesc;
typedef CpqrDescT<double> CpqrDesc;

#define PMX_LU_NB 32
#define PMX_QR_NB 32
#define PMX_TS_MAXLEV 4

enum { OP_N = 0, OP_T = 1, OP_C = 2 };

// C = alpha op(A) op(B) + beta C for a device list of GemmArgs.
template <class R>
void la_zgemm_list(int opa, int opb, const GemmArgsT<R>* d_list, int batch, int max_m, int max_n,
                   cx<R> alpha, cx<R> beta, hipStream_t s);
// C = A B (FP64) for a device list, as la_zgemm_list, under a kernel name of its own
// (k_zgemm...<FApplyList>) so that profiles count the operator apply's self-block products
// apart from the solver's FP64 products.
void la_zgemm_apply_list(const GemmArgsT<double>* d_list, int batch, int max_m, int max_n, hipStream_t s);
// algorithmic bytes and flops of the LU panels of one n x n factorisation; real_bytes is
// sizeof(R)
void la_getrf_work(int n, int real_bytes, double* bytes, double* flops);
// In-place LU with partial pivoting. info[b] = first zero pivot (1-based) or 0.
template <class R>
void la_getrf(const LuDescT<R>* d_lu, int batch, int max_n, int* d_info, hipStream_t s);
// One panel step [j0, j0 + PMX_LU_NB) of the LU of every matrix with a given kernel:
// 0 registers (256 threads x 1 row, <= 256 panel rows), 1 registers (256 x 2, <= 512),
// 2 registers (512 x 2, <= 1024, FP32 only), 3 global memory (any size); registers with
// the column loop unrolled: 4 (256 x 1, <= 256), 6 (512 x 1, <= 512), 8 (1024 x 1,
// <= 1024, FP32 only).
template <class R>
void la_lu_panel(int variant, const LuDescT<R>* d_lu, int batch, int j0, int* d_info, hipStream_t s);
// Solve A X = B in place in B (n x nrhs per entry) using the LU of getrf.
template <class R>
void la_getrs(const LuDescT<R>* d_lu, const MatT<R>* d_b, int batch, int max_n, int max_nrhs, hipStream_t s);
// The same for few right-hand sides (max_nrhs <= PMX_GETRS_SMALL_MAX): one fused launch, a
// workgroup per matrix and group of right-hand sides running the permutation and both
// substitutions; needs LuDesc::perm and a workspace per entry (w[b].p, n x nrhs, ld >= n).
#define PMX_GETRS_SMALL_MAX 64
// The same with each workgroup's solution block (max_n x 4 right-hand sides) in LDS, any
// number of right-hand sides (4 per workgroup); returns false, launching nothing, when the
// block exceeds 128 KiB.
template <class R>
bool la_getrs_lds(const LuDescT<R>* d_lu, const MatT<R>* d_b, int batch, int max_n, int max_nrhs, hipStream_t s);
// LDS bytes la_getrs_lds needs for max_n rows
inline size_t la_getrs_lds_bytes(int max_n, int real_bytes) { return (size_t)max_n * 4 * 2 * real_bytes; }
template <class R>
void la_getrs_small(const LuDescT<R>* d_lu, const MatT<R>* d_b, const MatT<R>* d_w, int batch, int max_n,
                    int max_nrhs, hipStream_t s);
// Householder QR of each M (destroyed); writes R (upper, zero below) to QrDesc::r.
int64_t la_geqrf_workspace(int m);
// algorithmic bytes and flops of the trailing updates and the leaf factorisations
void la_geqrf_work(int m, int c, int kc, int real_bytes, double* upd_bytes, double* upd_flops, double* leaf_bytes,
                   double* leaf_flops);
template <class R>
void la_geqrf_r(const QrDescT<R>* d_qr, int batch, int max_m, int max_c, hipStream_t s);
// Column pivoted QR with threshold rank on each CpqrDesc (in place).
// Runs steps until |R_jj| <= tol |R_11| (phase 1, tol > 0) or until the step count
// reaches kmin[b] (continuation, tol <= 0; kmin may be NULL).  A zero column stops both.
// Matrices with max_c >= PMX_CPQR_MULTI_MIN columns use the multi-workgroup variant, which
// needs d_work (one device int); every 16 steps it copies the done count to a pinned host
// buffer of the calling thread and waits for the count of the 16 steps before, so the
// stream never runs dry while the host checks (the call returns after its last copy has
// landed); a launch table
// may choose its persistent form instead (the whole loop in one cooperative launch, no
// host synchronisation).  Returns the first error of its progress polls (hipSuccess when
// there is none; launch errors stay with the stream as for every launcher).
#define PMX_CPQR_MULTI_MIN 256
template <class R>
hipError_t la_cpqr(const CpqrDescT<R>* d_cp, int batch, int max_c, double tol, const int* d_kmin, int init,
                   int* d_work, hipStream_t s);
// T = R11^-1 R12 in place: R11 = b[0:k,0:k] upper, R12 = b[0:k,k:c]; k from d_k.
template <class R>
void la_cpqr_tsolve(const CpqrDescT<R>* d_cp, const int* d_k, int batch, int max_k, int max_c, hipStream_t s);
// Squared norms of rows kc..m-1 of every column of each (truncated) QR: out[b] [c]
// (0 for the first kc columns).
template <class R>
void la_qr_tail_norms(const QrDescT<R>* d_qr, double* const* d_out, int batch, int max_c, hipStream_t s);
// Interpolation check after a CPQR stopped at k[b] columns: accept[b] = 1 when every
// remaining column (its downdated norm, outside b included) is at most tol |R_11|, and k[b]
// steps were taken.
template <class R>
void la_cpqr_judge(const CpqrDescT<R>* d_cp, const int* d_k, double tol, int* d_accept, int batch, hipStream_t s);
