// Kernel-matrix assembly, right-hand sides, gathers and the far field (FP64, gfx950).
#pragma once
#include "pmx_common.h"

// Node geometry (device, structure of arrays over all boundary nodes).
struct DevGeom {
  const double *x, *y, *nx, *ny, *w, *speed, *kappa;
  int n_nodes;
};

// Proxy points of one level (device).
struct DevProxy {
  const double *x, *y, *nx, *ny, *w;
};

// Material and wavenumber constants of the exterior medium.
struct ExtParams {
  double k;        // k+
  double eps;      // eps+
};

// A point code addresses a matrix row or column:
//   code >= 0 : boundary node code/2, type code&1
//   code <  0 : proxy point p = (-code-1)/2 of the current level, type (-code-1)&1
// Row types: 0 value equation, 1 normal-derivative equation.
// Column types: 0 density q (single layer), 1 density u (double layer).
__host__ __device__ inline int pmx_code_node(int node, int type) { return 2 * node + type; }
__host__ __device__ inline int pmx_code_proxy(int p, int type) { return -(2 * p + type) - 1; }

struct EntryMat {   // out[i + j ld] = entry(list a[i], list b[j])
  const int* a;
  const int* b;
  int na, nb;
  zd* out;
  int64_t ld;
  int a_is_target;  // 1: a = targets (rows of A), b = sources; 0: swapped (transposed block)
};

struct DiagDesc {   // one inclusion's self block
  int node0, n;
  double k_int, eps_int;
  int tbl;          // offset of this n's Kress/difference tables
  zd* out;          // 2n x 2n, ld 2n
  zd* scratch;      // n x n, holds S+/e+ + S-/e- then the Maue intermediate
  zd* scratch2;     // n x n
};

struct ParentDesc { // gathered parent block of the compressed system
  const int* rcode;
  const int* ccode;
  const int* rloc;  // child slot << 24 | local index (rows)
  const int* cloc;
  int s;
  zd* out;          // s x s
  const zd* at[4];  // children's compressed blocks
  int kc[4];        // their sizes
};

struct Mat2 {       // plain matrix view (n x n, leading dimension ld)
  zd* p;
  int64_t ld;
  int n;
};

struct RowSrc {     // source of one gathered row
  int64_t off;      // element offset of the row's first entry
  int64_t ld;       // distance between consecutive columns
};

struct GatherDesc {
  const RowSrc* src;
  int nrows, ncols;
  zd* dst;
  int64_t ld;
};

void asm_geometry(const double* dx, const double* dy, const double* ddx, const double* ddy,
                  const int* owner, const int64_t* node_off, double* nx, double* ny, double* w,
                  double* speed, double* kappa, int n_nodes, hipStream_t s);
void asm_tables(const int* ns, const int* tbl_off, int ntbl, int max_n, double* R, double* dt,
                hipStream_t s);
void asm_diag(DevGeom g, ExtParams e, const DiagDesc* d, int batch, int max_n, const double* R,
              const double* dt, hipStream_t s);
void asm_entries(DevGeom g, DevProxy p, ExtParams e, const EntryMat* d, int batch, int max_a,
                 int max_b, hipStream_t s);
void asm_parent(DevGeom g, ExtParams e, const ParentDesc* d, int batch, int max_s, hipStream_t s);
// leaf right-hand sides: rows [0,n) = -u^I, [n,2n) = -q^I per cell, column per angle
void asm_incident(DevGeom g, ExtParams e, const int* cell_node0, const int* cell_n,
                  const int64_t* cell_off, int ncell, int max_n, const double* angles, int nrhs,
                  zd* f, hipStream_t s);
// dst[i + c ld] = src[row_i.off + c row_i.ld] for i < nrows, c < ncols of each entry
void asm_gather(const zd* src, const GatherDesc* d, int batch, int max_rows, int max_cols,
                hipStream_t s);
// batched identity: a[i + j ld] = (i == j) for an n x n matrix per entry
void asm_identity(const Mat2* d, int batch, int max_n, hipStream_t s);
void asm_zero(zd* p, int64_t n, hipStream_t s);
// far field: out[r * ndir + t] for densities dens (ld = 2 * n_nodes, per inclusion [q; u])
void asm_far_field(DevGeom g, ExtParams e, const int* owner, const int64_t* node_off,
                   const zd* dens, int nrhs, const double* dirs, int ndir, zd* out, hipStream_t s);
// build the explicit L = blockdiag(Z_0^T, Z_1^T) (s x K) of a batch of cells
struct LDesc {
  zd* out;          // s x K, ld s
  int s0, s1, k0, k1;
  const int* piv0;  // row-ID pivots, type 0 and 1
  const int* piv1;
  const zd* t0;     // T blocks: t[i + j ldt]
  const zd* t1;
  int ldt0, ldt1;
};
void asm_build_l(const LDesc* d, int batch, int max_s, int max_k, hipStream_t s);
// y[i] += x[i] for complex arrays (used for the residual of iterative refinement)
void asm_axpy(zd* y, const zd* x, zd a, int64_t n, hipStream_t s);
// J0, J1, Y0, Y1 at z[i]: out[f * n + i]
void asm_probe_bessel(const double* z, int64_t n, double* out, hipStream_t s);
