/* pmx probe API: the library's own kernels on explicit inputs, for step-level checks.
 *
 * Each entry point runs exactly the kernel the factorisation uses, on caller data, so
 * that a test can compare one step of the method with an independent reference.
 * Pointers marked (device) are device memory; (host) host memory.  Results are written
 * in stream order on `stream`; every call synchronises it before returning.
 */
#ifndef PMX_PROBE_H
#define PMX_PROBE_H

#include "pmx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} pmx_c32;

/* J0, J1, Y0, Y1 at z[i] > 0 (device, n values); out (device) [4][n]. */
pmx_status pmx_probe_bessel(const double* z, int64_t n, double* out, void* stream);

/* Self block A_jj of inclusion j (Sec. 2.2 Omit form, Kress quadrature): out (device)
 * 2n_j x 2n_j column major. */
pmx_status pmx_probe_diag_block(const pmx_geometry* geom, int32_t j, pmx_c64* out, void* stream);
/* As pmx_probe_diag_block with the self-block quadrature of pmx_options.quadrature (0 Kress,
 * 1 zeta-corrected trapezoid, Sec. 2.2).  PMX_EINVAL for other values or fewer than 42
 * nodes with quadrature 1. */
pmx_status pmx_probe_diag_block_quad(const pmx_geometry* geom, int32_t j, int32_t quadrature, pmx_c64* out,
                                     void* stream);

/* Off-diagonal (exterior) matrix entries between boundary nodes: rows (host) [nr] node
 * indices with row types rtyp (0 value, 1 normal-derivative equation), cols (host) [nc]
 * with column types ctyp (0 q, 1 u); out (device) nr x nc column major. */
pmx_status pmx_probe_entries(const pmx_geometry* geom, int32_t nr, const int32_t* rows,
                             const int32_t* rtyp, int32_t nc, const int32_t* cols,
                             const int32_t* ctyp, pmx_c64* out, void* stream);

/* C = A B for a batch of column-major complex matrices packed back to back (device):
 * A [batch][m x k], B [batch][k x n], C [batch][m x n]; opa/opb 0 N, 1 T, 2 C (conjugate
 * transpose of the stored operand, whose shape is then k x m / n x k). */
pmx_status pmx_probe_zgemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t opa, int32_t opb,
                           const pmx_c64* A, const pmx_c64* B, pmx_c64* C, void* stream);

/* As pmx_probe_zgemm in complex FP32 (the FP32 MFMA kernel of the mixed-precision factor). */
pmx_status pmx_probe_cgemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t opa, int32_t opb,
                           const pmx_c32* A, const pmx_c32* B, pmx_c32* C, void* stream);

/* LU with partial pivoting of a batch of n x n matrices (device, in place) and solve with
 * nrhs right-hand sides B [batch][n x nrhs] (device, in place).  ipiv (device) [batch][n].
 * info (host) [batch]: first zero pivot (1-based) or 0.  variant selects the solve kernel:
 * 0 the fused substitution of the solves (<= 64 right-hand sides), 1 the blocked solve of
 * the factorisation, 2 the fused substitution with the solution in LDS (n x 4 complex
 * <= 128 KiB), -1 the solves' built-in rule; a variant that does not hold the shape falls
 * back to the built-in rule. */
pmx_status pmx_probe_lu_solve(int32_t batch, int32_t n, pmx_c64* A, int32_t* ipiv, int32_t nrhs,
                              pmx_c64* B, int32_t* info, int32_t variant, void* stream);

/* As pmx_probe_lu_solve in complex FP32. */
pmx_status pmx_probe_lu_solve_c32(int32_t batch, int32_t n, pmx_c32* A, int32_t* ipiv, int32_t nrhs,
                                  pmx_c32* B, int32_t* info, int32_t variant, void* stream);

/* Interpolative decomposition of a batch of m x c matrices (device, destroyed): QR, then
 * column-pivoted QR with threshold rank |R_jj| > tol |R_11|; k = max(rank, kmin[b]) pivots
 * are kept.  Outputs: piv (device) [batch][c] column order, rank (host) [batch] threshold
 * ranks, T (device) [batch][c x c] with T[0:k, 0:c-k] = R11^-1 R12 (leading dimension c).
 * kmin (host) [batch] or NULL. */
pmx_status pmx_probe_id(int32_t batch, int32_t m, int32_t c, pmx_c64* M, double tol,
                        const int32_t* kmin, int32_t* piv, int32_t* rank, pmx_c64* T, void* stream);

/* As pmx_probe_id in complex FP32 (column norms, |R_11| and pivot decisions stay FP64). */
pmx_status pmx_probe_id_c32(int32_t batch, int32_t m, int32_t c, pmx_c32* M, double tol,
                            const int32_t* kmin, int32_t* piv, int32_t* rank, pmx_c32* T, void* stream);

/* y = A x for the whole FP64 PMCHWT (Omit) matrix of Sec. 2.2 (self blocks by the Kress
 * rule, the exterior blocks between inclusions evaluated on the fly), the operator of the
 * refinement residual: x, y (device) [nrhs][2 node_off[m]] in the density layout of
 * pmx_solve; x and y may not overlap. */
pmx_status pmx_probe_apply(const pmx_geometry* geom, int32_t nrhs, const pmx_c64* x, pmx_c64* y,
                           void* stream);

/* One forward and backward pass of the network on a batch (all host memory): shape nin,
 * nhidden x nlayer hidden ReLU layers, nout outputs; params packed per layer as W (out x
 * in, column major) then b; X [B][nin], labels [B][nout] (first nout/2 binary, the rest
 * regression targets weighted by wmse).  Outputs: out [B][nout] (the last layer before
 * the loss), grad (as params) of the batch-mean loss, *loss the batch-mean loss. */
pmx_status pmx_probe_mlp(int32_t nin, int32_t nhidden, int32_t nlayer, int32_t nout, const float* params,
                         const float* X, const float* labels, int32_t B, float wmse, float* out, float* grad,
                         double* loss, void* stream);

/* Host only (no GPU work): the operator apply's structure for the refinement residual of a
 * geometry, built as a factor's first solve builds it (plan, target waves, dual tree walk
 * of the fast multipole part, the waves' walks).  stats [16]: 0-7 as pmx_info.apply_stats;
 * 8 the longest translation list of a local expansion, 9 the mean; 10 the longest far list
 * and 11 the longest near list of a wave; 12 with check != 0 the number of (wave, source
 * inclusion) pairs not taken exactly once (near, through a far source of the wave, or
 * through a translation into the wave's inclusion or an ancestor; none for the wave's own
 * inclusion), else -1; 13 waves; 14 the largest local order; 15 pairs checked. */
pmx_status pmx_probe_apply_structure(const pmx_geometry* geom, const pmx_options* opts, int32_t check,
                                     double* stats);

/* The plan's tree (either tree), host only (no GPU): per level the number of cells; per
 * centre, radius, proxy radius, proxy count and near list.  Buffers (host) are filled up
 * to their capacity; *n_levels, *n_cells_total and *n_near_total report the sizes
 * needed.  cell_level [cap_cells], cell_first_incl, cell_center [2 cap], cell_rc,
 * cell_rp, cell_p, near_off [cap_cells + 1], near [cap_near] (indices within the level). */
pmx_status pmx_plan_query(const pmx_geometry* geom, const pmx_options* opts, int32_t cap_cells,
                          int32_t cap_near, int32_t* n_levels, int32_t* n_cells_total,
                          int32_t* n_near_total, int32_t* cell_level, int32_t* cell_first_incl,
                          double* cell_center, double* cell_rc, double* cell_rp, int32_t* cell_p,
                          int32_t* near_off, int32_t* near);

/* The plan's membership, host only (no GPU), cells in the order of pmx_plan_query: per
 * cell its inclusions (ascending) and its children (indices within the level below).
 * Buffers (host) are filled up to their capacity; *n_cells_total, *n_incl_total and
 * *n_child_total report the sizes needed.  incl_off [cap_cells + 1], incl [cap_incl],
 * child_off [cap_cells + 1], child [cap_child]. */
pmx_status pmx_plan_members(const pmx_geometry* geom, const pmx_options* opts, int32_t cap_cells,
                            int32_t cap_incl, int32_t cap_child, int32_t* n_cells_total,
                            int32_t* n_incl_total, int32_t* n_child_total, int32_t* incl_off,
                            int32_t* incl, int32_t* child_off, int32_t* child);

#ifdef __cplusplus
}
#endif
#endif
