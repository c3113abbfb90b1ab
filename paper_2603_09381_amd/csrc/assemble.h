// Kernel-matrix assembly, right-hand sides, gathers and the far field (gfx950).  Matrix
// entries are always evaluated in FP64; the templated launchers store them as cx<R>.
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

template <class R>
struct EntryMatT {  // out[i + j ld] = entry(list a[i], list b[j]), computed in FP64, stored as R
  const int* a;
  const int* b;
  int na, nb;
  cx<R>* out;
  int64_t ld;
  int a_is_target;  // 1: a = targets (rows of A), b = sources; 0: swapped (transposed block)
};
typedef EntryMatT<double> EntryMat;

struct DiagDesc {   // one inclusion's self block
  int node0, n;
  double k_int, eps_int;
  int tbl;          // offset of this n's Kress/difference tables
  zd* out;          // 2n x 2n, ld 2n
  zd* scratch;      // n x n, holds S+/e+ + S-/e- then the Maue intermediate
  zd* scratch2;     // n x n
};

template <class R>
struct ParentDescT { // gathered parent block of the compressed system
  const int* rcode;
  const int* ccode;
  const int* rloc;  // child slot << 24 | local index (rows)
  const int* cloc;
  int s;
  cx<R>* out;          // s x s
  const cx<R>* at[4];  // children's compressed blocks
  int kc[4];           // their sizes
};

template <class R>
struct Mat2T {      // plain matrix view (n x n, leading dimension ld)
  cx<R>* p;
  int64_t ld;
  int n;
};

struct RowSrc {     // source of one gathered row
  int64_t off;      // element offset of the row's first entry
  int64_t ld;       // distance between consecutive columns
};

template <class R>
struct GatherDescT {
  const RowSrc* src;
  int nrows, ncols;
  cx<R>* dst;
  int64_t ld;
};
typedef GatherDescT<double> GatherDesc;

void asm_geometry(const double* dx, const double* dy, const double* ddx, const double* ddy,
                  const int* owner, const int64_t* node_off, double* nx, double* ny, double* w,
                  double* speed, double* kappa, int n_nodes, hipStream_t s);
void asm_tables(const int* ns, const int* tbl_off, int ntbl, int max_n, double* R, double* dt, int quad,
                hipStream_t s);
void asm_diag(DevGeom g, ExtParams e, const DiagDesc* d, int batch, int max_n, const double* R,
              const double* dt, hipStream_t s);
template <class R>
void asm_entries(DevGeom g, DevProxy p, ExtParams e, const EntryMatT<R>* d, int batch, int max_a, int max_b,
                 hipStream_t s);
// Node-node rows of the four ID matrices of a cell of one inclusion (own nodes own0 ..
// own0 + n_own - 1, all of them active, value / q rows before derivative / u rows) against a
// near cell of one inclusion (nodes near0 .. near0 + n_near - 1): out[kd] points at the near
// cell's first row in ID matrix kd (0 q columns, 1 u columns, 2 value rows, 3 derivative
// rows; column major, leading dimension ld); rows [0, n_near) take the near nodes' first
// type, [n_near, 2 n_near) the second.
template <class R>
struct LeafPairDescT {
  cx<R>* out[4];
  int64_t ld;
  int own0, n_own, near0, n_near;
};
template <class R>
void asm_leaf_pairs(DevGeom g, ExtParams e, const LeafPairDescT<R>* d, int n, hipStream_t s);
template <class R>
void asm_parent(DevGeom g, ExtParams e, const ParentDescT<R>* d, int batch, int max_s, hipStream_t s);
// leaf right-hand sides: rows [0,n) = -u^I, [n,2n) = -q^I per cell, column per angle
void asm_incident(DevGeom g, ExtParams e, const int* cell_node0, const int* cell_n,
                  const int64_t* cell_off, int ncell, int max_n, const double* angles, int nrhs,
                  zd* f, hipStream_t s);
// dst[i + c ld] = src[row_i.off + c row_i.ld] for i < nrows, c < ncols of each entry;
// the source may be of another real type (converted), and with acc = 1 the value is added
// to dst instead of stored
template <class RS, class RD>
void asm_gather(const cx<RS>* src, const GatherDescT<RD>* d, int batch, int max_rows, int max_cols, hipStream_t s,
                int acc = 0);
// batched identity: a[i + j ld] = (i == j) for an n x n matrix per entry
template <class R>
void asm_identity(const Mat2T<R>* d, int batch, int max_n, hipStream_t s);
template <class R>
void asm_zero(cx<R>* p, int64_t n, hipStream_t s);
// Near row and column code lists of the cells of a level: cell t's list starts at nro[t]
// and holds the codes rows / cols [offS[s], offS[s + 1]) of its near cells
// s = nidx[noff[t] .. noff[t + 1]) in order, then its proxy points poff[t] .. + np[t]
// (value type, then derivative type).  All arrays in device memory.
void asm_near_lists(const int* rows, const int* cols, const int64_t* offS, const int* noff, const int* nidx,
                    const int64_t* nro, const int* poff, const int* np, int ncell, int* nr, int* ncl, hipStream_t s);
// p[0 .. n) = 0 by a kernel (a node that graph capture records like any launch)
void asm_zero_i32(int* p, int64_t n, hipStream_t s);
// dst[i] = src[i] converted to the destination's real type
template <class RS, class RD>
void asm_convert(const cx<RS>* src, cx<RD>* dst, int64_t n, hipStream_t s);
// blocks of FP64 complex entries, block t from src + soff[t] to dst + doff[t] (len[t]
// entries), rounded to RD; the offset and length arrays in device memory
template <class RD>
void asm_convert_blocks(const zd* src, cx<RD>* dst, const int64_t* d_soff, const int64_t* d_doff,
                        const int64_t* d_len, int nblocks, int64_t max_len, hipStream_t s);
// far field: out[r * ndir + t] for densities dens (ld = 2 * n_nodes, per inclusion [q; u]);
// dirs is host memory [ndir] (angles), part device memory of far_field_part_bytes() for
// the partial sums of the split node sum
constexpr int PMX_FF_DIRS = 64;   // directions per launch, passed as kernel arguments
struct FarDirs {
  double c[PMX_FF_DIRS], s[PMX_FF_DIRS];   // cos, sin of the directions t0 .. t0 + nt - 1
  int t0, nt;
};
int far_field_splits(int64_t n_nodes, int nrhs, int ndir);
size_t far_field_part_bytes(int64_t n_nodes, int nrhs, int ndir);
void asm_far_field(DevGeom g, ExtParams e, const int* owner, const int64_t* node_off, const zd* dens, int nrhs,
                   const double* dirs, int ndir, zd* part, zd* out, hipStream_t s);
// Device address of this GPU's copy of the static partial-sum array of the allocation-free
// far field (PMX_FF_SCRATCH_BYTES, shared by every call on the GPU).
constexpr size_t PMX_FF_SCRATCH_BYTES = (size_t)8 << 20;
constexpr int PMX_MAX_DEVICES = 64;
hipError_t far_field_scratch(zd** out);
// build the explicit L = blockdiag(Z_0^T, Z_1^T) (s x K) of a batch of cells
template <class R>
struct LDescT {
  cx<R>* out;          // s x K, ld s
  int s0, s1, k0, k1;
  const int* piv0;     // row-ID pivots, type 0 and 1
  const int* piv1;
  const cx<R>* t0;     // T blocks: t[i + j ldt]
  const cx<R>* t1;
  int ldt0, ldt1;
};
template <class R>
void asm_build_l(const LDescT<R>* d, int batch, int max_s, int max_k, hipStream_t s);
// y[i] += a x[i] for complex FP64 arrays
void asm_axpy(zd* y, const zd* x, zd a, int64_t n, hipStream_t s);
// Dense FP64 operator apply between different inclusions (exterior kernels), for a block
// of right-hand sides in the density layout (ld = 2 n_nodes, per inclusion [q; u]).
// Targets are taken in waves of at most 64 consecutive nodes of one inclusion.  Tree
// nodes are the inclusions and the clusters of the plan's tree above them (index:
// inclusions first, then the clusters level by level upwards); each has a bounding circle.
// Every tree node is a source with a multipole expansion about its centre (Graf's addition
// theorem): an inclusion's coefficients come from its nodes (p2m kernel), a cluster's from
// its children's by the regular translation (m2m kernel, one launch per tree level).
// Far field (fast multipole method): a dual walk down the tree pairs target and source
// nodes; a pair whose circles are well separated ((r~_T + r_S) <= PMX_FMM_RATIO |c_T - c_S|,
// r~_T the radius about c_T of every circle below T) is translated into the target's
// local expansion (m2l kernel, with the pair's table of O_nu(c_T - c_S) made once per
// solve state); local expansions move down the tree (l2l kernel, one launch per level)
// and are evaluated at the target nodes (inside the far kernel).  Pairs left over at an
// inclusion (too close for a translation) start each of its waves' walks: far sources,
// taken through their expansions to the order the distance needs (far kernel, the list
// split in nsplit parts), and near inclusions, applied pair by pair (near kernel, split in
// nsplit_near parts, same-inclusion pairs left out).  In a wave's walk a cluster is far
// when its centre is farther than PMX_APPLY_RATIO cluster radii from the wave's circle and
// PMX_APPLY_PMAXC orders suffice; otherwise its children are examined.  An inclusion
// reached that way is near when its centre is closer than PMX_APPLY_RATIO radii or its
// expansion would need more than PMX_APPLY_PMAX orders, else far.  Partial sums go to
// part [nsplit + nsplit_near][nrhs][ld].
#define PMX_APPLY_RATIO 2.5
#define PMX_APPLY_PMAX 48
#define PMX_APPLY_PMAXC 96   // largest order of a cluster expansion
// truncation of a far pair: orders until (r_j / rho_min)^p <= e^-PMX_APPLY_TRUNC, about
// 1e-13, and of a source's own expansion: until its J_p decay reaches the same bound (on the
// star grids the sources' own order, from k r_j, is the larger one for most pairs).  The
// apply then stays within about 1e-13 of the assembled operator, three orders below the
// refinement's tolerances, which end at 1e-10.
#define PMX_APPLY_TRUNC 30.0
// coefficient records per source: orders m = 0 .. PMX_APPLY_PMAXC + 1, per right-hand side
// six complex numbers A_m, A_-m, B_m+1, B_-m+1, B_m-1, B_-m-1 (A: value rows, B: normal
// derivative rows; the -m entries are zero for m = 0); an inclusion fills orders up to
// PMX_APPLY_PMAX + 1 only
#define PMX_APPLY_NREC (PMX_APPLY_PMAX + 2)
#define PMX_APPLY_NRECA (PMX_APPLY_PMAXC + 2)
#define PMX_APPLY_MAXLEV 32
#ifndef PMX_APPLY_NR_NEAR
#define PMX_APPLY_NR_NEAR 8   // right-hand sides per group of the near part (8 or 16)
#endif
// fast multipole part: separation ratio of a translated pair, largest local order, and the
// local-expansion orders kept per target (m = -(PMX_FMM_PL + 1) .. PMX_FMM_PL + 1)
#ifndef PMX_FMM_RATIO
#define PMX_FMM_RATIO 0.5
#endif
#define PMX_FMM_PL 94     // at most 94: the m2l kernel's three passes hold orders -96 .. 95
#define PMX_FMM_NMAX 80   // largest source order of a translated pair (<= PMX_APPLY_PMAXC)
#define PMX_FMM_CHUNK 16  // translated pairs per work item of the m2l kernel
#define PMX_FMM_NL (2 * PMX_FMM_PL + 3)
struct ApplyArgs {
  const double *x, *y, *nx, *ny, *w;
  const int* owner;
  const int64_t* node_off;
  int n_nodes;
  double k, eps;
  const zd* xin;
  int nrhs;
  int64_t ld;
  zd* part;
  double* pack;          // [apply_pack_size] packed source data of one group of right-hand sides
  const int* near_off;   // [n_waves + 1]
  const int* near_idx;   // near inclusions of each wave, ascending
  const int* far_off;    // [n_waves + 1]
  const int* far_idx;    // far sources of each wave
  int nsplit_near;
  const double* incl_geo;  // per source: centre x, y, radius, order needed by the sources' decay
  const double* wave_geo;  // per wave: bounding-circle centre x, y, radius, unused
  const int* kid_off;    // [n_clus + 1] children of each cluster (source indices)
  const int* kid_idx;
  zd* coef;              // [n_src][PMX_APPLY_NRECA][nr][6] expansion records of one group
  int n_incl, n_clus;
  int n_lev;             // cluster levels; level l holds clusters lev_off[l] .. lev_off[l + 1] - 1
  int lev_off[PMX_APPLY_MAXLEV + 1];
  zd* near_blk;          // stored near coefficients (see k_apply_near_build) or NULL
  const int64_t* near_blk_off;  // per near-list entry: offset of its block
  const int* wave_node;  // [n_waves][2]: first node and node count of each target wave
  int n_waves;
  // fast multipole part
  zd* loc;               // [n_loc][2][PMX_FMM_NL][nr] local expansions (A, B) of one group
  zd* cm;                // [n_src][2][2 PMX_FMM_NMAX + 1][nr] translated sources' A_n, B_n
  const int* loc_id;     // [n_src] slot in loc of each tree node, -1: no local expansion
  const int* loc_p;      // [n_loc] order of each local expansion
  const double* loc_geo; // [n_loc][2] its centre
  int n_loc;
  const int* m2l_item;   // [n_m2l_items][3]: slot, first and last + 1 pair of each work item
  const int* m2l_item_off;  // [n_loc + 1] work items of each local expansion
  int n_m2l_items;
  zd* m2l_part;          // [n_m2l_items][2][PMX_FMM_NL][nr] partial local expansions
  const int* m2l_off;    // [n_loc + 1] translated sources of each local expansion
  const int* m2l_slot;   // local-expansion slot of each pair
  const int* m2l_src;    // source tree node of each pair
  const int* m2l_nmax;   // source order of each pair
  const int* m2l_mmax;   // local order of each pair (<= the slot's order)
  const int64_t* m2l_toff;  // offset of the pair's table O_nu(c_T - c_S), nu = -V .. V,
                            // V = mmax + 1 + nmax (complex entries)
  zd* m2l_tab;
  const int* l2l_child;  // [n_l2l] child slot of each parent-to-child translation, grouped
  const int* l2l_parent; //   by level from the top (l2l_lev[l] .. l2l_lev[l + 1] - 1)
  const int64_t* l2l_toff;  // offset of the pair's table I_nu(c_C - c_P), nu = -W .. W,
                            // W = p_P + p_C + 2
  zd* l2l_tab;
  int n_l2l_lev;
  int l2l_lev[PMX_APPLY_MAXLEV + 2];
};
// tables of the translations (once per solve state): O_nu(D) of every M2L pair and
// I_nu(d) of every L2L pair
void asm_apply_tables(const ApplyArgs& a, int n_m2l, int n_l2l, hipStream_t s);
// the stored near coefficients (once per solve state), when a.near_blk is set
void asm_apply_near_build(const ApplyArgs& a, hipStream_t s);
// budget of the stored near Bessel values; beyond it (or for fewer than 4 right-hand sides)
// the near pairs are evaluated in every apply
#define PMX_APPLY_NEAR_BYTES ((int64_t)48 << 30)
// orders needed for the sources of an inclusion of radius r: the smallest p with
// (e k r / 2p)^p <= e^-PMX_APPLY_TRUNC and p > e k r / 2 + 2
int apply_source_order(double kr);
// source splits giving about wg_target workgroups per launch
int apply_splits(int n_nodes, int wg_target);
// near-list splits giving about wg_target one-wave workgroups per launch
int apply_near_splits(int n_nodes, int wg_target);
// doubles of the packed source data for groups of up to nr_max right-hand sides
int64_t apply_pack_size(int n_nodes, int nr_max);
// complex entries of the expansion records for groups of up to nr_max right-hand sides
int64_t apply_coef_size(int n_src, int nr_max);
// complex entries of the translated sources' coefficients (m2l layout), the same groups
int64_t apply_m2l_coef_size(int n_src, int nr_max);
// partial sums of the off-diagonal operator (far ranges, then near parts), right-hand
// sides in groups of nr_max (1, 2, 4, 8) per thread
void asm_apply_off(const ApplyArgs& a, int nsplit, int nr_max, hipStream_t s);
// out = sf f + sa (ydiag + sum_p part[p]) elementwise over total entries (f may be NULL)
void asm_apply_finish(const zd* f, const zd* ydiag, const zd* part, int nsplit, int64_t total, double sf, double sa,
                      zd* out, hipStream_t s);
// squared column norms: part[c nblk + b], summed over b by the caller
void asm_colnorm2(const zd* a, int64_t n, int ncol, int64_t ld, int nblk, double* part, hipStream_t s);
// J0, J1, Y0, Y1 at z[i]: out[f * n + i]
void asm_probe_bessel(const double* z, int64_t n, double* out, hipStream_t s);
