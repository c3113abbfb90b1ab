/* pmx: proxy-method fast direct solver for 2-D Helmholtz transmission through many
 * disjoint inclusions, PMCHWT (Omit) Nystrom discretisation, on one AMD MI355X (gfx950).
 *
 * Method: arXiv 2603.09381.  Problem and boundary data: Sec. 2.1 (transmission
 * conditions, eqs. pressure and flux; unknowns u and q = (1/eps) du/dn on each
 * boundary).  System: the Omit form of Sec. 2.2 (exterior kernels only between
 * different inclusions), unknowns ordered per inclusion as (q_i; u_i) and right-hand
 * side (-u^I_i; -q^I_i).  Solver: Sec. 3 (proxy method + interpolative decomposition
 * by column-pivoted QR with threshold rank, compressed system of eq. compressed,
 * recovery formula, multi-level recursion), top system by partial-pivoted LU (Sec. 4).
 * Self-interaction quadrature: Kress' logarithmic product rule or the paper's
 * zeta-corrected trapezoid rule (options.quadrature), hypersingular operator through
 * Maue's identity.  Trees: the grid quadtree of Sec. 4 or the k-means clustering with
 * several inclusions per leaf of Sec. 4.4 (options.tree).
 *
 * Conventions.  Every function returns a pmx_status and never aborts; the text of the
 * last error of the calling thread is returned by pmx_last_error().  Host pointers are
 * only read during the call.  Device pointers must be device memory of the current
 * HIP device (e.g. torch tensors); device results are written in stream order on the
 * stream passed (a hipStream_t, NULL = default stream).
 */
#ifndef PMX_H
#define PMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} pmx_c64;

typedef enum {
  PMX_OK = 0,
  PMX_EINVAL = 1,     /* bad argument (sizes, NULL, odd node count, NaN, ...) */
  PMX_EGEOM = 2,      /* geometry not supported (shared grid cell, missing grid) */
  PMX_ENOMEM = 3,     /* device allocation failed */
  PMX_EHIP = 4,       /* a HIP runtime call failed */
  PMX_ESINGULAR = 5,  /* zero or non-finite pivot in an LU factorisation */
  PMX_ENOTCONV = 6    /* iterative refinement did not reach its tolerance */
} pmx_status;

/* Geometry: m closed, counterclockwise, smooth boundaries.  Inclusion j owns nodes
 * node_off[j] .. node_off[j+1]-1 (n_j = node_off[j+1]-node_off[j] even, >= 8), sampled at
 * t = 2 pi l / n_j with the curve x(t), its first and second t-derivatives.  The unit
 * normal n = (x2', -x1')/|x'| points into the exterior (Sec. 2.1).  Wavenumbers: k_ext
 * outside, k_int[j] inside inclusion j; material constants eps_ext and eps_int[j]
 * (NULL: eps_ext (k_int[j]/k_ext)^2, from k = omega sqrt(eps)).  grid_ij[2j], grid_ij[2j+1]
 * are the integer grid cell of inclusion j (one inclusion per cell); the quadtree is
 * built over these cells.  grid_ij NULL (scattered inclusions): the library places the
 * centres on a uniform grid of spacing 0.99 d_min / sqrt(2) (d_min the smallest centre
 * distance), one centre per cell, and prunes the empty cells of the quadtree.  All arrays
 * are host memory. */
typedef struct {
  int32_t m;
  const int64_t* node_off;   /* [m+1] */
  const double *x, *y;       /* [node_off[m]] */
  const double *dx, *dy;
  const double *ddx, *ddy;
  const double* center;      /* [2m] inclusion centres (cell centres are their means) */
  const int32_t* grid_ij;    /* [2m] or NULL */
  double k_ext, eps_ext;
  const double* k_int;       /* [m] */
  const double* eps_int;     /* [m] or NULL */
} pmx_geometry;

typedef struct {
  double id_tol;        /* CPQR threshold: keep |R_jj| > id_tol |R_11| (Sec. 3) */
  double proxy_ratio;   /* proxy radius >= proxy_ratio * cell radius */
  int32_t proxy_min;    /* minimum number of proxy points (exact number if proxy_rule = 1) */
  int32_t proxy_rule;   /* 0: radius max(ratio r_c, 0.9 rho_far), adaptive count; 1: fixed */
  int32_t near_rule;    /* 0: edge-adjacent cells + geometric test (Sec. 4); 1: geometric
                           (every cell with a node inside the proxy circle); 2: the
                           eta-admissibility test below + geometric */
  int32_t precision;    /* 0: FP64 throughout.  1: mixed: the factor (assembly storage,
                           QR, CPQR data, LU, Schur products) in complex FP32 with FP64 column
                           norms and pivot decisions, used as the inner solver of iterative
                           refinement against the FP64 operator (self blocks by the FP64
                           Kress rule, the rest evaluated on the fly); id_tol >= 1e-6.
                           2: the FP64 factor
                           (typically at a looser id_tol) refined the same way */
  int32_t timing;       /* 1: record per-phase device times in pmx_info */
  int32_t ir_max_iter;  /* precision 1, 2: at most this many refinement steps (1..100) */
  double ir_tol;        /* precision 1, 2: stop when max over right-hand sides of
                           |f - A x| / |f| <= ir_tol (2-norms) */
  int32_t solve_graph;  /* 1: every solve's launch sequence (per right-hand-side count) is
                           captured once as a HIP graph and replayed; 0: launched directly */
  int32_t learned;      /* 1: the leaf IDs start from the network of model_path: per ID its
                           proposed columns go first, QR stops after them, pivots are chosen
                           among them, and the result stands when every other column is
                           within id_tol |R_11| of their span (both IDs of both pairs of the
                           cell); otherwise the cell's IDs take the full CPQR */
  const char* model_path;  /* network file written by pmx_mlp_train (read at create) */
  uint32_t timing_kernels; /* with timing = 1: bit k selects kernel k of pmx_info.t_kernel_ms
                              for timing; 0: every kernel.  Solve sequences run launch by
                              launch (not as graphs) only when one of their kernels is timed */
  int32_t reserved0;
  const char* tune_path;   /* launch-parameter table written by pmx_autotune (read at create);
                              NULL: built-in rules */
  int32_t refactor;        /* 1: keep the numeric phase of the factorisation (its buffers,
                              descriptors and launch sequence) for pmx_factor_refactor; not
                              with learned = 1 */
  int32_t quadrature;      /* self blocks: 0 Kress' logarithmic product rule (spectral);
                              1 the zeta-corrected trapezoid rule with 41 local correction
                              points of Sec. 2.2 (needs >= 42 nodes per inclusion) */
  int32_t tree;            /* 0: quadtree over grid cells (Sec. 4; grid_ij, or the pruned grid
                              of scattered inclusions), one inclusion per leaf.  1: the
                              general arrangement of Sec. 4.4: a hierarchical k-means
                              clustering of the inclusions (node means weighted by node
                              counts, four clusters per split) with up to leaf_size
                              inclusions per leaf; grid_ij is ignored; needs near_rule 1 or 2
                              and learned = 0 */
  int32_t leaf_size;       /* tree 1: at most this many inclusions per leaf, 1..4; a leaf of
                              several inclusions is compressed as one cell (its own
                              inclusions interact through its dense block).  With
                              leaf_size > 1, pmx_factor_create returns PMX_EINVAL for plans of
                              more than 512 leaves */
  double eta;              /* near_rule 2 (Sec. 4.4): cells s, t of a level are near when
                              eta |c_s - c_t| < max(2 r_s, 2 r_t) (r: farthest own node from
                              the cell centre c), then the proxy-circle test of near_rule 1;
                              eta > 0 */
  int32_t reserved[2];
} pmx_options;

typedef struct {
  int32_t levels;            /* compressed levels below the root */
  int32_t root_size;         /* size of the top compressed system */
  int32_t n_unknowns;        /* 2 * total nodes */
  int32_t cells[32];         /* cells per level */
  int32_t rank_min[32], rank_max[32];   /* min / max skeleton count K per level */
  double rank_mean[32];
  double bytes_factor;       /* device bytes held by the factor */
  double t_factor_ms;        /* wall time of pmx_factor_create (host clock, synchronised) */
  double t_phase_ms[16];     /* host wall time of phases: 0 self blocks, 1 level compression,
                                2 level merges, 3 top LU, 4 plan; solves: 5 set-up of the
                                solve state for a new right-hand-side count, 6 of it the
                                operator apply set-up; 7 the leaf level's IDs (part of 1:
                                QR, CPQR, with learned proposals their judge and fallback),
                                8 the learned proposals (features and network, at create),
                                9 and 10 the solve program and the leaf maps (host parts of 5) */
  /* with options.timing = 1: per-kernel device time from HIP events around every launch
   * (of the kernels selected by options.timing_kernels) of the factorisation and of the
   * solves, summed over them (index: 0 QR leaf blocks, 1 QR trailing update, 2 LU panel, 3 CPQR
   * update, 4 CPQR single-workgroup, 5 complex GEMM, 6 small triangular solves, 7 entry
   * assembly, 8 self blocks, 9 dense operator apply of refinement residuals, 10 fused
   * substitutions of few right-hand sides), launch counts, and the algorithmic bytes and
   * flops of the kernels whose work the library counts (0, 1, 2, 9). */
  double t_kernel_ms[16];
  int32_t n_kernel_launch[16];
  double kernel_bytes[16];
  double kernel_flops[16];
  /* last solve: host wall time (synchronised), refinement steps and the final relative
   * residual max_r |f - A x| / |f| (precision 1, 2; 0 for precision 0) */
  double t_solve_ms;
  int32_t ir_iterations;
  double ir_residual;
  double ir_history[16];     /* relative residual after each of the first 16 steps */
  int32_t id_learned;        /* leaf cells whose IDs the learned proposals settled */
  int32_t id_fallback;       /* leaf cells that fell back to the full CPQR */
  /* refined forms, after the first solve: the operator apply's fast multipole structure:
   * 0 translated (target, source) pairs, 1 their mean source order, 2 their mean local
   * order, 3 local expansions, 4 parent-to-child translations, 5 near (target node, source
   * node) pairs, 6 (target node, far source) pairs evaluated directly, 7 bytes of the
   * translation tables */
  double apply_stats[8];
  /* host-side counts of the factorisation (create): kernel launches and host waits on the
   * device (downloads of ranks, pivots and LU checks, CPQR progress polls) */
  int64_t factor_launches;
  int64_t factor_host_syncs;
  /* last pmx_factor_refactor: launches from the host (1: the graph), kernel nodes of the
   * replayed graph, host waits, and its host wall time (synchronised) */
  int64_t refactor_launches;
  int64_t refactor_graph_nodes;
  int64_t refactor_host_syncs;
  double t_refactor_ms;
} pmx_info;

typedef struct pmx_factor pmx_factor;

/* Fills defaults: id_tol 1e-10, proxy_ratio 1.5, proxy_min 0, proxy_rule 0, near_rule 0,
 * precision 0, timing 0, ir_max_iter 10, ir_tol 1e-10, solve_graph 1, learned 0,
 * model_path NULL, timing_kernels 0, tune_path NULL, refactor 0, quadrature 0, tree 0,
 * leaf_size 4, eta 1. */
void pmx_options_default(pmx_options* o);

/* Builds the plan and the whole compressed factorisation on `hip_stream`.  Returns when
 * the factor is complete (the call synchronises the stream).  *out is owned by the
 * caller and released by pmx_factor_destroy.  Errors: PMX_EINVAL (bad sizes, odd or
 * small n_j, NaN, non-positive wavenumber), PMX_EGEOM (shared grid cells, coincident centres),
 * PMX_ENOMEM, PMX_EHIP, PMX_ESINGULAR. */
pmx_status pmx_factor_create(const pmx_geometry* geom, const pmx_options* opts, void* hip_stream,
                             pmx_factor** out);

/* Densities for plane waves u^I = exp(i k_ext (cos a, sin a).x) (Sec. 4): dens is device
 * memory [nrhs][2 * node_off[m]] of pmx_c64; column r holds, per inclusion j, q_j at its
 * nodes followed by u_j at its nodes (Sec. 2.2).  angles is host memory [nrhs]. */
pmx_status pmx_solve_plane_waves(pmx_factor* f, int32_t nrhs, const double* angles, pmx_c64* dens,
                                 void* hip_stream);

/* Densities for a general right-hand side f (device, same layout as dens, holding
 * (-u^I_j; -q^I_j) per inclusion).  f and dens may not overlap.
 * Both solves: with precision 1 or 2, PMX_ENOTCONV when refinement stops above ir_tol (dens
 * then holds the last iterate). */
pmx_status pmx_solve(pmx_factor* f, int32_t nrhs, const pmx_c64* rhs, pmx_c64* dens, void* hip_stream);

/* Far-field pattern u_inf(theta) of the scattered field, u^S ~ e^{ikr}/sqrt(r) u_inf:
 * out (device) [nrhs][ndir]; dirs host [ndir] angles; dens device as above. */
pmx_status pmx_far_field(const pmx_factor* f, int32_t nrhs, const pmx_c64* dens, int32_t ndir,
                         const double* dirs, pmx_c64* out, void* hip_stream);

/* pmx_far_field without any device allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and result as pmx_far_field.  The partial sums of
 * its split node sum live in a static array of 8 MiB per GPU, held by every GPU the
 * library runs on until the process ends; it holds at most 524288 (right-hand side,
 * direction) pairs, fewer when the node sum is split (small nrhs * ndir), and larger
 * requests return PMX_EINVAL before any GPU work.  Calls no hipMalloc or hipFree and does
 * not synchronise: the result is complete in stream order.  All calls on one GPU share the
 * array: calls that overlap on one GPU (different streams or threads without ordering)
 * race and may return wrong values; calls ordered on one stream do not.  Errors:
 * PMX_EINVAL, PMX_EHIP. */
pmx_status pmx_far_field_noalloc(const pmx_factor* f, int32_t nrhs, const pmx_c64* dens, int32_t ndir,
                                 const double* dirs, pmx_c64* out, void* hip_stream);

pmx_status pmx_factor_info(const pmx_factor* f, pmx_info* info);

/* Factors again for new interior media of the same inclusions.  In the PMCHWT-Omit system
 * (Sec. 2) the off-diagonal blocks, and with them every interpolative decomposition
 * (skeletons, interpolation matrices, ranks) and every size, use the exterior kernels
 * alone; only the self blocks depend on the interior media.  This call replays the
 * numeric phase of the factorisation kept at create (options.refactor = 1): self blocks,
 * Schur complements, parent blocks and the top LU, the same launches on the same device
 * buffers, as one HIP graph captured at the first call, followed by one wait for the
 * LU pivot checks.  k_int (host, [m]) > 0; eps_int (host, [m]) or NULL for
 * eps_ext (k_int / k_ext)^2.  Later solves use the new media, and give bit for bit what a
 * factor created with them gives.  Ordered after earlier work on hip_stream and on the
 * factor's solves; returns when the factor is complete.  Errors: PMX_EINVAL (factor
 * created without options.refactor, bad values), PMX_EHIP, PMX_ESINGULAR. */
pmx_status pmx_factor_refactor(pmx_factor* f, const double* k_int, const double* eps_int, void* hip_stream);

/* Autotuner of the launch parameters of the batched form.  Launches whose kernel has
 * alternatives (the LU panel kernel, the column-pivoted QR variant, the level-solve
 * variant, the dense apply's right-hand-side grouping and source splits) look their
 * choice up in a table keyed by the real type and size buckets of the launch; without a
 * table (or for a key it lacks) a built-in rule applies.  This call builds such a table
 * for a workload: it factors geom with opts (their timing, graph and table settings
 * ignored) and solves nrhs plane waves (angles 2 pi j / nrhs) while recording every
 * tunable launch shape, then times every candidate of every recorded shape on device
 * buffers of that shape (fixed seeded fills; best of reps timed runs after one warm-up;
 * the apply on the factor's own state, within a 30 s budget) and writes the fastest per
 * key to the text file `path` ("knob real_bytes a b c choice # candidate:us ...").
 * Factors created with options.tune_path = path use it.  nrhs in [1, 256], reps in
 * [1, 50].  Allocates device memory of the factor's size plus the largest timing case. */
pmx_status pmx_autotune(const pmx_geometry* geom, const pmx_options* opts, int32_t nrhs, int32_t reps,
                        const char* path, void* hip_stream);

/* Releases everything the factor holds; accepts NULL.  The factor's device blocks go to
 * a process-wide cache (after a device synchronisation), from which later factors take
 * their blocks before calling hipMalloc; see pmx_device_cache. */
void pmx_factor_destroy(pmx_factor* f);

/* Process-wide cache of device blocks left by destroyed factors (default limit 8 GiB).
 * limit >= 0 sets the limit and frees cached blocks beyond it (0 frees them all); limit < 0
 * keeps it.  held (may be NULL) receives the bytes the cache holds afterwards.  Factors
 * that cannot allocate empty the cache and try again.  limit 0 also frees the idle pinned
 * host chunks that factors stage their uploads in.  Thread-safe.  Errors: none. */
pmx_status pmx_device_cache(int64_t limit, int64_t* held);

/* Learned skeleton proposals (the leaf IDs of Sec. 3 as training labels).
 *
 * Features per leaf node (20): the cell's k+ r_c, k+ R_p, contrast k-/k+, n / 256, near
 * cells / 8, the relative Fourier magnitudes 2..6 of the node radii and mean radius / r_c;
 * the node's direction from the centre, normal, radius / r_c, curvature r_c, speed / r_c,
 * distance to the nearest near-cell node / r_c and to the proxy circle / r_c.
 * Outputs per node (8): skeleton logits of the four IDs (column q, column u, row value,
 * row derivative) and the four ranks as fractions k / n. */
typedef struct {
  int32_t epochs, batch;   /* passes over the training set; samples (nodes) per step */
  int32_t hidden, layers;  /* hidden width and number of hidden layers (ReLU) */
  float lr, wmse;          /* Adam step size; weight of the rank squared error */
  uint64_t seed;           /* initial weights and sample order */
} pmx_mlp_opts;

/* epochs 30, batch 4096, hidden 256, layers 3, lr 1e-3, wmse 10, seed 1 */
void pmx_mlp_opts_default(pmx_mlp_opts* o);

/* Runs the full leaf IDs of a geometry (plain FP64 path) and writes (append = 0) or appends
 * (append = 1) one training sample per leaf node to the file at path: features and labels
 * (membership of the node in the skeleton of each of the four IDs, and k / n). */
pmx_status pmx_id_dataset(const pmx_geometry* geom, const pmx_options* opts, const char* path, int32_t append,
                          void* hip_stream);

/* Trains the network on a training file with Adam (binary cross entropy on the logits,
 * wmse times squared error on the rank fractions, inputs standardised by the file's mean
 * and deviation) on the device and writes it to model_path; *final_loss (may be NULL) is
 * the mean loss of the last epoch. */
pmx_status pmx_mlp_train(const char* data_path, const pmx_mlp_opts* opts, const char* model_path, double* final_loss,
                         void* hip_stream);

/* The network's outputs for every boundary node of a geometry: out (host) [node][8]. */
pmx_status pmx_mlp_predict(const char* model_path, const pmx_geometry* geom, const pmx_options* opts, float* out,
                           void* hip_stream);

const char* pmx_status_string(pmx_status s);
const char* pmx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
