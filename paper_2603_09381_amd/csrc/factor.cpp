// Host orchestration of the recursive proxy solver (arXiv 2603.09381, Sec. 3) and the
// C-ABI of include/pmx.h and include/pmx_probe.h.
//
// Factorisation, level by level from the leaves (one inclusion per cell) to the root:
//   1. D_tau: the self block A_ii at the leaves; at a parent the block of the compressed
//      system gathered from the children (their At on the diagonal, kernel entries
//      between different children's skeletons off it, Sec. 3 multi-level remark).
//   2. Four interpolative decompositions per cell (q columns, u columns, value rows,
//      derivative rows): matrices of the cell's active columns against the near cells'
//      active rows plus proxy rows (and the transposed row versions), exterior kernel
//      only (the Omit property); Householder QR, then column-pivoted QR with the
//      threshold |R_jj| > tol |R_11|; pairs (q, value) and (u, derivative) keep the
//      larger of their two ranks; T = R11^-1 R12.
//   3. Schur step: LU(D), Y = D^-1 L, M = R Y, At = M^-1 (At = (R A^-1 L)^-1 of Sec. 3).
//   4. Skeleton rows and columns become the parent's active sets.
// The top system is factored by partial-pivoted LU (Sec. 4).  The solve runs the
// upward pass (y = D^-1 f, g = At R y), the root solve and the downward recovery
// x = y - Y (g - At psi), the recovery formula of Sec. 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pmx.h"
#include "../../include/pmx_probe.h"
#include "assemble.h"
#include "zeta_table.h"
#include "la.h"
#include "learn.h"
#include "plan.h"
#include "ktimer.h"
#include "tune.h"

thread_local KernelTimer* g_ktimer = nullptr;

namespace {
thread_local int64_t g_launches = 0, g_syncs = 0;
}
void pmx_count_launch() { ++g_launches; }
void pmx_count_sync() { ++g_syncs; }

namespace {

thread_local std::string g_last_error;

struct PmxErr {
  pmx_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) throw PmxErr{PMX_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

void fail(pmx_status st, const std::string& msg) { throw PmxErr{st, msg}; }

// Device blocks kept for reuse within one factorisation: the per-level temporaries of the
// factorisation are released level by level; giving their blocks back to hipFree would
// synchronise the device each time, and hipMalloc them anew costs host time.  Blocks come
// in size classes of one eighth of an octave (at least 256 bytes) and are reused only by
// later work of the same stream (the factorisation's), so stream order protects them.
// Host staging buffers of uploads are kept as well (an asynchronous copy may still read
// them).  Everything is freed when the pool is destroyed, after the stream is idle.
// Device blocks of destroyed factors, kept for later factors of the process so that a
// factorisation in steady state calls no hipMalloc: at most g_cache_limit bytes, blocks
// keyed by size class.  A block enters the cache only after the device has finished the
// work of the factor that held it.
std::mutex g_cache_mu;
std::map<size_t, std::vector<void*>> g_cache;
size_t g_cache_bytes = 0;
size_t g_cache_limit = (size_t)8 << 30;

void* cache_take(size_t c) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(c);
  if (it == g_cache.end() || it->second.empty()) return nullptr;
  void* p = it->second.back();
  it->second.pop_back();
  g_cache_bytes -= c;
  return p;
}

// frees cached blocks until at most `keep` bytes remain; returns the bytes freed
size_t cache_trim(size_t keep) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  size_t freed = 0;
  for (auto it = g_cache.rbegin(); it != g_cache.rend() && g_cache_bytes > keep; ++it)
    while (!it->second.empty() && g_cache_bytes > keep) {
      (void)hipFree(it->second.back());
      it->second.pop_back();
      g_cache_bytes -= it->first;
      freed += it->first;
    }
  return freed;
}

// Pinned host chunks for the staging of uploads, shared by the process.  An asynchronous
// copy from pageable memory waits for the stream to reach it, which takes away the host's
// lead over the device at every upload; from pinned memory it is queued like a kernel.  A
// factor's pool takes chunks as it needs them and gives them back when it is destroyed,
// after the device has finished every copy that reads them.
std::mutex g_pin_mu;
std::vector<std::pair<void*, size_t>> g_pin_free;
constexpr size_t PIN_CHUNK = (size_t)4 << 20;

std::pair<void*, size_t> pin_take(size_t n) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (size_t i = 0; i < g_pin_free.size(); ++i)
      if (g_pin_free[i].second >= n) {
        const auto c = g_pin_free[i];
        g_pin_free.erase(g_pin_free.begin() + (ptrdiff_t)i);
        return c;
      }
  }
  const size_t sz = (n + PIN_CHUNK - 1) / PIN_CHUNK * PIN_CHUNK;
  void* p = nullptr;
  if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return {nullptr, 0};
  }
  return {p, sz};
}

void pin_give(std::vector<std::pair<void*, size_t>>& v) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  for (const auto& c : v) g_pin_free.push_back(c);
  v.clear();
}

// Device blocks of one factor.  Temporary buffers of the factorisation are released level
// by level; giving their blocks back to hipFree would synchronise the device each time,
// and hipMalloc them anew costs host time.  Blocks come in size classes of one eighth of
// an octave (at least 256 bytes) and are reused by later work of the factor, in stream
// order: the factorisation's stream, then the solve stream, which waits for it.  Host
// staging buffers of uploads are kept as well (an asynchronous copy may still read them).
// When the pool is destroyed, the device is synchronised and the blocks go to the
// process cache (beyond its limit, to hipFree).
class DevPool {
 public:
  ~DevPool() {
    if (free_.empty() && pin_.empty()) return;
    (void)hipDeviceSynchronize();
    pin_give(pin_);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto& kv : free_)
      for (void* p : kv.second) {
        if (g_cache_bytes + kv.first <= g_cache_limit) {
          g_cache[kv.first].push_back(p);
          g_cache_bytes += kv.first;
        } else {
          (void)hipFree(p);
        }
      }
  }
  static size_t size_class(size_t n) {
    if (n <= 256) return 256;
    size_t oct = 1;
    while (oct * 2 <= n) oct *= 2;
    const size_t step = std::max<size_t>(oct / 8, 256);
    return (n + step - 1) / step * step;
  }
  void* get(size_t n) {
    const size_t c = size_class(n);
    auto it = free_.find(c);
    if (it != free_.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      return p;
    }
    if (void* p = cache_take(c)) return p;
    void* p = nullptr;
    if (hipMalloc(&p, c) != hipSuccess) {
      (void)hipGetLastError();
      // what is missing may be held by the cached blocks of earlier factors or by this
      // pool's idle blocks of other sizes: free both (after the device has finished with
      // them) and try once more
      cache_trim(0);
      release_idle();
      if (hipMalloc(&p, c) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    return p;
  }
  void release_idle() {
    if (free_.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipFree(p);
    free_.clear();
  }
  void put(void* p, size_t n) { free_[size_class(n)].push_back(p); }
  void retire(std::vector<std::vector<char>>& host) {
    for (auto& h : host) retired_.push_back(std::move(h));
    host.clear();
  }
  // a pinned copy of n bytes of src, kept until the pool is destroyed; nullptr when no
  // pinned memory can be had
  const void* stage(const void* src, size_t n) {
    const size_t n16 = (n + 15) / 16 * 16;
    if (pin_.empty() || pin_used_ + n16 > pin_.back().second) {
      const auto c = pin_take(n16);
      if (!c.first) return nullptr;
      pin_.push_back(c);
      pin_used_ = 0;
    }
    char* d = (char*)pin_.back().first + pin_used_;
    std::memcpy(d, src, n);
    pin_used_ += n16;
    return d;
  }

 private:
  std::map<size_t, std::vector<void*>> free_;
  std::vector<std::vector<char>> retired_;
  std::vector<std::pair<void*, size_t>> pin_;
  size_t pin_used_ = 0;
};

// Device allocations owned by one object, released together (to a pool when it has one).
class Arena {
 public:
  Arena() = default;
  explicit Arena(DevPool* pool) : pool_(pool) {}
  ~Arena() { release(); }
  void set_pool(DevPool* pool) {
    release();
    pool_ = pool;
  }
  template <class T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    if (pool_) {
      p = pool_->get(n * sizeof(T));
      if (!p) fail(PMX_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    } else {
      hipError_t e = hipMalloc(&p, n * sizeof(T));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(PMX_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
      }
    }
    ptrs_.push_back(p);
    sizes_.push_back(n * sizeof(T));
    bytes_ += n * sizeof(T);
    return (T*)p;
  }
  // The host data is copied into storage owned by the arena, so the asynchronous copy
  // never reads a buffer the caller has already released.
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) {
      const size_t nb = v.size() * sizeof(T);
      const void* src = pool_ ? pool_->stage(v.data(), nb) : nullptr;
      if (!src) {
        keep_.emplace_back((const char*)v.data(), (const char*)v.data() + nb);
        src = keep_.back().data();
      }
      HIPCHK(hipMemcpyAsync(p, src, nb, hipMemcpyHostToDevice, s));
    }
    return p;
  }
  void release() {
    if (pool_) {
      for (size_t i = 0; i < ptrs_.size(); ++i) pool_->put(ptrs_[i], sizes_[i]);
      pool_->retire(keep_);
    } else {
      for (void* p : ptrs_) (void)hipFree(p);
    }
    ptrs_.clear();
    sizes_.clear();
    keep_.clear();
    bytes_ = 0;
  }
  double bytes() const { return (double)bytes_; }

 private:
  DevPool* pool_ = nullptr;
  std::vector<void*> ptrs_;
  std::vector<size_t> sizes_;
  std::vector<std::vector<char>> keep_;
  size_t bytes_ = 0;
};

template <class T>
void download(std::vector<T>& v, const T* d, size_t n, hipStream_t s) {
  v.resize(n);
  if (n) HIPCHK(hipMemcpyAsync(v.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  pmx_count_sync();
  HIPCHK(hipStreamSynchronize(s));
}

void sync_check(hipStream_t s) {
  HIPCHK(hipGetLastError());
  pmx_count_sync();
  HIPCHK(hipStreamSynchronize(s));
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Data kept for one compressed level, in the factor's real type R.
template <class R>
struct LevelData {
  int ncell = 0;
  std::vector<int> s0, s1, k0, k1;            // active sizes and skeleton sizes per type
  std::vector<int64_t> offD, offY, offA, offT, offS, offK;
  std::vector<int> cpiv;                      // column-ID pivots, per cell [s0 | s1]
  std::vector<int64_t> offP;                  // offsets into cpiv (= offS)
  // active codes (rows, cols) and skeleton codes, host
  std::vector<int> rows, cols;                // concatenated per cell, offsets offS
  std::vector<int> rskel, cskel;              // concatenated per cell, offsets offK
  std::vector<std::vector<int>> children;     // plan children (only for the parent level)
  cx<R>* D = nullptr;                         // LU of D per cell
  int* ipiv = nullptr;
  int* perm = nullptr;                        // row permutations of the LUs
  cx<R>* Y = nullptr;                         // D^-1 L, s x K
  cx<R>* At = nullptr;                        // K x K
  cx<R>* Tc = nullptr;                        // column-ID T blocks, [k0 x (s0-k0)] then [k1 x (s1-k1)]
  LuDescT<R>* d_lu = nullptr;
  int max_s = 0, max_k = 0;
  int64_t tot_s = 0, tot_k = 0;
};

// Buffers and device launch descriptors of one level of a solve pass.
template <class R>
struct SolveLevel {
  cx<R>* F = nullptr;        // y / f vectors, sum s x nrhs
  cx<R>* G = nullptr;        // K x nrhs
  cx<R>* Red = nullptr;      // redundant rows
  cx<R>* Ry = nullptr;       // copy of R y
  cx<R>* W = nullptr;        // substitution workspace
  cx<R>* Psi = nullptr;      // parent solution rows of each cell
  MatT<R>* d_bm = nullptr;   // y = D^-1 f
  MatT<R>* d_w = nullptr;    // its workspace
  GatherDescT<R>* d_up = nullptr;    // R y: skeleton and redundant rows
  int n_up = 0, max_up = 0;
  GemmArgsT<R>* d_ga = nullptr;      // + T * redundant rows
  int n_ga = 0;
  GemmArgsT<R>* d_gb = nullptr;      // g = At (R y)
  GatherDescT<R>* d_par = nullptr;   // parent right-hand sides
  int n_par = 0, max_par = 0;
  GatherDescT<R>* d_psi = nullptr;   // psi gathers
  GemmArgsT<R>* d_g1 = nullptr;      // g -= At psi
  GemmArgsT<R>* d_g2 = nullptr;      // x = y - Y g
  int64_t tot_k = 0;
};

template <class R>
struct SolveProgram {
  int nrhs = -1;
  std::vector<SolveLevel<R>> lv;
  cx<R>* Froot = nullptr;
  cx<R>* leaf = nullptr;     // leaf vectors: input and output of a pass
  MatT<R>* d_bm_root = nullptr;
  MatT<R>* d_w_root = nullptr;
  zd *Wroot64 = nullptr, *Yroot64 = nullptr;   // top right-hand sides and solution in FP64
  GemmArgsT<double>* d_root_gemm = nullptr;    // Yroot64 = Ainv_root Wroot64
  Arena arena;
};

// The compressed factorisation in one real type: levels, top system and solve buffers.
template <class R>
struct Tier {
  std::vector<LevelData<R>> lev;
  int root_s = 0;
  cx<R>* Droot = nullptr;
  int* ipiv_root = nullptr;
  int* perm_root = nullptr;
  LuDescT<R>* d_lu_root = nullptr;
  // refined forms: the FP64 inverse of the top system's LU factors, so that each of the many
  // solves of a refinement takes one product instead of two sequential triangular sweeps
  zd* Ainv_root = nullptr;
  std::vector<int> root_rows, root_cols;
  SolveProgram<R> prog;
};

struct SolveState;
namespace {
struct ApplyGeo;
}

// The numeric phase of a factorisation kept for replays (options.refactor = 1): every
// launch after the interpolative decompositions, bound to device buffers and descriptors
// that live as long as the factor.  In the Omit form (Sec. 2) the IDs see exterior
// kernels only, so skeletons, interpolation matrices, ranks and every size stay valid
// when the interior media change; the self blocks, Schur complements, parent blocks and
// the top LU are what a replay recomputes.
struct NumProgram {
  bool on = false;
  std::vector<std::function<void(hipStream_t)>> steps;
  std::vector<std::pair<const int*, int>> infos;   // LU pivot checks (device arrays)
  struct Diag {                                     // self-block descriptors (interior media)
    std::vector<DiagDesc> host;
    DiagDesc* dev;
    std::vector<int> incl;
  };
  std::vector<Diag> diags;
  hipGraphExec_t graph = nullptr;
  int64_t nodes = 0;
  void add(std::function<void(hipStream_t)> f) {
    if (on) steps.push_back(std::move(f));
  }
  ~NumProgram() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

// Leaves of several inclusions: the largest first level accepted.  Batches of up to 324
// such leaves are verified; one of 1,231 leaves ended in a device memory fault whose cause
// is not known, so larger ones are refused.
#define PMX_MAX_MULTI_LEAVES 512

struct pmx_factor {
  // reuse of the factorisation's temporary device blocks (declared first: destroyed last)
  DevPool pool;
  // geometry (device)
  int m = 0, n_nodes = 0;
  double k_ext = 0, eps_ext = 1;
  std::vector<int64_t> node_off;
  std::vector<double> k_int, eps_int;
  double *x, *y, *nx, *ny, *w, *speed, *kappa;
  int* owner = nullptr;
  int64_t* d_node_off = nullptr;
  pmx_options opts;
  int lev0 = 0;   // plan level of the first compressed cells (1: leaves of several inclusions)
  std::vector<std::vector<CellPlan>> plan;
  Tier<double> t64;   // precision 0
  Tier<float> t32;    // precision 1
  // refined forms: the FP64 self blocks of the inclusions (inclusion order, offsets
  // selfOff) for the refinement residual
  zd* Dself = nullptr;
  std::vector<int> selfIncl;
  std::vector<int64_t> selfOff;
  Arena arena;
  pmx_info info;
  // solves: own stream (captured graphs), ordering events, per right-hand-side-count state
  hipStream_t gs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::unique_ptr<SolveState> ss;
  // learned leaf IDs: the network's outputs per leaf node (PMX_NOUT x nodes, leaf order)
  std::vector<float> leaf_pred;
  // launch-parameter table of options.tune_path (NULL: built-in rules)
  std::unique_ptr<TuneTable> tune;
  // options.refactor = 1: the numeric phase as a replayable launch sequence
  NumProgram num;
  // refined forms: the operator apply's geometry (tree walk per target wave), built on a
  // host thread while the device factors; read by the first solve
  std::future<std::shared_ptr<ApplyGeo>> apply_geo;
  pmx_factor() : arena(&pool) {
    t64.prog.arena.set_pool(&pool);
    t32.prog.arena.set_pool(&pool);
  }
  ~pmx_factor();
  DevGeom geom() const { return DevGeom{x, y, nx, ny, w, speed, kappa, n_nodes}; }
  ExtParams ext() const { return ExtParams{k_ext, eps_ext}; }
};

template <class R>
Tier<R>& tier(pmx_factor* F);
template <>
Tier<double>& tier<double>(pmx_factor* F) {
  return F->t64;
}
template <>
Tier<float>& tier<float>(pmx_factor* F) {
  return F->t32;
}

namespace {

// One launch step of the numeric phase: run now, and kept when the factor keeps its
// numeric program.  f takes the stream and may hold only values and device pointers that
// outlive the factor's creation.
template <class Fn>
void num_step(pmx_factor* F, hipStream_t s, Fn f) {
  f(s);
  F->num.add(std::function<void(hipStream_t)>(f));
}

// Device memory of the numeric phase: the factor's own arena when the program is kept,
// else the level's temporaries.
inline Arena& num_arena(pmx_factor* F, Arena& tmp) { return F->num.on ? F->arena : tmp; }

void validate(const pmx_geometry* g, const pmx_options* o) {
  if (!g) fail(PMX_EINVAL, "geometry is NULL");
  if (g->m <= 0) fail(PMX_EINVAL, "m must be positive");
  if (!g->node_off || !g->x || !g->y || !g->dx || !g->dy || !g->ddx || !g->ddy || !g->center || !g->k_int)
    fail(PMX_EINVAL, "a required geometry array is NULL");
  if (!(g->k_ext > 0) || !std::isfinite(g->k_ext)) fail(PMX_EINVAL, "k_ext must be positive");
  if (!(g->eps_ext > 0)) fail(PMX_EINVAL, "eps_ext must be positive");
  if (g->node_off[0] != 0) fail(PMX_EINVAL, "node_off[0] must be 0");
  for (int j = 0; j < g->m; ++j) {
    int64_t n = g->node_off[j + 1] - g->node_off[j];
    if (n < 8 || (n & 1)) fail(PMX_EINVAL, "inclusion " + std::to_string(j) + ": node count must be even and >= 8");
    if (!(g->k_int[j] > 0) || !std::isfinite(g->k_int[j])) fail(PMX_EINVAL, "k_int must be positive");
    if (g->eps_int && !(g->eps_int[j] > 0)) fail(PMX_EINVAL, "eps_int must be positive");
  }
  int64_t N = g->node_off[g->m];
  if (N > (int64_t)1 << 29) fail(PMX_EINVAL, "too many nodes");
  for (int64_t i = 0; i < N; ++i) {
    double v[6] = {g->x[i], g->y[i], g->dx[i], g->dy[i], g->ddx[i], g->ddy[i]};
    for (double t : v)
      if (!std::isfinite(t)) fail(PMX_EINVAL, "non-finite node data");
    if (g->dx[i] == 0.0 && g->dy[i] == 0.0) fail(PMX_EINVAL, "zero tangent");
  }
  if (o) {
    if (!(o->id_tol > 0) || o->id_tol >= 1) fail(PMX_EINVAL, "id_tol must be in (0, 1)");
    if (!(o->proxy_ratio > 1.0)) fail(PMX_EINVAL, "proxy_ratio must exceed 1");
    if (o->proxy_rule == 1 && o->proxy_min < 8) fail(PMX_EINVAL, "a fixed proxy count must be >= 8");
    if (o->precision < 0 || o->precision > 2) fail(PMX_EINVAL, "precision must be 0, 1 or 2");
    if (o->precision == 1 && o->id_tol < 1e-6)
      fail(PMX_EINVAL, "precision 1 needs id_tol >= 1e-6: FP32 column norms cannot resolve smaller ratios");
    if (o->precision != 0) {
      if (o->ir_max_iter < 1 || o->ir_max_iter > 100) fail(PMX_EINVAL, "ir_max_iter must be in [1, 100]");
      if (!(o->ir_tol > 0) || o->ir_tol >= 1) fail(PMX_EINVAL, "ir_tol must be in (0, 1)");
    }
    if (o->quadrature != 0 && o->quadrature != 1) fail(PMX_EINVAL, "quadrature must be 0 or 1");
    if (o->near_rule < 0 || o->near_rule > 2) fail(PMX_EINVAL, "near_rule must be 0, 1 or 2");
    if (o->near_rule == 2 && !(o->eta > 0 && std::isfinite(o->eta))) fail(PMX_EINVAL, "eta must be positive");
    if (o->tree != 0 && o->tree != 1) fail(PMX_EINVAL, "tree must be 0 or 1");
    if (o->tree == 1) {
      if (o->leaf_size < 1 || o->leaf_size > 4) fail(PMX_EINVAL, "leaf_size must be in 1..4");
      if (o->near_rule == 0) fail(PMX_EINVAL, "the k-means tree needs near_rule 1 or 2 (no grid adjacency)");
      if (o->learned) fail(PMX_EINVAL, "learned proposals need the grid quadtree (tree 0)");
    }
    if (o->quadrature == 1)
      for (int j = 0; j < g->m; ++j)
        if (g->node_off[j + 1] - g->node_off[j] < 2 * PMX_ZETA_P + 2)
          fail(PMX_EINVAL, "the zeta-corrected rule needs at least 2 * 20 + 2 nodes per inclusion");
  }
}

PlanOptions plan_options(const pmx_geometry* g, const pmx_options& o) {
  PlanOptions p;
  p.proxy_ratio = o.proxy_ratio;
  p.proxy_min = o.proxy_min;
  p.near_rule = o.near_rule;
  p.proxy_rule = o.proxy_rule;
  p.id_tol = o.id_tol;
  p.k_ext = g->k_ext;
  p.tree = o.tree;
  p.leaf_size = o.leaf_size;
  p.eta = o.eta;
  return p;
}

void make_plan(const pmx_geometry* g, const pmx_options& o, std::vector<std::vector<CellPlan>>& levels) {
  std::string err = build_plan(g->m, g->grid_ij, g->center, g->node_off, g->x, g->y, plan_options(g, o), levels);
  if (!err.empty()) fail(PMX_EGEOM, err);
}

void upload_geometry(pmx_factor* F, const pmx_geometry* g, hipStream_t s) {
  F->m = g->m;
  F->node_off.assign(g->node_off, g->node_off + g->m + 1);
  F->n_nodes = (int)F->node_off.back();
  F->k_ext = g->k_ext;
  F->eps_ext = g->eps_ext;
  F->k_int.assign(g->k_int, g->k_int + g->m);
  F->eps_int.resize(g->m);
  for (int j = 0; j < g->m; ++j)
    F->eps_int[j] = g->eps_int ? g->eps_int[j] : g->eps_ext * (g->k_int[j] / g->k_ext) * (g->k_int[j] / g->k_ext);
  const int N = F->n_nodes;
  Arena& A = F->arena;
  std::vector<int> owner(N);
  for (int j = 0; j < g->m; ++j)
    for (int64_t i = g->node_off[j]; i < g->node_off[j + 1]; ++i) owner[i] = j;
  auto up = [&](const double* h) {
    double* d = A.alloc<double>(N);
    HIPCHK(hipMemcpyAsync(d, h, N * sizeof(double), hipMemcpyHostToDevice, s));
    return d;
  };
  F->x = up(g->x);
  F->y = up(g->y);
  double* dx = up(g->dx);
  double* dy = up(g->dy);
  double* ddx = up(g->ddx);
  double* ddy = up(g->ddy);
  F->owner = A.upload(owner, s);
  F->d_node_off = A.upload(F->node_off, s);
  F->nx = A.alloc<double>(N);
  F->ny = A.alloc<double>(N);
  F->w = A.alloc<double>(N);
  F->speed = A.alloc<double>(N);
  F->kappa = A.alloc<double>(N);
  asm_geometry(dx, dy, ddx, ddy, F->owner, F->d_node_off, F->nx, F->ny, F->w, F->speed, F->kappa, N, s);
  sync_check(s);
}

// Kress / differentiation tables for the distinct node counts.
struct Tables {
  std::map<int, int> off;   // n -> offset
  double *R = nullptr, *dt = nullptr;
};

Tables make_tables(Arena& A, const std::vector<int>& ns_all, int quad, hipStream_t s) {
  Tables T;
  std::vector<int> ns, offs;
  int tot = 0, maxn = 0;
  for (int n : ns_all)
    if (!T.off.count(n)) {
      T.off[n] = tot;
      ns.push_back(n);
      offs.push_back(tot);
      tot += n;
      maxn = std::max(maxn, n);
    }
  T.R = A.alloc<double>(tot);
  T.dt = A.alloc<double>(tot);
  int* d_ns = A.upload(ns, s);
  int* d_off = A.upload(offs, s);
  asm_tables(d_ns, d_off, (int)ns.size(), maxn, T.R, T.dt, quad, s);
  return T;
}

// Leaf self blocks for the given inclusions into out[off_i], ld 2 n_i.
void assemble_diag(pmx_factor* F, Arena& tmp_, const std::vector<int>& incl, zd* D,
                   const std::vector<int64_t>& offD, hipStream_t s) {
  Arena& tmp = num_arena(F, tmp_);
  std::vector<int> ns;
  for (int j : incl) ns.push_back((int)(F->node_off[j + 1] - F->node_off[j]));
  Tables T = make_tables(tmp, ns, F->opts.quadrature, s);
  int64_t scr = 0;
  int maxn = 0;
  for (int n : ns) {
    scr += (int64_t)n * n;
    maxn = std::max(maxn, n);
  }
  zd* s1 = tmp.alloc<zd>(scr);
  zd* s2 = tmp.alloc<zd>(scr);
  std::vector<DiagDesc> dd(incl.size());
  int64_t so = 0;
  for (size_t t = 0; t < incl.size(); ++t) {
    int j = incl[t];
    DiagDesc& d = dd[t];
    d.node0 = (int)F->node_off[j];
    d.n = ns[t];
    d.k_int = F->k_int[j];
    d.eps_int = F->eps_int[j];
    d.tbl = T.off[d.n];
    d.out = D + offD[t];
    d.scratch = s1 + so;
    d.scratch2 = s2 + so;
    so += (int64_t)d.n * d.n;
  }
  DiagDesc* d_dd = tmp.upload(dd, s);
  const DevGeom g = F->geom();
  const ExtParams e = F->ext();
  const int cnt = (int)incl.size();
  const double *tr = T.R, *tdt = T.dt;
  num_step(F, s, [=](hipStream_t st) { asm_diag(g, e, d_dd, cnt, maxn, tr, tdt, st); });
  if (F->num.on) F->num.diags.push_back(NumProgram::Diag{dd, d_dd, incl});
}

// FP64 self blocks of every inclusion in inclusion order (the refined forms keep them for
// the residual); they need the geometry but not the plan
void self_blocks_by_inclusion(pmx_factor* F, hipStream_t s) {
  const double t0 = now_ms();
  std::vector<int> incl(F->m);
  std::vector<int64_t> off(F->m);
  int64_t td = 0;
  for (int j = 0; j < F->m; ++j) {
    incl[j] = j;
    off[j] = td;
    const int64_t n = F->node_off[j + 1] - F->node_off[j];
    td += 4 * n * n;
  }
  F->Dself = F->arena.alloc<zd>(td);
  F->selfIncl = incl;
  F->selfOff = off;
  Arena tmp(&F->pool);
  assemble_diag(F, tmp, incl, F->Dself, off, s);
  HIPCHK(hipGetLastError());
  F->info.t_phase_ms[0] += now_ms() - t0;
}

struct ProxyTable {
  DevProxy dev{nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<int> off;   // per cell first proxy index
};

ProxyTable make_proxies(Arena& A, const std::vector<CellPlan>& cells, hipStream_t s) {
  ProxyTable P;
  std::vector<double> px, py, pnx, pny, pw;
  for (const CellPlan& c : cells) {
    P.off.push_back((int)px.size());
    for (int k = 0; k < c.P; ++k) {
      double th = 2.0 * M_PI * k / c.P;
      double ct = std::cos(th), st = std::sin(th);
      px.push_back(c.cx + c.Rp * ct);
      py.push_back(c.cy + c.Rp * st);
      pnx.push_back(ct);
      pny.push_back(st);
      pw.push_back(2.0 * M_PI * c.Rp / c.P);
    }
  }
  if (px.empty()) return P;
  P.dev.x = A.upload(px, s);
  P.dev.y = A.upload(py, s);
  P.dev.nx = A.upload(pnx, s);
  P.dev.ny = A.upload(pny, s);
  P.dev.w = A.upload(pw, s);
  return P;
}

// Candidate columns proposed for the leaf IDs: for ID q = 4 t + kind, the column order
// (the first cand[q] are the candidates, best first) over the cell's active columns of the
// ID's type.
struct LearnedPlan {
  std::vector<int> cand;
  std::vector<std::vector<int>> order;
};

// Results of the ID stage of one level, per ID q = 4 t + kind (kinds 0/1: column IDs of
// type 0/1, 2/3: row IDs).  R and the pivots live at fixed offsets; the leading dimension
// of an ID's R is mbq[q] (rows of its CPQR matrix); pivots are original column indices.
template <class R>
struct IdOut {
  std::vector<int> idm, idc, mbq, kq, piv;
  std::vector<int64_t> offR, offC;
  cx<R>* Rb = nullptr;
  int* pivb = nullptr;
  int learned = 0, fallback = 0;
};

// Interpolative decompositions of the four matrices of every cell (Sec. 3): column IDs of
// [A(near rows, cell columns); proxy rows] per column type and row IDs of the transposed
// [A(cell rows, near columns), proxy columns] per row type, exterior kernel only (Omit).
// Full path: Householder QR, column-pivoted QR to the threshold |R_jj| <= tol |R_11|, the
// pairs (q, value) and (u, derivative) take the larger rank, T = R11^-1 R12.  Learned path
// (lp): the matrix is assembled with the proposed candidates first, QR stops after the
// candidates, pivots are chosen among them only, and the result stands when every
// remaining column (the part outside the candidates' span included) is at most
// tol |R_11|, for both IDs of both pairs; other cells take the full path.
template <class R>
void id_stage(pmx_factor* F, const LevelData<R>& L, const std::vector<CellPlan>& cells, const ProxyTable& PT,
              const LearnedPlan* lp, IdOut<R>& io, Arena& tmp, hipStream_t s, bool pairs) {
  const int nc = L.ncell;
  const double tol = F->opts.id_tol;
  // near code lists, built on the device from the level's code arrays (the host only
  // sums their lengths)
  std::vector<int64_t> nro(nc), mid(nc);
  std::vector<int> noff(nc + 1), nidx, poff(nc), np(nc);
  int64_t tot = 0;
  for (int t = 0; t < nc; ++t) {
    nro[t] = tot;
    noff[t] = (int)nidx.size();
    for (int sgm : cells[t].near) {
      nidx.push_back(sgm);
      tot += L.s0[sgm] + L.s1[sgm];
    }
    tot += 2 * (int64_t)cells[t].P;
    poff[t] = PT.off[t];
    np[t] = cells[t].P;
    mid[t] = tot - nro[t];
    if (mid[t] == 0) fail(PMX_EGEOM, "a cell has neither near cells nor a proxy circle");
  }
  noff[nc] = (int)nidx.size();
  int* d_rows = tmp.upload(L.rows, s);
  int* d_cols = tmp.upload(L.cols, s);
  int* d_nr = tmp.alloc<int>(std::max<int64_t>(tot, 1));
  int* d_ncol = tmp.alloc<int>(std::max<int64_t>(tot, 1));
  asm_near_lists(d_rows, d_cols, tmp.upload(L.offS, s), tmp.upload(noff, s), tmp.upload(nidx, s), tmp.upload(nro, s),
                 tmp.upload(poff, s), tmp.upload(np, s), nc, d_nr, d_ncol, s);
  const int nid = 4 * nc;
  io.idm.assign(nid, 0);
  io.idc.assign(nid, 0);
  io.mbq.assign(nid, 0);
  io.kq.assign(nid, 0);
  io.offR.assign(nid, 0);
  io.offC.assign(nid, 0);
  std::vector<int64_t> offM(nid), offV(nid);
  int64_t totM = 0, totR = 0, totV = 0, totC = 0;
  for (int t = 0; t < nc; ++t)
    for (int kd = 0; kd < 4; ++kd) {
      int q = 4 * t + kd;
      int c = (kd & 1) ? L.s1[t] : L.s0[t];
      int m = (int)mid[t];
      io.idm[q] = m;
      io.idc[q] = c;
      offM[q] = totM;
      totM += (int64_t)m * c;
      io.offR[q] = totR;
      totR += (int64_t)std::min(m, c) * c;
      offV[q] = totV;
      totV += la_geqrf_workspace(m);
      io.offC[q] = totC;
      totC += c;
    }
  cx<R>* Mb = tmp.alloc<cx<R>>(totM);
  // R factors (whose T blocks the row interpolation reads) and pivots outlive the level
  // when the numeric phase is kept for replays
  io.Rb = num_arena(F, tmp).alloc<cx<R>>(totR);
  cx<R>* Vb = tmp.alloc<cx<R>>(totV);
  cx<R>* VTb = tmp.alloc<cx<R>>(totV);
  cx<R>* CVb = tmp.alloc<cx<R>>(totC);
  double* taub = tmp.alloc<double>(nid);
  int* d_work = tmp.alloc<int>(1);
  io.pivb = num_arena(F, tmp).alloc<int>(totC);
  double* nrmb = tmp.alloc<double>(2 * totC);
  double* extrab = tmp.alloc<double>(totC);
  int* stb = tmp.alloc<int>(4 * nid);
  double* r11b = tmp.alloc<double>(nid);
  io.piv.assign(totC, 0);
  std::vector<char> done(nc, 0);

  // one pass over the cells `sel`, full or learned; returns per cell whether it stands
  auto pass = [&](const std::vector<int>& sel, bool learned) {
    const int nb = 4 * (int)sel.size();
    std::vector<EntryMatT<R>> em(nb);
    std::vector<QrDescT<R>> qd(nb);
    std::vector<CpqrDescT<R>> cd(nb);
    std::vector<double*> tails(nb);
    std::vector<int> ordcodes;
    std::vector<int64_t> ordoff(nb, 0);
    int maxm = 0, maxc = 0;
    if (learned) {
      for (int i = 0; i < nb; ++i) {
        const int q = 4 * sel[i / 4] + (i % 4), t = q / 4, kd = q % 4, ty = kd & 1;
        const std::vector<int>& src = (kd < 2) ? L.cols : L.rows;
        const int64_t base = L.offS[t] + (ty ? L.s0[t] : 0);
        ordoff[i] = (int64_t)ordcodes.size();
        for (int j : lp->order[q]) ordcodes.push_back(src[base + j]);
      }
    }
    const int* d_ord = learned ? tmp.upload(ordcodes, s) : nullptr;
    // cells of one inclusion with all nodes active (the inclusion level): the node-node rows
    // come from the pair kernel, one Bessel evaluation for the eight entries of a node pair,
    // and the general kernel fills the proxy rows
    const bool fused = pairs && !learned;
    std::vector<LeafPairDescT<R>> lpd;
    int maxa = 0;
    for (int i = 0; i < nb; ++i) {
      const int q = 4 * sel[i / 4] + (i % 4), t = q / 4, kd = q % 4, ty = kd & 1;
      const int m = io.idm[q], c = io.idc[q];
      const int kc = learned ? std::min(std::min(m, c), lp->cand[q]) : std::min(m, c);
      EntryMatT<R>& e = em[i];
      const int skip = fused ? m - 2 * cells[t].P : 0;   // node rows left to the pair kernel
      e.a = ((kd < 2) ? d_nr : d_ncol) + nro[t] + skip;
      e.na = m - skip;
      e.b = learned ? d_ord + ordoff[i] : ((kd < 2) ? d_cols : d_rows) + L.offS[t] + (ty ? L.s0[t] : 0);
      e.nb = c;
      e.out = Mb + offM[q] + skip;
      e.ld = m;
      e.a_is_target = (kd < 2) ? 1 : 0;
      maxa = std::max(maxa, e.na);
      if (fused && kd == 0) {
        int64_t o = 0;
        for (int sg : cells[t].near) {
          LeafPairDescT<R> d;
          for (int k = 0; k < 4; ++k) d.out[k] = Mb + offM[q + k] + o;
          d.ld = m;
          d.own0 = (int)F->node_off[cells[t].incl[0]];
          d.n_own = L.s0[t];
          d.near0 = (int)F->node_off[cells[sg].incl[0]];
          d.n_near = L.s0[sg];
          lpd.push_back(d);
          o += L.s0[sg] + L.s1[sg];
        }
      }
      QrDescT<R>& Q = qd[i];
      Q.a = Mb + offM[q];
      Q.ld = m;
      Q.m = m;
      Q.c = c;
      Q.r = io.Rb + io.offR[q];
      Q.v = Vb + offV[q];
      Q.t = VTb + offV[q];
      Q.kc = kc;
      CpqrDescT<R>& C = cd[i];
      C.b = io.Rb + io.offR[q];
      C.mb = kc;
      C.c = c;
      C.piv = io.pivb + io.offC[q];
      C.nrm = nrmb + 2 * io.offC[q];
      C.state = stb + 4 * q;
      C.r11 = r11b + q;
      C.v = CVb + io.offC[q];
      C.tau = taub + q;
      C.cpiv = learned ? kc : c;
      C.extra = learned ? extrab + io.offC[q] : nullptr;
      tails[i] = extrab + io.offC[q];
      io.mbq[q] = kc;
      maxm = std::max(maxm, m);
      maxc = std::max(maxc, c);
      la_geqrf_work(m, c, kc, (int)sizeof(R), &F->info.kernel_bytes[PK_TS_UPDATE], &F->info.kernel_flops[PK_TS_UPDATE],
                    &F->info.kernel_bytes[PK_TS_LEAF], &F->info.kernel_flops[PK_TS_LEAF]);
    }
    EntryMatT<R>* d_em = tmp.upload(em, s);
    QrDescT<R>* d_qd = tmp.upload(qd, s);
    CpqrDescT<R>* d_cd = tmp.upload(cd, s);
    asm_entries(F->geom(), PT.dev, F->ext(), d_em, nb, maxa, maxc, s);
    if (!lpd.empty()) asm_leaf_pairs(F->geom(), F->ext(), tmp.upload(lpd, s), (int)lpd.size(), s);
    la_geqrf_r(d_qd, nb, maxm, maxc, s);
    if (learned) la_qr_tail_norms(d_qd, tmp.upload(tails, s), nb, maxc, s);
    HIPCHK(la_cpqr(d_cd, nb, maxc, tol, nullptr, 1, d_work, s));
    std::vector<int> st;
    download(st, stb, 4 * nid, s);
    // common ranks per pair, continuation
    std::vector<int> kb(nb);
    for (int i = 0; i < nb; i += 4)
      for (int ty = 0; ty < 2; ++ty) {
        const int qc = 4 * sel[i / 4] + ty, qr = qc + 2;
        int k = std::max(st[4 * qc + 1], st[4 * qr + 1]);
        const int cap = std::min(io.idc[qc], std::min(io.idm[qc], io.idc[qc]));
        k = std::max(1, std::min(k, cap));
        kb[i + ty] = kb[i + 2 + ty] = k;
      }
    int* d_kb = tmp.upload(kb, s);
    HIPCHK(la_cpqr(d_cd, nb, maxc, 0.0, d_kb, 0, d_work, s));
    download(st, stb, 4 * nid, s);
    std::vector<char> ok(sel.size(), 1);
    if (learned) {
      int* d_acc = tmp.alloc<int>(nb);
      la_cpqr_judge(d_cd, d_kb, tol, d_acc, nb, s);
      std::vector<int> acc;
      download(acc, d_acc, nb, s);
      for (int i = 0; i < nb; ++i)
        if (!acc[i]) ok[i / 4] = 0;
    }
    for (int i = 0; i < nb; i += 4)
      for (int ty = 0; ty < 2; ++ty) {
        const int qc = 4 * sel[i / 4] + ty, qr = qc + 2;
        int k = std::min(kb[i + ty], std::min(st[4 * qc], st[4 * qr]));
        if (learned && k < kb[i + ty]) ok[i / 4] = 0;
        if (k < 1) fail(PMX_ESINGULAR, "an interpolative decomposition has rank 0");
        kb[i + ty] = kb[i + 2 + ty] = k;
        io.kq[qc] = io.kq[qr] = k;
      }
    HIPCHK(hipMemcpyAsync(d_kb, kb.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    la_cpqr_tsolve(d_cd, d_kb, nb, maxc, maxc, s);
    // pivots as original column indices
    std::vector<int> pv;
    download(pv, io.pivb, totC, s);
    for (int i = 0; i < nb; ++i) {
      const int q = 4 * sel[i / 4] + (i % 4);
      const int c = io.idc[q];
      for (int j = 0; j < c; ++j) {
        const int p = pv[io.offC[q] + j];
        io.piv[io.offC[q] + j] = learned ? lp->order[q][p] : p;
      }
    }
    return ok;
  };

  if (lp) {
    std::vector<int> all(nc);
    for (int t = 0; t < nc; ++t) all[t] = t;
    std::vector<char> ok = pass(all, true);
    for (int t = 0; t < nc; ++t) done[t] = ok[t];
  }
  std::vector<int> rest;
  for (int t = 0; t < nc; ++t)
    if (!done[t]) rest.push_back(t);
  io.learned = nc - (int)rest.size();
  io.fallback = lp ? (int)rest.size() : 0;
  if (!rest.empty()) pass(rest, false);
  if (lp) HIPCHK(hipMemcpyAsync(io.pivb, io.piv.data(), totC * sizeof(int), hipMemcpyHostToDevice, s));
}

// Compress one level whose active sets (L.rows, L.cols, s0, s1) and blocks D are set.
template <class R>
void compress_level(pmx_factor* F, LevelData<R>& L, const std::vector<CellPlan>& cells, const LearnedPlan* lp,
                    bool leaf, hipStream_t s) {
  const int nc = L.ncell;
  const double tol = F->opts.id_tol;
  Arena tmp(&F->pool);
  ProxyTable PT = make_proxies(tmp, cells, s);
  // ---- the four interpolative decompositions of every cell (learned proposals first at
  // the leaves when a model is loaded, the full CPQR for every cell they do not settle)
  IdOut<R> io;
  const double ti = now_ms();
  // the inclusion level: cells of one inclusion, all of its nodes active
  id_stage<R>(F, L, cells, PT, lp, io, tmp, s, leaf && F->lev0 == 0);
  if (leaf) F->info.t_phase_ms[7] += now_ms() - ti;   // id_stage ends with its ranks downloaded
  F->info.id_learned += io.learned;
  F->info.id_fallback += io.fallback;
  const std::vector<int>& kq = io.kq;
  const std::vector<int>& idc = io.idc;
  const std::vector<int>& mbq = io.mbq;
  const std::vector<int64_t>& offR = io.offR;
  const std::vector<int64_t>& offC = io.offC;
  const std::vector<int>& piv = io.piv;
  cx<R>* Rb = io.Rb;
  const int* pivb = io.pivb;
  L.k0.assign(nc, 0);
  L.k1.assign(nc, 0);
  for (int t = 0; t < nc; ++t) {
    L.k0[t] = kq[4 * t];
    L.k1[t] = kq[4 * t + 1];
  }
  // ---- level bookkeeping
  L.offK.resize(nc + 1);
  L.offY.resize(nc);
  L.offA.resize(nc);
  L.offT.resize(nc);
  int64_t tk = 0, ty_ = 0, ta = 0, tt = 0;
  L.max_k = 0;
  for (int t = 0; t < nc; ++t) {
    int K = L.k0[t] + L.k1[t];
    int sz = L.s0[t] + L.s1[t];
    L.offK[t] = tk;
    tk += K;
    L.offY[t] = ty_;
    ty_ += (int64_t)sz * K;
    L.offA[t] = ta;
    ta += (int64_t)K * K;
    L.offT[t] = tt;
    tt += (int64_t)L.k0[t] * (L.s0[t] - L.k0[t]) + (int64_t)L.k1[t] * (L.s1[t] - L.k1[t]);
    L.max_k = std::max(L.max_k, K);
  }
  L.offK[nc] = tk;
  L.tot_k = tk;
  L.cpiv.resize(L.tot_s);
  L.rskel.resize(tk);
  L.cskel.resize(tk);
  for (int t = 0; t < nc; ++t) {
    int64_t o = L.offK[t];
    for (int ty = 0; ty < 2; ++ty) {
      const int* pc = piv.data() + offC[4 * t + ty];
      const int* pr = piv.data() + offC[4 * t + 2 + ty];
      int kb = ty ? L.k1[t] : L.k0[t];
      int base = ty ? L.s0[t] : 0;
      int sb = ty ? L.s1[t] : L.s0[t];
      for (int j = 0; j < sb; ++j) L.cpiv[L.offS[t] + base + j] = pc[j];
      for (int i = 0; i < kb; ++i) {
        L.rskel[o + i] = L.rows[L.offS[t] + base + pr[i]];
        L.cskel[o + i] = L.cols[L.offS[t] + base + pc[i]];
      }
      o += kb;
    }
  }
  Arena& A = F->arena;
  L.Y = A.alloc<cx<R>>(ty_);
  L.At = A.alloc<cx<R>>(ta);
  L.Tc = A.alloc<cx<R>>(tt);
  // ---- compact copies of the column-ID T blocks
  {
    std::vector<RowSrc> rs;
    std::vector<GatherDescT<R>> gd;
    std::vector<int64_t> rso;
    int maxr = 0, maxcc = 0;
    for (int t = 0; t < nc; ++t)
      for (int ty = 0; ty < 2; ++ty) {
        int q = 4 * t + ty;
        int kb = kq[q];
        int mb = mbq[q];
        int ncol = idc[q] - kb;
        rso.push_back((int64_t)rs.size());
        for (int i = 0; i < kb; ++i) rs.push_back(RowSrc{offR[q] + i + (int64_t)kb * mb, mb});
        GatherDescT<R> g;
        g.nrows = ncol > 0 ? kb : 0;
        g.ncols = ncol;
        g.dst = L.Tc + L.offT[t] + (ty ? (int64_t)L.k0[t] * (L.s0[t] - L.k0[t]) : 0);
        g.ld = kb;
        gd.push_back(g);
        maxr = std::max(maxr, kb);
        maxcc = std::max(maxcc, ncol);
      }
    RowSrc* d_rs = tmp.upload(rs, s);
    for (size_t i = 0; i < gd.size(); ++i) gd[i].src = d_rs + rso[i];
    GatherDescT<R>* d_gd = tmp.upload(gd, s);
    asm_gather(Rb, d_gd, (int)gd.size(), maxr, maxcc, s);
  }
  // ---- L, LU(D), Y = D^-1 L (from here on the numeric phase: steps kept for replays)
  Arena& NA = num_arena(F, tmp);
  {
    cx<R>* Y = L.Y;
    num_step(F, s, [=](hipStream_t st) { asm_zero(Y, ty_, st); });
  }
  {
    std::vector<LDescT<R>> ld(nc);
    for (int t = 0; t < nc; ++t) {
      LDescT<R>& d = ld[t];
      d.out = L.Y + L.offY[t];
      d.s0 = L.s0[t];
      d.s1 = L.s1[t];
      d.k0 = L.k0[t];
      d.k1 = L.k1[t];
      int q0 = 4 * t + 2, q1 = 4 * t + 3;
      d.piv0 = pivb + offC[q0];
      d.piv1 = pivb + offC[q1];
      int mb0 = mbq[q0], mb1 = mbq[q1];
      d.t0 = Rb + offR[q0] + (int64_t)L.k0[t] * mb0;
      d.t1 = Rb + offR[q1] + (int64_t)L.k1[t] * mb1;
      d.ldt0 = mb0;
      d.ldt1 = mb1;
    }
    LDescT<R>* d_ld = NA.upload(ld, s);
    const int ms = L.max_s, mk = L.max_k;
    num_step(F, s, [=](hipStream_t st) { asm_build_l(d_ld, nc, ms, mk, st); });
  }
  std::vector<LuDescT<R>> lu(nc);
  for (int t = 0; t < nc; ++t) {
    int sz = L.s0[t] + L.s1[t];
    lu[t] = LuDescT<R>{L.D + L.offD[t], sz, sz, L.ipiv + L.offS[t], L.perm + L.offS[t]};
  }
  L.d_lu = A.upload(lu, s);
  int* d_info = NA.alloc<int>(nc);
  {
    const LuDescT<R>* dl = L.d_lu;
    const int ms = L.max_s;
    num_step(F, s, [=](hipStream_t st) {
      asm_zero_i32(d_info, nc, st);
      la_getrf(dl, nc, ms, d_info, st);
    });
  }
  for (int t = 0; t < nc; ++t)
    la_getrf_work(L.s0[t] + L.s1[t], (int)sizeof(R), &F->info.kernel_bytes[PK_GETRF_PANEL], &F->info.kernel_flops[PK_GETRF_PANEL]);
  std::vector<MatT<R>> ym(nc);
  for (int t = 0; t < nc; ++t) {
    int sz = L.s0[t] + L.s1[t];
    ym[t] = MatT<R>{L.Y + L.offY[t], sz, sz, L.k0[t] + L.k1[t]};
  }
  {
    MatT<R>* d_ym = NA.upload(ym, s);
    const LuDescT<R>* dl = L.d_lu;
    const int ms = L.max_s, mk = L.max_k;
    num_step(F, s, [=](hipStream_t st) { la_getrs(dl, d_ym, nc, ms, mk, st); });
  }
  // ---- M = R Y: skeleton rows of Y plus T times its redundant rows
  cx<R>* Mm = NA.alloc<cx<R>>(ta);
  int64_t totred = 0;
  for (int t = 0; t < nc; ++t) totred += (int64_t)(L.s0[t] + L.s1[t] - L.k0[t] - L.k1[t]) * (L.k0[t] + L.k1[t]);
  cx<R>* Red = NA.alloc<cx<R>>(std::max<int64_t>(totred, 1));
  {
    std::vector<RowSrc> rs;
    std::vector<int64_t> rso;
    std::vector<GatherDescT<R>> gd;
    std::vector<GemmArgsT<R>> ga;
    int maxr = 0;
    int64_t ro = 0;
    for (int t = 0; t < nc; ++t) {
      int K = L.k0[t] + L.k1[t];
      int sz = L.s0[t] + L.s1[t];
      // skeleton rows
      rso.push_back((int64_t)rs.size());
      for (int ty = 0; ty < 2; ++ty) {
        int kb = ty ? L.k1[t] : L.k0[t];
        int base = ty ? L.s0[t] : 0;
        for (int i = 0; i < kb; ++i) rs.push_back(RowSrc{L.offY[t] + base + L.cpiv[L.offS[t] + base + i], sz});
      }
      GatherDescT<R> g;
      g.nrows = K;
      g.ncols = K;
      g.dst = Mm + L.offA[t];
      g.ld = K;
      gd.push_back(g);
      maxr = std::max(maxr, K);
      for (int ty = 0; ty < 2; ++ty) {
        int kb = ty ? L.k1[t] : L.k0[t];
        int base = ty ? L.s0[t] : 0;
        int sb = ty ? L.s1[t] : L.s0[t];
        int nr = sb - kb;
        rso.push_back((int64_t)rs.size());
        for (int j = 0; j < nr; ++j) rs.push_back(RowSrc{L.offY[t] + base + L.cpiv[L.offS[t] + base + kb + j], sz});
        GatherDescT<R> h;
        h.nrows = nr;
        h.ncols = K;
        h.dst = Red + ro;
        h.ld = std::max(nr, 1);
        gd.push_back(h);
        maxr = std::max(maxr, nr);
        if (nr > 0) {
          GemmArgsT<R> a;
          a.m = kb;
          a.n = K;
          a.k = nr;
          a.A = L.Tc + L.offT[t] + (ty ? (int64_t)L.k0[t] * (L.s0[t] - L.k0[t]) : 0);
          a.lda = kb;
          a.B = Red + ro;
          a.ldb = nr;
          a.C = Mm + L.offA[t] + (ty ? L.k0[t] : 0);
          a.ldc = K;
          ga.push_back(a);
        }
        ro += (int64_t)nr * K;
      }
    }
    RowSrc* d_rs = NA.upload(rs, s);
    for (size_t i = 0; i < gd.size(); ++i) gd[i].src = d_rs + rso[i];
    GatherDescT<R>* d_gd = NA.upload(gd, s);
    const cx<R>* Y = L.Y;
    const int ngd = (int)gd.size(), mk = L.max_k;
    num_step(F, s, [=](hipStream_t st) { asm_gather(Y, d_gd, ngd, maxr, mk, st); });
    if (!ga.empty()) {
      GemmArgsT<R>* d_ga = NA.upload(ga, s);
      const int nga = (int)ga.size();
      num_step(F, s, [=](hipStream_t st) {
        la_zgemm_list(OP_N, OP_N, d_ga, nga, mk, mk, cmk<R>(1, 0), cmk<R>(1, 0), st);
      });
    }
  }
  // ---- At = M^-1
  int* d_info2 = NA.alloc<int>(nc);
  {
    std::vector<LuDescT<R>> lm(nc);
    std::vector<Mat2T<R>> id(nc);
    std::vector<MatT<R>> am(nc);
    int* ipm = NA.alloc<int>(std::max<int64_t>(tk, 1));
    for (int t = 0; t < nc; ++t) {
      int K = L.k0[t] + L.k1[t];
      lm[t] = LuDescT<R>{Mm + L.offA[t], K, K, ipm + L.offK[t]};
      id[t] = Mat2T<R>{L.At + L.offA[t], K, K};
      am[t] = MatT<R>{L.At + L.offA[t], K, K, K};
    }
    LuDescT<R>* d_lm = NA.upload(lm, s);
    Mat2T<R>* d_id = NA.upload(id, s);
    MatT<R>* d_am = NA.upload(am, s);
    const int mk = L.max_k;
    num_step(F, s, [=](hipStream_t st) {
      asm_zero_i32(d_info2, nc, st);
      la_getrf(d_lm, nc, mk, d_info2, st);
      asm_identity(d_id, nc, mk, st);
      la_getrs(d_lm, d_am, nc, mk, mk, st);
    });
    for (int t = 0; t < nc; ++t)
      la_getrf_work(L.k0[t] + L.k1[t], (int)sizeof(R), &F->info.kernel_bytes[PK_GETRF_PANEL], &F->info.kernel_flops[PK_GETRF_PANEL]);
  }
  std::vector<int> info;
  download(info, d_info, nc, s);
  for (int t = 0; t < nc; ++t)
    if (info[t]) fail(PMX_ESINGULAR, "zero or non-finite pivot in the LU of a cell block");
  download(info, d_info2, nc, s);
  for (int t = 0; t < nc; ++t)
    if (info[t]) fail(PMX_ESINGULAR, "zero or non-finite pivot in the LU of R D^-1 L");
  if (F->num.on) {
    F->num.infos.push_back({d_info, nc});
    F->num.infos.push_back({d_info2, nc});
  }
  sync_check(s);
}

// Active sets and block of every parent at level `lv` from the compressed children.
template <class R>
void merge_level(pmx_factor* F, const LevelData<R>& C, const std::vector<CellPlan>& cells, LevelData<R>& P,
                 Arena& tmp, hipStream_t s) {
  const int np = (int)cells.size();
  P.ncell = np;
  P.s0.assign(np, 0);
  P.s1.assign(np, 0);
  P.offS.resize(np + 1);
  P.offD.resize(np);
  P.rows.clear();
  P.cols.clear();
  std::vector<int> rloc, cloc;
  int64_t td = 0;
  P.max_s = 0;
  for (int p = 0; p < np; ++p) {
    if (cells[p].children.size() > 4) fail(PMX_EGEOM, "a tree cell with more than four children");
    P.offS[p] = (int64_t)P.rows.size();
    for (int ty = 0; ty < 2; ++ty)
      for (int sl = 0; sl < (int)cells[p].children.size(); ++sl) {
        int c = cells[p].children[sl];
        int kb = ty ? C.k1[c] : C.k0[c];
        int64_t o = C.offK[c] + (ty ? C.k0[c] : 0);
        for (int i = 0; i < kb; ++i) {
          P.rows.push_back(C.rskel[o + i]);
          P.cols.push_back(C.cskel[o + i]);
          int loc = (ty ? C.k0[c] : 0) + i;
          rloc.push_back((sl << 24) | loc);
          cloc.push_back((sl << 24) | loc);
        }
        (ty ? P.s1 : P.s0)[p] += kb;
      }
    int sz = P.s0[p] + P.s1[p];
    P.offD[p] = td;
    td += (int64_t)sz * sz;
    P.max_s = std::max(P.max_s, sz);
  }
  P.offS[np] = (int64_t)P.rows.size();
  P.tot_s = P.offS[np];
  P.D = F->arena.alloc<cx<R>>(td);
  P.ipiv = F->arena.alloc<int>(std::max<int64_t>(P.tot_s, 1));
  P.perm = F->arena.alloc<int>(std::max<int64_t>(P.tot_s, 1));
  Arena& NA = num_arena(F, tmp);
  int* d_r = NA.upload(P.rows, s);
  int* d_c = NA.upload(P.cols, s);
  int* d_rl = NA.upload(rloc, s);
  int* d_cl = NA.upload(cloc, s);
  std::vector<ParentDescT<R>> pd(np);
  for (int p = 0; p < np; ++p) {
    ParentDescT<R>& d = pd[p];
    d.rcode = d_r + P.offS[p];
    d.ccode = d_c + P.offS[p];
    d.rloc = d_rl + P.offS[p];
    d.cloc = d_cl + P.offS[p];
    d.s = P.s0[p] + P.s1[p];
    d.out = P.D + P.offD[p];
    for (int sl = 0; sl < 4; ++sl) {
      d.at[sl] = nullptr;
      d.kc[sl] = 0;
    }
    for (int sl = 0; sl < (int)cells[p].children.size(); ++sl) {
      int c = cells[p].children[sl];
      d.at[sl] = C.At + C.offA[c];
      d.kc[sl] = C.k0[c] + C.k1[c];
    }
  }
  ParentDescT<R>* d_pd = NA.upload(pd, s);
  const DevGeom g = F->geom();
  const ExtParams e = F->ext();
  const int ms = P.max_s;
  num_step(F, s, [=](hipStream_t st) { asm_parent(g, e, d_pd, np, ms, st); });
}

// Inclusion level (level 0 of the plan): one inclusion per cell, active rows and columns
// all its nodes (value / q first, then derivative / u); returns the size of the self
// blocks.
template <class R>
int64_t leaf_level(pmx_factor* F, LevelData<R>& L0, std::vector<int>& incl) {
  const std::vector<CellPlan>& leaves = F->plan[0];
  const int nc0 = (int)leaves.size();
  L0.ncell = nc0;
  L0.s0.resize(nc0);
  L0.s1.resize(nc0);
  L0.offS.resize(nc0 + 1);
  L0.offD.resize(nc0);
  int64_t td = 0;
  incl.assign(nc0, 0);
  L0.max_s = 0;
  for (int t = 0; t < nc0; ++t) {
    int j = leaves[t].incl[0];
    incl[t] = j;
    int n = (int)(F->node_off[j + 1] - F->node_off[j]);
    int node0 = (int)F->node_off[j];
    L0.s0[t] = L0.s1[t] = n;
    L0.offS[t] = (int64_t)L0.rows.size();
    for (int ty = 0; ty < 2; ++ty)
      for (int a = 0; a < n; ++a) {
        L0.rows.push_back(pmx_code_node(node0 + a, ty));
        L0.cols.push_back(pmx_code_node(node0 + a, ty));
      }
    L0.offD[t] = td;
    td += (int64_t)4 * n * n;
    L0.max_s = std::max(L0.max_s, 2 * n);
  }
  L0.offS[nc0] = (int64_t)L0.rows.size();
  L0.tot_s = L0.offS[nc0];
  return td;
}

// Candidate columns of the leaf IDs from the network's outputs.  Count: the pair (q,
// value) and the pair (u, derivative) each take c = min(n, ceil(1.1 k) + 8) candidates, k
// the larger of the two predicted ranks.  Choice: systematic sampling along the boundary
// with density proportional to 1/4 + the predicted skeleton probability, so that the
// candidates are spread over the whole boundary (a clustered subset interpolates the
// others poorly) and denser where the network expects skeleton nodes; nodes whose density
// would take more than one sample top the count up in the order of their scores.
LearnedPlan learned_plan(const pmx_factor* F, const std::vector<int>& s0) {
  const int nc = (int)s0.size();
  LearnedPlan lp;
  lp.cand.assign(4 * nc, 0);
  lp.order.resize(4 * nc);
  int64_t first = 0;
  for (int t = 0; t < nc; ++t) {
    const int n = s0[t];
    const float* o = F->leaf_pred.data() + (size_t)PMX_NOUT * first;
    for (int ty = 0; ty < 2; ++ty) {
      double fc = 0, fr = 0;
      for (int i = 0; i < n; ++i) {
        fc += o[(size_t)PMX_NOUT * i + 4 + ty];
        fr += o[(size_t)PMX_NOUT * i + 6 + ty];
      }
      const double khat = std::max(fc, fr);  // sums of the predicted k / n over the nodes
      const int c = std::max(1, std::min(n, (int)std::ceil(1.1 * khat) + 8));
      lp.cand[4 * t + ty] = lp.cand[4 * t + 2 + ty] = c;
    }
    for (int kd = 0; kd < 4; ++kd) {
      const int c = lp.cand[4 * t + kd];
      std::vector<double> dens(n);
      double tot = 0;
      for (int i = 0; i < n; ++i) {
        const double z = o[(size_t)PMX_NOUT * i + kd];
        dens[i] = 0.25 + 1.0 / (1.0 + std::exp(-z));
        tot += dens[i];
      }
      std::vector<char> used(n, 0);
      std::vector<int> ord;
      double cum = 0;
      for (int i = 0; i < n && (int)ord.size() < c; ++i) {
        const double prev = cum;
        cum += dens[i] * c / tot;
        if (std::floor(cum + 0.5) > std::floor(prev + 0.5)) {
          ord.push_back(i);
          used[i] = 1;
        }
      }
      std::vector<int> idx(n);
      for (int i = 0; i < n; ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return o[(size_t)PMX_NOUT * a + kd] > o[(size_t)PMX_NOUT * b + kd];
      });
      for (int i : idx)
        if ((int)ord.size() < c && !used[i]) {
          ord.push_back(i);
          used[i] = 1;
        }
      for (int i = 0; i < n; ++i)
        if (!used[i]) ord.push_back(i);
      lp.order[4 * t + kd] = ord;
    }
    first += n;
  }
  return lp;
}

template <class R>
void factor_all(pmx_factor* F, hipStream_t s) {
  Tier<R>& T = tier<R>(F);
  const double t0 = now_ms();
  const auto& plan = F->plan;
  const size_t lev0 = (size_t)F->lev0;
  // inclusion level (the leaf level unless leaves hold several inclusions)
  LevelData<R> L0;
  std::vector<int> incl;
  const int64_t td = leaf_level(F, L0, incl);
  // self blocks that only enter the leaves' blocks need not outlive the merge
  Arena pass(&F->pool);
  if (lev0) {
    L0.D = num_arena(F, pass).alloc<cx<R>>(td);
  } else {
    L0.D = F->arena.alloc<cx<R>>(td);
    L0.ipiv = F->arena.alloc<int>(L0.tot_s);
    L0.perm = F->arena.alloc<int>(L0.tot_s);
  }
  {
    Arena tmp(&F->pool);
    if (F->opts.precision == 0) {
      assemble_diag(F, tmp, incl, (zd*)L0.D, L0.offD, s);
    } else {
      // the FP64 self blocks (inclusion order, kept for the refinement residual) rounded
      // block by block into leaf order, where they are factored
      std::vector<int64_t> so(incl.size()), len(incl.size());
      int64_t ml = 0;
      for (size_t t = 0; t < incl.size(); ++t) {
        so[t] = F->selfOff[incl[t]];
        const int64_t n = F->node_off[incl[t] + 1] - F->node_off[incl[t]];
        len[t] = 4 * n * n;
        ml = std::max(ml, len[t]);
      }
      Arena& NA = num_arena(F, tmp);
      const int64_t *d_so = NA.upload(so, s), *d_do = NA.upload(L0.offD, s), *d_len = NA.upload(len, s);
      const zd* src = F->Dself;
      cx<R>* dst = L0.D;
      const int cnt = (int)incl.size();
      num_step(F, s, [=](hipStream_t st) { asm_convert_blocks(src, dst, d_so, d_do, d_len, cnt, ml, st); });
    }
    // no synchronisation: the temporaries go back to the pool, whose blocks only later
    // work of this stream reuses, and the host goes on building the next descriptors
    HIPCHK(hipGetLastError());
  }
  F->info.t_phase_ms[0] += now_ms() - t0;
  LevelData<R> cur = std::move(L0);
  if (lev0) {
    // leaves of several inclusions (Sec. 4.4): the inclusions enter whole, every node a
    // skeleton node and the self block itself the block to merge, so that a leaf's block
    // holds its self blocks and the exterior-kernel blocks between its inclusions
    const double tm = now_ms();
    cur.k0 = cur.s0;
    cur.k1 = cur.s1;
    cur.offK.assign(cur.offS.begin(), cur.offS.end() - 1);
    cur.rskel = cur.rows;
    cur.cskel = cur.cols;
    cur.At = cur.D;
    cur.offA = cur.offD;
    cur.tot_k = cur.tot_s;
    Arena tmp(&F->pool);
    LevelData<R> nxt;
    merge_level(F, cur, plan[lev0], nxt, tmp, s);
    HIPCHK(hipGetLastError());
    cur = std::move(nxt);
    F->info.t_phase_ms[2] += now_ms() - tm;
  }
  for (size_t lv = lev0; lv < plan.size(); ++lv) {
    if (lv > lev0) {
      const double tm = now_ms();
      Arena tmp(&F->pool);
      LevelData<R> nxt;
      merge_level(F, T.lev.back(), plan[lv], nxt, tmp, s);
      HIPCHK(hipGetLastError());
      cur = std::move(nxt);
      F->info.t_phase_ms[2] += now_ms() - tm;
    }
    if (plan[lv].size() == 1) {
      // root: dense partial-pivoted LU of the top compressed system
      const double tr = now_ms();
      T.root_s = cur.s0[0] + cur.s1[0];
      T.Droot = cur.D;
      T.ipiv_root = cur.ipiv;
      T.perm_root = cur.perm;
      T.root_rows = cur.rows;
      T.root_cols = cur.cols;
      Arena tmp(&F->pool);
      int* d_info = num_arena(F, tmp).alloc<int>(1);
      {
        std::vector<LuDescT<R>> lu{LuDescT<R>{T.Droot, T.root_s, T.root_s, T.ipiv_root, T.perm_root}};
        T.d_lu_root = F->arena.upload(lu, s);
        const LuDescT<R>* dl = T.d_lu_root;
        const int rs = T.root_s;
        num_step(F, s, [=](hipStream_t st) {
          asm_zero_i32(d_info, 1, st);
          la_getrf(dl, 1, rs, d_info, st);
        });
        la_getrf_work(T.root_s, (int)sizeof(R), &F->info.kernel_bytes[PK_GETRF_PANEL], &F->info.kernel_flops[PK_GETRF_PANEL]);
      }
      if (F->opts.precision != 0) {
        // refined forms: the inverse of the LU's factors, formed in FP64 (the LU's solves with
        // the identity as right-hand sides)
        const int rs = T.root_s;
        zd* LU64 = num_arena(F, tmp).alloc<zd>((int64_t)rs * rs);
        T.Ainv_root = F->arena.alloc<zd>((int64_t)rs * rs);
        std::vector<LuDescT<double>> lu{LuDescT<double>{LU64, rs, rs, T.ipiv_root, T.perm_root}};
        std::vector<Mat2T<double>> id{Mat2T<double>{T.Ainv_root, rs, rs}};
        std::vector<MatT<double>> am{MatT<double>{T.Ainv_root, rs, rs, rs}};
        const LuDescT<double>* dl = num_arena(F, tmp).upload(lu, s);
        const Mat2T<double>* d_id = num_arena(F, tmp).upload(id, s);
        const MatT<double>* d_am = num_arena(F, tmp).upload(am, s);
        const cx<R>* D = T.Droot;
        num_step(F, s, [=](hipStream_t st) {
          asm_convert(D, LU64, (int64_t)rs * rs, st);
          asm_identity(d_id, 1, rs, st);
          la_getrs(dl, d_am, 1, rs, rs, st);
        });
      }
      if (F->num.on) F->num.infos.push_back({d_info, 1});
      std::vector<int> info;
      download(info, d_info, 1, s);
      if (info[0]) fail(PMX_ESINGULAR, "zero or non-finite pivot in the LU of the top compressed system");
      F->info.t_phase_ms[3] += now_ms() - tr;
      break;
    }
    const double tc = now_ms();
    LearnedPlan lp;
    const bool learned = (lv == lev0 && !F->leaf_pred.empty());
    if (learned) {
      const double tq = now_ms();
      lp = learned_plan(F, cur.s0);
      F->info.t_phase_ms[8] += now_ms() - tq;
    }
    compress_level(F, cur, plan[lv], learned ? &lp : nullptr, lv == lev0, s);
    F->info.t_phase_ms[1] += now_ms() - tc;
    T.lev.push_back(std::move(cur));
    cur = LevelData<R>();
  }
}

template <class R>
void fill_info(pmx_factor* F) {
  Tier<R>& T = tier<R>(F);
  pmx_info& I = F->info;
  I.levels = (int)T.lev.size();
  I.root_size = T.root_s;
  I.n_unknowns = 2 * F->n_nodes;
  for (size_t l = 0; l < T.lev.size() && l < 32; ++l) {
    const LevelData<R>& L = T.lev[l];
    I.cells[l] = L.ncell;
    int mn = 1 << 30, mx = 0;
    double sum = 0;
    for (int t = 0; t < L.ncell; ++t) {
      int K = L.k0[t] + L.k1[t];
      mn = std::min(mn, K);
      mx = std::max(mx, K);
      sum += K;
    }
    I.rank_min[l] = mn;
    I.rank_max[l] = mx;
    I.rank_mean[l] = sum / std::max(1, L.ncell);
  }
  I.bytes_factor = F->arena.bytes();
}

// ---------------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------------
// solve programs
//
// A solve program holds, for one factor type and one right-hand-side count, every buffer
// and launch descriptor of the upward pass (y = D^-1 f, g = At R y), the top solve and the
// downward pass (x = y - Y (g - At psi)), so that running it only launches kernels.
// Vectors of a level are stored per cell, column major with leading dimension = rows.
template <class R>
void build_program(pmx_factor* F, int nrhs, hipStream_t s) {
  Tier<R>& T = tier<R>(F);
  SolveProgram<R>& P = T.prog;
  P.arena.release();
  P.lv.clear();
  P.nrhs = -1;
  Arena& A = P.arena;
  const int nl = (int)T.lev.size();
  P.lv.resize(nl);
  for (int l = 0; l < nl; ++l) {
    const LevelData<R>& L = T.lev[l];
    SolveLevel<R>& S = P.lv[l];
    S.F = A.alloc<cx<R>>(L.tot_s * nrhs);
    S.G = A.alloc<cx<R>>(std::max<int64_t>(L.tot_k, 1) * nrhs);
    S.Red = A.alloc<cx<R>>(std::max<int64_t>(L.tot_s - L.tot_k, 1) * nrhs);
    S.Ry = A.alloc<cx<R>>(std::max<int64_t>(L.tot_k, 1) * nrhs);
    S.W = A.alloc<cx<R>>(L.tot_s * nrhs);
  }
  P.Froot = A.alloc<cx<R>>((int64_t)T.root_s * nrhs);
  for (int l = 0; l < nl; ++l) {
    const LevelData<R>& L = T.lev[l];
    SolveLevel<R>& S = P.lv[l];
    const int nc = L.ncell;
    // y = D^-1 f
    std::vector<MatT<R>> bm(nc), wm(nc);
    for (int t = 0; t < nc; ++t) {
      int sz = L.s0[t] + L.s1[t];
      bm[t] = MatT<R>{S.F + L.offS[t] * nrhs, sz, sz, nrhs};
      wm[t] = MatT<R>{S.W + L.offS[t] * nrhs, sz, sz, nrhs};
    }
    S.d_bm = A.upload(bm, s);
    S.d_w = A.upload(wm, s);
    // R y -> G (skeleton rows, then + T * redundant rows)
    std::vector<RowSrc> rs;
    std::vector<int64_t> rso;
    std::vector<GatherDescT<R>> gd;
    std::vector<GemmArgsT<R>> ga, gb;
    int maxr = 0;
    int64_t ro = 0;
    for (int t = 0; t < nc; ++t) {
      int K = L.k0[t] + L.k1[t];
      int sz = L.s0[t] + L.s1[t];
      int64_t yo = L.offS[t] * nrhs;
      rso.push_back((int64_t)rs.size());
      for (int ty = 0; ty < 2; ++ty) {
        int kb = ty ? L.k1[t] : L.k0[t];
        int base = ty ? L.s0[t] : 0;
        for (int i = 0; i < kb; ++i) rs.push_back(RowSrc{yo + base + L.cpiv[L.offS[t] + base + i], sz});
      }
      gd.push_back(GatherDescT<R>{nullptr, K, nrhs, S.G + L.offK[t] * nrhs, K});
      maxr = std::max(maxr, K);
      for (int ty = 0; ty < 2; ++ty) {
        int kb = ty ? L.k1[t] : L.k0[t];
        int base = ty ? L.s0[t] : 0;
        int sb = ty ? L.s1[t] : L.s0[t];
        int nr = sb - kb;
        rso.push_back((int64_t)rs.size());
        for (int j = 0; j < nr; ++j) rs.push_back(RowSrc{yo + base + L.cpiv[L.offS[t] + base + kb + j], sz});
        gd.push_back(GatherDescT<R>{nullptr, nr, nrhs, S.Red + ro, std::max(nr, 1)});
        maxr = std::max(maxr, nr);
        if (nr > 0) {
          GemmArgsT<R> g;
          g.m = kb;
          g.n = nrhs;
          g.k = nr;
          g.A = L.Tc + L.offT[t] + (ty ? (int64_t)L.k0[t] * (L.s0[t] - L.k0[t]) : 0);
          g.lda = kb;
          g.B = S.Red + ro;
          g.ldb = nr;
          g.C = S.G + L.offK[t] * nrhs + (ty ? L.k0[t] : 0);
          g.ldc = K;
          ga.push_back(g);
        }
        ro += (int64_t)nr * nrhs;
      }
      gb.push_back(GemmArgsT<R>{K, nrhs, K, L.At + L.offA[t], K, S.Ry + L.offK[t] * nrhs, K,
                                S.G + L.offK[t] * nrhs, K});
    }
    RowSrc* d_rs = A.upload(rs, s);
    for (size_t i = 0; i < gd.size(); ++i) gd[i].src = d_rs + rso[i];
    S.d_up = A.upload(gd, s);
    S.n_up = (int)gd.size();
    S.max_up = maxr;
    S.n_ga = (int)ga.size();
    if (!ga.empty()) S.d_ga = A.upload(ga, s);
    S.d_gb = A.upload(gb, s);
    S.tot_k = L.tot_k;
    // parent right-hand sides
    const bool top = (l + 1 == nl);
    const std::vector<CellPlan>& pc = F->plan[l + 1 + F->lev0];
    cx<R>* dst = top ? P.Froot : P.lv[l + 1].F;
    std::vector<RowSrc> prs;
    std::vector<GatherDescT<R>> pgd;
    std::vector<int64_t> pro;
    int maxp = 0;
    int64_t po = 0;
    for (size_t q = 0; q < pc.size(); ++q) {
      pro.push_back((int64_t)prs.size());
      int cnt = 0;
      for (int ty = 0; ty < 2; ++ty)
        for (int c : pc[q].children) {
          int K = L.k0[c] + L.k1[c];
          int kb = ty ? L.k1[c] : L.k0[c];
          int base = ty ? L.k0[c] : 0;
          for (int i = 0; i < kb; ++i) prs.push_back(RowSrc{L.offK[c] * nrhs + base + i, K});
          cnt += kb;
        }
      pgd.push_back(GatherDescT<R>{nullptr, cnt, nrhs, dst + po * nrhs, cnt});
      po += cnt;
      maxp = std::max(maxp, cnt);
    }
    RowSrc* d_prs = A.upload(prs, s);
    for (size_t i = 0; i < pgd.size(); ++i) pgd[i].src = d_prs + pro[i];
    S.d_par = A.upload(pgd, s);
    S.n_par = (int)pgd.size();
    S.max_par = maxp;
    // downward: psi of each cell from its parent's solution, then g -= At psi, x = y - Y g
    const LevelData<R>* Pl = top ? nullptr : &T.lev[l + 1];
    std::vector<int64_t> psio(nc);
    int64_t o = 0;
    for (int t = 0; t < nc; ++t) {
      psio[t] = o;
      o += (int64_t)(L.k0[t] + L.k1[t]) * nrhs;
    }
    S.Psi = A.alloc<cx<R>>(std::max<int64_t>(o, 1));
    std::vector<RowSrc> xrs(L.tot_k);
    for (size_t q = 0; q < pc.size(); ++q) {
      int64_t pbase = top ? 0 : Pl->offS[q];
      int psz = top ? T.root_s : Pl->s0[q] + Pl->s1[q];
      int pos = 0;
      for (int ty = 0; ty < 2; ++ty)
        for (int c : pc[q].children) {
          int kb = ty ? L.k1[c] : L.k0[c];
          int base = ty ? L.k0[c] : 0;
          for (int i = 0; i < kb; ++i) xrs[L.offK[c] + base + i] = RowSrc{pbase * nrhs + pos + i, psz};
          pos += kb;
        }
    }
    RowSrc* d_xrs = A.upload(xrs, s);
    std::vector<GatherDescT<R>> xgd(nc);
    std::vector<GemmArgsT<R>> g1(nc), g2(nc);
    for (int t = 0; t < nc; ++t) {
      int K = L.k0[t] + L.k1[t];
      int sz = L.s0[t] + L.s1[t];
      xgd[t] = GatherDescT<R>{d_xrs + L.offK[t], K, nrhs, S.Psi + psio[t], K};
      g1[t] = GemmArgsT<R>{K, nrhs, K, L.At + L.offA[t], K, S.Psi + psio[t], K, S.G + L.offK[t] * nrhs, K};
      g2[t] = GemmArgsT<R>{sz, nrhs, K, L.Y + L.offY[t], sz, S.G + L.offK[t] * nrhs, K, S.F + L.offS[t] * nrhs, sz};
    }
    S.d_psi = A.upload(xgd, s);
    S.d_g1 = A.upload(g1, s);
    S.d_g2 = A.upload(g2, s);
  }
  std::vector<MatT<R>> rb{MatT<R>{P.Froot, T.root_s, T.root_s, nrhs}};
  P.d_bm_root = A.upload(rb, s);
  std::vector<MatT<R>> rw{MatT<R>{A.alloc<cx<R>>((int64_t)T.root_s * nrhs), T.root_s, T.root_s, nrhs}};
  P.d_w_root = A.upload(rw, s);
  P.d_root_gemm = nullptr;
  if (T.Ainv_root) {
    const int rs = T.root_s;
    P.Wroot64 = A.alloc<zd>((int64_t)rs * nrhs);
    P.Yroot64 = A.alloc<zd>((int64_t)rs * nrhs);
    std::vector<GemmArgsT<double>> rg{GemmArgsT<double>{rs, nrhs, rs, T.Ainv_root, rs, P.Wroot64, rs, P.Yroot64, rs}};
    P.d_root_gemm = A.upload(rg, s);
  }
  P.leaf = nl ? P.lv[0].F : P.Froot;
  P.nrhs = nrhs;
}

// level solves of `batch` LU factors of size <= n: 0 the fused kernel (few right-hand
// sides), 1 the blocked one, 2 the LDS-resident one; by default 2 when its LDS block fits,
// else 0 up to PMX_GETRS_SMALL_MAX right-hand sides, else 1
template <class R>
int getrs_variant(int n, int batch, int nrhs) {
  const bool lds_ok = la_getrs_lds_bytes(n, (int)sizeof(R)) <= 128 * 1024;
  const int dflt = lds_ok ? 2 : (nrhs <= PMX_GETRS_SMALL_MAX ? 0 : 1);
  int v = tune_choice(TK_GETRS, (int)sizeof(R), tune_bucket_size(n), tune_bucket_batch(batch), tune_bucket_pow2(nrhs),
                      dflt, n, batch, nrhs);
  if ((v == 2 && !lds_ok) || (v == 0 && nrhs > PMX_GETRS_SMALL_MAX) || v < 0 || v > 2) v = dflt;
  return v;
}

template <class R>
void level_getrs(const LuDescT<R>* d_lu, const MatT<R>* d_bm, const MatT<R>* d_w, int batch, int n, int nrhs,
                 hipStream_t s) {
  const int v = getrs_variant<R>(n, batch, nrhs);
  if (v == 2 && la_getrs_lds(d_lu, d_bm, batch, n, nrhs, s)) return;
  if (v == 0)
    la_getrs_small(d_lu, d_bm, d_w, batch, n, nrhs, s);
  else
    la_getrs(d_lu, d_bm, batch, n, nrhs, s);
}

// the launches of one solve pass on the leaf vectors P.leaf (in place); no host work
template <class R>
void launch_program(pmx_factor* F, hipStream_t s) {
  Tier<R>& T = tier<R>(F);
  SolveProgram<R>& P = T.prog;
  const int nrhs = P.nrhs;
  const int nl = (int)T.lev.size();
  const cx<R> one = cmk<R>(1, 0), mone = cmk<R>(-1, 0), zero = cmk<R>(0, 0);
  for (int l = 0; l < nl; ++l) {
    const LevelData<R>& L = T.lev[l];
    SolveLevel<R>& S = P.lv[l];
    level_getrs(L.d_lu, S.d_bm, S.d_w, L.ncell, L.max_s, nrhs, s);
    asm_gather(S.F, S.d_up, S.n_up, S.max_up, nrhs, s);
    if (S.n_ga) la_zgemm_list(OP_N, OP_N, S.d_ga, S.n_ga, L.max_k, nrhs, one, one, s);
    asm_convert(S.G, S.Ry, S.tot_k * nrhs, s);
    la_zgemm_list(OP_N, OP_N, S.d_gb, L.ncell, L.max_k, nrhs, one, zero, s);
    const bool top = (l + 1 == nl);
    (void)top;
    asm_gather(S.G, S.d_par, S.n_par, S.max_par, nrhs, s);
  }
  if (P.d_root_gemm) {
    const int64_t n = (int64_t)T.root_s * nrhs;
    asm_convert(P.Froot, P.Wroot64, n, s);
    la_zgemm_list(OP_N, OP_N, P.d_root_gemm, 1, T.root_s, nrhs, cmk<double>(1, 0), cmk<double>(0, 0), s);
    asm_convert(P.Yroot64, P.Froot, n, s);
  } else {
    level_getrs(T.d_lu_root, P.d_bm_root, P.d_w_root, 1, T.root_s, nrhs, s);
  }
  for (int l = nl - 1; l >= 0; --l) {
    const LevelData<R>& L = T.lev[l];
    SolveLevel<R>& S = P.lv[l];
    const cx<R>* xp = (l + 1 == nl) ? P.Froot : P.lv[l + 1].F;
    asm_gather(xp, S.d_psi, L.ncell, L.max_k, nrhs, s);
    la_zgemm_list(OP_N, OP_N, S.d_g1, L.ncell, L.max_k, nrhs, mone, one, s);
    la_zgemm_list(OP_N, OP_N, S.d_g2, L.ncell, L.max_s, nrhs, mone, one, s);
  }
}

// Row maps between three layouts of a block of nrhs vectors:
//  * leaf: the vectors of the first compressed level (the top system when there is none),
//    per cell its active rows in order, column major with leading dimension = rows;
//  * density: [nrhs][2 N], per inclusion [q; u] (value rows, then derivative rows);
//  * inclusion: per level-0 cell of the plan in plan order, [q; u] with leading dimension
//    2 n (what the plane-wave kernel writes).  With one inclusion per leaf it is the leaf
//    layout; with leaves of several inclusions the leaf rows of an inclusion are not
//    contiguous and the plane waves reach the leaves through the density layout.
struct LeafMap {
  int n2 = 0, max_cell = 0, ncell = 0;
  std::vector<int64_t> leaf_off;    // per cell: first leaf entry / nrhs
  std::vector<int> cell_rows;
  bool same = true;                 // inclusion layout == leaf layout
  RowSrc *d_to_dens = nullptr, *d_to_leaf = nullptr, *d_incl_to_dens = nullptr;
};

// rows, cols: the active codes of the leaf cells (node codes only), offsets offS [ncell + 1];
// same: the leaf cells are the plan's level-0 cells (one inclusion each, [q; u]), so that
// the inclusion layout is the leaf layout
void build_leaf_map(pmx_factor* F, int nrhs, const std::vector<int>& rows, const std::vector<int>& cols,
                    const std::vector<int64_t>& offS, int ncell, bool same, LeafMap& M, Arena& A, hipStream_t s) {
  const std::vector<int64_t>& no = F->node_off;
  const int N = F->n_nodes;
  M.n2 = 2 * N;
  M.ncell = ncell;
  M.same = same;
  std::vector<RowSrc> to_dens(M.n2), to_leaf(M.n2);
  M.leaf_off.assign(ncell, 0);
  M.cell_rows.assign(ncell, 0);
  M.max_cell = 0;
  // density index of each node code (2 node + type): base[node] + type * n_j
  std::vector<int64_t> base(N);
  std::vector<int> nj(N);
  for (int j = 0; j + 1 < (int)no.size(); ++j)
    for (int64_t i = no[j]; i < no[j + 1]; ++i) {
      base[i] = 2 * no[j] + (i - no[j]);
      nj[i] = (int)(no[j + 1] - no[j]);
    }
  auto dens = [&](int code) {
    if (code < 0 || (code >> 1) >= N) fail(PMX_EINVAL, "a leaf row that is not a boundary node");
    return base[code >> 1] + (int64_t)(code & 1) * nj[code >> 1];
  };
  for (int t = 0; t < ncell; ++t) {
    const int64_t off = offS[t];
    const int sz = (int)(offS[t + 1] - off);
    for (int r = 0; r < sz; ++r) {
      to_leaf[off + r] = RowSrc{dens(rows[off + r]), M.n2};
      to_dens[dens(cols[off + r])] = RowSrc{off * nrhs + r, sz};
    }
    M.leaf_off[t] = off;
    M.cell_rows[t] = sz;
    M.max_cell = std::max(M.max_cell, sz);
  }
  M.d_to_dens = A.upload(to_dens, s);
  M.d_to_leaf = A.upload(to_leaf, s);
  if (same) {
    M.d_incl_to_dens = M.d_to_dens;
    return;
  }
  std::vector<RowSrc> incl_to_dens(M.n2);
  int64_t o = 0;
  for (const CellPlan& c : F->plan[0]) {
    const int j = c.incl[0];
    const int n2j = (int)(2 * (no[j + 1] - no[j]));
    for (int r = 0; r < n2j; ++r) incl_to_dens[2 * no[j] + r] = RowSrc{o * nrhs + r, n2j};
    o += n2j;
  }
  M.d_incl_to_dens = A.upload(incl_to_dens, s);
}

// descriptors: leaf vectors -> one density-layout buffer, and back per cell
template <class RD>
GatherDescT<RD>* gather_to_dens(const LeafMap& M, cx<RD>* dens, int nrhs, Arena& A, hipStream_t s) {
  std::vector<GatherDescT<RD>> gd{GatherDescT<RD>{M.d_to_dens, M.n2, nrhs, dens, M.n2}};
  return A.upload(gd, s);
}

template <class RD>
GatherDescT<RD>* gather_incl_to_dens(const LeafMap& M, cx<RD>* dens, int nrhs, Arena& A, hipStream_t s) {
  std::vector<GatherDescT<RD>> gd{GatherDescT<RD>{M.d_incl_to_dens, M.n2, nrhs, dens, M.n2}};
  return A.upload(gd, s);
}

template <class RD>
GatherDescT<RD>* gather_to_leaf(const LeafMap& M, cx<RD>* leaf, int nrhs, Arena& A, hipStream_t s) {
  std::vector<GatherDescT<RD>> gd(M.ncell);
  for (int t = 0; t < M.ncell; ++t)
    gd[t] = GatherDescT<RD>{M.d_to_leaf + M.leaf_off[t], M.cell_rows[t], nrhs, leaf + M.leaf_off[t] * nrhs,
                            M.cell_rows[t]};
  return A.upload(gd, s);
}

// Dense FP64 operator apply y = A x, or the residual out = f - A x, for fixed buffers: the
// self blocks from FP64 storage (block of inclusion incl[t] at offset doff[t], 2 n x 2 n)
// by batched MFMA products, the blocks between inclusions evaluated on the fly.
struct DenseApply {
  int nrhs = -1, nsplit = 1, nblk = 1, nr_max = 8;
  int nslots = 1;                 // partial-sum slots: nsplit far-list parts + near parts
  int n_src = 0;                  // expansion sources: inclusions and clusters
  double flops_fixed = 0, flops_rhs = 0;   // algorithmic work of one apply (counted with timing)
  double self_sq = 0;             // sum over inclusions of (2 n_j)^2: the FP64 self-block entries
  double table_bytes = 0;         // translation tables of the fast multipole part
  double near_pairs_stored = 0;   // near (target, source node) pairs with stored coefficients
  int64_t total = 0;
  zd *ydiag = nullptr, *part = nullptr;
  double* d_norm = nullptr;
  GemmArgs* d_ga = nullptr;
  int n_ga = 0, max_s = 0;
  ApplyArgs aa;
  const zd* f = nullptr;
  zd* out = nullptr;
};

// Geometry of the dense apply.  Sources: every inclusion and every cell of the plan's tree
// above the leaves except the root (a cluster), each with its bounding circle (centre,
// radius) and the expansion order its sources need; waves of 64 consecutive target nodes
// with theirs.  Per wave, a walk down the tree from the top clusters gives the list of far
// sources (a cluster whose centre is farther than PMX_APPLY_RATIO radii from the wave's
// circle and whose order stays within PMX_APPLY_PMAXC; an inclusion reached because its
// parent was opened, when it is not near) and the sorted list of near inclusions (closer
// than PMX_APPLY_RATIO radii, or needing more than PMX_APPLY_PMAX orders).  A cluster is
// never taken whole when its own order exceeds PMX_APPLY_PMAXC or it holds an inclusion
// that is near for every wave.  With `count`, the algorithmic work per right-hand side and
// the fixed part are returned: per near pair 32 and 130 flops (the pair formulas); per
// (target, far source) of order p, (p + 2) 48 and 100 + 26 (p + 2) flops (orders
// m = 0 .. p + 1: six complex multiply-adds per right-hand side, the two O's and the
// recurrences; H0, H1 and the geometry once); per source node and order 72 flops per
// right-hand side for the expansion sums; per cluster, child and translated pair of
// orders 16 flops per right-hand side (two complex multiply-adds).
struct ApplyGeo {
  std::vector<int> off, idx;        // near inclusions per wave
  std::vector<int> foff, fidx;      // far sources per wave
  std::vector<double> incl, wave;   // per source (inclusions, then clusters) and per wave
  std::vector<int> wave_node;       // per wave: first node, node count (one inclusion)
  std::vector<int> kid_off, kid_idx;
  std::vector<int> lev_off;         // clusters of tree level 1, 2, ...: lev_off[l] .. lev_off[l + 1] - 1
  int n_clus = 0;
  // fast multipole part (see ApplyArgs)
  std::vector<int> loc_id, loc_p;
  std::vector<double> loc_geo;
  std::vector<int> m2l_off, m2l_slot, m2l_src, m2l_nmax, m2l_mmax;
  std::vector<int64_t> m2l_toff;
  std::vector<int> l2l_child, l2l_parent, l2l_lev;
  std::vector<int64_t> l2l_toff;
  int64_t m2l_tab = 0, l2l_tab = 0;   // complex entries of the translation tables
  double flops_fixed = 0, flops_rhs = 0;
  double stats[8] = {};               // pmx_info.apply_stats
};

void apply_geometry(const pmx_factor* F, const std::vector<double>& hx, const std::vector<double>& hy, ApplyGeo& G,
                    bool count) {
  const int m = F->m, N = F->n_nodes;
  // target waves: up to 64 consecutive nodes of one inclusion
  G.wave_node.clear();
  std::vector<int> wave_incl;
  for (int j = 0; j < m; ++j)
    for (int64_t o = F->node_off[j]; o < F->node_off[j + 1]; o += 64) {
      G.wave_node.push_back((int)o);
      G.wave_node.push_back((int)std::min<int64_t>(64, F->node_off[j + 1] - o));
      wave_incl.push_back(j);
    }
  const int nw = (int)G.wave_node.size() / 2;
  const double k = F->k_ext;
  const auto& plan = F->plan;
  // bounding circle of the nodes of the inclusions in `incs` (all nodes of inclusion j: node_off)
  auto circle = [&](const int* incs, int ninc, double& cx, double& cy, double& r) {
    const int64_t f0 = F->node_off[incs[0]];
    double x0 = hx[f0], x1 = hx[f0], y0 = hy[f0], y1 = hy[f0];
    for (int q = 0; q < ninc; ++q)
      for (int64_t b = F->node_off[incs[q]]; b < F->node_off[incs[q] + 1]; ++b) {
        x0 = std::min(x0, hx[b]);
        x1 = std::max(x1, hx[b]);
        y0 = std::min(y0, hy[b]);
        y1 = std::max(y1, hy[b]);
      }
    cx = 0.5 * (x0 + x1);
    cy = 0.5 * (y0 + y1);
    double r2 = 0;
    for (int q = 0; q < ninc; ++q)
      for (int64_t b = F->node_off[incs[q]]; b < F->node_off[incs[q] + 1]; ++b)
        r2 = std::max(r2, (hx[b] - cx) * (hx[b] - cx) + (hy[b] - cy) * (hy[b] - cy));
    r = std::sqrt(r2);
  };
  // clusters: plan levels 1 .. L - 2 (the root level is left out)
  const int L = (int)plan.size();
  const int nclev = std::max(0, std::min(L - 2, PMX_APPLY_MAXLEV));
  std::vector<std::vector<int>> cid(L);
  G.lev_off.assign(1, 0);
  int nc = 0;
  for (int l = 1; l <= nclev; ++l) {
    cid[l].resize(plan[l].size());
    for (size_t t = 0; t < plan[l].size(); ++t) cid[l][t] = nc++;
    G.lev_off.push_back(nc);
  }
  G.n_clus = nc;
  const int nsrc = m + nc;
  G.incl.assign(4 * (size_t)nsrc, 0.0);
  G.wave.assign(4 * (size_t)nw, 0.0);
  std::vector<char> always(m, 0), usable(nc, 0), holds_always(nc, 0);
  for (int j = 0; j < m; ++j) {
    double* g = &G.incl[4 * (size_t)j];
    circle(&j, 1, g[0], g[1], g[2]);
    g[3] = (double)apply_source_order(k * g[2]);
    if (g[3] > PMX_APPLY_PMAX) always[j] = 1;
  }
  G.kid_off.assign(1, 0);
  G.kid_idx.clear();
  std::vector<double> cterms(nc, 0.0);   // translation terms per cluster
  for (int l = 1; l <= nclev; ++l)
    for (size_t t = 0; t < plan[l].size(); ++t) {
      const CellPlan& cp = plan[l][t];
      const int c = cid[l][t];
      double* g = &G.incl[4 * (size_t)(m + c)];
      circle(cp.incl.data(), (int)cp.incl.size(), g[0], g[1], g[2]);
      g[3] = (double)apply_source_order(k * g[2]);
      bool ha = false;
      if (cp.children.size() > 4) fail(PMX_EGEOM, "a tree cell with more than four children");
      for (int ch : cp.children) {
        int src;
        if (l == 1) {
          src = plan[0][ch].incl[0];
          ha = ha || always[src];
          cterms[c] += 2.0 * (2 * (PMX_APPLY_PMAXC + 2) + 1) * (2 * PMX_APPLY_NREC);
        } else {
          src = m + cid[l - 1][ch];
          ha = ha || holds_always[cid[l - 1][ch]];
          cterms[c] += 2.0 * (2 * (PMX_APPLY_PMAXC + 2) + 1) * (2 * PMX_APPLY_NRECA);
        }
        G.kid_idx.push_back(src);
      }
      G.kid_off.push_back((int)G.kid_idx.size());
      holds_always[c] = ha;
      usable[c] = !ha && g[3] <= PMX_APPLY_PMAXC;
    }
  // levels above the last one with a usable cluster need no translated records (a parent
  // is never usable when none of its level is: its radius and order only grow)
  while (G.lev_off.size() > 1) {
    const int l0 = G.lev_off[G.lev_off.size() - 2], l1 = G.lev_off.back();
    bool any = false;
    for (int c = l0; c < l1; ++c) any = any || usable[c];
    if (any) break;
    G.lev_off.pop_back();
  }
  double m2m_terms = 0;
  for (int c = 0; c < G.lev_off.back(); ++c) m2m_terms += cterms[c];
  for (int w = 0; w < nw; ++w) {
    const int lo = G.wave_node[2 * w], hi = lo + G.wave_node[2 * w + 1];
    double* g = &G.wave[4 * (size_t)w];
    // the wave's nodes lie in consecutive inclusions: their circle over that node range
    double x0 = hx[lo], x1 = hx[lo], y0 = hy[lo], y1 = hy[lo];
    for (int b = lo; b < hi; ++b) {
      x0 = std::min(x0, hx[b]);
      x1 = std::max(x1, hx[b]);
      y0 = std::min(y0, hy[b]);
      y1 = std::max(y1, hy[b]);
    }
    g[0] = 0.5 * (x0 + x1);
    g[1] = 0.5 * (y0 + y1);
    double r2 = 0;
    for (int b = lo; b < hi; ++b) r2 = std::max(r2, (hx[b] - g[0]) * (hx[b] - g[0]) + (hy[b] - g[1]) * (hy[b] - g[1]));
    g[2] = std::sqrt(r2);
  }
  // tree: parents, the nested radius r~ (about the node's centre, covering every circle
  // below it), and the top nodes (no parent)
  const int nsrc_all = m + nc;
  std::vector<int> parent(nsrc_all, -1), lvl(nsrc_all, 0);
  for (int c = 0; c < nc; ++c)
    for (int q = G.kid_off[c]; q < G.kid_off[c + 1]; ++q) parent[G.kid_idx[q]] = m + c;
  for (int l = 1; l <= nclev; ++l)
    for (size_t t = 0; t < plan[l].size(); ++t) lvl[m + cid[l][t]] = l;
  std::vector<double> rt(nsrc_all);
  for (int j = 0; j < m; ++j) rt[j] = G.incl[4 * (size_t)j + 2];
  for (int c = 0; c < nc; ++c) {   // clusters are numbered level by level upwards
    const double* g = &G.incl[4 * (size_t)(m + c)];
    double r = g[2];
    for (int q = G.kid_off[c]; q < G.kid_off[c + 1]; ++q) {
      const int ch = G.kid_idx[q];
      const double* gc = &G.incl[4 * (size_t)ch];
      r = std::max(r, std::hypot(gc[0] - g[0], gc[1] - g[1]) + rt[ch]);
    }
    rt[m + c] = r;
  }
  std::vector<int> top;
  for (int v = 0; v < nsrc_all; ++v)
    if (parent[v] < 0 && (v >= m || nclev == 0)) top.push_back(v);
  // local-expansion orders: the targets' own decay order or the separation's, whichever is
  // larger; a node with an order above PMX_FMM_PL takes no local expansion
  const int p_sep = (int)std::ceil(PMX_APPLY_TRUNC / std::log(1.0 / PMX_FMM_RATIO));
  std::vector<int> ptgt(nsrc_all);
  for (int v = 0; v < nsrc_all; ++v) ptgt[v] = std::max(apply_source_order(k * rt[v]), p_sep);
  auto src_ok = [&](int v) { return v < m ? !always[v] : (bool)usable[v - m]; };
  // a pair (T, S) is translated when its circles are separated by the ratio, both orders
  // fit and the table's largest Hankel function stays far below the overflow threshold
  // orders of a pair: the double series sum_n sum_m X_n O_{n-m}(D) I_m(u) (|u| <= r~_T)
  // loses less than e^-PMX_APPLY_TRUNC beyond |n| = nmax when (r_S / (|D| - r~_T))^nmax is
  // that small, and beyond |m| = mmax when (r~_T / (|D| - r_S))^mmax is; neither goes
  // below the decay order of its own radius (the sources' J_n, the targets' J_m)
  auto accept = [&](int T, int S, int& nmax, int& mmax) {
    if (ptgt[T] > PMX_FMM_PL || !src_ok(S)) return false;
    const double* gt = &G.incl[4 * (size_t)T];
    const double* gs = &G.incl[4 * (size_t)S];
    const double d = std::hypot(gt[0] - gs[0], gt[1] - gs[1]);
    if (!(rt[T] + gs[2] <= PMX_FMM_RATIO * d)) return false;
    nmax = std::max((int)gs[3], (int)std::ceil(PMX_APPLY_TRUNC / std::log((d - rt[T]) / gs[2])));
    mmax = std::max(apply_source_order(k * rt[T]), (int)std::ceil(PMX_APPLY_TRUNC / std::log((d - gs[2]) / rt[T])));
    mmax = std::min(mmax, ptgt[T]);
    if (nmax > (S < m ? std::min(PMX_FMM_NMAX, PMX_APPLY_PMAX) : PMX_FMM_NMAX)) return false;   // within the records
    const double V = mmax + 1 + nmax, z = k * d;
    if (V > z && V * std::log(2.0 * V / (M_E * z)) > 600.0) return false;
    return true;
  };
  struct M2lPair {
    int src, nmax, mmax;
  };
  std::vector<std::vector<M2lPair>> m2l(nsrc_all);
  std::vector<std::vector<int>> leftover(m);
  std::function<void(int, int)> walk = [&](int T, int S) {
    if (T == S) {
      if (T < m) return;
      const int c = T - m;
      for (int a = G.kid_off[c]; a < G.kid_off[c + 1]; ++a)
        for (int b = G.kid_off[c]; b < G.kid_off[c + 1]; ++b) walk(G.kid_idx[a], G.kid_idx[b]);
      return;
    }
    int nmax = 0, mmax = 0;
    if (accept(T, S, nmax, mmax)) {
      m2l[T].push_back({S, nmax, mmax});
      return;
    }
    if (T < m) {   // a leaf target: its waves' walks take S, opening it as they need
      leftover[T].push_back(S);
      return;
    }
    if (S < m || rt[T] >= rt[S]) {
      const int c = T - m;
      for (int a = G.kid_off[c]; a < G.kid_off[c + 1]; ++a) walk(G.kid_idx[a], S);
    } else {
      const int c = S - m;
      for (int b = G.kid_off[c]; b < G.kid_off[c + 1]; ++b) walk(T, G.kid_idx[b]);
    }
  };
  for (int a : top)
    for (int b : top) walk(a, b);
  // local expansions: nodes with translated sources and everything below them, top down
  std::vector<char> has_local(nsrc_all, 0);
  std::vector<int> order;   // tree nodes from the top level down
  for (int l = nclev; l >= 1; --l)
    for (size_t t = 0; t < plan[l].size(); ++t) order.push_back(m + cid[l][t]);
  for (int j = 0; j < m; ++j) order.push_back(j);
  G.loc_id.assign(nsrc_all, -1);
  G.loc_p.clear();
  G.loc_geo.clear();
  for (int v : order) {
    has_local[v] = !m2l[v].empty() || (parent[v] >= 0 && has_local[parent[v]]);
    if (!has_local[v]) continue;
    if (ptgt[v] > PMX_FMM_PL) fail(PMX_EGEOM, "operator apply: a local expansion beyond its largest order");
    G.loc_id[v] = (int)G.loc_p.size();
    G.loc_p.push_back(ptgt[v]);
    G.loc_geo.push_back(G.incl[4 * (size_t)v]);
    G.loc_geo.push_back(G.incl[4 * (size_t)v + 1]);
  }
  const int nloc = (int)G.loc_p.size();
  G.m2l_off.assign(1, 0);
  G.m2l_slot.clear();
  G.m2l_src.clear();
  G.m2l_nmax.clear();
  G.m2l_mmax.clear();
  G.m2l_toff.clear();
  G.m2l_tab = 0;
  double m2l_terms = 0, l2l_terms = 0, l2p_terms = 0;
  for (int v : order) {
    const int t = G.loc_id[v];
    if (t < 0) continue;
    for (const M2lPair& pr : m2l[v]) {
      const int V = pr.mmax + 1 + pr.nmax;
      G.m2l_slot.push_back(t);
      G.m2l_src.push_back(pr.src);
      G.m2l_nmax.push_back(pr.nmax);
      G.m2l_mmax.push_back(pr.mmax);
      G.m2l_toff.push_back(G.m2l_tab);
      G.m2l_tab += 2 * V + 1;
      m2l_terms += 2.0 * (2 * pr.mmax + 3) * (2 * pr.nmax + 1);
    }
    G.m2l_off.push_back((int)G.m2l_src.size());
  }
  // parent-to-child translations, grouped by the child's level from the top
  G.l2l_child.clear();
  G.l2l_parent.clear();
  G.l2l_toff.clear();
  G.l2l_lev.assign(1, 0);
  G.l2l_tab = 0;
  for (int l = nclev; l >= 1; --l) {
    for (int v : order) {
      if (lvl[v] != l - 1 || (l - 1 == 0 && v >= m) || parent[v] < 0 || !has_local[parent[v]]) continue;
      const int c = G.loc_id[v], P = G.loc_id[parent[v]];
      const int W = ptgt[parent[v]] + ptgt[v] + 2;
      G.l2l_child.push_back(c);
      G.l2l_parent.push_back(P);
      G.l2l_toff.push_back(G.l2l_tab);
      G.l2l_tab += 2 * W + 1;
      l2l_terms += 2.0 * (2 * ptgt[v] + 3) * (2 * ptgt[parent[v]] + 3);
    }
    G.l2l_lev.push_back((int)G.l2l_child.size());
  }
  // the waves' walks start from what their inclusion left over
  G.off.assign(nw + 1, 0);
  G.foff.assign(nw + 1, 0);
  G.idx.clear();
  G.fidx.clear();
  std::vector<int> stack, nearv, farv;
  double near_pairs = 0, far_orders = 0, far_pairs = 0;
  for (int w = 0; w < nw; ++w) {
    const double* gw = &G.wave[4 * (size_t)w];
    const double nt = (double)G.wave_node[2 * w + 1];
    const int own = wave_incl[w];
    if (G.loc_id[own] >= 0) l2p_terms += nt * (2 * ptgt[own] + 1);
    nearv.clear();
    farv.clear();
    stack.assign(leftover[own].rbegin(), leftover[own].rend());
    while (!stack.empty()) {
      const int sidx = stack.back();
      stack.pop_back();
      const double* g = &G.incl[4 * (size_t)sidx];
      const double rmin = std::hypot(gw[0] - g[0], gw[1] - g[1]) - gw[2];
      if (sidx >= m) {
        const int c = sidx - m;
        if (usable[c] && rmin >= PMX_APPLY_RATIO * g[2]) {
          const double p = std::max(g[3], std::ceil(PMX_APPLY_TRUNC / std::log(rmin / g[2])));
          if (p <= PMX_APPLY_PMAXC) {
            farv.push_back(sidx);
            far_orders += nt * (p + 2);
            far_pairs += nt;
            continue;
          }
        }
        for (int q = G.kid_off[c + 1] - 1; q >= G.kid_off[c]; --q) stack.push_back(G.kid_idx[q]);
      } else if (always[sidx] || rmin < PMX_APPLY_RATIO * g[2]) {
        nearv.push_back(sidx);
        near_pairs += nt * (double)(F->node_off[sidx + 1] - F->node_off[sidx]);
      } else {
        const double p = std::min((double)PMX_APPLY_PMAX, std::max(g[3], std::ceil(PMX_APPLY_TRUNC / std::log(rmin / g[2]))));
        farv.push_back(sidx);
        far_orders += nt * (p + 2);
        far_pairs += nt;
      }
    }
    std::sort(nearv.begin(), nearv.end());
    std::sort(farv.begin(), farv.end());
    G.idx.insert(G.idx.end(), nearv.begin(), nearv.end());
    G.fidx.insert(G.fidx.end(), farv.begin(), farv.end());
    G.off[w + 1] = (int)G.idx.size();
    G.foff[w + 1] = (int)G.fidx.size();
  }
  {
    double sn = 0, sm = 0;
    for (size_t q = 0; q < G.m2l_nmax.size(); ++q) {
      sn += G.m2l_nmax[q];
      sm += G.m2l_mmax[q];
    }
    const double np = std::max<double>(1.0, (double)G.m2l_nmax.size());
    G.stats[0] = (double)G.m2l_nmax.size();
    G.stats[1] = sn / np;
    G.stats[2] = sm / np;
    G.stats[3] = (double)nloc;
    G.stats[4] = (double)G.l2l_child.size();
    G.stats[5] = near_pairs;
    G.stats[6] = far_pairs;
    G.stats[7] = 16.0 * (double)(G.m2l_tab + G.l2l_tab);
  }
  if (count) {
    const double p2m = (double)N * (2 * (PMX_APPLY_PMAX + 3) + 1);
    // translations: 8 flops per complex multiply-add; evaluation of a local expansion:
    // three complex multiply-adds per order (value row, both derivative sums)
    G.flops_rhs = 32.0 * near_pairs + 48.0 * far_orders + 72.0 * p2m + 8.0 * m2m_terms + 8.0 * m2l_terms +
                  8.0 * l2l_terms + 24.0 * l2p_terms;
    G.flops_fixed = 130.0 * near_pairs + 100.0 * far_pairs + 26.0 * far_orders;
  }
}

void build_dense_apply(pmx_factor* F, int nrhs, const zd* dself, const std::vector<int>& incl,
                       const std::vector<int64_t>& doff, const zd* x, const zd* f, zd* out, DenseApply& D, Arena& A,
                       hipStream_t s) {
  const int64_t N2 = 2 * (int64_t)F->n_nodes;
  D.total = N2 * nrhs;
  // right-hand sides per thread and workgroups per launch: built-in 8 and 8192, or the
  // launch-parameter table's choice for this node count and right-hand-side count
  const int ta = tune_bucket_pow2(F->n_nodes), tb = tune_bucket_pow2(nrhs);
  D.nr_max = tune_choice(TK_APPLY_NR, 8, ta, tb, 0, 8, F->n_nodes, nrhs, 0);
  if (D.nr_max != 1 && D.nr_max != 2 && D.nr_max != 4 && D.nr_max != 8) D.nr_max = 8;
  const int wg = std::max(64, std::min(1 << 20, tune_choice(TK_APPLY_WG, 8, ta, tb, 0, 8192, F->n_nodes, nrhs, 0)));
  D.nsplit = apply_splits(F->n_nodes, wg);
  ApplyGeo G;
  if (F->apply_geo.valid()) {
    G = *F->apply_geo.get();
  } else {
    std::vector<double> hx, hy;
    download(hx, F->x, F->n_nodes, s);
    download(hy, F->y, F->n_nodes, s);
    apply_geometry(F, hx, hy, G, F->opts.timing != 0);
  }
  D.flops_fixed = G.flops_fixed;
  D.flops_rhs = G.flops_rhs;
  for (int i = 0; i < 8; ++i) F->info.apply_stats[i] = G.stats[i];
  const int nnear = apply_near_splits(F->n_nodes, wg);
  D.nslots = D.nsplit + nnear;
  D.ydiag = A.alloc<zd>(D.total);
  D.part = A.alloc<zd>(D.total * D.nslots);
  D.nblk = (int)std::min<int64_t>(64, (N2 + 4095) / 4096);
  D.d_norm = A.alloc<double>((int64_t)D.nblk * nrhs);
  std::vector<GemmArgs> ga(incl.size());
  D.max_s = 0;
  for (size_t t = 0; t < incl.size(); ++t) {
    int j = incl[t];
    int n2 = (int)(2 * (F->node_off[j + 1] - F->node_off[j]));
    ga[t] = GemmArgs{n2, nrhs, n2, dself + doff[t], n2, x + 2 * F->node_off[j], N2, D.ydiag + 2 * F->node_off[j], N2};
    D.max_s = std::max(D.max_s, n2);
    D.self_sq += (double)n2 * n2;
  }
  D.d_ga = A.upload(ga, s);
  D.n_ga = (int)ga.size();
  ApplyArgs& aa = D.aa;
  aa.x = F->x;
  aa.y = F->y;
  aa.nx = F->nx;
  aa.ny = F->ny;
  aa.w = F->w;
  aa.owner = F->owner;
  aa.node_off = F->d_node_off;
  aa.n_nodes = F->n_nodes;
  aa.k = F->k_ext;
  aa.eps = F->eps_ext;
  aa.xin = x;
  aa.nrhs = nrhs;
  aa.ld = N2;
  aa.part = D.part;
  aa.pack = A.alloc<double>(apply_pack_size(F->n_nodes, std::max(PMX_APPLY_NR_NEAR, 16)));
  aa.near_off = A.upload(G.off, s);
  aa.near_idx = A.upload(G.idx, s);
  aa.far_off = A.upload(G.foff, s);
  aa.far_idx = A.upload(G.fidx, s);
  aa.nsplit_near = nnear;
  aa.incl_geo = A.upload(G.incl, s);
  aa.wave_geo = A.upload(G.wave, s);
  aa.kid_off = A.upload(G.kid_off, s);
  aa.kid_idx = A.upload(G.kid_idx, s);
  aa.coef = A.alloc<zd>(apply_coef_size(F->m + G.n_clus, 8));
  aa.n_incl = F->m;
  aa.n_clus = G.n_clus;
  aa.n_lev = (int)G.lev_off.size() - 1;
  for (int l = 0; l <= aa.n_lev; ++l) aa.lev_off[l] = G.lev_off[l];
  aa.wave_node = A.upload(G.wave_node, s);
  aa.n_waves = (int)G.wave_node.size() / 2;
  // fast multipole part: local expansions, translation lists and their tables (made here,
  // once per solve state; they depend on the geometry only)
  aa.n_loc = (int)G.loc_p.size();
  aa.loc_id = A.upload(G.loc_id, s);
  aa.loc_p = A.upload(G.loc_p, s);
  aa.loc_geo = A.upload(G.loc_geo, s);
  aa.loc = A.alloc<zd>((int64_t)std::max(1, aa.n_loc) * 2 * PMX_FMM_NL * 8);
  aa.cm = A.alloc<zd>(apply_m2l_coef_size(F->m + G.n_clus, 8));
  aa.m2l_off = A.upload(G.m2l_off, s);
  {
    // work items: runs of at most PMX_FMM_CHUNK pairs of one local expansion (every slot
    // has at least one, so that its partial sums exist)
    std::vector<int> item, item_off(1, 0);
    for (int t = 0; t < (int)G.loc_p.size(); ++t) {
      const int q0 = G.m2l_off[t], q1 = G.m2l_off[t + 1];
      int q = q0;
      do {
        const int qe = std::min(q1, q + PMX_FMM_CHUNK);
        item.push_back(t);
        item.push_back(q);
        item.push_back(qe);
        q = qe;
      } while (q < q1);
      item_off.push_back((int)item.size() / 3);
    }
    aa.n_m2l_items = (int)item.size() / 3;
    aa.m2l_item = A.upload(item, s);
    aa.m2l_item_off = A.upload(item_off, s);
    aa.m2l_part = A.alloc<zd>((int64_t)std::max(1, aa.n_m2l_items) * 2 * PMX_FMM_NL * 8);
  }
  aa.m2l_slot = A.upload(G.m2l_slot, s);
  aa.m2l_src = A.upload(G.m2l_src, s);
  aa.m2l_nmax = A.upload(G.m2l_nmax, s);
  aa.m2l_mmax = A.upload(G.m2l_mmax, s);
  aa.m2l_toff = A.upload(G.m2l_toff, s);
  aa.m2l_tab = A.alloc<zd>(std::max<int64_t>(1, G.m2l_tab));
  aa.l2l_child = A.upload(G.l2l_child, s);
  aa.l2l_parent = A.upload(G.l2l_parent, s);
  aa.l2l_toff = A.upload(G.l2l_toff, s);
  aa.l2l_tab = A.alloc<zd>(std::max<int64_t>(1, G.l2l_tab));
  if ((int)G.l2l_lev.size() > PMX_APPLY_MAXLEV + 2) fail(PMX_EGEOM, "operator apply: too many tree levels");
  aa.n_l2l_lev = (int)G.l2l_lev.size() - 1;
  for (int l = 0; l <= aa.n_l2l_lev; ++l) aa.l2l_lev[l] = G.l2l_lev[l];
  asm_apply_tables(aa, (int)G.m2l_src.size(), (int)G.l2l_child.size(), s);
  // near pairs: the Bessel values of every (target, source node) pair stored once, when
  // they fit the budget and at least four right-hand sides share them
  aa.near_blk = nullptr;
  aa.near_blk_off = nullptr;
  D.near_pairs_stored = 0;
  {
    std::vector<int64_t> boff(G.idx.size());
    int64_t tot = 0;
    for (size_t q = 0; q < G.idx.size(); ++q) {
      boff[q] = tot;
      const int j = G.idx[q];
      tot += 2 * 64 * (F->node_off[j + 1] - F->node_off[j]);
    }
    if (nrhs >= 4 && tot > 0 && 16 * tot <= PMX_APPLY_NEAR_BYTES) {
      aa.near_blk = A.alloc<zd>(tot);
      aa.near_blk_off = A.upload(boff, s);
      asm_apply_near_build(aa, s);
      D.near_pairs_stored = G.stats[5];
    }
  }
  D.table_bytes = 16.0 * (double)(G.m2l_tab + G.l2l_tab);
  D.n_src = F->m + G.n_clus;
  D.f = f;
  D.out = out;
  D.nrhs = nrhs;
}

void launch_dense_apply(const DenseApply& D, hipStream_t s) {
  la_zgemm_apply_list(D.d_ga, D.n_ga, D.max_s, D.nrhs, s);
  asm_apply_off(D.aa, D.nsplit, D.nr_max, s);
  if (D.f)
    asm_apply_finish(D.f, D.ydiag, D.part, D.nslots, D.total, 1.0, -1.0, D.out, s);
  else
    asm_apply_finish(nullptr, D.ydiag, D.part, D.nslots, D.total, 0.0, 1.0, D.out, s);
}

// squared column norms of v (density layout, nrhs columns), partial sums on the device
void launch_norms(const DenseApply& D, const zd* v, hipStream_t s) {
  const int64_t N2 = D.total / D.nrhs;
  asm_colnorm2(v, N2, D.nrhs, N2, D.nblk, D.d_norm, s);
}

std::vector<double> read_norms(const DenseApply& D, hipStream_t s) {
  std::vector<double> part;
  download(part, D.d_norm, (size_t)D.nblk * D.nrhs, s);
  std::vector<double> out(D.nrhs, 0.0);
  for (int c = 0; c < D.nrhs; ++c)
    for (int b = 0; b < D.nblk; ++b) out[c] += part[(size_t)c * D.nblk + b];
  return out;
}

}  // namespace

// Everything a solve with a given right-hand-side count needs besides the factor: the
// leaf maps, plane-wave tables, internal input / output vectors (density layout, FP64),
// the refinement buffers and the captured graphs (one per launch sequence).
struct SolveState {
  int nrhs = -1;
  LeafMap map;
  int *d_node0 = nullptr, *d_nn = nullptr;
  int64_t* d_off = nullptr;
  double* d_angles = nullptr;
  std::vector<double> h_angles;
  int maxn = 0;
  zd *fin = nullptr, *xout = nullptr;   // general right-hand side, solution
  zd *f = nullptr, *r = nullptr, *leaf64 = nullptr;
  GatherDescT<double>* d_fin_to_leaf = nullptr;    // precision 0: fin -> leaf vectors
  GatherDescT<double>* d_leaf_to_x = nullptr;      // leaf (FP64) -> xout
  GatherDescT<double>* d_leaf64_to_f = nullptr;    // plane waves (inclusion layout) -> f, or -> fin
                                                   // when the leaf layout differs
  void* d_r_to_leaf = nullptr;                     // refinement: r -> leaf vectors (factor type)
  void* d_leafr_to_x = nullptr;                    // refinement: leaf (factor type) += -> xout
  DenseApply apply;
  hipGraphExec_t g_plane = nullptr, g_general = nullptr, g_iter = nullptr, g_apply = nullptr;
  Arena arena;
  explicit SolveState(DevPool* pool) : arena(pool) {}
  void drop_graphs() {
    for (hipGraphExec_t* g : {&g_plane, &g_general, &g_iter, &g_apply})
      if (*g) {
        (void)hipGraphExecDestroy(*g);
        *g = nullptr;
      }
  }
  void reset() {
    drop_graphs();
    arena.release();
    nrhs = -1;
  }
  ~SolveState() { drop_graphs(); }
};

pmx_factor::~pmx_factor() {
  if (gs) (void)hipStreamSynchronize(gs);
  ss.reset();
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (ev_out) (void)hipEventDestroy(ev_out);
  if (gs) (void)hipStreamDestroy(gs);
}

namespace {

template <class Fn>
hipGraphExec_t capture_graph(hipStream_t gs, Fn&& fn) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
  fn();
  const hipError_t e1 = hipStreamEndCapture(gs, &g);
  if (e1 != hipSuccess || !g) {
    (void)hipGetLastError();
    fail(PMX_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e1));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) fail(PMX_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e2));
  return ex;
}

// run a launch sequence, through its captured graph when graphs are on
template <class Fn>
void run_seq(pmx_factor* F, hipGraphExec_t& g, unsigned kernels, Fn&& fn) {
  // with per-kernel timing of a kernel launched inside the sequence (bit k of `kernels`:
  // kernel k) it runs launch by launch, bracketed by events
  if (!F->opts.solve_graph || (g_ktimer && (g_ktimer->mask & kernels))) {
    fn();
    return;
  }
  if (!g) g = capture_graph(F->gs, fn);
  HIPCHK(hipGraphLaunch(g, F->gs));
}

template <class R>
void ensure_state(pmx_factor* F, int nrhs) {
  SolveState& S = *F->ss;
  if (S.nrhs == nrhs) return;
  const double t0 = now_ms();
  S.reset();
  hipStream_t s = F->gs;
  Arena& A = S.arena;
  const double tp = now_ms();
  build_program<R>(F, nrhs, s);
  const double tl = now_ms();
  F->info.t_phase_ms[9] += tl - tp;
  {
    const Tier<R>& T = tier<R>(F);
    const bool same = F->lev0 == 0;
    if (T.lev.empty()) {
      const std::vector<int64_t> offS{0, (int64_t)T.root_rows.size()};
      build_leaf_map(F, nrhs, T.root_rows, T.root_cols, offS, 1, same, S.map, A, s);
    } else {
      build_leaf_map(F, nrhs, T.lev[0].rows, T.lev[0].cols, T.lev[0].offS, T.lev[0].ncell, same, S.map, A, s);
    }
  }
  F->info.t_phase_ms[10] += now_ms() - tl;
  const std::vector<CellPlan>& leaves = F->plan[0];
  const int nc = (int)leaves.size();
  std::vector<int> node0(nc), nn(nc);
  std::vector<int64_t> off(nc);
  int64_t o = 0;
  S.maxn = 0;
  for (int t = 0; t < nc; ++t) {
    int j = leaves[t].incl[0];
    node0[t] = (int)F->node_off[j];
    nn[t] = (int)(F->node_off[j + 1] - F->node_off[j]);
    off[t] = o * nrhs;
    o += 2 * nn[t];
    S.maxn = std::max(S.maxn, nn[t]);
  }
  S.d_node0 = A.upload(node0, s);
  S.d_nn = A.upload(nn, s);
  S.d_off = A.upload(off, s);
  S.d_angles = A.alloc<double>(nrhs);
  S.h_angles.assign(nrhs, 0.0);
  const int64_t total = 2 * (int64_t)F->n_nodes * nrhs;
  S.fin = A.alloc<zd>(total);
  S.xout = A.alloc<zd>(total);
  cx<R>* leaf = tier<R>(F).prog.leaf;
  if (F->opts.precision == 0) {
    S.d_fin_to_leaf = gather_to_leaf(S.map, (zd*)leaf, nrhs, A, s);
    S.d_leaf_to_x = gather_to_dens(S.map, S.xout, nrhs, A, s);
    if (!S.map.same) {   // plane waves: inclusion layout -> fin -> leaf vectors
      S.leaf64 = A.alloc<zd>(total);
      S.d_leaf64_to_f = gather_incl_to_dens(S.map, S.fin, nrhs, A, s);
    }
  } else {
    S.f = A.alloc<zd>(total);
    S.r = A.alloc<zd>(total);
    S.leaf64 = A.alloc<zd>(total);
    S.d_leaf64_to_f = gather_incl_to_dens(S.map, S.f, nrhs, A, s);
    S.d_r_to_leaf = gather_to_leaf(S.map, leaf, nrhs, A, s);
    S.d_leaf_to_x = gather_to_dens(S.map, S.xout, nrhs, A, s);
    const double ta = now_ms();
    build_dense_apply(F, nrhs, F->Dself, F->selfIncl, F->selfOff, S.xout, S.f, S.r, S.apply, A, s);
    F->info.t_phase_ms[6] += now_ms() - ta;
  }
  HIPCHK(hipStreamSynchronize(s));
  S.nrhs = nrhs;
  F->info.t_phase_ms[5] += now_ms() - t0;
}

void upload_angles(pmx_factor* F, const double* angles) {
  SolveState& S = *F->ss;
  std::copy(angles, angles + S.nrhs, S.h_angles.begin());
  HIPCHK(hipMemcpyAsync(S.d_angles, S.h_angles.data(), S.nrhs * sizeof(double), hipMemcpyHostToDevice, F->gs));
}

// Algorithmic work of one operator apply: the near pairs, the far expansions and the
// expansion sums (apply_geometry counts them) and the FP64 self-block product (8 flops per
// complex multiply-add).  Bytes (inputs read once, the output written once): the node
// data (x, y, normal, weight, owner), the self blocks, the densities and the right-hand
// side, and the residual.  Expansion records and partial sums are the implementation's
// own traffic and are not counted.
void count_apply_work(pmx_factor* F, int nrhs) {
  const DenseApply& D = F->ss->apply;
  const double N2 = 2.0 * F->n_nodes;
  // with stored near Bessel values, their evaluation (90 of the pair's 130 flops; the
  // geometry and the four coefficients, 40 flops, stay) leaves the apply and their reading
  // (two complex numbers a pair) enters it
  F->info.kernel_flops[PK_APPLY] +=
      D.flops_fixed - 90.0 * D.near_pairs_stored + D.flops_rhs * nrhs + 8.0 * D.self_sq * nrhs;
  F->info.kernel_bytes[PK_APPLY] +=
      8.0 * 5 * F->n_nodes + 16.0 * D.self_sq + 16.0 * N2 * nrhs * 3 + 32.0 * D.near_pairs_stored;
}

// FP64 factor: right-hand side into the leaf vectors, one solve pass, solution to xout.
void solve_fp64(pmx_factor* F, int nrhs, const double* angles, const zd* rhs) {
  ensure_state<double>(F, nrhs);
  SolveState& S = *F->ss;
  hipStream_t gs = F->gs;
  zd* leaf = F->t64.prog.leaf;
  const LeafMap& M = S.map;
  if (angles) {
    upload_angles(F, angles);
    const int ninc = (int)F->plan[0].size();
    run_seq(F, S.g_plane, PK_SOLVE_MASK, [&] {
      if (M.same) {
        asm_incident(F->geom(), F->ext(), S.d_node0, S.d_nn, S.d_off, ninc, S.maxn, S.d_angles, nrhs, leaf, gs);
      } else {
        asm_incident(F->geom(), F->ext(), S.d_node0, S.d_nn, S.d_off, ninc, S.maxn, S.d_angles, nrhs, S.leaf64, gs);
        asm_gather(S.leaf64, S.d_leaf64_to_f, 1, M.n2, nrhs, gs, 0);
        asm_gather(S.fin, S.d_fin_to_leaf, M.ncell, M.max_cell, nrhs, gs, 0);
      }
      launch_program<double>(F, gs);
      asm_gather(leaf, S.d_leaf_to_x, 1, M.n2, nrhs, gs, 0);
    });
  } else {
    HIPCHK(hipMemcpyAsync(S.fin, rhs, 2 * (int64_t)F->n_nodes * nrhs * sizeof(zd), hipMemcpyDeviceToDevice, gs));
    run_seq(F, S.g_general, PK_SOLVE_MASK, [&] {
      asm_gather(S.fin, S.d_fin_to_leaf, M.ncell, M.max_cell, nrhs, gs, 0);
      launch_program<double>(F, gs);
      asm_gather(leaf, S.d_leaf_to_x, 1, M.n2, nrhs, gs, 0);
    });
  }
}

// Refinement: the factor of type R as the inner solver of iterative refinement with the
// FP64 operator, x_0 = 0, r_i = f - A x_i, x_{i+1} = x_i + solve(r_i), until
// max_r |r_i| / |f| <= ir_tol.  One step is two captured graphs (the gathers and the solve
// pass; the operator apply) and the residual norms.
template <class R>
void solve_refined(pmx_factor* F, int nrhs, const double* angles, const zd* rhs) {
  ensure_state<R>(F, nrhs);
  SolveState& S = *F->ss;
  hipStream_t gs = F->gs;
  const LeafMap& M = S.map;
  const int64_t total = S.apply.total;
  if (angles) {
    upload_angles(F, angles);
    asm_incident(F->geom(), F->ext(), S.d_node0, S.d_nn, S.d_off, (int)F->plan[0].size(), S.maxn, S.d_angles,
                 nrhs, S.leaf64, gs);
    asm_gather(S.leaf64, S.d_leaf64_to_f, 1, M.n2, nrhs, gs, 0);
  } else {
    HIPCHK(hipMemcpyAsync(S.f, rhs, total * sizeof(zd), hipMemcpyDeviceToDevice, gs));
  }
  asm_convert(S.f, S.r, total, gs);
  asm_zero(S.xout, total, gs);
  launch_norms(S.apply, S.f, gs);
  const std::vector<double> fn = read_norms(S.apply, gs);
  cx<R>* leaf = tier<R>(F).prog.leaf;
  const GatherDescT<R>* r_to_leaf = (const GatherDescT<R>*)S.d_r_to_leaf;
  const int maxit = std::max(1, F->opts.ir_max_iter);
  double rel = 0;
  int it = 0;
  for (int h = 0; h < 16; ++h) F->info.ir_history[h] = 0;
  for (it = 1; it <= maxit; ++it) {
    run_seq(F, S.g_iter, PK_SOLVE_MASK & ~(1u << PK_APPLY), [&] {
      asm_gather(S.r, r_to_leaf, M.ncell, M.max_cell, nrhs, gs, 0);
      launch_program<R>(F, gs);
      asm_gather(leaf, S.d_leaf_to_x, 1, M.n2, nrhs, gs, 1);
    });
    {
      // the operator apply is a graph of its own, so that events can bracket it (timer
      // slot k_apply_off: every kernel of one apply) while it still replays as a graph
      KScope ks(PK_APPLY, gs);
      run_seq(F, S.g_apply, 1u << PK_ZGEMM, [&] { launch_dense_apply(S.apply, gs); });
    }
    launch_norms(S.apply, S.r, gs);
    count_apply_work(F, nrhs);
    const std::vector<double> rn = read_norms(S.apply, gs);
    rel = 0;
    for (int c = 0; c < nrhs; ++c) rel = std::max(rel, fn[c] > 0 ? std::sqrt(rn[c] / fn[c]) : std::sqrt(rn[c]));
    if (it <= 16) F->info.ir_history[it - 1] = rel;
    if (rel <= F->opts.ir_tol) break;
  }
  F->info.ir_iterations = std::min(it, maxit);
  F->info.ir_residual = rel;
  if (rel > F->opts.ir_tol) {
    char buf[160];
    snprintf(buf, sizeof(buf), "iterative refinement stopped at relative residual %.3e after %d steps", rel, maxit);
    throw PmxErr{PMX_ENOTCONV, buf};
  }
}

// Solves run on the factor's own stream (so that their launch sequences can be captured
// as graphs), ordered after the caller's stream and before its later work.
void solve_any(pmx_factor* F, int nrhs, const double* angles, const zd* rhs, zd* dens, hipStream_t s) {
  const double t0 = now_ms();
  std::unique_ptr<KernelTimer> kt;
  if (F->opts.timing) {
    kt.reset(new KernelTimer());
    if (F->opts.timing_kernels) kt->mask = F->opts.timing_kernels;
    g_ktimer = kt.get();
  }
  struct Reset {
    const TuneTable* prev;
    ~Reset() {
      g_ktimer = nullptr;
      g_tune = prev;
    }
  } reset_timer{g_tune};
  g_tune = F->tune.get();
  HIPCHK(hipEventRecord(F->ev_in, s));
  HIPCHK(hipStreamWaitEvent(F->gs, F->ev_in, 0));
  pmx_status late = PMX_OK;
  std::string late_msg;
  try {
    if (F->opts.precision == 1)
      solve_refined<float>(F, nrhs, angles, rhs);
    else if (F->opts.precision == 2)
      solve_refined<double>(F, nrhs, angles, rhs);
    else
      solve_fp64(F, nrhs, angles, rhs);
  } catch (const PmxErr& e) {
    if (e.st != PMX_ENOTCONV) throw;
    late = e.st;
    late_msg = e.msg;
  }
  // the last iterate is returned also when refinement did not converge
  HIPCHK(hipMemcpyAsync(dens, F->ss->xout, 2 * (int64_t)F->n_nodes * nrhs * sizeof(zd), hipMemcpyDeviceToDevice,
                        F->gs));
  HIPCHK(hipEventRecord(F->ev_out, F->gs));
  HIPCHK(hipStreamWaitEvent(s, F->ev_out, 0));
  sync_check(F->gs);
  if (kt) kt->collect(F->info.t_kernel_ms, F->info.n_kernel_launch);
  F->info.t_solve_ms = now_ms() - t0;
  if (late != PMX_OK) throw PmxErr{late, late_msg};
}

// ---------------------------------------------------------------------------------
// probe bodies, shared by the complex FP64 and FP32 entry points
template <class R>
void probe_gemm(int batch, int m, int n, int k, int opa, int opb, const cx<R>* A, const cx<R>* B, cx<R>* Cm,
                hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0 || k < 0 || (k > 0 && (!A || !B)) || !Cm || opa < 0 || opa > 2 || opb < 0 ||
      opb > 2)
    fail(PMX_EINVAL, "bad arguments");
  std::vector<GemmArgsT<R>> ga(batch);
  for (int b = 0; b < batch; ++b) {
    GemmArgsT<R>& g = ga[b];
    g.m = m;
    g.n = n;
    g.k = k;
    g.A = A + (int64_t)b * m * k;
    g.lda = opa == OP_N ? m : k;
    g.B = B + (int64_t)b * k * n;
    g.ldb = opb == OP_N ? k : n;
    g.C = Cm + (int64_t)b * m * n;
    g.ldc = m;
  }
  Arena tmp;
  la_zgemm_list<R>(opa, opb, tmp.upload(ga, s), batch, m, n, cmk<R>(1, 0), cmk<R>(0, 0), s);
  sync_check(s);
}

template <class R>
void probe_lu(int batch, int n, cx<R>* A, int* ipiv, int nrhs, cx<R>* B, int* info, int variant, hipStream_t s) {
  if (batch <= 0 || n <= 0 || nrhs < 0 || !A || !ipiv || (nrhs > 0 && !B) || !info || variant < -1 || variant > 2)
    fail(PMX_EINVAL, "bad arguments");
  Arena tmp;
  const bool small = nrhs > 0;
  int* perm = small ? tmp.alloc<int>((int64_t)batch * n) : nullptr;
  cx<R>* work = small ? tmp.alloc<cx<R>>((int64_t)batch * n * nrhs) : nullptr;
  std::vector<LuDescT<R>> lu(batch);
  std::vector<MatT<R>> bm(batch), wm(batch);
  for (int b = 0; b < batch; ++b) {
    lu[b] = LuDescT<R>{A + (int64_t)b * n * n, n, n, ipiv + (int64_t)b * n, small ? perm + (int64_t)b * n : nullptr};
    bm[b] = MatT<R>{nrhs > 0 ? B + (int64_t)b * n * nrhs : nullptr, n, n, nrhs};
    wm[b] = MatT<R>{small ? work + (int64_t)b * n * nrhs : nullptr, n, n, nrhs};
  }
  LuDescT<R>* d_lu = tmp.upload(lu, s);
  int* d_info = tmp.alloc<int>(batch);
  HIPCHK(hipMemsetAsync(d_info, 0, batch * sizeof(int), s));
  la_getrf<R>(d_lu, batch, n, d_info, s);
  if (nrhs > 0) {
    const MatT<R>* d_bm = tmp.upload(bm, s);
    const MatT<R>* d_wm = tmp.upload(wm, s);
    if (variant < 0) {
      level_getrs<R>(d_lu, d_bm, d_wm, batch, n, nrhs, s);
    } else {
      TuneForce saved = g_tune_force;
      g_tune_force = TuneForce{TK_GETRS, variant};
      level_getrs<R>(d_lu, d_bm, d_wm, batch, n, nrhs, s);
      g_tune_force = saved;
    }
  }
  std::vector<int> hi;
  download(hi, d_info, batch, s);
  std::copy(hi.begin(), hi.end(), info);
  sync_check(s);
}

template <class R>
void probe_id(int batch, int m, int c, cx<R>* M, double tol, const int* kmin, int* piv, int* rank, cx<R>* T,
              hipStream_t s) {
  if (batch <= 0 || m <= 0 || c <= 0 || !M || !piv || !rank || !T || !(tol > 0)) fail(PMX_EINVAL, "bad arguments");
  Arena tmp;
  const int mb = std::min(m, c);
  cx<R>* Rb = tmp.alloc<cx<R>>((int64_t)batch * mb * c);
  const int64_t wsz = la_geqrf_workspace(m);
  cx<R>* Vb = tmp.alloc<cx<R>>((int64_t)batch * wsz);
  cx<R>* VTb = tmp.alloc<cx<R>>((int64_t)batch * wsz);
  cx<R>* CVb = tmp.alloc<cx<R>>((int64_t)batch * c);
  double* taub = tmp.alloc<double>(batch);
  int* d_work = tmp.alloc<int>(1);
  double* nrm = tmp.alloc<double>((int64_t)batch * 2 * c);
  int* st = tmp.alloc<int>(4 * batch);
  double* r11 = tmp.alloc<double>(batch);
  std::vector<QrDescT<R>> qd(batch);
  std::vector<CpqrDescT<R>> cd(batch);
  for (int b = 0; b < batch; ++b) {
    qd[b] = QrDescT<R>{M + (int64_t)b * m * c, m, m, c, Rb + (int64_t)b * mb * c, Vb + (int64_t)b * wsz,
                       VTb + (int64_t)b * wsz, mb};
    cd[b] = CpqrDescT<R>{Rb + (int64_t)b * mb * c, mb, c, piv + (int64_t)b * c, nrm + (int64_t)b * 2 * c, st + 4 * b,
                         r11 + b, CVb + (int64_t)b * c, taub + b, c, nullptr};
  }
  QrDescT<R>* d_qd = tmp.upload(qd, s);
  CpqrDescT<R>* d_cd = tmp.upload(cd, s);
  la_geqrf_r<R>(d_qd, batch, m, c, s);
  HIPCHK(la_cpqr<R>(d_cd, batch, c, tol, nullptr, 1, d_work, s));
  std::vector<int> sth;
  download(sth, st, 4 * batch, s);
  std::vector<int> k(batch);
  for (int b = 0; b < batch; ++b) {
    rank[b] = sth[4 * b + 1];
    k[b] = std::max(rank[b], kmin ? kmin[b] : 0);
    k[b] = std::max(1, std::min(k[b], mb));
  }
  int* d_k = tmp.upload(k, s);
  HIPCHK(la_cpqr<R>(d_cd, batch, c, 0.0, d_k, 0, d_work, s));
  download(sth, st, 4 * batch, s);
  for (int b = 0; b < batch; ++b) k[b] = std::min(k[b], sth[4 * b]);
  HIPCHK(hipMemcpyAsync(d_k, k.data(), batch * sizeof(int), hipMemcpyHostToDevice, s));
  la_cpqr_tsolve<R>(d_cd, d_k, batch, c, c, s);
  // T[b] (c x c, ld c): rows 0..k-1 hold R11^-1 R12 in columns 0..c-k-1
  std::vector<RowSrc> rs;
  std::vector<GatherDescT<R>> gd(batch);
  for (int b = 0; b < batch; ++b)
    for (int i = 0; i < k[b]; ++i) rs.push_back(RowSrc{(int64_t)b * mb * c + i + (int64_t)k[b] * mb, mb});
  RowSrc* d_rs = tmp.upload(rs, s);
  int64_t ro = 0;
  for (int b = 0; b < batch; ++b) {
    gd[b] = GatherDescT<R>{d_rs + ro, c - k[b] > 0 ? k[b] : 0, c - k[b], T + (int64_t)b * c * c, c};
    ro += k[b];
  }
  asm_gather(Rb, tmp.upload(gd, s), batch, c, c, s);
  sync_check(s);
}

HostGeom host_geom(const pmx_geometry* g) {
  HostGeom h;
  h.m = g->m;
  h.node_off = g->node_off;
  h.x = g->x;
  h.y = g->y;
  h.dx = g->dx;
  h.dy = g->dy;
  h.ddx = g->ddx;
  h.ddy = g->ddy;
  h.k_ext = g->k_ext;
  h.k_int = g->k_int;
  return h;
}

MlpModel load_model(const char* path) {
  if (!path) fail(PMX_EINVAL, "learned IDs need a model path");
  MlpModel m;
  std::string err = mlp_load(path, m);
  if (!err.empty()) fail(PMX_EINVAL, err);
  if (m.sh.nin != PMX_NFEAT || m.sh.nout != PMX_NOUT) fail(PMX_EINVAL, "model shape does not match the features");
  return m;
}

void leaf_predictions(pmx_factor* F, const pmx_geometry* g, const char* path, hipStream_t s) {
  const MlpModel m = load_model(path);
  std::vector<float> X;
  leaf_features(host_geom(g), F->plan[0], X);
  try {
    mlp_predict(m, X, (int64_t)X.size() / PMX_NFEAT, F->leaf_pred, s);
  } catch (const std::exception& e) {
    fail(PMX_EHIP, e.what());
  }
}

// Autotuner, dense apply: times the right-hand-side grouping and source-split candidates
// of the recorded apply shapes on the factor's own apply state (after a solve), best of
// reps launches after a warm-up, within a time budget (candidates in a fixed order, the
// built-in choice first), and stores the fastest pair.
void tune_apply(pmx_factor* F, const TuneRecorder& rec, TuneTable& t, int reps, hipStream_t s) {
  if (!F->ss || F->ss->nrhs <= 0 || F->opts.precision == 0) return;
  DenseApply& D = F->ss->apply;
  const int ta = tune_bucket_pow2(F->n_nodes), tb = tune_bucket_pow2(D.nrhs);
  const uint64_t knr = tune_key(TK_APPLY_NR, 8, ta, tb, 0), kwg = tune_key(TK_APPLY_WG, 8, ta, tb, 0);
  if (!rec.dims.count(knr) || !rec.dims.count(kwg)) return;
  int cnr[8], nnr = 0, cwg[8], nwg = 0;
  tune_candidates(TK_APPLY_NR, 8, F->n_nodes, D.nrhs, 0, cnr, &nnr);
  tune_candidates(TK_APPLY_WG, 8, F->n_nodes, D.nrhs, 0, cwg, &nwg);
  std::vector<std::pair<int, int>> cand{{8, 8192}};
  for (int i = 0; i < nnr; ++i)
    for (int j = 0; j < nwg; ++j)
      if (!(cnr[i] == 8 && cwg[j] == 8192)) cand.push_back({cnr[i], cwg[j]});
  Arena tmp;
  std::map<int, zd*> parts;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  ApplyArgs aa = D.aa;
  const double budget_ms = 30000.0;
  double spent = 0, best = 1e300;
  int bi = 0;
  std::string note;
  for (size_t c = 0; c < cand.size() && spent < budget_ms; ++c) {
    const int ns = apply_splits(F->n_nodes, cand[c].second);
    aa.nsplit_near = apply_near_splits(F->n_nodes, cand[c].second);
    const int slots = ns + aa.nsplit_near;
    if (!parts.count(slots)) parts[slots] = tmp.alloc<zd>(D.total * slots);
    aa.part = parts[slots];
    double tbest = 1e300;
    for (int r = 0; r <= reps; ++r) {
      HIPCHK(hipEventRecord(e0, s));
      asm_apply_off(aa, ns, cand[c].first, s);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      spent += ms;
      if (r > 0 || ms > 500.0f) tbest = std::min(tbest, (double)ms);   // long launches: no separate warm-up
      if (ms > 500.0f && r >= 1) break;
    }
    note += (note.empty() ? "" : " ") + std::to_string(cand[c].first) + "/" + std::to_string(cand[c].second) + ":" +
            std::to_string((int64_t)std::llround(1e3 * tbest));
    if (tbest < best) {
      best = tbest;
      bi = (int)c;
    }
  }
  HIPCHK(hipGetLastError());
  t.val[knr] = cand[bi].first;
  t.val[kwg] = cand[bi].second;
  t.note[knr] = "nr/wg:us " + note;
  t.note[kwg] = "chosen with apply_nr";
}

template <class Fn>
pmx_status guarded(Fn&& fn) {
  try {
    fn();
    return PMX_OK;
  } catch (const PmxErr& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PMX_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PMX_EINVAL;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------
extern "C" {

void pmx_options_default(pmx_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->id_tol = 1e-10;
  o->proxy_ratio = 1.5;
  o->proxy_min = 0;
  o->proxy_rule = 0;
  o->near_rule = 0;
  o->precision = 0;
  o->timing = 0;
  o->ir_max_iter = 10;
  o->ir_tol = 1e-10;
  o->solve_graph = 1;
  o->learned = 0;
  o->model_path = nullptr;
  o->tree = 0;
  o->leaf_size = 4;
  o->eta = 1.0;
}

pmx_status pmx_factor_create(const pmx_geometry* geom, const pmx_options* opts, void* hip_stream,
                             pmx_factor** out) {
  return guarded([&] {
    if (!out) fail(PMX_EINVAL, "out is NULL");
    *out = nullptr;
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    validate(geom, &o);
    hipStream_t s = (hipStream_t)hip_stream;
    std::unique_ptr<pmx_factor> F(new pmx_factor());
    std::memset(&F->info, 0, sizeof(F->info));
    F->opts = o;
    F->lev0 = plan_pass_through(plan_options(geom, o)) ? 1 : 0;
    if (o.refactor && o.learned) fail(PMX_EINVAL, "refactor = 1 needs learned = 0");
    F->num.on = o.refactor != 0;
    const int64_t launches0 = g_launches, syncs0 = g_syncs;
    if (o.tune_path) {
      F->tune.reset(new TuneTable());
      const std::string e = tune_load(o.tune_path, *F->tune);
      if (!e.empty()) fail(PMX_EINVAL, e);
    }
    F->opts.tune_path = nullptr;   // read here only
    const double t0 = now_ms();
    std::unique_ptr<KernelTimer> kt;
    if (o.timing) {
      kt.reset(new KernelTimer());
      if (o.timing_kernels) kt->mask = o.timing_kernels;
      g_ktimer = kt.get();
    }
    struct Reset {
      const TuneTable* prev;
      ~Reset() {
        g_ktimer = nullptr;
        g_tune = prev;
      }
    } reset_timer{g_tune};
    g_tune = F->tune.get();
    // the plan is made on a host thread while the geometry and, in the refined forms, the
    // FP64 self blocks (which need no plan) go to the device
    double plan_ms = 0;
    pmx_factor* Fp = F.get();
    auto plan_job = std::async(std::launch::async, [geom, &o, Fp, &plan_ms] {
      const double tp = now_ms();
      make_plan(geom, o, Fp->plan);
      if (Fp->lev0 && (int)Fp->plan[Fp->lev0].size() > PMX_MAX_MULTI_LEAVES)
        fail(PMX_EINVAL, "leaves of several inclusions are supported up to " + std::to_string(PMX_MAX_MULTI_LEAVES) +
                             " leaves (this plan has " + std::to_string(Fp->plan[Fp->lev0].size()) + ")");
      plan_ms = now_ms() - tp;
    });
    try {
      HIPCHK(hipStreamCreateWithFlags(&F->gs, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&F->ev_in, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&F->ev_out, hipEventDisableTiming));
      F->ss.reset(new SolveState(&F->pool));
      if (o.learned) {
        plan_job.get();
        const double tl = now_ms();
        leaf_predictions(F.get(), geom, o.model_path, s);
        F->info.t_phase_ms[8] = now_ms() - tl;
      }
      upload_geometry(F.get(), geom, s);
      if (o.precision != 0) self_blocks_by_inclusion(F.get(), s);
    } catch (...) {
      if (plan_job.valid()) plan_job.get();   // an unsupported geometry is reported first
      throw;
    }
    if (plan_job.valid()) plan_job.get();
    F->info.t_phase_ms[4] = plan_ms;
    if (o.precision != 0) {
      // host copies of the coordinates (the caller's arrays may go away after this call)
      const int64_t N = geom->node_off[geom->m];
      auto hx = std::make_shared<std::vector<double>>(geom->x, geom->x + N);
      auto hy = std::make_shared<std::vector<double>>(geom->y, geom->y + N);
      const pmx_factor* Fc = F.get();
      const bool count = o.timing != 0;
      F->apply_geo = std::async(std::launch::async, [Fc, hx, hy, count] {
        auto G = std::make_shared<ApplyGeo>();
        apply_geometry(Fc, *hx, *hy, *G, count);
        return G;
      });
    }
    if (o.precision == 1) {
      factor_all<float>(F.get(), s);
      fill_info<float>(F.get());
    } else {
      factor_all<double>(F.get(), s);
      fill_info<double>(F.get());
    }
    F->info.t_factor_ms = now_ms() - t0;
    F->info.factor_launches = g_launches - launches0;
    F->info.factor_host_syncs = g_syncs - syncs0;
    if (kt) {
      HIPCHK(hipStreamSynchronize(s));
      kt->collect(F->info.t_kernel_ms, F->info.n_kernel_launch);
    }
    *out = F.release();
  });
}

pmx_status pmx_autotune(const pmx_geometry* geom, const pmx_options* opts, int32_t nrhs, int32_t reps,
                        const char* path, void* hip_stream) {
  return guarded([&] {
    if (!geom || !path || nrhs < 1 || nrhs > 256 || reps < 1 || reps > 50) fail(PMX_EINVAL, "bad arguments to pmx_autotune");
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    o.timing = 0;
    o.tune_path = nullptr;
    o.solve_graph = 0;
    hipStream_t s = (hipStream_t)hip_stream;
    TuneRecorder rec;
    struct RecReset {
      ~RecReset() { g_tune_rec = nullptr; }
    } rec_reset;
    // pass 1: the workload with every tunable launch shape recorded
    g_tune_rec = &rec;
    pmx_factor* raw = nullptr;
    pmx_status st = pmx_factor_create(geom, &o, hip_stream, &raw);
    if (st != PMX_OK) throw PmxErr{st, g_last_error};
    std::unique_ptr<pmx_factor> F(raw);
    Arena tmp;
    zd* dens = tmp.alloc<zd>(2 * (int64_t)F->n_nodes * nrhs);
    std::vector<double> ang(nrhs);
    for (int r = 0; r < nrhs; ++r) ang[r] = 2.0 * M_PI * r / nrhs;
    st = pmx_solve_plane_waves(F.get(), nrhs, ang.data(), (pmx_c64*)dens, hip_stream);
    if (st != PMX_OK) throw PmxErr{st, g_last_error};
    g_tune_rec = nullptr;
    // pass 2: every candidate of every recorded shape, timed
    TuneTable t;
    const std::string e = tune_linear_algebra(rec, t, reps, s);
    if (!e.empty()) fail(PMX_EHIP, e);
    tune_apply(F.get(), rec, t, reps, s);
    sync_check(s);
    const std::string w = tune_save(path, t);
    if (!w.empty()) fail(PMX_EINVAL, w);
  });
}

pmx_status pmx_solve_plane_waves(pmx_factor* f, int32_t nrhs, const double* angles, pmx_c64* dens,
                                 void* hip_stream) {
  return guarded([&] {
    if (!f || !angles || !dens || nrhs <= 0) fail(PMX_EINVAL, "bad arguments to pmx_solve_plane_waves");
    for (int r = 0; r < nrhs; ++r)
      if (!std::isfinite(angles[r])) fail(PMX_EINVAL, "non-finite angle");
    solve_any(f, nrhs, angles, nullptr, (zd*)dens, (hipStream_t)hip_stream);
  });
}

pmx_status pmx_solve(pmx_factor* f, int32_t nrhs, const pmx_c64* rhs, pmx_c64* dens, void* hip_stream) {
  return guarded([&] {
    if (!f || !rhs || !dens || nrhs <= 0) fail(PMX_EINVAL, "bad arguments to pmx_solve");
    if ((const void*)rhs == (const void*)dens) fail(PMX_EINVAL, "rhs and dens overlap");
    solve_any(f, nrhs, nullptr, (const zd*)rhs, (zd*)dens, (hipStream_t)hip_stream);
  });
}

pmx_status pmx_far_field(const pmx_factor* f, int32_t nrhs, const pmx_c64* dens, int32_t ndir,
                         const double* dirs, pmx_c64* out, void* hip_stream) {
  return guarded([&] {
    if (!f || !dens || !dirs || !out || nrhs <= 0 || ndir <= 0) fail(PMX_EINVAL, "bad arguments to pmx_far_field");
    hipStream_t s = (hipStream_t)hip_stream;
    Arena tmp;
    zd* part = tmp.alloc<zd>(far_field_part_bytes(f->n_nodes, nrhs, ndir) / sizeof(zd));
    asm_far_field(f->geom(), f->ext(), f->owner, f->d_node_off, (const zd*)dens, nrhs, dirs, ndir, part, (zd*)out,
                  s);
    sync_check(s);
  });
}

pmx_status pmx_far_field_noalloc(const pmx_factor* f, int32_t nrhs, const pmx_c64* dens, int32_t ndir,
                                 const double* dirs, pmx_c64* out, void* hip_stream) {
  return guarded([&] {
    if (!f || !dens || !dirs || !out || nrhs <= 0 || ndir <= 0)
      fail(PMX_EINVAL, "bad arguments to pmx_far_field_noalloc");
    const size_t need = far_field_part_bytes(f->n_nodes, nrhs, ndir);
    if (need > PMX_FF_SCRATCH_BYTES)
      fail(PMX_EINVAL, "pmx_far_field_noalloc: " + std::to_string(nrhs) + " right-hand sides x " +
                           std::to_string(ndir) + " directions need " + std::to_string(need) +
                           " bytes of partial sums, more than its static " + std::to_string(PMX_FF_SCRATCH_BYTES) +
                           " (at most 524288 right-hand-side/direction pairs)");
    zd* part = nullptr;
    const hipError_t e = far_field_scratch(&part);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(PMX_EHIP, std::string("pmx_far_field_noalloc: no device address for its static array: ") +
                         hipGetErrorString(e));
    }
    hipStream_t s = (hipStream_t)hip_stream;
    asm_far_field(f->geom(), f->ext(), f->owner, f->d_node_off, (const zd*)dens, nrhs, dirs, ndir, part, (zd*)out,
                  s);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) fail(PMX_EHIP, std::string("pmx_far_field_noalloc launch: ") + hipGetErrorString(le));
  });
}

pmx_status pmx_factor_info(const pmx_factor* f, pmx_info* info) {
  return guarded([&] {
    if (!f || !info) fail(PMX_EINVAL, "NULL argument");
    *info = f->info;
  });
}

pmx_status pmx_factor_refactor(pmx_factor* F, const double* k_int, const double* eps_int, void* hip_stream) {
  return guarded([&] {
    if (!F) fail(PMX_EINVAL, "factor is NULL");
    if (!F->num.on) fail(PMX_EINVAL, "the factor was created without options.refactor = 1");
    if (!k_int) fail(PMX_EINVAL, "k_int is NULL");
    for (int j = 0; j < F->m; ++j) {
      if (!(k_int[j] > 0) || !std::isfinite(k_int[j])) fail(PMX_EINVAL, "k_int must be positive");
      if (eps_int && (!(eps_int[j] > 0) || !std::isfinite(eps_int[j]))) fail(PMX_EINVAL, "eps_int must be positive");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const double t0 = now_ms();
    const int64_t launches0 = g_launches, syncs0 = g_syncs;
    struct Reset {
      const TuneTable* prev;
      ~Reset() { g_tune = prev; }
    } reset_tune{g_tune};
    g_tune = F->tune.get();   // the launch choices of create, for the capture
    KernelTimer* kt_prev = g_ktimer;
    g_ktimer = nullptr;       // no events inside the captured sequence
    struct ResetT {
      KernelTimer* prev;
      ~ResetT() { g_ktimer = prev; }
    } reset_timer{kt_prev};
    for (int j = 0; j < F->m; ++j) {
      F->k_int[j] = k_int[j];
      const double r = k_int[j] / F->k_ext;
      F->eps_int[j] = eps_int ? eps_int[j] : F->eps_ext * r * r;
    }
    HIPCHK(hipEventRecord(F->ev_in, s));
    HIPCHK(hipStreamWaitEvent(F->gs, F->ev_in, 0));
    // the interior media enter through the self-block descriptors, rewritten in place
    // (stream-ordered, before the replay; the previous call's replay has completed)
    for (NumProgram::Diag& d : F->num.diags) {
      for (size_t t = 0; t < d.incl.size(); ++t) {
        d.host[t].k_int = F->k_int[d.incl[t]];
        d.host[t].eps_int = F->eps_int[d.incl[t]];
      }
      HIPCHK(hipMemcpyAsync(d.dev, d.host.data(), d.host.size() * sizeof(DiagDesc), hipMemcpyHostToDevice, F->gs));
    }
    int64_t captured = 0;   // launches recorded into the graph (not made) by this call
    if (!F->num.graph) {
      const int64_t l0 = g_launches;
      F->num.graph = capture_graph(F->gs, [&] {
        for (auto& f : F->num.steps) f(F->gs);
      });
      F->num.nodes = captured = g_launches - l0;
    }
    pmx_count_launch();
    HIPCHK(hipGraphLaunch(F->num.graph, F->gs));
    // one wait for every LU pivot check of the replay
    std::vector<std::vector<int>> hi(F->num.infos.size());
    for (size_t i = 0; i < hi.size(); ++i) {
      hi[i].resize(F->num.infos[i].second);
      HIPCHK(hipMemcpyAsync(hi[i].data(), F->num.infos[i].first, hi[i].size() * sizeof(int), hipMemcpyDeviceToHost,
                            F->gs));
    }
    sync_check(F->gs);
    for (const std::vector<int>& v : hi)
      for (int x : v)
        if (x) fail(PMX_ESINGULAR, "zero pivot in an LU of the refactorisation");
    HIPCHK(hipEventRecord(F->ev_out, F->gs));
    HIPCHK(hipStreamWaitEvent(s, F->ev_out, 0));
    F->info.refactor_launches = g_launches - launches0 - captured;
    F->info.refactor_graph_nodes = F->num.nodes;
    F->info.refactor_host_syncs = g_syncs - syncs0;
    F->info.t_refactor_ms = now_ms() - t0;
  });
}

void pmx_factor_destroy(pmx_factor* f) { delete f; }

pmx_status pmx_device_cache(int64_t limit, int64_t* held) {
  return guarded([&] {
    if (limit >= 0) {
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache_limit = (size_t)limit;
      }
      cache_trim((size_t)limit);
      if (limit == 0) {   // the idle pinned staging chunks go as well
        std::lock_guard<std::mutex> lk(g_pin_mu);
        for (const auto& c : g_pin_free) (void)hipHostFree(c.first);
        g_pin_free.clear();
      }
    }
    if (held) {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      *held = (int64_t)g_cache_bytes;
    }
  });
}

const char* pmx_status_string(pmx_status s) {
  switch (s) {
    case PMX_OK: return "ok";
    case PMX_EINVAL: return "invalid argument";
    case PMX_EGEOM: return "unsupported geometry";
    case PMX_ENOMEM: return "out of device memory";
    case PMX_EHIP: return "HIP runtime error";
    case PMX_ESINGULAR: return "singular block";
    case PMX_ENOTCONV: return "iterative refinement did not converge";
  }
  return "unknown status";
}

const char* pmx_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------------
// probes
pmx_status pmx_probe_bessel(const double* z, int64_t n, double* out, void* stream) {
  return guarded([&] {
    if (!z || !out || n <= 0) fail(PMX_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    asm_probe_bessel(z, n, out, s);
    sync_check(s);
  });
}

pmx_status pmx_probe_diag_block_quad(const pmx_geometry* geom, int32_t j, int32_t quadrature, pmx_c64* out,
                                     void* stream) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    o.quadrature = quadrature;
    validate(geom, &o);
    if (j < 0 || j >= geom->m || !out) fail(PMX_EINVAL, "bad inclusion index");
    hipStream_t s = (hipStream_t)stream;
    pmx_factor F;
    F.opts = o;
    upload_geometry(&F, geom, s);
    Arena tmp;
    std::vector<int> incl{j};
    std::vector<int64_t> off{0};
    assemble_diag(&F, tmp, incl, (zd*)out, off, s);
    sync_check(s);
  });
}

pmx_status pmx_probe_diag_block(const pmx_geometry* geom, int32_t j, pmx_c64* out, void* stream) {
  return pmx_probe_diag_block_quad(geom, j, 0, out, stream);
}

pmx_status pmx_probe_entries(const pmx_geometry* geom, int32_t nr, const int32_t* rows, const int32_t* rtyp,
                             int32_t nc, const int32_t* cols, const int32_t* ctyp, pmx_c64* out, void* stream) {
  return guarded([&] {
    validate(geom, nullptr);
    if (nr <= 0 || nc <= 0 || !rows || !rtyp || !cols || !ctyp || !out) fail(PMX_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    pmx_factor F;
    upload_geometry(&F, geom, s);
    std::vector<int> a(nr), b(nc);
    for (int i = 0; i < nr; ++i) {
      if (rows[i] < 0 || rows[i] >= F.n_nodes || (rtyp[i] & ~1)) fail(PMX_EINVAL, "bad row");
      a[i] = pmx_code_node(rows[i], rtyp[i]);
    }
    for (int i = 0; i < nc; ++i) {
      if (cols[i] < 0 || cols[i] >= F.n_nodes || (ctyp[i] & ~1)) fail(PMX_EINVAL, "bad column");
      b[i] = pmx_code_node(cols[i], ctyp[i]);
    }
    Arena tmp;
    std::vector<EntryMat> em{EntryMat{tmp.upload(a, s), tmp.upload(b, s), nr, nc, (zd*)out, nr, 1}};
    asm_entries(F.geom(), DevProxy{nullptr, nullptr, nullptr, nullptr, nullptr}, F.ext(), tmp.upload(em, s), 1, nr,
                nc, s);
    sync_check(s);
  });
}

pmx_status pmx_probe_zgemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t opa, int32_t opb,
                           const pmx_c64* A, const pmx_c64* B, pmx_c64* C, void* stream) {
  return guarded([&] { probe_gemm<double>(batch, m, n, k, opa, opb, (const zd*)A, (const zd*)B, (zd*)C,
                                          (hipStream_t)stream); });
}

pmx_status pmx_probe_cgemm(int32_t batch, int32_t m, int32_t n, int32_t k, int32_t opa, int32_t opb,
                           const pmx_c32* A, const pmx_c32* B, pmx_c32* C, void* stream) {
  return guarded([&] { probe_gemm<float>(batch, m, n, k, opa, opb, (const zf*)A, (const zf*)B, (zf*)C,
                                         (hipStream_t)stream); });
}

pmx_status pmx_probe_lu_solve(int32_t batch, int32_t n, pmx_c64* A, int32_t* ipiv, int32_t nrhs, pmx_c64* B,
                              int32_t* info, int32_t variant, void* stream) {
  return guarded(
      [&] { probe_lu<double>(batch, n, (zd*)A, ipiv, nrhs, (zd*)B, info, variant, (hipStream_t)stream); });
}

pmx_status pmx_probe_lu_solve_c32(int32_t batch, int32_t n, pmx_c32* A, int32_t* ipiv, int32_t nrhs, pmx_c32* B,
                                  int32_t* info, int32_t variant, void* stream) {
  return guarded(
      [&] { probe_lu<float>(batch, n, (zf*)A, ipiv, nrhs, (zf*)B, info, variant, (hipStream_t)stream); });
}

pmx_status pmx_probe_id(int32_t batch, int32_t m, int32_t c, pmx_c64* M, double tol, const int32_t* kmin,
                        int32_t* piv, int32_t* rank, pmx_c64* T, void* stream) {
  return guarded([&] { probe_id<double>(batch, m, c, (zd*)M, tol, kmin, piv, rank, (zd*)T, (hipStream_t)stream); });
}

pmx_status pmx_probe_id_c32(int32_t batch, int32_t m, int32_t c, pmx_c32* M, double tol, const int32_t* kmin,
                            int32_t* piv, int32_t* rank, pmx_c32* T, void* stream) {
  return guarded([&] { probe_id<float>(batch, m, c, (zf*)M, tol, kmin, piv, rank, (zf*)T, (hipStream_t)stream); });
}

pmx_status pmx_probe_apply(const pmx_geometry* geom, int32_t nrhs, const pmx_c64* x, pmx_c64* y, void* stream) {
  return guarded([&] {
    validate(geom, nullptr);
    if (nrhs <= 0 || !x || !y || (const void*)x == (const void*)y) fail(PMX_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    pmx_factor F;
    pmx_options_default(&F.opts);
    make_plan(geom, F.opts, F.plan);   // the tree of the expansion clusters
    upload_geometry(&F, geom, s);
    Arena tmp;
    std::vector<int> incl(geom->m);
    std::vector<int64_t> off(geom->m);
    int64_t o = 0;
    for (int j = 0; j < geom->m; ++j) {
      incl[j] = j;
      off[j] = o;
      const int64_t n = geom->node_off[j + 1] - geom->node_off[j];
      o += 4 * n * n;
    }
    zd* dself = tmp.alloc<zd>(o);
    assemble_diag(&F, tmp, incl, dself, off, s);
    DenseApply D;
    build_dense_apply(&F, nrhs, dself, incl, off, (const zd*)x, nullptr, (zd*)y, D, tmp, s);
    launch_dense_apply(D, s);
    sync_check(s);
  });
}

void pmx_mlp_opts_default(pmx_mlp_opts* o) {
  if (!o) return;
  TrainOpts d;
  o->epochs = d.epochs;
  o->batch = d.batch;
  o->hidden = d.hidden;
  o->layers = d.layers;
  o->lr = d.lr;
  o->wmse = d.wmse;
  o->seed = d.seed;
}

pmx_status pmx_id_dataset(const pmx_geometry* geom, const pmx_options* opts, const char* path, int32_t append,
                          void* stream) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    o.precision = 0;
    o.learned = 0;
    validate(geom, &o);
    if (!path) fail(PMX_EINVAL, "path is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (plan_pass_through(plan_options(geom, o))) fail(PMX_EINVAL, "leaf IDs need one inclusion per leaf");
    pmx_factor F;
    F.opts = o;
    make_plan(geom, o, F.plan);
    if (F.plan.size() < 2) fail(PMX_EGEOM, "a single cell has no leaf IDs");
    upload_geometry(&F, geom, s);
    LevelData<double> L0;
    std::vector<int> incl;
    leaf_level(&F, L0, incl);
    Arena tmp;
    ProxyTable PT = make_proxies(tmp, F.plan[0], s);
    IdOut<double> io;
    id_stage<double>(&F, L0, F.plan[0], PT, nullptr, io, tmp, s, false);
    // labels: skeleton membership of every node for the four IDs, and their ranks k / n
    const int nc = L0.ncell;
    std::vector<float> X, Y((size_t)PMX_NOUT * L0.tot_s / 2, 0.0f);
    leaf_features(host_geom(geom), F.plan[0], X);
    int64_t first = 0;
    for (int t = 0; t < nc; ++t) {
      const int n = L0.s0[t];
      for (int kd = 0; kd < 4; ++kd) {
        const int q = 4 * t + kd;
        const int k = io.kq[q];
        for (int i = 0; i < k; ++i) Y[(size_t)PMX_NOUT * (first + io.piv[io.offC[q] + i]) + kd] = 1.0f;
        for (int i = 0; i < n; ++i) Y[(size_t)PMX_NOUT * (first + i) + 4 + kd] = (float)k / n;
      }
      first += n;
    }
    std::string err = dataset_append(path, append != 0, X, Y, first, PMX_NFEAT, PMX_NOUT);
    if (!err.empty()) fail(PMX_EINVAL, err);
  });
}

pmx_status pmx_mlp_train(const char* data_path, const pmx_mlp_opts* opts, const char* model_path, double* final_loss,
                         void* stream) {
  return guarded([&] {
    if (!data_path || !model_path) fail(PMX_EINVAL, "NULL path");
    pmx_mlp_opts mo;
    pmx_mlp_opts_default(&mo);
    if (opts) mo = *opts;
    if (mo.epochs < 1 || mo.batch < 16 || mo.hidden < 8 || mo.hidden > 2048 || mo.layers < 1 || mo.layers > 16 ||
        !(mo.lr > 0) || !(mo.wmse >= 0))
      fail(PMX_EINVAL, "bad training options");
    std::vector<float> X, Y;
    int64_t n = 0;
    int nin = 0, nout = 0;
    std::string err = dataset_read(data_path, X, Y, n, nin, nout);
    if (!err.empty()) fail(PMX_EINVAL, err);
    if (nin != PMX_NFEAT || nout != PMX_NOUT) fail(PMX_EINVAL, "training file does not match the features");
    TrainOpts to;
    to.epochs = mo.epochs;
    to.batch = mo.batch;
    to.hidden = mo.hidden;
    to.layers = mo.layers;
    to.lr = mo.lr;
    to.wmse = mo.wmse;
    to.seed = mo.seed;
    MlpModel m;
    std::vector<double> hist;
    try {
      hist = mlp_train(X, Y, n, nin, nout, to, m, (hipStream_t)stream);
    } catch (const std::exception& e) {
      fail(PMX_EHIP, e.what());
    }
    err = mlp_save(model_path, m);
    if (!err.empty()) fail(PMX_EINVAL, err);
    if (final_loss) *final_loss = hist.empty() ? 0.0 : hist.back();
  });
}

pmx_status pmx_mlp_predict(const char* model_path, const pmx_geometry* geom, const pmx_options* opts, float* out,
                           void* stream) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    validate(geom, &o);
    if (!out) fail(PMX_EINVAL, "out is NULL");
    if (plan_pass_through(plan_options(geom, o))) fail(PMX_EINVAL, "leaf predictions need one inclusion per leaf");
    pmx_factor F;
    F.opts = o;
    make_plan(geom, o, F.plan);
    leaf_predictions(&F, geom, model_path, (hipStream_t)stream);
    int64_t first = 0;
    for (const CellPlan& c : F.plan[0]) {
      const int j = c.incl[0];
      const int64_t n = geom->node_off[j + 1] - geom->node_off[j];
      std::memcpy(out + (size_t)PMX_NOUT * geom->node_off[j], F.leaf_pred.data() + (size_t)PMX_NOUT * first,
                  (size_t)PMX_NOUT * n * sizeof(float));
      first += n;
    }
  });
}

pmx_status pmx_probe_mlp(int32_t nin, int32_t nhidden, int32_t nlayer, int32_t nout, const float* params,
                         const float* X, const float* labels, int32_t B, float wmse, float* out, float* grad,
                         double* loss, void* stream) {
  return guarded([&] {
    if (nin <= 0 || nhidden <= 0 || nlayer < 0 || nout < 2 || (nout & 1) || B <= 0 || !params || !X || !labels ||
        !out || !grad || !loss)
      fail(PMX_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    MlpShape sh;
    sh.nin = nin;
    sh.nhidden = nhidden;
    sh.nlayer = nlayer;
    sh.nout = nout;
    const std::vector<int64_t> off = mlp_param_offsets(sh);
    Arena tmp;
    float* P = tmp.alloc<float>(off.back());
    float* G = tmp.alloc<float>(off.back());
    float* Xd = tmp.alloc<float>((int64_t)nin * B);
    float* Yd = tmp.alloc<float>((int64_t)nout * B);
    float* lp = tmp.alloc<float>(B);
    HIPCHK(hipMemcpyAsync(P, params, off.back() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(Xd, X, (size_t)nin * B * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(Yd, labels, (size_t)nout * B * 4, hipMemcpyHostToDevice, s));
    MlpBatch wk;
    const int nl = sh.nlin();
    wk.cap = B;
    wk.Z.assign(nl + 1, nullptr);
    wk.H.assign(nl + 1, nullptr);
    wk.dZ.assign(nl + 1, nullptr);
    wk.dH.assign(nl + 1, nullptr);
    for (int l = 1; l <= nl; ++l) {
      wk.Z[l] = tmp.alloc<float>((int64_t)sh.dims(l) * B);
      wk.dZ[l] = tmp.alloc<float>((int64_t)sh.dims(l) * B);
      if (l < nl) {
        wk.H[l] = tmp.alloc<float>((int64_t)sh.dims(l) * B);
        wk.dH[l] = tmp.alloc<float>((int64_t)sh.dims(l) * B);
      }
    }
    mlp_forward(sh, P, off, Xd, B, wk, s);
    mlp_loss_grad(wk.Z[nl], Yd, nout, nout / 2, wmse, B, wk.dZ[nl], lp, s);
    mlp_backward(sh, P, off, B, wk, G, s);
    std::vector<float> lh;
    download(lh, lp, B, s);
    double L = 0;
    for (float v : lh) L += v;
    *loss = L / B;
    HIPCHK(hipMemcpyAsync(out, wk.Z[nl], (size_t)nout * B * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(grad, G, off.back() * 4, hipMemcpyDeviceToHost, s));
    sync_check(s);
  });
}

pmx_status pmx_probe_apply_structure(const pmx_geometry* geom, const pmx_options* opts, int32_t check,
                                     double* stats) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    validate(geom, &o);
    if (!stats) fail(PMX_EINVAL, "NULL stats");
    std::unique_ptr<pmx_factor> F(new pmx_factor());
    F->opts = o;
    F->m = geom->m;
    F->node_off.assign(geom->node_off, geom->node_off + geom->m + 1);
    F->n_nodes = (int)F->node_off.back();
    F->k_ext = geom->k_ext;
    make_plan(geom, o, F->plan);
    const std::vector<double> hx(geom->x, geom->x + F->n_nodes), hy(geom->y, geom->y + F->n_nodes);
    ApplyGeo G;
    apply_geometry(F.get(), hx, hy, G, true);
    const int m = F->m, nsrc = m + G.n_clus, nw = (int)G.wave_node.size() / 2;
    for (int i = 0; i < 16; ++i) stats[i] = 0;
    for (int i = 0; i < 8; ++i) stats[i] = G.stats[i];
    const int nloc = (int)G.loc_p.size();
    int mxl = 0, mxf = 0, mxn = 0, mxp = 0;
    for (int t = 0; t < nloc; ++t) {
      mxl = std::max(mxl, G.m2l_off[t + 1] - G.m2l_off[t]);
      mxp = std::max(mxp, G.loc_p[t]);
    }
    for (int w = 0; w < nw; ++w) {
      mxf = std::max(mxf, G.foff[w + 1] - G.foff[w]);
      mxn = std::max(mxn, G.off[w + 1] - G.off[w]);
    }
    stats[8] = mxl;
    stats[9] = nloc ? (double)G.m2l_src.size() / nloc : 0.0;
    stats[10] = mxf;
    stats[11] = mxn;
    stats[12] = -1;
    stats[13] = nw;
    stats[14] = mxp;
    if (check) {
      // every (wave, source inclusion) pair of different inclusions must be taken exactly
      // once: near, through a far source of the wave that holds it, or through a
      // translation into the wave's inclusion or one of its ancestors from a source that
      // holds it
      std::vector<int> parent(nsrc, -1);
      for (int c = 0; c < G.n_clus; ++c)
        for (int q = G.kid_off[c]; q < G.kid_off[c + 1]; ++q) parent[G.kid_idx[q]] = m + c;
      std::vector<std::vector<char>> holds(nsrc, std::vector<char>(m, 0));
      for (int j = 0; j < m; ++j)
        for (int v = j; v >= 0; v = parent[v]) holds[v][j] = 1;
      std::vector<int> node_of(nloc, -1);
      for (int v = 0; v < nsrc; ++v)
        if (G.loc_id[v] >= 0) node_of[G.loc_id[v]] = v;
      int64_t bad = 0, pairs = 0;
      std::vector<int> cnt(m);
      for (int w = 0; w < nw; ++w) {
        std::fill(cnt.begin(), cnt.end(), 0);
        int own = 0;
        while (own + 1 <= m && F->node_off[own + 1] <= G.wave_node[2 * w]) ++own;
        for (int q = G.off[w]; q < G.off[w + 1]; ++q) cnt[G.idx[q]] += 1;
        for (int q = G.foff[w]; q < G.foff[w + 1]; ++q)
          for (int j = 0; j < m; ++j) cnt[j] += holds[G.fidx[q]][j];
        for (int v = own; v >= 0; v = parent[v]) {
          const int t = G.loc_id[v];
          if (t < 0) continue;
          for (int q = G.m2l_off[t]; q < G.m2l_off[t + 1]; ++q)
            for (int j = 0; j < m; ++j) cnt[j] += holds[G.m2l_src[q]][j];
        }
        for (int j = 0; j < m; ++j) {
          bad += (j == own) ? (cnt[j] != 0) : (cnt[j] != 1);
          ++pairs;
        }
      }
      stats[12] = (double)bad;
      stats[15] = (double)pairs;
    }
  });
}

pmx_status pmx_plan_query(const pmx_geometry* geom, const pmx_options* opts, int32_t cap_cells, int32_t cap_near,
                          int32_t* n_levels, int32_t* n_cells_total, int32_t* n_near_total, int32_t* cell_level,
                          int32_t* cell_first_incl, double* cell_center, double* cell_rc, double* cell_rp,
                          int32_t* cell_p, int32_t* near_off, int32_t* near) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    validate(geom, &o);
    if (!n_levels || !n_cells_total || !n_near_total) fail(PMX_EINVAL, "NULL size outputs");
    std::vector<std::vector<CellPlan>> levels;
    make_plan(geom, o, levels);
    int tc = 0, tn = 0;
    for (auto& L : levels)
      for (auto& c : L) {
        if (tc < cap_cells) {
          if (cell_level) cell_level[tc] = (int)(&L - &levels[0]);
          if (cell_first_incl) cell_first_incl[tc] = c.incl[0];
          if (cell_center) {
            cell_center[2 * tc] = c.cx;
            cell_center[2 * tc + 1] = c.cy;
          }
          if (cell_rc) cell_rc[tc] = c.rc;
          if (cell_rp) cell_rp[tc] = c.Rp;
          if (cell_p) cell_p[tc] = c.P;
          if (near_off) near_off[tc] = tn;
        }
        for (int v : c.near) {
          if (near && tn < cap_near) near[tn] = v;
          ++tn;
        }
        ++tc;
      }
    if (near_off && tc <= cap_cells) near_off[tc] = tn;
    *n_levels = (int)levels.size();
    *n_cells_total = tc;
    *n_near_total = tn;
  });
}

pmx_status pmx_plan_members(const pmx_geometry* geom, const pmx_options* opts, int32_t cap_cells, int32_t cap_incl,
                            int32_t cap_child, int32_t* n_cells_total, int32_t* n_incl_total, int32_t* n_child_total,
                            int32_t* incl_off, int32_t* incl, int32_t* child_off, int32_t* child) {
  return guarded([&] {
    pmx_options o;
    pmx_options_default(&o);
    if (opts) o = *opts;
    validate(geom, &o);
    if (!n_cells_total || !n_incl_total || !n_child_total) fail(PMX_EINVAL, "NULL size outputs");
    std::vector<std::vector<CellPlan>> levels;
    make_plan(geom, o, levels);
    int tc = 0, ti = 0, tk = 0;
    for (auto& L : levels)
      for (auto& c : L) {
        if (tc < cap_cells) {
          if (incl_off) incl_off[tc] = ti;
          if (child_off) child_off[tc] = tk;
        }
        for (int v : c.incl) {
          if (incl && ti < cap_incl) incl[ti] = v;
          ++ti;
        }
        for (int v : c.children) {
          if (child && tk < cap_child) child[tk] = v;
          ++tk;
        }
        ++tc;
      }
    if (tc <= cap_cells) {
      if (incl_off) incl_off[tc] = ti;
      if (child_off) child_off[tc] = tk;
    }
    *n_cells_total = tc;
    *n_incl_total = ti;
    *n_child_total = tk;
  });
}

}  // extern "C"
