// Optional per-kernel timing with HIP events on the launch stream.  When a KernelTimer is
// active for the calling thread, every instrumented launch of a kernel in its mask is
// bracketed by two events; after the stream has been synchronised, collect() sums the
// elapsed times per kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

enum PmxKernelId {
  PK_TS_LEAF = 0,      // k_ts_leaf: in-LDS Householder QR of row blocks
  PK_TS_UPDATE = 1,    // k_ts_update: block reflectors applied to the trailing columns
  PK_GETRF_PANEL = 2,  // k_getrf_panel: LU panel with partial pivoting
  PK_CPQR_UPDATE = 3,  // k_cpqr_update: column-pivoted QR trailing update (multi-workgroup)
  PK_CPQR = 4,         // k_cpqr: column-pivoted QR, one workgroup per matrix
  PK_ZGEMM = 5,        // k_zgemm: every MFMA complex product
  PK_TRSM = 6,         // k_trsm_small: triangular solves on diagonal blocks
  PK_ENTRIES = 7,      // k_entries: interaction and proxy matrices
  PK_DIAG = 8,         // k_diag_*: self blocks (Kress quadrature, Maue products)
  PK_APPLY = 9,        // k_apply_off: dense FP64 operator apply for refinement residuals
  PK_GETRS = 10,       // k_getrs_small: fused permutation and substitutions, few right-hand sides
  PK_COUNT = 11
};

// kernels launched by solve sequences (captured as graphs unless one of them is timed)
constexpr unsigned PK_SOLVE_MASK = (1u << PK_ZGEMM) | (1u << PK_TRSM) | (1u << PK_APPLY) | (1u << PK_GETRS);

struct KernelTimer {
  unsigned mask = ~0u;   // bit k: time the launches of kernel k
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void collect(double* ms, int* n) {
    for (const Rec& r : recs) {
      float t = 0;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.kid] += t;
        n[r.kid] += 1;
      }
    }
    recs.clear();
    used = 0;
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

extern thread_local KernelTimer* g_ktimer;

struct KScope {
  hipEvent_t e0 = nullptr;
  int kid;
  hipStream_t s;
  KScope(int k, hipStream_t st) : kid(k), s(st) {
    if (g_ktimer && ((g_ktimer->mask >> k) & 1u)) {
      e0 = g_ktimer->get();
      if (e0) (void)hipEventRecord(e0, s);
    }
  }
  ~KScope() {
    if (e0) {
      hipEvent_t e1 = g_ktimer->get();
      if (e1) {
        (void)hipEventRecord(e1, s);
        g_ktimer->recs.push_back({kid, e0, e1});
      }
    }
  }
};
