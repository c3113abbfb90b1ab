// Launch-parameter table of the batched kernels and the lookups their launchers make.
//
// A table maps a key (knob, bytes of the real type, up to three size buckets) to a
// choice.  Launchers ask for the choice of the shape they are about to launch; without
// an active table, or for a key the table does not hold, the built-in rule applies.  The
// autotuner (pmx_autotune) fills a table in two passes: it first runs the workload with a
// recorder that collects every key the launchers ask for (and the largest shape seen per
// key), then times each candidate on device buffers of that shape with the choice forced,
// and keeps the fastest.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>

enum TuneKnob : int {
  TK_LU_PANEL = 0,  // LU panel kernel by panel rows, batch: 0 registers 256 x 1 row, 1 registers
                    // 256 x 2 rows, 2 registers 512 x 2 rows (FP32 only), 3 global memory;
                    // unrolled columns: 4 256 x 1, 6 512 x 1, 8 1024 x 1 (FP32 only);
                    // 10 tall panels, rows in memory (1024 threads FP32, 512 FP64)
  TK_CPQR = 1,      // column-pivoted QR by columns, batch: 0 one workgroup per matrix,
                    // 1 multi-workgroup steps, 2 the same steps in one cooperative launch
  TK_GETRS = 2,     // level LU solves by size, batch, right-hand sides: 0 one fused kernel per
                    // cell (<= 64 right-hand sides), 1 blocked (row swaps, triangular blocks, MFMA
                    // updates), 2 one fused kernel per cell and 4 right-hand sides with the
                    // solution in LDS (size x 4 x complex <= 128 KiB)
  TK_APPLY_NR = 3,  // dense operator apply by nodes, right-hand sides: right-hand sides per
                    // thread group (1, 2, 4 or 8)
  TK_APPLY_WG = 4,  // dense operator apply: workgroups a launch aims at (source splits)
  TK_TS_LEAF = 5,   // Householder QR by rows, batch, columns: threads per leaf block (256, 512,
                    // 1024 in FP32)
  TK_COUNT = 6
};

const char* tune_knob_name(int knob);
int tune_knob_from_name(const std::string& name);

// buckets: sizes {64,128,256,384,512,768,1024,1536,2048,3072,4096,6144,...} (index of the
// smallest bound >= n), batches ceil(log4 b), powers ceil(log2 n)
int tune_bucket_size(int64_t n);
int tune_bucket_batch(int64_t b);
int tune_bucket_pow2(int64_t n);

uint64_t tune_key(int knob, int rb, int a, int b, int c);
void tune_unkey(uint64_t key, int& knob, int& rb, int& a, int& b, int& c);

struct TuneTable {
  std::map<uint64_t, int> val;
  std::map<uint64_t, std::string> note;  // per key: the measured candidates, for the file
};

struct TuneRecorder {
  std::map<uint64_t, std::array<int64_t, 3>> dims;  // per key: largest shape asked for
};

struct TuneForce {
  int knob = -1;
  int value = 0;
};

extern thread_local const TuneTable* g_tune;      // table of the calling thread's factor
extern thread_local TuneRecorder* g_tune_rec;     // first autotuner pass
extern thread_local TuneForce g_tune_force;       // timing runs of the autotuner

// The choice for a key: the forced value of its knob, else the table's, else dflt.  With
// a recorder active the key and the shape (d0, d1, d2) are recorded.
int tune_choice(int knob, int rb, int a, int b, int c, int dflt, int64_t d0, int64_t d1, int64_t d2);

// text table: one line per key, "knob rb a b c value  # candidate:microseconds ..."
std::string tune_save(const std::string& path, const TuneTable& t);
std::string tune_load(const std::string& path, TuneTable& t);

// Candidate choices of a knob for a recorded shape (d0, d1, d2) and real type size rb.
void tune_candidates(int knob, int rb, int64_t d0, int64_t d1, int64_t d2, int* out, int* n);

// Times the candidates of every recorded LU-panel, CPQR, level-solve and QR key on device
// buffers of the recorded shape (a fixed seeded fill), best of `reps` runs each, and
// stores the fastest in t.  Returns an error text, empty on success.
std::string tune_linear_algebra(const TuneRecorder& rec, TuneTable& t, int reps, hipStream_t s);
