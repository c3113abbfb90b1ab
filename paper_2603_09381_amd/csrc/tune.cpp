// Launch-parameter table: buckets, lookups, the text file, and the timing of the linear
// algebra candidates (LU panels, column-pivoted QR, level solves) for the autotuner.
#include "tune.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "la.h"

thread_local const TuneTable* g_tune = nullptr;
thread_local TuneRecorder* g_tune_rec = nullptr;
thread_local TuneForce g_tune_force;

namespace {
const char* const kKnobNames[TK_COUNT] = {"lu_panel", "cpqr", "getrs", "apply_nr", "apply_wg", "ts_leaf"};
const int64_t kSizeBounds[] = {64, 128, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144, 8192, 12288, 16384};
}  // namespace

const char* tune_knob_name(int knob) { return (knob >= 0 && knob < TK_COUNT) ? kKnobNames[knob] : "?"; }

int tune_knob_from_name(const std::string& name) {
  for (int k = 0; k < TK_COUNT; ++k)
    if (name == kKnobNames[k]) return k;
  return -1;
}

int tune_bucket_size(int64_t n) {
  const int nb = (int)(sizeof(kSizeBounds) / sizeof(kSizeBounds[0]));
  for (int i = 0; i < nb; ++i)
    if (n <= kSizeBounds[i]) return i;
  return nb;
}

int tune_bucket_batch(int64_t b) {
  int i = 0;
  for (int64_t v = 1; v < b; v *= 4) ++i;
  return i;
}

int tune_bucket_pow2(int64_t n) {
  int i = 0;
  for (int64_t v = 1; v < n; v *= 2) ++i;
  return i;
}

uint64_t tune_key(int knob, int rb, int a, int b, int c) {
  return ((uint64_t)(knob & 0xff) << 56) | ((uint64_t)(rb & 0xff) << 48) | ((uint64_t)(a & 0xffff) << 32) |
         ((uint64_t)(b & 0xffff) << 16) | (uint64_t)(c & 0xffff);
}

void tune_unkey(uint64_t key, int& knob, int& rb, int& a, int& b, int& c) {
  knob = (int)((key >> 56) & 0xff);
  rb = (int)((key >> 48) & 0xff);
  a = (int)((key >> 32) & 0xffff);
  b = (int)((key >> 16) & 0xffff);
  c = (int)(key & 0xffff);
}

int tune_choice(int knob, int rb, int a, int b, int c, int dflt, int64_t d0, int64_t d1, int64_t d2) {
  const uint64_t key = tune_key(knob, rb, a, b, c);
  if (g_tune_rec) {
    auto it = g_tune_rec->dims.find(key);
    if (it == g_tune_rec->dims.end()) {
      g_tune_rec->dims[key] = {d0, d1, d2};
    } else {
      it->second[0] = std::max(it->second[0], d0);
      it->second[1] = std::max(it->second[1], d1);
      it->second[2] = std::max(it->second[2], d2);
    }
  }
  if (g_tune_force.knob == knob) return g_tune_force.value;
  if (g_tune) {
    auto it = g_tune->val.find(key);
    if (it != g_tune->val.end()) return it->second;
  }
  return dflt;
}

std::string tune_save(const std::string& path, const TuneTable& t) {
  std::ofstream f(path);
  if (!f) return "cannot open " + path + " for writing";
  f << "# pmx launch-parameter table: knob real_bytes bucket_a bucket_b bucket_c choice  # candidate:us\n";
  for (const auto& kv : t.val) {
    int knob, rb, a, b, c;
    tune_unkey(kv.first, knob, rb, a, b, c);
    f << tune_knob_name(knob) << ' ' << rb << ' ' << a << ' ' << b << ' ' << c << ' ' << kv.second;
    auto n = t.note.find(kv.first);
    if (n != t.note.end() && !n->second.empty()) f << "  # " << n->second;
    f << '\n';
  }
  if (!f) return "write to " + path + " failed";
  return "";
}

std::string tune_load(const std::string& path, TuneTable& t) {
  std::ifstream f(path);
  if (!f) return "cannot open launch-parameter table " + path;
  std::string line;
  int ln = 0;
  while (std::getline(f, line)) {
    ++ln;
    const size_t h = line.find('#');
    if (h != std::string::npos) line.resize(h);
    std::istringstream is(line);
    std::string name;
    if (!(is >> name)) continue;
    int rb, a, b, c, v;
    if (!(is >> rb >> a >> b >> c >> v)) return path + ":" + std::to_string(ln) + ": malformed line";
    const int knob = tune_knob_from_name(name);
    if (knob < 0) return path + ":" + std::to_string(ln) + ": unknown knob " + name;
    if ((rb != 4 && rb != 8) || a < 0 || b < 0 || c < 0 || a > 0xffff || b > 0xffff || c > 0xffff)
      return path + ":" + std::to_string(ln) + ": key out of range";
    t.val[tune_key(knob, rb, a, b, c)] = v;
  }
  return "";
}

void tune_candidates(int knob, int rb, int64_t d0, int64_t d1, int64_t d2, int* out, int* n) {
  *n = 0;
  (void)d1;
  switch (knob) {
    case TK_LU_PANEL:   // d0: panel rows
      if (d0 <= 256) out[(*n)++] = 0;
      if (d0 <= 512) out[(*n)++] = 1;
      if (rb == 4 && d0 <= 1024) out[(*n)++] = 2;
      out[(*n)++] = 3;
      if (d0 <= 256) out[(*n)++] = 4;
      if (d0 <= 512) out[(*n)++] = 6;
      if (rb == 4 && d0 <= 1024) out[(*n)++] = 8;
      out[(*n)++] = 10;
      break;
    case TK_CPQR:
      out[(*n)++] = 0;
      out[(*n)++] = 1;
      out[(*n)++] = 2;
      break;
    case TK_GETRS:      // d0: size, d2: right-hand sides
      if (d2 <= PMX_GETRS_SMALL_MAX) out[(*n)++] = 0;
      out[(*n)++] = 1;
      if (la_getrs_lds_bytes((int)d0, rb) <= 128 * 1024) out[(*n)++] = 2;
      break;
    case TK_APPLY_NR:   // d1: right-hand sides
      for (int v : {1, 2, 4, 8})
        if (v == 1 || v / 2 < d1) out[(*n)++] = v;
      break;
    case TK_APPLY_WG:
      for (int v : {512, 1024, 2048, 4096, 8192}) out[(*n)++] = v;
      break;
    case TK_TS_LEAF:
      for (int v : {256, 512, 1024})
        if (v < 1024 || rb == 4) out[(*n)++] = v;
      break;
    default:
      break;
  }
}

// ---------------------------------------------------------------------------------
// Timing of the linear algebra candidates

namespace {

// SplitMix64 finaliser of a counter: the fill of the tuning buffers
__device__ inline double tune_unit(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// count matrices of rows x cols (leading dimension rows, back to back): entries uniform in
// [-1, 1] + i [-1, 1], column j scaled by 10^(-decay j / cols), diag added on the diagonal
template <class R>
__global__ void k_tune_fill(cx<R>* p, int64_t rows, int64_t cols, int64_t count, uint64_t seed, double decay,
                            double diag) {
  const int64_t total = rows * cols * count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % (rows * cols);
    const int64_t r = e % rows, c = e / rows;
    const double sc = decay > 0 ? pow(10.0, -decay * (double)c / (double)cols) : 1.0;
    double re = tune_unit(seed ^ (2 * (uint64_t)i)) * sc, im = tune_unit(seed ^ (2 * (uint64_t)i + 1)) * sc;
    if (r == c) re += diag;
    p[i] = cmk<R>((R)re, (R)im);
  }
}

template <class R>
void fill(cx<R>* p, int64_t rows, int64_t cols, int64_t count, uint64_t seed, double decay, double diag,
          hipStream_t s) {
  const int64_t total = rows * cols * count;
  if (total <= 0) return;
  const int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
  PMX_LAUNCH(k_tune_fill<R>, dim3(blocks), dim3(256), 0, s, p, rows, cols, count, seed, decay, diag);
}

// device buffers of one timing case, released at the end of the case
struct Bufs {
  std::vector<void*> ptr;
  std::string err;
  template <class T>
  T* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      err = "device allocation of " + std::to_string(n * sizeof(T)) + " bytes for tuning failed";
      return nullptr;
    }
    ptr.push_back(p);
    return (T*)p;
  }
  template <class T>
  T* put(const std::vector<T>& v, hipStream_t s) {
    T* p = get<T>(v.size());
    if (p && !v.empty()) (void)hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return p;
  }
  ~Bufs() {
    for (void* p : ptr) (void)hipFree(p);
  }
};

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  template <class Prep, class Run>
  double best_us(int reps, hipStream_t s, Prep&& prep, Run&& run) {
    double best = 1e300;
    for (int r = 0; r <= reps; ++r) {   // the first run warms up and is not counted
      prep();
      (void)hipEventRecord(a, s);
      run();
      (void)hipEventRecord(b, s);
      (void)hipEventSynchronize(b);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, a, b);
      if (r > 0) best = std::min(best, 1e3 * (double)ms);
    }
    return best;
  }
};

template <class R>
std::string time_lu_panel(int64_t rows, int64_t batch, const int* cand, int nc, double* us, int reps, hipStream_t s) {
  Bufs B;
  const int64_t nr = std::max<int64_t>(rows, 1);
  cx<R>* a = B.get<cx<R>>(nr * PMX_LU_NB * batch);
  int* ipiv = B.get<int>(nr * batch);
  int* info = B.get<int>(batch);
  if (!B.err.empty()) return B.err;
  std::vector<LuDescT<R>> d(batch);
  for (int64_t b = 0; b < batch; ++b) d[b] = LuDescT<R>{a + b * nr * PMX_LU_NB, nr, (int)nr, ipiv + b * nr, nullptr};
  LuDescT<R>* dd = B.put(d, s);
  if (!B.err.empty()) return B.err;
  Timer T;
  for (int i = 0; i < nc; ++i)
    us[i] = T.best_us(
        reps, s,
        [&] {
          fill<R>(a, nr, PMX_LU_NB, batch, 0x5eed0001ull, 0.0, 0.0, s);
          (void)hipMemsetAsync(info, 0, batch * sizeof(int), s);
        },
        [&] { la_lu_panel<R>(cand[i], dd, (int)batch, 0, info, s); });
  return hipGetLastError() == hipSuccess ? "" : "a tuning launch failed";
}

template <class R>
std::string time_cpqr(int64_t c, int64_t batch, const int* cand, int nc, double* us, int reps, hipStream_t s) {
  Bufs B;
  cx<R>* m = B.get<cx<R>>(c * c * batch);
  int* piv = B.get<int>(c * batch);
  double* nrm = B.get<double>(2 * c * batch);
  int* st = B.get<int>(4 * batch);
  double* r11 = B.get<double>(batch);
  cx<R>* v = B.get<cx<R>>(c * batch);
  double* tau = B.get<double>(batch);
  int* work = B.get<int>(1);
  if (!B.err.empty()) return B.err;
  std::vector<CpqrDescT<R>> d(batch);
  for (int64_t b = 0; b < batch; ++b)
    d[b] = CpqrDescT<R>{m + b * c * c, (int)c, (int)c, piv + b * c, nrm + 2 * b * c, st + 4 * b, r11 + b,
                        v + b * c, tau + b, (int)c, nullptr};
  CpqrDescT<R>* dd = B.put(d, s);
  if (!B.err.empty()) return B.err;
  Timer T;
  const TuneForce saved = g_tune_force;
  hipError_t poll = hipSuccess;   // the first error of the CPQR progress polls
  for (int i = 0; i < nc; ++i) {
    g_tune_force = TuneForce{TK_CPQR, cand[i]};
    // singular values decaying over 12 decades: the threshold rank at 1e-10 is ~5/6 c
    us[i] = T.best_us(
        reps, s, [&] { fill<R>(m, c, c, batch, 0x5eed0002ull, 12.0, 0.0, s); },
        [&] {
          const hipError_t e = la_cpqr<R>(dd, (int)batch, (int)c, 1e-10, nullptr, 1, work, s);
          if (poll == hipSuccess) poll = e;
        });
  }
  g_tune_force = saved;
  if (poll != hipSuccess) return std::string("a CPQR progress poll failed: ") + hipGetErrorString(poll);
  return hipGetLastError() == hipSuccess ? "" : "a tuning launch failed";
}

template <class R>
std::string time_getrs(int64_t n, int64_t batch, int64_t nrhs, const int* cand, int nc, double* us, int reps,
                       hipStream_t s) {
  Bufs B;
  cx<R>* a = B.get<cx<R>>(n * n * batch);
  int* ipiv = B.get<int>(n * batch);
  int* perm = B.get<int>(n * batch);
  int* info = B.get<int>(batch);
  cx<R>* rhs = B.get<cx<R>>(n * nrhs * batch);
  cx<R>* w = B.get<cx<R>>(n * nrhs * batch);
  if (!B.err.empty()) return B.err;
  std::vector<LuDescT<R>> d(batch);
  std::vector<MatT<R>> bm(batch), wm(batch);
  for (int64_t b = 0; b < batch; ++b) {
    d[b] = LuDescT<R>{a + b * n * n, n, (int)n, ipiv + b * n, perm + b * n};
    bm[b] = MatT<R>{rhs + b * n * nrhs, n, (int)n, (int)nrhs};
    wm[b] = MatT<R>{w + b * n * nrhs, n, (int)n, (int)nrhs};
  }
  LuDescT<R>* dd = B.put(d, s);
  MatT<R>* db = B.put(bm, s);
  MatT<R>* dw = B.put(wm, s);
  if (!B.err.empty()) return B.err;
  fill<R>(a, n, n, batch, 0x5eed0003ull, 0.0, 2.0 * std::sqrt((double)n), s);
  (void)hipMemsetAsync(info, 0, batch * sizeof(int), s);
  la_getrf<R>(dd, (int)batch, (int)n, info, s);
  Timer T;
  for (int i = 0; i < nc; ++i)
    us[i] = T.best_us(
        reps, s, [&] { fill<R>(rhs, n, nrhs, batch, 0x5eed0004ull, 0.0, 0.0, s); },
        [&] {
          if (cand[i] == 2 && la_getrs_lds<R>(dd, db, (int)batch, (int)n, (int)nrhs, s)) return;
          if (cand[i] == 0)
            la_getrs_small<R>(dd, db, dw, (int)batch, (int)n, (int)nrhs, s);
          else
            la_getrs<R>(dd, db, (int)batch, (int)n, (int)nrhs, s);
        });
  return hipGetLastError() == hipSuccess ? "" : "a tuning launch failed";
}

template <class R>
std::string time_qr(int64_t m, int64_t batch, int64_t c, const int* cand, int nc, double* us, int reps, hipStream_t s) {
  Bufs B;
  const int64_t kc = std::min(m, c), ws = la_geqrf_workspace((int)m);
  cx<R>* a = B.get<cx<R>>(m * c * batch);
  cx<R>* r = B.get<cx<R>>(kc * c * batch);
  cx<R>* v = B.get<cx<R>>(ws * batch);
  cx<R>* t = B.get<cx<R>>(ws * batch);
  if (!B.err.empty()) return B.err;
  std::vector<QrDescT<R>> d(batch);
  for (int64_t b = 0; b < batch; ++b)
    d[b] = QrDescT<R>{a + b * m * c, m, (int)m, (int)c, r + b * kc * c, v + b * ws, t + b * ws, (int)kc};
  QrDescT<R>* dd = B.put(d, s);
  if (!B.err.empty()) return B.err;
  Timer T;
  const TuneForce saved = g_tune_force;
  for (int i = 0; i < nc; ++i) {
    g_tune_force = TuneForce{TK_TS_LEAF, cand[i]};
    us[i] = T.best_us(
        reps, s, [&] { fill<R>(a, m, c, batch, 0x5eed0005ull, 0.0, 0.0, s); },
        [&] { la_geqrf_r<R>(dd, (int)batch, (int)m, (int)c, s); });
  }
  g_tune_force = saved;
  return hipGetLastError() == hipSuccess ? "" : "a tuning launch failed";
}

std::string note_of(const int* cand, const double* us, int nc) {
  std::ostringstream o;
  for (int i = 0; i < nc; ++i) o << (i ? " " : "") << cand[i] << ':' << (int64_t)std::llround(us[i]);
  return o.str();
}

}  // namespace

std::string tune_linear_algebra(const TuneRecorder& rec, TuneTable& t, int reps, hipStream_t s) {
  for (const auto& kv : rec.dims) {
    int knob, rb, a, b, c;
    tune_unkey(kv.first, knob, rb, a, b, c);
    if (knob != TK_LU_PANEL && knob != TK_CPQR && knob != TK_GETRS && knob != TK_TS_LEAF) continue;
    const int64_t d0 = kv.second[0], d1 = kv.second[1], d2 = kv.second[2];
    if (d0 <= 0 || d1 <= 0) continue;
    int cand[16], nc = 0;
    tune_candidates(knob, rb, d0, d1, d2, cand, &nc);
    if (nc < 2) continue;
    double us[16];
    std::string e;
    if (knob == TK_LU_PANEL)
      e = rb == 8 ? time_lu_panel<double>(d0, d1, cand, nc, us, reps, s) : time_lu_panel<float>(d0, d1, cand, nc, us, reps, s);
    else if (knob == TK_CPQR)
      e = rb == 8 ? time_cpqr<double>(d0, d1, cand, nc, us, reps, s) : time_cpqr<float>(d0, d1, cand, nc, us, reps, s);
    else if (knob == TK_TS_LEAF)
      e = rb == 8 ? time_qr<double>(d0, d1, d2, cand, nc, us, reps, s) : time_qr<float>(d0, d1, d2, cand, nc, us, reps, s);
    else
      e = rb == 8 ? time_getrs<double>(d0, d1, d2, cand, nc, us, reps, s)
                  : time_getrs<float>(d0, d1, d2, cand, nc, us, reps, s);
    if (!e.empty()) return e;
    int best = 0;
    for (int i = 1; i < nc; ++i)
      if (us[i] < us[best]) best = i;
    t.val[kv.first] = cand[best];
    t.note[kv.first] = note_of(cand, us, nc) + " shape " + std::to_string(d0) + "," + std::to_string(d1) + "," +
                       std::to_string(d2);
  }
  return "";
}
