// Learned skeleton proposals: leaf-cell features, training and inference of the scoring
// network (FP32 on the device), model and training-set files.
#include "learn.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <thread>

namespace {

// device buffer released at scope exit
template <class T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) {
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct BatchBufs {
  std::vector<DevBuf<float>*> own;
  MlpBatch b;
  BatchBufs(const MlpShape& sh, int cap) {
    const int nl = sh.nlin();
    b.cap = cap;
    b.Z.assign(nl + 1, nullptr);
    b.H.assign(nl + 1, nullptr);
    b.dZ.assign(nl + 1, nullptr);
    b.dH.assign(nl + 1, nullptr);
    for (int l = 1; l <= nl; ++l) {
      const size_t sz = (size_t)sh.dims(l) * cap;
      b.Z[l] = get(sz);
      b.dZ[l] = get(sz);
      if (l < nl) {
        b.H[l] = get(sz);
        b.dH[l] = get(sz);
      }
    }
  }
  float* get(size_t n) {
    own.push_back(new DevBuf<float>(n));
    if (!own.back()->p) throw std::runtime_error("device allocation failed");
    return own.back()->p;
  }
  ~BatchBufs() {
    for (auto* d : own) delete d;
  }
};

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    const double u = uniform(), v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(2.0 * M_PI * v);
  }
};

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

void leaf_features(const HostGeom& g, const std::vector<CellPlan>& leaves, std::vector<float>& X) {
  const int nc = (int)leaves.size();
  std::vector<int64_t> first(nc + 1, 0);
  for (int t = 0; t < nc; ++t) {
    const int j = leaves[t].incl[0];
    first[t + 1] = first[t] + (g.node_off[j + 1] - g.node_off[j]);
  }
  X.assign((size_t)PMX_NFEAT * first[nc], 0.0f);
  auto work = [&](int t0, int t1) {
    for (int t = t0; t < t1; ++t) {
      const CellPlan& c = leaves[t];
      const int j = c.incl[0];
      const int64_t o = g.node_off[j];
      const int n = (int)(g.node_off[j + 1] - o);
      const double rc = c.rc > 0 ? c.rc : 1.0;
      std::vector<double> rho(n), phi(n);
      double mrho = 0;
      for (int i = 0; i < n; ++i) {
        rho[i] = std::hypot(g.x[o + i] - c.cx, g.y[o + i] - c.cy);
        phi[i] = std::atan2(g.y[o + i] - c.cy, g.x[o + i] - c.cx);
        mrho += rho[i];
      }
      mrho /= n;
      double modes[5];
      for (int mm = 2; mm <= 6; ++mm) {
        std::complex<double> acc = 0;
        for (int i = 0; i < n; ++i) acc += rho[i] * std::polar(1.0, -mm * phi[i]);
        modes[mm - 2] = std::abs(acc) / (n * mrho);
      }
      // nodes of the near cells
      std::vector<double> nx_, ny_;
      for (int s : c.near) {
        const int js = leaves[s].incl[0];
        for (int64_t i = g.node_off[js]; i < g.node_off[js + 1]; ++i) {
          nx_.push_back(g.x[i]);
          ny_.push_back(g.y[i]);
        }
      }
      for (int i = 0; i < n; ++i) {
        const int64_t a = o + i;
        const double sp = std::hypot(g.dx[a], g.dy[a]);
        const double kap = (g.dx[a] * g.ddy[a] - g.dy[a] * g.ddx[a]) / (sp * sp * sp);
        double d2 = 1e300;
        for (size_t q = 0; q < nx_.size(); ++q) {
          const double ex = nx_[q] - g.x[a], ey = ny_[q] - g.y[a];
          d2 = std::min(d2, ex * ex + ey * ey);
        }
        float* f = X.data() + (size_t)PMX_NFEAT * (first[t] + i);
        f[0] = (float)(g.k_ext * rc);
        f[1] = (float)(g.k_ext * c.Rp);
        f[2] = (float)(g.k_int[j] / g.k_ext);
        f[3] = (float)(n / 256.0);
        f[4] = (float)(c.near.size() / 8.0);
        for (int mm = 0; mm < 5; ++mm) f[5 + mm] = (float)modes[mm];
        f[10] = (float)(mrho / rc);
        f[11] = (float)std::cos(phi[i]);
        f[12] = (float)std::sin(phi[i]);
        f[13] = (float)(g.dy[a] / sp);
        f[14] = (float)(-g.dx[a] / sp);
        f[15] = (float)(rho[i] / rc);
        f[16] = (float)std::max(-10.0, std::min(10.0, kap * rc));
        f[17] = (float)(sp / rc);
        f[18] = (float)std::min(10.0, std::sqrt(d2) / rc);
        f[19] = (float)(c.Rp > 0 ? std::max(-10.0, std::min(10.0, (c.Rp - rho[i]) / rc)) : 10.0);
      }
    }
  };
  const int nth = std::max(1, std::min(8, nc / 16));
  std::vector<std::thread> th;
  for (int k = 0; k < nth; ++k) th.emplace_back(work, nc * k / nth, nc * (k + 1) / nth);
  for (auto& x : th) x.join();
}

static const char kModelMagic[8] = {'P', 'M', 'X', 'M', 'L', 'P', '0', '1'};
static const char kDataMagic[8] = {'P', 'M', 'X', 'I', 'D', 'S', '0', '1'};

std::string mlp_save(const std::string& path, const MlpModel& m) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return "cannot write " + path;
  int32_t hdr[4] = {m.sh.nin, m.sh.nhidden, m.sh.nlayer, m.sh.nout};
  int64_t np = (int64_t)m.params.size();
  bool ok = std::fwrite(kModelMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
            std::fwrite(m.mean.data(), 4, m.sh.nin, f) == (size_t)m.sh.nin &&
            std::fwrite(m.istd.data(), 4, m.sh.nin, f) == (size_t)m.sh.nin && std::fwrite(&np, 8, 1, f) == 1 &&
            std::fwrite(m.params.data(), 4, np, f) == (size_t)np;
  std::fclose(f);
  return ok ? "" : "short write to " + path;
}

std::string mlp_load(const std::string& path, MlpModel& m) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return "cannot read " + path;
  char mg[8];
  int32_t hdr[4];
  int64_t np = 0;
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kModelMagic, 8) == 0 && std::fread(hdr, 4, 4, f) == 4;
  if (ok) {
    m.sh.nin = hdr[0];
    m.sh.nhidden = hdr[1];
    m.sh.nlayer = hdr[2];
    m.sh.nout = hdr[3];
    ok = m.sh.nin > 0 && m.sh.nin < 4096 && m.sh.nhidden > 0 && m.sh.nhidden <= 4096 && m.sh.nlayer >= 0 &&
         m.sh.nlayer < 64 && m.sh.nout > 0 && m.sh.nout < 4096;
  }
  if (ok) {
    m.mean.resize(m.sh.nin);
    m.istd.resize(m.sh.nin);
    ok = std::fread(m.mean.data(), 4, m.sh.nin, f) == (size_t)m.sh.nin &&
         std::fread(m.istd.data(), 4, m.sh.nin, f) == (size_t)m.sh.nin && std::fread(&np, 8, 1, f) == 1 &&
         np == mlp_param_offsets(m.sh).back();
  }
  if (ok) {
    m.params.resize(np);
    ok = std::fread(m.params.data(), 4, np, f) == (size_t)np;
  }
  std::fclose(f);
  return ok ? "" : "not a valid model file: " + path;
}

void mlp_predict(const MlpModel& m, const std::vector<float>& X, int64_t n, std::vector<float>& out, hipStream_t s) {
  const MlpShape& sh = m.sh;
  out.assign((size_t)sh.nout * n, 0.0f);
  if (n <= 0) return;
  const std::vector<int64_t> off = mlp_param_offsets(sh);
  DevBuf<float> P(off.back()), mean(sh.nin), istd(sh.nin);
  const int B = (int)std::min<int64_t>(n, 65536);
  DevBuf<float> Xd((size_t)sh.nin * B);
  if (!P.p || !mean.p || !istd.p || !Xd.p) throw std::runtime_error("device allocation failed");
  check(hipMemcpyAsync(P.p, m.params.data(), off.back() * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemcpyAsync(mean.p, m.mean.data(), sh.nin * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemcpyAsync(istd.p, m.istd.data(), sh.nin * 4, hipMemcpyHostToDevice, s), "upload");
  BatchBufs wk(sh, B);
  for (int64_t c0 = 0; c0 < n; c0 += B) {
    const int b = (int)std::min<int64_t>(B, n - c0);
    check(hipMemcpyAsync(Xd.p, X.data() + (size_t)sh.nin * c0, (size_t)sh.nin * b * 4, hipMemcpyHostToDevice, s),
          "upload");
    mlp_standardise(Xd.p, mean.p, istd.p, sh.nin, b, s);
    mlp_forward(sh, P.p, off, Xd.p, b, wk.b, s);
    check(hipMemcpyAsync(out.data() + (size_t)sh.nout * c0, wk.b.Z[sh.nlin()], (size_t)sh.nout * b * 4,
                         hipMemcpyDeviceToHost, s),
          "download");
    check(hipStreamSynchronize(s), "predict");
  }
}

std::vector<double> mlp_train(const std::vector<float>& X, const std::vector<float>& Y, int64_t n, int nin, int nout,
                              const TrainOpts& o, MlpModel& model, hipStream_t s) {
  if (n <= 0 || nin <= 0 || nout < 4 || nout % 2) throw std::runtime_error("empty or malformed training set");
  MlpShape& sh = model.sh;
  sh.nin = nin;
  sh.nhidden = o.hidden;
  sh.nlayer = o.layers;
  sh.nout = nout;
  // standardisation of the inputs
  model.mean.assign(nin, 0.0f);
  model.istd.assign(nin, 1.0f);
  for (int r = 0; r < nin; ++r) {
    double s1 = 0, s2 = 0;
    for (int64_t c = 0; c < n; ++c) {
      const double v = X[(size_t)nin * c + r];
      s1 += v;
      s2 += v * v;
    }
    const double mu = s1 / n, var = std::max(0.0, s2 / n - mu * mu);
    model.mean[r] = (float)mu;
    model.istd[r] = (float)(1.0 / std::max(1e-6, std::sqrt(var)));
  }
  // He initialisation from the seeded generator, zero biases
  const std::vector<int64_t> off = mlp_param_offsets(sh);
  model.params.assign(off.back(), 0.0f);
  SplitMix rng{o.seed};
  for (int l = 0; l < sh.nlin(); ++l) {
    const double sd = std::sqrt(2.0 / sh.dims(l));
    for (int64_t e = off[2 * l]; e < off[2 * l + 1]; ++e) model.params[e] = (float)(sd * rng.normal());
  }
  DevBuf<float> P(off.back()), G(off.back()), M1(off.back()), V1(off.back());
  DevBuf<float> Xall((size_t)nin * n), Yall((size_t)nout * n), mean(nin), istd(nin);
  const int B = (int)std::min<int64_t>(o.batch, n);
  DevBuf<float> Xb((size_t)nin * B), Yb((size_t)nout * B), lp(B);
  DevBuf<int64_t> idx(B);
  if (!P.p || !G.p || !M1.p || !V1.p || !Xall.p || !Yall.p || !Xb.p || !Yb.p || !lp.p || !idx.p)
    throw std::runtime_error("device allocation failed");
  check(hipMemcpyAsync(P.p, model.params.data(), off.back() * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemsetAsync(M1.p, 0, off.back() * 4, s), "clear");
  check(hipMemsetAsync(V1.p, 0, off.back() * 4, s), "clear");
  check(hipMemcpyAsync(Xall.p, X.data(), (size_t)nin * n * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemcpyAsync(Yall.p, Y.data(), (size_t)nout * n * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemcpyAsync(mean.p, model.mean.data(), nin * 4, hipMemcpyHostToDevice, s), "upload");
  check(hipMemcpyAsync(istd.p, model.istd.data(), nin * 4, hipMemcpyHostToDevice, s), "upload");
  mlp_standardise(Xall.p, mean.p, istd.p, nin, n, s);
  BatchBufs wk(sh, B);
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::vector<float> lh(B);
  std::vector<double> hist;
  int step = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(rng.next() % (uint64_t)(i + 1))]);
    double lsum = 0;
    for (int64_t c0 = 0; c0 + B <= n; c0 += B) {
      check(hipMemcpyAsync(idx.p, perm.data() + c0, B * 8, hipMemcpyHostToDevice, s), "upload");
      mlp_gather_cols(Xall.p, idx.p, B, nin, Xb.p, s);
      mlp_gather_cols(Yall.p, idx.p, B, nout, Yb.p, s);
      mlp_forward(sh, P.p, off, Xb.p, B, wk.b, s);
      mlp_loss_grad(wk.b.Z[sh.nlin()], Yb.p, nout, nout / 2, o.wmse, B, wk.b.dZ[sh.nlin()], lp.p, s);
      mlp_backward(sh, P.p, off, B, wk.b, G.p, s);
      mlp_adam(P.p, G.p, M1.p, V1.p, off.back(), o.lr, 0.9f, 0.999f, 1e-8f, ++step, s);
      check(hipMemcpyAsync(lh.data(), lp.p, B * 4, hipMemcpyDeviceToHost, s), "download");
      check(hipStreamSynchronize(s), "train");
      for (int b = 0; b < B; ++b) lsum += lh[b];
    }
    hist.push_back(lsum / (double)((n / B) * B));
  }
  check(hipMemcpyAsync(model.params.data(), P.p, off.back() * 4, hipMemcpyDeviceToHost, s), "download");
  check(hipStreamSynchronize(s), "train");
  return hist;
}

std::string dataset_append(const std::string& path, bool append, const std::vector<float>& X,
                           const std::vector<float>& Y, int64_t n, int nin, int nout) {
  int64_t have = 0;
  FILE* f = nullptr;
  if (append) f = std::fopen(path.c_str(), "r+b");
  if (f) {
    char mg[8];
    int32_t hdr[2];
    if (std::fread(mg, 1, 8, f) != 8 || std::memcmp(mg, kDataMagic, 8) != 0 || std::fread(hdr, 4, 2, f) != 2 ||
        std::fread(&have, 8, 1, f) != 1 || hdr[0] != nin || hdr[1] != nout) {
      std::fclose(f);
      return "not a compatible training file: " + path;
    }
  } else {
    f = std::fopen(path.c_str(), "w+b");
    if (!f) return "cannot write " + path;
    int32_t hdr[2] = {nin, nout};
    if (std::fwrite(kDataMagic, 1, 8, f) != 8 || std::fwrite(hdr, 4, 2, f) != 2 || std::fwrite(&have, 8, 1, f) != 1) {
      std::fclose(f);
      return "short write to " + path;
    }
  }
  std::fseek(f, 0, SEEK_END);
  std::vector<float> row(nin + nout);
  bool ok = true;
  for (int64_t c = 0; c < n && ok; ++c) {
    std::memcpy(row.data(), X.data() + (size_t)nin * c, nin * 4);
    std::memcpy(row.data() + nin, Y.data() + (size_t)nout * c, nout * 4);
    ok = std::fwrite(row.data(), 4, nin + nout, f) == (size_t)(nin + nout);
  }
  have += n;
  ok = ok && std::fseek(f, 16, SEEK_SET) == 0 && std::fwrite(&have, 8, 1, f) == 1;
  std::fclose(f);
  return ok ? "" : "short write to " + path;
}

std::string dataset_read(const std::string& path, std::vector<float>& X, std::vector<float>& Y, int64_t& n, int& nin,
                         int& nout) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return "cannot read " + path;
  char mg[8];
  int32_t hdr[2];
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kDataMagic, 8) == 0 && std::fread(hdr, 4, 2, f) == 2 &&
            std::fread(&n, 8, 1, f) == 1 && hdr[0] > 0 && hdr[1] > 0 && n >= 0 && n < ((int64_t)1 << 34);
  if (ok) {
    nin = hdr[0];
    nout = hdr[1];
    X.resize((size_t)nin * n);
    Y.resize((size_t)nout * n);
    std::vector<float> row(nin + nout);
    for (int64_t c = 0; c < n && ok; ++c) {
      ok = std::fread(row.data(), 4, nin + nout, f) == (size_t)(nin + nout);
      std::memcpy(X.data() + (size_t)nin * c, row.data(), nin * 4);
      std::memcpy(Y.data() + (size_t)nout * c, row.data() + nin, nout * 4);
    }
  }
  std::fclose(f);
  return ok ? "" : "not a valid training file: " + path;
}
