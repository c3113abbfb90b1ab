// Learned skeleton proposals for the leaf IDs: per-node features of a leaf cell, the
// network that scores nodes and estimates ranks, its training and its file formats.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mlp.h"
#include "plan.h"

constexpr int PMX_NFEAT = 20;  // features per node
constexpr int PMX_NOUT = 8;    // per node: 4 skeleton logits (column IDs q, u; row IDs value,
                               // derivative), 4 rank fractions k / n of the same IDs

// Host copies of the geometry needed for the features.
struct HostGeom {
  int m = 0;
  const int64_t* node_off = nullptr;
  const double *x = nullptr, *y = nullptr, *dx = nullptr, *dy = nullptr, *ddx = nullptr, *ddy = nullptr;
  double k_ext = 0;
  const double* k_int = nullptr;
};

// Features of every node of the leaf cells (one inclusion per leaf), column major
// PMX_NFEAT x n_nodes with the nodes cell by cell in leaf order:
//   cell: k+ r_c, k+ R_p, k-/k+, n / 256, near cells / 8, |Fourier modes 2..6| of the
//         node radii (relative), mean radius / r_c;
//   node: direction from the centre (cos, sin), normal, radius / r_c, curvature r_c,
//         speed |x'| / r_c (node spacing times n / (2 pi r_c)), distance to the nearest node of a near
//         cell / r_c, distance to the proxy circle / r_c (clamped to [-10, 10]).
void leaf_features(const HostGeom& g, const std::vector<CellPlan>& leaves, std::vector<float>& X);

struct MlpModel {
  MlpShape sh;
  std::vector<float> mean, istd;  // input standardisation
  std::vector<float> params;      // packed as mlp_param_offsets
};

std::string mlp_save(const std::string& path, const MlpModel& m);
std::string mlp_load(const std::string& path, MlpModel& m);

// out (host, nout x n) = network(X (host, nin x n)) on the device
void mlp_predict(const MlpModel& m, const std::vector<float>& X, int64_t n, std::vector<float>& out, hipStream_t s);

struct TrainOpts {
  int epochs = 30, batch = 4096, hidden = 256, layers = 3;
  float lr = 1e-3f, wmse = 10.0f;
  uint64_t seed = 1;
};

// Adam on samples X (nin x n), labels Y (nout x n: 4 binary skeleton labels then 4 rank
// fractions); initial weights from a seeded generator; returns the mean loss per epoch.
std::vector<double> mlp_train(const std::vector<float>& X, const std::vector<float>& Y, int64_t n, int nin, int nout,
                              const TrainOpts& o, MlpModel& model, hipStream_t s);

// Training files: a header, then per sample nin features and nout labels (FP32).
std::string dataset_append(const std::string& path, bool append, const std::vector<float>& X,
                           const std::vector<float>& Y, int64_t n, int nin, int nout);
std::string dataset_read(const std::string& path, std::vector<float>& X, std::vector<float>& Y, int64_t& n, int& nin,
                         int& nout);
