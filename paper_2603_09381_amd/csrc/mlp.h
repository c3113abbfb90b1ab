// A small multilayer perceptron in FP32 on gfx950: dense layers with ReLU between them,
// forward and backward passes on MFMA, Adam updates.  Activations are column major
// (features x batch: one column per sample); a layer's weight is out x in, column major.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

// C (m x n) = alpha op(A) op(B) + beta C, column major, FP32 (op: 0 = N, 1 = T)
void mlp_sgemm(int opa, int opb, int m, int n, int k, float alpha, const float* A, int64_t lda, const float* B,
               int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s);

struct MlpShape {
  int nin = 0, nhidden = 0, nlayer = 0, nout = 0;   // nlayer hidden layers of nhidden units
  int dims(int l) const { return l == 0 ? nin : (l <= nlayer ? nhidden : nout); }   // width of activation l
  int nlin() const { return nlayer + 1; }                                           // linear maps
};

// Parameters (device): per linear map l (input dims(l), output dims(l+1)): W_l then b_l,
// packed in one array; offsets from mlp_param_offsets.
std::vector<int64_t> mlp_param_offsets(const MlpShape& sh);

// Workspace of one batch: Z_l (pre-activations) and H_l (activations) for every layer and
// their gradients.
struct MlpBatch {
  int cap = 0;
  std::vector<float*> Z, H, dZ, dH;
};

// forward on X (nin x B): H_0 = X, Z_{l+1} = W_l H_l + b_l, H = relu(Z) except the output
void mlp_forward(const MlpShape& sh, const float* params, const std::vector<int64_t>& off, const float* X, int B,
                 MlpBatch& wk, hipStream_t s);
// output gradients from the loss: rows 0..nscore-1 binary cross entropy with logits against
// labels in {0, 1}, rows nscore.. squared error (weight wmse); loss partial sums per column
// are written to loss_part [B]
void mlp_loss_grad(const float* out, const float* labels, int nout, int nscore, float wmse, int B, float* dout,
                   float* loss_part, hipStream_t s);
// backward: parameter gradients grad (same packing as params) from dZ of the output layer
void mlp_backward(const MlpShape& sh, const float* params, const std::vector<int64_t>& off, int B, MlpBatch& wk,
                  float* grad, hipStream_t s);
// Adam step t (1-based) on n parameters
void mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
              int t, hipStream_t s);
// gather columns: dst[:, i] = src[:, idx[i]] for rows r < rows (column major, ld = rows)
void mlp_gather_cols(const float* src, const int64_t* idx, int n, int rows, float* dst, hipStream_t s);
// standardise rows: x[r, c] = (x[r, c] - mean[r]) * istd[r]
void mlp_standardise(float* x, const float* mean, const float* istd, int rows, int64_t cols, hipStream_t s);
