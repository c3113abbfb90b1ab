// FP32 kernels of the skeleton-proposal network: MFMA GEMM (16x16x4 FP32 blocks, 64x64
// tiles per 256-thread workgroup, each wave a 32x32 sub-tile), bias and ReLU, the loss
// gradient, column sums and the Adam update.
#include "mlp.h"
#include "pmx_common.h"

#include <algorithm>
#include <cmath>

typedef float f4v __attribute__((ext_vector_type(4)));

// FP32 16x16x4 MFMA: operand A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; the
// accumulator holds element (i, j) in register i % 4 of lane j + 16 (i / 4).
template <int OPA, int OPB>
__global__ __launch_bounds__(256) void k_sgemm(int m, int n, int k, float alpha, const float* A, int64_t lda,
                                               const float* B, int64_t ldb, float beta, float* C, int64_t ldc) {
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0, 0, 0, 0};
  for (int k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
      int i, kk;
      if (OPA == 0) {
        i = tid & 63;
        kk = (tid >> 6) + 4 * pass;
      } else {
        kk = tid & 15;
        i = (tid >> 4) + 16 * pass;
      }
      const int gi = tm + i, gk = k0 + kk;
      const int ci = min(gi, m - 1), ck = min(gk, k - 1);
      const float v = (OPA == 0) ? A[ci + (int64_t)ck * lda] : A[ck + (int64_t)ci * lda];
      As[kk][i] = (gi < m && gk < k) ? v : 0.0f;
    }
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
      int j, kk;
      if (OPB == 0) {
        kk = tid & 15;
        j = (tid >> 4) + 16 * pass;
      } else {
        j = tid & 63;
        kk = (tid >> 6) + 4 * pass;
      }
      const int gj = tn + j, gk = k0 + kk;
      const int cj = min(gj, n - 1), ck = min(gk, k - 1);
      const float v = (OPB == 0) ? B[ck + (int64_t)cj * ldb] : B[cj + (int64_t)ck * ldb];
      Bs[kk][j] = (gj < n && gk < k) ? v : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[ks + (lane >> 4)][wm + t * 16 + (lane & 15)];
        b[t] = Bs[ks + (lane >> 4)][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm + wm + bi * 16 + 4 * (lane >> 4) + r;
        const int col = tn + wn + bj * 16 + (lane & 15);
        if (row < m && col < n) {
          float* cp = C + row + (int64_t)col * ldc;
          const float v = alpha * acc[bi][bj][r];
          *cp = (beta != 0.0f) ? v + beta * (*cp) : v;
        }
      }
}

void mlp_sgemm(int opa, int opb, int m, int n, int k, float alpha, const float* A, int64_t lda, const float* B,
               int64_t ldb, float beta, float* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((m + 63) / 64, (n + 63) / 64);
  if (opa == 0 && opb == 0)
    PMX_LAUNCH((k_sgemm<0, 0>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (opa == 0 && opb == 1)
    PMX_LAUNCH((k_sgemm<0, 1>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (opa == 1 && opb == 0)
    PMX_LAUNCH((k_sgemm<1, 0>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    PMX_LAUNCH((k_sgemm<1, 1>), grid, dim3(256), 0, s, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

// Z[:, c] += b; H = relu(Z) (H may be NULL: the output layer keeps Z)
__global__ void k_bias_relu(float* Z, const float* b, int rows, int64_t cols, float* H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int r = (int)(e % rows);
  const float z = Z[e] + b[r];
  Z[e] = z;
  if (H) H[e] = z > 0.0f ? z : 0.0f;
}

// dZ = dH where Z > 0, else 0
__global__ void k_relu_back(const float* Z, const float* dH, float* dZ, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dZ[e] = Z[e] > 0.0f ? dH[e] : 0.0f;
}

// row sums of the column-major rows x cols matrix X into out[rows] (one workgroup per row)
__global__ __launch_bounds__(256) void k_rowsum(const float* X, int rows, int cols, float* out) {
  const int r = blockIdx.x;
  float s = 0.0f;
  for (int c = threadIdx.x; c < cols; c += 256) s += X[r + (int64_t)c * rows];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

// loss and its gradient per column (one thread per column); the gradient carries the 1/B
// of the batch mean
__global__ void k_loss_grad(const float* out, const float* lab, int nout, int nscore, float wmse, int B, float* dout,
                            float* loss_part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= B) return;
  const float ib = 1.0f / (float)B;
  float L = 0.0f;
  for (int r = 0; r < nout; ++r) {
    const float z = out[r + (int64_t)c * nout], y = lab[r + (int64_t)c * nout];
    float g;
    if (r < nscore) {
      // binary cross entropy with logits, written to avoid overflow
      const float az = fabsf(z);
      L += fmaxf(z, 0.0f) - z * y + log1pf(expf(-az));
      const float sg = z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
      g = sg - y;
    } else {
      const float d = z - y;
      L += wmse * d * d;
      g = 2.0f * wmse * d;
    }
    dout[r + (int64_t)c * nout] = g * ib;
  }
  loss_part[c] = L;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_cols(const float* src, const int64_t* idx, int n, int rows, float* dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * rows) return;
  const int r = (int)(e % rows);
  const int64_t c = e / rows;
  dst[e] = src[r + idx[c] * rows];
}

__global__ void k_standardise(float* x, const float* mean, const float* istd, int rows, int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int r = (int)(e % rows);
  x[e] = (x[e] - mean[r]) * istd[r];
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

std::vector<int64_t> mlp_param_offsets(const MlpShape& sh) {
  std::vector<int64_t> off;
  int64_t o = 0;
  for (int l = 0; l < sh.nlin(); ++l) {
    off.push_back(o);                               // W_l
    o += (int64_t)sh.dims(l + 1) * sh.dims(l);
    off.push_back(o);                               // b_l
    o += sh.dims(l + 1);
  }
  off.push_back(o);                                 // total
  return off;
}

void mlp_forward(const MlpShape& sh, const float* params, const std::vector<int64_t>& off, const float* X, int B,
                 MlpBatch& wk, hipStream_t s) {
  const int nl = sh.nlin();
  const float* H = X;
  for (int l = 0; l < nl; ++l) {
    const int in = sh.dims(l), out = sh.dims(l + 1);
    const float* W = params + off[2 * l];
    const float* b = params + off[2 * l + 1];
    float* Z = wk.Z[l + 1];
    mlp_sgemm(0, 0, out, B, in, 1.0f, W, out, H, in, 0.0f, Z, out, s);
    float* Hn = (l + 1 < nl) ? wk.H[l + 1] : nullptr;
    PMX_LAUNCH(k_bias_relu, dim3(nblk((int64_t)out * B)), dim3(256), 0, s, Z, b, out, (int64_t)B, Hn);
    H = Hn;
  }
  wk.H[0] = const_cast<float*>(X);
}

void mlp_loss_grad(const float* out, const float* labels, int nout, int nscore, float wmse, int B, float* dout,
                   float* loss_part, hipStream_t s) {
  PMX_LAUNCH(k_loss_grad, dim3(nblk(B)), dim3(256), 0, s, out, labels, nout, nscore, wmse, B, dout,
                     loss_part);
}

void mlp_backward(const MlpShape& sh, const float* params, const std::vector<int64_t>& off, int B, MlpBatch& wk,
                  float* grad, hipStream_t s) {
  for (int l = sh.nlin() - 1; l >= 0; --l) {
    const int in = sh.dims(l), out = sh.dims(l + 1);
    const float* W = params + off[2 * l];
    const float* dZ = wk.dZ[l + 1];
    // dW = dZ H^T, db = row sums of dZ
    mlp_sgemm(0, 1, out, in, B, 1.0f, dZ, out, wk.H[l], in, 0.0f, grad + off[2 * l], out, s);
    PMX_LAUNCH(k_rowsum, dim3(out), dim3(256), 0, s, dZ, out, B, grad + off[2 * l + 1]);
    if (l > 0) {
      mlp_sgemm(1, 0, in, B, out, 1.0f, W, out, dZ, out, 0.0f, wk.dH[l], in, s);
      PMX_LAUNCH(k_relu_back, dim3(nblk((int64_t)in * B)), dim3(256), 0, s, wk.Z[l], wk.dH[l], wk.dZ[l],
                         (int64_t)in * B);
    }
  }
}

void mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
              int t, hipStream_t s) {
  const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
  PMX_LAUNCH(k_adam, dim3(nblk(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void mlp_gather_cols(const float* src, const int64_t* idx, int n, int rows, float* dst, hipStream_t s) {
  if (n <= 0) return;
  PMX_LAUNCH(k_gather_cols, dim3(nblk((int64_t)n * rows)), dim3(256), 0, s, src, idx, n, rows, dst);
}

void mlp_standardise(float* x, const float* mean, const float* istd, int rows, int64_t cols, hipStream_t s) {
  if (cols <= 0) return;
  PMX_LAUNCH(k_standardise, dim3(nblk(rows * cols)), dim3(256), 0, s, x, mean, istd, rows, cols);
}
