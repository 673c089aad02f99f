// Elementwise and reduction kernels of the warm-start perceptron (the
// products run on the BLAS library, BF16 in, FP32 accumulation and out).
//
// GELU in the erf form, g(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2, with
// g'(a) = Phi(a) + a phi(a); loss 1/(2B) sum ||y - t||^2, so the output
// gradient is (y - t) / B; Adam as published by Kingma and Ba.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_dev.h"

namespace rkkt {
namespace {

constexpr int kT = 256;
inline unsigned blocks(long long n) { return (unsigned)((n + kT - 1) / kT); }

// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * expf(-0.5f * a * a) * 0.39894228040143268f;
}

__global__ void k_to_bf16(const float* __restrict__ s, uint16_t* __restrict__ d, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) d[i] = to_bf16(s[i]);
}

// Z [rows][cols] += b; hidden layers also A = bf16(g(Z)); the output layer
// also copies Z to y when y is given
__global__ void k_bias_act(float* __restrict__ Z, const float* __restrict__ b, uint16_t* __restrict__ A,
                           float* __restrict__ y, int rows, int cols, int act) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= (long long)rows * cols) return;
  const float z = Z[i] + b[i % cols];
  Z[i] = z;
  if (act) A[i] = to_bf16(gelu(z));
  else if (y) y[i] = z;
}

// dZ = (Y - T) / B (FP32 and BF16), and per-block partial sums of (Y - T)^2
__global__ void k_out_grad(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dZ,
                           uint16_t* __restrict__ dZb, float* __restrict__ part, long long n, float inv_b) {
  __shared__ float red[kT];
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  float sq = 0.0f;
  if (i < n) {
    const float r = Y[i] - T[i];
    sq = r * r;
    const float g = r * inv_b;
    dZ[i] = g;
    dZb[i] = to_bf16(g);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = 0.5 inv_b sum of the partials, in a fixed order
__global__ void k_loss_final(const float* __restrict__ part, int np, float inv_b, float* __restrict__ loss) {
  __shared__ float red[kT];
  float s = 0.0f;
  for (int i = threadIdx.x; i < np; i += kT) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = 0.5f * inv_b * red[0];
}

// dZ = dA g'(Z) (FP32 and BF16)
__global__ void k_act_back(const float* __restrict__ dA, const float* __restrict__ Z, float* __restrict__ dZ,
                           uint16_t* __restrict__ dZb, long long n) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float g = dA[i] * gelu_grad(Z[i]);
  dZ[i] = g;
  dZb[i] = to_bf16(g);
}

// db[c] = sum over rows of dZ[r][c] (rows in order)
__global__ void k_col_sum(const float* __restrict__ dZ, int rows, int cols, float* __restrict__ db) {
  const int c = blockIdx.x * kT + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += dZ[(long long)r * cols + c];
  db[c] = s;
}

// Adam on the master parameters, then their BF16 copies
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, long long n, float lr, float b1,
                       float b2, float c1, float c2, float eps) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = to_bf16(pi);
}

}  // namespace

void mlp_to_bf16(const float* s, uint16_t* d, long long n, hipStream_t st) {
  k_to_bf16<<<blocks(n), kT, 0, st>>>(s, d, n);
}

void mlp_bias_act(float* Z, const float* b, uint16_t* A, float* y, int rows, int cols, bool act, hipStream_t st) {
  k_bias_act<<<blocks((long long)rows * cols), kT, 0, st>>>(Z, b, A, y, rows, cols, act ? 1 : 0);
}

int mlp_out_grad_blocks(long long n) { return (int)blocks(n); }

void mlp_out_grad(const float* Y, const float* T, float* dZ, uint16_t* dZb, float* part, float* loss,
                  long long n, int batch, hipStream_t st) {
  const float inv_b = 1.0f / (float)batch;
  k_out_grad<<<blocks(n), kT, 0, st>>>(Y, T, dZ, dZb, part, n, inv_b);
  k_loss_final<<<1, kT, 0, st>>>(part, (int)blocks(n), inv_b, loss);
}

void mlp_act_back(const float* dA, const float* Z, float* dZ, uint16_t* dZb, long long n, hipStream_t st) {
  k_act_back<<<blocks(n), kT, 0, st>>>(dA, Z, dZ, dZb, n);
}

void mlp_col_sum(const float* dZ, int rows, int cols, float* db, hipStream_t st) {
  k_col_sum<<<blocks(cols), kT, 0, st>>>(dZ, rows, cols, db);
}

void mlp_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, long long n, float lr, int t,
              hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  k_adam<<<blocks(n), kT, 0, st>>>(p, g, m, v, pb, n, lr, b1, b2, c1, c2, 1e-8f);
}

}  // namespace rkkt
