// Kernels of the warm-start perceptron: BF16 products on the matrix cores
// with FP32 accumulation and fused epilogues, the output-layer gradient and
// loss, and the Adam step.
//
// GELU in the erf form, g(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2, with
// g'(a) = Phi(a) + a phi(a); loss 1/(2B) sum ||y - t||^2, so the output
// gradient is (y - t) / B; Adam as published by Kingma and Ba.
//
// Products.  Every product of a layer is C[m][n] = sum_k A[m][k] B[n][k] with
// both operands stored k-contiguous in BF16 (row pitch a multiple of 8
// elements, so 8 consecutive k are one aligned 16-byte load):
//   forward   Z_l  = A_l W_l + b_l   A = A_l [B][fi],   B = W_l^T [fo][fi]
//   dW        dW_l = A_l^T dZ_l      A = A_l^T [fi][B], B = dZ_l^T [fo][B]
//   dA        dA   = dZ_l W_l^T      A = dZ_l [B][fo],  B = W_l [fi][fo]
// so the parameters keep two BF16 copies per layer (W_l and W_l^T) and the
// forward and backward epilogues write each activation and output gradient in
// both orientations.  The transposed activations carry one extra row of ones
// (row fi of A_l^T): the dW product over fi + 1 rows then also yields the
// bias gradient, the column sums of dZ_l, in the row that follows W_l in the
// parameter layout.
//
// Each 32 x 32 output tile is 2 x 2 blocks of v_mfma_f32_16x16x32_bf16 (A
// operand: lane holds row lane % 16, k group lane / 16 of 8 consecutive k;
// B operand: column lane % 16, the same k group; result register r of a
// lane: row 4 (lane / 16) + r, column lane % 16).  Operands come straight
// from global memory (each 16-byte fragment is used by two products), the
// next k step's fragments loaded while the current step's products run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_dev.h"

namespace rkkt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// 8 consecutive BF16 values row[kk .. kk + 7], zero from k = K on.  The row's
// pitch is at least K rounded up to 8, so a granule that starts below K lies
// inside the row.
__device__ __forceinline__ uint4 frag8(const uint16_t* __restrict__ row, int kk, int K) {
  if (kk >= K) return make_uint4(0u, 0u, 0u, 0u);
  uint4 v = *reinterpret_cast<const uint4*>(row + kk);
  const int nv = K - kk;
  if (nv < 8) {
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t lo = 2 * q < nv ? 0x0000ffffu : 0u;
      const uint32_t hi = 2 * q + 1 < nv ? 0xffff0000u : 0u;
      w[q] &= lo | hi;
    }
    v = make_uint4(w[0], w[1], w[2], w[3]);
  }
  return v;
}

__device__ __forceinline__ f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}

// One workgroup of four wavefronts per 32 x 32 output tile: wavefront w
// takes the k steps w, w + 4, ... (so each wavefront's chain of dependent
// loads is a quarter of K long), the four partial tiles are added in LDS in
// wavefront order, and wavefront w then applies the epilogue to block
// (w / 2, w % 2) of the tile.
constexpr int kGemmWaves = 4;

template <int EPI>
__global__ __launch_bounds__(64 * kGemmWaves) void k_gemm(MlpGemm g) {
  __shared__ f32x4 part[kGemmWaves][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t* pa[2];
  const uint16_t* pb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    pa[i] = g.A + (long long)min(m0 + 16 * i + r16, g.M - 1) * g.lda;
    pb[i] = g.B + (long long)min(n0 + 16 * i + r16, g.N - 1) * g.ldb;
  }
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int kStride = 32 * kGemmWaves;
  uint4 a[2], b[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    a[i] = frag8(pa[i], 32 * w + kq, g.K);
    b[i] = frag8(pb[i], 32 * w + kq, g.K);
  }
  for (int k0 = 32 * w; k0 < g.K; k0 += kStride) {
    uint4 an[2], bn[2];
    const int kn = k0 + kStride + kq;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      an[i] = frag8(pa[i], kn, g.K);
      bn[i] = frag8(pb[i], kn, g.K);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = an[i];
      b[i] = bn[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) part[w][2 * i + j][lane] = acc[i][j];
  __syncthreads();
  // epilogue of block (i, j) = (w / 2, w % 2): lane holds rows mr .. mr + 3 of column nc
  const int i = w >> 1, j = w & 1;
  f32x4 t = part[0][w][lane];
#pragma unroll
  for (int q = 1; q < kGemmWaves; ++q) t += part[q][w][lane];
  const int mr = m0 + 16 * i + 4 * (lane >> 4);
  const int nc = n0 + 16 * j + r16;
  if (nc >= g.N) return;
  float v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = t[r];
  uint16_t h[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = mr + r;
    if (m >= g.M) break;
    const long long o = (long long)m * g.ldz + nc;
    if (EPI == kMlpStore) {
      g.zout[o] = v[r];
    } else if (EPI == kMlpBiasGelu || EPI == kMlpBiasOut) {
      const float z = v[r] + g.bias[nc];
      if (g.zout) g.zout[o] = z;
      if (EPI == kMlpBiasOut) {
        if (g.y) g.y[(long long)m * g.N + nc] = z;
      } else {
        h[r] = to_bf16(gelu(z));
        g.hout[(long long)m * g.ldh + nc] = h[r];
      }
    } else {  // kMlpGeluBack: dZ_{l-1} = dA g'(Z_{l-1})
      h[r] = to_bf16(v[r] * gelu_grad(g.zin[o]));
      g.hout[(long long)m * g.ldh + nc] = h[r];
    }
  }
  if ((EPI == kMlpBiasGelu || EPI == kMlpGeluBack) && g.tout) {
    uint16_t* tp = g.tout + (long long)nc * g.ldt + mr;
    if (mr + 3 < g.M) {
      *reinterpret_cast<uint2*>(tp) = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                 (uint32_t)h[2] | ((uint32_t)h[3] << 16));
    } else {
      for (int r = 0; r < 4 && mr + r < g.M; ++r) tp[r] = h[r];
    }
  }
}

// x [rows][cols] FP32 -> BF16 row-major (pitch ldh) and transposed (pitch ldt)
__global__ void k_input_bf16(const float* __restrict__ x, int rows, int cols, uint16_t* __restrict__ h, int ldh,
                             uint16_t* __restrict__ t, int ldt) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= (long long)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  const uint16_t v = to_bf16(x[i]);
  h[(long long)r * ldh + c] = v;
  if (t) t[(long long)c * ldt + r] = v;
}

// dZ = (Y - T) / B in BF16, row-major and transposed, and the per-tile
// partial sums of (Y - T)^2: one workgroup per 32 x 32 tile, the transposed
// copy written through LDS so both stores are coalesced
constexpr int kOG = 32, kOGT = 256;
__global__ __launch_bounds__(kOGT) void k_out_grad(const float* __restrict__ Y, const float* __restrict__ T,
                                                   int rows, int cols, float inv_b, uint16_t* __restrict__ h,
                                                   int ldh, uint16_t* __restrict__ t, int ldt,
                                                   float* __restrict__ part) {
  __shared__ uint16_t tile[kOG][kOG + 2];
  __shared__ float red[kOGT];
  const int c0 = blockIdx.x * kOG, r0 = blockIdx.y * kOG;
  const int tx = threadIdx.x % kOG, ty = threadIdx.x / kOG;
  float sq = 0.0f;
  for (int rr = ty; rr < kOG; rr += kOGT / kOG) {
    const int r = r0 + rr, c = c0 + tx;
    uint16_t v = 0;
    if (r < rows && c < cols) {
      const long long i = (long long)r * cols + c;
      const float d = Y[i] - T[i];
      sq = fmaf(d, d, sq);
      v = to_bf16(d * inv_b);
      h[(long long)r * ldh + c] = v;
    }
    tile[rr][tx] = v;
  }
  __syncthreads();
  for (int cc = ty; cc < kOG; cc += kOGT / kOG) {
    const int c = c0 + cc, r = r0 + tx;
    if (c < cols && r < rows) t[(long long)c * ldt + r] = tile[tx][cc];
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = kOGT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// loss = 0.5 inv_b sum of the partials, in a fixed order
constexpr int kLossT = 256;
__global__ __launch_bounds__(kLossT) void k_loss_final(const float* __restrict__ part, int np, float inv_b,
                                                       float* __restrict__ loss) {
  __shared__ float red[kLossT];
  float sum = 0.0f;
  for (int i = threadIdx.x; i < np; i += kLossT) sum += part[i];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int w = kLossT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = 0.5f * inv_b * red[0];
}

// BF16 copies of parameter i: W_l entries into W_l [fi][pitch fo] and
// W_l^T [fo][pitch fi], biases nowhere (they stay FP32)
__device__ __forceinline__ void store_copies(const MlpLayers& L, long long i, float p, uint16_t* __restrict__ wb,
                                             uint16_t* __restrict__ wt) {
  for (int l = 0; l < L.n; ++l) {
    const long long rel = i - L.woff[l];
    const long long nw = (long long)L.fi[l] * L.fo[l];
    if (rel >= 0 && rel < nw) {
      const int r = (int)(rel / L.fo[l]), c = (int)(rel % L.fo[l]);
      const uint16_t v = to_bf16(p);
      wb[L.wb_off[l] + (long long)r * L.fo_p[l] + c] = v;
      wt[L.wt_off[l] + (long long)c * L.fi_p[l] + r] = v;
      return;
    }
  }
}

__global__ void k_param_copies(const float* __restrict__ p, long long n, MlpLayers L, uint16_t* __restrict__ wb,
                               uint16_t* __restrict__ wt) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) store_copies(L, i, p[i], wb, wt);
}

// Adam on the master parameters, then their BF16 copies
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float c1, float c2,
                       float eps, MlpLayers L, uint16_t* __restrict__ wb, uint16_t* __restrict__ wt) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  store_copies(L, i, pi, wb, wt);
}

__global__ void k_fill_bf16(uint16_t* __restrict__ d, long long n, uint16_t v) {
  const long long i = (long long)blockIdx.x * kT + threadIdx.x;
  if (i < n) d[i] = v;
}

}  // namespace

void mlp_gemm(int epi, const MlpGemm& g, hipStream_t st) {
  const dim3 grid((unsigned)((g.N + 31) / 32), (unsigned)((g.M + 31) / 32));
  switch (epi) {
    case kMlpStore: k_gemm<kMlpStore><<<grid, 64 * kGemmWaves, 0, st>>>(g); break;
    case kMlpBiasGelu: k_gemm<kMlpBiasGelu><<<grid, 64 * kGemmWaves, 0, st>>>(g); break;
    case kMlpBiasOut: k_gemm<kMlpBiasOut><<<grid, 64 * kGemmWaves, 0, st>>>(g); break;
    default: k_gemm<kMlpGeluBack><<<grid, 64 * kGemmWaves, 0, st>>>(g); break;
  }
}

void mlp_input_bf16(const float* x, int rows, int cols, uint16_t* h, int ldh, uint16_t* t, int ldt,
                    hipStream_t st) {
  k_input_bf16<<<blocks((long long)rows * cols), kT, 0, st>>>(x, rows, cols, h, ldh, t, ldt);
}

int mlp_out_grad_tiles(int rows, int cols) { return ((rows + kOG - 1) / kOG) * ((cols + kOG - 1) / kOG); }

void mlp_out_grad(const float* Y, const float* T, int rows, int cols, uint16_t* h, int ldh, uint16_t* t,
                  int ldt, float* part, float* loss, hipStream_t st) {
  const dim3 grid((unsigned)((cols + kOG - 1) / kOG), (unsigned)((rows + kOG - 1) / kOG));
  const float inv_b = 1.0f / (float)rows;
  k_out_grad<<<grid, kOGT, 0, st>>>(Y, T, rows, cols, inv_b, h, ldh, t, ldt, part);
  k_loss_final<<<1, kLossT, 0, st>>>(part, mlp_out_grad_tiles(rows, cols), inv_b, loss);
}

void mlp_param_copies(const float* p, long long n, const MlpLayers& L, uint16_t* wb, uint16_t* wt,
                      hipStream_t st) {
  k_param_copies<<<blocks(n), kT, 0, st>>>(p, n, L, wb, wt);
}

void mlp_adam(float* p, const float* g, float* m, float* v, long long n, float lr, int t, const MlpLayers& L,
              uint16_t* wb, uint16_t* wt, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  k_adam<<<blocks(n), kT, 0, st>>>(p, g, m, v, n, lr, b1, b2, c1, c2, 1e-8f, L, wb, wt);
}

void mlp_fill_bf16(uint16_t* d, long long n, float v, hipStream_t st) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  k_fill_bf16<<<blocks(n), kT, 0, st>>>(d, n, (uint16_t)(u >> 16));
}

}  // namespace rkkt
