// Launchers of the warm-start perceptron's kernels (k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rkkt {

// epilogues of the product kernel
enum { kMlpStore = 0, kMlpBiasGelu = 1, kMlpBiasOut = 2, kMlpGeluBack = 3 };

// C[m][n] = sum_k A[m][k] B[n][k] (BF16 operands, k-contiguous rows whose
// pitches lda, ldb are multiples of 8 and at least K rounded up to 8; FP32
// accumulation), then the epilogue:
//   kMlpStore:    zout[m][n] = C                         (pitch ldz)
//   kMlpBiasGelu: z = C + bias[n]; zout[m][n] = z when zout is set;
//                 hout[m][n] = bf16(g(z)) (pitch ldh); tout[n][m] likewise
//                 when tout is set (pitch ldt, a multiple of 8)
//   kMlpBiasOut:  z = C + bias[n]; zout[m][n] = z when set; y[m][n] = z when
//                 set (pitch N)
//   kMlpGeluBack: d = bf16(C g'(zin[m][n])) (zin pitch ldz); hout[m][n] = d,
//                 tout[n][m] = d when set
struct MlpGemm {
  const uint16_t* A;
  const uint16_t* B;
  int lda, ldb, M, N, K;
  const float* bias;
  const float* zin;
  float* zout;
  int ldz;
  uint16_t* hout;
  int ldh;
  uint16_t* tout;
  int ldt;
  float* y;
};

// where each layer's BF16 weight copies live: W_l as [fi][fo_p] at wb_off,
// W_l^T as [fo][fi_p] at wt_off (fo_p, fi_p: fo, fi rounded up to 8)
constexpr int kMlpMaxLayers = 8;
struct MlpLayers {
  int n;
  long long woff[kMlpMaxLayers], wb_off[kMlpMaxLayers], wt_off[kMlpMaxLayers];
  int fi[kMlpMaxLayers], fo[kMlpMaxLayers], fi_p[kMlpMaxLayers], fo_p[kMlpMaxLayers];
};

inline int mlp_pad8(int n) { return (n + 7) / 8 * 8; }

void mlp_gemm(int epi, const MlpGemm& g, hipStream_t st);
void mlp_input_bf16(const float* x, int rows, int cols, uint16_t* h, int ldh, uint16_t* t, int ldt,
                    hipStream_t st);
// partial sums per 32 x 32 tile of the output gradient (the part buffer's length)
int mlp_out_grad_tiles(int rows, int cols);
void mlp_out_grad(const float* Y, const float* T, int rows, int cols, uint16_t* h, int ldh, uint16_t* t,
                  int ldt, float* part, float* loss, hipStream_t st);
void mlp_param_copies(const float* p, long long n, const MlpLayers& L, uint16_t* wb, uint16_t* wt,
                      hipStream_t st);
void mlp_adam(float* p, const float* g, float* m, float* v, long long n, float lr, int t, const MlpLayers& L,
              uint16_t* wb, uint16_t* wt, hipStream_t st);
void mlp_fill_bf16(uint16_t* d, long long n, float v, hipStream_t st);

}  // namespace rkkt
