// Launchers of the warm-start perceptron's kernels (k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rkkt {

void mlp_to_bf16(const float* s, uint16_t* d, long long n, hipStream_t st);
void mlp_bias_act(float* Z, const float* b, uint16_t* A, float* y, int rows, int cols, bool act, hipStream_t st);
int mlp_out_grad_blocks(long long n);
void mlp_out_grad(const float* Y, const float* T, float* dZ, uint16_t* dZb, float* part, float* loss,
                  long long n, int batch, hipStream_t st);
void mlp_act_back(const float* dA, const float* Z, float* dZ, uint16_t* dZb, long long n, hipStream_t st);
void mlp_col_sum(const float* dZ, int rows, int cols, float* db, hipStream_t st);
void mlp_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, long long n, float lr, int t,
              hipStream_t st);

}  // namespace rkkt
