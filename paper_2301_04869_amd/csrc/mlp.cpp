// The warm-start perceptron behind the C ABI of rkkt_mlp.h: workspace,
// forward pass, backward pass and Adam step.  Products C = op(A) op(B) of
// row-major BF16 operands with FP32 accumulation and output go to rocBLAS
// (a row-major product is the column-major product of the transposes, so
// the operands are passed swapped with their transpose flags unchanged);
// everything else runs in k_mlp.hip.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <string>
#include <vector>

#include "mlp_dev.h"
#include "rkkt_mlp.h"

struct rkkt_mlp {
  int L = 0, bmax = 0;
  std::vector<int> sz;
  std::vector<long long> woff, boff;  // parameter offsets of W_l, b_l
  long long P = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t* pb = nullptr;           // BF16 copy of the parameters
  std::vector<uint16_t*> A;         // A_l [bmax][sz[l]], BF16 (A_0 = input)
  std::vector<float*> Z;            // Z_l [bmax][sz[l + 1]], FP32 pre-activations
  float *dZ = nullptr, *dA = nullptr, *part = nullptr;
  uint16_t* dZb = nullptr;
  int t = 0;
  rocblas_handle h = nullptr;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

std::string g_mlp_err;

int fail(rkkt_mlp* m, int code, const std::string& msg) {
  (m ? m->err : g_mlp_err) = msg;
  return code;
}

template <typename T>
hipError_t dalloc(rkkt_mlp* m, T** ptr, long long n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)std::max(n, 1LL) * sizeof(T));
  if (e == hipSuccess) m->allocs.push_back(q);
  *ptr = static_cast<T*>(q);
  return e;
}

// row-major C [M][N] = op(A) op(B) + beta C, op(A) [M][K], op(B) [K][N]
rocblas_status rm_gemm(rocblas_handle h, bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda,
                       const uint16_t* B, int ldb, float beta, float* C, int ldc) {
  const float one = 1.0f;
  return rocblas_gemm_ex(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                         ta ? rocblas_operation_transpose : rocblas_operation_none, N, M, K, &one, B,
                         rocblas_datatype_bf16_r, ldb, A, rocblas_datatype_bf16_r, lda, &beta, C,
                         rocblas_datatype_f32_r, ldc, C, rocblas_datatype_f32_r, ldc,
                         rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0);
}

int check(rkkt_mlp* m, const char* where, rocblas_status bs = rocblas_status_success) {
  if (bs != rocblas_status_success)
    return fail(m, -2, std::string(where) + ": rocBLAS status " + std::to_string((int)bs));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(m, -2, std::string(where) + ": " + hipGetErrorString(e));
  return 0;
}

int forward_impl(rkkt_mlp* m, const float* x, int B, float* y, hipStream_t st) {
  rocblas_set_stream(m->h, st);
  rkkt::mlp_to_bf16(x, m->A[0], (long long)B * m->sz[0], st);
  for (int l = 0; l < m->L; ++l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    const rocblas_status bs = rm_gemm(m->h, false, false, B, fo, fi, m->A[l], fi, m->pb + m->woff[l], fo,
                                      0.0f, m->Z[l], fo);
    if (int rc = check(m, "rkkt_mlp forward", bs)) return rc;
    const bool act = l + 1 < m->L;
    rkkt::mlp_bias_act(m->Z[l], m->p + m->boff[l], act ? m->A[l + 1] : nullptr, act ? nullptr : y, B, fo,
                       act, st);
  }
  return check(m, "rkkt_mlp forward");
}

int gradients_impl(rkkt_mlp* m, const float* x, const float* t, int B, float* loss, hipStream_t st) {
  if (int rc = forward_impl(m, x, B, nullptr, st)) return rc;
  const int L = m->L;
  const long long nout = (long long)B * m->sz[L];
  rkkt::mlp_out_grad(m->Z[L - 1], t, m->dZ, m->dZb, m->part, loss, nout, B, st);
  for (int l = L - 1; l >= 0; --l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    // dW_l = A_l^T dZ_l, db_l = column sums of dZ_l
    rocblas_status bs = rm_gemm(m->h, true, false, fi, fo, B, m->A[l], fi, m->dZb, fo, 0.0f,
                                m->g + m->woff[l], fo);
    if (int rc = check(m, "rkkt_mlp backward", bs)) return rc;
    rkkt::mlp_col_sum(m->dZ, B, fo, m->g + m->boff[l], st);
    if (l == 0) break;
    // dA_{l-1} = dZ_l W_l^T, dZ_{l-1} = dA_{l-1} g'(Z_{l-1})
    bs = rm_gemm(m->h, false, true, B, fi, fo, m->dZb, fo, m->pb + m->woff[l], fo, 0.0f, m->dA, fi);
    if (int rc = check(m, "rkkt_mlp backward", bs)) return rc;
    rkkt::mlp_act_back(m->dA, m->Z[l - 1], m->dZ, m->dZb, (long long)B * fi, st);
  }
  return check(m, "rkkt_mlp backward");
}

int args_ok(rkkt_mlp* m, int B, const char* where) {
  if (!m) return fail(nullptr, -1, std::string(where) + ": null handle");
  if (B < 1 || B > m->bmax) return fail(m, -1, std::string(where) + ": batch outside [1, batch_max]");
  return 0;
}

}  // namespace

extern "C" {

int rkkt_mlp_create(const int* sizes, int n_layers, int batch_max, rkkt_mlp** out) {
  if (!sizes || !out || n_layers < 1 || batch_max < 1) return fail(nullptr, -1, "rkkt_mlp_create: bad argument");
  for (int l = 0; l <= n_layers; ++l)
    if (sizes[l] < 1) return fail(nullptr, -1, "rkkt_mlp_create: layer width < 1");
  *out = nullptr;
  rkkt_mlp* m = new rkkt_mlp();
  m->L = n_layers;
  m->bmax = batch_max;
  m->sz.assign(sizes, sizes + n_layers + 1);
  int wmax = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->woff.push_back(m->P);
    m->P += (long long)m->sz[l] * m->sz[l + 1];
    m->boff.push_back(m->P);
    m->P += m->sz[l + 1];
  }
  for (int w : m->sz) wmax = std::max(wmax, w);
  const long long bw = (long long)batch_max * wmax;
  hipError_t e = hipSuccess;
  m->A.assign(n_layers, nullptr);
  m->Z.assign(n_layers, nullptr);
  if (e == hipSuccess) e = dalloc(m, &m->p, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->m, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->v, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->g, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->pb, m->P);
  for (int l = 0; l < n_layers && e == hipSuccess; ++l) {
    e = dalloc(m, &m->A[l], (long long)batch_max * m->sz[l]);
    if (e == hipSuccess) e = dalloc(m, &m->Z[l], (long long)batch_max * m->sz[l + 1]);
  }
  if (e == hipSuccess) e = dalloc(m, &m->dZ, bw);
  if (e == hipSuccess) e = dalloc(m, &m->dA, bw);
  if (e == hipSuccess) e = dalloc(m, &m->dZb, bw);
  if (e == hipSuccess) e = dalloc(m, &m->part, rkkt::mlp_out_grad_blocks((long long)batch_max * m->sz[n_layers]));
  if (e != hipSuccess) {
    std::string msg = std::string("rkkt_mlp_create: ") + hipGetErrorString(e);
    rkkt_mlp_destroy(m);
    return fail(nullptr, -6, msg);
  }
  if (rocblas_create_handle(&m->h) != rocblas_status_success) {
    rkkt_mlp_destroy(m);
    return fail(nullptr, -2, "rkkt_mlp_create: rocblas_create_handle");
  }
  *out = m;
  return 0;
}

int rkkt_mlp_destroy(rkkt_mlp* m) {
  if (!m) return 0;
  if (m->h) rocblas_destroy_handle(m->h);
  for (void* q : m->allocs) (void)hipFree(q);
  delete m;
  return 0;
}

const char* rkkt_mlp_last_error(const rkkt_mlp* m) { return m ? m->err.c_str() : g_mlp_err.c_str(); }

long long rkkt_mlp_n_params(const rkkt_mlp* m) { return m ? m->P : 0; }

int rkkt_mlp_set_params(rkkt_mlp* m, const float* params, hipStream_t st) {
  if (!m || !params) return fail(m, -1, "rkkt_mlp_set_params: null argument");
  hipError_t e = hipMemcpyAsync(m->p, params, m->P * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, m->P * sizeof(float), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, m->P * sizeof(float), st);
  if (e != hipSuccess) return fail(m, -2, std::string("rkkt_mlp_set_params: ") + hipGetErrorString(e));
  rkkt::mlp_to_bf16(m->p, m->pb, m->P, st);
  m->t = 0;
  return check(m, "rkkt_mlp_set_params");
}

int rkkt_mlp_get_params(const rkkt_mlp* m, float* params, hipStream_t st) {
  if (!m || !params) return fail(const_cast<rkkt_mlp*>(m), -1, "rkkt_mlp_get_params: null argument");
  hipError_t e = hipMemcpyAsync(params, m->p, m->P * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail(const_cast<rkkt_mlp*>(m), -2, std::string("rkkt_mlp_get_params: ") + hipGetErrorString(e));
  return 0;
}

int rkkt_mlp_forward(rkkt_mlp* m, const float* x, int batch, float* y, hipStream_t st) {
  if (int rc = args_ok(m, batch, "rkkt_mlp_forward")) return rc;
  if (!x || !y) return fail(m, -1, "rkkt_mlp_forward: null array");
  (void)hipGetLastError();
  return forward_impl(m, x, batch, y, st);
}

int rkkt_mlp_gradients(rkkt_mlp* m, const float* x, const float* t, int batch, float* grads, float* loss,
                       hipStream_t st) {
  if (int rc = args_ok(m, batch, "rkkt_mlp_gradients")) return rc;
  if (!x || !t || !loss) return fail(m, -1, "rkkt_mlp_gradients: null array");
  (void)hipGetLastError();
  if (int rc = gradients_impl(m, x, t, batch, loss, st)) return rc;
  if (grads) {
    hipError_t e = hipMemcpyAsync(grads, m->g, m->P * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(m, -2, std::string("rkkt_mlp_gradients: ") + hipGetErrorString(e));
  }
  return 0;
}

int rkkt_mlp_train_step(rkkt_mlp* m, const float* x, const float* t, int batch, float lr, float* loss,
                        hipStream_t st) {
  if (int rc = args_ok(m, batch, "rkkt_mlp_train_step")) return rc;
  if (!x || !t || !loss) return fail(m, -1, "rkkt_mlp_train_step: null array");
  (void)hipGetLastError();
  if (int rc = gradients_impl(m, x, t, batch, loss, st)) return rc;
  m->t += 1;
  rkkt::mlp_adam(m->p, m->g, m->m, m->v, m->pb, m->P, lr, m->t, st);
  return check(m, "rkkt_mlp_train_step");
}

}  // extern "C"
