// The warm-start perceptron behind the C ABI of rkkt_mlp.h: workspace,
// forward pass, backward pass and Adam step, all in k_mlp.hip (BF16 products
// on the matrix cores with FP32 accumulation and fused epilogues).
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "mlp_dev.h"
#include "rkkt_mlp.h"

using rkkt::mlp_pad8;

struct rkkt_mlp {
  int L = 0, bmax = 0, bpit = 0;      // bpit: batch_max rounded up to 8
  std::vector<int> sz;
  std::vector<long long> woff, boff;  // parameter offsets of W_l, b_l
  long long P = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  rkkt::MlpLayers lay{};
  uint16_t *wb = nullptr, *wt = nullptr;  // BF16 W_l [fi][fo_p] and W_l^T [fo][fi_p]
  std::vector<uint16_t*> A;           // A_l [bmax][pad8(sz[l])], BF16 (A_0 = input)
  std::vector<uint16_t*> AT;          // A_l^T [sz[l] + 1][bpit], BF16, last row ones
  std::vector<float*> Z;              // Z_l [bmax][sz[l + 1]], FP32 pre-activations
  uint16_t *dZb[2] = {nullptr, nullptr}, *dZT[2] = {nullptr, nullptr};  // output gradients, both orientations
  float* lpart = nullptr;             // loss partial sums, one per output-gradient tile
  int t = 0;
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
  const size_t bytes = (size_t)std::max(n, 1LL) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e == hipSuccess) {
    m->allocs.push_back(q);
    e = hipMemset(q, 0, bytes);
  }
  *ptr = static_cast<T*>(q);
  return e;
}

int check(rkkt_mlp* m, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(m, -2, std::string(where) + ": " + hipGetErrorString(e));
  return 0;
}

// Forward pass over B rows of x.  With `train`, the FP32 pre-activations and
// the transposed activations (operands of the dW products) are kept;
// otherwise only y is written.
int forward_impl(rkkt_mlp* m, const float* x, int B, float* y, bool train, hipStream_t st) {
  const int L = m->L;
  rkkt::mlp_input_bf16(x, B, m->sz[0], m->A[0], mlp_pad8(m->sz[0]), train ? m->AT[0] : nullptr, m->bpit, st);
  for (int l = 0; l < L; ++l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    const bool last = l + 1 == L;
    rkkt::MlpGemm g{};
    g.A = m->A[l];
    g.lda = mlp_pad8(fi);
    g.B = m->wt + m->lay.wt_off[l];
    g.ldb = m->lay.fi_p[l];
    g.M = B;
    g.N = fo;
    g.K = fi;
    g.bias = m->p + m->boff[l];
    g.zout = train ? m->Z[l] : nullptr;
    g.ldz = fo;
    if (!last) {
      g.hout = m->A[l + 1];
      g.ldh = mlp_pad8(fo);
      g.tout = train ? m->AT[l + 1] : nullptr;
      g.ldt = m->bpit;
    } else {
      g.y = y;
    }
    rkkt::mlp_gemm(last ? rkkt::kMlpBiasOut : rkkt::kMlpBiasGelu, g, st);
  }
  return check(m, "rkkt_mlp forward");
}

int gradients_impl(rkkt_mlp* m, const float* x, const float* t, int B, float* loss, hipStream_t st) {
  if (int rc = forward_impl(m, x, B, nullptr, true, st)) return rc;
  const int L = m->L;
  int c = 0;
  rkkt::mlp_out_grad(m->Z[L - 1], t, B, m->sz[L], m->dZb[c], mlp_pad8(m->sz[L]), m->dZT[c], m->bpit, m->lpart,
                     loss, st);
  for (int l = L - 1; l >= 0; --l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    // [dW_l; db_l] = [A_l^T; 1^T] dZ_l: fi + 1 rows, the last one lands on b_l
    rkkt::MlpGemm gw{};
    gw.A = m->AT[l];
    gw.lda = m->bpit;
    gw.B = m->dZT[c];
    gw.ldb = m->bpit;
    gw.M = fi + 1;
    gw.N = fo;
    gw.K = B;
    gw.zout = m->g + m->woff[l];
    gw.ldz = fo;
    rkkt::mlp_gemm(rkkt::kMlpStore, gw, st);
    if (l == 0) break;
    // dZ_{l-1} = (dZ_l W_l^T) g'(Z_{l-1})
    rkkt::MlpGemm ga{};
    ga.A = m->dZb[c];
    ga.lda = mlp_pad8(fo);
    ga.B = m->wb + m->lay.wb_off[l];
    ga.ldb = m->lay.fo_p[l];
    ga.M = B;
    ga.N = fi;
    ga.K = fo;
    ga.zin = m->Z[l - 1];
    ga.ldz = fi;
    ga.hout = m->dZb[c ^ 1];
    ga.ldh = mlp_pad8(fi);
    ga.tout = m->dZT[c ^ 1];
    ga.ldt = m->bpit;
    rkkt::mlp_gemm(rkkt::kMlpGeluBack, ga, st);
    c ^= 1;
  }
  return check(m, "rkkt_mlp backward");
}

// ---- forward pass without the handle's workspace (rkkt_mlp_forward_static)
// The BF16 input and hidden activations of that call live in `scratch`, one
// copy per GPU for the life of the process.  In host code the array's name
// only stands for the device symbol: its device address comes from
// hipGetSymbolAddress, looked up once per device with that device current
// (by rkkt_mlp_create, else by the first call on the device) and kept in
// g_scratch_dev.
constexpr size_t kMlpStaticBytes = 8u << 20;
static __device__ __align__(256) unsigned char scratch[kMlpStaticBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// device address of `scratch` on the current device, or nullptr
void* scratch_address(std::string* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = std::string("no usable current device: ") + hipGetErrorString(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

inline size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// bytes of `scratch` that B rows need: A_l [B][pad8(sz[l])] BF16 for every
// layer input, each region 256-byte aligned
size_t static_bytes(const rkkt_mlp* m, long long B) {
  size_t n = 0;
  for (int l = 0; l < m->L; ++l) n += align256((size_t)B * mlp_pad8(m->sz[l]) * sizeof(uint16_t));
  return n;
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
  if (n_layers > rkkt::kMlpMaxLayers)
    return fail(nullptr, -1, "rkkt_mlp_create: more than " + std::to_string(rkkt::kMlpMaxLayers) + " layers");
  for (int l = 0; l <= n_layers; ++l)
    if (sizes[l] < 1) return fail(nullptr, -1, "rkkt_mlp_create: layer width < 1");
  *out = nullptr;
  rkkt_mlp* m = new rkkt_mlp();
  m->L = n_layers;
  m->bmax = batch_max;
  m->bpit = mlp_pad8(batch_max);
  m->sz.assign(sizes, sizes + n_layers + 1);
  int wmax = 0;
  long long nwb = 0, nwt = 0;
  m->lay.n = n_layers;
  for (int l = 0; l < n_layers; ++l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    m->woff.push_back(m->P);
    m->P += (long long)fi * fo;
    m->boff.push_back(m->P);
    m->P += fo;
    m->lay.woff[l] = m->woff[l];
    m->lay.fi[l] = fi;
    m->lay.fo[l] = fo;
    m->lay.fi_p[l] = mlp_pad8(fi);
    m->lay.fo_p[l] = mlp_pad8(fo);
    m->lay.wb_off[l] = nwb;
    m->lay.wt_off[l] = nwt;
    nwb += (long long)fi * m->lay.fo_p[l];
    nwt += (long long)fo * m->lay.fi_p[l];
  }
  for (int w : m->sz) wmax = std::max(wmax, w);
  hipError_t e = hipSuccess;
  m->A.assign(n_layers, nullptr);
  m->AT.assign(n_layers, nullptr);
  m->Z.assign(n_layers, nullptr);
  if (e == hipSuccess) e = dalloc(m, &m->p, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->m, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->v, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->g, m->P);
  if (e == hipSuccess) e = dalloc(m, &m->wb, nwb);
  if (e == hipSuccess) e = dalloc(m, &m->wt, nwt);
  for (int l = 0; l < n_layers && e == hipSuccess; ++l) {
    e = dalloc(m, &m->A[l], (long long)batch_max * mlp_pad8(m->sz[l]));
    if (e == hipSuccess) e = dalloc(m, &m->AT[l], (long long)(m->sz[l] + 1) * m->bpit);
    if (e == hipSuccess) e = dalloc(m, &m->Z[l], (long long)batch_max * m->sz[l + 1]);
  }
  for (int c = 0; c < 2 && e == hipSuccess; ++c) {
    e = dalloc(m, &m->dZb[c], (long long)batch_max * mlp_pad8(wmax));
    if (e == hipSuccess) e = dalloc(m, &m->dZT[c], (long long)wmax * m->bpit);
  }
  if (e == hipSuccess) e = dalloc(m, &m->lpart, rkkt::mlp_out_grad_tiles(batch_max, m->sz[n_layers]));
  if (e == hipSuccess) {
    for (int l = 0; l < n_layers; ++l)
      rkkt::mlp_fill_bf16(m->AT[l] + (long long)m->sz[l] * m->bpit, m->bpit, 1.0f, nullptr);
    e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (e == hipSuccess) {
    std::string msg;
    if (!scratch_address(&msg)) {
      rkkt_mlp_destroy(m);
      return fail(nullptr, -2, "rkkt_mlp_create: " + msg);
    }
  }
  if (e != hipSuccess) {
    std::string msg = std::string("rkkt_mlp_create: ") + hipGetErrorString(e);
    rkkt_mlp_destroy(m);
    return fail(nullptr, -6, msg);
  }
  *out = m;
  return 0;
}

int rkkt_mlp_destroy(rkkt_mlp* m) {
  if (!m) return 0;
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
  rkkt::mlp_param_copies(m->p, m->P, m->lay, m->wb, m->wt, st);
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
  return forward_impl(m, x, batch, y, false, st);
}

int rkkt_mlp_forward_static(const rkkt_mlp* mc, const float* x, int batch, float* y, hipStream_t st) {
  rkkt_mlp* m = const_cast<rkkt_mlp*>(mc);  // only its error string is written
  if (!m) return fail(nullptr, -1, "rkkt_mlp_forward_static: null handle");
  if (!x || !y) return fail(m, -1, "rkkt_mlp_forward_static: null array");
  if (batch < 1) return fail(m, -1, "rkkt_mlp_forward_static: batch < 1");
  const size_t need = static_bytes(m, batch);
  if (need > kMlpStaticBytes) {
    long long rows = 0;
    while (static_bytes(m, rows + 1) <= kMlpStaticBytes) ++rows;
    return fail(m, -1, "rkkt_mlp_forward_static: " + std::to_string(batch) + " rows need " +
                           std::to_string(need) + " bytes of the " + std::to_string(kMlpStaticBytes) +
                           "-byte static workspace (at most " + std::to_string(rows) +
                           " rows for this network)");
  }
  std::string msg;
  unsigned char* base = static_cast<unsigned char*>(scratch_address(&msg));
  if (!base) return fail(m, -2, "rkkt_mlp_forward_static: " + msg);
  (void)hipGetLastError();
  std::vector<uint16_t*> act(m->L);
  size_t off = 0;
  for (int l = 0; l < m->L; ++l) {
    act[l] = reinterpret_cast<uint16_t*>(base + off);
    off += align256((size_t)batch * mlp_pad8(m->sz[l]) * sizeof(uint16_t));
  }
  rkkt::mlp_input_bf16(x, batch, m->sz[0], act[0], mlp_pad8(m->sz[0]), nullptr, 0, st);
  for (int l = 0; l < m->L; ++l) {
    const int fi = m->sz[l], fo = m->sz[l + 1];
    const bool last = l + 1 == m->L;
    rkkt::MlpGemm g{};
    g.A = act[l];
    g.lda = mlp_pad8(fi);
    g.B = m->wt + m->lay.wt_off[l];
    g.ldb = m->lay.fi_p[l];
    g.M = batch;
    g.N = fo;
    g.K = fi;
    g.bias = m->p + m->boff[l];
    g.ldz = fo;
    if (!last) {
      g.hout = act[l + 1];
      g.ldh = mlp_pad8(fo);
    } else {
      g.y = y;
    }
    rkkt::mlp_gemm(last ? rkkt::kMlpBiasOut : rkkt::kMlpBiasGelu, g, st);
  }
  return check(m, "rkkt_mlp_forward_static");
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
  rkkt::mlp_adam(m->p, m->g, m->m, m->v, m->P, lr, m->t, m->lay, m->wb, m->wt, st);
  return check(m, "rkkt_mlp_train_step");
}

}  // extern "C"
