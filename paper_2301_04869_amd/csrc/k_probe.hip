// Machine-balance probes for the roofline: the rates that a plain device copy,
// independent FP64 multiply-add chains and independent FP64 matrix-core
// products reach on this device, measured beside the datasheet peaks.  They
// are measurement infrastructure; no stage of the hot path calls them.
#include <hip/hip_runtime.h>

#include "rkkt.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kProbeThreads = 256;

// dst = src in 16-byte units, grid-stride, eight loads in flight per thread,
// streaming (non-temporal) accesses
constexpr int kCopyUnroll = 8;
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const v2d* __restrict__ src,
                                                              v2d* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    v2d v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// eight independent chains x <- a x + b per thread; one sum per thread stored
constexpr int kChains = 8;
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma(double* out, int iters, double a, double b) {
  double x[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) x[j] = 1e-3 * threadIdx.x + j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = fma(x[j], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// four independent 16x16x4 FP64 matrix-core accumulations per wavefront
constexpr int kAcc = 4;
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(double* out, int iters) {
  v4d acc[kAcc];
#pragma unroll
  for (int j = 0; j < kAcc; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * (threadIdx.x & 63), b = 1.0 - 1e-6 * threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// best of `reps` timed launches after one untimed one, in ms
template <typename F>
hipError_t best_ms(hipStream_t st, int reps, F launch, float* best) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  *best = 0.0f;
  launch();
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
    launch();
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    if (r == 0 || ms < *best) *best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" int rkkt_probe_peaks(int device, double* hbm_gbs, double* fp64_vec_tfs, double* fp64_mfma_tfs) {
  if (!hbm_gbs || !fp64_vec_tfs || !fp64_mfma_tfs) return RKKT_ERR_ARG;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return RKKT_ERR_HIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    return RKKT_ERR_HIP;
  const long long n16 = 1LL << 26;                 // 16-byte units: 1 GiB per buffer
  const int blocks = 8 * cus, iters_fma = 4096, iters_mfma = 2048;
  const long long threads = (long long)blocks * kProbeThreads;
  v2d *src = nullptr, *dst = nullptr;
  double* out = nullptr;
  hipStream_t st = nullptr;
  float ms = 0.0f;
  int rc = RKKT_OK;
  if (hipMalloc(&src, n16 * sizeof(v2d)) != hipSuccess || hipMalloc(&dst, n16 * sizeof(v2d)) != hipSuccess ||
      hipMalloc(&out, threads * sizeof(double)) != hipSuccess) {
    rc = RKKT_ERR_NOMEM;
    goto done;
  }
  if (hipStreamCreate(&st) != hipSuccess || hipMemsetAsync(src, 0, n16 * sizeof(v2d), st) != hipSuccess) {
    rc = RKKT_ERR_HIP;
    goto done;
  }
  if (best_ms(st, 5, [&] { k_probe_copy<<<blocks * 4, kProbeThreads, 0, st>>>(src, dst, n16); }, &ms) !=
          hipSuccess || ms <= 0.0f) {
    rc = RKKT_ERR_HIP;
    goto done;
  }
  *hbm_gbs = 2.0 * 16.0 * (double)n16 / (ms * 1e-3) / 1e9;
  if (best_ms(st, 5, [&] { k_probe_fma<<<blocks, kProbeThreads, 0, st>>>(out, iters_fma, 0.999999, 1e-6); },
              &ms) != hipSuccess || ms <= 0.0f) {
    rc = RKKT_ERR_HIP;
    goto done;
  }
  *fp64_vec_tfs = 2.0 * kChains * (double)iters_fma * (double)threads / (ms * 1e-3) / 1e12;
  if (best_ms(st, 5, [&] { k_probe_mfma<<<blocks, kProbeThreads, 0, st>>>(out, iters_mfma); }, &ms) !=
          hipSuccess || ms <= 0.0f) {
    rc = RKKT_ERR_HIP;
    goto done;
  }
  // 2 * 16 * 16 * 4 flops per product, kAcc products per wavefront and step
  *fp64_mfma_tfs = 2048.0 * kAcc * (double)iters_mfma * (double)(threads / 64) / (ms * 1e-3) / 1e12;
done:
  if (st) (void)hipStreamSynchronize(st);
  if (st) (void)hipStreamDestroy(st);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  if (out) (void)hipFree(out);
  return rc;
}
