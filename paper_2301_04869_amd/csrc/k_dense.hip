// Dense n_u x n_u stages: the global sum of the scenario contributions (the
// paper's MPI all-reduce of K_hat, here a fixed-order on-device sum), the
// Cholesky factorisation of K_hat (the paper factorises it densely with
// LAPACK on the GPU) and the two triangular solves for p_u.
#include "device.h"

namespace rkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kNB = 64;          // panel width of the blocked factorisation
constexpr int kSmallN = 120;     // whole matrix in LDS up to this order

__global__ void k_set_int(int* p, int v) { *p = v; }

// K_hat = sum_i part_i + diag(sigma_u) + delta_w I, scenarios summed in index order
__global__ void k_scenario_sum(DP d, const double* su, double dw, double* khat) {
  const long long nn = (long long)d.nu * d.nu;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn) return;
  double acc = 0.0;
  for (int k = 0; k < d.N; ++k) acc += d.part[(long long)k * nn + t];
  const int r = (int)(t / d.nu), c = (int)(t % d.nu);
  if (r == c) acc += su[r] + dw;
  if (!isfinite(acc)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
  khat[t] = acc;
}

// Unblocked right-looking Cholesky of an n x n block held in LDS (row-major,
// leading dimension ld).  Returns 0 or the 1-based failing column.
__device__ int chol_lds(double* a, int n, int ld, int* sflag) {
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double p = a[j * ld + j];
      if (!(p > 0.0) || !isfinite(p)) *sflag = j + 1;
      else a[j * ld + j] = sqrt(p);
    }
    __syncthreads();
    if (*sflag) return *sflag;
    const double dj = a[j * ld + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) a[i * ld + j] /= dj;
    __syncthreads();
    const int m = n - j - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = j + 1 + idx / m, l = j + 1 + idx % m;
      if (l <= i) a[i * ld + l] -= a[i * ld + j] * a[l * ld + j];
    }
    __syncthreads();
  }
  return 0;
}

__global__ __launch_bounds__(kThreads) void k_chol_small(double* A, int n, int* info) {
  extern __shared__ double sa[];
  __shared__ int sflag;
  if (threadIdx.x == 0) sflag = 0;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) sa[t] = A[t];
  __syncthreads();
  const int r = chol_lds(sa, n, n, &sflag);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, l = t % n;
    if (l <= i) A[t] = sa[t];
  }
  if (threadIdx.x == 0) *info = r;
}

// blocked: factor the diagonal block at jb
__global__ __launch_bounds__(kThreads) void k_chol_diag(double* A, int n, int jb, int* info) {
  if (*info != 0) return;
  __shared__ double sa[kNB * kNB];
  __shared__ int sflag;
  const int nb = min(kNB, n - jb);
  if (threadIdx.x == 0) sflag = 0;
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x)
    sa[t] = A[(long long)(jb + t / nb) * n + jb + t % nb];
  __syncthreads();
  const int r = chol_lds(sa, nb, nb, &sflag);
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    const int i = t / nb, l = t % nb;
    if (l <= i) A[(long long)(jb + i) * n + jb + l] = sa[t];
  }
  if (threadIdx.x == 0 && r) *info = jb + r;
}

// blocked: A[i, jb:jb+nb] <- A[i, jb:jb+nb] L_jj^-T for rows below the block
__global__ __launch_bounds__(kThreads) void k_chol_trsm(double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  __shared__ double sl[kNB * kNB];
  const int nb = min(kNB, n - jb);
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x)
    sl[t] = A[(long long)(jb + t / nb) * n + jb + t % nb];
  __syncthreads();
  const int i = jb + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* row = A + (long long)i * n + jb;
  double x[kNB];
  for (int p = 0; p < nb; ++p) {
    double acc = row[p];
    for (int q = 0; q < p; ++q) acc -= x[q] * sl[p * nb + q];
    x[p] = acc / sl[p * nb + p];
  }
  for (int p = 0; p < nb; ++p) row[p] = x[p];
}

// blocked: trailing update A[i, l] -= sum_p A[i, p] A[l, p] over the lower
// 64 x 64 tiles, on the FP64 matrix cores.  Each of the 4 waves owns a 32 x 32
// quarter as 2 x 2 blocks of v_mfma_f64_16x16x4f64 (A operand: lane holds
// row lane%16, k = lane/16; B operand: k = lane/16, column lane%16; result
// register r of a lane: row lane/16 + 4 r, column lane%16).
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_chol_update(double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  const int nb = min(kNB, n - jb);
  const int s0 = jb + nb;
  const int ti = blockIdx.y, tl = blockIdx.x;
  if (tl > ti) return;
  const int i0 = s0 + ti * 64, l0 = s0 + tl * 64;
  __shared__ double sa[64][kNB + 1];
  __shared__ double sb[64][kNB + 1];
  for (int t = threadIdx.x; t < 64 * kNB; t += blockDim.x) {
    const int r = t / kNB, p = t % kNB;
    const bool kin = p < nb;
    sa[r][p] = (kin && i0 + r < n) ? A[(long long)(i0 + r) * n + jb + p] : 0.0;
    sb[r][p] = (kin && l0 + r < n) ? A[(long long)(l0 + r) * n + jb + p] : 0.0;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;   // wave's quarter
  const int lm = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kNB; k0 += 4) {
    const double a0 = sa[rb + lm][k0 + lk], a1 = sa[rb + 16 + lm][k0 + lk];
    const double b0 = sb[cb + lm][k0 + lk], b1 = sb[cb + 16 + lm][k0 + lk];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + rb + 16 * a + lk + 4 * r, l = l0 + cb + 16 * b + lm;
        if (i < n && l <= i) A[(long long)i * n + l] -= acc[a][b][r];
      }
}

// p_u = K_hat^-1 rhs with rhs = -r1u + sum_i rpart_i (fixed scenario order).
// One wavefront: lanes own rows, the forward and backward column sweeps need
// only wavefront-scope ordering of LDS accesses (no workgroup barriers).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64) void k_reduced_solve(DP d, const double* r1u, const double* L,
                                                      double* pu) {
  extern __shared__ double y[];
  const int n = d.nu, lane = threadIdx.x;
  for (int c = lane; c < n; c += 64) {
    double acc = -r1u[c];
    for (int k = 0; k < d.N; ++k) acc += d.rpart[(long long)k * n + c];
    y[c] = acc;
  }
  wave_lds_sync();
  // L y = rhs (column sweep)
  for (int j = 0; j < n; ++j) {
    const double yj = y[j] / L[(long long)j * n + j];
    wave_lds_sync();
    if (lane == 0) y[j] = yj;
    for (int i = j + 1 + lane; i < n; i += 64) y[i] -= L[(long long)i * n + j] * yj;
    wave_lds_sync();
  }
  // L^T p = y (column sweep of L^T = row sweep of L)
  for (int j = n - 1; j >= 0; --j) {
    const double yj = y[j] / L[(long long)j * n + j];
    wave_lds_sync();
    if (lane == 0) y[j] = yj;
    for (int i = lane; i < j; i += 64) y[i] -= L[(long long)j * n + i] * yj;
    wave_lds_sync();
  }
  for (int c = lane; c < n; c += 64) pu[c] = y[c];
}

}  // namespace

// raise the dynamic LDS limit of a kernel to what this problem needs (never lowered)
static hipError_t allow_lds(const void* fn, int* cur, int need) {
  if (need <= *cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, need);
  if (e == hipSuccess) *cur = need;
  return e;
}

hipError_t configure_dense_kernels(const DP& d) {
  static int c1 = 0, c2 = 0;
  hipError_t e = hipSuccess;
  if (d.nu <= kSmallN) e = allow_lds((const void*)k_chol_small, &c1, 8 * d.nu * d.nu);
  if (e == hipSuccess) e = allow_lds((const void*)k_reduced_solve, &c2, 8 * d.nu);
  return e;
}

__global__ void k_copy(const double* a, double* b, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = a[t];
}

void launch_copy(const double* a, double* b, long long n, hipStream_t s) {
  k_copy<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(a, b, n);
}

void launch_scenario_sum(const DP& d, const double* su, double dw, double* khat, hipStream_t s) {
  const long long nn = (long long)d.nu * d.nu;
  k_scenario_sum<<<(unsigned)((nn + kThreads - 1) / kThreads), kThreads, 0, s>>>(d, su, dw, khat);
}

void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s) {
  const int n = d.nu;
  if (n <= kSmallN) {
    size_t lds = 8 * (size_t)n * n;
    k_chol_small<<<1, kThreads, lds, s>>>(a, n, info);
    return;
  }
  k_set_int<<<1, 1, 0, s>>>(info, 0);
  for (int jb = 0; jb < n; jb += kNB) {
    k_chol_diag<<<1, kThreads, 0, s>>>(a, n, jb, info);
    const int nb = n - jb < kNB ? n - jb : kNB;
    const int rest = n - jb - nb;
    if (rest <= 0) break;
    k_chol_trsm<<<(rest + kThreads - 1) / kThreads, kThreads, 0, s>>>(a, n, jb, info);
    const int nt = (rest + 63) / 64;
    k_chol_update<<<dim3(nt, nt), kThreads, 0, s>>>(a, n, jb, info);
  }
}

void launch_reduced_solve(const DP& d, const double* r1u, const double* chol, double* pu,
                          hipStream_t s) {
  size_t lds = 8 * (size_t)d.nu;
  k_reduced_solve<<<1, 64, lds, s>>>(d, r1u, chol, pu);
}

}  // namespace rkkt
