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

// blocked: trailing update A[i, l] -= sum_p A[i, p] A[l, p], lower tiles only
__global__ __launch_bounds__(kThreads) void k_chol_update(double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  const int nb = min(kNB, n - jb);
  const int s0 = jb + nb;
  const int ti = blockIdx.y, tl = blockIdx.x;
  if (tl > ti) return;
  const int i0 = s0 + ti * 64, l0 = s0 + tl * 64;
  __shared__ double sa[64][kNB + 1];
  __shared__ double sb[64][kNB + 1];
  for (int t = threadIdx.x; t < 64 * nb; t += blockDim.x) {
    const int r = t / nb, p = t % nb;
    sa[r][p] = (i0 + r < n) ? A[(long long)(i0 + r) * n + jb + p] : 0.0;
    sb[r][p] = (l0 + r < n) ? A[(long long)(l0 + r) * n + jb + p] : 0.0;
  }
  __syncthreads();
  // each thread: 4 x 4 outputs
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  for (int p = 0; p < nb; ++p) {
    double av[4], bv[4];
    for (int q = 0; q < 4; ++q) { av[q] = sa[tr + q][p]; bv[q] = sb[tc + q][p]; }
    for (int q = 0; q < 4; ++q)
      for (int w = 0; w < 4; ++w) acc[q][w] += av[q] * bv[w];
  }
  for (int q = 0; q < 4; ++q)
    for (int w = 0; w < 4; ++w) {
      const int i = i0 + tr + q, l = l0 + tc + w;
      if (i < n && l < n && l <= i) A[(long long)i * n + l] -= acc[q][w];
    }
}

// p_u = K_hat^-1 rhs with rhs = -r1u + sum_i rpart_i (fixed scenario order)
__global__ __launch_bounds__(1024) void k_reduced_solve(DP d, const double* r1u, const double* L,
                                                        double* pu) {
  extern __shared__ double y[];
  const int n = d.nu;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double acc = -r1u[c];
    for (int k = 0; k < d.N; ++k) acc += d.rpart[(long long)k * n + c];
    y[c] = acc;
  }
  __syncthreads();
  // L y = rhs
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) y[j] /= L[(long long)j * n + j];
    __syncthreads();
    const double yj = y[j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) y[i] -= L[(long long)i * n + j] * yj;
    __syncthreads();
  }
  // L^T p = y
  for (int j = n - 1; j >= 0; --j) {
    if (threadIdx.x == 0) y[j] /= L[(long long)j * n + j];
    __syncthreads();
    const double yj = y[j];
    for (int i = threadIdx.x; i < j; i += blockDim.x) y[i] -= L[(long long)j * n + i] * yj;
    __syncthreads();
  }
  for (int c = threadIdx.x; c < n; c += blockDim.x) pu[c] = y[c];
}

}  // namespace

void configure_dense_kernels() {
  const int lds = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)k_chol_small, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_reduced_solve, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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
  k_reduced_solve<<<1, 1024, lds, s>>>(d, r1u, chol, pu);
}

}  // namespace rkkt
