// Dense n_u x n_u stages: the global sum of the scenario contributions (the
// paper's MPI all-reduce of K_hat, here a fixed-order on-device sum), the
// Cholesky factorisation of K_hat (the paper factorises it densely with
// LAPACK on the GPU) and the two triangular solves for p_u.
#include "device.h"

namespace rkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kNB = 64;          // panel width of the blocked factorisation
constexpr int kSmallN = 140;     // whole matrix in LDS up to this order
constexpr int kWavesD = kThreads / 64;

__global__ void k_set_int(int* p, int v) { *p = v; }

// K_hat = sum_i part_i + diag(sigma_u) + delta_w I.  A workgroup owns 64
// entries; its 8 wavefronts each sum a contiguous eighth of the scenarios in
// index order and the eight partial sums are added in wavefront order, so the
// result does not depend on scheduling.
constexpr int kSumEntries = 64, kSumWaves = 8;

__global__ __launch_bounds__(kSumEntries * kSumWaves) void k_scenario_sum(DP d, const double* su,
                                                                           double dw, double* khat) {
  __shared__ double part[kSumWaves][kSumEntries];
  const long long nn = (long long)d.nu * d.nu;
  const int lane = threadIdx.x % kSumEntries, wv = threadIdx.x / kSumEntries;
  const long long t = (long long)blockIdx.x * kSumEntries + lane;
  const int per = (d.N + kSumWaves - 1) / kSumWaves;
  const int k0 = wv * per, k1 = min(d.N, k0 + per);
  double acc = 0.0;
  if (t < nn)
    for (int k = k0; k < k1; ++k) acc += d.part[(long long)k * nn + t];
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && t < nn) {
    double s = part[0][lane];
    for (int q = 1; q < kSumWaves; ++q) s += part[q][lane];
    const int r = (int)(t / d.nu), c = (int)(t % d.nu);
    if (r == c) s += su[r] + dw;
    if (!isfinite(s)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
    khat[t] = s;
  }
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

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Whole matrix in LDS (leading dimension n + 1), right-looking blocked
// Cholesky with 16-column panels: the diagonal block is factorised by one
// wavefront, the panel below by a triangular solve per row, and the trailing
// lower triangle is updated in 16 x 16 tiles on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; result register r of lane l is row l/16 + 4r,
// column l%16).
constexpr int kPB = 16;

__global__ __launch_bounds__(kThreads) void k_chol_small(double* A, int n, int* info) {
  extern __shared__ double sa[];
  __shared__ int sflag;
  const int ld = n + 1, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int t = tid; t < n * n; t += kThreads) {
    const int i = t / n, l = t % n;
    if (l <= i) sa[i * ld + l] = A[t];
  }
  if (tid == 0) sflag = 0;
  __syncthreads();
  for (int jb = 0; jb < n; jb += kPB) {
    const int nb = min(kPB, n - jb);
    if (wv == 0) {
      for (int j = jb; j < jb + nb; ++j) {
        const double p = sa[j * ld + j];
        if (!(p > 0.0) || !isfinite(p)) {
          if (lane == 0) sflag = j + 1;
          break;
        }
        const double sq = sqrt(p);
        wave_lds_sync();
        if (lane == 0) sa[j * ld + j] = sq;
        const int i = j + 1 + lane;
        if (i < jb + nb) sa[i * ld + j] /= sq;
        wave_lds_sync();
        const int m = jb + nb - j - 1;
        for (int idx = lane; idx < m * m; idx += 64) {
          const int ii = j + 1 + idx / m, ll = j + 1 + idx % m;
          if (ll <= ii) sa[ii * ld + ll] -= sa[ii * ld + j] * sa[ll * ld + j];
        }
        wave_lds_sync();
      }
    }
    __syncthreads();
    if (sflag) break;
    const int s0 = jb + nb, rest = n - s0;
    if (rest <= 0) break;
    for (int i = s0 + tid; i < n; i += kThreads) {
      double x[kPB];
      for (int p = 0; p < kPB; ++p) {
        double acc = sa[i * ld + jb + p];
        for (int q = 0; q < p; ++q) acc -= x[q] * sa[(jb + p) * ld + jb + q];
        x[p] = acc / sa[(jb + p) * ld + jb + p];
      }
      for (int p = 0; p < kPB; ++p) sa[i * ld + jb + p] = x[p];
    }
    __syncthreads();
    const int nt = (rest + 15) / 16;
    const int lm = lane & 15, lk = lane >> 4;
    int cnt = 0;
    for (int ti = 0; ti < nt; ++ti)
      for (int tl = 0; tl <= ti; ++tl, ++cnt) {
        if (cnt % kWavesD != wv) continue;
        const int i0 = s0 + 16 * ti, l0 = s0 + 16 * tl;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < kPB; k0 += 4) {
          const double a = i0 + lm < n ? sa[(i0 + lm) * ld + jb + k0 + lk] : 0.0;
          const double b = l0 + lm < n ? sa[(l0 + lm) * ld + jb + k0 + lk] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r, l = l0 + lm;
          if (i < n && l <= i) sa[i * ld + l] -= acc[r];
        }
      }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += kThreads) {
    const int i = t / n, l = t % n;
    if (l <= i) A[t] = sa[i * ld + l];
  }
  if (tid == 0) *info = sflag;
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
// Small orders: L copied into LDS, then one wavefront sweeps columns (lanes
// own rows; wavefront-scope ordering only).
__global__ __launch_bounds__(kThreads) void k_reduced_solve(DP d, const double* r1u, const double* L,
                                                            double* pu) {
  extern __shared__ double sm[];
  const int n = d.nu, ld = n + 1, tid = threadIdx.x, lane = tid & 63;
  double* sl = sm;
  double* y = sm + (size_t)n * ld;
  for (int t = tid; t < n * n; t += kThreads) {
    const int i = t / n, l = t % n;
    if (l <= i) sl[i * ld + l] = L[t];
  }
  for (int c = tid; c < n; c += kThreads) {
    double acc = -r1u[c];
    for (int k = 0; k < d.N; ++k) acc += d.rpart[(long long)k * n + c];
    y[c] = acc;
  }
  __syncthreads();
  if (tid >= 64) return;
  for (int j = 0; j < n; ++j) {
    const double yj = y[j] / sl[j * ld + j];
    wave_lds_sync();
    if (lane == 0) y[j] = yj;
    for (int i = j + 1 + lane; i < n; i += 64) y[i] -= sl[i * ld + j] * yj;
    wave_lds_sync();
  }
  for (int j = n - 1; j >= 0; --j) {
    const double yj = y[j] / sl[j * ld + j];
    wave_lds_sync();
    if (lane == 0) y[j] = yj;
    for (int i = lane; i < j; i += 64) y[i] -= sl[j * ld + i] * yj;
    wave_lds_sync();
  }
  for (int c = lane; c < n; c += 64) pu[c] = y[c];
}

// Large orders: one workgroup, 64-row blocks.  Forward: each block first
// subtracts L[block, :jb] y[:jb] (waves over rows, lanes over contiguous
// columns of a row), then one wavefront solves the 64 x 64 diagonal triangle.
// Backward (L^T): each block first subtracts sum_{i beyond} L[i, block] x_i
// (waves over rows i, lanes over the 64 contiguous columns of the block),
// then one wavefront solves the transposed triangle.
constexpr int kRB = 64, kRThreads = 1024, kRWaves = kRThreads / 64;

__global__ __launch_bounds__(kRThreads) void k_reduced_solve_blocked(DP d, const double* r1u,
                                                                     const double* L, double* pu) {
  extern __shared__ double y[];
  __shared__ double red[kRWaves][kRB];
  const int n = d.nu, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int c = tid; c < n; c += kRThreads) {
    double acc = -r1u[c];
    for (int k = 0; k < d.N; ++k) acc += d.rpart[(long long)k * n + c];
    y[c] = acc;
  }
  __syncthreads();
  for (int jb = 0; jb < n; jb += kRB) {
    const int nb = min(kRB, n - jb);
    // y[jb + r] -= L[jb + r, 0:jb] . y[0:jb]
    for (int r = wv; r < nb; r += kRWaves) {
      const double* row = L + (long long)(jb + r) * n;
      double acc = 0.0;
      for (int q = lane; q < jb; q += 64) acc += row[q] * y[q];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
      if (lane == 0) y[jb + r] -= acc;
    }
    __syncthreads();
    if (wv == 0) {
      for (int j = jb; j < jb + nb; ++j) {
        const double yj = y[j] / L[(long long)j * n + j];
        wave_lds_sync();
        if (lane == 0) y[j] = yj;
        const int i = j + 1 + lane;
        if (i < jb + nb) y[i] -= L[(long long)i * n + j] * yj;
        wave_lds_sync();
      }
    }
    __syncthreads();
  }
  for (int jb = ((n - 1) / kRB) * kRB; jb >= 0; jb -= kRB) {
    const int nb = min(kRB, n - jb);
    // y[jb + lane] -= sum_{i >= jb + nb} L[i, jb + lane] y[i]
    double acc = 0.0;
    if (lane < nb)
      for (int i = jb + nb + wv; i < n; i += kRWaves) acc += L[(long long)i * n + jb + lane] * y[i];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
      double s = 0.0;
      for (int q = 0; q < kRWaves; ++q) s += red[q][lane];
      if (lane < nb) y[jb + lane] -= s;
      wave_lds_sync();
      for (int j = jb + nb - 1; j >= jb; --j) {
        const double yj = y[j] / L[(long long)j * n + j];
        wave_lds_sync();
        if (lane == 0) y[j] = yj;
        const int i = jb + lane;
        if (i < j) y[i] -= L[(long long)j * n + i] * yj;
        wave_lds_sync();
      }
    }
    __syncthreads();
  }
  for (int c = tid; c < n; c += kRThreads) pu[c] = y[c];
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
  static int c1 = 0, c2 = 0, c3 = 0;
  hipError_t e = hipSuccess;
  if (d.nu <= kSmallN) {
    e = allow_lds((const void*)k_chol_small, &c1, 8 * d.nu * (d.nu + 1));
    if (e == hipSuccess) e = allow_lds((const void*)k_reduced_solve, &c2, 8 * (d.nu * (d.nu + 1) + d.nu));
  } else {
    e = allow_lds((const void*)k_reduced_solve_blocked, &c3, 8 * d.nu);
  }
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
  k_scenario_sum<<<(unsigned)((nn + kSumEntries - 1) / kSumEntries), kSumEntries * kSumWaves, 0, s>>>(
      d, su, dw, khat);
}

void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s) {
  const int n = d.nu;
  if (n <= kSmallN) {
    size_t lds = 8 * (size_t)n * (n + 1);
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
  if (d.nu <= kSmallN)
    k_reduced_solve<<<1, kThreads, 8 * ((size_t)d.nu * (d.nu + 1) + d.nu), s>>>(d, r1u, chol, pu);
  else
    k_reduced_solve_blocked<<<1, kRThreads, 8 * (size_t)d.nu, s>>>(d, r1u, chol, pu);
}

}  // namespace rkkt
