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

// K_hat = sum_c src_c + diag(sigma_u) + delta_w I over `cnt` n_u x n_u
// matrices (the scenario contributions, or the chunk partials of the stacked
// product), lower triangle, mirrored into the upper one so K_hat is exactly
// symmetric.  A workgroup owns 64 entries of the lower triangle (row-major
// order); its 8 wavefronts each sum a contiguous eighth of the matrices in
// index order and the eight partial sums are added in wavefront order, so the
// result does not depend on scheduling.
constexpr int kSumEntries = 64, kSumWaves = 8;

__global__ __launch_bounds__(kSumEntries * kSumWaves) void k_sym_sum(DP d, const double* src, int cnt,
                                                                      const double* su, double dw,
                                                                      double* khat) {
  __shared__ double part[kSumWaves][kSumEntries];
  const int n = d.nu;
  const long long nn = (long long)n * n, ntri = (long long)n * (n + 1) / 2;
  const int lane = threadIdx.x % kSumEntries, wv = threadIdx.x / kSumEntries;
  const long long t = (long long)blockIdx.x * kSumEntries + lane;
  // t -> (r, c), c <= r, rows in order
  int r = 0, c = 0;
  if (t < ntri) {
    r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)r * (r + 1) / 2 > t) --r;
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    c = (int)(t - (long long)r * (r + 1) / 2);
  }
  const long long off = (long long)r * n + c;
  const int per = (cnt + kSumWaves - 1) / kSumWaves;
  const int k0 = wv * per, k1 = min(cnt, k0 + per);
  double acc = 0.0;
  if (t < ntri)
    for (int k = k0; k < k1; ++k) acc += src[(long long)k * nn + off];
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && t < ntri) {
    double s = part[0][lane];
    for (int q = 1; q < kSumWaves; ++q) s += part[q][lane];
    if (r == c) s += su[r] + dw;
    if (!isfinite(s)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
    khat[off] = s;
    khat[(long long)c * n + r] = s;
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Stacked product of the reduction's product variant: for chunk c of the
// stacked rows rho (all scenarios, x rows then u rows of each),
//   gpart_c[i][j] = sum_rho Z[rho][i] (K Z)[rho][j],   i >= j,
// so that sum_c gpart_c = sum_k Z_k^T K_k Z_k.  One workgroup per (32 x 32
// lower output tile, chunk); its 4 wavefronts take interleaved 4-row slices
// of the chunk and each accumulates the whole tile as 2 x 2 blocks of
// v_mfma_f64_16x16x4f64 (A operand: lane holds Z[rho + lane/16][i + lane%16];
// B operand: (K Z)[rho + lane/16][j + lane%16]; result register r of a lane:
// row lane/16 + 4 r, column lane%16); the four tiles are added in wavefront
// order.
__global__ __launch_bounds__(256) void k_stacked_product(DP d) {
  int t = blockIdx.x, ti = 0;
  while (t > ti) { t -= ti + 1; ++ti; }
  const int tj = t, chunk = blockIdx.y;
  const long long rows = (long long)d.N * d.nz;
  const long long per = ((rows + d.nchunk - 1) / d.nchunk + 15) / 16 * 16;
  const long long r0 = (long long)chunk * per, r1 = min(rows, r0 + per);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lm = lane & 15, lk = lane >> 4;
  const int i0 = ti * 32, j0 = tj * 32;
  const long long ld = d.nu_pad;
  const double* Z = d.Zst;
  const double* KZ = d.KZst;
  v4d acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  // kU 4-row slices per wavefront in flight: all their operand loads are
  // issued before the first of their matrix-core products
  constexpr int kU = 4;
  for (long long r = r0 + 4 * wv; r < r1; r += 16 * kU) {
    double a0[kU], a1[kU], b0[kU], b1[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long rr = r + 16 * u + lk;
      const bool ok = rr < r1;
      a0[u] = ok ? Z[rr * ld + i0 + lm] : 0.0;
      a1[u] = ok ? Z[rr * ld + i0 + 16 + lm] : 0.0;
      b0[u] = ok ? KZ[rr * ld + j0 + lm] : 0.0;
      b1[u] = ok ? KZ[rr * ld + j0 + 16 + lm] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b0[u], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[u], b1[u], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b0[u], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[u], b1[u], acc[1][1], 0, 0, 0);
    }
  }
  __shared__ double red[4][32][33];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) red[wv][16 * a + lk + 4 * r][16 * b + lm] = acc[a][b][r];
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int i = e >> 5, j = e & 31;
    const double s = ((red[0][i][j] + red[1][i][j]) + red[2][i][j]) + red[3][i][j];
    const int gi = i0 + i, gj = j0 + j;
    if (gi < d.nu && gj <= gi) d.gpart[((long long)chunk * d.nu + gi) * d.nu + gj] = s;
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// 1/sqrt(d) for d > 0: the hardware reciprocal square root estimate refined by
// two Newton-Raphson steps r <- r (3 - d r^2) / 2 (quadratic convergence from
// the estimate's accuracy to double precision).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  double e = fma(-d * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  e = fma(-d * r, r, 1.0);
  return fma(0.5 * r, e, r);
}

// 1/d: the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r (2 - d r).
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Right-looking blocked Cholesky of the lower triangle of an n x n block held
// in LDS (row-major, leading dimension ld), n <= 64 kR, by a workgroup of
// 64 kWaves threads.  Panels of kPB columns: wavefront 0 factorises the panel
// in registers (lane l holds rows jb + l + 64 t; the diagonal row jb + p is
// in lane p, so its entries are broadcast with readlane and no
// synchronisation is needed inside the panel).  Inside the panel the
// elimination runs in the square-root-free form A = W D^-1 W^T (column p of W
// is the updated column p of A, D its diagonal), so the dependency chain from
// one column to the next holds one reciprocal; the panel's columns are then
// scaled to L = W D^-1/2 together.  The trailing lower triangle is updated in
// 16 x 16 tiles on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A operand
// lane holds row lane%16, k = lane/16; B operand k = lane/16, column lane%16;
// result register r of a lane is row lane/16 + 4 r, column lane%16).
// Returns 0 or the 1-based first column whose pivot is not positive.
constexpr int kPB = 16;

template <int kWaves, int kR>
__device__ int chol_blocked_lds(double* sa, int n, int ld, int* sflag) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) *sflag = 0;
  __syncthreads();
  for (int jb = 0; jb < n; jb += kPB) {
    const int nb = min(kPB, n - jb);
    if (wv == 0) {
      double x[kR][kPB];
#pragma unroll
      for (int t = 0; t < kR; ++t) {
        const int r = jb + lane + 64 * t;
#pragma unroll
        for (int p = 0; p < kPB; ++p) x[t][p] = (r < n && p < nb) ? sa[r * ld + jb + p] : 0.0;
      }
      int bad = 0;
      double dpiv[kPB];
#pragma unroll
      for (int p = 0; p < kPB; ++p) {
        dpiv[p] = 1.0;
        if (p < nb && !bad) {
          const double dv = readlane_d(x[0][p], p);
          if (!(dv > 0.0) || !isfinite(dv)) {
            bad = jb + p + 1;
          } else {
            dpiv[p] = dv;
            const double inv = rcp_nr(dv);
#pragma unroll
            for (int q = p + 1; q < kPB; ++q) {
              if (q < nb) {
                const double lq = readlane_d(x[0][p], q) * inv;  // w_qp / d_p
#pragma unroll
                for (int t = 0; t < kR; ++t) x[t][q] = fma(-x[t][p], lq, x[t][q]);
              }
            }
          }
        }
      }
      if (bad) {
        if (lane == 0) *sflag = bad;
      } else {
        // L = W D^-1/2 for the whole panel (independent chains)
#pragma unroll
        for (int p = 0; p < kPB; ++p) {
          const double rs = rsqrt_nr(dpiv[p]);
#pragma unroll
          for (int t = 0; t < kR; ++t) {
            const int r = jb + lane + 64 * t;
            if (r < n && p < nb && jb + p <= r) sa[r * ld + jb + p] = r == jb + p ? dpiv[p] * rs : x[t][p] * rs;
          }
        }
      }
    }
    __syncthreads();
    if (*sflag) return *sflag;
    const int s0 = jb + nb, rest = n - s0;
    if (rest <= 0) break;
    const int nt = (rest + 15) / 16;
    const int lm = lane & 15, lk = lane >> 4;
    int cnt = 0;
    for (int ti = 0; ti < nt; ++ti)
      for (int tl = 0; tl <= ti; ++tl, ++cnt) {
        if (cnt % kWaves != wv) continue;
        const int i0 = s0 + 16 * ti, l0 = s0 + 16 * tl;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < kPB; k0 += 4) {
          const double a = i0 + lm < n ? sa[(i0 + lm) * ld + jb + k0 + lk] : 0.0;
          const double b = l0 + lm < n ? sa[(l0 + lm) * ld + jb + k0 + lk] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + lk + 4 * r, l = l0 + lm;
          if (i < n && l <= i) sa[i * ld + l] -= acc[r];
        }
      }
    __syncthreads();
  }
  return 0;
}

// whole matrix in LDS (leading dimension n + 1); kR = rows per lane of the
// panel factorisation (n <= 64 kR)
constexpr int kCholSmallThreads = 512;

template <int kR>
__global__ __launch_bounds__(kCholSmallThreads) void k_chol_small(const double* src, double* A,
                                                                   int n, int* info) {
  extern __shared__ double sa[];
  __shared__ int sflag;
  const int ld = n + 1, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  copy2d_overlapped(sa, ld, src, n, n, n, threadIdx.x, kCholSmallThreads);
  __syncthreads();
  const int r = chol_blocked_lds<kCholSmallThreads / 64, kR>(sa, n, ld, &sflag);
  for (int i = wv; i < n; i += kCholSmallThreads / 64)
    for (int l = lane; l <= i; l += 64) A[(long long)i * n + l] = sa[i * ld + l];
  if (threadIdx.x == 0) *info = r;
}

// blocked: factor the 64 x 64 diagonal block at jb
__global__ __launch_bounds__(kThreads) void k_chol_diag(double* A, int n, int jb, int* info) {
  if (*info != 0) return;
  __shared__ double sa[kNB * (kNB + 1)];
  __shared__ int sflag;
  const int nb = min(kNB, n - jb), ld = kNB + 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  copy2d_overlapped(sa, ld, A + (long long)jb * n + jb, n, nb, nb, threadIdx.x, kThreads);
  __syncthreads();
  const int r = chol_blocked_lds<kWavesD, 1>(sa, nb, ld, &sflag);
  for (int i = wv; i < nb; i += kWavesD)
    for (int l = lane; l <= i; l += 64) A[(long long)(jb + i) * n + jb + l] = sa[i * ld + l];
  if (threadIdx.x == 0 && r) *info = jb + r;
}

// blocked: A[i, jb:jb+nb] <- A[i, jb:jb+nb] L_jj^-T for rows below the block.
// A wavefront takes one row at a time with lane q holding column q; lane q
// keeps row q of L_jj in registers, so the forward substitution is 64
// readlane broadcasts and fused multiply-adds with no memory traffic.
constexpr int kTrsmRowsPerWave = 4;

__global__ __launch_bounds__(kThreads) void k_chol_trsm(double* A, int n, int jb, const int* info) {
  if (*info != 0) return;
  __shared__ double sinv[kNB];
  const int nb = min(kNB, n - jb);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double lrow[kNB];
#pragma unroll
  for (int p = 0; p < kNB; ++p)
    lrow[p] = (lane < nb && p <= lane) ? A[(long long)(jb + lane) * n + jb + p] : 0.0;
  if (threadIdx.x < kNB)
    sinv[threadIdx.x] = threadIdx.x < nb ? 1.0 / A[(long long)(jb + threadIdx.x) * n + jb + threadIdx.x] : 0.0;
  __syncthreads();
  const int rows = n - jb - nb;
  for (int r = blockIdx.x * kWavesD + wv; r < rows; r += gridDim.x * kWavesD) {
    double* row = A + (long long)(jb + nb + r) * n + jb;
    double v = lane < nb ? row[lane] : 0.0;
#pragma unroll
    for (int p = 0; p < kNB; ++p) {
      if (p < nb) {
        const double xp = readlane_d(v, p) * sinv[p];
        if (lane == p) v = xp;
        else if (lane > p) v = fma(-xp, lrow[p], v);
      }
    }
    if (lane < nb) row[lane] = v;
  }
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

// p_u = K_hat^-1 rhs with rhs = -r1u + sum_i rpart_i, from the Cholesky
// factor L (lower triangle of `L`, row-major).  One workgroup of kRThreads
// (16 wavefronts).  The right-hand side is summed over scenarios in a fixed
// order (wavefront w takes a contiguous 1/16 of the scenarios, partial sums
// added in wavefront order).  Both triangular solves go by blocks of 16 rows:
// the off-diagonal part is a matrix-vector product (one wavefront per row of
// the block for L, per column for L^T, lanes over the long dimension, then a
// shuffle reduction), and the 16 x 16 diagonal triangle is solved by one
// wavefront in registers (lane r holds unknown r; readlane broadcasts).
// kLDS: L staged in LDS (leading dimension n + 1); else read from global.
constexpr int kRB = 16, kRThreads = 1024, kRWaves = kRThreads / 64;

// the reduced solve stages L in LDS when it fits next to its reduction buffer
__host__ __device__ inline bool rsolve_lds(int n) {
  return 8LL * ((long long)n * (n + 1) + n) + 8LL * kRWaves * 64 <= 160 * 1024;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <bool kLDS>
__global__ __launch_bounds__(kRThreads) void k_reduced_solve(DP d, const double* r1u, const double* Lg,
                                                             double* pu) {
  extern __shared__ double sm[];
  __shared__ double red[kRWaves][64];
  const int n = d.nu, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ld = kLDS ? n + 1 : n;
  double* y = sm;
  const double* L = Lg;
  if (kLDS) {
    double* sl = sm + n;
    copy2d_overlapped(sl, ld, Lg, n, n, n, tid, kRThreads);
    L = sl;
  }
  // right-hand side
  const int per = (d.N + kRWaves - 1) / kRWaves;
  const int k0 = wv * per, k1 = min(d.N, k0 + per);
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = c0 + lane;
    double acc = 0.0;
    if (c < n)
      for (int k = k0; k < k1; ++k) acc += d.rpart[(long long)k * n + c];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && c < n) {
      double sum = -r1u[c];
      for (int q = 0; q < kRWaves; ++q) sum += red[q][lane];
      y[c] = sum;
    }
    __syncthreads();
  }
  // forward: L y = b
  for (int jb = 0; jb < n; jb += kRB) {
    const int nb = min(kRB, n - jb);
    if (wv < nb) {
      const double* row = L + (long long)(jb + wv) * ld;
      double acc = 0.0;
      for (int q = lane; q < jb; q += 64) acc = fma(row[q], y[q], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[jb + wv] -= acc;
    }
    __syncthreads();
    if (wv == 0) {
      const int r = lane;
      double lrow[kRB];
#pragma unroll
      for (int p = 0; p < kRB; ++p) lrow[p] = (r < nb && p <= r) ? L[(long long)(jb + r) * ld + jb + p] : 0.0;
      const double myinv = r < nb ? rcp_nr(L[(long long)(jb + r) * ld + jb + r]) : 0.0;  // 1/L_rr
      double v = r < nb ? y[jb + r] : 0.0;
#pragma unroll
      for (int p = 0; p < kRB; ++p) {
        if (p < nb) {
          const double vp = readlane_d(v, p) * readlane_d(myinv, p);
          if (r == p) v = vp;
          else if (r > p) v = fma(-lrow[p], vp, v);
        }
      }
      if (r < nb) y[jb + r] = v;
    }
    __syncthreads();
  }
  // backward: L^T x = y
  for (int jb = ((n - 1) / kRB) * kRB; jb >= 0; jb -= kRB) {
    const int nb = min(kRB, n - jb);
    if (wv < nb) {
      double acc = 0.0;
      for (int i = jb + nb + lane; i < n; i += 64) acc = fma(L[(long long)i * ld + jb + wv], y[i], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[jb + wv] -= acc;
    }
    __syncthreads();
    if (wv == 0) {
      const int r = lane;
      // lane r holds column r of the diagonal block: L[jb + p][jb + r], p >= r
      double lcol[kRB];
#pragma unroll
      for (int p = 0; p < kRB; ++p) lcol[p] = (r < nb && p < nb && p >= r) ? L[(long long)(jb + p) * ld + jb + r] : 0.0;
      const double myinv = r < nb ? rcp_nr(L[(long long)(jb + r) * ld + jb + r]) : 0.0;
      double v = r < nb ? y[jb + r] : 0.0;
#pragma unroll
      for (int p = kRB - 1; p >= 0; --p) {
        if (p < nb) {
          const double vp = readlane_d(v, p) * readlane_d(myinv, p);
          if (r == p) v = vp;
          else if (r < p) v = fma(-lcol[p], vp, v);
        }
      }
      if (r < nb) y[jb + r] = v;
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
  static int c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
  hipError_t e = hipSuccess;
  if (d.nu <= kSmallN) {
    const void* f = d.nu <= 64 ? (const void*)k_chol_small<1>
                    : d.nu <= 128 ? (const void*)k_chol_small<2> : (const void*)k_chol_small<3>;
    int* cur = d.nu <= 64 ? &c1 : d.nu <= 128 ? &c4 : &c5;
    e = allow_lds(f, cur, 8 * d.nu * (d.nu + 1));
  }
  if (e == hipSuccess) {
    if (rsolve_lds(d.nu))
      e = allow_lds((const void*)k_reduced_solve<true>, &c2, 8 * (d.nu * (d.nu + 1) + d.nu));
    else
      e = allow_lds((const void*)k_reduced_solve<false>, &c3, 8 * d.nu);
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
  const long long ntri = (long long)d.nu * (d.nu + 1) / 2;
  const unsigned grid = (unsigned)((ntri + kSumEntries - 1) / kSumEntries);
  if (d.variant == 2)
    k_sym_sum<<<grid, kSumEntries * kSumWaves, 0, s>>>(d, d.gpart, d.nchunk, su, dw, khat);
  else
    k_sym_sum<<<grid, kSumEntries * kSumWaves, 0, s>>>(d, d.part, d.N, su, dw, khat);
}

void launch_stacked_product(const DP& d, hipStream_t s) {
  const int T = d.nu_pad / 32;
  k_stacked_product<<<dim3(T * (T + 1) / 2, d.nchunk), 256, 0, s>>>(d);
}

void launch_cholesky_from(const DP& d, const double* src, double* a, int* info, hipStream_t s) {
  const int n = d.nu;
  if (n <= kSmallN) {
    size_t lds = 8 * (size_t)n * (n + 1);
    if (n <= 64) k_chol_small<1><<<1, kCholSmallThreads, lds, s>>>(src, a, n, info);
    else if (n <= 128) k_chol_small<2><<<1, kCholSmallThreads, lds, s>>>(src, a, n, info);
    else k_chol_small<3><<<1, kCholSmallThreads, lds, s>>>(src, a, n, info);
    return;
  }
  if (src != a) launch_copy(src, a, (long long)n * n, s);
  k_set_int<<<1, 1, 0, s>>>(info, 0);
  for (int jb = 0; jb < n; jb += kNB) {
    k_chol_diag<<<1, kThreads, 0, s>>>(a, n, jb, info);
    const int nb = n - jb < kNB ? n - jb : kNB;
    const int rest = n - jb - nb;
    if (rest <= 0) break;
    k_chol_trsm<<<(rest + kWavesD * kTrsmRowsPerWave - 1) / (kWavesD * kTrsmRowsPerWave), kThreads, 0, s>>>(
        a, n, jb, info);
    const int nt = (rest + 63) / 64;
    k_chol_update<<<dim3(nt, nt), kThreads, 0, s>>>(a, n, jb, info);
  }
}

void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s) {
  launch_cholesky_from(d, a, a, info, s);
}

void launch_reduced_solve(const DP& d, const double* r1u, const double* chol, double* pu,
                          hipStream_t s) {
  if (rsolve_lds(d.nu))
    k_reduced_solve<true><<<1, kRThreads, 8 * ((size_t)d.nu * (d.nu + 1) + d.nu), s>>>(d, r1u, chol, pu);
  else
    k_reduced_solve<false><<<1, kRThreads, 8 * (size_t)d.nu, s>>>(d, r1u, chol, pu);
}

}  // namespace rkkt
