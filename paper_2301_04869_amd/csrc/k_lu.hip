// Batched sparse LU refactorisation of G_x and the local reduction (paper,
// parallel KKT solver section: the scenario blocks of G_x share one pattern,
// so their LU factorisations can be batched; the reduced matrix is formed by
// the three-step product K_hat V over column batches of the identity).
//
// G_x of every scenario is refactorised on one filled pattern with a fixed
// symmetric fill-reducing permutation and static diagonal pivots.  Rows are
// processed by an up-looking (row-by-row) elimination in level-schedule order:
// rows of one level depend only on rows of earlier levels, so a level's rows
// run concurrently (one wavefront per row, lanes over the row updates).
//
// The reduction of one scenario and one tile of W columns of V = I runs in one
// workgroup: the right-hand-side panel -G_u[:, tile] is solved with L and U
// (T = -G_x^-1 G_u, step 1), multiplied by K (L_x = K_xx T + K_xu, step 2),
// solved with U^T and L^T and reduced with G_u^T (step 3,
// K_hat V = L_u - G_u^T G_x^-T L_x).  Every level of every triangular solve
// is one barrier-separated sweep with lanes over (row in level, column).
#include "device.h"

namespace rkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline void raise_status(const DP& d, int code, int k) {
  if (atomicCAS(d.status, 0, code) == 0) d.status[1] = k;
}

// ------------------------------------------------------------ refactorisation
template <bool kLDS>
__global__ __launch_bounds__(kThreads) void k_refactor(DP d) {
  const int k = blockIdx.x;
  const int nx = d.nx;
  extern __shared__ double smem[];
  double *lu, *invd, *rmax;
  int* map;
  if (kLDS) {
    lu = smem;
    invd = lu + d.nnz_f;
    rmax = invd + nx;
    map = reinterpret_cast<int*>(rmax + nx);
  } else {
    lu = d.LU + (long long)k * d.nnz_f;
    invd = d.invd + (long long)k * nx;
    rmax = d.rhat1 + (long long)k * nx;
    map = d.imap + (long long)k * kWaves * nx;
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* gv = d.EV + (long long)k * d.n_ev + d.off_gx;
  for (int e = tid; e < d.nnz_f; e += kThreads) lu[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < d.nnz_gx; e += kThreads) lu[d.gx2f[e]] = gv[e];
  for (int i = tid; i < nx; i += kThreads) {
    double mx = 0.0;
    for (int e = d.gx_ptr[i]; e < d.gx_ptr[i + 1]; ++e) mx = fmax(mx, fabs(gv[e]));
    rmax[i] = mx;
  }
  __syncthreads();
  int* mp = map + wv * nx;
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    const int r1 = d.lvu_ptr[lev + 1];
    for (int ri = d.lvu_ptr[lev] + wv; ri < r1; ri += kWaves) {
      const int i = d.lvu_rows[ri];
      const int f0 = d.f_ptr[i], fd = d.f_diag[i], f1 = d.f_ptr[i + 1];
      for (int e = f0 + lane; e < f1; e += 64) mp[d.f_col[e]] = e;
      wave_sync();
      for (int e = f0; e < fd; ++e) {
        const int kk = d.f_col[e];
        const double l = lu[e] * invd[kk];
        wave_sync();
        if (lane == 0) lu[e] = l;
        const int q1 = d.f_ptr[kk + 1];
        for (int q = d.f_diag[kk] + 1 + lane; q < q1; q += 64) lu[mp[d.f_col[q]]] -= l * lu[q];
        wave_sync();
      }
      if (lane == 0) {
        const double p = lu[fd];
        if (!(fabs(p) > 0.0 && fabs(p) >= 1e-10 * rmax[i]) || !isfinite(p)) raise_status(d, RKKT_ERR_SINGULAR_GX, k);
        invd[i] = 1.0 / p;
      }
      wave_sync();
    }
    __syncthreads();
  }
  if (kLDS) {
    double* glu = d.LU + (long long)k * d.nnz_f;
    for (int e = tid; e < d.nnz_f; e += kThreads) glu[e] = lu[e];
    double* gid = d.invd + (long long)k * nx;
    for (int i = tid; i < nx; i += kThreads) gid[i] = invd[i];
  }
}

// --------------------------------------------- multi-RHS level-scheduled solves
// X is an nx x W panel (row-major, column fastest).  lu/invd hold one
// scenario's factors of P G_x P^T = L U (L unit lower, U upper).

__device__ __forceinline__ void panel_L(const DP& d, const double* lu, double* X, int W) {
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    const int r0 = d.lvu_ptr[lev], n = (d.lvu_ptr[lev + 1] - r0) * W;
    for (int it = threadIdx.x; it < n; it += kThreads) {
      const int i = d.lvu_rows[r0 + it / W], c = it % W;
      double acc = X[i * W + c];
      for (int e = d.f_ptr[i]; e < d.f_diag[i]; ++e) acc -= lu[e] * X[d.f_col[e] * W + c];
      X[i * W + c] = acc;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void panel_U(const DP& d, const double* lu, const double* invd,
                                        double* X, int W) {
  for (int lev = 0; lev < d.nlev_dn; ++lev) {
    const int r0 = d.lvd_ptr[lev], n = (d.lvd_ptr[lev + 1] - r0) * W;
    for (int it = threadIdx.x; it < n; it += kThreads) {
      const int i = d.lvd_rows[r0 + it / W], c = it % W;
      double acc = X[i * W + c];
      for (int e = d.f_diag[i] + 1; e < d.f_ptr[i + 1]; ++e) acc -= lu[e] * X[d.f_col[e] * W + c];
      X[i * W + c] = acc * invd[i];
    }
    __syncthreads();
  }
}

// U^T v = b: row i of U^T has the pattern of the L part of row i
__device__ __forceinline__ void panel_Ut(const DP& d, const double* lu, const double* invd,
                                         double* X, int W) {
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    const int r0 = d.lvu_ptr[lev], n = (d.lvu_ptr[lev + 1] - r0) * W;
    for (int it = threadIdx.x; it < n; it += kThreads) {
      const int i = d.lvu_rows[r0 + it / W], c = it % W;
      double acc = X[i * W + c];
      for (int e = d.f_ptr[i]; e < d.f_diag[i]; ++e) acc -= lu[d.f_tpos[e]] * X[d.f_col[e] * W + c];
      X[i * W + c] = acc * invd[i];
    }
    __syncthreads();
  }
}

// L^T z = v: row i of L^T has the pattern of the U part of row i
__device__ __forceinline__ void panel_Lt(const DP& d, const double* lu, double* X, int W) {
  for (int lev = 0; lev < d.nlev_dn; ++lev) {
    const int r0 = d.lvd_ptr[lev], n = (d.lvd_ptr[lev + 1] - r0) * W;
    for (int it = threadIdx.x; it < n; it += kThreads) {
      const int i = d.lvd_rows[r0 + it / W], c = it % W;
      double acc = X[i * W + c];
      for (int e = d.f_diag[i] + 1; e < d.f_ptr[i + 1]; ++e) acc -= lu[d.f_tpos[e]] * X[d.f_col[e] * W + c];
      X[i * W + c] = acc;
    }
    __syncthreads();
  }
}

// value of K at (row r, column col) of the u block, 0 if structurally zero
__device__ __forceinline__ double k_ucol(const DP& d, const double* Kv, int r, int col) {
  for (int e = d.k_usplit[r]; e < d.k_ptr[r + 1]; ++e)
    if (d.k_col[e] == col) return Kv[e];
  return 0.0;
}

// ---------------------------------------------------------- local reduction
template <bool kLDS>
__global__ __launch_bounds__(kThreads) void k_reduce(DP d) {
  const int k = blockIdx.y, tile = blockIdx.x;
  const int W = d.col_tile, c0 = tile * W;
  const int nx = d.nx, nu = d.nu;
  const int ntile = gridDim.x;
  extern __shared__ double smem[];
  const double *lu, *invd;
  double *T, *Lx;
  if (kLDS) {
    double* slu = smem;
    double* sid = slu + d.nnz_f;
    T = sid + nx;
    Lx = T + nx * W;
    const double* glu = d.LU + (long long)k * d.nnz_f;
    for (int e = threadIdx.x; e < d.nnz_f; e += kThreads) slu[e] = glu[e];
    const double* gid = d.invd + (long long)k * nx;
    for (int i = threadIdx.x; i < nx; i += kThreads) sid[i] = gid[i];
    lu = slu;
    invd = sid;
  } else {
    lu = d.LU + (long long)k * d.nnz_f;
    invd = d.invd + (long long)k * nx;
    T = d.panel + ((long long)k * ntile + tile) * 2LL * nx * W;
    Lx = T + (long long)nx * W;
  }
  const double* Kv = d.K + (long long)k * d.nnz_k;
  const double* guv = d.EV + (long long)k * d.n_ev + d.off_gu;
  double* out = d.part + (long long)k * nu * nu;

  // right-hand side -G_u[:, c0:c0+W]
  for (int i = threadIdx.x; i < nx * W; i += kThreads) T[i] = 0.0;
  __syncthreads();
  for (int c = 0; c < W && c0 + c < nu; ++c) {
    const int cc = c0 + c;
    for (int j = d.guc_ptr[cc] + threadIdx.x; j < d.guc_ptr[cc + 1]; j += kThreads)
      T[d.guc_row[j] * W + c] = -guv[d.guc_pos[j]];
  }
  __syncthreads();
  // step 1: T = -G_x^-1 G_u V
  panel_L(d, lu, T, W);
  panel_U(d, lu, invd, T, W);
  // step 2: L_x = K_xx T + K_xu V, L_u = K_ux T + K_uu V
  for (int it = threadIdx.x; it < nx * W; it += kThreads) {
    const int r = it / W, c = it % W;
    double acc = k_ucol(d, Kv, r, nx + c0 + c);
    for (int e = d.k_ptr[r]; e < d.k_usplit[r]; ++e) acc += Kv[e] * T[d.k_col[e] * W + c];
    Lx[it] = acc;
  }
  for (int it = threadIdx.x; it < nu * W; it += kThreads) {
    const int ru = it / W, c = it % W;
    if (c0 + c >= nu) continue;
    const int r = nx + ru;
    double acc = k_ucol(d, Kv, r, nx + c0 + c);
    for (int e = d.k_ptr[r]; e < d.k_usplit[r]; ++e) acc += Kv[e] * T[d.k_col[e] * W + c];
    out[(long long)ru * nu + c0 + c] = acc;
  }
  __syncthreads();
  // step 3: K_hat V = L_u - G_u^T G_x^-T L_x
  panel_Ut(d, lu, invd, Lx, W);
  panel_Lt(d, lu, Lx, W);
  for (int it = threadIdx.x; it < nu * W; it += kThreads) {
    const int ru = it / W, c = it % W;
    if (c0 + c >= nu) continue;
    double acc = out[(long long)ru * nu + c0 + c];
    for (int j = d.guc_ptr[ru]; j < d.guc_ptr[ru + 1]; ++j)
      acc -= guv[d.guc_pos[j]] * Lx[d.guc_row[j] * W + c];
    out[(long long)ru * nu + c0 + c] = acc;
  }
}

// ------------------------------------------------ single-column solves (step)
__device__ __forceinline__ void vec_L(const DP& d, const double* lu, double* x) {
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    for (int ri = d.lvu_ptr[lev] + threadIdx.x; ri < d.lvu_ptr[lev + 1]; ri += kThreads) {
      const int i = d.lvu_rows[ri];
      double acc = x[i];
      for (int e = d.f_ptr[i]; e < d.f_diag[i]; ++e) acc -= lu[e] * x[d.f_col[e]];
      x[i] = acc;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void vec_U(const DP& d, const double* lu, const double* invd, double* x) {
  for (int lev = 0; lev < d.nlev_dn; ++lev) {
    for (int ri = d.lvd_ptr[lev] + threadIdx.x; ri < d.lvd_ptr[lev + 1]; ri += kThreads) {
      const int i = d.lvd_rows[ri];
      double acc = x[i];
      for (int e = d.f_diag[i] + 1; e < d.f_ptr[i + 1]; ++e) acc -= lu[e] * x[d.f_col[e]];
      x[i] = acc * invd[i];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void vec_Ut(const DP& d, const double* lu, const double* invd, double* x) {
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    for (int ri = d.lvu_ptr[lev] + threadIdx.x; ri < d.lvu_ptr[lev + 1]; ri += kThreads) {
      const int i = d.lvu_rows[ri];
      double acc = x[i];
      for (int e = d.f_ptr[i]; e < d.f_diag[i]; ++e) acc -= lu[d.f_tpos[e]] * x[d.f_col[e]];
      x[i] = acc * invd[i];
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void vec_Lt(const DP& d, const double* lu, double* x) {
  for (int lev = 0; lev < d.nlev_dn; ++lev) {
    for (int ri = d.lvd_ptr[lev] + threadIdx.x; ri < d.lvd_ptr[lev + 1]; ri += kThreads) {
      const int i = d.lvd_rows[ri];
      double acc = x[i];
      for (int e = d.f_diag[i] + 1; e < d.f_ptr[i + 1]; ++e) acc -= lu[d.f_tpos[e]] * x[d.f_col[e]];
      x[i] = acc;
    }
    __syncthreads();
  }
}

// Reduced right-hand side contributions of one scenario (eq. "kkt:reduced"):
//   rhat1 = r1x + H_x^T (Sigma_s r4 - r2),  q = G_x^-1 r3,
//   a = G_x^-T (rhat1 - K_xx q),
//   rpart = -H_u^T (Sigma_s r4 - r2) + G_u^T a + K_ux q
__global__ __launch_bounds__(kThreads) void k_step_rhs(DP d, const double* r1x, const double* r2,
                                                       const double* r3, const double* r4,
                                                       const double* ss) {
  const int k = blockIdx.x;
  const int nx = d.nx, nu = d.nu;
  const double* lu = d.LU + (long long)k * d.nnz_f;
  const double* invd = d.invd + (long long)k * nx;
  const double* Kv = d.K + (long long)k * d.nnz_k;
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* hv = ev + d.off_h;
  const double* guv = ev + d.off_gu;
  const double* r2k = r2 + (long long)k * d.m;
  const double* r4k = r4 + (long long)k * d.m;
  const double* ssk = ss + (long long)k * d.m;
  double* rh1 = d.rhat1 + (long long)k * nx;
  double* q = d.panel + (long long)k * 2 * nx;  // scratch: two nx vectors per scenario
  double* a = q + nx;
  for (int i = threadIdx.x; i < nx; i += kThreads) {
    double acc = r1x[(long long)k * nx + d.perm[i]];
    for (int j = d.ht_ptr[i]; j < d.ht_ptr[i + 1]; ++j) {
      const int r = d.ht_row[j];
      acc += hv[d.ht_pos[j]] * (ssk[r] * r4k[r] - r2k[r]);
    }
    rh1[i] = acc;
    q[i] = r3[(long long)k * nx + d.perm[i]];
  }
  __syncthreads();
  vec_L(d, lu, q);
  vec_U(d, lu, invd, q);
  for (int i = threadIdx.x; i < nx; i += kThreads) {
    double acc = rh1[i];
    for (int e = d.k_ptr[i]; e < d.k_usplit[i]; ++e) acc -= Kv[e] * q[d.k_col[e]];
    a[i] = acc;
  }
  __syncthreads();
  vec_Ut(d, lu, invd, a);
  vec_Lt(d, lu, a);
  for (int c = threadIdx.x; c < nu; c += kThreads) {
    const int v = nx + c;
    double acc = 0.0;
    for (int j = d.ht_ptr[v]; j < d.ht_ptr[v + 1]; ++j) {
      const int r = d.ht_row[j];
      acc -= hv[d.ht_pos[j]] * (ssk[r] * r4k[r] - r2k[r]);
    }
    for (int j = d.guc_ptr[c]; j < d.guc_ptr[c + 1]; ++j) acc += guv[d.guc_pos[j]] * a[d.guc_row[j]];
    for (int e = d.k_ptr[v]; e < d.k_usplit[v]; ++e) acc += Kv[e] * q[d.k_col[e]];
    d.rpart[(long long)k * nu + c] = acc;
  }
}

// Recovery of one scenario (propositions "Reduction" and "Condensed KKT system"):
//   p_x = -G_x^-1 (r3 + G_u p_u), p_y = -G_x^-T (rhat1 + K_xx p_x + K_xu p_u),
//   p_s = -(r4 + H p_d), p_z = Sigma_s (H p_d + r4) - r2
__global__ __launch_bounds__(kThreads) void k_step_recover(DP d, const double* r2, const double* r3,
                                                           const double* r4, const double* ss,
                                                           const double* pu, double* px, double* ps,
                                                           double* py, double* pz) {
  const int k = blockIdx.x;
  const int nx = d.nx;
  const double* lu = d.LU + (long long)k * d.nnz_f;
  const double* invd = d.invd + (long long)k * nx;
  const double* Kv = d.K + (long long)k * d.nnz_k;
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* hv = ev + d.off_h;
  const double* guv = ev + d.off_gu;
  const double* rh1 = d.rhat1 + (long long)k * nx;
  double* xv = d.panel + (long long)k * 2 * nx;
  double* yv = xv + nx;
  for (int i = threadIdx.x; i < nx; i += kThreads) {
    double acc = r3[(long long)k * nx + d.perm[i]];
    for (int e = d.gu_ptr[i]; e < d.gu_ptr[i + 1]; ++e) acc += guv[e] * pu[d.gu_col[e]];
    xv[i] = -acc;
  }
  __syncthreads();
  vec_L(d, lu, xv);
  vec_U(d, lu, invd, xv);
  for (int i = threadIdx.x; i < nx; i += kThreads) {
    px[(long long)k * nx + d.perm[i]] = xv[i];
    double acc = rh1[i];
    for (int e = d.k_ptr[i]; e < d.k_ptr[i + 1]; ++e) {
      const int c = d.k_col[e];
      acc += Kv[e] * (c < nx ? xv[c] : pu[c - nx]);
    }
    yv[i] = -acc;
  }
  __syncthreads();
  vec_Ut(d, lu, invd, yv);
  vec_Lt(d, lu, yv);
  for (int i = threadIdx.x; i < nx; i += kThreads) py[(long long)k * nx + d.perm[i]] = yv[i];
  const double* r2k = r2 + (long long)k * d.m;
  const double* r4k = r4 + (long long)k * d.m;
  const double* ssk = ss + (long long)k * d.m;
  for (int r = threadIdx.x; r < d.m; r += kThreads) {
    double hp = 0.0;
    for (int e = d.h_ptr[r]; e < d.h_ptr[r + 1]; ++e) {
      const int c = d.h_col[e];
      hp += hv[e] * (c < nx ? xv[c] : pu[c - nx]);
    }
    ps[(long long)k * d.m + r] = -(r4k[r] + hp);
    pz[(long long)k * d.m + r] = ssk[r] * (hp + r4k[r]) - r2k[r];
  }
}

}  // namespace

static hipError_t allow_lds(const void* fn, int* cur, int need) {
  if (need <= *cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, need);
  if (e == hipSuccess) *cur = need;
  return e;
}

hipError_t configure_lu_kernels(const DP& d) {
  static int c1 = 0, c2 = 0;
  if (!d.lds) return hipSuccess;
  const int lr = (int)(8 * ((size_t)d.nnz_f + 2 * (size_t)d.nx) + 4 * (size_t)kWaves * d.nx);
  const int lc = (int)(8 * ((size_t)d.nnz_f + (size_t)d.nx + 2 * (size_t)d.nx * d.col_tile));
  hipError_t e = allow_lds((const void*)k_refactor<true>, &c1, lr);
  if (e == hipSuccess) e = allow_lds((const void*)k_reduce<true>, &c2, lc);
  return e;
}

void launch_refactor(const DP& d, hipStream_t s) {
  if (d.lds) {
    size_t lds = 8 * ((size_t)d.nnz_f + 2 * (size_t)d.nx) + 4 * (size_t)kWaves * d.nx;
    k_refactor<true><<<d.N, kThreads, lds, s>>>(d);
  } else {
    k_refactor<false><<<d.N, kThreads, 0, s>>>(d);
  }
}

void launch_reduce(const DP& d, hipStream_t s) {
  const int ntile = (d.nu + d.col_tile - 1) / d.col_tile;
  dim3 grid(ntile, d.N);
  if (d.lds) {
    size_t lds = 8 * ((size_t)d.nnz_f + (size_t)d.nx + 2 * (size_t)d.nx * d.col_tile);
    k_reduce<true><<<grid, kThreads, lds, s>>>(d);
  } else {
    k_reduce<false><<<grid, kThreads, 0, s>>>(d);
  }
}

void launch_step_rhs(const DP& d, const double* r1x, const double* r2, const double* r3,
                     const double* r4, const double* ss, hipStream_t s) {
  k_step_rhs<<<d.N, kThreads, 0, s>>>(d, r1x, r2, r3, r4, ss);
}

void launch_step_recover(const DP& d, const double* r2, const double* r3, const double* r4,
                         const double* ss, const double* pu, double* px, double* ps, double* py,
                         double* pz, hipStream_t s) {
  k_step_recover<<<d.N, kThreads, 0, s>>>(d, r2, r3, r4, ss, pu, px, ps, py, pz);
}

}  // namespace rkkt
