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
// is one barrier-separated sweep.  Each thread keeps one fixed (row slot,
// column) pair for the whole kernel.
//
// When the problem fits (kLDS), every value and index the sweeps touch -- LU
// values, K values, G_u values, the filled pattern, the level schedules, the
// K pattern -- is copied into LDS once per workgroup, so the dependent loads
// on the critical path of a level are LDS loads; otherwise they read global
// memory (large grids).
#include "device.h"

namespace rkkt {

namespace {

constexpr int kThreads = 256;
constexpr int kRefactorWideThreads = 1024;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline void raise_status(const DP& d, int code, int k) {
  if (atomicCAS(d.status, 0, code) == 0) d.status[1] = k;
}

template <typename T>
__device__ __forceinline__ void copy_in(T* dst, const T* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__host__ __device__ __forceinline__ LdsSizes sizes_of(const DP& d) {
  LdsSizes z;
  z.nx = d.nx; z.nu = d.nu; z.nz = d.nz; z.nnz_f = d.nnz_f; z.nnz_k = d.nnz_k;
  z.nnz_gu = d.nnz_gu; z.nlu = d.nlev_up; z.nld = d.nlev_dn; z.w = d.col_tile;
  return z;
}

// pattern of the filled LU and its level schedules
struct SolveMeta {
  const int *f_ptr, *f_diag, *f_col, *f_tpos, *lvu_ptr, *lvu_rows, *lvd_ptr, *lvd_rows;
  int nlu, nld;
};

__device__ __forceinline__ SolveMeta global_meta(const DP& d) {
  return SolveMeta{d.f_ptr, d.f_diag, d.f_col, d.f_tpos, d.lvu_ptr, d.lvu_rows, d.lvd_ptr,
                   d.lvd_rows, d.nlev_up, d.nlev_dn};
}

// copies the solve metadata into LDS at `ip`; returns the pointer past it
__device__ __forceinline__ int* stage_meta(const DP& d, int* ip, SolveMeta& m) {
  const int nx = d.nx;
  int* p = ip;
  int* f_ptr = p; copy_in(f_ptr, d.f_ptr, nx + 1); p += nx + 1;
  int* f_diag = p; copy_in(f_diag, d.f_diag, nx); p += nx;
  int* f_col = p; copy_in(f_col, d.f_col, d.nnz_f); p += d.nnz_f;
  int* f_tpos = p; copy_in(f_tpos, d.f_tpos, d.nnz_f); p += d.nnz_f;
  int* lvu_ptr = p; copy_in(lvu_ptr, d.lvu_ptr, d.nlev_up + 1); p += d.nlev_up + 1;
  int* lvu_rows = p; copy_in(lvu_rows, d.lvu_rows, nx); p += nx;
  int* lvd_ptr = p; copy_in(lvd_ptr, d.lvd_ptr, d.nlev_dn + 1); p += d.nlev_dn + 1;
  int* lvd_rows = p; copy_in(lvd_rows, d.lvd_rows, nx); p += nx;
  m = SolveMeta{f_ptr, f_diag, f_col, f_tpos, lvu_ptr, lvu_rows, lvd_ptr, lvd_rows,
                d.nlev_up, d.nlev_dn};
  return p;
}

// One barrier-separated sweep per level; thread (slot, c) handles the rows
// slot, slot + nslot, ... of every level.
template <typename Row>
__device__ __forceinline__ void sweep(const int* lv_ptr, const int* lv_rows, int nlev, int slot,
                                      int nslot, bool active, Row row) {
  for (int lev = 0; lev < nlev; ++lev) {
    if (active) {
      const int r1 = lv_ptr[lev + 1];
      for (int ri = lv_ptr[lev] + slot; ri < r1; ri += nslot) row(lv_rows[ri]);
    }
    __syncthreads();
  }
}

// X (nx x W, column c of this thread): X <- L^-1 X, then U^-1
__device__ __forceinline__ void solve_LU(const SolveMeta& m, const double* lu, const double* invd,
                                         double* X, int W, int c, int slot, int nslot, bool act) {
  sweep(m.lvu_ptr, m.lvu_rows, m.nlu, slot, nslot, act, [&](int i) {
    double acc = X[i * W + c];
    const int e1 = m.f_diag[i];
    for (int e = m.f_ptr[i]; e < e1; ++e) acc -= lu[e] * X[m.f_col[e] * W + c];
    X[i * W + c] = acc;
  });
  sweep(m.lvd_ptr, m.lvd_rows, m.nld, slot, nslot, act, [&](int i) {
    double acc = X[i * W + c];
    const int e1 = m.f_ptr[i + 1];
    for (int e = m.f_diag[i] + 1; e < e1; ++e) acc -= lu[e] * X[m.f_col[e] * W + c];
    X[i * W + c] = acc * invd[i];
  });
}

// X <- U^-T X, then L^-T (row i of U^T / L^T has the pattern of the L / U part of row i)
__device__ __forceinline__ void solve_LUt(const SolveMeta& m, const double* lu, const double* invd,
                                          double* X, int W, int c, int slot, int nslot, bool act) {
  sweep(m.lvu_ptr, m.lvu_rows, m.nlu, slot, nslot, act, [&](int i) {
    double acc = X[i * W + c];
    const int e1 = m.f_diag[i];
    for (int e = m.f_ptr[i]; e < e1; ++e) acc -= lu[m.f_tpos[e]] * X[m.f_col[e] * W + c];
    X[i * W + c] = acc * invd[i];
  });
  sweep(m.lvd_ptr, m.lvd_rows, m.nld, slot, nslot, act, [&](int i) {
    double acc = X[i * W + c];
    const int e1 = m.f_ptr[i + 1];
    for (int e = m.f_diag[i] + 1; e < e1; ++e) acc -= lu[m.f_tpos[e]] * X[m.f_col[e] * W + c];
    X[i * W + c] = acc;
  });
}

// ------------------------------------------------------------ refactorisation
template <bool kLDS, int kRT>
__global__ __launch_bounds__(kRT) void k_refactor(DP d) {
  constexpr int kRW = kRT / 64;
  const int k = blockIdx.x;
  const int nx = d.nx;
  extern __shared__ double smem[];
  double *lu, *invd, *rmax;
  int* map;
  const int *f_ptr, *f_diag, *f_col, *lvu_ptr, *lvu_rows;
  if (kLDS) {
    lu = smem;
    invd = lu + d.nnz_f;
    rmax = invd + nx;
    int* p = reinterpret_cast<int*>(rmax + nx);
    int* a = p; copy_in(a, d.f_ptr, nx + 1); f_ptr = a; p += nx + 1;
    a = p; copy_in(a, d.f_diag, nx); f_diag = a; p += nx;
    a = p; copy_in(a, d.f_col, d.nnz_f); f_col = a; p += d.nnz_f;
    a = p; copy_in(a, d.lvu_ptr, d.nlev_up + 1); lvu_ptr = a; p += d.nlev_up + 1;
    a = p; copy_in(a, d.lvu_rows, nx); lvu_rows = a; p += nx;
    map = p;
  } else {
    lu = d.LU + (long long)k * d.nnz_f;
    invd = d.invd + (long long)k * nx;
    rmax = d.rhat1 + (long long)k * nx;
    map = d.imap + (long long)k * kRW * nx;
    f_ptr = d.f_ptr; f_diag = d.f_diag; f_col = d.f_col; lvu_ptr = d.lvu_ptr; lvu_rows = d.lvu_rows;
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* gv = d.EV + (long long)k * d.n_ev + d.off_gx;
  for (int e = tid; e < d.nnz_f; e += kRT) lu[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < d.nnz_gx; e += kRT) lu[d.gx2f[e]] = gv[e];
  for (int i = tid; i < nx; i += kRT) {
    double mx = 0.0;
    for (int e = d.gx_ptr[i]; e < d.gx_ptr[i + 1]; ++e) mx = fmax(mx, fabs(gv[e]));
    rmax[i] = mx;
  }
  __syncthreads();
  int* mp = map + wv * nx;
  for (int lev = 0; lev < d.nlev_up; ++lev) {
    const int r1 = lvu_ptr[lev + 1];
    for (int ri = lvu_ptr[lev] + wv; ri < r1; ri += kRW) {
      const int i = lvu_rows[ri];
      const int f0 = f_ptr[i], fd = f_diag[i], f1 = f_ptr[i + 1];
      for (int e = f0 + lane; e < f1; e += 64) mp[f_col[e]] = e;
      wave_sync();
      for (int e = f0; e < fd; ++e) {
        const int kk = f_col[e];
        const double l = lu[e] * invd[kk];
        wave_sync();
        if (lane == 0) lu[e] = l;
        const int q1 = f_ptr[kk + 1];
        for (int q = f_diag[kk] + 1 + lane; q < q1; q += 64) lu[mp[f_col[q]]] -= l * lu[q];
        wave_sync();
      }
      if (lane == 0) {
        const double p = lu[fd];
        if (!(fabs(p) > 0.0 && fabs(p) >= 1e-10 * rmax[i]) || !isfinite(p))
          raise_status(d, RKKT_ERR_SINGULAR_GX, k);
        invd[i] = 1.0 / p;
      }
      wave_sync();
    }
    __syncthreads();
  }
  if (kLDS) {
    double* glu = d.LU + (long long)k * d.nnz_f;
    for (int e = tid; e < d.nnz_f; e += kRT) glu[e] = lu[e];
    double* gid = d.invd + (long long)k * nx;
    for (int i = tid; i < nx; i += kRT) gid[i] = invd[i];
  }
}

// ---------------------------------------------------------- local reduction
template <bool kLDS>
__global__ __launch_bounds__(kThreads) void k_reduce(DP d) {
  const int k = blockIdx.y, tile = blockIdx.x;
  const int W = d.col_tile, c0 = tile * W;
  const int nx = d.nx, nu = d.nu;
  const int ntile = gridDim.x;
  const int tid = threadIdx.x;
  const int nslot = kThreads / W, slot = tid / W, c = tid % W;
  const bool act = slot < nslot;
  extern __shared__ double smem[];
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double *lu, *invd, *kv, *guv;
  double *T, *Lx;
  SolveMeta m;
  const int *k_ptr, *k_usplit, *k_col, *guc_ptr, *guc_row;
  if (kLDS) {
    const LdsSizes z = sizes_of(d);
    double* p = smem;
    double* slu = p; copy_in(slu, d.LU + (long long)k * d.nnz_f, d.nnz_f); p += d.nnz_f;
    double* sid = p; copy_in(sid, d.invd + (long long)k * nx, nx); p += nx;
    double* skv = p; copy_in(skv, d.K + (long long)k * d.nnz_k, d.nnz_k); p += d.nnz_k;
    double* sgu = p;
    for (int j = tid; j < d.nnz_gu; j += kThreads) sgu[j] = ev[d.off_gu + d.guc_pos[j]];
    p += d.nnz_gu;
    T = p; p += nx * W;
    Lx = p; p += nx * W;
    int* ip = reinterpret_cast<int*>(smem + reduce_lds_doubles(z));
    ip = stage_meta(d, ip, m);
    int* a = ip; copy_in(a, d.k_ptr, d.nz + 1); k_ptr = a; ip += d.nz + 1;
    a = ip; copy_in(a, d.k_usplit, d.nz); k_usplit = a; ip += d.nz;
    a = ip; copy_in(a, d.k_col, d.nnz_k); k_col = a; ip += d.nnz_k;
    a = ip; copy_in(a, d.guc_ptr, nu + 1); guc_ptr = a; ip += nu + 1;
    a = ip; copy_in(a, d.guc_row, d.nnz_gu); guc_row = a;
    lu = slu; invd = sid; kv = skv; guv = sgu;
  } else {
    lu = d.LU + (long long)k * d.nnz_f;
    invd = d.invd + (long long)k * nx;
    kv = d.K + (long long)k * d.nnz_k;
    guv = nullptr;
    T = d.panel + ((long long)k * ntile + tile) * 2LL * nx * W;
    Lx = T + (long long)nx * W;
    m = global_meta(d);
    k_ptr = d.k_ptr; k_usplit = d.k_usplit; k_col = d.k_col;
    guc_ptr = d.guc_ptr; guc_row = d.guc_row;
  }
  auto gu_val = [&](int j) -> double { return kLDS ? guv[j] : ev[d.off_gu + d.guc_pos[j]]; };
  auto k_ucol = [&](int r, int col) -> double {
    const int e1 = k_ptr[r + 1];
    for (int e = k_usplit[r]; e < e1; ++e)
      if (k_col[e] == col) return kv[e];
    return 0.0;
  };
  double* out = d.part + (long long)k * nu * nu;
  const bool colok = c0 + c < nu;

  // right-hand side -G_u[:, c0:c0+W]
  for (int i = tid; i < nx * W; i += kThreads) T[i] = 0.0;
  __syncthreads();
  if (act && colok)
    for (int j = guc_ptr[c0 + c] + slot; j < guc_ptr[c0 + c + 1]; j += nslot)
      T[guc_row[j] * W + c] = -gu_val(j);
  __syncthreads();
  // step 1: T = -G_x^-1 G_u V
  solve_LU(m, lu, invd, T, W, c, slot, nslot, act);
  // step 2: L_x = K_xx T + K_xu V, L_u = K_ux T + K_uu V
  if (act) {
    for (int r = slot; r < nx; r += nslot) {
      double acc = k_ucol(r, nx + c0 + c);
      const int e1 = k_usplit[r];
      for (int e = k_ptr[r]; e < e1; ++e) acc += kv[e] * T[k_col[e] * W + c];
      Lx[r * W + c] = acc;
    }
    if (colok)
      for (int ru = slot; ru < nu; ru += nslot) {
        const int r = nx + ru;
        double acc = k_ucol(r, nx + c0 + c);
        const int e1 = k_usplit[r];
        for (int e = k_ptr[r]; e < e1; ++e) acc += kv[e] * T[k_col[e] * W + c];
        out[(long long)ru * nu + c0 + c] = acc;
      }
  }
  __syncthreads();
  // step 3: K_hat V = L_u - G_u^T G_x^-T L_x
  solve_LUt(m, lu, invd, Lx, W, c, slot, nslot, act);
  if (act && colok)
    for (int ru = slot; ru < nu; ru += nslot) {
      double acc = out[(long long)ru * nu + c0 + c];
      const int j1 = guc_ptr[ru + 1];
      for (int j = guc_ptr[ru]; j < j1; ++j) acc -= gu_val(j) * Lx[guc_row[j] * W + c];
      out[(long long)ru * nu + c0 + c] = acc;
    }
}

// ------------------------------------- local reduction, large grids (global)
// One workgroup of 16 wavefronts per (scenario, tile of 64 columns); a
// wavefront owns one row at a time and its lanes the 64 columns, so the row's
// pattern and LU values are wavefront-uniform (one broadcast load each) and
// the panel accesses X[col][lane] are coalesced.  Panels live in global memory.
constexpr int kWideThreads = 1024, kWideWaves = kWideThreads / 64, kWideW = 64;

template <bool kTrans, bool kUpper, bool kScale>
__device__ __forceinline__ void wide_sweep(const DP& d, const double* __restrict__ lu,
                                           const double* __restrict__ invd, double* X, int wv,
                                           int lane) {
  const int* lv_ptr = kUpper ? d.lvd_ptr : d.lvu_ptr;
  const int* lv_rows = kUpper ? d.lvd_rows : d.lvu_rows;
  const int nlev = kUpper ? d.nlev_dn : d.nlev_up;
  for (int lev = 0; lev < nlev; ++lev) {
    const int r1 = lv_ptr[lev + 1];
    for (int ri = lv_ptr[lev] + wv; ri < r1; ri += kWideWaves) {
      const int i = __builtin_amdgcn_readfirstlane(lv_rows[ri]);
      const int e0 = kUpper ? d.f_diag[i] + 1 : d.f_ptr[i];
      const int e1 = kUpper ? d.f_ptr[i + 1] : d.f_diag[i];
      double acc = X[(long long)i * kWideW + lane];
      double acc2 = 0.0;
      int e = e0;
      for (; e + 4 <= e1; e += 4) {
        const int c0 = d.f_col[e], c1 = d.f_col[e + 1], c2 = d.f_col[e + 2], c3 = d.f_col[e + 3];
        const double v0 = lu[kTrans ? d.f_tpos[e] : e], v1 = lu[kTrans ? d.f_tpos[e + 1] : e + 1];
        const double v2 = lu[kTrans ? d.f_tpos[e + 2] : e + 2], v3 = lu[kTrans ? d.f_tpos[e + 3] : e + 3];
        const double x0 = X[(long long)c0 * kWideW + lane], x1 = X[(long long)c1 * kWideW + lane];
        const double x2 = X[(long long)c2 * kWideW + lane], x3 = X[(long long)c3 * kWideW + lane];
        acc -= v0 * x0;
        acc2 -= v1 * x1;
        acc -= v2 * x2;
        acc2 -= v3 * x3;
      }
      for (; e < e1; ++e) acc -= lu[kTrans ? d.f_tpos[e] : e] * X[(long long)d.f_col[e] * kWideW + lane];
      acc += acc2;
      X[(long long)i * kWideW + lane] = kScale ? acc * invd[i] : acc;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kWideThreads) void k_reduce_wide(DP d) {
  const int k = blockIdx.y, tile = blockIdx.x;
  const int c0 = tile * kWideW, nx = d.nx, nu = d.nu;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* lu = d.LU + (long long)k * d.nnz_f;
  const double* invd = d.invd + (long long)k * nx;
  const double* kv = d.K + (long long)k * d.nnz_k;
  double* T = d.panel + ((long long)k * gridDim.x + tile) * 2LL * nx * kWideW;
  double* Lx = T + (long long)nx * kWideW;
  double* out = d.part + (long long)k * nu * nu;
  const int col = c0 + lane;
  const bool colok = col < nu;
  for (long long q = tid; q < (long long)nx * kWideW; q += kWideThreads) T[q] = 0.0;
  __syncthreads();
  if (colok)
    for (int j = d.guc_ptr[col] + wv; j < d.guc_ptr[col + 1]; j += kWideWaves)
      T[(long long)d.guc_row[j] * kWideW + lane] = -ev[d.off_gu + d.guc_pos[j]];
  __syncthreads();
  wide_sweep<false, false, false>(d, lu, invd, T, wv, lane);
  wide_sweep<false, true, true>(d, lu, invd, T, wv, lane);
  auto k_ucol = [&](int r, int cc) -> double {
    for (int e = d.k_usplit[r]; e < d.k_ptr[r + 1]; ++e)
      if (d.k_col[e] == cc) return kv[e];
    return 0.0;
  };
  for (int r = wv; r < nx + nu; r += kWideWaves) {
    const int rr = __builtin_amdgcn_readfirstlane(r);
    double acc = k_ucol(rr, nx + col);
    const int e1 = d.k_usplit[rr];
    for (int e = d.k_ptr[rr]; e < e1; ++e) acc += kv[e] * T[(long long)d.k_col[e] * kWideW + lane];
    if (rr < nx) Lx[(long long)rr * kWideW + lane] = acc;
    else if (colok) out[(long long)(rr - nx) * nu + col] = acc;
  }
  __syncthreads();
  wide_sweep<true, false, true>(d, lu, invd, Lx, wv, lane);
  wide_sweep<true, true, false>(d, lu, invd, Lx, wv, lane);
  for (int ru = wv; ru < nu; ru += kWideWaves) {
    const int rr = __builtin_amdgcn_readfirstlane(ru);
    if (!colok) continue;
    double acc = out[(long long)rr * nu + col];
    for (int j = d.guc_ptr[rr]; j < d.guc_ptr[rr + 1]; ++j)
      acc -= ev[d.off_gu + d.guc_pos[j]] * Lx[(long long)d.guc_row[j] * kWideW + lane];
    out[(long long)rr * nu + col] = acc;
  }
}

// ------------------------------------------------ single-column solves (step)
// Workspace of a step workgroup: LU values, 1/u_ii and three nx vectors in LDS
// (with the solve metadata) when they fit, else per-scenario global memory.
struct StepWs {
  const double *lu, *invd;
  double *v0, *v1, *v2;
  SolveMeta m;
};

template <bool kLDS>
__device__ __forceinline__ StepWs step_ws(const DP& d, int k, double* smem) {
  StepWs w;
  const int nx = d.nx;
  if (kLDS) {
    double* p = smem;
    double* slu = p; copy_in(slu, d.LU + (long long)k * d.nnz_f, d.nnz_f); p += d.nnz_f;
    double* sid = p; copy_in(sid, d.invd + (long long)k * nx, nx); p += nx;
    w.v0 = p; p += nx;
    w.v1 = p; p += nx;
    w.v2 = p; p += nx;
    stage_meta(d, reinterpret_cast<int*>(p), w.m);
    w.lu = slu;
    w.invd = sid;
  } else {
    w.lu = d.LU + (long long)k * d.nnz_f;
    w.invd = d.invd + (long long)k * nx;
    w.v0 = d.panel + (long long)k * 2 * nx;
    w.v1 = w.v0 + nx;
    w.v2 = d.rhat1 + (long long)k * nx;
    w.m = global_meta(d);
  }
  __syncthreads();
  return w;
}

// Reduced right-hand side contributions of one scenario (eq. "kkt:reduced"):
//   rhat1 = r1x + H_x^T (Sigma_s r4 - r2),  q = G_x^-1 r3,
//   a = G_x^-T (rhat1 - K_xx q),
//   rpart = -H_u^T (Sigma_s r4 - r2) + G_u^T a + K_ux q
template <bool kLDS>
__global__ __launch_bounds__(kThreads) void k_step_rhs(DP d, const double* r1x, const double* r2,
                                                       const double* r3, const double* r4,
                                                       const double* ss) {
  extern __shared__ double smem[];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int nx = d.nx, nu = d.nu;
  const StepWs w = step_ws<kLDS>(d, k, smem);
  const double* Kv = d.K + (long long)k * d.nnz_k;
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* hv = ev + d.off_h;
  const double* guv = ev + d.off_gu;
  const double* r2k = r2 + (long long)k * d.m;
  const double* r4k = r4 + (long long)k * d.m;
  const double* ssk = ss + (long long)k * d.m;
  double* rh1 = w.v2;  // rhat1; the global copy is kept for the recovery
  double* q = w.v0;
  double* a = w.v1;
  double* grh1 = d.rhat1 + (long long)k * nx;
  for (int i = tid; i < nx; i += kThreads) {
    double acc = r1x[(long long)k * nx + d.perm[i]];
    for (int j = d.ht_ptr[i]; j < d.ht_ptr[i + 1]; ++j) {
      const int r = d.ht_row[j];
      acc += hv[d.ht_pos[j]] * (ssk[r] * r4k[r] - r2k[r]);
    }
    rh1[i] = acc;
    q[i] = r3[(long long)k * nx + d.perm[i]];
  }
  __syncthreads();
  solve_LU(w.m, w.lu, w.invd, q, 1, 0, tid, kThreads, true);
  for (int i = tid; i < nx; i += kThreads) {
    double acc = rh1[i];
    for (int e = d.k_ptr[i]; e < d.k_usplit[i]; ++e) acc -= Kv[e] * q[d.k_col[e]];
    a[i] = acc;
    if (kLDS) grh1[i] = rh1[i];
  }
  __syncthreads();
  solve_LUt(w.m, w.lu, w.invd, a, 1, 0, tid, kThreads, true);
  for (int c = tid; c < nu; c += kThreads) {
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
template <bool kLDS>
__global__ __launch_bounds__(kThreads) void k_step_recover(DP d, const double* r2, const double* r3,
                                                           const double* r4, const double* ss,
                                                           const double* pu, double* px, double* ps,
                                                           double* py, double* pz) {
  extern __shared__ double smem[];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int nx = d.nx;
  const StepWs w = step_ws<kLDS>(d, k, smem);
  const double* Kv = d.K + (long long)k * d.nnz_k;
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* hv = ev + d.off_h;
  const double* guv = ev + d.off_gu;
  const double* rh1 = d.rhat1 + (long long)k * nx;
  double* xv = w.v0;
  double* yv = w.v1;
  for (int i = tid; i < nx; i += kThreads) {
    double acc = r3[(long long)k * nx + d.perm[i]];
    for (int e = d.gu_ptr[i]; e < d.gu_ptr[i + 1]; ++e) acc += guv[e] * pu[d.gu_col[e]];
    xv[i] = -acc;
  }
  __syncthreads();
  solve_LU(w.m, w.lu, w.invd, xv, 1, 0, tid, kThreads, true);
  for (int i = tid; i < nx; i += kThreads) {
    px[(long long)k * nx + d.perm[i]] = xv[i];
    double acc = rh1[i];
    for (int e = d.k_ptr[i]; e < d.k_ptr[i + 1]; ++e) {
      const int cc = d.k_col[e];
      acc += Kv[e] * (cc < nx ? xv[cc] : pu[cc - nx]);
    }
    yv[i] = -acc;
  }
  __syncthreads();
  solve_LUt(w.m, w.lu, w.invd, yv, 1, 0, tid, kThreads, true);
  for (int i = tid; i < nx; i += kThreads) py[(long long)k * nx + d.perm[i]] = yv[i];
  const double* r2k = r2 + (long long)k * d.m;
  const double* r4k = r4 + (long long)k * d.m;
  const double* ssk = ss + (long long)k * d.m;
  for (int r = tid; r < d.m; r += kThreads) {
    double hp = 0.0;
    for (int e = d.h_ptr[r]; e < d.h_ptr[r + 1]; ++e) {
      const int cc = d.h_col[e];
      hp += hv[e] * (cc < nx ? xv[cc] : pu[cc - nx]);
    }
    ps[(long long)k * d.m + r] = -(r4k[r] + hp);
    pz[(long long)k * d.m + r] = ssk[r] * (hp + r4k[r]) - r2k[r];
  }
}

hipError_t allow_lds(const void* fn, int* cur, long long need) {
  if (need <= *cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
  if (e == hipSuccess) *cur = (int)need;
  return e;
}

}  // namespace

hipError_t configure_lu_kernels(const DP& d) {
  static int c1 = 0, c2 = 0, c3 = 0, c4 = 0;
  if (!d.lds) return hipSuccess;
  const LdsSizes z = sizes_of(d);
  hipError_t e = allow_lds((const void*)k_refactor<true, kThreads>, &c1, refactor_lds_bytes(z));
  if (e == hipSuccess) e = allow_lds((const void*)k_reduce<true>, &c2, reduce_lds_bytes(z));
  if (e == hipSuccess) e = allow_lds((const void*)k_step_rhs<true>, &c3, step_lds_bytes(z));
  if (e == hipSuccess) e = allow_lds((const void*)k_step_recover<true>, &c4, step_lds_bytes(z));
  return e;
}

void launch_refactor(const DP& d, hipStream_t s) {
  if (d.lds)
    k_refactor<true, kThreads><<<d.N, kThreads, refactor_lds_bytes(sizes_of(d)), s>>>(d);
  else
    k_refactor<false, kRefactorWideThreads><<<d.N, kRefactorWideThreads, 0, s>>>(d);
}

void launch_reduce(const DP& d, hipStream_t s) {
  const int ntile = (d.nu + d.col_tile - 1) / d.col_tile;
  dim3 grid(ntile, d.N);
  if (d.lds)
    k_reduce<true><<<grid, kThreads, reduce_lds_bytes(sizes_of(d)), s>>>(d);
  else if (d.col_tile == kWideW)
    k_reduce_wide<<<grid, kWideThreads, 0, s>>>(d);
  else
    k_reduce<false><<<grid, kThreads, 0, s>>>(d);
}

void launch_step_rhs(const DP& d, const double* r1x, const double* r2, const double* r3,
                     const double* r4, const double* ss, hipStream_t s) {
  if (d.lds)
    k_step_rhs<true><<<d.N, kThreads, step_lds_bytes(sizes_of(d)), s>>>(d, r1x, r2, r3, r4, ss);
  else
    k_step_rhs<false><<<d.N, kThreads, 0, s>>>(d, r1x, r2, r3, r4, ss);
}

void launch_step_recover(const DP& d, const double* r2, const double* r3, const double* r4,
                         const double* ss, const double* pu, double* px, double* ps, double* py,
                         double* pz, hipStream_t s) {
  if (d.lds)
    k_step_recover<true><<<d.N, kThreads, step_lds_bytes(sizes_of(d)), s>>>(
        d, r2, r3, r4, ss, pu, px, ps, py, pz);
  else
    k_step_recover<false><<<d.N, kThreads, 0, s>>>(d, r2, r3, r4, ss, pu, px, ps, py, pz);
}

}  // namespace rkkt
