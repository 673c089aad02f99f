// Batched evaluation of the scenario blocks and condensation of the KKT matrix.
//
// Paper: block evaluation through a nonlinear basis (eq. "AST", "eval:block"):
// every scenario's f, g, h are linear maps of per-line basis terms
// (V_f^2, V_t^2, V_f V_t cos, V_f V_t sin).  Here the basis is evaluated per
// (scenario, line) and every output -- bus injections, Jacobian values of the
// fixed patterns, Hessian values -- is a fixed gather over per-line
// quantities, so no value is ever accumulated with atomics.  Derivatives are
// the analytic derivatives of the basis (the paper uses forward-mode and
// forward-over-reverse AD on the same structure).
#include "device.h"

namespace rkkt {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline double bus_theta(const DP& d, const double* xk, int b) {
  int s = d.th_src[b];
  return s >= 0 ? xk[s] : 0.0;
}

__device__ inline double bus_vm(const DP& d, const double* xk, const double* u, int b) {
  int s = d.v_src[b];
  return s >= 0 ? xk[s] : u[-s - 1];
}

// The four line-end functions F = A vf^2 + B vt^2 + vf vt (C cos + D sin)
// of the pi-model (order: P_from, Q_from, P_to, Q_to).
__device__ inline void line_coeffs(double gs, double bs, double bc, double A[4], double B[4],
                                   double C[4], double D[4]) {
  A[0] = gs;          B[0] = 0.0;          C[0] = -gs; D[0] = -bs;
  A[1] = -(bs + bc);  B[1] = 0.0;          C[1] = bs;  D[1] = -gs;
  A[2] = 0.0;         B[2] = gs;           C[2] = -gs; D[2] = bs;
  A[3] = 0.0;         B[3] = -(bs + bc);   C[3] = bs;  D[3] = gs;
}

__global__ void k_bus_loads(DP d, const double* pd, const double* qd) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nb) return;
  int k = (int)(t / d.nb), b = (int)(t % d.nb);
  int j = d.load_of_bus[b];
  d.pdb[t] = j >= 0 ? pd[(long long)k * d.nload + j] : 0.0;
  d.qdb[t] = j >= 0 ? qd[(long long)k * d.nload + j] : 0.0;
}

// a1: basis terms and first derivatives of the four line-end functions of
// line l; o = its 28 values
__device__ inline void line_eval_one(const DP& d, int k, int l, const double* x, const double* u,
                                     double* o) {
  const double* xk = x + (long long)k * d.nx;
  int bf = d.line_f[l], bt = d.line_t[l];
  double dth = bus_theta(d, xk, bf) - bus_theta(d, xk, bt);
  double vf = bus_vm(d, xk, u, bf), vt = bus_vm(d, xk, u, bt);
  double sn, cs;
  sincos(dth, &sn, &cs);
  double A[4], B[4], C[4], D[4];
  const double st = d.lstat[(long long)k * d.nl + l];  // 0 for a tripped line
  line_coeffs(st * d.gs[l], st * d.bs[l], st * d.bc[l], A, B, C, D);
  double val[4], grad[4][4];
  for (int q = 0; q < 4; ++q) {
    double T = C[q] * cs + D[q] * sn;
    double Tp = -C[q] * sn + D[q] * cs;
    val[q] = A[q] * vf * vf + B[q] * vt * vt + vf * vt * T;
    grad[q][0] = vf * vt * Tp;
    grad[q][1] = -vf * vt * Tp;
    grad[q][2] = 2.0 * A[q] * vf + vt * T;
    grad[q][3] = 2.0 * B[q] * vt + vf * T;
  }
  for (int e = 0; e < 2; ++e) {
    double P = val[2 * e], Q = val[2 * e + 1];
    double* oe = o + 14 * e;
    oe[0] = P;
    oe[1] = Q;
    for (int q = 0; q < 4; ++q) {
      oe[2 + q] = grad[2 * e][q];
      oe[6 + q] = grad[2 * e + 1][q];
      oe[10 + q] = 2.0 * (P * grad[2 * e][q] + Q * grad[2 * e + 1][q]);
    }
  }
}

// one bus injection or Jacobian value on the fixed patterns; lv = the
// scenario's line values
__device__ inline double gather_ev_one(const DP& d, int e, const double* lv) {
  // terms added in list order, the source indices of kEb terms loaded
  // together before their values are read
  constexpr int kEb = 4;
  const int j0 = d.ev_ptr[e], j1 = d.ev_ptr[e + 1];
  double acc = d.ev_const[e];
  for (int j = j0; j < j1; j += kEb) {
    int src[kEb];
#pragma unroll
    for (int q = 0; q < kEb; ++q) src[q] = d.ev_src[min(j + q, j1 - 1)];
#pragma unroll
    for (int q = 0; q < kEb; ++q)
      if (j + q < j1) acc += lv[src[q]];
  }
  return acc;
}

// one entry of g, h or the gradient of f (item i of 2 nx + m + nu); ev,
// lv = the scenario's values
__device__ inline void assemble_one(const DP& d, int k, int i, const double* u, double w,
                                    double* gx, double* gu, double* g, double* h,
                                    const double* ev, const double* lv) {
  const double* pdb = d.pdb + (long long)k * d.nb;
  const double* qdb = d.qdb + (long long)k * d.nb;
  double pref = ev[d.off_P + d.ref] + pdb[d.ref];
  double cref = w * (2.0 * d.aref * pref + d.bref);
  if (i < d.nx) {
    int b = d.grow_bus[i];
    double v;
    if (i < d.nb - 1) {
      int pu = d.pg_u[b];
      v = ev[d.off_P + b] - (pu >= 0 ? u[pu] : 0.0) + pdb[b];
    } else {
      v = ev[d.off_Q + b] + qdb[b];
    }
    g[(long long)k * d.nx + i] = v;
    return;
  }
  i -= d.nx;
  if (i < d.m) {
    double v;
    if (i == 0) {
      v = pref;
    } else if (i <= d.ng) {
      int b = d.gen_bus[i - 1];
      v = ev[d.off_Q + b] + qdb[b];
    } else {
      int r = i - 1 - d.ng;
      int e = r >= d.nl ? 1 : 0;
      int l = r - e * d.nl;
      const double* le = lv + (long long)l * kLVsize + 14 * e;
      v = le[0] * le[0] + le[1] * le[1];
    }
    h[(long long)k * d.m + i] = v;
    return;
  }
  i -= d.m;
  if (i < d.nx) {
    int p = d.h0pos[d.pinv[i]];
    gx[(long long)k * d.nx + i] = p >= 0 ? cref * ev[d.off_h + p] : 0.0;
    return;
  }
  i -= d.nx;
  if (i < d.nu) {
    double v;
    if (i < d.ng) {
      int p = d.h0pos[d.nx + i];
      v = p >= 0 ? cref * ev[d.off_h + p] : 0.0;
    } else {
      int gg = d.gnr[i - d.ng];
      v = w * (2.0 * d.ca[gg] * u[i] + d.cb[gg]);
    }
    gu[(long long)k * d.nu + i] = v;
  }
}

// the objective f of scenario k by one wavefront: lane j adds the costs of
// generators j, j + 64, ... in order, then the 64 partial sums meet in a
// fixed butterfly, so the result does not depend on the run
__device__ inline void objective_wave(const DP& d, int k, int lane, const double* u, double w, double* f) {
  const double pref = d.EV[(long long)k * d.n_ev + d.off_P + d.ref] + d.pdb[(long long)k * d.nb + d.ref];
  double acc = 0.0;
  for (int gg = lane; gg < d.ng; gg += 64) {
    const int ui = d.gen_u[gg];
    const double pg = ui >= 0 ? u[ui] : pref;
    acc += d.ca[gg] * pg * pg + d.cb[gg] * pg + d.cc[gg];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) f[k] = w * acc;
}

// threads of k_assemble: one per entry of g, h and the gradients (2 nx + m +
// nu per scenario), then, from the next wavefront boundary, one wavefront per
// scenario for f
__host__ __device__ inline long long assemble_f_base(const DP& d) {
  return ((long long)d.N * (2 * d.nx + d.m + d.nu) + 63) / 64 * 64;
}
__host__ __device__ inline long long assemble_threads(const DP& d) { return assemble_f_base(d) + 64LL * d.N; }

// a3: local 4x4 Hessian of line l's share of f + y^T g + z^T h; le = the
// line's 28 values, o = its 10 Hessian values
__device__ inline void line_hess_one(const DP& d, int k, int l, const double* x, const double* u,
                                     const double* y, const double* z, double w,
                                     const double* ev, const double* le0, double* o) {
  const double* xk = x + (long long)k * d.nx;
  const double* yk = y + (long long)k * d.nx;
  const double* zk = z + (long long)k * d.m;
  int bus[2] = {d.line_f[l], d.line_t[l]};
  double dth = bus_theta(d, xk, bus[0]) - bus_theta(d, xk, bus[1]);
  double vf = bus_vm(d, xk, u, bus[0]), vt = bus_vm(d, xk, u, bus[1]);
  double sn, cs;
  sincos(dth, &sn, &cs);
  double A[4], B[4], C[4], D[4];
  const double st = d.lstat[(long long)k * d.nl + l];
  line_coeffs(st * d.gs[l], st * d.bs[l], st * d.bc[l], A, B, C, D);
  const double pgref = ev[d.off_P + d.ref] + d.pdb[(long long)k * d.nb + d.ref];
  double H[kLHsize];
  for (int q = 0; q < kLHsize; ++q) H[q] = 0.0;
  for (int e = 0; e < 2; ++e) {
    int b = bus[e];
    double wP, wQ;
    if (d.prow[b] >= 0) wP = yk[d.prow[b]];
    else wP = zk[0] + w * (2.0 * d.aref * pgref + d.bref);
    wQ = d.qrow[b] >= 0 ? yk[d.qrow[b]] : zk[1 + (-d.qrow[b] - 1)];
    double zs = zk[1 + d.ng + e * d.nl + l];
    const double* le = le0 + 14 * e;
    double mu[2] = {wP + 2.0 * zs * le[0], wQ + 2.0 * zs * le[1]};
    for (int f2 = 0; f2 < 2; ++f2) {
      int q = 2 * e + f2;
      double T = C[q] * cs + D[q] * sn;
      double Tp = -C[q] * sn + D[q] * cs;
      double m = mu[f2];
      double vv = vf * vt * T;
      H[0] += m * (-vv);
      H[1] += m * vv;
      H[2] += m * vt * Tp;
      H[3] += m * vf * Tp;
      H[4] += m * (-vv);
      H[5] += m * (-vt * Tp);
      H[6] += m * (-vf * Tp);
      H[7] += m * 2.0 * A[q];
      H[8] += m * T;
      H[9] += m * 2.0 * B[q];
      const double* gr = le + (f2 == 0 ? 2 : 6);
      double c2 = 2.0 * zs;
      for (int a = 0; a < 4; ++a)
        for (int bq = a; bq < 4; ++bq) H[lh_index(a, bq)] += c2 * gr[a] * gr[bq];
    }
  }
  for (int q = 0; q < kLHsize; ++q) o[q] = H[q];
}

// Hessian of the Lagrangian at entry e of the pattern of K; lh = the
// scenario's line Hessians, hv = its Jacobian values of h
__device__ inline double w_gather_one(const DP& d, int e, double w, const double* lh,
                                      const double* hv) {
  // terms added in list order; the loads of kWb terms are issued before
  // they are added, so a long list costs one round of dependent loads per
  // kWb terms instead of one per term
  constexpr int kWb = 4;
  const int w0 = d.w_ptr[e], w1 = d.w_ptr[e + 1], p0 = d.wp_ptr[e], p1 = d.wp_ptr[e + 1];
  double acc = 0.0;
  for (int j = w0; j < w1; j += kWb) {
    double v[kWb];
#pragma unroll
    for (int q = 0; q < kWb; ++q) v[q] = lh[d.w_src[min(j + q, w1 - 1)]];
#pragma unroll
    for (int q = 0; q < kWb; ++q)
      if (j + q < w1) acc += v[q];
  }
  double prod = d.w_const[e];
  for (int j = p0; j < p1; j += kWb) {
    double cf[kWb], va[kWb], vb[kWb];
#pragma unroll
    for (int q = 0; q < kWb; ++q) {
      const int jj = min(j + q, p1 - 1);
      cf[q] = d.wp_coef[jj];
      va[q] = hv[d.wp_a[jj]];
      vb[q] = hv[d.wp_b[jj]];
    }
#pragma unroll
    for (int q = 0; q < kWb; ++q)
      if (j + q < p1) prod += cf[q] * va[q] * vb[q];
  }
  return acc + w * prod;
}

// line values and the bus / Jacobian values of one scenario in one
// workgroup, the line values in LDS (they feed only the gathers and, from
// HBM, the kernels after; both copies are written)
// kLvSplit workgroups per scenario: each evaluates every line of its
// scenario into LDS (the first also writes them out) and takes a strided
// share of the gathers, so the gathers of a scenario run on several CUs.
constexpr int kLvT = 512, kLvSplit = 4;

// Every kernel of the pass is a body taking the instance (d) and its block
// index, with two entry points: k_* (one instance, block index from the
// grid) and k_*_m (several instances: block b is block blk[b].bx of instance
// blk[b].inst, arguments from that instance's rkkt_iteration).
__device__ __forceinline__ void line_eval_gather_body(const DP& d, int bx, const double* x, const double* u) {
  extern __shared__ double lv[];
  const int k = bx / kLvSplit, part = bx % kLvSplit, tid = threadIdx.x;
  double* glv = d.LV + (long long)k * d.nl * kLVsize;
  for (int l = tid; l < d.nl; l += kLvT) {
    double* o = lv + (long long)l * kLVsize;
    line_eval_one(d, k, l, x, u, o);
    if (part == 0) {
#pragma unroll
      for (int q = 0; q < kLVsize; ++q) glv[(long long)l * kLVsize + q] = o[q];
    }
  }
  __syncthreads();
  double* gev = d.EV + (long long)k * d.n_ev;
  for (int e = part * kLvT + tid; e < d.n_ev; e += kLvSplit * kLvT) gev[e] = gather_ev_one(d, e, lv);
}

__device__ __forceinline__ void line_eval_body(const DP& d, int bx, const double* x, const double* u) {
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nl) return;
  line_eval_one(d, (int)(t / d.nl), (int)(t % d.nl), x, u, d.LV + t * kLVsize);
}

__device__ __forceinline__ void gather_ev_body(const DP& d, int bx) {
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.n_ev) return;
  int k = (int)(t / d.n_ev), e = (int)(t % d.n_ev);
  d.EV[t] = gather_ev_one(d, e, d.LV + (long long)k * d.nl * kLVsize);
}

__device__ __forceinline__ void assemble_body(const DP& d, int bx, const double* u, double w, double* f,
                                              double* gx, double* gu, double* g, double* h) {
  const int per = 2 * d.nx + d.m + d.nu;
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  const long long fb = assemble_f_base(d);
  if (t >= fb) {  // whole wavefronts (fb and the block size are multiples of 64)
    const long long r = t - fb;
    if (r < 64LL * d.N) objective_wave(d, (int)(r >> 6), (int)(r & 63), u, w, f);
    return;
  }
  if (t >= (long long)d.N * per) return;
  int k = (int)(t / per), i = (int)(t % per);
  assemble_one(d, k, i, u, w, gx, gu, g, h, d.EV + (long long)k * d.n_ev,
               d.LV + (long long)k * d.nl * kLVsize);
}

__device__ __forceinline__ void line_hess_body(const DP& d, int bx, const double* x, const double* u,
                                               const double* y, const double* z, double w) {
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nl) return;
  int k = (int)(t / d.nl), l = (int)(t % d.nl);
  line_hess_one(d, k, l, x, u, y, z, w, d.EV + (long long)k * d.n_ev, d.LV + t * kLVsize,
                d.LH + t * kLHsize);
}

__device__ __forceinline__ void w_gather_body(const DP& d, int bx, double w) {
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nnz_k) return;
  int k = (int)(t / d.nnz_k), e = (int)(t % d.nnz_k);
  d.W[t] = w_gather_one(d, e, w, d.LH + (long long)k * d.nl * kLHsize,
                        d.EV + (long long)k * d.n_ev + d.off_h);
}

// a4: entry e of K = W + H^T Sigma_s H + diag(Sigma_x) + delta_w on the x
// block; wv = W at e, hv = the scenario's Jacobian values of h
__device__ inline double condense_value(const DP& d, int k, int e, double wv, const double* hv,
                                        const double* sx, const double* ss, double dw) {
  const double* sk = ss + (long long)k * d.m;
  double acc = wv;
  for (int j = d.t_ptr[e]; j < d.t_ptr[e + 1]; ++j) acc += sk[d.t_row[j]] * hv[d.t_a[j]] * hv[d.t_b[j]];
  int r = d.k_row[e];
  if (r < d.nx && d.k_col[e] == r) acc += sx[(long long)k * d.nx + d.perm[r]] + dw;
  if (!isfinite(acc)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
  return acc;
}

__device__ __forceinline__ void condense_values_body(const DP& d, int bx, const double* sx, const double* ss,
                                                     double dw) {
  long long t = (long long)bx * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * d.nnz_k) return;
  int k = (int)(t / d.nnz_k), e = (int)(t % d.nnz_k);
  d.K[t] = condense_value(d, k, e, d.W[t], d.EV + (long long)k * d.n_ev + d.off_h, sx, ss, dw);
}

// The same values with the work of a scenario in d.cv_split workgroups of
// kCvT threads, each taking a contiguous range of the K entries: the
// scenario's sigma_s and H values and the range's triplet lists are staged
// in LDS first (all of their loads in flight together), so a value's terms
// cost LDS reads instead of dependent global gathers.  The terms are added
// in the same order as in condense_value.
constexpr int kCvT = 256;

__host__ __device__ inline long long cv_lds_bytes(const DP& d) {
  const int per = (d.nnz_k + d.cv_split - 1) / d.cv_split;
  return (8LL * (d.m + d.nnz_h) + 4LL * (per + 1 + 3LL * d.cv_nt) + 7) / 8 * 8;
}

__device__ __forceinline__ void condense_lds_body(const DP& d, int bx, const double* sx, const double* ss,
                                                  double dw) {
  const int G = d.cv_split, k = bx / G, g = bx % G, E = d.nnz_k;
  const int per = (E + G - 1) / G, e0 = min(E, g * per), e1 = min(E, e0 + per), ne = e1 - e0;
  const int tid = threadIdx.x;
  extern __shared__ double smem[];
  double* ssl = smem;
  double* hvl = ssl + d.m;
  int* tp = reinterpret_cast<int*>(hvl + d.nnz_h);
  int* tr = tp + per + 1;
  int* ta = tr + d.cv_nt;
  int* tb = ta + d.cv_nt;
  const int j0 = d.t_ptr[e0], nt = d.t_ptr[e1] - j0;
  const double* hv = d.EV + (long long)k * d.n_ev + d.off_h;
  const double* sk = ss + (long long)k * d.m;
  {
    constexpr int kB = 4;  // elements per thread and array in flight
    const int nmax = max(max(d.m, d.nnz_h), max(ne + 1, nt));
    for (int i0 = tid; i0 < nmax; i0 += kB * kCvT) {
      double vs[kB], vh[kB];
      int ip[kB], ir[kB], ia[kB], ib[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int i = i0 + u * kCvT;
        if (i < d.m) vs[u] = sk[i];
        if (i < d.nnz_h) vh[u] = hv[i];
        if (i <= ne) ip[u] = d.t_ptr[e0 + i];
        if (i < nt) {
          ir[u] = d.t_row[j0 + i];
          ia[u] = d.t_a[j0 + i];
          ib[u] = d.t_b[j0 + i];
        }
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int i = i0 + u * kCvT;
        if (i < d.m) ssl[i] = vs[u];
        if (i < d.nnz_h) hvl[i] = vh[u];
        if (i <= ne) tp[i] = ip[u] - j0;
        if (i < nt) {
          tr[i] = ir[u];
          ta[i] = ia[u];
          tb[i] = ib[u];
        }
      }
    }
  }
  __syncthreads();
  for (int e = e0 + tid; e < e1; e += kCvT) {
    const long long o = (long long)k * E + e;
    double acc = d.W[o];
    const int r = d.k_row[e], cdiag = d.k_col[e];
    const int ja = tp[e - e0], jb = tp[e - e0 + 1];
    for (int j = ja; j < jb; ++j) acc += ssl[tr[j]] * hvl[ta[j]] * hvl[tb[j]];
    if (r < d.nx && cdiag == r) acc += sx[(long long)k * d.nx + d.perm[r]] + dw;
    if (!isfinite(acc)) atomicCAS(d.status, 0, RKKT_ERR_NONFINITE);
    d.K[o] = acc;
  }
}

// ---- entry points: one instance
__global__ __launch_bounds__(kCvT) void k_condense_lds(DP d, const double* sx, const double* ss, double dw) {
  condense_lds_body(d, blockIdx.x, sx, ss, dw);
}
__global__ __launch_bounds__(kLvT) void k_line_eval_gather(DP d, const double* x, const double* u) {
  line_eval_gather_body(d, blockIdx.x, x, u);
}
__global__ void k_line_eval(DP d, const double* x, const double* u) { line_eval_body(d, blockIdx.x, x, u); }
__global__ void k_gather_ev(DP d) { gather_ev_body(d, blockIdx.x); }
__global__ void k_assemble(DP d, const double* u, double w, double* f, double* gx, double* gu, double* g,
                           double* h) {
  assemble_body(d, blockIdx.x, u, w, f, gx, gu, g, h);
}
__global__ void k_line_hess(DP d, const double* x, const double* u, const double* y, const double* z,
                            double w) {
  line_hess_body(d, blockIdx.x, x, u, y, z, w);
}
__global__ void k_w_gather(DP d, double w) { w_gather_body(d, blockIdx.x, w); }
__global__ void k_condense_values(DP d, const double* sx, const double* ss, double dw) {
  condense_values_body(d, blockIdx.x, sx, ss, dw);
}

// ---- entry points: several instances
#define RKKT_MULTI_PROLOGUE                          \
  const MultiBlk mb = blk[blockIdx.x];               \
  const DP& d = dps[mb.inst];                        \
  const rkkt_iteration& it = its[mb.inst];           \
  (void)it;
__global__ __launch_bounds__(kLvT) void k_line_eval_gather_m(const DP* __restrict__ dps,
                                                             const rkkt_iteration* __restrict__ its,
                                                             const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  line_eval_gather_body(d, mb.bx, it.x, it.u);
}
__global__ void k_line_eval_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                              const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  line_eval_body(d, mb.bx, it.x, it.u);
}
__global__ void k_gather_ev_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                              const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  gather_ev_body(d, mb.bx);
}
__global__ void k_assemble_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                             const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  assemble_body(d, mb.bx, it.u, it.obj_weight, it.f, it.grad_x, it.grad_u, it.g, it.h);
}
__global__ void k_line_hess_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                              const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  line_hess_body(d, mb.bx, it.x, it.u, it.y, it.z, it.obj_weight);
}
__global__ void k_w_gather_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                             const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  w_gather_body(d, mb.bx, it.obj_weight);
}
__global__ __launch_bounds__(kCvT) void k_condense_lds_m(const DP* __restrict__ dps,
                                                          const rkkt_iteration* __restrict__ its,
                                                          const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  condense_lds_body(d, mb.bx, it.sigma_x, it.sigma_s, it.delta_w);
}
__global__ void k_condense_values_m(const DP* __restrict__ dps, const rkkt_iteration* __restrict__ its,
                                    const MultiBlk* __restrict__ blk) {
  RKKT_MULTI_PROLOGUE
  condense_values_body(d, mb.bx, it.sigma_x, it.sigma_s, it.delta_w);
}

}  // namespace

__global__ void k_line_status(DP d, const double* st) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (long long)d.N * d.nl) d.lstat[t] = st ? st[t] : 1.0;
}

// copies the status into the handle (st == nullptr: every line in service)
void launch_line_status(const DP& d, const double* st, hipStream_t s) {
  const long long n = (long long)d.N * d.nl;
  k_line_status<<<grid_for(n), kBlock, 0, s>>>(d, st);
}

void launch_bus_loads(const DP& d, const double* pd, const double* qd, hipStream_t s) {
  long long n = (long long)d.N * d.nb;
  k_bus_loads<<<grid_for(n), kBlock, 0, s>>>(d, pd, qd);
}

// the fused line / gather kernel where a scenario's line values fit in LDS
static long long line_lds_bytes(const DP& d) { return 8LL * d.nl * kLVsize; }
static bool line_fused(const DP& d) { return line_lds_bytes(d) <= 96 * 1024; }

hipError_t configure_eval_kernels(const DP& d) {
  static int cur = 0;
  if (!line_fused(d) || line_lds_bytes(d) <= cur) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_line_eval_gather, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)line_lds_bytes(d));
  if (e == hipSuccess) cur = (int)line_lds_bytes(d);
  return e;
}

void launch_evaluate_values(const DP& d, const double* x, const double* u, hipStream_t s) {
  if (line_fused(d)) {
    k_line_eval_gather<<<d.N * kLvSplit, kLvT, (size_t)line_lds_bytes(d), s>>>(d, x, u);
    return;
  }
  long long nl = (long long)d.N * d.nl;
  k_line_eval<<<grid_for(nl), kBlock, 0, s>>>(d, x, u);
  long long ne = (long long)d.N * d.n_ev;
  k_gather_ev<<<grid_for(ne), kBlock, 0, s>>>(d);
}

void launch_evaluate_rest(const DP& d, const double* x, const double* u, const double* y,
                          const double* z, double w, double* f, double* gx, double* gu, double* g,
                          double* h, hipStream_t s) {
  k_assemble<<<grid_for(assemble_threads(d)), kBlock, 0, s>>>(d, u, w, f, gx, gu, g, h);
  long long nl = (long long)d.N * d.nl;
  k_line_hess<<<grid_for(nl), kBlock, 0, s>>>(d, x, u, y, z, w);
  long long nk = (long long)d.N * d.nnz_k;
  k_w_gather<<<grid_for(nk), kBlock, 0, s>>>(d, w);
}

void launch_evaluate(const DP& d, const double* x, const double* u, const double* y,
                     const double* z, double w, double* f, double* gx, double* gu, double* g,
                     double* h, hipStream_t s) {
  launch_evaluate_values(d, x, u, s);
  launch_evaluate_rest(d, x, u, y, z, w, f, gx, gu, g, h, s);
}

void launch_condense_values(const DP& d, const double* sx, const double* ss, double dw,
                            hipStream_t s) {
  if (d.cv_split > 0) {
    k_condense_lds<<<d.N * d.cv_split, kCvT, (size_t)cv_lds_bytes(d), s>>>(d, sx, ss, dw);
    return;
  }
  long long nk = (long long)d.N * d.nnz_k;
  k_condense_values<<<grid_for(nk), kBlock, 0, s>>>(d, sx, ss, dw);
}

// the launches of launch_evaluate_values, launch_evaluate_rest and
// launch_condense_values, in that order
void launches_eval(const DP& d, std::vector<Launch>& out) {
  auto add = [&](int key, int kernel, long long grid, int threads, long long lds) {
    out.push_back(Launch{key, kernel, 0, (int)grid, 1, threads, 0, lds});
  };
  if (line_fused(d)) {
    add(kStEvalValues * 4096, kKLineEvalGather, (long long)d.N * kLvSplit, kLvT, line_lds_bytes(d));
  } else {
    add(kStEvalValues * 4096, kKLineEval, grid_for((long long)d.N * d.nl), kBlock, 0);
    add(kStEvalValues * 4096 + 1, kKGatherEv, grid_for((long long)d.N * d.n_ev), kBlock, 0);
  }
  add(kStEvalRest * 4096, kKAssemble, grid_for(assemble_threads(d)), kBlock, 0);
  add(kStEvalRest * 4096 + 1, kKLineHess, grid_for((long long)d.N * d.nl), kBlock, 0);
  add(kStEvalRest * 4096 + 2, kKWGather, grid_for((long long)d.N * d.nnz_k), kBlock, 0);
  if (d.cv_split > 0)
    add(kStCondense * 4096, kKCondenseLds, (long long)d.N * d.cv_split, kCvT, cv_lds_bytes(d));
  else
    add(kStCondense * 4096, kKCondense, grid_for((long long)d.N * d.nnz_k), kBlock, 0);
}

hipError_t multi_eval(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                      const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled) {
  *handled = true;
  if (prepare) {
    static int cur = 0;
    if (l.kernel != kKLineEvalGather || lds <= cur) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_line_eval_gather_m,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) cur = (int)lds;
    return e;
  }
  switch (l.kernel) {
    case kKLineEvalGather: k_line_eval_gather_m<<<nblk, kLvT, (size_t)lds, s>>>(dps, its, blk); break;
    case kKLineEval: k_line_eval_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKGatherEv: k_gather_ev_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKAssemble: k_assemble_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKLineHess: k_line_hess_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKWGather: k_w_gather_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKCondense: k_condense_values_m<<<nblk, kBlock, 0, s>>>(dps, its, blk); break;
    case kKCondenseLds: k_condense_lds_m<<<nblk, kCvT, (size_t)lds, s>>>(dps, its, blk); break;
    default: *handled = false;
  }
  return hipSuccess;
}

}  // namespace rkkt
