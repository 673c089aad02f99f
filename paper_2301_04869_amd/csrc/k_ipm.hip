// Interior-point glue around the hot path: IPM diagonals and residuals of the
// augmented system (paper: KKT conditions with barrier homotopy, residuals
// r1..r4), the scaled KKT error, the barrier objective and constraint
// violation of the filter line search, fraction-to-boundary step lengths and
// the iterate update.  Reductions run in one workgroup with a fixed tree, so
// every scalar is reproducible run to run.
#include "ipm.h"

namespace rkkt {

namespace {

constexpr int kBlock = 256;
constexpr int kRed = 1024;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline bool fin(double v) { return isfinite(v); }

// Sigma contribution and barrier gradient of one boxed variable
__device__ inline void box_terms(double v, double lo, double hi, double zl, double zu, double mu,
                                 double* sigma, double* bgrad, double* bdual) {
  double sg = 0.0, bg = 0.0, bd = 0.0;
  if (fin(lo)) { double dl = v - lo; sg += zl / dl; bg -= mu / dl; bd -= zl; }
  if (fin(hi)) { double du = hi - v; sg += zu / du; bg += mu / du; bd += zu; }
  *sigma = sg;
  *bgrad = bg;
  *bdual = bd;
}

// r1x, dx, Sigma_x (x part); per-scenario u gradient of the Lagrangian (u part);
// r2, ds, r4, Sigma_s (s part)
__global__ void k_resid(DP d, IpmDev s, double mu) {
  const long long per = (long long)d.nx + d.nu + d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)d.N * per) return;
  const int k = (int)(t / per);
  int i = (int)(t % per);
  const double* ev = d.EV + (long long)k * d.n_ev;
  const double* hv = ev + d.off_h;
  const double* yk = s.y + (long long)k * d.nx;
  const double* zk = s.z + (long long)k * d.m;
  if (i < d.nx) {
    const int ih = d.pinv[i];
    double acc = s.gx[(long long)k * d.nx + i];
    for (int j = d.gxc_ptr[ih]; j < d.gxc_ptr[ih + 1]; ++j)
      acc += ev[d.off_gx + d.gxc_pos[j]] * yk[d.perm[d.gxc_row[j]]];
    for (int j = d.ht_ptr[ih]; j < d.ht_ptr[ih + 1]; ++j) acc += hv[d.ht_pos[j]] * zk[d.ht_row[j]];
    const long long q = (long long)k * d.nx + i;
    double sg, bg, bd;
    box_terms(s.x[q], s.xl[i], s.xu[i], s.zlx[q], s.zux[q], mu, &sg, &bg, &bd);
    s.sx[q] = sg;
    s.r1x[q] = acc + bg;
    s.dx[q] = acc + bd;
    s.r3[q] = s.g[q];
    return;
  }
  i -= d.nx;
  if (i < d.nu) {
    double acc = s.gu[(long long)k * d.nu + i];
    for (int j = d.guc_ptr[i]; j < d.guc_ptr[i + 1]; ++j)
      acc += ev[d.off_gu + d.guc_pos[j]] * yk[d.perm[d.guc_row[j]]];
    const int v = d.nx + i;
    for (int j = d.ht_ptr[v]; j < d.ht_ptr[v + 1]; ++j) acc += hv[d.ht_pos[j]] * zk[d.ht_row[j]];
    s.cu[(long long)k * d.nu + i] = acc;
    return;
  }
  i -= d.nu;
  const long long q = (long long)k * d.m + i;
  double sg, bg, bd;
  box_terms(s.s[q], s.sl[i], s.su[i], s.zls[q], s.zus[q], mu, &sg, &bg, &bd);
  s.ss[q] = sg;
  s.r2[q] = zk[i] + bg;
  s.ds[q] = zk[i] + bd;
  s.r4[q] = s.h[q] + s.s[q];
}

__global__ void k_resid_u(DP d, IpmDev s, double mu) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.nu) return;
  double acc = 0.0;
  for (int k = 0; k < d.N; ++k) acc += s.cu[(long long)k * d.nu + c];
  double sg, bg, bd;
  box_terms(s.u[c], s.ul[c], s.uu[c], s.zlu[c], s.zuu[c], mu, &sg, &bg, &bd);
  s.sgu[c] = sg;
  s.r1u[c] = acc + bg;
  s.du[c] = acc + bd;
}

// block reductions in one workgroup (fixed tree)
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_min(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// complementarity of one boxed variable
__device__ inline void comp_terms(double v, double lo, double hi, double zl, double zu, double mu,
                                  double* cm, double* c0, double* zs) {
  if (fin(lo)) {
    double a = (v - lo) * zl;
    *cm = fmax(*cm, fabs(a - mu));
    *c0 = fmax(*c0, fabs(a));
    *zs += fabs(zl);
  }
  if (fin(hi)) {
    double a = (hi - v) * zu;
    *cm = fmax(*cm, fabs(a - mu));
    *c0 = fmax(*c0, fabs(a));
    *zs += fabs(zu);
  }
}

// out: [0] max dual, [1] max primal, [2] max |comp - mu|, [3] max |comp|,
//      [4] sum |y| + |z|, [5] sum |bound duals|
__global__ __launch_bounds__(kRed) void k_kkt_scalars(DP d, IpmDev s, double mu, double* out) {
  __shared__ double sh[kRed];
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  double dmax = 0.0, pmax = 0.0, cm = 0.0, c0 = 0.0, ysum = 0.0, zs = 0.0;
  for (long long q = threadIdx.x; q < nxN; q += kRed) {
    const int i = (int)(q % d.nx);
    dmax = fmax(dmax, fabs(s.dx[q]));
    pmax = fmax(pmax, fabs(s.g[q]));
    ysum += fabs(s.y[q]);
    comp_terms(s.x[q], s.xl[i], s.xu[i], s.zlx[q], s.zux[q], mu, &cm, &c0, &zs);
  }
  for (long long q = threadIdx.x; q < nmN; q += kRed) {
    const int i = (int)(q % d.m);
    dmax = fmax(dmax, fabs(s.ds[q]));
    pmax = fmax(pmax, fabs(s.h[q] + s.s[q]));
    ysum += fabs(s.z[q]);
    comp_terms(s.s[q], s.sl[i], s.su[i], s.zls[q], s.zus[q], mu, &cm, &c0, &zs);
  }
  for (int c = threadIdx.x; c < d.nu; c += kRed) {
    dmax = fmax(dmax, fabs(s.du[c]));
    comp_terms(s.u[c], s.ul[c], s.uu[c], s.zlu[c], s.zuu[c], mu, &cm, &c0, &zs);
  }
  dmax = block_max(dmax, sh);
  pmax = block_max(pmax, sh);
  cm = block_max(cm, sh);
  c0 = block_max(c0, sh);
  ysum = block_sum(ysum, sh);
  zs = block_sum(zs, sh);
  if (threadIdx.x == 0) {
    out[0] = dmax; out[1] = pmax; out[2] = cm; out[3] = c0; out[4] = ysum; out[5] = zs;
  }
}

__device__ inline double logbox(double v, double lo, double hi, int* bad) {
  double r = 0.0;
  if (fin(lo)) { double a = v - lo; if (!(a > 0.0)) *bad = 1; else r += log(a); }
  if (fin(hi)) { double b = hi - v; if (!(b > 0.0)) *bad = 1; else r += log(b); }
  return r;
}

// merit of a primal point (x, u, s) with its f, g, h:
// out: [0] sum f, [1] theta = |g|_1 + |h + s|_1, [2] log-barrier sum, [3] bad (1 if outside)
__global__ __launch_bounds__(kRed) void k_merit(DP d, IpmDev s, const double* x, const double* u,
                                                const double* sv, const double* f, const double* g,
                                                const double* h, double* out) {
  __shared__ double sh[kRed];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  int bad = 0;
  double fs = 0.0, th = 0.0, lg = 0.0;
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  for (long long q = threadIdx.x; q < nxN; q += kRed) {
    th += fabs(g[q]);
    lg += logbox(x[q], s.xl[q % d.nx], s.xu[q % d.nx], &bad);
  }
  for (long long q = threadIdx.x; q < nmN; q += kRed) {
    th += fabs(h[q] + sv[q]);
    lg += logbox(sv[q], s.sl[q % d.m], s.su[q % d.m], &bad);
  }
  for (int c = threadIdx.x; c < d.nu; c += kRed) lg += logbox(u[c], s.ul[c], s.uu[c], &bad);
  for (int k = threadIdx.x; k < d.N; k += kRed) fs += f[k];
  if (bad) atomicOr(&sbad, 1);
  fs = block_sum(fs, sh);
  th = block_sum(th, sh);
  lg = block_sum(lg, sh);
  if (threadIdx.x == 0) { out[0] = fs; out[1] = th; out[2] = lg; out[3] = sbad ? 1.0 : 0.0; }
}

// bound-dual steps: p_zL = mu/(v-l) - zL - zL/(v-l) p, p_zU = mu/(u-v) - zU + zU/(u-v) p
__device__ inline void dual_step(double v, double p, double lo, double hi, double zl, double zu,
                                 double mu, double* pl, double* pu) {
  *pl = 0.0;
  *pu = 0.0;
  if (fin(lo)) { double a = v - lo; *pl = mu / a - zl - zl / a * p; }
  if (fin(hi)) { double b = hi - v; *pu = mu / b - zu + zu / b * p; }
}

__global__ void k_dual_steps(DP d, IpmDev s, double mu) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    dual_step(s.x[t], s.px[t], s.xl[i], s.xu[i], s.zlx[t], s.zux[t], mu, &s.pzlx[t], &s.pzux[t]);
    return;
  }
  t -= nxN;
  if (t < nmN) {
    const int i = (int)(t % d.m);
    dual_step(s.s[t], s.ps[t], s.sl[i], s.su[i], s.zls[t], s.zus[t], mu, &s.pzls[t], &s.pzus[t]);
    return;
  }
  t -= nmN;
  if (t < d.nu) {
    const int c = (int)t;
    dual_step(s.u[c], s.pu[c], s.ul[c], s.uu[c], s.zlu[c], s.zuu[c], mu, &s.pzlu[c], &s.pzuu[c]);
  }
}

__device__ inline double primal_ratio(double v, double p, double lo, double hi, double tau) {
  double a = 1.0;
  if (fin(lo) && p < 0.0) a = fmin(a, -tau * (v - lo) / p);
  if (fin(hi) && p > 0.0) a = fmin(a, tau * (hi - v) / p);
  return a;
}

__device__ inline double dual_ratio(double z, double p, double tau) {
  return p < 0.0 ? fmin(1.0, -tau * z / p) : 1.0;
}

// out: [0] alpha_max primal, [1] alpha_z, [2] grad(phi)^T d
__global__ __launch_bounds__(kRed) void k_step_scalars(DP d, IpmDev s, double mu, double tau,
                                                       double* out) {
  __shared__ double sh[kRed];
  double ap = 1.0, az = 1.0, dphi = 0.0;
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  for (long long q = threadIdx.x; q < nxN; q += kRed) {
    const int i = (int)(q % d.nx);
    ap = fmin(ap, primal_ratio(s.x[q], s.px[q], s.xl[i], s.xu[i], tau));
    az = fmin(az, fmin(dual_ratio(s.zlx[q], s.pzlx[q], tau), dual_ratio(s.zux[q], s.pzux[q], tau)));
    double sg, bg, bd;
    box_terms(s.x[q], s.xl[i], s.xu[i], 0.0, 0.0, mu, &sg, &bg, &bd);
    dphi += (s.gx[q] + bg) * s.px[q];
  }
  for (long long q = threadIdx.x; q < nmN; q += kRed) {
    const int i = (int)(q % d.m);
    ap = fmin(ap, primal_ratio(s.s[q], s.ps[q], s.sl[i], s.su[i], tau));
    az = fmin(az, fmin(dual_ratio(s.zls[q], s.pzls[q], tau), dual_ratio(s.zus[q], s.pzus[q], tau)));
    double sg, bg, bd;
    box_terms(s.s[q], s.sl[i], s.su[i], 0.0, 0.0, mu, &sg, &bg, &bd);
    dphi += bg * s.ps[q];
  }
  for (int c = threadIdx.x; c < d.nu; c += kRed) {
    ap = fmin(ap, primal_ratio(s.u[c], s.pu[c], s.ul[c], s.uu[c], tau));
    az = fmin(az, fmin(dual_ratio(s.zlu[c], s.pzlu[c], tau), dual_ratio(s.zuu[c], s.pzuu[c], tau)));
    double gsum = 0.0;
    for (int k = 0; k < d.N; ++k) gsum += s.gu[(long long)k * d.nu + c];
    double sg, bg, bd;
    box_terms(s.u[c], s.ul[c], s.uu[c], 0.0, 0.0, mu, &sg, &bg, &bd);
    dphi += (gsum + bg) * s.pu[c];
  }
  ap = block_min(ap, sh);
  az = block_min(az, sh);
  dphi = block_sum(dphi, sh);
  if (threadIdx.x == 0) { out[0] = ap; out[1] = az; out[2] = dphi; }
}

__global__ void k_trial(DP d, IpmDev s, double alpha) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) { s.xt[t] = s.x[t] + alpha * s.px[t]; return; }
  t -= nxN;
  if (t < nmN) { s.st[t] = s.s[t] + alpha * s.ps[t]; return; }
  t -= nmN;
  if (t < d.nu) s.ut[t] = s.u[t] + alpha * s.pu[t];
}

__device__ inline void safeguard(double v, double lo, double hi, double mu, double ks, double* zl,
                                 double* zu) {
  if (fin(lo)) { double a = v - lo; *zl = fmax(fmin(*zl, ks * mu / a), mu / (ks * a)); } else *zl = 0.0;
  if (fin(hi)) { double b = hi - v; *zu = fmax(fmin(*zu, ks * mu / b), mu / (ks * b)); } else *zu = 0.0;
}

__global__ void k_accept(DP d, IpmDev s, double alpha, double alpha_z, double mu, double ks) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    s.x[t] += alpha * s.px[t];
    s.y[t] += alpha * s.py[t];
    double zl = s.zlx[t] + alpha_z * s.pzlx[t], zu = s.zux[t] + alpha_z * s.pzux[t];
    safeguard(s.x[t], s.xl[i], s.xu[i], mu, ks, &zl, &zu);
    s.zlx[t] = zl;
    s.zux[t] = zu;
    return;
  }
  t -= nxN;
  if (t < nmN) {
    const int i = (int)(t % d.m);
    s.s[t] += alpha * s.ps[t];
    s.z[t] += alpha * s.pz[t];
    double zl = s.zls[t] + alpha_z * s.pzls[t], zu = s.zus[t] + alpha_z * s.pzus[t];
    safeguard(s.s[t], s.sl[i], s.su[i], mu, ks, &zl, &zu);
    s.zls[t] = zl;
    s.zus[t] = zu;
    return;
  }
  t -= nmN;
  if (t < d.nu) {
    const int c = (int)t;
    s.u[c] += alpha * s.pu[c];
    double zl = s.zlu[c] + alpha_z * s.pzlu[c], zu = s.zuu[c] + alpha_z * s.pzuu[c];
    safeguard(s.u[c], s.ul[c], s.uu[c], mu, ks, &zl, &zu);
    s.zlu[c] = zl;
    s.zuu[c] = zu;
  }
}

// push v inside [lo, hi]: distance min(k1 max(1,|bound|), k2 (hi - lo))
__device__ inline double push(double v, double lo, double hi, double k1, double k2) {
  double pl = fin(lo) ? k1 * fmax(1.0, fabs(lo)) : 0.0;
  double pu = fin(hi) ? k1 * fmax(1.0, fabs(hi)) : 0.0;
  if (fin(lo) && fin(hi)) { pl = fmin(pl, k2 * (hi - lo)); pu = fmin(pu, k2 * (hi - lo)); }
  if (fin(lo)) v = fmax(v, lo + pl);
  if (fin(hi)) v = fmin(v, hi - pu);
  return v;
}

// start point: theta 0, V 1, Pg mid-range, pushed inside; y = z = 0; bound duals 1
__global__ void k_init_primal(DP d, IpmDev s, double k1, double k2) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    double v0 = i < d.nb - 1 ? 0.0 : 1.0;
    s.x[t] = push(v0, s.xl[i], s.xu[i], k1, k2);
    s.y[t] = 0.0;
    s.zlx[t] = fin(s.xl[i]) ? 1.0 : 0.0;
    s.zux[t] = fin(s.xu[i]) ? 1.0 : 0.0;
    return;
  }
  t -= nxN;
  if (t < nmN) {
    const int i = (int)(t % d.m);
    s.z[t] = 0.0;
    s.s[t] = 0.0;
    s.zls[t] = fin(s.sl[i]) ? 1.0 : 0.0;
    s.zus[t] = fin(s.su[i]) ? 1.0 : 0.0;
    return;
  }
  t -= nmN;
  if (t < d.nu) {
    const int c = (int)t;
    double v0 = c < d.ng ? 1.0 : 0.5 * (s.ul[c] + s.uu[c]);
    s.u[c] = push(v0, s.ul[c], s.uu[c], k1, k2);
    s.zlu[c] = fin(s.ul[c]) ? 1.0 : 0.0;
    s.zuu[c] = fin(s.uu[c]) ? 1.0 : 0.0;
  }
}

__global__ void k_init_slack(DP d, IpmDev s, double k1, double k2) {
  const long long nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nmN) return;
  const int i = (int)(t % d.m);
  s.s[t] = push(-s.h[t], s.sl[i], s.su[i], k1, k2);
}

// warm start, primal part: x0, u0 pushed into the boxes
__global__ void k_warm_primal(DP d, IpmDev s, const double* x0, const double* u0, double k1, double k2) {
  const long long nxN = (long long)d.N * d.nx;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    s.x[t] = push(x0[t], s.xl[i], s.xu[i], k1, k2);
  } else if (t - nxN < d.nu) {
    const int c = (int)(t - nxN);
    s.u[c] = push(u0[c], s.ul[c], s.uu[c], k1, k2);
  }
}

// warm start, dual part: y = mult y0, z = mult z0, and every bound
// multiplier from complementarity at mu0 (mu0 / gap), after the slacks
__global__ void k_warm_duals(DP d, IpmDev s, const double* y0, const double* z0, double mult, double mu0) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    s.y[t] = mult * y0[t];
    s.zlx[t] = fin(s.xl[i]) ? mu0 / (s.x[t] - s.xl[i]) : 0.0;
    s.zux[t] = fin(s.xu[i]) ? mu0 / (s.xu[i] - s.x[t]) : 0.0;
    return;
  }
  t -= nxN;
  if (t < nmN) {
    const int i = (int)(t % d.m);
    s.z[t] = mult * z0[t];
    s.zls[t] = fin(s.sl[i]) ? mu0 / (s.s[t] - s.sl[i]) : 0.0;
    s.zus[t] = fin(s.su[i]) ? mu0 / (s.su[i] - s.s[t]) : 0.0;
    return;
  }
  t -= nmN;
  if (t < d.nu) {
    const int c = (int)t;
    s.zlu[c] = fin(s.ul[c]) ? mu0 / (s.u[c] - s.ul[c]) : 0.0;
    s.zuu[c] = fin(s.uu[c]) ? mu0 / (s.uu[c] - s.u[c]) : 0.0;
  }
}

// warm start, bound multipliers implied by stationarity (after k_resid with
// the complementarity multipliers of k_warm_duals): v = the derivative of the
// Lagrangian without bound terms (dual infeasibility plus the current bound
// terms), lower multiplier mu0 / gap + max(v, 0), upper mu0 / gap + max(-v, 0)
__device__ inline void implied_pair(double val, double lo, double hi, double v, double mu0, double* zl,
                                    double* zu) {
  *zl = fin(lo) ? mu0 / (val - lo) + fmax(v, 0.0) : 0.0;
  *zu = fin(hi) ? mu0 / (hi - val) + fmax(-v, 0.0) : 0.0;
}

__global__ void k_warm_implied(DP d, IpmDev s, double mu0) {
  const long long nxN = (long long)d.N * d.nx, nmN = (long long)d.N * d.m;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nxN) {
    const int i = (int)(t % d.nx);
    const double v = s.dx[t] + s.zlx[t] - s.zux[t];
    implied_pair(s.x[t], s.xl[i], s.xu[i], v, mu0, &s.zlx[t], &s.zux[t]);
    return;
  }
  t -= nxN;
  if (t < nmN) {
    const int i = (int)(t % d.m);
    const double v = s.ds[t] + s.zls[t] - s.zus[t];
    implied_pair(s.s[t], s.sl[i], s.su[i], v, mu0, &s.zls[t], &s.zus[t]);
    return;
  }
  t -= nmN;
  if (t < d.nu) {
    const int c = (int)t;
    const double v = s.du[c] + s.zlu[c] - s.zuu[c];
    implied_pair(s.u[c], s.ul[c], s.uu[c], v, mu0, &s.zlu[c], &s.zuu[c]);
  }
}

// out[0] = max(max |grad_x f_i|, max |sum_i grad_u f_i|)
__global__ __launch_bounds__(kRed) void k_grad_max(DP d, IpmDev s, double* out) {
  __shared__ double sh[kRed];
  double mx = 0.0;
  const long long nxN = (long long)d.N * d.nx;
  for (long long q = threadIdx.x; q < nxN; q += kRed) mx = fmax(mx, fabs(s.gx[q]));
  for (int c = threadIdx.x; c < d.nu; c += kRed) {
    double acc = 0.0;
    for (int k = 0; k < d.N; ++k) acc += s.gu[(long long)k * d.nu + c];
    mx = fmax(mx, fabs(acc));
  }
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) out[0] = mx;
}

}  // namespace

void ipm_resid(const DP& d, const IpmDev& s, double mu, hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.nu + d.m);
  k_resid<<<grid_for(n), kBlock, 0, st>>>(d, s, mu);
  k_resid_u<<<grid_for(d.nu), kBlock, 0, st>>>(d, s, mu);
}

void ipm_kkt_scalars(const DP& d, const IpmDev& s, double mu, double* out, hipStream_t st) {
  k_kkt_scalars<<<1, kRed, 0, st>>>(d, s, mu, out);
}

void ipm_merit(const DP& d, const IpmDev& s, bool trial, double* out, hipStream_t st) {
  if (trial) k_merit<<<1, kRed, 0, st>>>(d, s, s.xt, s.ut, s.st, s.ft, s.gt, s.ht, out);
  else k_merit<<<1, kRed, 0, st>>>(d, s, s.x, s.u, s.s, s.f, s.g, s.h, out);
}

void ipm_step_scalars(const DP& d, const IpmDev& s, double mu, double tau, double* out,
                      hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_dual_steps<<<grid_for(n), kBlock, 0, st>>>(d, s, mu);
  k_step_scalars<<<1, kRed, 0, st>>>(d, s, mu, tau, out);
}

void ipm_trial(const DP& d, const IpmDev& s, double alpha, hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_trial<<<grid_for(n), kBlock, 0, st>>>(d, s, alpha);
}

void ipm_accept(const DP& d, const IpmDev& s, double alpha, double alpha_z, double mu, double ks,
                hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_accept<<<grid_for(n), kBlock, 0, st>>>(d, s, alpha, alpha_z, mu, ks);
}

void ipm_init_primal(const DP& d, const IpmDev& s, double k1, double k2, hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_init_primal<<<grid_for(n), kBlock, 0, st>>>(d, s, k1, k2);
}

void ipm_init_slack(const DP& d, const IpmDev& s, double k1, double k2, hipStream_t st) {
  const long long n = (long long)d.N * d.m;
  k_init_slack<<<grid_for(n), kBlock, 0, st>>>(d, s, k1, k2);
}

void ipm_warm_primal(const DP& d, const IpmDev& s, const double* x0, const double* u0, double k1, double k2,
                     hipStream_t st) {
  const long long n = (long long)d.N * d.nx + d.nu;
  k_warm_primal<<<grid_for(n), kBlock, 0, st>>>(d, s, x0, u0, k1, k2);
}

void ipm_warm_implied(const DP& d, const IpmDev& s, double mu0, hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_warm_implied<<<grid_for(n), kBlock, 0, st>>>(d, s, mu0);
}

void ipm_warm_duals(const DP& d, const IpmDev& s, const double* y0, const double* z0, double mult, double mu0,
                    hipStream_t st) {
  const long long n = (long long)d.N * (d.nx + d.m) + d.nu;
  k_warm_duals<<<grid_for(n), kBlock, 0, st>>>(d, s, y0, z0, mult, mu0);
}

void ipm_grad_max(const DP& d, const IpmDev& s, double* out, hipStream_t st) {
  k_grad_max<<<1, kRed, 0, st>>>(d, s, out);
}

}  // namespace rkkt
