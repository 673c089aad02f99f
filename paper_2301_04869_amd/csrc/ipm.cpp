// Interior-point driver on the device: the outer loop around evaluate /
// condense / factor / step.  The paper runs its linear algebra inside an
// IPOPT-style primal-dual solver and does not specify the loop; the rules
// here are the published filter line-search method (Waechter & Biegler 2006)
// with the same simplifications as the CPU oracle's loop: start point pushed
// into the boxes, monotone barrier update, fraction to boundary, inertia
// correction on the reduced matrix, filter line search with switching and
// Armijo conditions, no second-order correction and no restoration phase.
// Every vector operation runs in the kernels of k_ipm.hip; the host reads a
// few scalars per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <utility>
#include <vector>

#include "handle.h"

namespace {

struct Opt {
  double tol = 1e-8, mu0 = 0.1, kappa1 = 1e-2, kappa2 = 1e-2, tau_min = 0.99;
  double kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5, s_max = 100.0;
  double delta0 = 1e-4, delta_min = 1e-20, delta_max = 1e20, kw_minus = 1.0 / 3.0;
  double kw_plus = 8.0, kw_plus_bar = 100.0;
  double gamma_theta = 1e-5, gamma_phi = 1e-8, s_theta = 1.1, s_phi = 2.3, delta_sw = 1.0;
  double eta_phi = 1e-8, gamma_alpha = 0.05, kappa_sigma = 1e10, obj_grad_max = 100.0;
  int max_iter = 200;
  double kappa_warm = 1e-6;  // interior push of a warm start point
};

template <typename T>
hipError_t ialloc(rkkt_problem* p, T** out, size_t n) {
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, (n ? n : 1) * sizeof(T));
  if (e != hipSuccess) return e;
  p->ipm_allocs.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return hipSuccess;
}

template <typename T>
hipError_t iupload(rkkt_problem* p, const T** out, const std::vector<T>& v) {
  T* ptr = nullptr;
  hipError_t e = ialloc(p, &ptr, v.size());
  if (e == hipSuccess) e = hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  *out = ptr;
  return e;
}

hipError_t ipm_workspace(rkkt_problem* p) {
  if (p->ipm_ready) return hipSuccess;
  const rkkt::Sym& sy = p->sym;
  rkkt::IpmDev& s = p->ipm;
  const size_t N = sy.N, nx = sy.nx, nu = sy.nu, m = sy.m;
  hipError_t e;
#define A(ptr, n) \
  if ((e = ialloc(p, &s.ptr, n)) != hipSuccess) return e;
  if ((e = iupload(p, &s.xl, sy.xl)) != hipSuccess) return e;
  if ((e = iupload(p, &s.xu, sy.xu)) != hipSuccess) return e;
  if ((e = iupload(p, &s.ul, sy.ul)) != hipSuccess) return e;
  if ((e = iupload(p, &s.uu, sy.uu)) != hipSuccess) return e;
  if ((e = iupload(p, &s.sl, sy.sl)) != hipSuccess) return e;
  if ((e = iupload(p, &s.su, sy.su)) != hipSuccess) return e;
  A(x, N * nx) A(u, nu) A(s, N * m) A(y, N * nx) A(z, N * m)
  A(zlx, N * nx) A(zux, N * nx) A(zlu, nu) A(zuu, nu) A(zls, N * m) A(zus, N * m)
  A(xt, N * nx) A(ut, nu) A(st, N * m)
  A(f, N) A(gx, N * nx) A(gu, N * nu) A(g, N * nx) A(h, N * m)
  A(ft, N) A(gxt, N * nx) A(gut, N * nu) A(gt, N * nx) A(ht, N * m)
  A(sx, N * nx) A(sgu, nu) A(ss, N * m)
  A(r1x, N * nx) A(r1u, nu) A(r2, N * m) A(r3, N * nx) A(r4, N * m)
  A(dx, N * nx) A(du, nu) A(ds, N * m) A(cu, N * nu)
  A(px, N * nx) A(pu, nu) A(ps, N * m) A(py, N * nx) A(pz, N * m)
  A(pzlx, N * nx) A(pzux, N * nx) A(pzlu, nu) A(pzuu, nu) A(pzls, N * m) A(pzus, N * m)
  A(khat, nu * nu) A(chol, nu * nu) A(info, 1) A(scal, 32)
#undef A
  p->ipm_ready = true;
  return hipSuccess;
}

}  // namespace

// warm: x0, u0, y0, z0 (device) or all null for the cold start
static int solve_impl(rkkt_problem* p, const rkkt_ipm_options* uopt, const double* x0, const double* u0,
                      const double* y0, const double* z0, double* x_out, double* u_out, double* y_out,
                      double* z_out, double* s_out, rkkt_ipm_result* res, hipStream_t st) {
  if (!p || !res) return RKKT_ERR_ARG;
  const bool warm = x0 != nullptr;
  Opt o;
  int verbose = 0;
  bool warm_implied = true;
  if (uopt) {
    if (uopt->tol > 0) o.tol = uopt->tol;
    if (uopt->max_iter >= 0) o.max_iter = uopt->max_iter;
    if (uopt->mu0 > 0) o.mu0 = uopt->mu0;
    verbose = uopt->verbose;
    warm_implied = uopt->warm_duals == 0;
  }
  *res = rkkt_ipm_result{};
  hipError_t e = ipm_workspace(p);
  if (e != hipSuccess) {
    p->err = std::string("rkkt_solve: workspace: ") + hipGetErrorString(e);
    return RKKT_ERR_NOMEM;
  }
  const rkkt::DP& d = p->d;
  rkkt::IpmDev& s = p->ipm;
  const int N = d.N;
  double hs[32];
  auto fetch = [&](int n) -> hipError_t {
    hipError_t r = hipMemcpyAsync(hs, s.scal, n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    return r;
  };
  auto eval = [&](bool trial, double w) -> int {
    if (trial)
      return rkkt_evaluate(p, s.xt, s.ut, s.y, s.z, w, s.ft, s.gxt, s.gut, s.gt, s.ht, st);
    return rkkt_evaluate(p, s.x, s.u, s.y, s.z, w, s.f, s.gx, s.gu, s.g, s.h, st);
  };
  const double n_var = (double)N * (d.nx + d.m) + d.nu;
  const double n_con = (double)N * (d.nx + d.m);
  auto kkt_err = [&](double mu, double* e_mu, double* e_0) -> hipError_t {
    rkkt::ipm_kkt_scalars(d, s, mu, s.scal, st);
    hipError_t r = fetch(6);
    if (r != hipSuccess) return r;
    const double sd = std::max(o.s_max, (hs[4] + hs[5]) / (n_var + n_con)) / o.s_max;
    const double sc = std::max(o.s_max, hs[5] / n_var) / o.s_max;
    *e_mu = std::max({hs[0] / sd, hs[1], hs[2] / sc});
    *e_0 = std::max({hs[0] / sd, hs[1], hs[3] / sc});
    return hipSuccess;
  };
  int rc;
#define CK(call)                                                      \
  do {                                                                \
    hipError_t _e = (call);                                           \
    if (_e != hipSuccess) {                                           \
      p->err = std::string("rkkt_solve: ") + hipGetErrorString(_e);   \
      res->status = 4;                                                \
      return RKKT_ERR_HIP;                                            \
    }                                                                 \
  } while (0)
#define CR(call)                \
  do {                          \
    rc = (call);                \
    if (rc != RKKT_OK) {        \
      res->status = 4;          \
      return rc;                \
    }                           \
  } while (0)

  // ---- start point and objective scaling
  rkkt::ipm_init_primal(d, s, o.kappa1, o.kappa2, st);
  if (warm) rkkt::ipm_warm_primal(d, s, x0, u0, o.kappa_warm, o.kappa_warm, st);
  CK(hipGetLastError());
  CR(eval(false, 1.0 / N));
  rkkt::ipm_init_slack(d, s, warm ? o.kappa_warm : o.kappa1, warm ? o.kappa_warm : o.kappa2, st);
  rkkt::ipm_grad_max(d, s, s.scal, st);
  CK(fetch(1));
  const double scale = hs[0] > 0 ? std::min(1.0, o.obj_grad_max / hs[0]) : 1.0;
  const double w = scale / N;
  // warm multipliers are given for objective weight 1 / N: scale them by w N
  if (warm) rkkt::ipm_warm_duals(d, s, y0, z0, w * N, o.mu0, st);
  double mu = o.mu0;
  double tau = std::max(o.tau_min, 1.0 - mu);
  CR(eval(false, w));
  if (warm && warm_implied) {
    rkkt::ipm_resid(d, s, mu, st);
    rkkt::ipm_warm_implied(d, s, o.mu0, st);
  }
  rkkt::ipm_resid(d, s, mu, st);
  rkkt::ipm_merit(d, s, false, s.scal, st);
  CK(fetch(4));
  const double th0 = hs[1];
  const double th_max = 1e4 * std::max(1.0, th0), th_min = 1e-4 * std::max(1.0, th0);
  std::vector<std::pair<double, double>> filt;
  double delta_last = 0.0;
  int status = 1, k = 0, nfac = 0;
  double e0 = 0.0, emu = 0.0;
  for (k = 0; k <= o.max_iter; ++k) {
    rkkt::ipm_resid(d, s, mu, st);
    CK(kkt_err(mu, &emu, &e0));
    if (e0 <= o.tol) { status = 0; break; }
    if (k == o.max_iter) break;
    while (emu <= o.kappa_eps * mu && mu > o.tol / 10 + 1e-300) {
      const double nm = std::max(o.tol / 10, std::min(o.kappa_mu * mu, std::pow(mu, o.theta_mu)));
      if (nm >= mu) break;
      mu = nm;
      tau = std::max(o.tau_min, 1.0 - mu);
      filt.clear();
      CK(kkt_err(mu, &emu, &e0));
    }
    rkkt::ipm_resid(d, s, mu, st);
    // inertia correction: the reduced matrix factorises iff the condensed
    // KKT matrix has the right inertia (G_x invertible)
    double dw = 0.0;
    bool ok = false;
    for (int attempt = 0;; ++attempt) {
      CR(rkkt_condense(p, s.sx, s.sgu, s.ss, dw, s.khat, st));
      CK(hipMemcpyAsync(s.chol, s.khat, sizeof(double) * d.nu * d.nu, hipMemcpyDeviceToDevice, st));
      CR(rkkt_factor(p, s.chol, s.info, st));
      int info = 0;
      CK(hipMemcpyAsync(&info, s.info, sizeof(int), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      ++nfac;
      if (info == 0) { ok = true; if (dw > 0) delta_last = dw; break; }
      if (attempt == 0) dw = delta_last == 0.0 ? o.delta0 : std::max(o.delta_min, o.kw_minus * delta_last);
      else dw *= delta_last == 0.0 ? o.kw_plus_bar : o.kw_plus;
      if (dw > o.delta_max) break;
    }
    if (!ok) { status = 3; break; }
    {
      int code = 0, sc = -1;
      CR(rkkt_status(p, st, &code, &sc));
      if (code != 0) { status = 4; p->err = "rkkt_solve: device status raised"; break; }
    }
    CR(rkkt_step(p, s.r1x, s.r1u, s.r2, s.r3, s.r4, s.ss, s.chol, s.px, s.pu, s.ps, s.py, s.pz, st));
    rkkt::ipm_step_scalars(d, s, mu, tau, s.scal, st);
    CK(fetch(3));
    const double a_max = hs[0], a_z = hs[1], dphi = hs[2];
    rkkt::ipm_merit(d, s, false, s.scal, st);
    CK(fetch(4));
    const double phi0 = hs[0] - mu * hs[2], th = hs[1];
    double a_min;
    if (dphi < 0 && th <= th_min)
      a_min = o.gamma_alpha * std::min({o.gamma_theta, o.gamma_phi * th / -dphi,
                                        o.delta_sw * std::pow(th, o.s_theta) / std::pow(-dphi, o.s_phi)});
    else if (dphi < 0)
      a_min = o.gamma_alpha * std::min(o.gamma_theta, o.gamma_phi * th / -dphi);
    else
      a_min = o.gamma_alpha * o.gamma_theta;
    double alpha = a_max;
    bool accepted = false, augment = false;
    while (true) {
      rkkt::ipm_trial(d, s, alpha, st);
      CR(eval(true, w));
      rkkt::ipm_merit(d, s, true, s.scal, st);
      CK(fetch(4));
      const double th_t = hs[1];
      const double phi_t = hs[3] != 0.0 ? NAN : hs[0] - mu * hs[2];
      bool acc = std::isfinite(phi_t) && std::isfinite(th_t) && th_t <= th_max;
      if (acc)
        for (auto& fe : filt)
          if (!(th_t < fe.first || phi_t < fe.second)) { acc = false; break; }
      if (acc) {
        const bool sw = dphi < 0 && th <= th_min &&
                        alpha * std::pow(-dphi, o.s_phi) > o.delta_sw * std::pow(th, o.s_theta);
        if (sw) {
          if (phi_t <= phi0 + o.eta_phi * alpha * dphi) accepted = true;
        } else if (th_t <= (1 - o.gamma_theta) * th || phi_t <= phi0 - o.gamma_phi * th) {
          accepted = true;
          augment = true;
        }
      }
      if (accepted) break;
      alpha *= 0.5;
      if (alpha < a_min) break;
    }
    if (!accepted) { status = 2; break; }
    if (augment) filt.push_back({(1 - o.gamma_theta) * th, phi0 - o.gamma_phi * th});
    rkkt::ipm_accept(d, s, alpha, a_z, mu, o.kappa_sigma, st);
    CK(hipGetLastError());
    CR(eval(false, w));
    if (verbose) {
      rkkt::ipm_merit(d, s, false, s.scal, st);
      CK(fetch(4));
      std::printf("%3d obj=%.8e E0=%.2e mu=%.1e dw=%.1e a=%.2e az=%.2e\n", k, hs[0] / (w * N), e0,
                  mu, dw, alpha, a_z);
    }
  }
  rkkt::ipm_resid(d, s, mu, st);
  CK(kkt_err(0.0, &emu, &e0));
  rkkt::ipm_merit(d, s, false, s.scal, st);
  CK(fetch(4));
  res->status = status;
  res->iters = k;
  res->obj = hs[0] / (w * N);
  res->kkt_error = e0;
  res->mu = mu;
  res->obj_weight = w;
  res->factorizations = nfac;
  const size_t nxb = sizeof(double) * N * d.nx, nmb = sizeof(double) * N * d.m;
  if (x_out) CK(hipMemcpyAsync(x_out, s.x, nxb, hipMemcpyDeviceToDevice, st));
  if (u_out) CK(hipMemcpyAsync(u_out, s.u, sizeof(double) * d.nu, hipMemcpyDeviceToDevice, st));
  if (y_out) CK(hipMemcpyAsync(y_out, s.y, nxb, hipMemcpyDeviceToDevice, st));
  if (z_out) CK(hipMemcpyAsync(z_out, s.z, nmb, hipMemcpyDeviceToDevice, st));
  if (s_out) CK(hipMemcpyAsync(s_out, s.s, nmb, hipMemcpyDeviceToDevice, st));
  CK(hipStreamSynchronize(st));
#undef CK
#undef CR
  return RKKT_OK;
}

extern "C" int rkkt_solve(rkkt_problem* p, const rkkt_ipm_options* opt, double* x, double* u, double* y,
                          double* z, double* s, rkkt_ipm_result* res, hipStream_t stream) {
  return solve_impl(p, opt, nullptr, nullptr, nullptr, nullptr, x, u, y, z, s, res, stream);
}

extern "C" int rkkt_solve_warm(rkkt_problem* p, const rkkt_ipm_options* opt, const double* x0,
                               const double* u0, const double* y0, const double* z0, double* x, double* u,
                               double* y, double* z, double* s, rkkt_ipm_result* res, hipStream_t stream) {
  if (!x0 || !u0 || !y0 || !z0) {
    if (p) p->err = "rkkt_solve_warm: null start point";
    return RKKT_ERR_ARG;
  }
  return solve_impl(p, opt, x0, u0, y0, z0, x, u, y, z, s, res, stream);
}

