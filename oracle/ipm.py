"""Oracle: the outer interior-point iteration (test infrastructure).

Parity status: pinned by invariants only (power-flow residual and scaled KKT
error below tolerance at convergence, reduced Hessian positive definite at
the solution).  The objective value itself has no printed counterpart in the
paper.

The paper runs its linear algebra inside an IPOPT-style primal-dual
interior-point solver and does not spell out the outer loop; the rules below
are the published filter line-search method (Waechter & Biegler, 2006) with
the simplifications listed, and the GPU-side driver follows the same rules:

* start: angles 0, magnitudes 1, generator outputs at mid-range, pushed inside
  their boxes (kappa_1 = kappa_2 = 1e-2); slacks s = -h pushed inside; equality
  and inequality multipliers 0; bound multipliers 1; mu_0 = 0.1; objective
  scaled by min(1, 100 / max|grad f(x_0)|);
* barrier update: while E_mu <= 10 mu, mu <- max(tol/10, min(0.2 mu, mu^1.5))
  and the filter is reset;
* fraction to boundary tau = max(0.99, 1 - mu), separately for the primal
  variables and the bound multipliers;
* inertia correction on the reduced Hessian: Cholesky success means correct
  inertia; on failure delta_w = 1e-4 (first time) or max(1e-20, delta_last/3),
  then x100 (first time) or x8 until success, failure above 1e20;
* filter line search with halving backtracking, switching condition,
  Armijo condition on the barrier objective, filter augmentation on
  non-f-type steps; no second-order correction and no restoration phase
  (a failed line search ends the run with status "line_search_failed");
* stop when the scaled KKT error E_0 <= tol (s_max = 100).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

from . import kkt


@dataclass
class Options:
    tol: float = 1e-8
    max_iter: int = 200
    mu0: float = 0.1
    kappa1: float = 1e-2
    kappa2: float = 1e-2
    tau_min: float = 0.99
    kappa_eps: float = 10.0
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    s_max: float = 100.0
    delta0: float = 1e-4
    delta_min: float = 1e-20
    delta_max: float = 1e20
    kw_minus: float = 1.0 / 3.0
    kw_plus: float = 8.0
    kw_plus_bar: float = 100.0
    gamma_theta: float = 1e-5
    gamma_phi: float = 1e-8
    s_theta: float = 1.1
    s_phi: float = 2.3
    delta_sw: float = 1.0
    eta_phi: float = 1e-8
    gamma_alpha: float = 0.05
    kappa_sigma: float = 1e10
    obj_scale_max_grad: float = 100.0


@dataclass
class Result:
    status: str
    iters: int
    obj: float                 # unscaled average cost
    it: kkt.Iterate
    wf: float
    mu: float
    kkt_error: float
    history: list = field(default_factory=list)


def _push(v, lo, hi, k1, k2):
    v = np.array(v, dtype=float, copy=True)
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    both = fl & fu
    pl = np.where(fl, k1 * np.maximum(1.0, np.abs(np.where(fl, lo, 0.0))), 0.0)
    pu = np.where(fu, k1 * np.maximum(1.0, np.abs(np.where(fu, hi, 0.0))), 0.0)
    rng = np.where(both, np.where(both, hi, 0.0) - np.where(both, lo, 0.0), np.inf)
    pl = np.where(both, np.minimum(pl, k2 * rng), pl)
    pu = np.where(both, np.minimum(pu, k2 * rng), pu)
    v = np.where(fl, np.maximum(v, np.where(fl, lo, 0.0) + pl), v)
    v = np.where(fu, np.minimum(v, np.where(fu, hi, 0.0) - pu), v)
    return v


def initial_point(prob: kkt.Problem, opt: Options):
    md = prob.model
    N = prob.N
    net = md.net
    x0 = np.concatenate([np.zeros(md.nb - 1), np.ones(len(md.pq))])
    x = np.tile(_push(x0, prob.xl, prob.xu, opt.kappa1, opt.kappa2), (N, 1))
    u = np.concatenate([np.ones(md.ng), 0.5 * (net.pmin[md.gnr] + net.pmax[md.gnr])])
    u = _push(u, prob.ul, prob.uu, opt.kappa1, opt.kappa2)
    zero = np.zeros((N, prob.m))
    it = kkt.Iterate(x, u, zero.copy(), np.zeros((N, prob.n_x)), zero.copy(),
                     np.isfinite(prob.xl) * np.ones((N, 1)), np.isfinite(prob.xu) * np.ones((N, 1)),
                     np.isfinite(prob.ul) * 1.0, np.isfinite(prob.uu) * 1.0,
                     np.isfinite(prob.sl) * np.ones((N, 1)), np.isfinite(prob.su) * np.ones((N, 1)))
    ev = kkt.evaluate(prob, it, 1.0 / N, derivs=True, hess=False)
    it.s = _push(-ev.h, prob.sl, prob.su, opt.kappa1, opt.kappa2)
    gmax = max(np.abs(ev.gx).max(), np.abs(ev.gu.sum(axis=0)).max())
    scale = min(1.0, opt.obj_scale_max_grad / gmax) if gmax > 0 else 1.0
    return it, scale / N


def _logsum(v, lo, hi):
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    a = np.where(fl, v - np.where(fl, lo, 0.0), 1.0)
    b = np.where(fu, np.where(fu, hi, 0.0) - v, 1.0)
    if np.any(a <= 0) or np.any(b <= 0):
        return np.nan
    return float(np.sum(np.log(a)) + np.sum(np.log(b)))


def barrier_objective(prob, it, f, mu):
    return f - mu * (_logsum(it.x, prob.xl, prob.xu) + _logsum(it.u, prob.ul, prob.uu)
                     + _logsum(it.s, prob.sl, prob.su))


def constraint_violation(ev, it):
    return float(np.abs(ev.g).sum() + np.abs(ev.h + it.s).sum())


def kkt_error(prob, it, ev, mu, opt):
    N = prob.N
    dx = np.zeros((N, prob.n_x))
    du = -it.zlu + it.zuu
    for k in range(N):
        dx[k] = ev.gx[k] + ev.Gx[k].T @ it.y[k] + ev.Hx[k].T @ it.z[k] - it.zlx[k] + it.zux[k]
        du = du + ev.gu[k] + ev.Gu[k].T @ it.y[k] + ev.Hu[k].T @ it.z[k]
    ds = it.z - it.zls + it.zus
    dual = max(np.abs(dx).max(), np.abs(du).max(), np.abs(ds).max())
    primal = max(np.abs(ev.g).max(), np.abs(ev.h + it.s).max())
    comp = 0.0
    zsum = 0.0
    for v, lo, hi, zl, zu in ((it.x, prob.xl, prob.xu, it.zlx, it.zux),
                              (it.u, prob.ul, prob.uu, it.zlu, it.zuu),
                              (it.s, prob.sl, prob.su, it.zls, it.zus)):
        fl, fu = np.isfinite(lo), np.isfinite(hi)
        cl = np.where(fl, (v - np.where(fl, lo, 0.0)) * zl - mu, 0.0)
        cu = np.where(fu, (np.where(fu, hi, 0.0) - v) * zu - mu, 0.0)
        comp = max(comp, np.abs(cl).max(), np.abs(cu).max())
        zsum += np.abs(zl).sum() + np.abs(zu).sum()
    n_var = N * (prob.n_x + prob.m) + prob.n_u
    n_con = N * (prob.n_x + prob.m)
    sd = max(opt.s_max, (np.abs(it.y).sum() + np.abs(it.z).sum() + zsum) / (n_var + n_con)) / opt.s_max
    sc = max(opt.s_max, zsum / n_var) / opt.s_max
    return max(dual / sd, primal, comp / sc)


def _max_step(v, p, lo, hi, tau):
    a = 1.0
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    with np.errstate(divide="ignore", invalid="ignore"):
        ml = fl & (p < 0)
        if np.any(ml):
            a = min(a, float(np.min((-tau * (v - np.where(fl, lo, 0.0)) / p)[ml])))
        mu_ = fu & (p > 0)
        if np.any(mu_):
            a = min(a, float(np.min((tau * (np.where(fu, hi, 0.0) - v) / p)[mu_])))
    return a


def _max_dual_step(z, p, tau):
    m = p < 0
    if not np.any(m):
        return 1.0
    return min(1.0, float(np.min(-tau * z[m] / p[m])))


def _safeguard(v, lo, hi, zl, zu, mu, ks):
    fl, fu = np.isfinite(lo), np.isfinite(hi)
    dl = np.where(fl, v - np.where(fl, lo, 0.0), 1.0)
    du = np.where(fu, np.where(fu, hi, 0.0) - v, 1.0)
    zl = np.where(fl, np.maximum(np.minimum(zl, ks * mu / dl), mu / (ks * dl)), 0.0)
    zu = np.where(fu, np.maximum(np.minimum(zu, ks * mu / du), mu / (ks * du)), 0.0)
    return zl, zu


def factor_with_inertia_correction(prob, ev, dg, delta_last, opt):
    """Returns (reduced data, delta_w, new delta_last, number of factorizations)."""
    red = kkt.reduced_hessian(prob, ev, dg, 0.0)
    info, _ = kkt.cholesky_info(red.khat)
    nfac = 1
    if info == 0:
        return red, 0.0, delta_last, nfac
    dw = opt.delta0 if delta_last == 0.0 else max(opt.delta_min, opt.kw_minus * delta_last)
    while True:
        red = kkt.reduced_hessian(prob, ev, dg, dw)
        info, _ = kkt.cholesky_info(red.khat)
        nfac += 1
        if info == 0:
            return red, dw, dw, nfac
        dw *= opt.kw_plus_bar if delta_last == 0.0 else opt.kw_plus
        if dw > opt.delta_max:
            return None, dw, delta_last, nfac


def solve(prob: kkt.Problem, opt: Options | None = None, verbose=False,
          snapshot_iters=(), max_iter=None) -> Result:
    opt = opt or Options()
    it, wf = initial_point(prob, opt)
    mu = opt.mu0
    tau = max(opt.tau_min, 1.0 - mu)
    ev = kkt.evaluate(prob, it, wf)
    th0 = constraint_violation(ev, it)
    th_max = 1e4 * max(1.0, th0)
    th_min = 1e-4 * max(1.0, th0)
    filt = []
    delta_last = 0.0
    hist = []
    status = "max_iter"
    n_iter = opt.max_iter if max_iter is None else max_iter
    k = 0
    for k in range(n_iter + 1):
        e0 = kkt_error(prob, it, ev, 0.0, opt)
        if e0 <= opt.tol:
            status = "converged"
            break
        if k == n_iter:
            break
        while kkt_error(prob, it, ev, mu, opt) <= opt.kappa_eps * mu and mu > opt.tol / 10 + 1e-300:
            new_mu = max(opt.tol / 10, min(opt.kappa_mu * mu, mu ** opt.theta_mu))
            if new_mu >= mu:
                break
            mu = new_mu
            tau = max(opt.tau_min, 1.0 - mu)
            filt = []
        dg = kkt.diagonals(prob, it)
        rs = kkt.residuals(prob, it, ev, mu)
        red, dw, delta_last, nfac = factor_with_inertia_correction(prob, ev, dg, delta_last, opt)
        if red is None:
            status = "inertia_correction_failed"
            break
        step = kkt.newton_reduced(prob, ev, dg, rs, dw, red)
        if k in snapshot_iters:
            hist.append(dict(k=k, it=it.copy(), mu=mu, wf=wf, delta_w=dw, step=step,
                             khat=red.khat.copy()))
        dz = kkt.bound_dual_steps(prob, it, step, mu)
        a_max = min(_max_step(it.x, step["px"], prob.xl, prob.xu, tau),
                    _max_step(it.u, step["pu"], prob.ul, prob.uu, tau),
                    _max_step(it.s, step["ps"], prob.sl, prob.su, tau))
        a_z = min(_max_dual_step(getattr(it, n), dz[n], tau)
                  for n in ("zlx", "zux", "zlu", "zuu", "zls", "zus"))
        # line search
        phi0 = barrier_objective(prob, it, ev.f, mu)
        th = constraint_violation(ev, it)
        _, bx = kkt._bound_parts(it.x, prob.xl, prob.xu, it.zlx, it.zux, mu)
        _, bu = kkt._bound_parts(it.u, prob.ul, prob.uu, it.zlu, it.zuu, mu)
        _, bs = kkt._bound_parts(it.s, prob.sl, prob.su, it.zls, it.zus, mu)
        dphi = float(np.sum((ev.gx + bx) * step["px"]) + np.dot(ev.gu.sum(axis=0) + bu, step["pu"])
                     + np.sum(bs * step["ps"]))
        if dphi < 0 and th <= th_min:
            a_min = opt.gamma_alpha * min(opt.gamma_theta, opt.gamma_phi * th / -dphi,
                                          opt.delta_sw * th ** opt.s_theta / (-dphi) ** opt.s_phi)
        elif dphi < 0:
            a_min = opt.gamma_alpha * min(opt.gamma_theta, opt.gamma_phi * th / -dphi)
        else:
            a_min = opt.gamma_alpha * opt.gamma_theta
        alpha = a_max
        accepted = False
        augment = False
        n_bt = 0
        while True:
            tr = it.copy()
            tr.x = it.x + alpha * step["px"]
            tr.u = it.u + alpha * step["pu"]
            tr.s = it.s + alpha * step["ps"]
            evt = kkt.evaluate(prob, tr, wf, derivs=False, hess=False)
            th_t = constraint_violation(evt, tr)
            phi_t = barrier_objective(prob, tr, evt.f, mu)
            ok = np.isfinite(phi_t) and np.isfinite(th_t) and th_t <= th_max
            if ok:
                ok = all(th_t < tf or phi_t < pf for tf, pf in filt)
            if ok:
                switching = (dphi < 0 and th <= th_min and
                             alpha * (-dphi) ** opt.s_phi > opt.delta_sw * th ** opt.s_theta)
                if switching:
                    if phi_t <= phi0 + opt.eta_phi * alpha * dphi:
                        accepted = True
                else:
                    if th_t <= (1 - opt.gamma_theta) * th or phi_t <= phi0 - opt.gamma_phi * th:
                        accepted = True
                        augment = True
            if accepted:
                break
            alpha *= 0.5
            n_bt += 1
            if alpha < a_min:
                break
        if not accepted:
            status = "line_search_failed"
            break
        if augment:
            filt.append(((1 - opt.gamma_theta) * th, phi0 - opt.gamma_phi * th))
        new = it.copy()
        new.x = it.x + alpha * step["px"]
        new.u = it.u + alpha * step["pu"]
        new.s = it.s + alpha * step["ps"]
        new.y = it.y + alpha * step["py"]
        new.z = it.z + alpha * step["pz"]
        for n in ("zlx", "zux", "zlu", "zuu", "zls", "zus"):
            setattr(new, n, getattr(it, n) + a_z * dz[n])
        for v, lo, hi, a, b in (("x", prob.xl, prob.xu, "zlx", "zux"),
                                ("u", prob.ul, prob.uu, "zlu", "zuu"),
                                ("s", prob.sl, prob.su, "zls", "zus")):
            zl, zu = _safeguard(getattr(new, v), lo, hi, getattr(new, a), getattr(new, b),
                                mu, opt.kappa_sigma)
            setattr(new, a, zl)
            setattr(new, b, zu)
        it = new
        ev = kkt.evaluate(prob, it, wf)
        if verbose:
            print(f"{k:3d} obj={ev.f / (wf * prob.N):.8e} inf_pr={max(np.abs(ev.g).max(), np.abs(ev.h + it.s).max()):.2e} "
                  f"E0={e0:.2e} mu={mu:.1e} dw={dw:.1e} a={alpha:.2e} az={a_z:.2e} bt={n_bt}")
    e0 = kkt_error(prob, it, ev, 0.0, opt)
    return Result(status=status, iters=k, obj=ev.f / (wf * prob.N), it=it, wf=wf, mu=mu,
                  kkt_error=e0, history=hist)
