"""Oracle: IPM Newton systems, condensation and reduction (test infrastructure).

Parity status: pinned (dense augmented solve = condensed solve = reduced
solve on tiny instances; the Schur complement of the block-angular condensed
system equals Z^T K Z; the closed-form inverse of the 2x2 block A_i;
Cholesky against LAPACK and against the inertia of the condensed system).

Arrays here are scenario-major: x[N, n_x], s[N, m], y[N, n_x], z[N, m];
u[n_u] is shared.

Paper passages followed:
* KKT conditions with barrier homotopy and the augmented Newton system
  (eq. of the augmented system, residuals r1..r4), extended to two-sided
  boxes: every finite bound contributes Z_L (X - X_L)^-1 or Z_U (X_U - X)^-1
  to the diagonal Sigma and -mu (X - X_L)^-1 e or +mu (X_U - X)^-1 e to the
  residual;
* condensation (proposition "Condensed KKT system"): K = W + H^T Sigma_s H,
  right-hand side r1 + H^T (Sigma_s r4 - r2), p_z = Sigma_s (H p_d + r4) - r2;
* block-angular condensed matrix (K_xixi, K_uxi, K_uu);
* reduction (proposition "Reduction"): K_hat = Z^T K Z with
  Z = [-(G_x^i)^-1 G_u^i ; I], the reduced right-hand side and the recovery
  of p_x and p_y.

Readings where the paper is silent (both the oracle and the GPU path use them):
* Sigma_x and delta_w enter every K_xixi; Sigma_u and delta_w enter K_uu once
  (the paper's K has no Sigma_p, the condensed system adds it);
* p_s is recovered from the fourth block row of the augmented system,
  p_s = -(r4 + H p_d), which equals the paper's -Sigma_s^-1 (r2 + p_z) in exact
  arithmetic but does not divide by a vanishing Sigma_s.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .model import Model


@dataclass
class Iterate:
    x: np.ndarray      # [N, n_x]
    u: np.ndarray      # [n_u]
    s: np.ndarray      # [N, m]
    y: np.ndarray      # [N, n_x]
    z: np.ndarray      # [N, m]
    zlx: np.ndarray    # bound duals, zero where the bound is infinite
    zux: np.ndarray
    zlu: np.ndarray
    zuu: np.ndarray
    zls: np.ndarray
    zus: np.ndarray

    def copy(self):
        return Iterate(**{k: np.array(v, copy=True) for k, v in self.__dict__.items()})


class Problem:
    """One block-structured OPF instance: model, loads, bounds."""

    def __init__(self, inst):
        self.inst = inst
        self.model = Model(inst.net)
        self.pd = inst.scen.pd          # [n_load][N]
        self.qd = inst.scen.qd
        self.N = inst.scen.n_scen
        md = self.model
        self.n_x, self.n_u, self.m = md.n_x, md.n_u, md.m
        self.xl, self.xu, self.ul, self.uu, self.sl, self.su = md.bounds()

    def scen_loads(self, k):
        return self.pd[:, k], self.qd[:, k]


# ---------------------------------------------------------------- evaluation
@dataclass
class Eval:
    f: float
    fk: np.ndarray
    g: np.ndarray          # [N, n_x]
    h: np.ndarray          # [N, m]
    gx: np.ndarray         # [N, n_x]  gradient of f_i w.r.t. x_i
    gu: np.ndarray         # [N, n_u]  gradient of f_i w.r.t. u
    Gx: list = field(default_factory=list)
    Gu: list = field(default_factory=list)
    Hx: list = field(default_factory=list)
    Hu: list = field(default_factory=list)
    Wxx: list = field(default_factory=list)
    Wxu: list = field(default_factory=list)
    Wuu: list = field(default_factory=list)


def evaluate(prob: Problem, it: Iterate, wf: float, derivs=True, hess=True) -> Eval:
    md = prob.model
    N = prob.N
    fk = np.zeros(N)
    g = np.zeros((N, prob.n_x))
    h = np.zeros((N, prob.m))
    gx = np.zeros((N, prob.n_x))
    gu = np.zeros((N, prob.n_u))
    ev = Eval(0.0, fk, g, h, gx, gu)
    for k in range(N):
        pdk, qdk = prob.scen_loads(k)
        fk[k], g[k], h[k] = md.evaluate(it.x[k], it.u, pdk, qdk, wf)
        if derivs:
            Gx, Gu, Hx, Hu, gx[k], gu[k] = md.jacobians(it.x[k], it.u, pdk, qdk, wf)
            ev.Gx.append(Gx); ev.Gu.append(Gu); ev.Hx.append(Hx); ev.Hu.append(Hu)
        if hess:
            Wxx, Wxu, Wuu = md.hessian(it.x[k], it.u, pdk, qdk, it.y[k], it.z[k], wf)
            ev.Wxx.append(Wxx); ev.Wxu.append(Wxu); ev.Wuu.append(Wuu)
    ev.f = float(fk.sum())
    return ev


# -------------------------------------------------------- diagonals, residuals
def _bound_parts(v, lo, hi, zl, zu, mu):
    hl = np.isfinite(lo)
    hu = np.isfinite(hi)
    dl = np.where(hl, v - lo, 1.0)
    du = np.where(hu, hi - v, 1.0)
    sigma = np.where(hl, zl / dl, 0.0) + np.where(hu, zu / du, 0.0)
    bgrad = np.where(hl, -mu / dl, 0.0) + np.where(hu, mu / du, 0.0)
    return sigma, bgrad


@dataclass
class Diag:
    sx: np.ndarray    # [N, n_x]
    su: np.ndarray    # [n_u]
    ss: np.ndarray    # [N, m]


@dataclass
class Resid:
    r1x: np.ndarray   # [N, n_x]
    r1u: np.ndarray   # [n_u]
    r2: np.ndarray    # [N, m]
    r3: np.ndarray    # [N, n_x]
    r4: np.ndarray    # [N, m]


def diagonals(prob: Problem, it: Iterate) -> Diag:
    sx, _ = _bound_parts(it.x, prob.xl, prob.xu, it.zlx, it.zux, 0.0)
    su, _ = _bound_parts(it.u, prob.ul, prob.uu, it.zlu, it.zuu, 0.0)
    ss, _ = _bound_parts(it.s, prob.sl, prob.su, it.zls, it.zus, 0.0)
    return Diag(sx, su, ss)


def residuals(prob: Problem, it: Iterate, ev: Eval, mu: float) -> Resid:
    """r1 = grad f + G^T y + H^T z + barrier gradient; r2 = z + barrier
    gradient in s; r3 = g; r4 = h + s (the augmented system's right-hand side)."""
    N = prob.N
    _, bx = _bound_parts(it.x, prob.xl, prob.xu, it.zlx, it.zux, mu)
    _, bu = _bound_parts(it.u, prob.ul, prob.uu, it.zlu, it.zuu, mu)
    _, bs = _bound_parts(it.s, prob.sl, prob.su, it.zls, it.zus, mu)
    r1x = np.zeros((N, prob.n_x))
    r1u = bu.copy()
    for k in range(N):
        r1x[k] = ev.gx[k] + ev.Gx[k].T @ it.y[k] + ev.Hx[k].T @ it.z[k] + bx[k]
        r1u += ev.gu[k] + ev.Gu[k].T @ it.y[k] + ev.Hu[k].T @ it.z[k]
    return Resid(r1x, r1u, it.z + bs, ev.g.copy(), ev.h + it.s)


# ---------------------------------------------------------- global assembly
def global_matrices(prob: Problem, ev: Eval):
    """Dense block-angular W, G, H of the whole problem (tiny instances only).

    Primal order: (x_1, ..., x_N, u).  W_uu is the sum of the scenario blocks.
    """
    N, nx, nu, m = prob.N, prob.n_x, prob.n_u, prob.m
    nd = N * nx + nu
    W = np.zeros((nd, nd))
    G = np.zeros((N * nx, nd))
    H = np.zeros((N * m, nd))
    uo = N * nx
    for k in range(N):
        xs = slice(k * nx, (k + 1) * nx)
        W[xs, xs] = ev.Wxx[k].toarray()
        W[xs, uo:] = ev.Wxu[k].toarray()
        W[uo:, xs] = ev.Wxu[k].toarray().T
        W[uo:, uo:] += ev.Wuu[k].toarray()
        G[xs, xs] = ev.Gx[k].toarray()
        G[xs, uo:] = ev.Gu[k].toarray()
        H[k * m:(k + 1) * m, xs] = ev.Hx[k].toarray()
        H[k * m:(k + 1) * m, uo:] = ev.Hu[k].toarray()
    return W, G, H


def _split_step(prob, pd, ps, py, pz):
    N, nx, m = prob.N, prob.n_x, prob.m
    return dict(px=pd[: N * nx].reshape(N, nx), pu=pd[N * nx:].copy(),
                ps=ps.reshape(N, m), py=py.reshape(N, nx), pz=pz.reshape(N, m))


def newton_full(prob: Problem, ev: Eval, dg: Diag, rs: Resid, delta_w: float):
    """Dense LU solve of the augmented system [W+Sigma_p, 0, G^T, H^T;
    0, Sigma_s, 0, I; G, 0, 0, 0; H, I, 0, 0] p = -r (LAPACK, partial pivots)."""
    N, nx, nu, m = prob.N, prob.n_x, prob.n_u, prob.m
    W, G, H = global_matrices(prob, ev)
    nd, ns, ny = N * nx + nu, N * m, N * nx
    Sp = np.concatenate([dg.sx.ravel(), dg.su])
    A = np.zeros((nd + ns + ny + ns,) * 2)
    o1, o2, o3 = nd, nd + ns, nd + ns + ny
    A[:nd, :nd] = W + np.diag(Sp + delta_w)
    A[:nd, o2:o3] = G.T
    A[:nd, o3:] = H.T
    A[o1:o2, o1:o2] = np.diag(dg.ss.ravel())
    A[o1:o2, o3:] = np.eye(ns)
    A[o2:o3, :nd] = G
    A[o3:, :nd] = H
    A[o3:, o1:o2] = np.eye(ns)
    r = np.concatenate([rs.r1x.ravel(), rs.r1u, rs.r2.ravel(), rs.r3.ravel(), rs.r4.ravel()])
    p = sla.lu_solve(sla.lu_factor(A), -r)
    return _split_step(prob, p[:nd], p[o1:o2], p[o2:o3], p[o3:])


def newton_condensed(prob: Problem, ev: Eval, dg: Diag, rs: Resid, delta_w: float):
    """Condensed system [K+Sigma_p, G^T; G, 0] (p_d, p_y) = -(r1 + H^T(Sigma_s r4 - r2), r3)."""
    N, nx, nu, m = prob.N, prob.n_x, prob.n_u, prob.m
    W, G, H = global_matrices(prob, ev)
    nd = N * nx + nu
    ss = dg.ss.ravel()
    K = W + H.T @ (ss[:, None] * H)
    Sp = np.concatenate([dg.sx.ravel(), dg.su])
    A = np.block([[K + np.diag(Sp + delta_w), G.T], [G, np.zeros((N * nx, N * nx))]])
    r1 = np.concatenate([rs.r1x.ravel(), rs.r1u])
    r2, r4 = rs.r2.ravel(), rs.r4.ravel()
    rhs = -np.concatenate([r1 + H.T @ (ss * r4 - r2), rs.r3.ravel()])
    p = sla.lu_solve(sla.lu_factor(A), rhs)
    pd, py = p[:nd], p[nd:]
    ps = -(r4 + H @ pd)
    pz = ss * (H @ pd + r4) - r2
    return _split_step(prob, pd, ps, py, pz)


# --------------------------------------------------------------- reduction
# Largest n_x factorised densely (LAPACK); larger G_x blocks go to SuperLU.
DENSE_MAX = 3000


class _GxFactor:
    """LU of one G_x block (dense LAPACK for n_x <= DENSE_MAX, SuperLU beyond)."""

    def __init__(self, Gx):
        self.n = Gx.shape[0]
        if self.n <= DENSE_MAX:
            self.lu = sla.lu_factor(Gx.toarray())
            self.sparse = False
        else:
            self.lu = spla.splu(sp.csc_matrix(Gx))
            self.sparse = True

    def solve(self, b, trans=False):
        if self.sparse:
            return self.lu.solve(np.asarray(b, order="F"), trans="T" if trans else "N")
        return sla.lu_solve(self.lu, b, trans=1 if trans else 0)


@dataclass
class Reduced:
    khat: np.ndarray              # [n_u, n_u]
    Kxx: list
    Kxu: list
    Kuu: list
    fac: list
    S: list                       # S_i = -(G_x^i)^-1 G_u^i, dense [n_x, n_u]


def condensed_blocks(ev: Eval, dg: Diag, k: int, delta_w: float):
    """K_xixi (+ Sigma_x + delta_w), K_xiu and the scenario's share of K_uu."""
    ss = sp.diags(dg.ss[k])
    Hx, Hu = ev.Hx[k], ev.Hu[k]
    Kxx = (ev.Wxx[k] + Hx.T @ ss @ Hx + sp.diags(dg.sx[k] + delta_w)).tocsr()
    Kxu = (ev.Wxu[k] + Hx.T @ ss @ Hu).tocsr()
    Kuu = (ev.Wuu[k] + Hu.T @ ss @ Hu).tocsr()
    return Kxx, Kxu, Kuu


def reduced_hessian(prob: Problem, ev: Eval, dg: Diag, delta_w: float,
                    keep=True) -> Reduced:
    """K_hat = sum_i [K_uu^i + K_ux^i S_i + S_i^T K_xu^i + S_i^T K_xx^i S_i]
    + Sigma_u + delta_w I, with S_i = -(G_x^i)^-1 G_u^i (= Z^T K Z)."""
    nu = prob.n_u
    khat = np.zeros((nu, nu))
    red = Reduced(khat, [], [], [], [], [])
    for k in range(prob.N):
        Kxx, Kxu, Kuu = condensed_blocks(ev, dg, k, delta_w)
        fac = _GxFactor(ev.Gx[k])
        S = -fac.solve(ev.Gu[k].toarray())
        KxuS = Kxu.T @ S
        khat += Kuu.toarray() + KxuS + KxuS.T + S.T @ (Kxx @ S)
        if keep:
            red.Kxx.append(Kxx); red.Kxu.append(Kxu); red.Kuu.append(Kuu)
            red.fac.append(fac); red.S.append(S)
    khat += np.diag(dg.su + delta_w)
    return red


def reduced_rhs(prob: Problem, ev: Eval, dg: Diag, rs: Resid, red: Reduced):
    """hat r pieces and the right-hand side of the reduced system:
    -r2_hat + sum_i [G_u^T G_x^-T r1_hat^i + (K_ux - G_u^T G_x^-T K_xx) G_x^-1 r3^i]."""
    rhat1 = np.zeros((prob.N, prob.n_x))
    rhat2 = rs.r1u.copy()
    for k in range(prob.N):
        w = dg.ss[k] * rs.r4[k] - rs.r2[k]
        rhat1[k] = rs.r1x[k] + ev.Hx[k].T @ w
        rhat2 += ev.Hu[k].T @ w
    rhs = -rhat2
    for k in range(prob.N):
        fac = red.fac[k]
        a = fac.solve(rhat1[k], trans=True)
        q = fac.solve(rs.r3[k])
        b = fac.solve(red.Kxx[k] @ q, trans=True)
        rhs = rhs + ev.Gu[k].T @ a + red.Kxu[k].T @ q - ev.Gu[k].T @ b
    return rhat1, rhat2, rhs


def newton_reduced(prob: Problem, ev: Eval, dg: Diag, rs: Resid, delta_w: float,
                   red: Reduced | None = None):
    """Reduced solve: Cholesky of K_hat, then per-scenario recovery of
    p_x = -G_x^-1 (r3_hat + G_u p_u), p_y = -G_x^-T (r1_hat + K_xx p_x + K_xu p_u),
    then p_s and p_z from the condensation."""
    if red is None:
        red = reduced_hessian(prob, ev, dg, delta_w)
    rhat1, rhat2, rhs = reduced_rhs(prob, ev, dg, rs, red)
    L = sla.cholesky(red.khat, lower=True)
    pu = sla.cho_solve((L, True), rhs)
    N, nx, m = prob.N, prob.n_x, prob.m
    px = np.zeros((N, nx)); py = np.zeros((N, nx))
    ps = np.zeros((N, m)); pz = np.zeros((N, m))
    for k in range(N):
        fac = red.fac[k]
        px[k] = -fac.solve(rs.r3[k] + ev.Gu[k] @ pu)
        py[k] = -fac.solve(rhat1[k] + red.Kxx[k] @ px[k] + red.Kxu[k] @ pu, trans=True)
        hp = ev.Hx[k] @ px[k] + ev.Hu[k] @ pu
        ps[k] = -(rs.r4[k] + hp)
        pz[k] = dg.ss[k] * (hp + rs.r4[k]) - rs.r2[k]
    return dict(px=px, pu=pu, ps=ps, py=py, pz=pz)


def cholesky_info(A):
    """LAPACK-style Cholesky status: 0 on success, else the 1-based column of
    the first non-positive pivot (plain right-looking outer-product form)."""
    A = np.array(A, dtype=float, copy=True)
    n = A.shape[0]
    for j in range(n):
        d = A[j, j] - A[j, :j] @ A[j, :j]
        if not d > 0.0:
            return j + 1, None
        A[j, j] = np.sqrt(d)
        A[j + 1:, j] = (A[j + 1:, j] - A[j + 1:, :j] @ A[j, :j]) / A[j, j]
    return 0, np.tril(A)


def bound_dual_steps(prob: Problem, it: Iterate, step: dict, mu: float):
    """p_zL = mu (X - X_L)^-1 e - z_L - Sigma_L p, p_zU = mu (X_U - X)^-1 e - z_U + Sigma_U p."""
    out = {}
    for name, v, p, lo, hi, zl, zu in (
            ("x", it.x, step["px"], prob.xl, prob.xu, it.zlx, it.zux),
            ("u", it.u, step["pu"], prob.ul, prob.uu, it.zlu, it.zuu),
            ("s", it.s, step["ps"], prob.sl, prob.su, it.zls, it.zus)):
        hl, hu = np.isfinite(lo), np.isfinite(hi)
        dl = np.where(hl, v - lo, 1.0)
        du = np.where(hu, hi - v, 1.0)
        out["zl" + name] = np.where(hl, mu / dl - zl - zl / dl * p, 0.0)
        out["zu" + name] = np.where(hu, mu / du - zu + zu / du * p, 0.0)
    return out


def reduced_hessian_columns(prob: Problem, ev: Eval, dg: Diag, delta_w: float, cols):
    """Selected columns K_hat V of the reduced matrix, V = unit vectors e_j,
    by the paper's three-step product (parallel KKT solver section):
    T_x = -G_x^-1 (G_u V);  [L_x; L_u] = [K_xx K_xu; K_ux K_uu] [T_x; V];
    K_hat V = L_u - G_u^T G_x^-T L_x; summed over scenarios, plus
    (Sigma_u + delta_w) on the selected diagonal entries."""
    cols = np.asarray(cols, dtype=np.int64)
    nu = prob.n_u
    V = np.zeros((nu, len(cols)))
    V[cols, np.arange(len(cols))] = 1.0
    out = V * (dg.su + delta_w)[:, None]
    for k in range(prob.N):
        Kxx, Kxu, Kuu = condensed_blocks(ev, dg, k, delta_w)
        fac = _GxFactor(ev.Gx[k])
        Tx = -fac.solve(ev.Gu[k] @ V)
        Lx = Kxx @ Tx + Kxu @ V
        Lu = Kxu.T @ Tx + Kuu @ V
        out += Lu - ev.Gu[k].T @ fac.solve(Lx, trans=True)
    return out


def augmented_residual(prob: Problem, ev: Eval, dg: Diag, rs: Resid, delta_w: float, step: dict,
                       blocks=False):
    """Block rows of the augmented Newton system (eq. of the augmented system)
    evaluated at a candidate step, scenario by scenario with sparse blocks:
      row 1 (x_i): (W_xx + Sigma_x + dw) p_x + W_xu p_u + G_x^T p_y + H_x^T p_z + r1x
      row 1 (u):   sum_i [W_ux p_x + W_uu p_u + G_u^T p_y + H_u^T p_z] + (Sigma_u + dw) p_u + r1u
      row 2:       Sigma_s p_s + p_z + r2
      row 3:       G_x p_x + G_u p_u + r3
      row 4:       H_x p_x + H_u p_u + p_s + r4
    Returns (residual 2-norm, scale) with scale the 2-norm of all terms; with
    blocks=True also a dict of (residual, scale) per block row."""
    pu = step["pu"]
    res = []
    scale = []
    per = {"x": [0.0, 0.0], "s": [0.0, 0.0], "g": [0.0, 0.0], "h": [0.0, 0.0], "u": [0.0, 0.0]}
    ru = (dg.su + delta_w) * pu + rs.r1u
    su_terms = [np.linalg.norm((dg.su + delta_w) * pu), np.linalg.norm(rs.r1u)]
    for k in range(prob.N):
        px, py, ps, pz = step["px"][k], step["py"][k], step["ps"][k], step["pz"][k]
        t1 = [ev.Wxx[k] @ px + (dg.sx[k] + delta_w) * px, ev.Wxu[k] @ pu, ev.Gx[k].T @ py,
              ev.Hx[k].T @ pz, rs.r1x[k]]
        tu = [ev.Wxu[k].T @ px, ev.Wuu[k] @ pu, ev.Gu[k].T @ py, ev.Hu[k].T @ pz]
        ru = ru + sum(tu)
        su_terms += [np.linalg.norm(t) for t in tu]
        t2 = [dg.ss[k] * ps, pz, rs.r2[k]]
        t3 = [ev.Gx[k] @ px, ev.Gu[k] @ pu, rs.r3[k]]
        t4 = [ev.Hx[k] @ px, ev.Hu[k] @ pu, ps, rs.r4[k]]
        for name, terms in (("x", t1), ("s", t2), ("g", t3), ("h", t4)):
            rv = sum(terms)
            res.append(rv)
            sc = [np.linalg.norm(t) for t in terms]
            scale += sc
            per[name][0] += float(np.dot(rv, rv))
            per[name][1] += float(np.sum(np.square(sc)))
    res.append(ru)
    scale += su_terms
    per["u"] = [float(np.dot(ru, ru)), float(np.sum(np.square(su_terms)))]
    r = float(np.sqrt(sum(float(np.dot(v, v)) for v in res)))
    if blocks:
        return r, float(np.linalg.norm(scale)), {k: (np.sqrt(a), np.sqrt(b)) for k, (a, b) in per.items()}
    return r, float(np.linalg.norm(scale))
