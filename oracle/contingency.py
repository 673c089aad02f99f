"""Oracle for scenarios with a tripped line (test infrastructure; only the
tests may use it).

Parity status: pinned (with no outage it is the plain oracle's K_hat and
Newton step; an outage in scenario k changes K_hat by exactly the difference
of scenario k's terms computed by the plain oracle on one-scenario instances
of the grid with and without the line; the step with outages satisfies every
block row of each scenario's own augmented system).

The paper's scenarios may carry contingencies next to the loads (case-study
section).  Here a scenario with a tripped line is evaluated on its own grid,
the grid with that line deleted (its two flow limits deleted with it), and
its term of the reduced matrix is the term of the proposition "Reduction" on
that grid:
    Z_k^T K_k Z_k = K_uu + K_xu^T S + S^T K_xu + S^T K_xx S,
    S = -(G_x^k)^-1 G_u^k,  K = W + H^T Sigma_s H (+ Sigma_x + delta_w on x),
and K_hat is the sum of the terms plus Sigma_u + delta_w I (proposition
"Condensed KKT system" for K).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .model import Model


def without_line(net, l):
    """The grid with line l deleted."""
    keep = np.arange(net.n_line) != l
    return dataclasses.replace(
        net, n_line=net.n_line - 1, line_from=net.line_from[keep], line_to=net.line_to[keep],
        r=net.r[keep], x=net.x[keep], b=net.b[keep], rate=net.rate[keep])


def kept_rows(net, l):
    """Rows of h kept when line l is deleted: h = [Pg_ref; Qg (n_gen);
    |S_from|^2 (n_line); |S_to|^2 (n_line)]."""
    m = 1 + net.n_gen + 2 * net.n_line
    drop = {1 + net.n_gen + l, 1 + net.n_gen + net.n_line + l}
    return np.array([r for r in range(m) if r not in drop], dtype=np.int64)


def scenario_term(net, xk, u, pdk, qdk, yk, zk, sxk, ssk, wf, delta_w):
    """Z_k^T K_k Z_k of one scenario on the grid `net` (dense)."""
    md = Model(net)
    Gx, Gu, Hx, Hu, _, _ = md.jacobians(xk, u, pdk, qdk, wf)
    Wxx, Wxu, Wuu = md.hessian(xk, u, pdk, qdk, yk, zk, wf)
    Gx, Gu, Hx, Hu = (a.toarray() for a in (Gx, Gu, Hx, Hu))
    Wxx, Wxu, Wuu = (a.toarray() for a in (Wxx, Wxu, Wuu))
    Kxx = Wxx + Hx.T @ (ssk[:, None] * Hx) + np.diag(sxk + delta_w)
    Kxu = Wxu + Hx.T @ (ssk[:, None] * Hu)
    Kuu = Wuu + Hu.T @ (ssk[:, None] * Hu)
    S = -sla.solve(Gx, Gu)
    KxuS = Kxu.T @ S
    return Kuu + KxuS + KxuS.T + S.T @ Kxx @ S


def khat_with_outages(inst, it, delta_w, tripped):
    """K_hat of an instance whose scenario k has line tripped[k] deleted
    (tripped[k] < 0: no outage).  `it` holds the iterate and diagonals in the
    full grid's row order (rows of a deleted line's limits are dropped)."""
    net = inst.net
    N = inst.scen.n_scen
    nu = 2 * net.n_gen - 1
    khat = np.zeros((nu, nu))
    for k in range(N):
        l = int(tripped[k])
        rows = kept_rows(net, l) if l >= 0 else np.arange(1 + net.n_gen + 2 * net.n_line)
        net_k = without_line(net, l) if l >= 0 else net
        khat += scenario_term(net_k, it["x"][k], it["u"], inst.scen.pd[:, k], inst.scen.qd[:, k],
                              it["y"][k], it["z"][k][rows], it["sigma_x"][k], it["sigma_s"][k][rows],
                              it["obj_weight"], delta_w)
    return khat + np.diag(it["sigma_u"] + delta_w)


def evaluate_with_outages(inst, it, tripped):
    """g [N, n_x] and h [N, m] (a deleted line's flow rows set to 0, as its
    flows are)."""
    net = inst.net
    N = inst.scen.n_scen
    m = 1 + net.n_gen + 2 * net.n_line
    g, h = [], np.zeros((N, m))
    for k in range(N):
        l = int(tripped[k])
        net_k = without_line(net, l) if l >= 0 else net
        rows = kept_rows(net, l) if l >= 0 else np.arange(m)
        _, gk, hk = Model(net_k).evaluate(it["x"][k], it["u"], inst.scen.pd[:, k], inst.scen.qd[:, k],
                                          it["obj_weight"])
        g.append(gk)
        h[k, rows] = hk
    return np.array(g), h


def _dense_blocks(net, xk, u, pdk, qdk, yk, zk, wf):
    md = Model(net)
    Gx, Gu, Hx, Hu, _, _ = md.jacobians(xk, u, pdk, qdk, wf)
    Wxx, Wxu, Wuu = md.hessian(xk, u, pdk, qdk, yk, zk, wf)
    return [a.toarray() for a in (Gx, Gu, Hx, Hu, Wxx, Wxu, Wuu)]


def step_with_outages(inst, it, delta_w, tripped):
    """Newton step of the augmented system (right-hand side -r) when scenario
    k has line tripped[k] deleted, each scenario on its own grid (dense):
    condensation (proposition "Condensed KKT system") and reduction
    (proposition "Reduction"):
        K_hat = sum_k [K_uu + K_xu^T S + S^T K_xu + S^T K_xx S] + Sigma_u + dw,
        rhs   = -r2_hat + sum_k [G_u^T G_x^-T r1_hat + K_xu^T q - G_u^T G_x^-T K_xx q],
                q = G_x^-1 r3, r1_hat = r1x + H_x^T w, r2_hat = r1u + sum H_u^T w,
                w = Sigma_s r4 - r2,
        p_u = K_hat^-1 rhs,  p_x = -G_x^-1 (r3 + G_u p_u),
        p_y = -G_x^-T (r1_hat + K_xx p_x + K_xu p_u),
        p_s = -(r4 + H p_d),  p_z = Sigma_s (H p_d + r4) - r2.
    The two flow-limit rows of a deleted line have no H row, so they decouple:
    p_s = -r4 and p_z = Sigma_s r4 - r2 there.  `it` holds the iterate,
    diagonals and residuals in the full grid's row order.  Returns the step
    in that order (dict px, pu, ps, py, pz)."""
    net = inst.net
    N = inst.scen.n_scen
    nu = 2 * net.n_gen - 1
    m = 1 + net.n_gen + 2 * net.n_line
    wf = it["obj_weight"]
    khat = np.diag(it["sigma_u"] + delta_w)
    rhat2 = np.array(it["r1u"], dtype=float, copy=True)
    per = []
    for k in range(N):
        l = int(tripped[k])
        rows = kept_rows(net, l) if l >= 0 else np.arange(m)
        net_k = without_line(net, l) if l >= 0 else net
        Gx, Gu, Hx, Hu, Wxx, Wxu, Wuu = _dense_blocks(
            net_k, it["x"][k], it["u"], inst.scen.pd[:, k], inst.scen.qd[:, k], it["y"][k],
            it["z"][k][rows], wf)
        ss = it["sigma_s"][k][rows]
        r2, r4 = it["r2"][k][rows], it["r4"][k][rows]
        Kxx = Wxx + Hx.T @ (ss[:, None] * Hx) + np.diag(it["sigma_x"][k] + delta_w)
        Kxu = Wxu + Hx.T @ (ss[:, None] * Hu)
        Kuu = Wuu + Hu.T @ (ss[:, None] * Hu)
        S = -sla.solve(Gx, Gu)
        KxuS = Kxu.T @ S
        khat += Kuu + KxuS + KxuS.T + S.T @ Kxx @ S
        w = ss * r4 - r2
        r1h = it["r1x"][k] + Hx.T @ w
        rhat2 += Hu.T @ w
        per.append((rows, Gx, Gu, Hx, Hu, Kxx, Kxu, ss, r1h))
    rhs = -rhat2
    for k, (rows, Gx, Gu, Hx, Hu, Kxx, Kxu, ss, r1h) in enumerate(per):
        q = sla.solve(Gx, it["r3"][k])
        rhs += Gu.T @ sla.solve(Gx.T, r1h) + Kxu.T @ q - Gu.T @ sla.solve(Gx.T, Kxx @ q)
    pu = sla.solve(khat, rhs)
    nx = per[0][1].shape[0]
    out = dict(px=np.zeros((N, nx)), pu=pu, ps=np.zeros((N, m)), py=np.zeros((N, nx)),
               pz=np.zeros((N, m)))
    for k, (rows, Gx, Gu, Hx, Hu, Kxx, Kxu, ss, r1h) in enumerate(per):
        px = -sla.solve(Gx, it["r3"][k] + Gu @ pu)
        out["px"][k] = px
        out["py"][k] = -sla.solve(Gx.T, r1h + Kxx @ px + Kxu @ pu)
        # decoupled rows (no H row) first, then the kept rows
        out["ps"][k] = -it["r4"][k]
        out["pz"][k] = it["sigma_s"][k] * it["r4"][k] - it["r2"][k]
        hp = Hx @ px + Hu @ pu
        out["ps"][k][rows] = -(it["r4"][k][rows] + hp)
        out["pz"][k][rows] = ss * (hp + it["r4"][k][rows]) - it["r2"][k][rows]
    return out
