"""Oracle for scenarios with a tripped line (test infrastructure; only the
tests may use it).

Parity status: pinned (with no outage it is the plain oracle's K_hat; an
outage in scenario k changes K_hat by exactly the difference of scenario k's
terms computed by the plain oracle on one-scenario instances of the grid with
and without the line).

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
