"""Real-arithmetic (analytic in every input) evaluation of f, g, h, used by the
tests to pin the oracle: complex-step differentiation needs a function with no
conjugates or absolute values, and a per-line loop with cos/sin is a second,
independent way to write the power-flow equations (textbook pi-line model).
"""
import numpy as np


def line_flows(md, th, v):
    net = md.net
    ys = 1.0 / (net.r + 1j * net.x)
    gs, bs = ys.real, ys.imag
    bc = 0.5 * net.b
    f, t = net.line_from, net.line_to
    dt = th[f] - th[t]
    vf, vt = v[f], v[t]
    c, s = np.cos(dt), np.sin(dt)
    # from end: S_f = conj(y_ff) V_f^2 + conj(y_ft) V_f V_t e^{j dt}
    pf = gs * vf * vf - vf * vt * (gs * c + bs * s)
    qf = -(bs + bc) * vf * vf - vf * vt * (gs * s - bs * c)
    pt = gs * vt * vt - vf * vt * (gs * c - bs * s)
    qt = -(bs + bc) * vt * vt - vf * vt * (-gs * s - bs * c)
    return pf, qf, pt, qt


def evaluate(md, xk, u, pdk, qdk, wf):
    net = md.net
    nb, ng = md.nb, md.ng
    dt = np.result_type(xk, u, float)
    th = np.zeros(nb, dtype=dt)
    v = np.zeros(nb, dtype=dt)
    th[md.nonref] = xk[: nb - 1]
    v[md.pq] = xk[nb - 1:]
    v[net.gen_bus] = u[:ng]
    pg_nr = u[ng:]
    pf, qf, pt, qt = line_flows(md, th, v)
    P = np.zeros(nb, dtype=dt)
    Q = np.zeros(nb, dtype=dt)
    np.add.at(P, net.line_from, pf)
    np.add.at(P, net.line_to, pt)
    np.add.at(Q, net.line_from, qf)
    np.add.at(Q, net.line_to, qt)
    Pd = np.zeros(nb)
    Qd = np.zeros(nb)
    np.add.at(Pd, net.load_bus, pdk)
    np.add.at(Qd, net.load_bus, qdk)
    Pg = np.zeros(nb, dtype=dt)
    Pg[md.pg_bus] = pg_nr
    g = np.concatenate([P[md.nonref] - Pg[md.nonref] + Pd[md.nonref], Q[md.pq] + Qd[md.pq]])
    pref = P[md.ref] + Pd[md.ref]
    gb = net.gen_bus
    h = np.concatenate([[pref], Q[gb] + Qd[gb], pf * pf + qf * qf, pt * pt + qt * qt])
    pg = np.zeros(ng, dtype=dt)
    pg[md.gnr] = pg_nr
    pg[md.gref] = pref
    f = wf * np.sum(1e4 * net.c2 * pg * pg + 1e2 * net.c1 * pg + net.c0)
    return f, g, h
