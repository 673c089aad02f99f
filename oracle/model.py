"""Oracle: the block-structured AC-OPF and its derivatives (test infrastructure).

Parity status: pinned (complex-step first derivatives, central differences of
the analytic gradient for the Hessian, the paper's dimension tables, the
lossless-grid identity, textbook power-flow convergence).

Formulation (paper, problem statement and case-study section; eq. of the
two-stage problem and its slack form):

* one scenario block i has state x_i, shared control u, state equation
  g_i(x_i, u) = 0 and operational constraints h_i(x_i, u) <= 0, written as
  h_i + s_i = 0 with a slack s_i;
* buses: the reference bus (the bus of the largest generator), PV buses (the
  other generator buses) and PQ buses (no generator);
* x_i = [voltage angles of the non-reference buses (bus order);
         voltage magnitudes of the PQ buses (bus order)]
  so n_x = 2 n_bus - n_gen - 1 (the paper's Table 1 column);
* u = [voltage magnitudes of the generator buses (generator order);
       active output of the non-reference generators (generator order)]
  so n_u = 2 n_gen - 1;  the reference generator's output is a per-scenario
  recourse quantity;
* g_i = [P_b(theta, V) - Pg_b + Pd_b for every non-reference bus b;
         Q_b(theta, V) + Qd_b for every PQ bus b];
* h_i = [Pg_ref = P_ref + Pd_ref;  Qg_k = Q_bus(k) + Qd_bus(k) for every
         generator k;  |S_from,l|^2 for every line; |S_to,l|^2 for every line]
  so m = 2 n_line + n_gen + 1;
* f_i = w * sum_k [c2_k (100 Pg_k)^2 + c1_k (100 Pg_k) + c0_k], with w the
  objective weight (1/N times the objective scale; the problem averages the
  scenario costs).

Lines are pi-models: series admittance 1/(r + jx), half the charging
susceptance at each end, no transformers.  Powers are per unit on 100 MVA.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _diag(v):
    return sp.diags(v, 0, format="csr")


class Model:
    """Per-scenario evaluation of f, g, h and their first and second derivatives."""

    def __init__(self, net):
        self.net = net
        nb, nl, ng = net.n_bus, net.n_line, net.n_gen
        self.nb, self.nl, self.ng = nb, nl, ng
        self.ref = int(net.ref_bus)
        self.gref = int(net.ref_gen)
        is_gen = np.zeros(nb, dtype=bool)
        is_gen[net.gen_bus] = True
        self.nonref = np.array([b for b in range(nb) if b != self.ref], dtype=np.int64)
        self.pq = np.nonzero(~is_gen)[0]
        self.gnr = np.array([k for k in range(ng) if k != self.gref], dtype=np.int64)
        self.n_x = len(self.nonref) + len(self.pq)
        self.n_u = 2 * ng - 1
        self.m = 1 + ng + 2 * nl
        # admittances
        ys = 1.0 / (net.r + 1j * net.x)
        ysh = 0.5j * net.b
        yff, yft, ytf, ytt = ys + ysh, -ys, -ys, ys + ysh
        li = np.arange(nl)
        self.Cf = sp.csr_matrix((np.ones(nl), (li, net.line_from)), shape=(nl, nb))
        self.Ct = sp.csr_matrix((np.ones(nl), (li, net.line_to)), shape=(nl, nb))
        self.Yf = (_diag(yff) @ self.Cf + _diag(yft) @ self.Ct).tocsr()
        self.Yt = (_diag(ytf) @ self.Cf + _diag(ytt) @ self.Ct).tocsr()
        self.Ybus = (self.Cf.T @ self.Yf + self.Ct.T @ self.Yt).tocsr()
        # columns of the full coordinate vector (theta[0:nb], v[0:nb]) that x and
        # the voltage part of u select
        self.xcols = np.concatenate([self.nonref, nb + self.pq])
        self.ucols_v = nb + np.asarray(net.gen_bus, dtype=np.int64)
        # equation rows: P rows of non-ref buses, Q rows of PQ buses
        self.gbus_P = self.nonref
        self.gbus_Q = self.pq
        # objective coefficients in per unit: cost = a*Pg^2 + b*Pg + c
        self.ca = 1e4 * np.asarray(net.c2)
        self.cb = 1e2 * np.asarray(net.c1)
        self.cc = np.asarray(net.c0, dtype=float)
        # Pg column of u for every non-ref generator, and its bus
        self.pg_bus = np.asarray(net.gen_bus, dtype=np.int64)[self.gnr]

    # ------------------------------------------------------------------ state
    def unpack(self, xk, u):
        nb, ng = self.nb, self.ng
        th = np.zeros(nb, dtype=np.result_type(xk, u))
        v = np.zeros(nb, dtype=np.result_type(xk, u))
        th[self.nonref] = xk[: nb - 1]
        v[self.pq] = xk[nb - 1:]
        v[self.net.gen_bus] = u[:ng]
        pg_nr = u[ng:]
        return th, v, pg_nr

    def bus_loads(self, pdk, qdk):
        Pd = np.zeros(self.nb)
        Qd = np.zeros(self.nb)
        np.add.at(Pd, self.net.load_bus, pdk)
        np.add.at(Qd, self.net.load_bus, qdk)
        return Pd, Qd

    # -------------------------------------------------------------- functions
    def powers(self, th, v):
        V = v * np.exp(1j * th)
        I = self.Ybus @ V
        S = V * np.conj(I)
        Sf = (self.Cf @ V) * np.conj(self.Yf @ V)
        St = (self.Ct @ V) * np.conj(self.Yt @ V)
        return V, I, S, Sf, St

    def evaluate(self, xk, u, pdk, qdk, wf):
        """f_i, g_i, h_i of one scenario (paper: state equation and constraints)."""
        th, v, pg_nr = self.unpack(xk, u)
        Pd, Qd = self.bus_loads(pdk, qdk)
        V, I, S, Sf, St = self.powers(th, v)
        P, Q = S.real, S.imag
        Pg_bus = np.zeros(self.nb)
        Pg_bus[self.pg_bus] = pg_nr
        g = np.concatenate([P[self.gbus_P] - Pg_bus[self.gbus_P] + Pd[self.gbus_P],
                            Q[self.gbus_Q] + Qd[self.gbus_Q]])
        pg_ref = P[self.ref] + Pd[self.ref]
        gb = self.net.gen_bus
        h = np.concatenate([[pg_ref], Q[gb] + Qd[gb],
                            Sf.real ** 2 + Sf.imag ** 2, St.real ** 2 + St.imag ** 2])
        pg = np.zeros(self.ng)
        pg[self.gnr] = pg_nr
        pg[self.gref] = pg_ref
        f = wf * np.sum(self.ca * pg ** 2 + self.cb * pg + self.cc)
        return f, g, h

    # ---------------------------------------------------- first derivatives
    def _dS_bus(self, V, I, v):
        """Textbook polar derivatives of bus injections S = V conj(Ybus V)."""
        E = V / v
        dS_dth = 1j * _diag(V) @ np.conj(_diag(I) - self.Ybus @ _diag(V))
        dS_dv = _diag(V) @ np.conj(self.Ybus @ _diag(E)) + np.conj(_diag(I)) @ _diag(E)
        return sp.csr_matrix(dS_dth), sp.csr_matrix(dS_dv)

    def _dS_br(self, C, Y, V, v):
        """Polar derivatives of line-end flows S_l = (C V)_l conj((Y V)_l)."""
        E = V / v
        Ib = Y @ V
        dth = 1j * (np.conj(_diag(Ib)) @ C @ _diag(V) - _diag(C @ V) @ np.conj(Y @ _diag(V)))
        dv = np.conj(_diag(Ib)) @ C @ _diag(E) + _diag(C @ V) @ np.conj(Y @ _diag(E))
        return sp.csr_matrix(dth), sp.csr_matrix(dv)

    def jacobians(self, xk, u, pdk, qdk, wf):
        """Sparse G_x, G_u, H_x, H_u and the gradient of f_i w.r.t. (x_i, u).

        Returned matrices use the x and u column orders of the module docstring.
        """
        th, v, pg_nr = self.unpack(xk, u)
        Pd, Qd = self.bus_loads(pdk, qdk)
        V, I, S, Sf, St = self.powers(th, v)
        dth, dv = self._dS_bus(V, I, v)
        J = sp.hstack([dth, dv]).tocsr()          # d S_bus / d(theta, v)
        JP, JQ = J.real.tocsr(), J.imag.tocsr()
        fth, fv = self._dS_br(self.Cf, self.Yf, V, v)
        tth, tv = self._dS_br(self.Ct, self.Yt, V, v)
        Jf = sp.hstack([fth, fv]).tocsr()
        Jt = sp.hstack([tth, tv]).tocsr()
        Jsf = 2 * (_diag(Sf.real) @ Jf.real + _diag(Sf.imag) @ Jf.imag)
        Jst = 2 * (_diag(St.real) @ Jt.real + _diag(St.imag) @ Jt.imag)
        gb = self.net.gen_bus
        Jg = sp.vstack([JP[self.gbus_P], JQ[self.gbus_Q]]).tocsr()
        Jh = sp.vstack([JP[[self.ref]], JQ[gb], Jsf, Jst]).tocsr()
        Gx = Jg[:, self.xcols]
        Hx = Jh[:, self.xcols]
        # u columns: voltage part from the full coordinates, Pg part explicit
        pgcol = np.zeros((self.n_x, self.ng - 1))
        row_of_bus = -np.ones(self.nb, dtype=np.int64)
        row_of_bus[self.gbus_P] = np.arange(len(self.gbus_P))
        for j, b in enumerate(self.pg_bus):
            pgcol[row_of_bus[b], j] = -1.0
        Gu = sp.hstack([Jg[:, self.ucols_v], sp.csr_matrix(pgcol)]).tocsr()
        Hu = sp.hstack([Jh[:, self.ucols_v], sp.csr_matrix((self.m, self.ng - 1))]).tocsr()
        # objective gradient
        pg_ref = S.real[self.ref] + Pd[self.ref]
        dref = JP[self.ref].toarray().ravel()
        dcost_ref = wf * (2 * self.ca[self.gref] * pg_ref + self.cb[self.gref])
        gx = dcost_ref * dref[self.xcols]
        gu = np.concatenate([dcost_ref * dref[self.ucols_v],
                             wf * (2 * self.ca[self.gnr] * pg_nr + self.cb[self.gnr])])
        return Gx.tocsr(), Gu, Hx.tocsr(), Hu, gx, gu

    # --------------------------------------------------- second derivatives
    @staticmethod
    def _quadform_hessian(c, th, v):
        """Hessian of F = Re sum_ik c_ik V_i conj(V_k) w.r.t. (theta, v).

        With D_ik = c_ik exp(j(theta_i - theta_k)), R = -Im D, Q = Re D and
        M = diag(v) Q diag(v):
          F_thth = M + M^T - diag(M 1 + M^T 1)
          F_thv  = diag(R v - R^T v) + diag(v) (R - R^T)
          F_vv   = Q + Q^T
        (derived by differentiating v_i v_k Re(D_ik) term by term).
        """
        c = sp.coo_matrix(c)
        n = len(th)
        d = c.data * np.exp(1j * (th[c.row] - th[c.col]))
        R = sp.csr_matrix((-d.imag, (c.row, c.col)), shape=(n, n))
        Q = sp.csr_matrix((d.real, (c.row, c.col)), shape=(n, n))
        M = _diag(v) @ Q @ _diag(v)
        Htt = M + M.T - _diag(M @ np.ones(n) + M.T @ np.ones(n))
        Htv = _diag(R @ v - R.T @ v) + _diag(v) @ (R - R.T)
        Hvv = Q + Q.T
        return sp.bmat([[Htt, Htv], [Htv.T, Hvv]]).tocsr()

    def hessian(self, xk, u, pdk, qdk, yk, zk, wf):
        """Hessian of f_i + y_i^T g_i + z_i^T h_i w.r.t. (x_i, u): W_xx, W_xu, W_uu^i."""
        nb, ng, nl = self.nb, self.ng, self.nl
        th, v, pg_nr = self.unpack(xk, u)
        Pd, Qd = self.bus_loads(pdk, qdk)
        V, I, S, Sf, St = self.powers(th, v)
        gb = self.net.gen_bus
        pg_ref = S.real[self.ref] + Pd[self.ref]
        wP = np.zeros(nb)
        wQ = np.zeros(nb)
        wP[self.gbus_P] = yk[: nb - 1]
        wQ[self.gbus_Q] = yk[nb - 1:]
        dcost_ref = wf * (2 * self.ca[self.gref] * pg_ref + self.cb[self.gref])
        wP[self.ref] += zk[0] + dcost_ref
        wQ[gb] += zk[1: 1 + ng]
        Hfull = self._quadform_hessian(_diag(wP - 1j * wQ) @ np.conj(self.Ybus), th, v)
        zf = zk[1 + ng: 1 + ng + nl]
        zt = zk[1 + ng + nl:]
        for C, Y, Sb, zb in ((self.Cf, self.Yf, Sf, zf), (self.Ct, self.Yt, St, zt)):
            w = 2 * zb * Sb.real - 1j * 2 * zb * Sb.imag
            Hfull = Hfull + self._quadform_hessian(C.T @ _diag(w) @ np.conj(Y), th, v)
            dth, dv = self._dS_br(C, Y, V, v)
            Jb = sp.hstack([dth, dv]).tocsr()
            Hfull = Hfull + 2 * (Jb.real.T @ _diag(zb) @ Jb.real + Jb.imag.T @ _diag(zb) @ Jb.imag)
        # rank-one curvature of the reference generator's cost
        dth, dv = self._dS_bus(V, I, v)
        dref = sp.hstack([dth, dv]).tocsr()[[self.ref]].real
        Hfull = Hfull + 2 * wf * self.ca[self.gref] * (dref.T @ dref)
        Hfull = Hfull.tocsr()
        Wxx = Hfull[self.xcols][:, self.xcols]
        Wxv = Hfull[self.xcols][:, self.ucols_v]
        Wvv = Hfull[self.ucols_v][:, self.ucols_v]
        Wxu = sp.hstack([Wxv, sp.csr_matrix((self.n_x, ng - 1))]).tocsr()
        Wuu = sp.bmat([[Wvv, None],
                       [None, _diag(2 * wf * self.ca[self.gnr])]]).tocsr()
        return Wxx.tocsr(), Wxu, Wuu

    # ------------------------------------------------------------- bounds
    def bounds(self):
        """Boxes on x, u and on the slack s = -h (s in [-h_upper, -h_lower])."""
        net = self.net
        nb, ng, nl = self.nb, self.ng, self.nl
        xl = np.concatenate([np.full(nb - 1, -np.inf), net.vmin[self.pq]])
        xu = np.concatenate([np.full(nb - 1, np.inf), net.vmax[self.pq]])
        ul = np.concatenate([net.vmin[net.gen_bus], net.pmin[self.gnr]])
        uu = np.concatenate([net.vmax[net.gen_bus], net.pmax[self.gnr]])
        hl = np.concatenate([[net.pmin[self.gref]], net.qmin, np.full(2 * nl, -np.inf)])
        hu = np.concatenate([[net.pmax[self.gref]], net.qmax, net.rate ** 2, net.rate ** 2])
        return xl, xu, ul, uu, -hu, -hl
