"""Pins of the CPU oracle against facts fixed outside it (paper tables, closed
forms, calculus, textbook identities).  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synthgrid as sg
from oracle import kkt, ipm
from oracle.model import Model
import realeval

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_point(md, rng, N=None):
    def one():
        return np.concatenate([rng.normal(0, 0.1, md.nb - 1), rng.uniform(0.93, 1.07, len(md.pq))])
    x = one() if N is None else np.stack([one() for _ in range(N)])
    u = np.concatenate([rng.uniform(0.93, 1.07, md.ng), rng.uniform(0.1, 0.6, md.ng - 1)])
    return x, u


def rand_iterate(prob, rng, slack_noise=0.05):
    md = prob.model
    N = prob.N
    x, u = rand_point(md, rng, N)

    def duals(lo, hi, shape):
        return (np.where(np.isfinite(lo), rng.uniform(0.05, 2.0, shape), 0.0),
                np.where(np.isfinite(hi), rng.uniform(0.05, 2.0, shape), 0.0))
    it = kkt.Iterate(x, u, np.zeros((N, prob.m)), rng.normal(size=(N, prob.n_x)),
                     rng.normal(size=(N, prob.m)), *duals(prob.xl, prob.xu, (N, prob.n_x)),
                     *duals(prob.ul, prob.uu, prob.n_u), *duals(prob.sl, prob.su, (N, prob.m)))
    ev = kkt.evaluate(prob, it, 0.01, derivs=False, hess=False)
    s = -ev.h + rng.uniform(-slack_noise, slack_noise, ev.h.shape)
    width = np.where(np.isfinite(prob.su - prob.sl), prob.su - prob.sl, 1.0)
    it.s = np.clip(s, prob.sl + 1e-3 * width, prob.su - 1e-3 * width)
    return it


# ----------------------------------------------------------- paper tables
def test_dimensions_match_paper_tables():
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    per_case = {}
    for row in tab["table1"]:
        d = sg.dims(row["n_bus"], row["n_line"], row["n_gen"])
        assert d["n_x"] == row["n_x"] and d["n_u"] == row["n_u"], row["name"]
        per_case[row["name"]] = (row, d)
    for row in tab["table3"]:
        t1, d = per_case[row["name"]]
        N = row["N"]
        assert N * d["n_x"] + d["n_u"] == row["nvar"]
        assert N * (d["n_x"] + d["m"]) == row["ncon"]
        assert round(8 * d["n_u"] ** 2 / 2 ** 20, 1) == row["khat_mb"]


def test_oracle_model_sizes_on_case118_shape():
    """The oracle's variable split, built on a drawn grid with the case118 counts,
    has the paper's n_x and n_u (Table 1)."""
    md = Model(sg.preset("c1", n_scen=1).net)
    assert (md.n_x, md.n_u, md.m) == (181, 107, 2 * 186 + 54 + 1)


# --------------------------------------------------------------- functions
@pytest.mark.parametrize("name", ["tiny9", "c0", "c1"])
def test_complex_matrix_equals_per_line_real_form(name):
    inst = sg.preset(name, n_scen=1)
    md = Model(inst.net)
    rng = np.random.default_rng(3)
    x, u = rand_point(md, rng)
    pd, qd = inst.scen.pd[:, 0], inst.scen.qd[:, 0]
    f1, g1, h1 = md.evaluate(x, u, pd, qd, 0.37)
    f2, g2, h2 = realeval.evaluate(md, x, u, pd, qd, 0.37)
    assert abs(f1 - f2) <= 1e-12 * abs(f2)
    assert np.abs(g1 - g2).max() <= 1e-12 * max(1.0, np.abs(g2).max())
    assert np.abs(h1 - h2).max() <= 1e-12 * max(1.0, np.abs(h2).max())


def test_lossless_grid_conserves_active_power():
    inst = sg.preset("c0")
    net = inst.net
    net.r = np.zeros_like(net.r)
    net.b = np.zeros_like(net.b)
    md = Model(net)
    rng = np.random.default_rng(5)
    for _ in range(3):
        x, u = rand_point(md, rng)
        th, v, _ = md.unpack(x, u)
        _, _, S, Sf, St = md.powers(th, v)
        assert abs(S.real.sum()) < 1e-12
        assert np.abs(Sf.real + St.real).max() < 1e-12


# ----------------------------------------------------------- derivatives
@pytest.mark.parametrize("name", ["tiny9", "c0"])
def test_jacobians_by_complex_step(name):
    inst = sg.preset(name, n_scen=1)
    md = Model(inst.net)
    rng = np.random.default_rng(7)
    x, u = rand_point(md, rng)
    pd, qd = inst.scen.pd[:, 0], inst.scen.qd[:, 0]
    wf = 0.013
    Gx, Gu, Hx, Hu, gx, gu = md.jacobians(x, u, pd, qd, wf)
    A = np.vstack([np.concatenate([gx, gu])[None, :],
                   np.hstack([Gx.toarray(), Gu.toarray()]),
                   np.hstack([Hx.toarray(), Hu.toarray()])])
    z = np.concatenate([x, u]).astype(complex)
    n_x = len(x)
    J = np.zeros_like(A)
    hstep = 1e-30
    for j in range(len(z)):
        zz = z.copy()
        zz[j] += 1j * hstep
        f, g, h = realeval.evaluate(md, zz[:n_x], zz[n_x:], pd, qd, wf)
        J[:, j] = np.concatenate([[f], g, h]).imag / hstep
    scale = np.abs(J).max(axis=1, keepdims=True) + 1.0
    assert np.abs((A - J) / scale).max() < 1e-13


@pytest.mark.parametrize("name", ["tiny9", "c0"])
def test_hessian_by_central_differences(name):
    inst = sg.preset(name, n_scen=1)
    md = Model(inst.net)
    rng = np.random.default_rng(11)
    x, u = rand_point(md, rng)
    pd, qd = inst.scen.pd[:, 0], inst.scen.qd[:, 0]
    wf = 0.02
    y = rng.normal(size=md.n_x)
    z = rng.normal(size=md.m)
    Wxx, Wxu, Wuu = md.hessian(x, u, pd, qd, y, z, wf)
    W = np.block([[Wxx.toarray(), Wxu.toarray()], [Wxu.toarray().T, Wuu.toarray()]])
    n_x = len(x)

    def grad(zv):
        Gx, Gu, Hx, Hu, gx, gu = md.jacobians(zv[:n_x], zv[n_x:], pd, qd, wf)
        return (np.concatenate([gx, gu]) + np.hstack([Gx.toarray(), Gu.toarray()]).T @ y
                + np.hstack([Hx.toarray(), Hu.toarray()]).T @ z)
    z0 = np.concatenate([x, u])
    H = np.zeros_like(W)
    eps = 1e-6
    for j in range(len(z0)):
        e = np.zeros(len(z0))
        e[j] = eps
        H[:, j] = (grad(z0 + e) - grad(z0 - e)) / (2 * eps)
    assert np.abs(W - W.T).max() <= 1e-13 * np.abs(W).max()
    assert np.abs(H - W).max() <= 1e-6 * np.abs(W).max()


def test_newton_power_flow_converges_quadratically():
    """G_x is the exact Jacobian: Newton's method on g(., u) = 0 converges
    quadratically from a flat start (textbook power-flow behaviour)."""
    inst = sg.preset("c1", n_scen=1)
    md = Model(inst.net)
    net = inst.net
    pd, qd = 0.5 * inst.scen.pd[:, 0], 0.5 * inst.scen.qd[:, 0]
    pm = net.pmax.copy()
    pm[md.gref] = np.median(pm)
    pg = pm * pd.sum() / pm.sum()
    u = np.concatenate([np.ones(md.ng), pg[md.gnr]])
    x = np.concatenate([np.zeros(md.nb - 1), np.ones(len(md.pq))])
    errs = []
    for _ in range(8):
        _, g, _ = md.evaluate(x, u, pd, qd, 1.0)
        errs.append(np.abs(g).max())
        if errs[-1] < 1e-13:
            break
        x = x - spla.spsolve(md.jacobians(x, u, pd, qd, 1.0)[0].tocsc(), g)
    assert errs[-1] < 1e-12
    tail = [e for e in errs if e < 1e-2]
    for a, b in zip(tail[:-1], tail[1:]):
        if b > 1e-12:
            assert b <= 10 * a * a


# ------------------------------------------------------------ KKT systems
@pytest.mark.parametrize("name,dw", [("tiny5", 0.0), ("tiny9", 3.0), ("c0", 0.5)])
def test_full_condensed_reduced_steps_agree(name, dw):
    prob = kkt.Problem(sg.preset(name))
    rng = np.random.default_rng(13)
    it = rand_iterate(prob, rng)
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    rs = kkt.residuals(prob, it, ev, 0.05)
    red = kkt.reduced_hessian(prob, ev, dg, dw)
    if np.linalg.eigvalsh(red.khat).min() <= 0:
        dw = dw + 1.0 - np.linalg.eigvalsh(red.khat).min()
    a = kkt.newton_full(prob, ev, dg, rs, dw)
    b = kkt.newton_condensed(prob, ev, dg, rs, dw)
    c = kkt.newton_reduced(prob, ev, dg, rs, dw)
    va = np.concatenate([a[k].ravel() for k in ("px", "pu", "ps", "py", "pz")])
    for other in (b, c):
        vo = np.concatenate([other[k].ravel() for k in ("px", "pu", "ps", "py", "pz")])
        assert np.linalg.norm(vo - va) <= 1e-9 * np.linalg.norm(va)


def test_schur_complement_equals_reduced_matrix():
    """S_uu = A_0 - sum_i B_i A_i^-1 B_i^T with the blocks of the block-angular
    condensed system equals Z^T K Z, and the closed-form A_i^-1 inverts A_i."""
    prob = kkt.Problem(sg.preset("tiny9"))
    rng = np.random.default_rng(17)
    it = rand_iterate(prob, rng)
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    dw = 0.3
    red = kkt.reduced_hessian(prob, ev, dg, dw)
    nx = prob.n_x
    A0 = np.diag(dg.su + dw)
    S = A0.copy()
    for k in range(prob.N):
        Kxx, Kxu, Kuu = kkt.condensed_blocks(ev, dg, k, dw)
        Gx, Gu = ev.Gx[k].toarray(), ev.Gu[k].toarray()
        Ai = np.block([[Kxx.toarray(), Gx.T], [Gx, np.zeros((nx, nx))]])
        Bi = np.hstack([Kxu.toarray().T, Gu.T])
        Gi = np.linalg.inv(Gx)
        Ai_inv = np.block([[np.zeros((nx, nx)), Gi], [Gi.T, -Gi.T @ Kxx.toarray() @ Gi]])
        bound = 1e-14 * np.abs(Ai).max() * np.abs(Ai_inv).max() * 2 * nx
        assert np.abs(Ai @ Ai_inv - np.eye(2 * nx)).max() <= bound
        S += Kuu.toarray() - Bi @ np.linalg.solve(Ai, Bi.T)
    assert np.abs(S - red.khat).max() <= 1e-10 * np.abs(S).max()


def _solve_pf(md, x, u, pd, qd):
    for _ in range(30):
        _, g, _ = md.evaluate(x, u, pd, qd, 1.0)
        if np.abs(g).max() < 1e-14:
            break
        x = x - spla.spsolve(md.jacobians(x, u, pd, qd, 1.0)[0].tocsc(), g)
    return x


def test_reduced_hessian_is_derivative_of_reduced_gradient():
    """At power-flow-feasible points x_i(u), with adjoints
    y_i = -G_x^-T grad_x(f_i + z_i^T h_i), the Jacobian of the reduced gradient
    grad_u l(u) = sum_i grad_u(f_i + z_i^T h_i) + G_u^T y_i equals Z^T W Z
    (Sigma = 0, delta_w = 0)."""
    inst = sg.preset("tiny9")
    prob = kkt.Problem(inst)
    md = prob.model
    N = prob.N
    rng = np.random.default_rng(19)
    wf = 0.01
    z = rng.normal(size=(N, prob.m))
    u0 = np.concatenate([np.full(md.ng, 1.02), 0.4 * np.ones(md.ng - 1)])
    xs0 = np.zeros((N, prob.n_x))
    for k in range(N):
        xs0[k] = _solve_pf(md, np.concatenate([np.zeros(md.nb - 1), np.ones(len(md.pq))]),
                           u0, *prob.scen_loads(k))

    def reduced_grad(u):
        gsum = np.zeros(prob.n_u)
        ys = np.zeros((N, prob.n_x))
        xs = np.zeros((N, prob.n_x))
        for k in range(N):
            pd, qd = prob.scen_loads(k)
            xs[k] = _solve_pf(md, xs0[k].copy(), u, pd, qd)
            Gx, Gu, Hx, Hu, gx, gu = md.jacobians(xs[k], u, pd, qd, wf)
            ys[k] = -np.linalg.solve(Gx.toarray().T, gx + Hx.T @ z[k])
            gsum += gu + Hu.T @ z[k] + Gu.T @ ys[k]
        return gsum, xs, ys
    g0, xs, ys = reduced_grad(u0)
    zeros = lambda *s: np.zeros(s)  # noqa: E731
    it = kkt.Iterate(xs, u0, zeros(N, prob.m), ys, z, zeros(N, prob.n_x), zeros(N, prob.n_x),
                     zeros(prob.n_u), zeros(prob.n_u), zeros(N, prob.m), zeros(N, prob.m))
    ev = kkt.evaluate(prob, it, wf)
    dg = kkt.Diag(zeros(N, prob.n_x), zeros(prob.n_u), zeros(N, prob.m))
    khat = kkt.reduced_hessian(prob, ev, dg, 0.0).khat
    H = np.zeros((prob.n_u, prob.n_u))
    eps = 1e-5
    for j in range(prob.n_u):
        e = np.zeros(prob.n_u)
        e[j] = eps
        H[:, j] = (reduced_grad(u0 + e)[0] - reduced_grad(u0 - e)[0]) / (2 * eps)
    assert np.abs(khat - khat.T).max() <= 1e-12 * np.abs(khat).max()
    assert np.abs(H - khat).max() <= 1e-6 * np.abs(khat).max()


def test_cholesky_matches_lapack_and_inertia():
    prob = kkt.Problem(sg.preset("tiny9"))
    rng = np.random.default_rng(23)
    it = rand_iterate(prob, rng)
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    W, G, H = kkt.global_matrices(prob, ev)
    nd = W.shape[0]
    ny = G.shape[0]
    ss = dg.ss.ravel()
    for dw in (-50.0, -5.0, -0.5, 0.0, 0.5, 5.0, 50.0):
        red = kkt.reduced_hessian(prob, ev, dg, dw, keep=False)
        info, L = kkt.cholesky_info(red.khat)
        K = W + H.T @ (ss[:, None] * H) + np.diag(np.concatenate([dg.sx.ravel(), dg.su]) + dw)
        A = np.block([[K, G.T], [G, np.zeros((ny, ny))]])
        ev_ = np.linalg.eigvalsh(A)
        inertia_ok = (ev_ > 0).sum() == nd and (ev_ < 0).sum() == ny
        assert (info == 0) == inertia_ok
        if info == 0:
            Lr = sla.cholesky(red.khat, lower=True)
            assert np.abs(L - Lr).max() <= 1e-12 * np.abs(Lr).max()
            assert np.abs(L @ L.T - red.khat).max() <= 1e-13 * np.abs(red.khat).max() * red.khat.shape[0]


# ------------------------------------------------------------------- IPM
@pytest.mark.parametrize("name", ["tiny5", "tiny9", "c0"])
def test_ipm_converges_with_kkt_invariants(name):
    prob = kkt.Problem(sg.preset(name))
    res = ipm.solve(prob)
    assert res.status == "converged"
    ev = kkt.evaluate(prob, res.it, res.wf)
    assert np.abs(ev.g).max() <= 1e-8
    assert np.abs(ev.h + res.it.s).max() <= 1e-8
    assert res.kkt_error <= 1e-8
    dg = kkt.Diag(np.zeros_like(res.it.x), np.zeros(prob.n_u), np.zeros_like(res.it.s))
    # second-order sufficiency in the reduced space with the final diagonals
    dg = kkt.diagonals(prob, res.it)
    khat = kkt.reduced_hessian(prob, ev, dg, 0.0, keep=False).khat
    assert np.linalg.eigvalsh(khat).min() > 0


# -------------------------------------------------- the pins have teeth
def test_planted_hessian_sign_error_is_caught(monkeypatch):
    """Flipping the sign of one curvature term in the oracle Hessian must make
    the finite-difference pin fail."""
    orig = Model._quadform_hessian

    def broken(c, th, v):
        H = orig(c, th, v).tolil()
        n = len(th)
        H[n:, n:] = -H[n:, n:]       # wrong sign on the magnitude block
        return H.tocsr()
    monkeypatch.setattr(Model, "_quadform_hessian", staticmethod(broken))
    with pytest.raises(AssertionError):
        test_hessian_by_central_differences("tiny9")


def test_planted_reduction_error_is_caught(monkeypatch):
    """Dropping the S^T K_xu cross term from the reduced matrix must break the
    equality of the reduced and the full Newton step."""
    orig = kkt.reduced_hessian

    def broken(prob, ev, dg, dw, keep=True):
        red = orig(prob, ev, dg, dw, keep)
        for k in range(prob.N):
            KxuS = red.Kxu[k].T @ red.S[k]
            red.khat -= KxuS.T
        return red
    monkeypatch.setattr(kkt, "reduced_hessian", broken)
    with pytest.raises(AssertionError):
        test_full_condensed_reduced_steps_agree("tiny9", 3.0)


def test_three_step_columns_equal_reduced_matrix():
    """The paper's three-step K_hat V product equals the reduced matrix built
    from S = -G_x^-1 G_u (two independent oracle paths)."""
    prob = kkt.Problem(sg.preset("tiny9"))
    rng = np.random.default_rng(29)
    it = rand_iterate(prob, rng)
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    full = kkt.reduced_hessian(prob, ev, dg, 0.7).khat
    cols = [0, 2, prob.n_u - 1]
    part = kkt.reduced_hessian_columns(prob, ev, dg, 0.7, cols)
    assert np.abs(part - full[:, cols]).max() <= 1e-11 * np.abs(full).max()


def test_augmented_residual_vanishes_at_the_newton_step():
    prob = kkt.Problem(sg.preset("tiny9"))
    rng = np.random.default_rng(31)
    it = rand_iterate(prob, rng)
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    rs = kkt.residuals(prob, it, ev, 0.05)
    dw = 3.0
    st = kkt.newton_full(prob, ev, dg, rs, dw)
    r, s = kkt.augmented_residual(prob, ev, dg, rs, dw, st)
    assert r <= 1e-12 * s
    bad = dict(st)
    bad["pu"] = st["pu"] * (1 + 1e-6)
    r2, _ = kkt.augmented_residual(prob, ev, dg, rs, dw, bad)
    assert r2 > 1e3 * r


# ------------------------------------------- sparse and dense G_x factors
@pytest.mark.parametrize("n_bus,n_line,n_gen", [(118, 186, 54), (2000, 3000, 300)])
def test_sparse_and_dense_gx_factors_agree(monkeypatch, n_bus, n_line, n_gen):
    """The SuperLU branch of the G_x factor (taken when n_x > 3000, as at the
    9241-bus size) and the dense LAPACK branch give the same solves, plain
    and transposed, on a grid below and one above the threshold; both solve
    the system to rounding (residual against the sparse matrix)."""
    inst = sg.make_instance(n_bus, n_line, n_gen, 1, 4242)
    prob = kkt.Problem(inst)
    rng = np.random.default_rng(5)
    x, u = rand_point(prob.model, rng)
    Gx, Gu = prob.model.jacobians(x, u, inst.scen.pd[:, 0], inst.scen.qd[:, 0], 0.01)[:2]
    B = np.concatenate([Gu.toarray()[:, :7], rng.normal(size=(prob.n_x, 3))], axis=1)
    out = {}
    for dense_max in (0, 10 ** 9):
        monkeypatch.setattr(kkt, "DENSE_MAX", dense_max)
        fac = kkt._GxFactor(Gx)
        assert fac.sparse == (dense_max == 0)
        X, Y = fac.solve(B), fac.solve(B, trans=True)
        scale = spla.norm(Gx, 1) * np.abs(X).max()
        assert np.abs(Gx @ X - B).max() <= 1e-11 * scale
        assert np.abs(Gx.T @ Y - B).max() <= 1e-11 * spla.norm(Gx, 1) * np.abs(Y).max()
        out[dense_max] = (X, Y)
    for a, b in zip(out[0], out[10 ** 9]):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def test_reduced_matrix_same_with_sparse_gx_factor(monkeypatch):
    inst = sg.preset("c1", n_scen=3)
    prob = kkt.Problem(inst)
    it = rand_iterate(prob, np.random.default_rng(17))
    ev = kkt.evaluate(prob, it, 0.01)
    dg = kkt.diagonals(prob, it)
    a = kkt.reduced_hessian(prob, ev, dg, 0.5).khat
    monkeypatch.setattr(kkt, "DENSE_MAX", 0)
    b = kkt.reduced_hessian(prob, ev, dg, 0.5).khat
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


# ------------------------------------------------ bounds of the slack form
def _network_quantities(md, inst, xk, u, k):
    """Bus voltages, generator outputs and line flows at a point, written from
    the network data (textbook pi-line flows of realeval), not from the
    oracle's h or its bounds."""
    net = inst.net
    th = np.zeros(md.nb)
    v = np.zeros(md.nb)
    th[md.nonref] = xk[: md.nb - 1]
    v[md.pq] = xk[md.nb - 1:]
    v[net.gen_bus] = u[: md.ng]
    pf, qf, pt, qt = realeval.line_flows(md, th, v)
    P = np.zeros(md.nb)
    Q = np.zeros(md.nb)
    np.add.at(P, net.line_from, pf)
    np.add.at(P, net.line_to, pt)
    np.add.at(Q, net.line_from, qf)
    np.add.at(Q, net.line_to, qt)
    Pd = np.zeros(md.nb)
    Qd = np.zeros(md.nb)
    np.add.at(Pd, net.load_bus, inst.scen.pd[:, k])
    np.add.at(Qd, net.load_bus, inst.scen.qd[:, k])
    pg = np.zeros(md.ng)
    pg[md.gnr] = u[md.ng:]
    pg[md.gref] = P[md.ref] + Pd[md.ref]
    qg = Q[net.gen_bus] + Qd[net.gen_bus]
    return v, pg, qg, pf ** 2 + qf ** 2, pt ** 2 + qt ** 2


@pytest.mark.parametrize("name,n_scen", [("c0", None), ("c1", 4)])
def test_converged_point_respects_the_network_limits(name, n_scen):
    """The boxes of the slack form (s in [-h_U, -h_L] and the x, u boxes) are
    the network's limits: at a converged interior point every bus voltage is
    in [Vmin, Vmax], every generator's active and reactive output in its
    range and every line end's |S|^2 <= rate^2 (1e-8), and in each family at
    least one limit is active (1e-6), so a misplaced or mis-signed bound
    would show."""
    inst = sg.preset(name, n_scen=n_scen)
    prob = kkt.Problem(inst)
    res = ipm.solve(prob)
    assert res.status == "converged"
    md, net = prob.model, inst.net
    slack = {"V": [], "Pg": [], "Qg": [], "flow": []}
    for k in range(prob.N):
        v, pg, qg, sf, st = _network_quantities(md, inst, res.it.x[k], res.it.u, k)
        slack["V"].append(np.concatenate([v - net.vmin, net.vmax - v]))
        slack["Pg"].append(np.concatenate([pg - net.pmin, net.pmax - pg]))
        slack["Qg"].append(np.concatenate([qg - net.qmin, net.qmax - qg]))
        slack["flow"].append(np.concatenate([net.rate ** 2 - sf, net.rate ** 2 - st]))
    for fam, parts in slack.items():
        a = np.concatenate(parts)
        assert a.min() >= -1e-8, fam
        assert a.min() <= 1e-6, fam


# ---------------------------- two FP64 steps and the conditioning of K_hat
def test_full_and_reduced_steps_agree_within_the_conditioning_bound():
    """On interior-point iterates from the first to the last (the oracle's own
    trajectory on the 30-bus grid, Sigma spreading over up to 20 decades near
    the end), the dense LU solve of the augmented system and the reduced
    Cholesky solve agree block by block within eps kappa_2(K_hat): the reading
    of a relative 1e-10 step tolerance when kappa_2(K_hat) eps exceeds it."""
    prob = kkt.Problem(sg.preset("c0"))
    res = ipm.solve(prob, snapshot_iters=tuple(range(0, 40, 3)) + (19, 20))
    assert len(res.history) >= 6
    eps = np.finfo(float).eps
    worst = 0.0
    for h in res.history:
        it = h["it"]
        ev = kkt.evaluate(prob, it, h["wf"])
        dg = kkt.diagonals(prob, it)
        rs = kkt.residuals(prob, it, ev, h["mu"])
        red = kkt.reduced_hessian(prob, ev, dg, h["delta_w"])
        a = kkt.newton_reduced(prob, ev, dg, rs, h["delta_w"], red)
        b = kkt.newton_full(prob, ev, dg, rs, h["delta_w"])
        bound = max(1e-12, eps * np.linalg.cond(red.khat))
        for k in ("px", "pu", "ps", "py", "pz"):
            e = np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])
            assert e <= bound, (h["k"], k, e, bound)
            worst = max(worst, e / bound)
    assert worst > 0
