"""Contingency scenarios on the CPU: the outage draw keeps the grid
connected, and the outage oracle is pinned to the plain oracle (no outage:
the same K_hat; one outage: K_hat moves by exactly the difference of that
scenario's terms, each computed by the plain oracle on a one-scenario
instance of the grid with and without the line)."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import synthgrid as sg
from synthgrid.iterates import random_iterate
from oracle import kkt
from oracle import contingency as ct


def _plain_khat(inst, it, dw):
    prob = kkt.Problem(inst)
    N = prob.N
    z0 = np.zeros
    I = kkt.Iterate(it["x"], it["u"], z0((N, prob.m)), it["y"], it["z"], z0((N, prob.n_x)),
                    z0((N, prob.n_x)), z0(prob.n_u), z0(prob.n_u), z0((N, prob.m)), z0((N, prob.m)))
    ev = kkt.evaluate(prob, I, it["obj_weight"])
    dg = kkt.Diag(it["sigma_x"], it["sigma_u"], it["sigma_s"])
    return kkt.reduced_hessian(prob, ev, dg, dw).khat


def _one_scenario(inst, it, k, net, rows):
    sc = sg.Scenarios(inst.scen.pd[:, k:k + 1], inst.scen.qd[:, k:k + 1], inst.scen.sigma, inst.scen.seed)
    i1 = sg.Instance(inst.name, net, sc)
    it1 = {key: (v[k:k + 1] if isinstance(v, np.ndarray) and v.ndim == 2 else v) for key, v in it.items()}
    it1["z"] = it1["z"][:, rows]
    it1["sigma_s"] = it1["sigma_s"][:, rows]
    it1["sigma_u"] = np.zeros_like(it["sigma_u"])
    return i1, it1


def test_outages_keep_the_grid_connected_and_are_seeded():
    inst = sg.preset("c1")
    out = sg.line_outages(inst.net, 64, seed=5)
    assert np.array_equal(out, sg.line_outages(inst.net, 64, seed=5))
    assert (out >= 0).any() and (out < 0).any()
    net = inst.net
    for l in set(out[out >= 0].tolist()):
        keep = np.arange(net.n_line) != l
        adj = sp.coo_matrix((np.ones(keep.sum()), (net.line_from[keep], net.line_to[keep])),
                            shape=(net.n_bus, net.n_bus))
        assert connected_components(adj, directed=False)[0] == 1


def test_no_outage_is_the_plain_oracle():
    inst = sg.preset("c1", n_scen=3)
    it = random_iterate(inst.net, 3, 7)
    a = ct.khat_with_outages(inst, it, 0.5, np.full(3, -1))
    b = _plain_khat(inst, it, 0.5)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_one_outage_moves_khat_by_that_scenarios_terms():
    inst = sg.preset("c1", n_scen=3)
    it = random_iterate(inst.net, 3, 8)
    l = int(sg.line_outages(inst.net, 50, seed=1, frac=1.0)[0])
    tripped = np.array([-1, l, -1])
    full_rows = np.arange(1 + inst.net.n_gen + 2 * inst.net.n_line)
    a = ct.khat_with_outages(inst, it, 0.0, tripped) - ct.khat_with_outages(inst, it, 0.0, np.full(3, -1))
    i_del, it_del = _one_scenario(inst, it, 1, ct.without_line(inst.net, l), ct.kept_rows(inst.net, l))
    i_all, it_all = _one_scenario(inst, it, 1, inst.net, full_rows)
    b = _plain_khat(i_del, it_del, 0.0) - _plain_khat(i_all, it_all, 0.0)
    assert np.linalg.norm(b) > 0
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def _plain_step(inst, it, dw):
    prob = kkt.Problem(inst)
    N = prob.N
    z0 = np.zeros
    I = kkt.Iterate(it["x"], it["u"], z0((N, prob.m)), it["y"], it["z"], z0((N, prob.n_x)),
                    z0((N, prob.n_x)), z0(prob.n_u), z0(prob.n_u), z0((N, prob.m)), z0((N, prob.m)))
    ev = kkt.evaluate(prob, I, it["obj_weight"])
    dg = kkt.Diag(it["sigma_x"], it["sigma_u"], it["sigma_s"])
    rs = kkt.Resid(it["r1x"], it["r1u"], it["r2"], it["r3"], it["r4"])
    return kkt.newton_reduced(prob, ev, dg, rs, dw)


def test_step_without_outages_is_the_plain_oracle():
    inst = sg.preset("c1", n_scen=3)
    it = random_iterate(inst.net, 3, 11)
    it["y"] *= 0.01
    it["z"] *= 0.01
    a = ct.step_with_outages(inst, it, 0.5, np.full(3, -1))
    b = _plain_step(inst, it, 0.5)
    for k in ("px", "pu", "ps", "py", "pz"):
        assert np.linalg.norm(a[k] - b[k]) <= 1e-10 * np.linalg.norm(b[k]), k


def test_step_with_outages_solves_each_scenarios_own_system():
    """Every block row of the augmented system (eq. of the augmented system),
    written out with each scenario's deleted-line matrices, vanishes at the
    step; the deleted line's flow rows carry Sigma_s p_s + p_z + r2 = 0 and
    p_s + r4 = 0."""
    from oracle.model import Model
    inst = sg.preset("c1", n_scen=4)
    it = random_iterate(inst.net, 4, 12)
    it["y"] *= 0.01
    it["z"] *= 0.01
    net = inst.net
    tripped = np.array([-1, 3, -1, 7])
    tripped[1] = sg.line_outages(net, 50, seed=2, frac=1.0)[0]
    tripped[3] = sg.line_outages(net, 50, seed=3, frac=1.0)[0]
    dw = 0.5
    st = ct.step_with_outages(inst, it, dw, tripped)
    m = 1 + net.n_gen + 2 * net.n_line
    pu = st["pu"]
    ru = (it["sigma_u"] + dw) * pu + it["r1u"]
    scale_u = np.abs(ru).max()
    for k in range(4):
        l = int(tripped[k])
        rows = ct.kept_rows(net, l) if l >= 0 else np.arange(m)
        net_k = ct.without_line(net, l) if l >= 0 else net
        md = Model(net_k)
        Gx, Gu, Hx, Hu, _, _ = md.jacobians(it["x"][k], it["u"], inst.scen.pd[:, k], inst.scen.qd[:, k],
                                            it["obj_weight"])
        Wxx, Wxu, Wuu = md.hessian(it["x"][k], it["u"], inst.scen.pd[:, k], inst.scen.qd[:, k],
                                   it["y"][k], it["z"][k][rows], it["obj_weight"])
        px, py = st["px"][k], st["py"][k]
        ps, pz = st["ps"][k], st["pz"][k]
        ss = it["sigma_s"][k]
        r1 = (Wxx @ px + (it["sigma_x"][k] + dw) * px + Wxu @ pu + Gx.T @ py + Hx.T @ pz[rows]
              + it["r1x"][k])
        r2 = ss * ps + pz + it["r2"][k]
        r3 = Gx @ px + Gu @ pu + it["r3"][k]
        r4 = it["r4"][k] + ps
        r4[rows] += Hx @ px + Hu @ pu
        ru = ru + Wxu.T @ px + Wuu @ pu + Gu.T @ py + Hu.T @ pz[rows]
        for r in (r1, r2, r3, r4):
            assert np.abs(r).max() <= 1e-9 * max(1.0, np.abs(st["px"]).max(), np.abs(st["pz"]).max())
        scale_u = max(scale_u, np.abs(Wuu @ pu).max(), np.abs(Gu.T @ py).max())
    assert np.abs(ru).max() <= 1e-9 * scale_u
