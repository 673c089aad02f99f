"""Pick the accepted attempt of every named workload (writes attempts.json).

Rule: the first attempt whose base-case power flow (distributed slack, load
continuation from 5% to 100%, all generator magnitudes at 1.0) converges and,
for grids of at most a few hundred buses, whose N = 1 interior-point solve by
the oracle converges.  The 9241-bus grid is checked by the power flow only:
an oracle interior-point solve at that size takes hours.

Calls only the oracle and the instance generator.  Run from the repository
root:  python tests/golden/select_attempts.py [names...]
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import scipy.sparse.linalg as spla

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import synthgrid as sg  # noqa: E402
from oracle import kkt, ipm  # noqa: E402


def base_power_flow(inst, vg=1.0):
    prob = kkt.Problem(inst)
    md, net = prob.model, inst.net
    x = np.concatenate([np.zeros(md.nb - 1), np.ones(len(md.pq))])
    pd0 = inst.net.pd
    qd0 = inst.net.qd
    pm = net.pmax.copy()
    pm[md.gref] = np.median(pm)
    loss = 0.0
    for lam in np.arange(0.05, 1.0001, 0.05):
        pdk, qdk = lam * pd0, lam * qd0
        for _ in range(6):
            pg = pm * (pdk.sum() + loss) / pm.sum()
            u = np.concatenate([np.full(md.ng, vg), pg[md.gnr]])
            for _ in range(20):
                _, g, h = md.evaluate(x, u, pdk, qdk, 1.0)
                if not np.all(np.isfinite(g)) or np.abs(g).max() < 1e-9:
                    break
                Gx = md.jacobians(x, u, pdk, qdk, 1.0)[0]
                x = x - spla.spsolve(Gx.tocsc(), g)
            if not np.all(np.isfinite(g)) or np.abs(g).max() > 1e-6:
                return False
            if abs(h[0] - pg[md.gref]) < 1e-3:
                break
            loss = h[0] + pg[md.gnr].sum() - pdk.sum()
    return True


def accept(name, attempt, ipm_check=True):
    inst = sg.preset(name, attempt=attempt)
    if not base_power_flow(inst):
        return False, "power flow"
    if not ipm_check:
        return True, "power flow only"
    one = sg.preset(name, attempt=attempt, n_scen=1)
    res = ipm.solve(kkt.Problem(one))
    return res.status == "converged", f"ipm {res.status} in {res.iters}"


def main(names):
    path = os.path.join(os.path.dirname(__file__), "attempts.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        for a in range(50):
            ok, why = accept(name, a, ipm_check=(name != "c4"))
            print(name, a, ok, why, flush=True)
            if ok:
                table[name] = a
                break
    json.dump(table, open(path, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["tiny5", "tiny9", "c0", "c1", "c4"])
