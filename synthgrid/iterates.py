"""Seeded synthetic interior-point iterates and right-hand sides.

Plain random draws with the shapes and value ranges of an interior-point
iterate of the block AC-OPF (no model arithmetic): angles ~ N(0, 0.1),
magnitudes ~ U[0.93, 1.07], generator outputs inside their boxes,
multipliers ~ N(0, 1), IPM diagonals ~ U[lo, hi] >= 0, Newton residuals
~ N(0, 1).  Arrays are scenario-major ([N][n]).
"""
from __future__ import annotations

import numpy as np

from .grid import dims


def random_iterate(net, n_scen: int, seed: int, sigma_range=(0.1, 10.0)) -> dict:
    rng = np.random.default_rng(seed)
    d = dims(net.n_bus, net.n_line, net.n_gen)
    nx, nu, m = d["n_x"], d["n_u"], d["m"]
    n_th = net.n_bus - 1
    x = np.empty((n_scen, nx))
    x[:, :n_th] = rng.normal(0.0, 0.1, (n_scen, n_th))
    x[:, n_th:] = rng.uniform(0.93, 1.07, (n_scen, nx - n_th))
    ref_gen = int(np.nonzero(net.gen_bus == net.ref_bus)[0][0])
    gnr = [g for g in range(net.n_gen) if g != ref_gen]
    lo, hi = net.pmin[gnr], net.pmax[gnr]
    u = np.concatenate([rng.uniform(0.93, 1.07, net.n_gen), lo + (hi - lo) * rng.uniform(0.1, 0.9, len(gnr))])
    a, b = sigma_range
    return dict(
        x=x, u=u,
        y=rng.normal(size=(n_scen, nx)), z=rng.normal(size=(n_scen, m)),
        obj_weight=float(rng.uniform(0.001, 0.05)) / n_scen,
        sigma_x=rng.uniform(a, b, (n_scen, nx)), sigma_u=rng.uniform(a, b, nu),
        sigma_s=rng.uniform(a, b, (n_scen, m)),
        r1x=rng.normal(size=(n_scen, nx)), r1u=rng.normal(size=nu),
        r2=rng.normal(size=(n_scen, m)), r3=rng.normal(size=(n_scen, nx)),
        r4=rng.normal(size=(n_scen, m)),
    )
