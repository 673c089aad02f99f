"""Instance generator: determinism, structure, counts.  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import synthgrid as sg


@pytest.mark.parametrize("name", ["tiny5", "tiny9", "c0", "c1"])
def test_preset_counts_and_connectivity(name):
    inst = sg.preset(name)
    net = inst.net
    _, nb, nl, ng, ns, loads, sigma, _, _ = sg.PRESETS[name]
    assert (net.n_bus, net.n_line, net.n_gen, inst.scen.n_scen) == (nb, nl, ng, ns)
    A = sp.csr_matrix((np.ones(nl), (net.line_from, net.line_to)), shape=(nb, nb))
    ncomp, _ = csg.connected_components(A, directed=False)
    assert ncomp == 1
    pairs = set(zip(np.minimum(net.line_from, net.line_to), np.maximum(net.line_from, net.line_to)))
    assert len(pairs) == nl and np.all(net.line_from != net.line_to)
    assert len(set(net.gen_bus.tolist())) == ng
    assert net.ref_bus == net.gen_bus[np.argmax(net.pmax)]
    assert np.all((net.r >= 0.01) & (net.r <= 0.1) & (net.x >= 0.05) & (net.x <= 0.4))
    assert np.all((net.b >= 0) & (net.b <= 0.05))
    assert np.allclose(net.qd, 0.3 * net.pd)
    if loads == "pq":
        assert net.n_load == nb - ng
    else:
        assert net.n_load == loads
    fac = inst.scen.pd / net.pd[:, None]
    assert np.all((fac >= 0.5 - 1e-15) & (fac <= 1.5 + 1e-15))
    assert np.allclose(inst.scen.qd, 0.3 * inst.scen.pd)


def test_generator_is_deterministic():
    a = sg.preset("c1")
    b = sg.preset("c1")
    for k in ("line_from", "line_to", "r", "x", "b", "rate", "gen_bus", "pmax", "c2", "c1"):
        assert np.array_equal(getattr(a.net, k), getattr(b.net, k))
    assert np.array_equal(a.scen.pd, b.scen.pd)


def test_accepted_attempts_match_table():
    path = os.path.join(os.path.dirname(__file__), "golden", "attempts.json")
    table = json.load(open(path))
    for name, att in table.items():
        assert sg.PRESETS[name][-1] == att, name
