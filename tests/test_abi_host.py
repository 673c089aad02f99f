"""The C ABI library loads on the CPU, exports every symbol include/*.h
declare, and its host-only analysis gives the documented sizes.  No GPU."""
import os
import re

import numpy as np
import pytest

import synthgrid as sg

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"\b(rkkt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2301_04869_amd as R
    L = R.lib()
    headers = sorted(h for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h"))
    assert headers == ["rkkt.h", "rkkt_mlp.h"]
    for h in headers:
        for n in _declared(h):
            assert hasattr(L, n), (h, n)
    assert set(_declared("rkkt.h")) == set(R.EXPORTS)
    assert set(_declared("rkkt_mlp.h")) == set(R.MLP_EXPORTS)


@pytest.mark.parametrize("name", ["tiny5", "c0", "c1", "c4"])
def test_host_analysis_sizes(name):
    import paper_2301_04869_amd as R
    inst = sg.preset(name)
    net = inst.net
    d = R.rkkt_analyze(net, inst.scen.n_scen)
    dd = sg.dims(net.n_bus, net.n_line, net.n_gen)
    assert (d["n_x"], d["n_u"], d["m"]) == (dd["n_x"], dd["n_u"], dd["m"])
    assert d["nnz_lu"] >= d["nnz_gx"] >= d["n_x"]
    assert d["levels_up"] >= 1 and d["levels_down"] >= 1


def test_host_analysis_rejects_bad_networks():
    import paper_2301_04869_amd as R
    net = sg.preset("tiny9").net
    bad = sg.preset("tiny9").net
    bad.ref_bus = int(np.setdiff1d(np.arange(bad.n_bus), bad.gen_bus)[0])
    with pytest.raises(R.RkktError) as e:
        R.rkkt_analyze(bad, 1)
    assert e.value.code == -1
    bad = sg.preset("tiny9").net
    bad.line_to = bad.line_from.copy()
    with pytest.raises(R.RkktError):
        R.rkkt_analyze(bad, 1)
    with pytest.raises(R.RkktError):
        R.rkkt_analyze(net, 0)
