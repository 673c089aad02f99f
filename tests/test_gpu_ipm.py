"""The device interior-point driver against the oracle's outer loop (same
written rules, separate code): both converge, same iteration count within a
small margin, final objective within 1e-6 relative, KKT error <= 1e-8."""
import numpy as np
import pytest

import synthgrid as sg
from oracle import kkt, ipm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,n_scen", [("tiny5", None), ("tiny9", None), ("c0", None), ("c1", 8)])
def test_device_ipm_matches_oracle(name, n_scen):
    import paper_2301_04869_amd as R
    inst = sg.preset(name, n_scen=n_scen)
    ref = ipm.solve(kkt.Problem(inst))
    p = R.rkkt_create(inst.net, inst.scen.pd.T, inst.scen.qd.T)
    d = p.dims
    x = torch.zeros(d["n_scen"], d["n_x"], dtype=torch.float64, device="cuda")
    u = torch.zeros(d["n_u"], dtype=torch.float64, device="cuda")
    res = R.rkkt_solve(p, x=x, u=u)
    print(f"\n{name}: oracle {ref.status} it={ref.iters} obj={ref.obj:.10e} | "
          f"device {res['status']} it={res['iters']} obj={res['obj']:.10e} "
          f"kkt={res['kkt_error']:.2e} fact={res['factorizations']}", flush=True)
    assert ref.status == "converged"
    assert res["status"] == "converged"
    assert res["kkt_error"] <= 1e-8
    assert abs(res["obj"] - ref.obj) <= 1e-6 * abs(ref.obj)
    assert abs(res["iters"] - ref.iters) <= 2
    assert np.abs(u.cpu().numpy() - ref.it.u).max() <= 1e-5
