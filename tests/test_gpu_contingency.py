"""Contingency scenarios on the GPU: with a line tripped (zero admittance on
the shared pattern) in some scenarios, the reduced matrix and the evaluation
equal those of the oracle that deletes the line from those scenarios' grids."""
import numpy as np
import pytest

import gpu_common as gc
import synthgrid as sg
from oracle import contingency as ct

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("variant", [1, 2])
def test_tripped_lines_match_the_deleted_line_oracle(variant):
    import paper_2301_04869_amd as R
    inst = gc.instance("c1", 16)
    it = gc.iterate(inst, seed=31)
    N, nl = inst.scen.n_scen, inst.net.n_line
    tripped = sg.line_outages(inst.net, N, seed=9)
    print(f"\ntripped lines per scenario: {tripped.tolist()}", flush=True)
    status = np.ones((N, nl))
    for k, l in enumerate(tripped):
        if l >= 0:
            status[k, l] = 0.0
    dw = 0.5
    run = gc.GpuRun(inst, it, dw, torch, variant=variant)
    R.rkkt_set_line_status(run.p, torch.tensor(status, dtype=torch.float64, device="cuda"))
    run.evaluate()
    run.condense()
    code, scen = R.rkkt_status(run.p)
    assert code == 0, (code, scen)
    torch.cuda.synchronize()
    g_o, h_o = ct.evaluate_with_outages(inst, it, tripped)
    for nm, a, b in (("g", run.g, g_o), ("h", run.h, h_o)):
        err = np.abs(a.cpu().numpy() - b).max() / np.abs(b).max()
        print(f"  {nm}: max rel err {err:.2e}")
        assert err <= 1e-12, nm
    kh = run.khat.cpu().numpy()
    ko = ct.khat_with_outages(inst, it, dw, tripped)
    e = gc.rel_fro(kh, ko)
    print(f"  khat: rel err {e:.2e} against the deleted-line oracle")
    assert e <= 1e-12
    # back in service: the plain reduced matrix again
    R.rkkt_set_line_status(run.p, torch.ones((N, nl), dtype=torch.float64, device="cuda"))
    run.evaluate()
    run.condense()
    torch.cuda.synchronize()
    e0 = gc.rel_fro(run.khat.cpu().numpy(), ct.khat_with_outages(inst, it, dw, np.full(N, -1)))
    print(f"  khat with every line in service: rel err {e0:.2e}")
    assert e0 <= 1e-12


@pytest.mark.parametrize("variant", [1, 2])
def test_step_with_tripped_lines_matches_the_deleted_line_oracle(variant):
    """The Newton step (reduced right-hand side, p_u, recovery) with lines
    tripped in some scenarios equals the step of the oracle that deletes the
    lines (each block within gpu_common.step_bar)."""
    import paper_2301_04869_amd as R
    inst = gc.instance("c1", 16)
    it = gc.iterate(inst, seed=33)
    it["y"] *= 0.01
    it["z"] *= 0.01
    N, nl = inst.scen.n_scen, inst.net.n_line
    tripped = sg.line_outages(inst.net, N, seed=10)
    status = np.ones((N, nl))
    for k, l in enumerate(tripped):
        if l >= 0:
            status[k, l] = 0.0
    dw = 0.5
    ko = ct.khat_with_outages(inst, it, dw, tripped)
    assert np.linalg.eigvalsh(ko).min() > 0
    run = gc.GpuRun(inst, it, dw, torch, variant=variant)
    R.rkkt_set_line_status(run.p, torch.tensor(status, dtype=torch.float64, device="cuda"))
    run.evaluate()
    run.condense()
    run.factor()
    run.step()
    code, scen = R.rkkt_status(run.p)
    assert code == 0, (code, scen)
    torch.cuda.synchronize()
    assert int(run.info.item()) == 0
    e = gc.rel_fro(run.khat.cpu().numpy(), ko)
    print(f"\ntripped {tripped.tolist()} khat {e:.2e}", flush=True)
    assert e <= 1e-10
    st = ct.step_with_outages(inst, it, dw, tripped)
    gc.check_step({k: v.cpu().numpy() for k, v in run.out.items()}, st, gc.cond2(ko))
