"""Parity at interior-point iterates of the oracle's own trajectory (first,
middle and last iterations: the IPM diagonals spread over many decades near
the end), on the 30-bus grid and the 118-bus grid with 8 scenarios, both
reduction variants, with the snapshot's delta_w (inertia correction, > 0 at
one of them) and with a forced delta_w = 1e-2.  The reduced matrix at
1e-10 relative Frobenius; every Newton-step block separately within
gpu_common.step_bar (1e-10, or 10 eps kappa_2(K_hat) when the conditioning
makes 1e-10 unreachable in FP64)."""
import numpy as np
import pytest

import gpu_common as gc
from oracle import kkt, ipm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (preset, scenarios, oracle iterations kept)
SNAPS = {("c0", None): (0, 1, 8, 12, 15, 19, 20), ("c1", 8): (0, 10, 21, 27, 29)}
_cache = {}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _trajectory(name, n_scen):
    key = (name, n_scen)
    if key not in _cache:
        inst = gc.instance(name, n_scen)
        prob = kkt.Problem(inst)
        res = ipm.solve(prob, snapshot_iters=SNAPS[key])
        assert res.status == "converged"
        _cache[key] = (inst, prob, res.history)
    return _cache[key]


CASES = [(n, s, v) for (n, s) in SNAPS for v in (1, 2)]


@pytest.mark.parametrize("name,n_scen,variant", CASES,
                         ids=[f"{n}-N{s or 1}-v{v}" for n, s, v in CASES])
def test_snapshot_iterates(name, n_scen, variant):
    inst, prob, hist = _trajectory(name, n_scen)
    assert [h["k"] for h in hist] == [k for k in SNAPS[(name, n_scen)] if k <= hist[-1]["k"]]
    ran_dw = []
    for h in hist:
        it = gc.snapshot_inputs(prob, h)
        for dw in (h["delta_w"], 1e-2):
            if dw != h["delta_w"] and dw < h["delta_w"]:
                continue          # the snapshot needed a larger correction
            prob_, ev, dg, red, _ = gc.oracle_state(inst, it, delta_w=dw)
            assert kkt.cholesky_info(red.khat)[0] == 0
            st = gc.oracle_step(prob_, ev, dg, red, dw, it)
            kappa = gc.cond2(red.khat)
            run = gc.GpuRun(inst, it, dw, torch, variant=variant)
            run.evaluate()
            run.condense()
            run.factor()
            run.step()
            code, scen = run.R.rkkt_status(run.p)
            assert code == 0, (code, scen)
            torch.cuda.synchronize()
            assert int(run.info.item()) == 0
            kh = run.khat.cpu().numpy()
            e_k = gc.rel_fro(kh, red.khat)
            s_min, s_max = dg.ss.min(), dg.ss.max()
            print(f"\n{name} k={h['k']} mu={h['mu']:.1e} delta_w={dw:g} Sigma_s in [{s_min:.1e}, "
                  f"{s_max:.1e}] khat {e_k:.2e}", flush=True)
            assert e_k <= 1e-10
            gc.check_step({k: v.cpu().numpy() for k, v in run.out.items()}, st, kappa)
            ran_dw.append(dw)
    assert any(d > 0 for d in ran_dw)
