"""Parity of the path the benchmark times: the 118-bus workload with all 128
scenarios, in the launch configuration bench.py uses (automatic reduction
variant and column tile), run as one rkkt_iterate pass and as replays of its
captured graph, against the oracle on the same seeded iterate.  Every output
is compared: evaluation (1e-12), the reduced matrix (1e-10 relative
Frobenius), its Cholesky factor and each Newton-step block (p_x, p_u, p_s,
p_y, p_z) separately at 1e-10 (or the conditioning bound of
gpu_common.step_bar)."""
import numpy as np
import pytest

import gpu_common as gc
from oracle import kkt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 2024          # bench.py's default iterate seed


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bench_delta_w(inst, it):
    """bench.py's inertia correction: delta_w = 0, then 1e-4, x100 until the
    reduced matrix factorises (decided here by the oracle's Cholesky)."""
    dw = 0.0
    while True:
        prob, ev, dg, red, _ = gc.oracle_state(inst, it, delta_w=dw)
        if kkt.cholesky_info(red.khat)[0] == 0:
            return prob, ev, dg, red, dw
        dw = 1e-4 if dw == 0.0 else 100.0 * dw


def _check(run, prob, ev, red, st, kappa, label):
    np_ = lambda t: t.cpu().numpy()  # noqa: E731
    for nm, gpu, orc in (("f", run.f, ev.fk), ("g", run.g, ev.g), ("h", run.h, ev.h),
                         ("grad_x", run.gx, ev.gx), ("grad_u", run.gu, ev.gu)):
        err = np.abs(np_(gpu) - orc).max() / max(np.abs(orc).max(), 1e-300)
        assert err <= 1e-12, (label, nm, err)
    kh = np_(run.khat)
    e_k = gc.rel_fro(kh, red.khat)
    assert int(run.info.item()) == 0, label
    L = np.tril(np_(run.chol))
    e_l = gc.rel_fro(L, gc.chol_lower(kh))
    e_lo = gc.rel_fro(L, gc.chol_lower(red.khat))
    print(f"  {label}: khat {e_k:.2e}  chol {e_l:.2e} (own K_hat) {e_lo:.2e} (oracle)", flush=True)
    assert e_k <= 1e-10, label
    assert e_l <= 1e-10, label
    assert e_lo <= max(1e-10, 10.0 * kappa * e_k), label
    gc.check_step({k: np_(v) for k, v in run.out.items()}, st, kappa, label=" " + label)


def test_bench_configuration_iterate_and_graph_match_oracle():
    import paper_2301_04869_amd as R
    inst = gc.instance("c1")
    it = gc.iterate(inst, seed=SEED)
    prob, ev, dg, red, dw = _bench_delta_w(inst, it)
    st = gc.oracle_step(prob, ev, dg, red, dw, it)
    kappa = gc.cond2(red.khat)
    run = gc.GpuRun(inst, it, dw, torch)
    dm = run.p.dims
    print(f"\nbench configuration: N={dm['n_scen']} variant={dm['variant']} tile={dm['col_tile']} "
          f"lds_reduce={dm['lds_reduce']} lds_group={dm['lds_group']} lds_step={dm['lds_step']} "
          f"delta_w={dw:g} kappa={kappa:.2e}", flush=True)
    assert dm["n_scen"] == 128
    run.chol = torch.zeros_like(run.khat)
    args = gc.iter_args(run)
    R.rkkt_iterate(run.p, args)
    code, scen = R.rkkt_status(run.p)
    assert code == 0, (code, scen)
    _check(run, prob, ev, red, st, kappa, "rkkt_iterate")
    R.rkkt_graph_capture(run.p, args)
    for rep in range(3):
        for v in list(run.out.values()) + [run.khat, run.chol, run.f, run.g, run.h, run.gx, run.gu]:
            v.fill_(float("nan"))
        run.info.fill_(-1)
        torch.cuda.synchronize()
        R.rkkt_graph_launch(run.p)
        torch.cuda.synchronize()
        _check(run, prob, ev, red, st, kappa, f"graph replay {rep}")
