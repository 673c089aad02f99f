"""Parity at the full size of the 9241-bus workload (N = 16), in the launch
configuration the benchmark times (rkkt_iterate and its captured graph, whose
replays must equal the eager calls bit for bit), against the whole oracle:
its reduced matrix over all 2889 columns (about two minutes of CPU) and its
Newton step.

  * evaluation outputs element by element (1e-12);
  * the reduced matrix: relative Frobenius 1e-10, and column by column on 64
    sampled columns (both column tiles' ends, the ragged last one included);
  * the Cholesky factor against the factor of the GPU's own reduced matrix
    (isolates the dense factorisation, 1e-10) and against the oracle's;
  * every Newton-step block separately within gpu_common.step_bar
    (1e-10, or 10 eps kappa_2(K_hat));
  * the error of p_u split between its sources: the reduced matrix (the
    oracle's right-hand side solved with the GPU's K_hat on the CPU) and the
    right-hand side, factorisation and triangular solves of the GPU."""
import numpy as np
import pytest
import scipy.linalg as sla

import gpu_common as gc
from oracle import kkt

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.timeout(1200)
def test_c4_full_size():
    import paper_2301_04869_amd as R
    inst = gc.instance("c4")
    it = gc.iterate(inst, seed=404)
    it["y"] *= 0.01
    it["z"] *= 0.01
    dw = 1.0
    run = gc.GpuRun(inst, it, dw, torch)
    dm = run.p.dims
    print(f"\ncase c4 N={dm['n_scen']} n_x={dm['n_x']} n_u={dm['n_u']} variant={dm['variant']} "
          f"tile={dm['col_tile']} lds_reduce={dm['lds_reduce']}", flush=True)
    np_ = lambda t: t.cpu().numpy()  # noqa: E731
    # eager calls
    run.evaluate()
    run.condense()
    run.factor()
    run.step()
    code, scen = R.rkkt_status(run.p)
    assert code == 0, (code, scen)
    assert int(run.info.item()) == 0
    eager = {k: np_(v) for k, v in run.out.items()}
    eager["khat"] = np_(run.khat)
    chol_eager = np.tril(np_(run.chol))
    # the timed path: rkkt_iterate captured and replayed
    run.chol = torch.zeros_like(run.khat)
    args = gc.iter_args(run)
    R.rkkt_graph_capture(run.p, args)
    for v in list(run.out.values()) + [run.khat]:
        v.fill_(float("nan"))
    torch.cuda.synchronize()
    R.rkkt_graph_launch(run.p)
    torch.cuda.synchronize()
    assert int(run.info.item()) == 0
    fails = [k for k, v in run.out.items() if not np.array_equal(np_(v), eager[k])]
    kh = np_(run.khat)
    L = np.tril(np_(run.chol))
    if not np.array_equal(kh, eager["khat"]):
        fails.append("khat")
    if not np.array_equal(L, chol_eager):
        fails.append("chol")
    print(f"  graph replay against the eager calls: differing outputs {fails}", flush=True)

    prob, ev, dg, _, _ = gc.oracle_state(inst, it, delta_w=dw, reduced=False)
    for nm, gpu, orc in (("f", run.f, ev.fk), ("g", run.g, ev.g), ("h", run.h, ev.h),
                         ("grad_x", run.gx, ev.gx), ("grad_u", run.gu, ev.gu)):
        err = np.abs(np_(gpu) - orc).max() / max(np.abs(orc).max(), 1e-300)
        print(f"  {nm}: max rel err {err:.2e}")
        assert err <= 1e-12, nm
    red = kkt.reduced_hessian(prob, ev, dg, dw)
    nu = prob.n_u
    kappa = gc.cond2(red.khat)
    e_k = gc.rel_fro(kh, red.khat)
    tile = dm["col_tile"]
    rng = np.random.default_rng(5)
    edges = sorted({0, 1, tile - 1, tile, nu - 2, nu - 1, (nu - 1) // tile * tile})
    cols = sorted(set(edges) | set(rng.choice(nu, 64 - len(edges), replace=False).tolist()))
    ce = (np.linalg.norm(kh[:, cols] - red.khat[:, cols], axis=0)
          / np.linalg.norm(red.khat[:, cols], axis=0))
    print(f"  khat: rel err {e_k:.2e} (all columns), {ce.max():.2e} worst of {len(cols)} sampled "
          f"columns; kappa_2(K_hat) {kappa:.2e}", flush=True)
    assert e_k <= 1e-10
    assert ce.max() <= 1e-10
    # dense factorisation
    Lc = gc.chol_lower(kh)
    e_l = gc.rel_fro(L, Lc)
    e_lo = gc.rel_fro(L, gc.chol_lower(red.khat))
    print(f"  chol: rel err {e_l:.2e} (own K_hat), {e_lo:.2e} (oracle)", flush=True)
    assert e_l <= 1e-10
    assert e_lo <= max(1e-10, 10.0 * kappa * e_k)
    # Newton step
    rs = kkt.Resid(it["r1x"], it["r1u"], it["r2"], it["r3"], it["r4"])
    _, _, rhs = kkt.reduced_rhs(prob, ev, dg, rs, red)
    st = kkt.newton_reduced(prob, ev, dg, rs, dw, red)
    gpu = {k: np_(v) for k, v in run.out.items()}
    pu_k = sla.cho_solve((Lc, True), rhs)       # oracle rhs, GPU K_hat
    e_from_k = np.linalg.norm(pu_k - st["pu"]) / np.linalg.norm(st["pu"])
    e_rest = np.linalg.norm(gpu["pu"] - pu_k) / np.linalg.norm(st["pu"])
    print(f"  p_u error split: from K_hat {e_from_k:.2e}, from the GPU's right-hand side, factor "
          f"and solves {e_rest:.2e}", flush=True)
    r, s, per = kkt.augmented_residual(prob, ev, dg, rs, dw, gpu, blocks=True)
    ro, so, per_o = kkt.augmented_residual(prob, ev, dg, rs, dw, st, blocks=True)
    print(f"  augmented residual relative: GPU {r / s:.2e}, oracle {ro / so:.2e}")
    for k in per:
        print(f"    block {k}: GPU {per[k][0] / per[k][1]:.2e}  oracle {per_o[k][0] / per_o[k][1]:.2e}")
    gc.check_step(gpu, st, kappa)
    assert not fails, fails
