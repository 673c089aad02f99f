"""Parity of the HIP path (through the C ABI) with the CPU oracle on seeded
inputs.  Needs an MI355X and the built librkkt.so.

Tolerances: 1e-12 (relative, per array) on evaluation outputs, 1e-10
relative Frobenius on the reduced matrix and on its Cholesky factor (against
the factor of the same matrix; against the oracle's factor the bound widens
to 10 kappa(K_hat) times the reduced-matrix difference when that is larger),
1e-10 relative 2-norm on the concatenated Newton step (p_x, p_u, p_s, p_y,
p_z); the two-norm condition number of the reduced matrix is printed with
every check."""
import numpy as np
import pytest

import gpu_common as gc
from oracle import kkt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (preset, scenarios or None for the preset's, column tile (0: automatic),
# reduction variant (0: automatic, 1: adjoint solves, 2: stacked product))
CASES = [("tiny5", None, 0, 1), ("tiny5", None, 0, 2), ("tiny9", None, 0, 1), ("tiny9", None, 0, 2),
         ("c0", None, 0, 1), ("c0", None, 0, 2), ("c1", 8, 0, 1), ("c1", 8, 0, 2), ("c1", 8, 4, 1),
         ("c1", 8, 7, 2), ("c1", 8, 64, 1), ("c1", 8, 64, 2), ("c1", None, 0, 0), ("c1", None, 0, 1),
         ("mid300", None, 0, 1), ("mid300", None, 0, 2)]


def _ids(c):
    return f"{c[0]}-N{c[1] or 'full'}-w{c[2]}-v{c[3]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_evaluate_condense_factor_step(case):
    name, n_scen, tile, variant = case
    inst = gc.instance(name, n_scen)
    it = gc.iterate(inst, seed=101)
    prob, ev, dg, red, dw = gc.oracle_state(inst, it)
    run = gc.GpuRun(inst, it, dw, torch, col_tile=tile, variant=variant)
    dm = run.p.dims
    print(f"\ncase {name} N={prob.N} tile={dm['col_tile']} variant={dm['variant']} "
          f"lds_reduce={dm['lds_reduce']} lds_group={dm['lds_group']} lds_step={dm['lds_step']} delta_w={dw:g}", flush=True)
    run.evaluate()
    run.condense()
    run.factor()
    run.step()
    code, scen = run.R.rkkt_status(run.p)
    assert code == 0, (code, scen)
    torch.cuda.synchronize()
    # evaluation
    np_ = lambda t: t.cpu().numpy()  # noqa: E731
    for nm, gpu, orc in (("f", run.f, ev.fk), ("g", run.g, ev.g), ("h", run.h, ev.h),
                         ("grad_x", run.gx, ev.gx), ("grad_u", run.gu, ev.gu)):
        a, b = np_(gpu), orc
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        print(f"  {nm}: max rel err {err:.2e}")
        assert err <= 1e-12, nm
    # reduced matrix (exactly symmetric: the lower triangle is mirrored)
    kh = np_(run.khat)
    assert np.array_equal(kh, kh.T)
    e_k = gc.rel_fro(kh, red.khat)
    kappa = gc.cond2(red.khat)
    print(f"  khat: rel err {e_k:.2e}  cond {kappa:.2e}")
    assert e_k <= 1e-10
    # Cholesky: the factor of the GPU's own reduced matrix (isolates the
    # factorisation), and next to the oracle's factor within the bound the
    # conditioning of K_hat allows for the reduced-matrix difference
    assert int(run.info.item()) == 0
    L = np.tril(np_(run.chol))
    e_l = gc.rel_fro(L, gc.chol_lower(kh))
    e_lo = gc.rel_fro(L, gc.chol_lower(red.khat))
    print(f"  chol: rel err {e_l:.2e} (own K_hat), {e_lo:.2e} (oracle)")
    assert e_l <= 1e-10
    assert e_lo <= max(1e-10, 10.0 * kappa * e_k)
    # Newton step
    st = gc.oracle_step(prob, ev, dg, red, dw, it)
    keys = ("px", "pu", "ps", "py", "pz")
    a = np.concatenate([np_(run.out[k]).ravel() for k in keys])
    b = np.concatenate([st[k].ravel() for k in keys])
    e_s = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"  step: rel err {e_s:.2e}")
    assert e_s <= 1e-10


def test_condense_is_deterministic():
    inst = gc.instance("c1", 16)
    it = gc.iterate(inst, seed=7)
    run = gc.GpuRun(inst, it, 1.0, torch)
    run.evaluate()
    run.condense()
    a = run.khat.clone()
    run.condense()
    assert torch.equal(a, run.khat)


def test_not_positive_definite_reports_column():
    inst = gc.instance("c0")
    it = gc.iterate(inst, seed=3)
    prob, ev, dg, red, _ = gc.oracle_state(inst, it, delta_w=-50.0)
    info_orc, _ = kkt.cholesky_info(red.khat)
    assert info_orc > 0
    run = gc.GpuRun(inst, it, -50.0, torch)
    run.evaluate()
    run.condense()
    run.factor()
    torch.cuda.synchronize()
    assert int(run.info.item()) == info_orc


def test_singular_state_jacobian_is_flagged():
    """All voltage magnitudes zero: every G_x pivot is zero."""
    inst = gc.instance("tiny9")
    it = gc.iterate(inst, seed=5)
    nb = inst.net.n_bus
    it["x"][:, nb - 1:] = 0.0
    it["u"][: inst.net.n_gen] = 0.0
    run = gc.GpuRun(inst, it, 1.0, torch)
    run.evaluate()
    run.condense()
    code, scen = run.R.rkkt_status(run.p)
    assert code == run.R.RkktError(-3, "").code and scen >= 0


def test_bad_arguments_raise_before_launch():
    import paper_2301_04869_amd as R
    inst = gc.instance("tiny5")
    it = gc.iterate(inst, seed=1)
    run = gc.GpuRun(inst, it, 1.0, torch)
    with pytest.raises(ValueError):
        R.rkkt_evaluate(run.p, run.inp["x"][:1], run.inp["u"], run.inp["y"], run.inp["z"],
                        0.1, run.f, run.gx, run.gu, run.g, run.h)
    with pytest.raises(R.RkktError):
        R.rkkt_condense(run.p, run.inp["sigma_x"], run.inp["sigma_u"], run.inp["sigma_s"],
                        float("nan"), run.khat)


def _iter_args(run):
    i, o = run.inp, run.out
    return dict(x=i["x"], u=i["u"], y=i["y"], z=i["z"], obj_weight=run.w, f=run.f, grad_x=run.gx,
                grad_u=run.gu, g=run.g, h=run.h, sigma_x=i["sigma_x"], sigma_u=i["sigma_u"],
                sigma_s=i["sigma_s"], delta_w=run.delta_w, khat=run.khat, chol=run.chol,
                info=run.info, r1x=i["r1x"], r1u=i["r1u"], r2=i["r2"], r3=i["r3"], r4=i["r4"],
                px=o["px"], pu=o["pu"], ps=o["ps"], py=o["py"], pz=o["pz"])


def test_graph_replays_match_eager():
    """The captured pass, replayed several times with eager work and host
    synchronisation between replays, reproduces the eager pass bit for bit."""
    import paper_2301_04869_amd as R
    inst = gc.instance("c1", 16)
    it = gc.iterate(inst, seed=21)
    _, _, _, _, dw = gc.oracle_state(inst, it)
    run = gc.GpuRun(inst, it, dw, torch)
    run.chol = torch.zeros_like(run.khat)
    args = _iter_args(run)
    R.rkkt_iterate(run.p, args)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in run.out.items()}
    ref["khat"] = run.khat.clone()
    R.rkkt_graph_capture(run.p, args)
    for rep in range(4):
        for v in list(run.out.values()) + [run.khat, run.chol]:
            v.fill_(float("nan"))
        run.evaluate()             # eager work between replays
        torch.cuda.synchronize()
        R.rkkt_graph_launch(run.p)
        torch.cuda.synchronize()
        for k, v in run.out.items():
            assert torch.equal(v, ref[k]), (rep, k)
        assert torch.equal(run.khat, ref["khat"]), rep
        assert int(run.info.item()) == 0
