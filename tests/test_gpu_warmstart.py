"""Warm starts of the device interior-point solver: from the cold solve's own
solution it converges again, to the same objective, in a few iterations; a
perceptron trained on a few seeded load draws gives warm starts that converge
to the cold objectives; and on the 118-bus grid the trained perceptron cuts
the mean iterations below the cold start on held-out draws at equal 1e-6
objective accuracy, fallbacks counted (the full-size comparison is
bench.py --config warm)."""
import numpy as np
import pytest

import synthgrid as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_warm_start_from_the_solution_converges_at_once():
    from paper_2301_04869_amd import warmstart as ws
    inst = sg.preset("c0")
    solver = ws.Solver(inst.net, torch)
    solver.set_loads(inst.scen.pd[:, 0], inst.scen.qd[:, 0])
    r0, sol = solver.solve()
    assert r0["status"] == "converged"
    r1, sol1 = solver.solve(warm=solver.split(sol), mu0=1e-8)
    print(f"\n  cold {r0['iters']} iterations, obj {r0['obj']:.10f}; warm from the solution "
          f"{r1['iters']} iterations, obj {r1['obj']:.10f}")
    assert r1["status"] == "converged"
    assert abs(r1["obj"] - r0["obj"]) <= 1e-6 * abs(r0["obj"])
    assert r1["iters"] <= 5 and r1["iters"] < r0["iters"]


def test_learned_warm_starts_reach_the_cold_objectives():
    from paper_2301_04869_amd import warmstart as ws
    inst = sg.preset("c0", n_scen=48, sigma=0.15)
    res = ws.experiment(torch, inst.net, inst.scen.pd, inst.scen.qd, n_train=40, steps=300,
                        log=lambda s: print("  " + s))
    assert res["n_test"] >= 6
    assert res["fallback_rate"] <= 0.5
    assert res["train_loss"][-1] < res["train_loss"][0]


def test_learned_warm_start_cuts_iterations_on_held_out_draws():
    """118-bus grid, sigma 0.15 load draws: 4000 training, 40 validation
    (choice of mu0), 100 held-out draws.  Every held-out warm solve whose
    objective is more than 1e-6 (relative) from the cold one, or that fails,
    counts its iterations plus the cold solve's.  The learned start must take
    fewer mean iterations than the cold start and than the start from the mean
    training solution at the same mu0 (the ablation that separates the
    network's contribution from that of a warm barrier parameter)."""
    from paper_2301_04869_amd import warmstart as ws
    inst = sg.preset("c3", n_scen=4140)
    res = ws.experiment(torch, inst.net, inst.scen.pd, inst.scen.qd, n_train=4000, n_val=40,
                        mu0s=(1e-6, 1e-7, 1e-8), steps=8000, log=lambda s: print("  " + s, flush=True))
    assert res["n_test"] >= 95
    assert res["warm_mean_iters"] < res["cold_mean_iters"]
    assert res["warm_mean_iters"] < res["mean_start_mean_iters"]
    assert res["fallback_rate"] <= 0.05
