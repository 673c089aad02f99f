"""Independent instances of uneven sizes, one launch per kernel configuration
(rkkt_multi_*): eight instances of 113 to 922 buses (one with 8 scenarios,
one with narrow column tiles), which between them take the reduction in LDS
and in device memory, both reduction variants, push and pull schedules,
refactorisation groups of 1, 2 and 4 scenarios and in device memory, the
small and the blocked Cholesky.  The multi-instance pass, eager and as three
replays of its captured graph with eager work between them, must equal every
instance's own rkkt_iterate bit for bit, and match the oracle (reduced
matrix 1e-10, every Newton-step block within gpu_common.step_bar)."""
import numpy as np
import pytest

import gpu_common as gc
import synthgrid as sg
from synthgrid.iterates import random_iterate

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _outputs(run):
    return dict(run.out, khat=run.khat, chol=run.chol, f=run.f, g=run.g, h=run.h, gx=run.gx, gu=run.gu,
                info=run.info)


def _instances():
    """(instance, scenarios, column tile) of the test: six single-scenario
    grids of 113 to 922 buses, the 118-bus grid with 8 scenarios, and a small
    grid with 16-column tiles."""
    out = [(inst, 1, 0) for inst in sg.batch_instances(6, seed=81, lo=60, hi=1200)]
    out.append((sg.preset("c1", n_scen=8), 8, 0))
    out.append((sg.batch_instances(1, seed=82, lo=80, hi=150)[0], 1, 16))
    return out


def test_multi_pass_equals_each_instance_and_the_oracle():
    import paper_2301_04869_amd as R
    runs, refs, orcs = [], [], []
    for j, (inst, n_scen, tile) in enumerate(_instances()):
        it = random_iterate(inst.net, n_scen, 900 + j)
        prob, ev, dg, red, dw = gc.oracle_state(inst, it)
        st = gc.oracle_step(prob, ev, dg, red, dw, it)
        run = gc.GpuRun(inst, it, dw, torch, col_tile=tile)
        run.chol = torch.zeros_like(run.khat)
        R.rkkt_iterate(run.p, gc.iter_args(run))
        torch.cuda.synchronize()
        code, scen = R.rkkt_status(run.p)
        assert code == 0, (j, code, scen)
        refs.append({k: v.clone() for k, v in _outputs(run).items()})
        orcs.append((red.khat, st, gc.cond2(red.khat)))
        runs.append(run)
        dm = run.p.dims
        print(f"\ninstance {j}: n_bus={inst.net.n_bus} N={dm['n_scen']} n_x={dm['n_x']} n_u={dm['n_u']} "
              f"variant={dm['variant']} tile={dm['col_tile']} lds_reduce={dm['lds_reduce']} "
              f"sweep_form={dm['sweep_form']} lds_group={dm['lds_group']} spw={dm['scen_per_group']} "
              f"lds_step={dm['lds_step']} delta_w={dw:g}", flush=True)
    with pytest.raises(R.RkktError):
        R.Multi([runs[0].p, runs[0].p], [gc.iter_args(runs[0])] * 2)
    m = R.Multi([r.p for r in runs], [gc.iter_args(r) for r in runs])
    print(f"multi-instance pass: {m.n_launches} launches for {len(runs)} instances", flush=True)

    def check(label):
        for j, (r, ref, (kho, sto, kappa)) in enumerate(zip(runs, refs, orcs)):
            for k, v in _outputs(r).items():
                assert torch.equal(v, ref[k]), (label, j, k)
            assert gc.rel_fro(r.khat.cpu().numpy(), kho) <= 1e-10, (label, j)
            gc.check_step({k: v.cpu().numpy() for k, v in r.out.items()}, sto, kappa,
                          label=f" instance {j} {label}")

    def poison():
        # every output NaN (info -7), except the factor's buffer: the Cholesky
        # leaves entries outside the factor as they were, so it starts from
        # zeros, as in the eager reference
        for r in runs:
            for k, v in _outputs(r).items():
                v.fill_(-7 if k == "info" else 0.0 if k == "chol" else float("nan"))

    poison()
    torch.cuda.synchronize()
    m.iterate()
    torch.cuda.synchronize()
    check("eager")
    m.capture()
    for rep in range(3):
        poison()
        runs[0].evaluate()          # eager work between the replays
        torch.cuda.synchronize()
        m.launch()
        torch.cuda.synchronize()
        check(f"replay {rep}")
