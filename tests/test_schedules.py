"""The level-sliced schedules and the chain that the kernels follow, exported
by the host analysis and replayed here in Python with random values on the
filled pattern: the four unit triangular sweeps must reproduce dense
triangular solves, and the refactorisation items plus the chain elimination
must reproduce a dense LU without pivoting.  Within a phase every source is
read from the state before the phase, so a schedule that let a row be a
source and a destination in one phase would fail here.  Host logic only."""
import numpy as np
import pytest
import scipy.linalg as sla

import synthgrid as sg
import paper_2301_04869_amd as R

CASES = [("tiny5", None), ("tiny9", None), ("c0", None), ("c1", 4), ("mid300", 2)]


def _pattern(net, n):
    perm, fp, fc = R.rkkt_analyze_lu(net, n)
    nx = len(fp) - 1
    rows = np.repeat(np.arange(nx), np.diff(fp))
    return nx, fp, fc, rows


def _sweep(sc, vals, b, nx, up, trans):
    x = b.copy()
    S, ptr, ent, t = sc["slots"], sc["ptr"], sc["ent"], sc["chain_rows"]
    c0, P = nx - t, sc["chain_pos"]

    def phases():
        for q in range(sc["nphase"]):
            snap = x.copy()
            for e in range(ptr[q * S], ptr[(q + 1) * S]):
                dest, src, pos, tpos = ent[e]
                x[dest] -= vals[tpos if trans else pos] * snap[src]

    def chain():  # column order, as the kernels take it
        order = range(t) if up else range(t - 1, -1, -1)
        for bb in order:
            rows_a = range(bb + 1, t) if up else range(bb)
            for a in rows_a:
                pp = P[bb, a] if trans else P[a, bb]
                if pp >= 0:
                    x[c0 + a] -= vals[pp] * x[c0 + bb]

    if up:
        phases()
        chain()
    else:
        chain()
        phases()
    return x


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-N{c[1]}")
def test_sweeps_reproduce_dense_triangular_solves(case):
    name, n = case
    inst = sg.preset(name)
    n = n or inst.scen.n_scen
    nx, fp, fc, rows = _pattern(inst.net, n)
    rng = np.random.default_rng(3)
    vals = rng.uniform(-0.5, 0.5, len(fc))
    Lm = np.zeros((nx, nx))
    Um = np.zeros((nx, nx))
    for e, (i, j) in enumerate(zip(rows, fc)):
        if j < i:
            Lm[i, j] = vals[e]
        elif j > i:
            Um[i, j] = vals[e]
    eye = np.eye(nx)
    b = rng.standard_normal(nx)
    for which, up, form in (("reduce_up", True, 0), ("reduce_down", False, 0), ("reduce_up", True, 2),
                            ("reduce_down", False, 2), ("step_up", True, 0), ("step_down", False, 0)):
        sc = R.rkkt_analyze_schedule(inst.net, n, which, sweep_form=form)
        for trans in (False, True):
            got = _sweep(sc, vals, b, nx, up, trans)
            if up:
                M = eye + (Um.T if trans else Lm)
                ref = sla.solve_triangular(M, b, lower=True, unit_diagonal=True)
            else:
                M = eye + (Lm.T if trans else Um)
                ref = sla.solve_triangular(M, b, lower=False, unit_diagonal=True)
            err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err < 1e-12, (which, trans, err)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-N{c[1]}")
def test_refactor_schedule_reproduces_dense_lu(case):
    name, n = case
    inst = sg.preset(name)
    n = n or inst.scen.n_scen
    nx, fp, fc, rows = _pattern(inst.net, n)
    rng = np.random.default_rng(5)
    A = np.zeros((nx, nx))
    A[rows, fc] = rng.uniform(-1.0, 1.0, len(fc))
    A[np.arange(nx), np.arange(nx)] = nx + rng.uniform(1.0, 2.0, nx)   # no pivoting needed
    lu = A[rows, fc].copy()
    sc = R.rkkt_analyze_schedule(inst.net, n, "refactor")
    S, ptr, ent, upd, t = sc["slots"], sc["ptr"], sc["ent"], sc["upd"], sc["chain_rows"]
    for q in range(sc["nphase"]):
        for e in range(ptr[q * S], ptr[(q + 1) * S]):
            pos, diag, ulen, ub = ent[e]
            l = lu[pos] / lu[diag]
            lu[pos] = l
            for j in range(ulen):
                lu[upd[ub + j]] -= l * lu[diag + 1 + j]
    c0, P = nx - t, sc["chain_pos"]
    for j in range(t):
        for a in range(j + 1, t):
            if P[a, j] < 0:
                continue
            l = lu[P[a, j]] / lu[P[j, j]]
            lu[P[a, j]] = l
            for bb in range(j + 1, t):
                if P[j, bb] >= 0:
                    lu[P[a, bb]] -= l * lu[P[j, bb]]
    # dense Doolittle LU without pivoting
    U = A.copy()
    Lf = np.eye(nx)
    for k in range(nx - 1):
        Lf[k + 1:, k] = U[k + 1:, k] / U[k, k]
        U[k + 1:, k:] -= np.outer(Lf[k + 1:, k], U[k, k:])
    ref = np.where(fc < rows, Lf[rows, fc], U[rows, fc])
    err = np.abs(lu - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err
    # the filled pattern holds every nonzero of the factors
    mask = np.zeros((nx, nx), bool)
    mask[rows, fc] = True
    assert np.abs(np.tril(Lf, -1)[~mask]).max(initial=0.0) == 0.0
    assert np.abs(np.triu(U, 1)[~mask]).max(initial=0.0) < 1e-300


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("which,form", [("reduce_up", 0), ("reduce_down", 0), ("reduce_up", 2),
                                        ("reduce_down", 2), ("step_up", 0), ("step_down", 0)])
def test_sweep_phases_group_destinations(case, which, form):
    """What the sweeps that read a phase's values ahead rely on: within a
    phase no row is both a destination and a source, every destination
    belongs to one slot, and a slot's entries for one destination are
    contiguous (push and pull forms of the reduction's schedules)."""
    name, n = case
    inst = sg.preset(name)
    n = n or inst.scen.n_scen
    sc = R.rkkt_analyze_schedule(inst.net, n, which, sweep_form=form)
    P, S, ptr, ent = sc["nphase"], sc["slots"], sc["ptr"], sc["ent"]
    for q in range(P):
        dsts, srcs, owner = set(), set(), {}
        for sl in range(S):
            runs = []
            for e in range(ptr[q * S + sl], ptr[q * S + sl + 1]):
                d, s = int(ent[e][0]), int(ent[e][1])
                dsts.add(d)
                srcs.add(s)
                assert owner.setdefault(d, sl) == sl, (q, d)
                if not runs or runs[-1] != d:
                    assert d not in runs, (q, sl, d)
                    runs.append(d)
        assert not (dsts & srcs), q


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("which", ["reduce_up", "reduce_down"])
def test_pull_form_writes_each_row_in_few_pieces(case, which):
    """The pull form writes a row once per piece of at most 16 terms (a row's
    pieces lie in distinct phases, each in one slot), far fewer row writes
    than the push form, and it holds the same pairs as the push form."""
    name, n = case
    inst = sg.preset(name)
    n = n or inst.scen.n_scen
    pull = R.rkkt_analyze_schedule(inst.net, n, which, sweep_form=2)
    push = R.rkkt_analyze_schedule(inst.net, n, which, sweep_form=1)

    def pieces(sc):
        P, S, ptr, ent = sc["nphase"], sc["slots"], sc["ptr"], sc["ent"]
        out = {}
        for q in range(P):
            for sl in range(S):
                for e in range(ptr[q * S + sl], ptr[q * S + sl + 1]):
                    out.setdefault((int(ent[e][0]), q), set()).add(sl)
        return out
    pp, pu = pieces(pull), pieces(push)
    assert all(len(v) == 1 for v in pp.values())
    terms = {}
    for d in pull["ent"][:, 0]:
        terms[int(d)] = terms.get(int(d), 0) + 1
    per_row = {}
    for (d, q) in pp:
        per_row[d] = per_row.get(d, 0) + 1
    assert all(per_row[d] <= -(-terms[d] // 16) for d in terms)
    assert len(pp) <= len(pu)
    key = lambda a: sorted(map(tuple, a.tolist()))  # noqa: E731
    assert key(pull["ent"]) == key(push["ent"])
