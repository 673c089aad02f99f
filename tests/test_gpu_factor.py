"""The dense factorisation (rkkt_factor) on seeded synthetic matrices of the
orders n_u = 2 n_gen - 1 that grids with 2 .. 64 generators give: one tile
(3, 15), a ragged last tile of one row (17, 33, 65, 113), full or nearly full
tiles (63, 127), the single-workgroup path's limit (127 <= 128).

Checks, against the oracle's right-looking Cholesky (oracle.kkt.cholesky_info):
  - the lower triangle within 1e-13 relative Frobenius on well-conditioned
    matrices, and the backward error ||A - L L^T||_F <= 1e-14 n ||A||_F on
    one with condition number 1e10;
  - the strict upper triangle of each 16 x 16 diagonal block holds the
    transpose of that block's inverse, (L_bb^-1)[p][r] at [r][p], within
    1e-12 relative to the largest entry of the inverse;
  - the rest of the strict upper triangle is left exactly as it was;
  - a matrix whose first non-positive pivot is column j (a negative entry
    of D in A = L D L^T, or a NaN on the diagonal) reports j + 1 in info,
    the same column as the oracle."""
import numpy as np
import pytest

import synthgrid as sg
from oracle import kkt

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GENS = [2, 8, 9, 17, 32, 33, 57, 64]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_handles = {}


def _handle(n_gen):
    """An N = 1 problem whose reduced matrix has order 2 n_gen - 1."""
    import paper_2301_04869_amd as R
    if n_gen not in _handles:
        nb = max(3 * n_gen, 20)
        inst = sg.make_instance(nb, int(nb * 1.4), n_gen, 1, 500 + n_gen)
        _handles[n_gen] = R.rkkt_create(inst.net, inst.scen.pd.T, inst.scen.qd.T)
    return _handles[n_gen]


def _factor(n_gen, a):
    import paper_2301_04869_amd as R
    p = _handle(n_gen)
    n = p.dims["n_u"]
    assert a.shape == (n, n)
    print(f"\nfactor n_gen={n_gen} n={n}", flush=True)
    t = torch.tensor(a, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    R.rkkt_factor(p, t, info)
    torch.cuda.synchronize()
    return t.cpu().numpy(), int(info.item())


def _spd(n, seed, cond=None):
    rng = np.random.default_rng(seed)
    if cond is None:
        b = rng.standard_normal((n, n))
        return b @ b.T / n + np.eye(n)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.logspace(0.0, -np.log10(cond), n)
    return (q * ev) @ q.T


def _with_upper_marker(a):
    """The lower triangle of a, a recognisable pattern in the strict upper."""
    n = a.shape[0]
    out = np.tril(a)
    iu = np.triu_indices(n, 1)
    out[iu] = 1000.0 + np.arange(len(iu[0]))
    return out


def _check_blocks(out, L):
    n = L.shape[0]
    for b0 in range(0, n, 16):
        b1 = min(n, b0 + 16)
        inv = np.linalg.inv(L[b0:b1, b0:b1])
        got = np.triu(out[b0:b1, b0:b1], 1)
        want = np.triu(inv.T, 1)
        err = np.abs(got - want).max() / np.abs(inv).max()
        assert err <= 1e-12, (b0, err)


@pytest.mark.parametrize("n_gen", GENS)
def test_factor_matches_oracle(n_gen):
    n = 2 * n_gen - 1
    a = _spd(n, 10 + n_gen)
    inp = _with_upper_marker(a)
    out, info = _factor(n_gen, inp)
    assert info == 0
    info_o, L_o = kkt.cholesky_info(a)
    assert info_o == 0
    L = np.tril(out)
    err = np.linalg.norm(L - L_o) / np.linalg.norm(L_o)
    print(f"  rel err {err:.2e}")
    assert err <= 1e-13
    _check_blocks(out, L)
    # strict upper triangle outside the diagonal blocks untouched
    blk = np.arange(n) // 16
    outside = np.triu(np.ones((n, n), dtype=bool), 1) & (blk[:, None] != blk[None, :])
    assert np.array_equal(out[outside], inp[outside])


@pytest.mark.parametrize("n_gen", [17, 57, 64])
def test_factor_ill_conditioned_backward_error(n_gen):
    n = 2 * n_gen - 1
    a = _spd(n, 20 + n_gen, cond=1e10)
    out, info = _factor(n_gen, a)
    assert info == 0
    L = np.tril(out)
    berr = np.linalg.norm(a - L @ L.T) / np.linalg.norm(a)
    print(f"  backward err {berr:.2e}")
    assert berr <= 1e-14 * n


def _indefinite(n, j, seed):
    """A = L D L^T with unit lower L (entries of size 0.1) and D = 1 but
    D[j] = -1: the first non-positive pivot is column j."""
    rng = np.random.default_rng(seed)
    Lu = np.tril(0.1 * rng.standard_normal((n, n)), -1) + np.eye(n)
    d = np.ones(n)
    d[j] = -1.0
    return (Lu * d) @ Lu.T


@pytest.mark.parametrize("n_gen,j", [(2, 0), (2, 2), (9, 5), (9, 16), (33, 15), (33, 16), (33, 47),
                                     (64, 0), (64, 63), (64, 100), (64, 126)])
def test_factor_reports_first_bad_pivot(n_gen, j):
    n = 2 * n_gen - 1
    a = _indefinite(n, j, 30 + j)
    info_o, _ = kkt.cholesky_info(a)
    assert info_o == j + 1
    _, info = _factor(n_gen, a)
    assert info == j + 1


@pytest.mark.parametrize("n_gen,j", [(9, 3), (64, 70)])
def test_factor_nan_pivot(n_gen, j):
    n = 2 * n_gen - 1
    a = _spd(n, 40 + j)
    a[j, j] = np.nan
    _, info = _factor(n_gen, a)
    assert info == j + 1


def test_factor_twice_in_a_row():
    """Consecutive calls on one handle: the second result does not depend on
    the first."""
    n_gen = 57
    n = 2 * n_gen - 1
    a, b = _spd(n, 50), _spd(n, 51)
    _factor(n_gen, a)
    out, info = _factor(n_gen, b)
    assert info == 0
    _, L_o = kkt.cholesky_info(b)
    assert np.linalg.norm(np.tril(out) - L_o) / np.linalg.norm(L_o) <= 1e-13
