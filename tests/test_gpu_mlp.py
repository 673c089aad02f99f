"""The warm-start perceptron on the GPU (rkkt_mlp.h) against the FP64 oracle
MLP: loss and gradients at the full size 198 -> 512 -> 512 -> 512 -> 896 to a
BF16-level tolerance, the Adam step exactly (FP32), and a short training run
that lowers the loss."""
import numpy as np
import pytest

from oracle import mlp as om

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [198, 512, 512, 512, 896]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flat(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)])


def _unflat(p, sizes):
    import paper_2301_04869_amd as R
    Ws, bs = [], []
    for (wo, bo), (fi, fo) in zip(R.mlp_layout(sizes), zip(sizes[:-1], sizes[1:])):
        Ws.append(p[wo:wo + fi * fo].reshape(fi, fo))
        bs.append(p[bo:bo + fo])
    return Ws, bs


def _setup(batch, seed):
    import paper_2301_04869_amd as R
    Ws, bs = om.init_params(SIZES, seed)
    rng = np.random.default_rng(seed + 1)
    bs = [rng.normal(0.0, 0.1, b.shape) for b in bs]           # nonzero biases exercise db
    p32 = _flat(Ws, bs).astype(np.float32)
    X = rng.normal(size=(batch, SIZES[0])).astype(np.float32)
    T = rng.normal(size=(batch, SIZES[-1])).astype(np.float32)
    m = R.Mlp(SIZES, batch)
    dev = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    m.set_params(dev(p32))
    return m, p32, X, T, dev


def test_gradients_match_the_oracle_to_bf16_accuracy():
    batch = 64
    m, p32, X, T, dev = _setup(batch, 3)
    g = torch.zeros(m.n_params, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.gradients(dev(X), dev(T), g, loss)
    torch.cuda.synchronize()
    Ws, bs = _unflat(p32.astype(np.float64), SIZES)
    lo, gW, gb = om.loss_and_grads(Ws, bs, X.astype(np.float64), T.astype(np.float64))
    e_loss = abs(float(loss.item()) - lo) / lo
    print(f"\n  loss gpu {float(loss.item()):.6f} oracle {lo:.6f} rel err {e_loss:.2e}")
    assert e_loss <= 1e-2
    gw_gpu, gb_gpu = _unflat(g.cpu().numpy().astype(np.float64), SIZES)
    for l in range(len(Ws)):
        for nm, a, b in (("W", gw_gpu[l], gW[l]), ("b", gb_gpu[l], gb[l])):
            e = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = float(np.sum(a * b) / (np.linalg.norm(a) * np.linalg.norm(b)))
            print(f"  layer {l} d{nm}: rel err {e:.2e}, cosine {cos:.6f}")
            # BF16 operands (unit roundoff 2^-8 = 3.9e-3), FP32 accumulation:
            # a few roundoffs relative, about 5 allowed
            assert e <= 2e-2 and cos >= 0.9995, (l, nm)


def test_adam_step_is_exact():
    batch = 32
    m, p32, X, T, dev = _setup(batch, 5)
    g = torch.zeros(m.n_params, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.gradients(dev(X), dev(T), g, loss)
    lr = 1e-3
    m.train_step(dev(X), dev(T), lr, loss)
    p1 = torch.zeros(m.n_params, dtype=torch.float32, device="cuda")
    m.get_params(p1)
    torch.cuda.synchronize()
    g64 = g.cpu().numpy().astype(np.float64)
    ref, _, _ = om.adam_step(p32.astype(np.float64), g64, np.zeros_like(g64), np.zeros_like(g64), 1, lr=lr)
    got = p1.cpu().numpy().astype(np.float64)
    e = np.abs(got - ref).max() / np.abs(ref - p32).max()
    print(f"\n  Adam step: max abs diff {np.abs(got - ref).max():.2e} (step size {np.abs(ref - p32).max():.2e})")
    assert e <= 1e-3


def test_training_lowers_the_loss():
    batch = 256
    m, p32, X, T, dev = _setup(batch, 7)
    rng = np.random.default_rng(11)
    A = rng.normal(size=(SIZES[0], SIZES[-1])).astype(np.float32) / np.sqrt(SIZES[0])
    Xd = dev(X)
    Td = dev((X @ A).astype(np.float32))   # a linear teacher
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(200):
        m.train_step(Xd, Td, 1e-3, loss)
        if step % 50 == 0 or step == 199:
            hist.append(float(loss.item()))
    print(f"\n  loss over 200 Adam steps: {hist}")
    assert hist[-1] < 0.2 * hist[0]


def test_bad_batch_raises():
    import paper_2301_04869_amd as R
    m = R.Mlp([4, 8, 3], 16)
    x = torch.zeros(17, 4, dtype=torch.float32, device="cuda")
    y = torch.zeros(17, 3, dtype=torch.float32, device="cuda")
    with pytest.raises(R.RkktError):
        m.forward(x, y)
