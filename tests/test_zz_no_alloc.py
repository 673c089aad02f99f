"""rkkt_mlp_forward_static, the forward pass of the warm-start perceptron in
the library's static device workspace (for callers that cannot allocate),
against rkkt_mlp_forward through the C ABI: equal outputs on two calls in a
row, the second with a smaller batch, and a clear error beyond the
workspace's row limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [198, 512, 512, 512, 896]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_static_forward_equals_the_handle_forward():
    import paper_2301_04869_amd as R
    from paper_2301_04869_amd import warmstart as ws
    m = R.Mlp(SIZES, 512)
    m.set_params(torch.tensor(ws.init_params(SIZES, 4), device="cuda"))
    rng = np.random.default_rng(9)
    for rows in (300, 37):
        x = torch.tensor(rng.standard_normal((rows, SIZES[0])).astype(np.float32), device="cuda")
        ref = torch.full((rows, SIZES[-1]), float("nan"), dtype=torch.float32, device="cuda")
        got = torch.full_like(ref, float("nan"))
        m.forward(x, ref)
        m.forward_static(x, got)
        torch.cuda.synchronize()
        print(f"\n  {rows} rows: max |static - handle| = {float((got - ref).abs().max()):.3e}")
        assert torch.isfinite(ref).all()
        assert torch.equal(got, ref), rows
    # beyond the workspace: 2416 rows fit for these sizes, 2417 do not
    big = torch.zeros(2417, SIZES[0], dtype=torch.float32, device="cuda")
    out = torch.zeros(2417, SIZES[-1], dtype=torch.float32, device="cuda")
    with pytest.raises(R.RkktError, match="static workspace"):
        m.forward_static(big, out)
    ok = torch.zeros(2416, SIZES[-1], dtype=torch.float32, device="cuda")
    m.forward_static(big[:2416].contiguous(), ok)
    torch.cuda.synchronize()
    assert torch.isfinite(ok).all()
