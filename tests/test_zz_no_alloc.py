"""mlp_forward_noalloc (the entry point for callers that cannot allocate)
against mlp_forward: the same kernels on the library's static device scratch
instead of a caller's workspace, so the outputs must agree bit for bit, on two
calls in a row (the second smaller), at the row limit, and the limit enforced."""
import pytest
import torch

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]
if gpu_available():
    import paper_1208_0302_amd as g

DEV = "cuda"


def _x(n, seed):
    gen = torch.Generator(device="cpu").manual_seed(seed)
    # network inputs are Stokes samples divided by the continuum: I near 1,
    # Q, U, V small
    x = 0.05 * torch.randn((n, 1024), generator=gen, dtype=torch.float32)
    x[:, :256] += 0.9
    return x.to(DEV)


@pytest.mark.parametrize("precision", [0, 1])
def test_forward_noalloc_matches_forward(precision):
    net = g.MLP(seed=11, device=DEV, precision=precision)
    for n, seed in ((700, 1), (77, 2)):
        x = _x(n, seed)
        ref = net.forward(x)
        got = net.forward_noalloc(x)
        torch.cuda.synchronize()
        print("n %d: max |noalloc - forward| = %.3g" % (n, (got - ref).abs().max().item()))
        assert torch.equal(got, ref)


def test_forward_noalloc_row_limit():
    net = g.MLP(seed=12, device=DEV)
    m = int(g.lib().mlp_noalloc_max_rows())
    assert m >= 256
    x = _x(m, 3)
    assert torch.equal(net.forward_noalloc(x), net.forward(x))
    with pytest.raises(g.GenesisError):
        net.forward_noalloc(_x(m + 1, 4))
    with pytest.raises(g.GenesisError):
        net.forward_noalloc(_x(0, 5))
