"""GPU: the STREAM-triad probe computes a = b + s c exactly (one fma per
element), with and without non-temporal hints, on lengths that leave a
ragged last pass."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


@pytest.mark.parametrize("n", [2, 1030, 4 * 256 * 7 + 18, 3 << 20])
@pytest.mark.parametrize("nt", [False, True])
def test_triad_exact(H, n, nt):
    g = torch.Generator(device="cpu").manual_seed(n)
    b = torch.randn(n, dtype=torch.float64, generator=g)
    # c with 41 significant bits: s c is exact, so b + s c rounds once with
    # or without a fused multiply-add
    c = torch.randint(-(1 << 40), 1 << 40, (n,), generator=g).to(torch.float64) * 2.0 ** -20
    a = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    H.hmc_stream_triad(a, b.cuda(), c.cuda(), -1.75, nt)
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), b + (-1.75) * c)
