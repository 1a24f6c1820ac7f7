"""The allocation-free norm2 (hmc_norm2_static: partial sums in the library's
static device array) against hmc_norm2 through the C ABI: two calls in a
row, the second on a smaller lattice, each bit-identical to hmc_norm2 on the
same input (same kernels, same partial count and summation order)."""
import ctypes as C

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


def source(H, F, prec, full, seed):
    """A Gaussian spinor of storage prec (full: both halves)."""
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, H.SOURCE_GAUSS, seed, 0)
    if prec == H.F64:
        return b if full else b[: H.hmc_field_bytes(F.L, H.F64, H.KIND_HALF_SPINOR)]
    hb64 = H.hmc_field_bytes(F.L, H.F64, H.KIND_HALF_SPINOR)
    low = F.spinor(prec=prec, full=full)
    hbl = H.hmc_field_bytes(F.L, prec, H.KIND_HALF_SPINOR)
    for h in range(2 if full else 1):
        H.hmc_convert_spinor(F, low[h * hbl:(h + 1) * hbl], prec, b[h * hb64:(h + 1) * hb64], H.F64)
    return low


# (lattice, halves, storage): the second call is smaller than the first
CASES = [((16, 16, 16, 32), 2, 0), ((8, 6, 6, 10), 1, 0), ((24, 24, 24, 48), 2, 1), ((4, 4, 4, 4), 1, 2),
         ((8, 8, 8, 8), 2, 3)]


def test_norm2_static_matches_norm2(H):
    out = torch.full((len(CASES),), float("nan"), dtype=torch.float64, device="cuda")
    want = []
    keep = []
    for i, (L, nh, prec) in enumerate(CASES):
        F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
        x = source(H, F, prec, nh == 2, 7 + i)
        want.append(H.hmc_norm2(F, x, nh, prec))
        st = H.lib().hmc_norm2_static(C.byref(H.geom(L)), x.data_ptr(), nh, prec, out[i:].data_ptr(),
                                      torch.cuda.current_stream().cuda_stream)
        assert st == H.HMC_OK, H.last_error()
        keep.append((F, x))
    torch.cuda.synchronize()
    got = out.cpu().tolist()
    for i in range(len(CASES)):
        assert got[i] == want[i] and want[i] > 0, (CASES[i], got[i], want[i])


def test_norm2_static_repeated_calls_and_errors(H):
    L = (8, 6, 6, 10)
    F = H.Fields(L, 5.6, 0.15)
    x = source(H, F, H.F64, True, 3)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    for k in range(2):
        H.hmc_norm2_static(L, x, 2, H.F64, out[k:])
    torch.cuda.synchronize()
    assert out[0].item() == out[1].item() == H.hmc_norm2(F, x, 2, H.F64)
    lib = H.lib()
    g = H.geom(L)
    assert lib.hmc_norm2_static(C.byref(g), x.data_ptr(), 3, 0, out.data_ptr(), None) == H.HMC_E_ARG
    assert lib.hmc_norm2_static(C.byref(g), None, 1, 0, out.data_ptr(), None) == H.HMC_E_ARG
    assert lib.hmc_norm2_static(C.byref(H.geom((5, 4, 4, 4))), x.data_ptr(), 1, 0, out.data_ptr(), None) \
        == H.HMC_E_ARG
