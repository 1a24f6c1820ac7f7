"""GPU: launch auto-tuning picks shapes that still reproduce the oracle."""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_gpu_parity import get_spinor, put_gauge, put_spinor, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def test_autotune_then_parity(H, tmp_path):
    L = (8, 6, 6, 10)
    k = 0.157
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = O.weak_field(L, 1, 0.5)
    put_gauge(H, F, U)
    db = tmp_path / "tune.txt"
    H.hmc_autotune(F, str(db))
    lines = [ln.split() for ln in db.read_text().splitlines() if ln and not ln.startswith("#")]
    assert len(lines) >= 5
    for prec in (0, 1, 2, 3):
        ch, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH, prec)
        assert tuned and ch in (1, 2, 4)
    assert H.hmc_tune_query(L, H.TUNE_GAUGE_FORCE)[1]
    psi = synth.spinor(12, L)
    want = O.dslash(L, U, psi, 0, 0)
    for prec, tol in ((0, 1e-14), (1, 1e-6), (2, 3e-3), (3, 2e-2)):
        b = put_spinor(H, F, psi, 1, prec=prec)
        out = F.spinor(prec=prec)
        H.hmc_wilson_dslash(F, out, b, 0, 0, prec)
        assert rel(get_spinor(H, F, out, 0, prec=prec), want) < tol, prec
    # solves under the tuned shapes (partial counts follow the shape)
    b = O.source(L, 0, 3, 0)
    bb = put_spinor(H, F, b, -1)
    xw, _ = O.wilson_solve(L, U, k, b, tol=1e-10)
    for prec in (0, 1, 2):
        x = F.spinor(full=True)
        st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, mode=H.CG_WILSON_SOLVE, prec=prec, maxiter=20000))
        assert st["status"] == 0 and st["true_rel_res"] <= 1e-10
        assert rel(get_spinor(H, F, x, -1), xw) < 1e-7
    # the staple force under the tuned shape
    P = synth.hermitian_traceless(5, L)
    from tests.test_gpu_parity import get_momenta, put_momenta
    put_momenta(H, F, P)
    H.hmc_gauge_force(F, 0.3)
    assert rel(get_momenta(H, F), P - 0.3 * O.gauge_force(L, U, 5.6)) < 1e-13
