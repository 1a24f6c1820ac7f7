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


def test_autotune_site_orders_then_parity(H, tmp_path):
    """A lattice that admits the tiled order and y-blocks (32 x 16 / 2 = 256
    sites per z-plane = 4 chunks: whole planes or y-blocks of 2): the tuner
    times the orders x workgroups per CU for the one-site shape, stores its
    choice for every storage, and the Dslash and a solve reproduce the oracle
    under it."""
    L = (32, 16, 4, 8)
    k = 0.15
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = synth.gauge_field(71, L, eps=0.5)
    put_gauge(H, F, U)
    db = tmp_path / "tune.txt"
    H.hmc_autotune(F, str(db))
    kinds = {ln.split()[0] for ln in db.read_text().splitlines() if ln and not ln.startswith("#")}
    assert {"dslash_order", "dslash_occupancy"} <= kinds
    for prec in (0, 1, 2, 3):
        order, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_ORDER, prec)
        assert tuned and order in (0, 1, 2), (prec, order)
        occ, tuned = H.hmc_tune_query(L, H.TUNE_DSLASH_OCC, prec)
        assert tuned and occ in (0, 2), (prec, occ)
    psi = synth.spinor(72, L)
    for par, dag in ((0, 0), (1, 1)):
        want = O.dslash(L, U, psi, par, dag)
        for prec, tol in ((0, 1e-14), (1, 1e-6), (2, 3e-3), (3, 2e-2)):
            b = put_spinor(H, F, psi, 1 - par, prec=prec)
            out = F.spinor(prec=prec)
            H.hmc_wilson_dslash(F, out, b, par, dag, prec)
            assert rel(get_spinor(H, F, out, par, prec=prec), want) < tol, (prec, par, dag)
    odd = O.parity_mask(L)
    b = synth.spinor(73, L, odd, 0)
    want, _ = O.cg_mhat(L, U, k, b, tol=1e-12)
    bb = put_spinor(H, F, b, 0)
    for prec in (0, 1, 2):
        x = F.spinor()
        st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, prec=prec, maxiter=20000))
        assert st["status"] == 0 and st["true_rel_res"] <= 1e-10, prec
        assert rel(get_spinor(H, F, x, 0), want) < 1e-8, prec
