"""GPU tests of the trajectory failure paths (the rejection rules of the
HMC accept/reject step, Sec. 1).

* A force solve that stops at maxiter forces a reject: hmc_trajectory
  returns HMC_E_NOCONV, counts every failed solve and restores U bit for
  bit; the next trajectory with a working solver matches the oracle.
* A non-finite link forces a reject with HMC_E_NAN, which takes precedence
  over the non-convergence the same field causes in every solve; U is
  restored bit for bit (the non-finite entry included).
* A non-finite right-hand side stops a solve at once with HMC_E_NAN.

Every failure is forced from the host (a tiny iteration limit, a NaN written
into an input); each kernel still runs to its normal end.
"""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = (4, 4, 4, 4)
SEED, BETA, KAPPA = 12120785, 5.6, 0.15


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def get_gauge(H, F):
    c = H.canon_gauge_zeros(F.L)
    H.hmc_export_gauge(F, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def put_gauge(H, F, U):
    H.hmc_import_gauge(F, H.to_device_c128(np.ascontiguousarray(U)))


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def test_nonconverged_solves_reject_and_restore(H):
    F = H.Fields(L, BETA, KAPPA)
    H.hmc_weak_field_start(F, SEED, 0.3)
    U0 = get_gauge(H, F)
    r = H.hmc_trajectory(F, SEED, 0, 1.0, 10, H.cg_params(tol=1e-10, maxiter=2))
    assert r["status"] == H.HMC_E_NOCONV
    assert r["nonconverged"] == 11 and r["accepted"] == 0
    assert r["cg_iters_max"] == 2
    assert np.isfinite(r["dH"])
    assert np.array_equal(bits(get_gauge(H, F)), bits(U0))
    # the same fields object then runs a normal trajectory that matches the oracle
    r = H.hmc_trajectory(F, SEED, 0, 1.0, 10, H.cg_params(tol=1e-10))
    U1, o = O.hmc_trajectory(L, U0, BETA, KAPPA, SEED, 0, 1.0, 10, tol=1e-10)
    assert r["status"] == H.HMC_OK and r["accepted"] == o["accepted"]
    assert abs(r["dH"] - o["dH"]) < 1e-12 * abs(o["H_old"])
    assert np.linalg.norm(get_gauge(H, F) - U1) < 1e-12 * np.linalg.norm(U1)


def test_leapfrog_reports_nonconvergence(H):
    F = H.Fields(L, BETA, KAPPA)
    H.hmc_weak_field_start(F, SEED, 0.3)
    H.hmc_refresh(F, SEED, 0)
    st = H.hmc_md_leapfrog(F, 1.0, 10, H.cg_params(tol=1e-10, maxiter=2), allow_noconv=True)
    assert st["status"] == H.HMC_E_NOCONV
    assert st["solves"] == 11 and st["nonconverged"] == 11 and st["nonfinite"] == 0


@pytest.mark.parametrize("where", [(0, 0, 0, 0), (37, 2, 1, 2)])
def test_nonfinite_link_rejects_with_nan(H, where):
    F = H.Fields(L, BETA, KAPPA)
    U = O.weak_field(L, SEED, 0.3)
    site, mu, a, b = where
    U[site, mu, a, b] = complex(np.nan, 0.0)
    put_gauge(H, F, U)
    U0 = get_gauge(H, F)
    assert np.isnan(U0[site, mu, a, b])
    r = H.hmc_trajectory(F, SEED, 0, 1.0, 10, H.cg_params(tol=1e-10))
    assert r["status"] == H.HMC_E_NAN  # not HMC_E_NOCONV, although no solve converged
    assert r["accepted"] == 0 and r["nonconverged"] == 11
    assert not np.isfinite(r["dH"])
    assert r["cg_iters_max"] == 0  # every solve stopped at its non-finite |b|^2
    assert np.array_equal(bits(get_gauge(H, F)), bits(U0))


def test_nonfinite_link_in_leapfrog_and_mts(H):
    F = H.Fields(L, BETA, KAPPA)
    U = O.weak_field(L, SEED, 0.3)
    U[5, 3, 1, 1] = complex(0.0, np.inf)
    put_gauge(H, F, U)
    U0 = get_gauge(H, F)
    H.hmc_refresh(F, SEED, 0)
    st = H.hmc_md_leapfrog(F, 1.0, 4, H.cg_params(tol=1e-10), allow_noconv=True)
    assert st["status"] == H.HMC_E_NAN and st["nonfinite"] == st["solves"] == 5
    put_gauge(H, F, U)
    p = H.mts_params(1.0, 0.12, 2, 2, 2, H.cg_params(tol=1e-10))
    r = H.hmc_trajectory_mts(F, SEED, 0, p)
    assert r["status"] == H.HMC_E_NAN and r["accepted"] == 0
    assert r["nonfinite"] > 0
    assert np.array_equal(bits(get_gauge(H, F)), bits(U0))


@pytest.mark.parametrize("prec", [0, 1])
def test_nonfinite_source_stops_solve(H, prec):
    F = H.Fields(L, BETA, KAPPA, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, SEED, 0.3)
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, H.SOURCE_GAUSS, 3, 0)
    b.view(torch.float64)[17] = float("nan")
    x = F.spinor(full=True)
    st = H.hmc_cg_solve(F, x, b, H.cg_params(tol=1e-10, mode=H.CG_WILSON_SOLVE, prec=prec), allow_noconv=True)
    assert st["status"] == H.HMC_E_NAN and st["iters"] == 0
    bh = F.spinor()
    H.hmc_make_source(F, b, H.SOURCE_GAUSS, 3, 0)
    bh.copy_(b[: bh.numel()])
    bh.view(torch.float64)[5] = float("inf")
    xh = F.spinor()
    st = H.hmc_cg_solve(F, xh, bh, H.cg_params(tol=1e-10, prec=prec), allow_noconv=True)
    assert st["status"] == H.HMC_E_NAN and st["iters"] == 0
