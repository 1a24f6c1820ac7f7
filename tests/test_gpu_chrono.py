"""GPU parity of the CG started from a guess and of HMC trajectories whose
force solves start from the chronological (minimal-residual) guess."""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_gpu_parity import get_gauge, get_spinor, put_gauge, put_spinor, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEED = 12120785


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


@pytest.mark.parametrize("prec", [0, 1])
def test_cg_from_a_guess(H, prec):
    L = (8, 6, 6, 10)
    k = 0.15
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = synth.gauge_field(61, L, eps=0.5)
    put_gauge(H, F, U)
    odd = O.parity_mask(L)
    b = synth.spinor(62, L, odd, 0)
    x0 = synth.spinor(63, L, odd, 0)
    bb = put_spinor(H, F, b, 0)
    x = put_spinor(H, F, x0, 0)
    st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, prec=prec, initial_guess=1))
    want, ost = O.cg_mhat_x0(L, U, k, b, x0, tol=1e-10)
    assert st["status"] == 0 and st["true_rel_res"] <= 1.01e-10
    assert rel(get_spinor(H, F, x, 0), want) < (1e-12 if prec == 0 else 1e-8)
    if prec == 0:
        assert abs(st["iters"] - ost["iters"]) <= 1
    # the solution as guess needs no iteration
    st2 = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-8, initial_guess=1))
    assert st2["iters"] == 0


@pytest.mark.parametrize("tau,nsteps,nc", [(0.1, 4, 1), (0.1, 4, 3), (1.0, 10, 4)])
def test_trajectory_chrono_parity_c1(H, tau, nsteps, nc):
    L = (4, 4, 4, 4)
    F = H.Fields(L, 5.6, 0.15)
    H.hmc_weak_field_start(F, SEED, 0.3)
    U = O.weak_field(L, SEED, 0.3)
    r = H.hmc_trajectory(F, SEED, 0, tau, nsteps, H.cg_params(tol=1e-10), n_chrono=nc)
    Uo, o = O.hmc_trajectory_chrono(L, U, 5.6, 0.15, SEED, 0, tau, nsteps, nc, tol=1e-10)
    rp = O.hmc_trajectory(L, U, 5.6, 0.15, SEED, 0, tau, nsteps, tol=1e-10)[1]
    assert r["status"] == 0 and o["status"] == 0
    assert r["accepted"] == o["accepted"] and r["u"] == o["u"]
    for key in ("H_old", "H_new", "KE_new", "S_g_new", "S_f_new"):
        assert abs(r[key] - o[key]) < 1e-10 * abs(o[key]), key
    assert abs(r["dH"] - o["dH"]) < 1e-10 * abs(o["H_old"])
    assert rel(get_gauge(H, F), Uo) < 1e-10
    # same iteration counts up to one per solve, fewer than the plain chain
    assert abs(r["cg_iters_total"] - o["cg_iters_total"]) <= nsteps + 1
    assert r["cg_iters_total"] < rp["cg_iters_total"]
