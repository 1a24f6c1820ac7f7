"""GPU parity of the mass-preconditioned (Hasenbusch) HMC on nested time
scales against the FP64 oracle: the general Wilson-force bilinear, the
nested integrator, and whole trajectories (4^4, C1 action, kappa_h 0.13)."""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_gpu_parity import get_gauge, get_momenta, get_spinor, put_gauge, put_momenta, put_spinor, rel

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


def field_view(H, F, which, nbytes):
    off = F.pointer(which) - F.arena.data_ptr()
    return F.arena[off:off + nbytes]


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 6, 6, 10)])
def test_fermion_force_bilinear_parity(H, L):
    kc, coef = 0.13, 0.37
    F = H.Fields(L, 5.6, 0.15)
    U = synth.gauge_field(51, L, eps=0.5)
    put_gauge(H, F, U)
    P = synth.hermitian_traceless(52, L)
    put_momenta(H, F, P)
    odd = O.parity_mask(L)
    Xe = synth.spinor(53, L, odd, 0)
    Ye = synth.spinor(54, L, odd, 0)
    H.hmc_fermion_force_bilinear(F, put_spinor(H, F, Xe, 0), put_spinor(H, F, Ye, 0), kc, coef)
    X, Y = Xe.copy(), Ye.copy()
    X[odd] = O.dslash(L, U, Xe, 1)[odd]
    Y[odd] = O.dslash(L, U, Ye, 1, dagger=True)[odd]
    want = P - coef * O.fermion_force(L, U, kc * kc, X, Y)
    assert rel(get_momenta(H, F), want) < 1e-13


def test_md_mts_parity_c1(H):
    L = (4, 4, 4, 4)
    k, kh = 0.15, 0.13
    F = H.Fields(L, 5.6, k)
    U = O.weak_field(L, SEED, 0.3)
    P = O.refresh_momenta(L, SEED, 0)
    phi1 = O.mhat(L, U, kh, O.eta(L, SEED, 0), dagger=True)
    phi2 = O.mhat(L, U, kh, O.eta2(L, SEED, 0))
    put_gauge(H, F, U)
    put_momenta(H, F, P)
    hb = H.hmc_field_bytes(L, H.F64, H.KIND_HALF_SPINOR)
    field_view(H, F, H.FIELD_PHI, hb).copy_(put_spinor(H, F, phi1, 0))
    p = H.mts_params(0.5, kh, 3, 2, 2, H.cg_params(tol=1e-12))
    ms = H.hmc_md_mts(F, put_spinor(H, F, phi2, 0), p)
    a = O.mts_action(5.6, k, kh, 3, 2, 2, tol=1e-12)
    Uo, Po, X1, X2, chi, mo, s = O.mts_integrate(L, U, P, phi1, phi2, a, 0.5)
    assert s == 0 and ms["status"] == 0
    for key in ("solves_ratio", "solves_heavy", "gauge_forces", "link_updates"):
        assert ms[key] == mo[key], key
    assert rel(get_gauge(H, F), Uo) < 1e-12
    assert rel(get_momenta(H, F), Po) < 1e-12
    assert rel(get_spinor(H, F, field_view(H, F, H.FIELD_XE, hb), 0), X1) < 1e-10


def test_trajectory_mts_parity_c1(H):
    L = (4, 4, 4, 4)
    k, kh = 0.15, 0.13
    F = H.Fields(L, 5.6, k)
    H.hmc_weak_field_start(F, SEED, 0.3)
    U = O.weak_field(L, SEED, 0.3)
    a = O.mts_action(5.6, k, kh, 4, 2, 2, tol=1e-10)
    p = H.mts_params(1.0, kh, 4, 2, 2, H.cg_params(tol=1e-10))
    for traj in range(3):
        r = H.hmc_trajectory_mts(F, SEED, traj, p)
        U, o = O.hmc_trajectory_mts(L, U, a, SEED, traj, 1.0)
        assert r["status"] == 0 and o["status"] == 0
        assert r["u"] == o["u"]
        assert r["accepted"] == o["accepted"]
        for key in ("H_old", "H_new", "KE_old", "KE_new", "S_g_old", "S_g_new", "S_f_old", "S_f_new",
                    "S1_old", "S2_old", "S1_new", "S2_new"):
            assert abs(r[key] - o[key]) < 1e-11 * abs(o[key]), key
        assert abs(r["dH"] - o["dH"]) < 1e-11 * abs(o["H_old"])
        assert abs(r["plaquette"] - o["plaquette"]) < 1e-12
        for key in ("solves_ratio", "solves_heavy", "gauge_forces", "link_updates"):
            assert r[key] == o[key], key
        assert rel(get_gauge(H, F), U) < 1e-12


def test_trajectory_mts_reduces_to_plain_at_equal_kappa(H):
    L = (4, 4, 4, 4)
    F1 = H.Fields(L, 5.6, 0.15)
    F2 = H.Fields(L, 5.6, 0.15)
    for F in (F1, F2):
        H.hmc_weak_field_start(F, SEED, 0.3)
    cg = H.cg_params(tol=1e-12)
    r1 = H.hmc_trajectory_mts(F1, SEED, 0, H.mts_params(1.0, 0.15, 10, 1, 1, cg))
    r2 = H.hmc_trajectory(F2, SEED, 0, 1.0, 10, cg)
    assert abs(r1["S2_new"] - r1["S2_old"]) < 1e-9 * r1["S2_old"]
    assert abs(r1["dH"] - r2["dH"]) < 1e-7 * abs(r2["H_old"])
    assert r1["accepted"] == r2["accepted"]
