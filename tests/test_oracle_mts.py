"""Pins of the oracle's mass-preconditioned (Hasenbusch) action and its
nested multi-time-scale integrator (CPU only).

What fixes the result independently of the oracle's own code:
* the integrator schedule: per level the kicks add up to tau, the link
  steps add up to tau, the schedule is a palindrome (time reversal), and
  its evaluation counts are those of nested leapfrog with merged kicks;
* the ratio force equals the finite-difference derivative of the ratio
  action (a converged solve), the heavy force equals the plain Wilson
  force at kappa_h;
* at kappa_h = kappa the ratio factor is the identity: its force vanishes
  and the trajectory reduces to plain HMC;
* reversibility and dH ~ eps^2 of the integrator.
"""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_oracle_pins import _dS_predicted, _force_vectors, _rotate

SEED = 12120785


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 3, 2), (3, 1, 4), (5, 2, 1)])
def test_schedule_structure(n):
    tau = 0.7
    coef, eps = O.mts_schedule(*n, tau)
    n0, n1, n2 = n
    assert coef.shape == (n0 * n1 * n2 + 1, 3)
    assert np.allclose(coef.sum(0), tau, rtol=0, atol=1e-15)
    assert abs(eps.sum() - tau) < 1e-15 and eps[-1] == 0
    # palindrome: reversing the stretches gives the same schedule
    assert np.allclose(coef, coef[::-1], rtol=0, atol=1e-15)
    assert np.allclose(eps[:-1], eps[:-1][::-1], rtol=0, atol=1e-15)
    # force evaluations per level (kicks between two link steps merged)
    counts = (coef != 0).sum(0)
    assert counts.tolist() == [n0 + 1, n0 * n1 + 1, n0 * n1 * n2 + 1]
    # every link step is the innermost step size
    assert np.allclose(eps[:-1], tau / (n0 * n1 * n2), rtol=0, atol=1e-15)


def test_single_level_schedule_is_plain_leapfrog():
    coef, eps = O.mts_schedule(4, 1, 1, 1.0)
    want = np.array([0.125, 0.25, 0.25, 0.25, 0.125])
    for lvl in range(3):
        assert np.allclose(coef[:, lvl], want, rtol=0, atol=1e-16)


@pytest.fixture(scope="module")
def small():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 7, 0.4)
    P = synth.hermitian_traceless(8, L)
    odd = O.parity_mask(L)
    phi = synth.spinor(9, L, odd, 0)
    return L, U, P, phi


def test_ratio_force_finite_difference(small):
    L, U, P, phi2 = small
    a = O.mts_action(5.6, 0.15, 0.12, 1, 1, 1, tol=1e-14)
    h = 1e-4
    F, X, s = O.mts_force(L, U, a, 0, phi2)
    assert s == 0
    fd = (O.ratio_action(L, _rotate(U, P, h), a, phi2) - O.ratio_action(L, _rotate(U, P, -h), a, phi2)) / (2 * h)
    pred = _dS_predicted(P, F)
    assert abs(fd - pred) < 1e-6 * abs(pred)
    Fm = F.reshape(-1, 3, 3)
    assert np.abs(Fm - np.conj(np.swapaxes(Fm, 1, 2))).max() < 1e-14
    assert np.abs(np.trace(Fm, axis1=1, axis2=2)).max() < 1e-13


def test_heavy_force_is_wilson_force_at_kappa_h(small):
    L, U, P, phi1 = small
    kh = 0.12
    a = O.mts_action(5.6, 0.15, kh, 1, 1, 1, tol=1e-14)
    F, X1, s = O.mts_force(L, U, a, 1, phi1)
    Xe, _ = O.cg_mhat(L, U, kh, phi1, tol=1e-14)
    Xf, Yf = _force_vectors(L, U, kh, Xe)
    want = O.fermion_force(L, U, kh * kh, Xf, Yf)
    assert np.abs(F - want).max() <= 1e-14 * np.abs(want).max()
    Fg, _, _ = O.mts_force(L, U, a, 2)
    assert np.array_equal(Fg, O.gauge_force(L, U, 5.6))


def test_ratio_force_vanishes_at_equal_kappa(small):
    L, U, P, phi = small
    a = O.mts_action(5.6, 0.15, 0.15, 1, 1, 1, tol=1e-14)
    Fr, _, _ = O.mts_force(L, U, a, 0, phi)
    Fh, _, _ = O.mts_force(L, U, a, 1, phi)
    assert np.abs(Fr).max() < 1e-10 * np.abs(Fh).max()
    # and the ratio action is |phi|^2
    assert abs(O.ratio_action(L, U, a, phi) - O.norm2(phi)) < 1e-12 * O.norm2(phi)


def test_reduces_to_plain_hmc_at_equal_kappa():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, SEED, 0.3)
    a = O.mts_action(5.6, 0.15, 0.15, 10, 1, 1, tol=1e-13)
    Um, rm = O.hmc_trajectory_mts(L, U, a, SEED, 0, 1.0)
    Up, rp = O.hmc_trajectory(L, U, 5.6, 0.15, SEED, 0, 1.0, 10, tol=1e-13)
    assert rm["S1_old"] == rp["S_f_old"]
    assert rm["S2_old"] == O.norm2(O.eta2(L, SEED, 0))
    assert abs(rm["S2_new"] - rm["S2_old"]) < 1e-9 * rm["S2_old"]
    assert abs(rm["dH"] - rp["dH"]) < 1e-7 * abs(rp["H_old"])
    assert rm["accepted"] == rp["accepted"]
    # the links after the trajectory (rejected: both equal the start)
    P = O.refresh_momenta(L, SEED, 0)
    eta = O.eta(L, SEED, 0, 0)
    phi1 = O.mhat(L, U, 0.15, eta, dagger=True)
    phi2 = O.eta2(L, SEED, 0)  # at kappa_h = kappa, phi_2 = eta_2
    Ui, Pi, *_ = O.mts_integrate(L, U, P, phi1, phi2, a, 1.0)
    Ul, Pl, _, _ = O.leapfrog(L, U, P, phi1, 5.6, 0.15, 1.0, 10, tol=1e-13)
    assert np.abs(Ui - Ul).max() < 1e-9 and np.abs(Pi - Pl).max() < 1e-8


def test_eta2_is_an_independent_stream():
    L = [4, 4, 4, 4]
    e1, e2 = O.eta(L, SEED, 3), O.eta2(L, SEED, 3)
    assert not np.allclose(e1, e2)
    assert abs(O.norm2(e2) / (12 * 128) - 1) < 0.1  # E|eta_k|^2 = 1 on the 128 even sites
    assert np.all(e2[O.parity_mask(L)] == 0)


def test_mts_integrator_is_reversible():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, SEED, 0.3)
    P = O.refresh_momenta(L, SEED, 0)
    a = O.mts_action(5.6, 0.15, 0.13, 3, 2, 2, tol=1e-14)
    phi1 = O.mhat(L, U, 0.13, O.eta(L, SEED, 0), dagger=True)
    phi2 = O.mhat(L, U, 0.13, O.eta2(L, SEED, 0))
    U1, P1, *_ = O.mts_integrate(L, U, P, phi1, phi2, a, 0.5)
    U2, P2, *_ = O.mts_integrate(L, U1, -P1, phi1, phi2, a, 0.5)
    assert np.abs(U2 - U).max() < 1e-10
    assert np.abs(-P2 - P).max() < 1e-9


def test_mts_dH_scales_as_eps_squared():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, SEED, 0.3)
    dH = []
    for n0 in (6, 12, 24):
        a = O.mts_action(5.6, 0.15, 0.13, n0, 2, 2, tol=1e-14)
        dH.append(O.hmc_trajectory_mts(L, U, a, SEED, 0, 0.5)[1]["dH"])
    for x, y in zip(dH, dH[1:]):
        assert 0.2 < y / x < 0.3, dH


def test_mts_trajectory_bookkeeping():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, SEED, 0.3)
    a = O.mts_action(5.6, 0.15, 0.13, 4, 2, 2)
    U1, r = O.hmc_trajectory_mts(L, U, a, SEED, 1, 1.0)
    assert r["status"] == 0
    assert r["S1_old"] == O.norm2(O.eta(L, SEED, 1))
    assert r["S2_old"] == O.norm2(O.eta2(L, SEED, 1))
    assert abs(r["S_f_old"] - (r["S1_old"] + r["S2_old"])) < 1e-12 * r["S_f_old"]
    assert abs(r["dH"] - (r["H_new"] - r["H_old"])) < 1e-9
    assert r["solves_ratio"] == 4 + 1 and r["solves_heavy"] == 4 * 2 + 1 + 1  # + the heatbath solve
    assert r["gauge_forces"] == 4 * 2 * 2 + 1 and r["link_updates"] == 16
    acc = r["dH"] <= 0 or r["u"] < np.exp(-r["dH"])
    assert r["accepted"] == int(acc)
    if not acc:
        assert np.array_equal(U1, U)
