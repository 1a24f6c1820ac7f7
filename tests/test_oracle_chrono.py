"""Pins of the oracle's chronological initial guess (minimal-residual
extrapolation over previous solutions) and the CG started from a guess
(CPU only)."""
import numpy as np

import oracle as O
from tests import synth

SEED = 12120785


def A(L, U, k, x):
    return O.mhat(L, U, k, O.mhat(L, U, k, x), dagger=True)


def setup():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 7, 0.4)
    odd = O.parity_mask(L)
    b = synth.spinor(9, L, odd, 0)
    return L, U, odd, b


def test_cg_from_zero_guess_is_plain_cg():
    L, U, odd, b = setup()
    x1, s1 = O.cg_mhat(L, U, 0.15, b, tol=1e-12)
    x2, s2 = O.cg_mhat_x0(L, U, 0.15, b, np.zeros_like(b), tol=1e-12)
    assert s1["iters"] == s2["iters"] and np.array_equal(x1, x2)


def test_cg_from_the_solution_takes_no_iteration():
    L, U, odd, b = setup()
    x, _ = O.cg_mhat(L, U, 0.15, b, tol=1e-13)
    x2, s = O.cg_mhat_x0(L, U, 0.15, b, x, tol=1e-10)
    assert s["iters"] == 0 and np.array_equal(x2, x)
    # a guess from a history holding the solution reproduces it
    x0, st = O.chrono_guess(L, U, 0.15, b, [synth.spinor(3, L, odd, 0), x])
    assert st == 0 and np.abs(x0 - x).max() < 1e-10 * np.abs(x).max()


def test_guess_satisfies_the_galerkin_condition():
    L, U, odd, b = setup()
    k = 0.15
    hist = [synth.spinor(s, L, odd, 0) for s in (11, 12, 13)]
    x0, st = O.chrono_guess(L, U, k, b, hist)
    assert st == 0
    r = b - A(L, U, k, x0)
    for y in hist:  # <y_j, b - A x0> = 0 for every history vector
        assert abs(O.inner(y, r)) < 1e-12 * np.sqrt(O.norm2(y) * O.norm2(b))
    # and x0 lies in their span: least squares against the history basis
    Yb = np.stack([h[~odd].ravel() for h in hist], 1)
    c, *_ = np.linalg.lstsq(Yb, x0[~odd].ravel(), rcond=None)
    assert np.abs(Yb @ c - x0[~odd].ravel()).max() < 1e-12 * np.abs(x0).max()


def test_guess_is_a_norm_optimal_in_the_span():
    # A-norm error of the Galerkin guess is below that of perturbed combinations
    L, U, odd, b = setup()
    k = 0.15
    x, _ = O.cg_mhat(L, U, k, b, tol=1e-13)
    hist = [synth.spinor(s, L, odd, 0) for s in (21, 22)]
    x0, _ = O.chrono_guess(L, U, k, b, hist)

    def err(v):
        e = v - x
        return O.inner(e, A(L, U, k, e)).real

    base = err(x0)
    for dc in ([1e-3, 0], [0, 1e-3], [1e-3j, -1e-3]):
        assert err(x0 + dc[0] * hist[0] + dc[1] * hist[1]) > base


def test_chrono_trajectory_saves_iterations_and_keeps_the_result():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, SEED, 0.3)
    # tau 0.1 in 4 steps: accepted, so the compared links are the evolved ones
    Up, rp = O.hmc_trajectory(L, U, 5.6, 0.15, SEED, 0, 0.1, 4)
    assert rp["accepted"] == 1 and np.abs(Up - U).max() > 1e-3
    for n in (1, 2, 4):
        Uc, rc = O.hmc_trajectory_chrono(L, U, 5.6, 0.15, SEED, 0, 0.1, 4, n)
        assert rc["status"] == 0
        assert rc["cg_iters_total"] < rp["cg_iters_total"]
        assert abs(rc["dH"] - rp["dH"]) < 1e-7 * abs(rp["H_old"])
        assert rc["accepted"] == rp["accepted"]
        assert np.abs(Uc - Up).max() < 1e-8
    assert O.hmc_trajectory_chrono(L, U, 5.6, 0.15, SEED, 0, 1.0, 10, 0)[1]["status"] == -1
    assert O.hmc_trajectory_chrono(L, U, 5.6, 0.15, SEED, 0, 1.0, 10, 9)[1]["status"] == -1
