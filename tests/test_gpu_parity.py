"""GPU parity: every step of the HIP path against the FP64 oracle.

Inputs are seeded synthetic fields from tests/synth.py (or each side's own
Philox draws from the same seed).  All calls go through the C ABI
(libhmc.so via the ctypes binding).  Tolerances: bit-exact for indexing,
layout conversion and random words; relative 1e-12 on FP64 fields
(observed ~1e-15 per kernel); solver and trajectory tolerances as noted.
Lattices: 4^4 (one partial block), 8x6x6x10 (Vh = 1440: several blocks and
a ragged tail) and 16^3x32 (the HMC benchmark volume).
"""
import numpy as np
import pytest

import oracle as O
from tests import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = [(4, 4, 4, 4), (8, 6, 6, 10)]
ALL = SMALL + [(16, 16, 16, 32)]


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def put_gauge(H, F, U):
    H.hmc_import_gauge(F, H.to_device_c128(np.ascontiguousarray(U)))


def get_gauge(H, F):
    c = H.canon_gauge_zeros(F.L)
    H.hmc_export_gauge(F, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def put_spinor(H, F, psi, parity, prec=0):
    buf = F.spinor(full=(parity < 0))
    H.hmc_import_spinor(F, buf, H.to_device_c128(np.ascontiguousarray(psi)), parity)
    if prec:
        low = F.spinor(prec=prec, full=False)
        H.hmc_convert_spinor(F, low, prec, buf, 0)
        return low
    return buf


def get_spinor(H, F, buf, parity, prec=0):
    if prec:
        b64 = F.spinor()
        H.hmc_convert_spinor(F, b64, 0, buf, prec)
        buf = b64
    c = H.canon_spinor_zeros(F.L)
    H.hmc_export_spinor(F, c, buf, parity)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def put_momenta(H, F, P):
    H.hmc_import_momenta(F, H.to_device_c128(np.ascontiguousarray(P)))


def get_momenta(H, F):
    c = H.canon_gauge_zeros(F.L)
    H.hmc_export_momenta(F, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def odd_mask(L):
    return synth.site_coords(L).sum(1) % 2 == 1


# ------------------------------------------------------- layout and RNG


@pytest.mark.parametrize("L", SMALL)
def test_layout_roundtrip_bit_exact(H, L):
    F = H.Fields(L, 5.6, 0.15)
    U = synth.gauge_field(1, L)
    put_gauge(H, F, U)
    assert np.array_equal(get_gauge(H, F), U)
    psi = synth.spinor(2, L)
    odd = odd_mask(L)
    for par in (0, 1):
        b = put_spinor(H, F, psi, par)
        want = psi.copy()
        want[odd != bool(par)] = 0
        assert np.array_equal(get_spinor(H, F, b, par), want)
    b = put_spinor(H, F, psi, -1)
    assert np.array_equal(get_spinor(H, F, b, -1), psi)
    P = synth.hermitian_traceless(3, L)
    put_momenta(H, F, P)
    back = get_momenta(H, F)
    assert np.array_equal(back[..., 0, 1], P[..., 0, 1]) and np.array_equal(back[..., 1, 2], P[..., 1, 2])
    assert rel(back, P) < 1e-15


@pytest.mark.parametrize("stream,epoch", [(0, 0), (1, 3), (2, 7), (4, 1)])
def test_random_words_bit_exact(H, stream, epoch):
    seed = 12120785
    sites = np.array([0, 1, 2, 255, 4096, 131071, 10616831, 123456789], dtype=np.int64)
    got = H.hmc_random_words(seed, stream, epoch, torch.from_numpy(sites).cuda(), 8).cpu().numpy().view(np.uint64)
    for k, i in enumerate(sites):
        assert np.array_equal(got[k], O.site_words(seed, int(i), stream, epoch, 8))


def test_random_gaussians_match(H):
    seed = 99
    sites = np.arange(0, 5000, 7, dtype=np.int64)
    got = H.hmc_random_gaussians(seed, 1, 2, torch.from_numpy(sites).cuda(), 32).cpu().numpy()
    want = np.array([O.site_gaussians(seed, int(i), 1, 2, 32) for i in sites])
    # uniforms are bit-exact; log/sin/cos of host libm and device math may
    # differ by an ulp or two
    assert np.abs(got - want).max() <= 8 * np.finfo(float).eps * np.abs(want).max()


# ----------------------------------------------------------- operators


def test_dslash_indexing_bit_exact(H):
    # unit links and small-integer spinors: every hop is exact in FP64, so
    # any indexing, shift or boundary-sign difference shows as a bit change
    L = (8, 6, 6, 10)
    F = H.Fields(L, 5.6, 0.15)
    put_gauge(H, F, O.unit_gauge(L))
    psi = synth.integer_spinor(5, L)
    for dag in (0, 1):
        for par in (0, 1):
            b = put_spinor(H, F, psi, 1 - par)
            out = F.spinor()
            H.hmc_wilson_dslash(F, out, b, par, dag)
            got = get_spinor(H, F, out, par)
            want = O.dslash(L, O.unit_gauge(L), psi, par, dag)
            assert np.array_equal(got, want), (dag, par)


@pytest.mark.parametrize("L", ALL)
def test_dslash_parity(H, L):
    F = H.Fields(L, 5.6, 0.15)
    U = synth.gauge_field(7, L)
    put_gauge(H, F, U)
    psi = synth.spinor(8, L)
    for dag in (0, 1):
        for par in (0, 1):
            b = put_spinor(H, F, psi, 1 - par)
            out = F.spinor()
            H.hmc_wilson_dslash(F, out, b, par, dag)
            got = get_spinor(H, F, out, par)
            assert rel(got, O.dslash(L, U, psi, par, dag)) < 1e-14


@pytest.mark.parametrize("L", SMALL)
def test_mhat_and_wilson_m_parity(H, L):
    k = 0.156
    F = H.Fields(L, 5.6, k)
    U = synth.gauge_field(9, L, eps=0.6)
    put_gauge(H, F, U)
    psi = synth.spinor(10, L)
    for dag in (0, 1):
        b = put_spinor(H, F, psi, 0)
        out = F.spinor()
        H.hmc_mhat(F, out, b, dag)
        assert rel(get_spinor(H, F, out, 0), O.mhat(L, U, k, psi, dag)) < 1e-14
        bf = put_spinor(H, F, psi, -1)
        of = F.spinor(full=True)
        H.hmc_wilson_m(F, of, bf, dag)
        assert rel(get_spinor(H, F, of, -1), O.wilson_m(L, U, k, psi, dag)) < 1e-14


@pytest.mark.parametrize("prec,tol", [(1, 1e-6), (2, 3e-3), (3, 2e-2)])
def test_low_precision_dslash(H, prec, tol):
    L = (8, 6, 6, 10)
    F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
    U = synth.gauge_field(11, L, eps=0.5)
    put_gauge(H, F, U)
    psi = synth.spinor(12, L)
    b = put_spinor(H, F, psi, 1, prec=prec)
    out = F.spinor(prec=prec)
    H.hmc_wilson_dslash(F, out, b, 0, 0, prec)
    got = get_spinor(H, F, out, 0, prec=prec)
    assert rel(got, O.dslash(L, U, psi, 0, 0)) < tol


# ---------------------------------------------------------- global sums


def test_reductions_exact_on_integers(H):
    L = (8, 6, 6, 10)
    F = H.Fields(L, 5.6, 0.15)
    a = synth.integer_spinor(1, L)
    b = synth.integer_spinor(2, L)
    ba, bb = put_spinor(H, F, a, -1), put_spinor(H, F, b, -1)
    assert H.hmc_norm2(F, ba, 2) == O.norm2(a)
    assert H.hmc_inner(F, ba, bb, 2) == O.inner(a, b)
    # sumMulti over time slices in the field's own site order ([parity][Vh])
    t = synth.site_coords(L)[:, 3]
    odd = odd_mask(L)
    sub = np.concatenate([t[~odd], t[odd]]).astype(np.int32)  # cb order = lex order within a parity
    got = H.hmc_sum_multi(F, ba, 2, torch.from_numpy(sub).cuda(), L[3])
    dens = (np.abs(a) ** 2).reshape(synth.volume(L), -1)
    assert got == list(O.sum_multi(dens, t, L[3]))


def test_reductions_random(H):
    L = (16, 16, 16, 32)
    F = H.Fields(L, 5.6, 0.15)
    a, b = synth.spinor(3, L), synth.spinor(4, L)
    ba, bb = put_spinor(H, F, a, -1), put_spinor(H, F, b, -1)
    assert abs(H.hmc_norm2(F, ba, 2) - O.norm2(a)) < 1e-13 * O.norm2(a)
    ip, want = H.hmc_inner(F, ba, bb, 2), O.inner(a, b)
    assert abs(ip - want) < 1e-13 * np.sqrt(O.norm2(a) * O.norm2(b))
    # deterministic: same bits twice
    assert H.hmc_norm2(F, ba, 2) == H.hmc_norm2(F, ba, 2)


# ------------------------------------------------ gauge-field kernels


@pytest.mark.parametrize("L", ALL)
def test_plaquette_and_action(H, L):
    F = H.Fields(L, 5.6, 0.15)
    put_gauge(H, F, O.unit_gauge(L))
    assert H.hmc_plaquette(F) == 1.0
    U = synth.gauge_field(13, L, eps=0.7)
    put_gauge(H, F, U)
    assert abs(H.hmc_plaquette(F) - O.plaquette(L, U)) < 1e-14
    sg = O.gauge_action(L, U, 5.6)
    assert abs(H.hmc_gauge_action(F) - sg) < 1e-13 * sg


@pytest.mark.parametrize("L", SMALL)
def test_plaquette_on_links_that_are_not_su3(H, L):
    """Links that fail the SU(3) check (scaled by 1.1) take the per-site sum
    over all nine entries instead of the plane-paired two-row one."""
    F = H.Fields(L, 5.6, 0.15)
    U = 1.1 * synth.gauge_field(23, L, eps=0.7)
    put_gauge(H, F, U)
    assert abs(H.hmc_plaquette(F) - O.plaquette(L, U)) < 1e-14 * abs(O.plaquette(L, U))


@pytest.mark.parametrize("L", ALL)
def test_gauge_force_parity(H, L):
    F = H.Fields(L, 5.7, 0.15)
    U = synth.gauge_field(14, L, eps=0.6)
    P = synth.hermitian_traceless(15, L)
    put_gauge(H, F, U)
    put_momenta(H, F, P)
    H.hmc_gauge_force(F, 0.05)
    want = P - 0.05 * O.gauge_force(L, U, 5.7)
    assert rel(get_momenta(H, F), want) < 1e-14


@pytest.mark.parametrize("L", ALL)
def test_fermion_force_parity(H, L):
    k = 0.156
    F = H.Fields(L, 5.6, k)
    U = synth.gauge_field(16, L, eps=0.6)
    P = synth.hermitian_traceless(17, L)
    odd = odd_mask(L)
    Xe = synth.spinor(18, L, odd, 0)
    put_gauge(H, F, U)
    put_momenta(H, F, P)
    bx = put_spinor(H, F, Xe, 0)
    H.hmc_fermion_force(F, bx, 0.05)
    X = Xe.copy()
    X[odd] = O.dslash(L, U, Xe, 1)[odd]
    Y = O.mhat(L, U, k, Xe)
    Y[odd] = O.dslash(L, U, Y, 1, dagger=True)[odd]
    want = P - 0.05 * O.fermion_force(L, U, k * k, X, Y)
    assert rel(get_momenta(H, F), want) < 1e-13


@pytest.mark.parametrize("L", ALL)
def test_exp_update_reunit_parity(H, L):
    F = H.Fields(L, 5.6, 0.15)
    U = synth.gauge_field(19, L)
    P = synth.hermitian_traceless(20, L, scale=2.0)
    put_gauge(H, F, U)
    put_momenta(H, F, P)
    H.hmc_exp_update_reunit(F, 0.1)
    got = get_gauge(H, F)
    assert rel(got, O.update_links(L, U, P, 0.1)) < 1e-14
    g = got.reshape(-1, 3, 3)
    assert np.abs(g @ np.conj(np.swapaxes(g, 1, 2)) - np.eye(3)).max() < 1e-14


# ------------------------------------------------------- random fields


@pytest.mark.parametrize("L", ALL)
def test_refresh_and_weak_field_parity(H, L):
    seed, traj, k = 12120785, 3, 0.15
    F = H.Fields(L, 5.6, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    U = O.weak_field(L, seed, 0.3)
    assert rel(get_gauge(H, F), U) < 1e-14
    H.hmc_refresh(F, seed, traj)
    assert rel(get_momenta(H, F), O.refresh_momenta(L, seed, traj)) < 1e-14
    eta = O.eta(L, seed, traj, 0)
    assert rel(get_spinor(H, F, F.pointer(H.FIELD_ETA), 0), eta) < 1e-15
    assert rel(get_spinor(H, F, F.pointer(H.FIELD_PHI), 0), O.mhat(L, U, k, eta, dagger=True)) < 1e-14


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_sources(H, kind):
    L = (8, 6, 6, 10)
    F = H.Fields(L, 5.6, 0.15)
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, kind, 77, 5)
    got = get_spinor(H, F, b, -1)
    want = O.source(L, kind, 77, 5)
    if kind == 0:
        assert rel(got, want) < 1e-15
    else:
        assert np.array_equal(got, want)


# ---------------------------------------------------------------- solvers


@pytest.mark.parametrize("L", ALL)
def test_cg_fixed_iterations_parity(H, L):
    k = 0.156
    F = H.Fields(L, 5.6, k)
    U = synth.gauge_field(21, L, eps=0.4)
    put_gauge(H, F, U)
    b = synth.spinor(22, L, odd_mask(L), 0)
    bb = put_spinor(H, F, b, 0)
    x = F.spinor()
    n = 20
    st = H.hmc_cg_solve(F, x, bb, H.cg_params(fixed_iters=n))
    assert st["iters"] == n
    want, ost = O.cg_mhat(L, U, k, b, fixed_iters=n)
    assert rel(get_spinor(H, F, x, 0), want) < 1e-12
    assert abs(st["true_rel_res"] - ost["true_rel_res"]) < 1e-10


@pytest.mark.parametrize("L", SMALL)
def test_cg_converged_parity(H, L):
    k = 0.15
    F = H.Fields(L, 5.6, k)
    U = O.weak_field(L, 5, 0.3)
    put_gauge(H, F, U)
    b = synth.spinor(23, L, odd_mask(L), 0)
    bb = put_spinor(H, F, b, 0)
    x = F.spinor()
    st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10))
    want, ost = O.cg_mhat(L, U, k, b, tol=1e-10)
    assert st["status"] == 0 and st["true_rel_res"] < 2e-10
    assert abs(st["iters"] - ost["iters"]) <= 1
    assert rel(get_spinor(H, F, x, 0), want) < 1e-8


def test_cg_nonconvergence_reported(H):
    L = (4, 4, 4, 4)
    F = H.Fields(L, 5.6, 0.15)
    put_gauge(H, F, O.weak_field(L, 5, 0.3))
    bb = put_spinor(H, F, synth.spinor(24, L, odd_mask(L), 0), 0)
    x = F.spinor()
    st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, maxiter=3), allow_noconv=True)
    assert st["status"] == H.HMC_E_NOCONV and st["iters"] == 3


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_wilson_solve_parity(H, prec):
    L = (8, 6, 6, 10)
    k = 0.157
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = O.weak_field(L, 1, 0.5)
    put_gauge(H, F, U)
    b = O.source(L, 0, 3, 0)
    bb = put_spinor(H, F, b, -1)
    x = F.spinor(full=True)
    st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, mode=H.CG_WILSON_SOLVE, prec=prec, maxiter=20000))
    assert st["status"] == 0 and st["true_rel_res"] <= 1e-10
    want, ost = O.wilson_solve(L, U, k, b, tol=1e-10)
    assert ost["true_rel_res"] <= 1e-10
    got = get_spinor(H, F, x, -1)
    # both solutions satisfy |b - M x| <= 1e-10 |b|; they agree to ~cond * 1e-10
    assert rel(got, want) < 1e-7
    if prec:
        assert st["reliable_updates"] >= 1


def test_wilson_solves_at_24c48_against_oracle(H):
    """The precision study's configuration (24^3x48, kappa 0.157, weak-field
    eps 0.5 seed 1, Gaussian source seed 1 epoch 0), generated on each side
    from the seeds: FP64 and the three mixed-precision solves against the
    oracle's FP64 CGLS solution."""
    L = (24, 24, 24, 48)
    k = 0.157
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 1, 0.5)
    bb = F.spinor(full=True)
    H.hmc_make_source(F, bb, 0, 1, 0)
    U = O.weak_field(L, 1, 0.5)
    b = O.source(L, 0, 1, 0)
    assert rel(get_spinor(H, F, bb, -1), b) < 1e-15
    want, ost = O.wilson_solve(L, U, k, b, tol=1e-10, maxiter=50000)
    assert ost["status"] == 0 and ost["true_rel_res"] <= 1e-10
    for prec in (0, 1, 2, 3):
        x = F.spinor(full=True)
        st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, mode=H.CG_WILSON_SOLVE, prec=prec, maxiter=50000))
        assert st["status"] == 0 and st["true_rel_res"] <= 1e-10, prec
        got = get_spinor(H, F, x, -1)
        # both solutions satisfy |b - M x| <= 1e-10 |b|; FP64 runs the same
        # iteration as the oracle and agrees far closer than the bound
        assert rel(got, want) < (1e-10 if prec == 0 else 1e-8), (prec, rel(got, want))


# ------------------------------------------------------------------ HMC


def test_leapfrog_parity_c1(H):
    L = (4, 4, 4, 4)
    seed, beta, k = 12120785, 5.6, 0.15
    F = H.Fields(L, beta, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    H.hmc_refresh(F, seed, 0)
    U0 = O.weak_field(L, seed, 0.3)
    P0 = O.refresh_momenta(L, seed, 0)
    phi = O.mhat(L, U0, k, O.eta(L, seed, 0, 0), dagger=True)
    st = H.hmc_md_leapfrog(F, 1.0, 10, H.cg_params(tol=1e-10))
    U1, P1, Xe, ost = O.leapfrog(L, U0, P0, phi, beta, k, 1.0, 10, tol=1e-10)
    assert st["solves"] == ost["solves"] == 11
    assert rel(get_gauge(H, F), U1) < 1e-12
    assert rel(get_momenta(H, F), P1) < 1e-12


def test_trajectory_parity_c1(H):
    L = (4, 4, 4, 4)
    seed, beta, k = 12120785, 5.6, 0.15
    F = H.Fields(L, beta, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    U = O.weak_field(L, seed, 0.3)
    for traj in range(3):
        r = H.hmc_trajectory(F, seed, traj, 1.0, 10, H.cg_params(tol=1e-10))
        U, o = O.hmc_trajectory(L, U, beta, k, seed, traj, 1.0, 10, tol=1e-10)
        assert r["status"] == 0
        assert r["u"] == o["u"]  # bit-exact uniform
        assert r["accepted"] == o["accepted"]
        for key in ("H_old", "H_new", "KE_old", "KE_new", "S_g_old", "S_g_new", "S_f_old", "S_f_new"):
            assert abs(r[key] - o[key]) < 1e-12 * abs(o[key]), key
        assert abs(r["dH"] - o["dH"]) < 1e-12 * abs(o["H_old"])
        assert abs(r["plaquette"] - o["plaquette"]) < 1e-12
        assert rel(get_gauge(H, F), U) < 1e-12


def test_trajectory_parity_c2_short(H):
    """The benchmark's 16^3x32 HMC (beta 5.6, kappa 0.156, weak-field start
    eps 0.3, seed 12120785, step 0.05) over a shortened trajectory (tau 0.1,
    two leapfrog steps: three force evaluations and solves at full size):
    energies, plaquette, links and the accept decision against the oracle."""
    L = (16, 16, 16, 32)
    seed, beta, k = 12120785, 5.6, 0.156
    F = H.Fields(L, beta, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    U = O.weak_field(L, seed, 0.3)
    assert rel(get_gauge(H, F), U) < 1e-14
    r = H.hmc_trajectory(F, seed, 0, 0.1, 2, H.cg_params(tol=1e-10))
    U, o = O.hmc_trajectory(L, U, beta, k, seed, 0, 0.1, 2, tol=1e-10)
    assert r["status"] == 0 and o["status"] == 0
    assert r["u"] == o["u"]
    assert r["accepted"] == o["accepted"]
    for key in ("H_old", "H_new", "KE_old", "KE_new", "S_g_old", "S_g_new", "S_f_old", "S_f_new"):
        assert abs(r[key] - o[key]) < 1e-12 * abs(o[key]), key
    assert abs(r["dH"] - o["dH"]) < 1e-12 * abs(o["H_old"])
    assert abs(r["plaquette"] - o["plaquette"]) < 1e-12
    assert rel(get_gauge(H, F), U) < 1e-12


@pytest.mark.timeout(900)
def test_full_trajectory_parity_c2(H):
    """The headline's whole 16^3x32 integration in the benchmark's launch
    configuration (beta 5.6, kappa 0.156, weak-field start eps 0.3 seed
    12120785, trajectory 0, tau 1 with 20 leapfrog steps: 21 force solves
    to 1e-10) against the oracle.  Trajectory 0 is rejected (dH ~ 1.4e3), so
    the integrated fields are compared after hmc_md_leapfrog from the same
    refresh; the energies, the uniform and the decision of hmc_trajectory
    against the oracle's energies of those fields.  Tolerances (relative,
    whole field): links and momenta 1e-13, the last solve X_e 1e-12 (21
    solves of condition ~1e3 could amplify rounding; measured on MI355X:
    4e-16, 7e-16, 7e-16, printed by the test), every energy 1e-12, dH 1e-12
    of H_old (measured 4e-14), plaquette 1e-12, identical decision."""
    L = (16, 16, 16, 32)
    seed, beta, k = 12120785, 5.6, 0.156
    F = H.Fields(L, beta, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    H.hmc_refresh(F, seed, 0)
    st = H.hmc_md_leapfrog(F, 1.0, 20, H.cg_params(tol=1e-10))
    Ug, Pg = get_gauge(H, F), get_momenta(H, F)
    Xg = get_spinor(H, F, F.pointer(H.FIELD_XE), 0)
    H.hmc_weak_field_start(F, seed, 0.3)
    r = H.hmc_trajectory(F, seed, 0, 1.0, 20, H.cg_params(tol=1e-10))

    U0 = O.weak_field(L, seed, 0.3)
    P0 = O.refresh_momenta(L, seed, 0)
    eta = O.eta(L, seed, 0, 0)
    phi = O.mhat(L, U0, k, eta, dagger=True)
    U1, P1, Xe, ost = O.leapfrog(L, U0, P0, phi, beta, k, 1.0, 20, tol=1e-10)
    want = {"KE_old": O.kinetic(L, P0), "S_g_old": O.gauge_action(L, U0, beta), "S_f_old": O.norm2(eta),
            "KE_new": O.kinetic(L, P1), "S_g_new": O.gauge_action(L, U1, beta), "S_f_new": O.inner(phi, Xe).real}
    want["H_old"] = want["KE_old"] + want["S_g_old"] + want["S_f_old"]
    want["H_new"] = want["KE_new"] + want["S_g_new"] + want["S_f_new"]
    dH = want["H_new"] - want["H_old"]
    u = O.accept_uniform(seed, 0)

    dev = {"U": rel(Ug, U1), "P": rel(Pg, P1), "X_e": rel(Xg, Xe), "dH": abs(r["dH"] - dH) / abs(want["H_old"]),
           "plaq_md": abs(O.plaquette(L, Ug) - O.plaquette(L, U1))}
    dev.update({key: abs(r[key] - want[key]) / abs(want[key]) for key in want})
    print("C2 full-trajectory deviations:", {kk: f"{v:.2e}" for kk, v in dev.items()},
          f"dH gpu {r['dH']:.10f} oracle {dH:.10f}, CG iterations gpu {st['iters_total']} oracle {ost['iters_total']}")
    assert st["status"] == 0 and ost["status"] == 0 and st["solves"] == ost["solves"] == 21
    assert abs(st["iters_total"] - ost["iters_total"]) <= 21
    assert dev["U"] < 1e-13 and dev["P"] < 1e-13 and dev["X_e"] < 1e-12
    assert dev["plaq_md"] < 1e-12
    for key in want:
        assert dev[key] < 1e-12, key
    assert dev["dH"] < 1e-12
    assert r["u"] == u
    assert r["accepted"] == int(dH <= 0 or u < np.exp(-dH))
    assert abs(r["plaquette"] - O.plaquette(L, U0 if not r["accepted"] else U1)) < 1e-12


def test_leapfrog_reversible_at_c2(H):
    """At the benchmark's 16^3x32 shape and launch configuration, with no
    oracle: leapfrog over tau = 0.2 and back over -0.2 returns to the start
    (links and momenta), the full-size check that the integrator and every
    force kernel are time-reversible."""
    L = (16, 16, 16, 32)
    seed = 12120785
    F = H.Fields(L, 5.6, 0.156)
    H.hmc_weak_field_start(F, seed, 0.3)
    H.hmc_refresh(F, seed, 0)
    U0, P0 = get_gauge(H, F), get_momenta(H, F)
    prm = H.cg_params(tol=1e-12)
    st = H.hmc_md_leapfrog(F, 0.2, 4, prm)
    U1 = get_gauge(H, F)
    assert st["solves"] == 5 and rel(U1, U0) > 1e-3
    H.hmc_md_leapfrog(F, -0.2, 4, prm)
    assert rel(get_gauge(H, F), U0) < 1e-11
    assert rel(get_momenta(H, F), P0) < 1e-10


def test_trajectory_accepts_at_small_step(H):
    # a finer integration gives |dH| small enough to accept; both sides agree
    L = (4, 4, 4, 4)
    seed, beta, k = 4, 5.6, 0.15
    F = H.Fields(L, beta, k)
    H.hmc_weak_field_start(F, seed, 0.3)
    U = O.weak_field(L, seed, 0.3)
    r = H.hmc_trajectory(F, seed, 0, 0.2, 20, H.cg_params(tol=1e-12))
    U2, o = O.hmc_trajectory(L, U, beta, k, seed, 0, 0.2, 20, tol=1e-12)
    assert r["accepted"] == o["accepted"] == 1
    assert abs(r["dH"] - o["dH"]) < 1e-10
    assert rel(get_gauge(H, F), U2) < 1e-12


# -------------------------------------- full-size sampled check (48^3x96)


def _coords48(lex):
    return np.stack([lex % 48, (lex // 48) % 48, (lex // 2304) % 48, lex // 110592], 1)


def test_dslash_sampled_at_48c96(H):
    """The 48^3 x 96 bandwidth workload in the launch configuration the
    benchmark times (FP64, and the FP32 / FP16 / BF16 storages): GPU
    weak-field links and Gaussian spinor from their seeds; ~260 even output
    sites recomputed by the oracle from its own draws (only the links and
    spinors those sites touch are generated)."""
    L = (48, 48, 48, 96)
    V = synth.volume(L)
    F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 2, 0.3)
    H.hmc_sync_lowprec(F)
    src = F.spinor(full=True)
    H.hmc_make_source(F, src, 0, 2, 0)
    out = F.spinor()
    hb = H.hmc_field_bytes(L, 0, H.KIND_HALF_SPINOR)
    H.hmc_wilson_dslash(F, out, src[hb:], 0, 0)  # even <- odd
    torch.cuda.synchronize()
    cand = np.random.default_rng(1).integers(0, V, 2048)
    lex = cand[_coords48(cand).sum(1) % 2 == 0][:256]
    corners = [O.lex_index(L, 0, 0, 0, 0), O.lex_index(L, 47, 0, 0, 95), O.lex_index(L, 0, 47, 47, 94),
               O.lex_index(L, 47, 47, 47, 95)]
    lex = np.unique(np.concatenate([lex, corners])).astype(np.int64)
    assert np.all(_coords48(lex).sum(1) % 2 == 0)
    need = set(int(i) for i in lex)
    for x, y, z, t in _coords48(lex):
        for d in ((1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)):
            for sg in (1, -1):
                need.add(O.lex_index(L, (x + sg * d[0]) % 48, (y + sg * d[1]) % 48, (z + sg * d[2]) % 48,
                                     (t + sg * d[3]) % 96))
    need = np.array(sorted(need), dtype=np.int64)
    U = np.zeros((V, 4, 3, 3), np.complex128)  # lazily zero pages: only the needed sites are touched
    psi = np.zeros((V, 4, 3), np.complex128)
    O.weak_field_sites(L, 2, 0.3, need, U)
    O.gauss_source_sites(2, 0, need, psi)
    want = O.dslash_sites(L, U, psi, lex)
    cb = torch.from_numpy(lex // 2).cuda()

    def sampled(o):
        gv = o.view(torch.float64).view(12, -1, 2)[:, cb, :].cpu().numpy()  # component-major [12][Vh]
        return (gv[..., 0] + 1j * gv[..., 1]).T.reshape(-1, 4, 3)

    assert rel(sampled(out), want) < 1e-14
    for prec, tol in ((1, 1e-6), (2, 3e-3), (3, 2e-2)):
        inl, outl = F.spinor(prec=prec), F.spinor(prec=prec)
        H.hmc_convert_spinor(F, inl, prec, src[hb:], H.F64)
        H.hmc_wilson_dslash(F, outl, inl, 0, 0, prec)
        H.hmc_convert_spinor(F, out, H.F64, outl, prec)
        torch.cuda.synchronize()
        assert rel(sampled(out), want) < tol, prec


def test_gauge_force_sampled_at_48c96(H):
    """Staple force at 48^3 x 96 (the kernel shape chosen for large volumes):
    P_after - P_before = -F at ~130 sites of both parities (all four
    directions), the oracle's force from its own weak-field draws of the
    links those staples touch."""
    L = (48, 48, 48, 96)
    V = synth.volume(L)
    Vh = V // 2
    F = H.Fields(L, 5.6, 0.15)
    H.hmc_weak_field_start(F, 2, 0.3)
    H.hmc_refresh(F, 5, 0, H.REFRESH_MOM)
    P = F.arena[F.pointer(H.FIELD_MOMENTA) - F.arena.data_ptr():].view(torch.float64)[: 4 * 2 * 8 * Vh]
    P = P.view(4, 2, 8, Vh)
    lex = np.random.default_rng(3).integers(0, V, 128)
    lex = np.unique(np.concatenate([lex, [O.lex_index(L, 0, 0, 0, 0), O.lex_index(L, 47, 47, 47, 95)]]))
    lex = lex.astype(np.int64)
    c = _coords48(lex)
    par = torch.from_numpy(c.sum(1) % 2).cuda()
    cb = torch.from_numpy(lex // 2).cuda()
    before = P[:, par, :, cb].clone()  # (n, 4, 8)
    H.hmc_gauge_force(F, 1.0)
    torch.cuda.synchronize()
    dP = (P[:, par, :, cb] - before).cpu().numpy()
    need = set()
    offs = [np.array(o) for o in np.ndindex(3, 3, 3, 3) if sum(v != 1 for v in o) <= 2]
    for x in c:
        for o in offs:
            y = (x + o - 1) % np.array(L)
            need.add(O.lex_index(L, *[int(v) for v in y]))
    need = np.array(sorted(need), dtype=np.int64)
    U = np.zeros((V, 4, 3, 3), np.complex128)  # lazily zero pages: only the needed sites are touched
    O.weak_field_sites(L, 2, 0.3, need, U)
    Fo = O.gauge_force_sites(L, U, 5.6, lex)  # (n, 4, 3, 3), Hermitian traceless
    want = -np.stack([Fo[..., 0, 0].real, Fo[..., 1, 1].real, Fo[..., 0, 1].real, Fo[..., 0, 1].imag,
                      Fo[..., 0, 2].real, Fo[..., 0, 2].imag, Fo[..., 1, 2].real, Fo[..., 1, 2].imag], -1)
    assert rel(dP, want) < 1e-12


def _ball48(lex, r):
    """The lexicographic sites within lattice (L1) distance r of the listed
    ones on the 48^3 x 96 torus."""
    L = np.array([48, 48, 48, 96])
    offs = [np.array(o) - r for o in np.ndindex(*(2 * r + 1,) * 4) if sum(abs(v - r) for v in o) <= r]
    c = _coords48(np.asarray(lex))
    out = set()
    for o in offs:
        y = (c + o) % L
        out.update((y[:, 0] + 48 * (y[:, 1] + 48 * (y[:, 2] + 48 * y[:, 3]))).tolist())
    return np.array(sorted(out), dtype=np.int64)


def test_plaquette_at_48c96(H):
    """The plaquette sum over the whole 48^3 x 96 lattice in the launch
    configuration the benchmark times: exactly 1 on the unit gauge, and the
    GPU's weak-field start (seed 2, eps 0.3) against the oracle's plaquette
    of its own draws of the same field."""
    L = (48, 48, 48, 96)
    F = H.Fields(L, 5.6, 0.15)
    put_gauge(H, F, O.unit_gauge(L))
    assert H.hmc_plaquette(F) == 1.0
    H.hmc_weak_field_start(F, 2, 0.3)
    p = H.hmc_plaquette(F)
    want = O.plaquette(L, O.weak_field(L, 2, 0.3))
    assert abs(p - want) < 1e-12 * abs(want)


def test_fermion_force_sampled_at_48c96(H):
    """The fermion force at 48^3 x 96 (the launch configuration the
    benchmark times): P_after - P_before = -F_f at ~70 sites of both
    parities, all four directions.  The oracle builds X = (X_e, D_oe X_e)
    and Y = (Mhat X_e, D^dag_oe Mhat X_e) at the sites the force reads from
    its own draws of the links and of the Gaussian X_e, on the ball of
    radius four around the samples that those hops reach."""
    L = (48, 48, 48, 96)
    V = synth.volume(L)
    Vh = V // 2
    k = 0.15
    F = H.Fields(L, 5.6, k)
    H.hmc_weak_field_start(F, 2, 0.3)
    H.hmc_refresh(F, 5, 0, H.REFRESH_MOM)
    src = F.spinor(full=True)
    H.hmc_make_source(F, src, 0, 2, 0)
    hb = H.hmc_field_bytes(L, 0, H.KIND_HALF_SPINOR)
    P = F.arena[F.pointer(H.FIELD_MOMENTA) - F.arena.data_ptr():].view(torch.float64)[: 4 * 2 * 8 * Vh]
    P = P.view(4, 2, 8, Vh)
    lex = np.random.default_rng(4).integers(0, V, 64)
    lex = np.unique(np.concatenate([lex, [O.lex_index(L, 0, 0, 0, 0), O.lex_index(L, 47, 47, 47, 95),
                                          O.lex_index(L, 47, 0, 0, 95)]])).astype(np.int64)
    c = _coords48(lex)
    par = torch.from_numpy(c.sum(1) % 2).cuda()
    cb = torch.from_numpy(lex // 2).cuda()
    before = P[:, par, :, cb].clone()  # (n, 4, 8)
    H.hmc_fermion_force(F, src[:hb], 1.0)  # X_e: the even half of the Gaussian source
    torch.cuda.synchronize()
    dP = (P[:, par, :, cb] - before).cpu().numpy()

    def even(s):
        return s[_coords48(s).sum(1) % 2 == 0]

    def odd(s):
        return s[_coords48(s).sum(1) % 2 == 1]

    ball = _ball48(lex, 4)
    U = np.zeros((V, 4, 3, 3), np.complex128)  # lazily zero pages: only the ball is touched
    O.weak_field_sites(L, 2, 0.3, ball, U)
    X = np.zeros((V, 4, 3), np.complex128)
    Y = np.zeros((V, 4, 3), np.complex128)
    O.gauss_source_sites(2, 0, even(ball), X)  # X_e on the even sites of the ball
    o3 = odd(_ball48(lex, 3))
    X[o3] = O.dslash_sites(L, U, X, o3)  # X_o = D_oe X_e
    e2 = even(_ball48(lex, 2))
    Y[e2] = X[e2] - k * k * O.dslash_sites(L, U, X, e2)  # Y_e = Mhat X_e
    o1 = odd(_ball48(lex, 1))
    Y[o1] = O.dslash_sites(L, U, Y, o1, dagger=True)  # Y_o = D^dag_oe Y_e
    Fo = O.fermion_force_sites(L, U, k * k, X, Y, lex)  # (n, 4, 3, 3), Hermitian traceless
    want = -np.stack([Fo[..., 0, 0].real, Fo[..., 1, 1].real, Fo[..., 0, 1].real, Fo[..., 0, 1].imag,
                      Fo[..., 0, 2].real, Fo[..., 0, 2].imag, Fo[..., 1, 2].real, Fo[..., 1, 2].imag], -1)
    assert rel(dP, want) < 1e-12


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_trajectory_with_mixed_precision_solves_c1(H, prec):
    """The 4^4 chain with the force solves in mixed precision (FP32 / FP16 /
    BF16 inner storage, device-driven FP64 reliable updates, the same 1e-10
    FP64 true-residual stop) against the FP64 oracle: every energy within
    1e-10 of H_old (the solves differ from the oracle's by their residual
    tolerance, not by rounding), the same Metropolis decision, links after
    the integration within 1e-9."""
    L = (4, 4, 4, 4)
    seed, beta, k = 12120785, 5.6, 0.15
    F = H.Fields(L, beta, k, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, seed, 0.3)
    U = O.weak_field(L, seed, 0.3)
    prm = H.cg_params(tol=1e-10, prec=prec)
    for traj in range(2):
        r = H.hmc_trajectory(F, seed, traj, 1.0, 10, prm)
        U_md = O.leapfrog(L, U, O.refresh_momenta(L, seed, traj),
                          O.mhat(L, U, k, O.eta(L, seed, traj, 0), dagger=True), beta, k, 1.0, 10, tol=1e-10)[0]
        U, o = O.hmc_trajectory(L, U, beta, k, seed, traj, 1.0, 10, tol=1e-10)
        assert r["status"] == 0 and r["accepted"] == o["accepted"] and r["u"] == o["u"]
        dev = {key: abs(r[key] - o[key]) / abs(o["H_old"]) for key in ("H_old", "H_new", "dH", "S_f_new")}
        print(f"prec {prec} trajectory {traj}: deviations relative to H_old", {kk: f"{v:.1e}" for kk, v in dev.items()})
        assert max(dev.values()) < 1e-10, dev
        if not r["accepted"]:
            assert rel(get_gauge(H, F), U) < 1e-14  # restored start
        else:
            assert rel(get_gauge(H, F), U_md) < 1e-9
