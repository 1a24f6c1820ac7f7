"""The oracle pins catch plausible mistakes.

Each mutant is oracle.c with one planted error (a flipped projector, a
dropped boundary sign, a missing dagger, a wrong coefficient, a transposed
product, ...).  It is compiled to a temporary library and swapped in for the
real oracle; at least one of the listed pin tests must then fail.  Mistakes
are planted only in the CPU oracle.
"""
import os

import pytest

import oracle as O
from tests import synth
from tests import test_oracle_chrono as CH
from tests import test_oracle_mts as M
from tests import test_oracle_pins as P

SRC = open(os.path.join(os.path.dirname(O.__file__), "oracle.c")).read()


def c1():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, 12120785, 0.3)
    Pm = O.refresh_momenta(L, 12120785, 0)
    eta = O.eta(L, 12120785, 0, 0)
    phi = O.mhat(L, U, 0.15, eta, dagger=True)
    return L, U, Pm, eta, phi


def small():
    L = [4, 2, 2, 4]
    return L, O.weak_field(L, 7, 0.4), synth.hermitian_traceless(8, L), synth.spinor(9, L, O.parity_mask(L), 0)


def schedules():
    for n in [(1, 1, 1), (2, 3, 2)]:
        M.test_schedule_structure(n)


def free_field():
    for n in [(0, 0, 0, 0), (1, 2, 0, 3), (3, 5, 1, 7)]:
        P.test_free_field_closed_form(n)


MUTANTS = {
    "forward/backward projectors swapped": (
        "int sgn = (dir > 0) ? s_fwd : -s_fwd;", "int sgn = (dir > 0) ? -s_fwd : s_fwd;",
        [free_field]),
    "antiperiodic time sign dropped": (
        "double bc = wraps ? -1.0 : 1.0;\n            /* colour matrix", "double bc = 1.0;\n            /* colour matrix",
        [free_field]),
    "backward link not daggered": (
        "mat_dag(&U[(j * 4 + mu) * 9], Um);", "memcpy(Um, &U[(j * 4 + mu) * 9], sizeof Um);",
        [P.test_gamma5_hermiticity_and_dagger, P.test_gauge_covariance]),
    "dagger flag ignored": (
        "int s_fwd = dagger ? +1 : -1;", "int s_fwd = -1;",
        [P.test_gamma5_hermiticity_and_dagger]),
    "Mhat uses kappa instead of kappa^2": (
        "in[i * 12 + k] - kappa * kappa * u[i * 12 + k]", "in[i * 12 + k] - kappa * u[i * 12 + k]",
        [P.test_schur_determinant_and_solvers]),
    "gauge force coefficient beta/6": (
        "-I * beta / 12.0 * Z[k]", "-I * beta / 6.0 * Z[k]",
        [P.test_gauge_force_finite_difference]),
    "lower staple orientation": (
        "mat_mul(a, &U[(xmnu * 4 + nu) * 9], a);", "mat_mul(&U[(xmnu * 4 + nu) * 9], a, a);",
        [P.test_gauge_force_finite_difference, P.test_forces_gauge_covariant]),
    "fermion force boundary sign dropped": (
        "double s = wraps ? -1.0 : 1.0;\n    cplx M1[9]", "double s = 1.0;\n    cplx M1[9]",
        [P.test_fermion_force_finite_difference]),
    "fermion force projectors swapped": (
        "cplx pm = proj_el(mu, -1, a, b), pp = proj_el(mu, +1, a, b);",
        "cplx pm = proj_el(mu, +1, a, b), pp = proj_el(mu, -1, a, b);",
        [P.test_fermion_force_finite_difference]),
    "fermion force W term transposed": (
        "mat_mul(M2, Ud, t);", "mat_mul(Ud, M2, t);",
        [P.test_fermion_force_finite_difference]),
    "reunit third row not conjugated": (
        "u[6] = conj(u[1] * u[5] - u[2] * u[4]);", "u[6] = (u[1] * u[5] - u[2] * u[4]);",
        [P.test_reunit_projects_to_su3_and_fixes_su3]),
    "Philox key increment typo": (
        "inc1 = 0xBB67AE8584CAA73BULL", "inc1 = 0xBB67AE8584CAA73AULL",
        [P.test_philox_known_answer_vectors]),
    "Philox round output order": (
        "x0 = hi1 ^ x1 ^ k0;", "x0 = hi0 ^ x1 ^ k0;",
        [P.test_philox_known_answer_vectors, P.test_philox_matches_numpy]),
    "CG beta inverted": (
        "double beta = rr_new / rr;", "double beta = rr / rr_new;",
        [P.test_schur_determinant_and_solvers]),
    "plaquette missing dagger": (
        "mat_dag(&U[(xnu * 4 + mu) * 9], t);\n            mat_mul(a, t, a);",
        "memcpy(t, &U[(xnu * 4 + mu) * 9], sizeof t);\n            mat_mul(a, t, a);",
        [P.test_plaquette_single_abelian_link, P.test_gauge_covariance]),
    "generator normalisation lambda instead of lambda/2": (
        "H[1] = 0.5 * (om[0] - I * om[1]);", "H[1] = (om[0] - I * om[1]);",
        [P.test_algebra_generators]),
    "leapfrog first kick a full step": (
        "status |= force_kick(L, U, P, phi, a, 0.5 * eps, Xe, ms);", "status |= force_kick(L, U, P, phi, a, eps, Xe, ms);",
        [lambda: P.test_leapfrog_reversibility(c1())]),
    "Metropolis with exp(+dH)": (
        "(dH <= 0 || u < exp(-dH))", "(dH <= 0 || u < exp(dH))",
        [lambda: P.test_trajectory_bookkeeping(c1())]),
    "ratio force: second bilinear added": (
        "for (long k = 0; k < V * 36; ++k) F[k] -= F2[k];", "for (long k = 0; k < V * 36; ++k) F[k] += F2[k];",
        [lambda: M.test_ratio_force_finite_difference(small())]),
    "ratio force: kappa in place of kappa_h": (
        "or_fermion_force(L, U, a->kappa_h * a->kappa_h, X, Y, F2);", "or_fermion_force(L, U, a->kappa * a->kappa, X, Y, F2);",
        [lambda: M.test_ratio_force_finite_difference(small())]),
    "nested leapfrog: last kick a full step": (
        "mts_emit(ops, nops, level, k < n ? e : 0.5 * e);", "mts_emit(ops, nops, level, e);",
        [schedules]),
    "ratio heatbath without the heavy solve": (
        "or_mhat(L, U, a->kappa_h, X1, phi2, 0);", "or_mhat(L, U, a->kappa_h, t, phi2, 0);",
        [M.test_reduces_to_plain_hmc_at_equal_kappa]),
    "chronological guess: Gram matrix conjugated": (
        "G[j * m + k] = ri[0] + I * ri[1];", "G[j * m + k] = ri[0] - I * ri[1];",
        [CH.test_guess_satisfies_the_galerkin_condition]),
    "CG from a guess: residual not recomputed": (
        "for (long k = 0; k < n; ++k) { r[k] = b[k] - q[k]; p[k] = r[k]; }",
        "for (long k = 0; k < n; ++k) { r[k] = b[k]; p[k] = r[k]; }",
        [CH.test_cg_from_the_solution_takes_no_iteration]),
    "Z2 sign from bit 0 instead of bit 63": (
        "double re = (w[2 * k] >> 63) ? -s : s;", "double re = (w[2 * k] & 1) ? -s : s;",
        [lambda: P.test_z2_source(12120785, 0)]),
    "Z2 without the 1/sqrt2": (
        "double re = (w[2 * k] >> 63) ? -s : s;\n                double im = (w[2 * k + 1] >> 63) ? -s : s;",
        "double re = (w[2 * k] >> 63) ? -1.0 : 1.0;\n                double im = (w[2 * k + 1] >> 63) ? -1.0 : 1.0;",
        [lambda: P.test_z2_source(12120785, 0), P.test_z2_source_statistics]),
    "Z2 imaginary sign from the real part's word": (
        "double im = (w[2 * k + 1] >> 63) ? -s : s;", "double im = (w[2 * k] >> 63) ? -s : s;",
        [lambda: P.test_z2_source(3, 17)]),
    "point source on the last site": (
        "b[i * 12 + k] = (i == 0 && k == 0) ? 1.0 : 0.0;", "b[i * 12 + k] = (i == V - 1 && k == 0) ? 1.0 : 0.0;",
        [P.test_point_source]),
    "link update right-multiplies": (
        "mat_mul(E, &U[l * 9], &U[l * 9]);", "mat_mul(&U[l * 9], E, &U[l * 9]);",
        [P.test_update_links_is_left_multiplication_by_exp]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new, checks = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    path = O.compile_variant(SRC.replace(old, new), str(tmp_path / "liboracle_mutant.so"))
    real = O._load()
    O._lib = O.bind(path)
    try:
        caught = []
        for chk in checks:
            try:
                chk()
            except (AssertionError, ValueError, FloatingPointError):
                caught.append(chk)
        assert caught, f"no pin detected the planted mistake: {name}"
    finally:
        O._lib = real
