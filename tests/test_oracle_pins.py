"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against mathematics or an independent
implementation, never against a retyped copy of its own formula:

* Philox words: published known-answer vectors and numpy's Philox.
* Dirac basis: Clifford algebra, hermiticity, gamma5.
* Dslash / Wilson matrix: free-field momentum-space closed form with the
  antiperiodic time momenta, gamma5-hermiticity, adjointness of the dagger
  flag, gauge covariance under a random SU(3) transformation.
* Even/odd Schur operator: det M = det Mhat on a dense 4x2x2x4 lattice.
* Solvers: dense numpy solves.
* Plaquette and gauge action: unit gauge, gauge invariance, and the
  independent-link expectation u0(eps)^4 of the weak-field start.
* Forces: central finite differences of the actions along a random
  algebra direction, using scipy's expm for the link rotation.
* Exponential / reunitarisation: scipy expm, unitarity, det = 1.
* Integrator: reversibility and dH ~ eps^2.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from tests import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- RNG


def test_philox_known_answer_vectors():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) if not ln.startswith("#")]
    assert rows
    for r in rows:
        v = [int(h, 16) for h in r]
        out = O.philox(v[0:4], v[4:6])
        assert [int(w) for w in out] == v[6:10]


def test_philox_matches_numpy():
    g = np.random.default_rng(11)
    for _ in range(20):
        ctr = [int(c) for c in g.integers(0, 2**63, 4, dtype=np.uint64)]
        key = [int(c) for c in g.integers(0, 2**63, 2, dtype=np.uint64)]
        # numpy's Philox increments the counter before its first block
        bg = np.random.Philox(counter=[(ctr[0] - 1) % 2**64, ctr[1], ctr[2], ctr[3]], key=key)
        ref = [int(w) for w in bg.random_raw(4)]
        assert [int(w) for w in O.philox(ctr, key)] == ref


def test_site_words_counter_layout():
    # counter = (block, site, stream, epoch), key = (seed, 0)
    w = O.site_words(12120785, 37, 2, 5, 3)
    for b in range(3):
        assert [int(x) for x in w[4 * b:4 * b + 4]] == [int(x) for x in O.philox([b, 37, 2, 5], [12120785, 0])]


def test_u53_range_and_exactness():
    assert O.u53(0) == 2.0**-54
    assert O.u53(2**64 - 1) == 1.0 - 2.0**-54
    w = 0x123456789ABCDEF0
    assert O.u53(w) == ((w >> 11) + 0.5) / 2.0**53


def test_gaussian_moments():
    g = np.concatenate([O.site_gaussians(5, i, 1, 0, 32) for i in range(4000)])
    n = g.size
    assert abs(g.mean()) < 4 / np.sqrt(n)
    assert abs(g.var() - 1) < 4 * np.sqrt(2 / n)
    k = ((g - g.mean()) ** 4).mean() / g.var() ** 2
    assert abs(k - 3) < 4 * np.sqrt(24 / n)



def _numpy_site_words(seed, site, stream, epoch, nblocks):
    """Philox4x64-10 words of counter (block, site, stream, epoch), key
    (seed, 0), drawn from numpy's own Philox (independent of the oracle)."""
    out = []
    for blk in range(nblocks):
        # numpy increments its 256-bit counter before the first block
        c = (blk + (site << 64) + (stream << 128) + (epoch << 192) - 1) % 2**256
        ctr = np.array([(c >> (64 * j)) % 2**64 for j in range(4)], dtype=np.uint64)
        bg = np.random.Philox(counter=ctr, key=np.array([seed, 0], dtype=np.uint64))
        out.extend(int(w) for w in bg.random_raw(4))
    return out


@pytest.mark.parametrize("seed,epoch", [(12120785, 0), (3, 17)])
def test_z2_source(seed, epoch):
    """Z2 noise: each real component is +-1/sqrt2, the sign of component
    (spin, colour, re/im) at site i being bit 63 of Philox word
    (spin*3 + colour)*2 + re/im of that site (stream 4, epoch = source
    index).  The words come from numpy's Philox, the magnitude from the
    definition |b_k|^2 = 1."""
    L = [4, 2, 2, 4]
    b = O.source(L, O.Z2, seed, epoch)
    V = b.shape[0]
    comp = b.reshape(V, 12)
    # every component is (+-1 +- i)/sqrt2: unit modulus, |re| = |im|
    assert np.all(np.abs(comp.real) == np.abs(comp.imag))
    assert np.abs(np.abs(comp) ** 2 - 1).max() < 1e-15
    assert np.all(np.abs(comp.real) == 0.7071067811865476)
    for i in range(V):
        w = _numpy_site_words(seed, i, O.ST_SOURCE, epoch, 6)
        signs = np.array([-1.0 if (x >> 63) else 1.0 for x in w[:24]])
        assert np.array_equal(np.sign(comp[i].real), signs[0::2]), i
        assert np.array_equal(np.sign(comp[i].imag), signs[1::2]), i
    # a different epoch gives a different (independent) noise vector
    b2 = O.source(L, O.Z2, seed, epoch + 1)
    agree = np.mean(np.sign(b2.real) == np.sign(b.real))
    assert 0.35 < agree < 0.65


def test_z2_source_statistics():
    """Z2 noise has E[b] = 0 and E[b b^dag] = 1 between components."""
    L = [4, 4, 4, 4]
    b = O.source(L, O.Z2, 99, 0).reshape(-1)
    n = b.size
    assert abs(b.real.mean()) < 4 * np.sqrt(0.5 / n) and abs(b.imag.mean()) < 4 * np.sqrt(0.5 / n)
    assert abs(np.vdot(b, b).real / n - 1) < 1e-15
    off = np.vdot(b[:-1], b[1:]) / (n - 1)
    assert abs(off) < 4 / np.sqrt(n)


def test_point_source():
    """Point source: 1 at site 0, spin 0, colour 0; zero everywhere else,
    whatever the seed and epoch."""
    for L in ([4, 2, 2, 4], [2, 4, 6, 2]):
        for seed, epoch in [(1, 0), (12120785, 9)]:
            b = O.source(L, O.POINT, seed, epoch)
            ref = np.zeros_like(b)
            ref[0, 0, 0] = 1.0
            assert np.array_equal(b, ref)


# ------------------------------------------------------- Dirac algebra


def test_gamma_basis():
    g = O.gamma_matrices()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * (m == n) * np.eye(4), atol=0)
        for s in (+1, -1):
            assert np.linalg.matrix_rank(np.eye(4) + s * g[m]) == 2
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], np.diag([1, 1, -1, -1]), atol=0)


def test_algebra_generators():
    T = [O.algebra_matrix(np.eye(8)[a]) for a in range(8)]
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T, atol=1e-16)
        assert abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15
    # su(3) structure constants f_123 = 1, f_458 = sqrt(3)/2: [T1,T2] = i T3
    assert np.allclose(T[0] @ T[1] - T[1] @ T[0], 1j * T[2], atol=1e-15)
    assert np.allclose(T[3] @ T[4] - T[4] @ T[3], 1j * (0.5 * T[2] + np.sqrt(3) / 2 * T[7]), atol=1e-15)


# ------------------------------------------------------------ geometry


def test_neighbor_table_and_parity():
    L = [4, 6, 2, 8]
    nb = O.neighbor_table(L)
    par = O.parity_mask(L)
    V = synth.volume(L)
    for i in range(V):
        for mu in range(4):
            assert nb[nb[i, mu, 0], mu, 1] == i
            assert par[nb[i, mu, 0]] != par[i]
    c = synth.site_coords(L)
    assert np.array_equal(par, (c.sum(1) % 2).astype(bool))
    for i in (0, 1, 57, V - 1):
        assert O.lex_index(L, *c[i]) == i


# ------------------------------------------------------- Wilson matrix


def plane_wave(L, p, chi):
    c = synth.site_coords(L)
    ph = np.exp(1j * (c @ np.asarray(p)))
    return ph[:, None, None] * chi[None]


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (3, 5, 1, 7)])
def test_free_field_closed_form(n):
    L = [4, 6, 2, 8]
    kappa = 0.137
    p = [2 * np.pi * n[m] / L[m] for m in range(3)] + [(2 * n[3] + 1) * np.pi / L[3]]
    chi = synth.spinor(3, [1, 1, 1, 1])[0]
    psi = plane_wave(L, p, chi)
    g = O.gamma_matrices()
    Mp = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
    want = np.einsum("ab,ibc->iac", Mp, psi)
    got = O.wilson_m(L, O.unit_gauge(L), kappa, psi)
    assert np.abs(got - want).max() < 1e-14 * np.abs(want).max()
    # and the periodic time momentum is NOT an eigenvector (boundary sign matters)
    pp = p[:3] + [2 * np.pi * n[3] / L[3]]
    psi2 = plane_wave(L, pp, chi)
    Mp2 = (1 - 2 * kappa * np.sum(np.cos(pp))) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(pp[m]) for m in range(4))
    assert np.abs(O.wilson_m(L, O.unit_gauge(L), kappa, psi2) - np.einsum("ab,ibc->iac", Mp2, psi2)).max() > 1e-3


def test_gamma5_hermiticity_and_dagger():
    L = [4, 4, 2, 6]
    U = synth.gauge_field(1, L)
    x, y = synth.spinor(2, L), synth.spinor(3, L)
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    k = 0.155
    lhs = np.vdot(x, g5 * O.wilson_m(L, U, k, y))
    rhs = np.vdot(O.wilson_m(L, U, k, x), g5 * y)
    assert abs(lhs - rhs) < 1e-14 * abs(lhs)
    lhs = np.vdot(x, O.wilson_m(L, U, k, y, dagger=True))
    rhs = np.vdot(O.wilson_m(L, U, k, x), y)
    assert abs(lhs - rhs) < 1e-14 * abs(lhs)
    # D^dagger = gamma5 D gamma5 as an operator identity
    assert np.abs(O.dslash(L, U, y, dagger=True) - g5 * O.dslash(L, U, g5 * y)).max() < 1e-14


def transform_gauge(L, U, G):
    nb = O.neighbor_table(L)
    Gd = np.conj(np.swapaxes(G, -1, -2))
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = G @ U[:, mu] @ Gd[nb[:, mu, 0]]
    return Ug


def test_gauge_covariance():
    L = [4, 2, 4, 4]
    U = synth.gauge_field(4, L, eps=0.5)
    G = synth.gauge_transform(5, L)
    psi = synth.spinor(6, L)
    Ug = transform_gauge(L, U, G)
    psig = np.einsum("iab,isb->isa", G, psi)
    k = 0.15
    lhs = O.wilson_m(L, Ug, k, psig)
    rhs = np.einsum("iab,isb->isa", G, O.wilson_m(L, U, k, psi))
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(rhs).max()
    assert abs(np.vdot(psig, O.wilson_m(L, Ug, k, psig)) - np.vdot(psi, O.wilson_m(L, U, k, psi))) < 1e-12
    assert abs(O.plaquette(L, Ug) - O.plaquette(L, U)) < 1e-15


def dense(op, n_sites, mask=None):
    """Dense matrix of a linear map over spinors (restricted to mask sites)."""
    sites = np.arange(n_sites) if mask is None else np.nonzero(mask)[0]
    cols = []
    for i in sites:
        for k in range(12):
            e = np.zeros((n_sites, 4, 3), complex)
            e[i].flat[k] = 1
            cols.append(op(e)[sites].reshape(-1))
    return np.array(cols).T


def test_schur_determinant_and_solvers():
    L = [4, 2, 2, 4]
    V = synth.volume(L)
    U = synth.gauge_field(7, L, eps=0.6)
    k = 0.15
    odd = O.parity_mask(L)
    M = dense(lambda e: O.wilson_m(L, U, k, e), V)
    Mh = dense(lambda e: O.mhat(L, U, k, e), V, ~odd)
    Mhd = dense(lambda e: O.mhat(L, U, k, e, dagger=True), V, ~odd)
    s1, l1 = np.linalg.slogdet(M)
    s2, l2 = np.linalg.slogdet(Mh)
    assert abs(l1 - l2) < 1e-11 and abs(s1 - s2) < 1e-11
    assert np.abs(Mhd - Mh.conj().T).max() < 1e-14
    # CG on Mhat^dag Mhat against a dense solve
    b = synth.spinor(8, L, odd, 0)
    x, st = O.cg_mhat(L, U, k, b, tol=1e-13)
    assert st["status"] == 0 and st["true_rel_res"] < 1e-12
    xd = np.linalg.solve(Mh.conj().T @ Mh, b[~odd].reshape(-1))
    assert np.abs(x[~odd].reshape(-1) - xd).max() < 1e-11 * np.abs(xd).max()
    assert np.abs(x[odd]).max() == 0
    # Wilson solve through the Schur complement against a dense solve of M
    bf = synth.spinor(9, L)
    xw, st = O.wilson_solve(L, U, k, bf, tol=1e-12)
    assert st["status"] == 0 and st["true_rel_res"] < 1e-11
    xd = np.linalg.solve(M, bf.reshape(-1))
    assert np.abs(xw.reshape(-1) - xd).max() < 1e-10 * np.abs(xd).max()


def test_cg_nonconvergence_status():
    L = [4, 2, 2, 4]
    U = synth.gauge_field(7, L, eps=0.6)
    b = synth.spinor(8, L, O.parity_mask(L), 0)
    x, st = O.cg_mhat(L, U, 0.15, b, tol=1e-10, maxiter=1)
    assert st["status"] == -4 and st["iters"] == 1


def test_cg_fixed_iterations():
    L = [4, 2, 2, 4]
    U = synth.gauge_field(7, L, eps=0.6)
    b = synth.spinor(8, L, O.parity_mask(L), 0)
    x, st = O.cg_mhat(L, U, 0.15, b, fixed_iters=5)
    assert st["status"] == 0 and st["iters"] == 5


# -------------------------------------------------------- global sums


def test_reductions_exact_on_integers():
    L = [4, 4, 2, 2]
    a = synth.integer_spinor(1, L)
    b = synth.integer_spinor(2, L)
    assert O.norm2(a) == float(np.sum(np.abs(a) ** 2).round())
    ip = O.inner(a, b)
    want = np.sum(np.conj(a) * b)
    assert ip == complex(round(want.real), round(want.imag))
    f = np.abs(a.reshape(synth.volume(L), -1)) ** 2
    t = synth.site_coords(L)[:, 3]
    s = O.sum_multi(f, t, L[3])
    assert np.array_equal(s, np.array([f[t == k].sum() for k in range(L[3])]))


# ------------------------------------------------- plaquette and action


def test_plaquette_unit_gauge():
    L = [4, 4, 4, 4]
    assert O.plaquette(L, O.unit_gauge(L)) == 1.0
    assert O.gauge_action(L, O.unit_gauge(L), 5.6) == 0.0


def test_plaquette_single_abelian_link():
    # One link set to diag(e^{ia}, e^{-ia}, 1): it sits in 6 plaquettes,
    # each with Re Tr = 1 + 2 cos a; every other plaquette is 3.
    L = [4, 4, 2, 2]
    V = synth.volume(L)
    U = O.unit_gauge(L)
    a = 0.7
    U[5, 2] = np.diag([np.exp(1j * a), np.exp(-1j * a), 1.0])
    want = ((6 * V - 6) * 3 + 6 * (1 + 2 * np.cos(a))) / (18 * V)
    assert abs(O.plaquette(L, U) - want) < 1e-15


def test_weak_field_plaquette_expectation():
    # Independent links with E[U] = u0 * 1 give <plaquette> = u0^4;
    # u0 = E[Re Tr exp(i eps H)]/3 estimated with numpy Gaussians + expm.
    eps = 0.3
    L = [8, 8, 8, 8]
    U = O.weak_field(L, 4242, eps)
    g = np.random.default_rng(99)
    T = [O.algebra_matrix(np.eye(8)[a]) for a in range(8)]
    n = 20000
    om = g.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", om, np.array(T))
    tr = np.array([np.trace(sla.expm(1j * eps * h)).real / 3 for h in H])
    u0, du0 = tr.mean(), tr.std() / np.sqrt(n)
    want, dwant = u0**4, 4 * u0**3 * du0
    # per-plaquette spread from the sample itself
    P = O.plaquette(L, U)
    sigma_plaq = 0.05 / np.sqrt(6 * synth.volume(L))
    assert abs(P - want) < 4 * np.hypot(dwant, sigma_plaq) + 1e-4


def test_weak_field_links_are_su3():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 1, 0.5).reshape(-1, 3, 3)
    assert np.abs(U @ np.conj(np.swapaxes(U, 1, 2)) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


# ------------------------------------------------- exp and reunitarise


def test_exp_matches_scipy():
    g = np.random.default_rng(3)
    # Arguments up to the largest met in HMC (weak-field start eps=0.5);
    # a summed Taylor series loses about exp(|A|) ulps to cancellation.
    for scale in (0.02, 0.1, 0.3, 0.6):
        a = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
        h = 0.5 * (a + a.conj().T)
        h -= np.trace(h) / 3 * np.eye(3)
        A = 1j * scale * h
        E = O.mat_exp(A)
        bound = 8e-16 * np.exp(np.linalg.norm(A, 2))
        assert np.abs(E - sla.expm(A)).max() < bound
        assert np.abs(E @ E.conj().T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(E) - 1) < 1e-14


def test_reunit_projects_to_su3_and_fixes_su3():
    g = np.random.default_rng(4)
    u = synth.random_su3(g, 1)[0]
    assert np.abs(O.reunit(u) - u).max() < 1e-15
    v = O.reunit(u + 1e-3 * (g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))))
    assert np.abs(v @ v.conj().T - np.eye(3)).max() < 1e-15
    assert abs(np.linalg.det(v) - 1) < 1e-15


def test_update_links_is_left_multiplication_by_exp():
    L = [2, 2, 2, 2]
    U = synth.gauge_field(5, L)
    P = synth.hermitian_traceless(6, L)
    eps = 0.1
    U2 = O.update_links(L, U, P, eps)
    for i in range(synth.volume(L)):
        for mu in range(4):
            assert np.abs(U2[i, mu] - sla.expm(1j * eps * P[i, mu]) @ U[i, mu]).max() < 1e-14


# ------------------------------------------------------------- forces


def _rotate(U, P, h):
    E = np.array([sla.expm(1j * h * p) for p in P.reshape(-1, 3, 3)])
    return (E @ U.reshape(-1, 3, 3)).reshape(U.shape)


def _dS_predicted(P, F):
    return 2 * np.einsum("lab,lba->", P.reshape(-1, 3, 3), F.reshape(-1, 3, 3)).real


def test_gauge_force_finite_difference():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 7, 0.4)
    P = synth.hermitian_traceless(8, L)
    beta, h = 5.6, 1e-4
    fd = (O.gauge_action(L, _rotate(U, P, h), beta) - O.gauge_action(L, _rotate(U, P, -h), beta)) / (2 * h)
    pred = _dS_predicted(P, O.gauge_force(L, U, beta))
    assert abs(fd - pred) < 1e-6 * abs(pred)


def _force_vectors(L, U, k, Xe):
    odd = O.parity_mask(L)
    X = Xe.copy()
    X[odd] = O.dslash(L, U, Xe, 1)[odd]
    Y = O.mhat(L, U, k, Xe)
    Y[odd] = O.dslash(L, U, Y, 1, dagger=True)[odd]
    return X, Y


def test_fermion_force_finite_difference():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 7, 0.4)
    P = synth.hermitian_traceless(8, L)
    k, h = 0.15, 1e-4
    odd = O.parity_mask(L)
    phi = synth.spinor(9, L, odd, 0)

    def S_f(U):
        x, st = O.cg_mhat(L, U, k, phi, tol=1e-14)
        assert st["status"] == 0
        return O.inner(phi, x).real

    Xe, _ = O.cg_mhat(L, U, k, phi, tol=1e-14)
    X, Y = _force_vectors(L, U, k, Xe)
    F = O.fermion_force(L, U, k * k, X, Y)
    fd = (S_f(_rotate(U, P, h)) - S_f(_rotate(U, P, -h))) / (2 * h)
    pred = _dS_predicted(P, F)
    assert abs(fd - pred) < 1e-6 * abs(pred)
    Fm = F.reshape(-1, 3, 3)
    assert np.abs(Fm - np.conj(np.swapaxes(Fm, 1, 2))).max() < 1e-14
    assert np.abs(np.trace(Fm, axis1=1, axis2=2)).max() < 1e-13


def test_unpreconditioned_fermion_force_finite_difference():
    # Same routine with coef = kappa and X = (M^dag M)^-1 phi, Y = M X
    L = [4, 2, 2, 4]
    V = synth.volume(L)
    U = O.weak_field(L, 3, 0.4)
    P = synth.hermitian_traceless(4, L)
    k, h = 0.13, 1e-4
    phi = synth.spinor(5, L)

    def solve(U):
        M = dense(lambda e: O.wilson_m(L, U, k, e), V)
        return np.linalg.solve(M.conj().T @ M, phi.reshape(-1)).reshape(V, 4, 3)

    X = solve(U)
    Y = O.wilson_m(L, U, k, X)
    F = O.fermion_force(L, U, k, X, Y)
    S = lambda U: np.vdot(phi, solve(U)).real
    fd = (S(_rotate(U, P, h)) - S(_rotate(U, P, -h))) / (2 * h)
    assert abs(fd - _dS_predicted(P, F)) < 1e-6 * abs(fd)


def test_forces_gauge_covariant():
    L = [4, 2, 2, 4]
    U = O.weak_field(L, 11, 0.4)
    G = synth.gauge_transform(12, L)
    Ug = transform_gauge(L, U, G)
    Gd = np.conj(np.swapaxes(G, -1, -2))
    F = O.gauge_force(L, U, 5.6)
    Fg = O.gauge_force(L, Ug, 5.6)
    assert np.abs(Fg - G[:, None] @ F @ Gd[:, None]).max() < 1e-13


# ---------------------------------------------------------- integrator


@pytest.fixture(scope="module")
def c1_setup():
    L = [4, 4, 4, 4]
    U = O.weak_field(L, 12120785, 0.3)
    P = O.refresh_momenta(L, 12120785, 0)
    eta = O.eta(L, 12120785, 0, 0)
    phi = O.mhat(L, U, 0.15, eta, dagger=True)
    return L, U, P, eta, phi


def test_momenta_kinetic_expectation(c1_setup):
    L, U, P, eta, phi = c1_setup
    Pm = P.reshape(-1, 3, 3)
    assert np.abs(Pm - np.conj(np.swapaxes(Pm, 1, 2))).max() == 0
    assert np.abs(np.trace(Pm, axis1=1, axis2=2)).max() < 1e-15
    ke = O.kinetic(L, P) / Pm.shape[0]
    # Tr P^2 = sum_a omega_a^2 / 2 has mean 4 and variance 4 per link
    assert abs(ke - 4) < 4 * 2 / np.sqrt(Pm.shape[0])


def test_pseudofermion_variance(c1_setup):
    L, U, P, eta, phi = c1_setup
    odd = O.parity_mask(L)
    assert np.abs(eta[odd]).max() == 0
    v = np.abs(eta[~odd]) ** 2
    assert abs(v.mean() - 1) < 4 / np.sqrt(v.size)


def test_leapfrog_reversibility(c1_setup):
    L, U, P, eta, phi = c1_setup
    U1, P1, _, st = O.leapfrog(L, U, P, phi, 5.6, 0.15, 1.0, 10, tol=1e-14)
    assert st["solves"] == 11 and st["nonconverged"] == 0
    U2, P2, _, _ = O.leapfrog(L, U1, -P1, phi, 5.6, 0.15, 1.0, 10, tol=1e-14)
    assert np.linalg.norm(U2 - U) / np.linalg.norm(U) < 1e-12
    assert np.linalg.norm(P2 + P) / np.linalg.norm(P) < 1e-12


def test_dH_scales_as_eps_squared(c1_setup):
    L, U = c1_setup[0], c1_setup[1]
    dH = [O.hmc_trajectory(L, U, 5.6, 0.15, 12120785, 0, 1.0, n, tol=1e-14)[1]["dH"] for n in (10, 20, 40)]
    for a, b in zip(dH, dH[1:]):
        assert 0.2 < b / a < 0.3


def test_trajectory_bookkeeping(c1_setup):
    L, U = c1_setup[0], c1_setup[1]
    U1, r = O.hmc_trajectory(L, U, 5.6, 0.15, 12120785, 0, 1.0, 10)
    assert r["status"] == 0 and r["nonconverged"] == 0
    assert r["S_f_old"] == O.norm2(O.eta(L, 12120785, 0, 0))
    assert abs(r["dH"] - (r["H_new"] - r["H_old"])) < 1e-9
    assert r["u"] == O.accept_uniform(12120785, 0)
    acc = r["dH"] <= 0 or r["u"] < np.exp(-r["dH"])
    assert r["accepted"] == int(acc)
    if not acc:
        assert np.array_equal(U1, U)
    assert abs(r["plaquette"] - O.plaquette(L, U1)) == 0
    # the energies are those of the refreshed fields before and of the
    # integrated fields after the leapfrog (the assembly the full-size GPU
    # test repeats from these primitives)
    P0 = O.refresh_momenta(L, 12120785, 0)
    eta = O.eta(L, 12120785, 0, 0)
    phi = O.mhat(L, U, 0.15, eta, dagger=True)
    U2, P2, Xe, st = O.leapfrog(L, U, P0, phi, 5.6, 0.15, 1.0, 10)
    assert st["solves"] == 11 and st["iters_total"] == r["cg_iters_total"]
    assert r["H_old"] == O.kinetic(L, P0) + O.gauge_action(L, U, 5.6) + O.norm2(eta)
    assert r["H_new"] == O.kinetic(L, P2) + O.gauge_action(L, U2, 5.6) + O.inner(phi, Xe).real


def test_site_list_functions_match_full_lattice():
    """The site-list forms used for sampled checks at large volume agree
    bit for bit with the full-lattice functions pinned above."""
    L = (4, 6, 4, 6)
    V = synth.volume(L)
    sites = np.array([0, 5, 17, 100, V - 1], dtype=np.int64)
    U = synth.gauge_field(41, L, eps=0.6)
    psi = synth.spinor(42, L)
    full = O.dslash(L, U, psi, -1, 0)
    assert np.array_equal(O.dslash_sites(L, U, psi, sites), full[sites])
    fg = O.gauge_force(L, U, 5.6)
    assert np.array_equal(O.gauge_force_sites(L, U, 5.6, sites), fg[sites])
    chi = synth.spinor(43, L)
    ff = O.fermion_force(L, U, 0.02, psi, chi)
    assert np.array_equal(O.fermion_force_sites(L, U, 0.02, psi, chi, sites), ff[sites])
    Uw = np.zeros_like(U)
    O.weak_field_sites(L, 3, 0.3, sites, Uw)
    assert np.array_equal(Uw[sites], O.weak_field(L, 3, 0.3)[sites])
    b = np.zeros_like(psi)
    O.gauss_source_sites(7, 2, sites, b)
    assert np.array_equal(b[sites], O.source(L, 0, 7, 2)[sites])


def test_results_do_not_depend_on_thread_count():
    """The CPU baseline is timed at several thread counts: the oracle's
    results are bit-identical at each (site loops write disjoint outputs,
    global sums are serial)."""
    L = (4, 4, 4, 4)
    U = synth.gauge_field(5, L, eps=0.5)
    b = synth.spinor(6, L, O.parity_mask(L), 0)
    got = []
    prev = O.set_threads(0)
    try:
        for n in (1, 3):
            O.set_threads(n)
            x, st = O.cg_mhat(L, U, 0.15, b, tol=1e-10)
            assert st["status"] == 0
            got.append((O.plaquette(L, U), O.gauge_force(L, U, 5.6), x, st["iters"], O.dslash(L, U, b, -1, 0)))
    finally:
        O.set_threads(prev)
    for a, c in zip(got[0], got[1]):
        assert np.array_equal(a, c)
