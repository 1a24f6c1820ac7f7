"""GPU: the link-load forms of the hopping and staple kernels.

On SU(3) fields the kernels read a compact form of each link: rows 0 and 1
(row 2 rebuilt as conj(row0 x row1)), or row 0 and column 2 (u10, u11 from
orthogonality and det = 1, exact reads where |u02| is close to 1), with or
without non-temporal hints on those loads and the output stores; on any
other field they read all nine entries.  Every form must reproduce the
oracle, and the library must use a compact form only when every link is
SU(3) to rounding.
"""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_gpu_parity import SMALL, get_spinor, put_gauge, put_spinor, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def u3_field(seed, L):
    """Unitary links with det != 1 (a random U(1) phase per link): the
    third row is not conj(row0 x row1)."""
    U = synth.gauge_field(seed, L, eps=0.5)
    phi = synth.rng(seed + 1000).uniform(0.3, 2.5, size=U.shape[:-2])
    return U * np.exp(1j * phi)[..., None, None]


def test_two_row_flag_follows_the_field(H):
    L = (4, 4, 4, 4)
    F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
    assert not H.hmc_links_two_row(F)  # fresh arena: unknown contents
    put_gauge(H, F, synth.gauge_field(3, L))
    assert H.hmc_links_two_row(F)
    F.pointer(H.FIELD_GAUGE)  # the caller may now write U in place
    assert not H.hmc_links_two_row(F)
    H.hmc_sync_lowprec(F)
    assert H.hmc_links_two_row(F)
    put_gauge(H, F, u3_field(4, L))
    assert not H.hmc_links_two_row(F)
    H.hmc_refresh(F, 1, 0, H.REFRESH_MOM)
    H.hmc_exp_update_reunit(F, 0.1)  # reunitarised: SU(3) again
    assert H.hmc_links_two_row(F)
    put_gauge(H, F, u3_field(5, L))
    H.hmc_weak_field_start(F, 2, 0.3)
    assert H.hmc_links_two_row(F)
    # one perturbed third-row entry above the 1e-14 threshold
    U = synth.gauge_field(6, L)
    U[17, 2, 2, 1] += 1e-12
    put_gauge(H, F, U)
    assert not H.hmc_links_two_row(F)
    # third row = conj(row0 x row1) but rows 0, 1 not orthonormal
    U = synth.gauge_field(7, L)
    U[5, 1, 0, :] *= 1.0 + 1e-12
    U[5, 1, 2, :] = np.conj(np.cross(U[5, 1, 0, :], U[5, 1, 1, :]))
    put_gauge(H, F, U)
    assert not H.hmc_links_two_row(F)


@pytest.mark.parametrize("L", SMALL)
def test_full_link_path_matches_oracle(H, L):
    k = 0.15
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = u3_field(21, L)
    put_gauge(H, F, U)
    assert not H.hmc_links_two_row(F)
    psi = synth.spinor(22, L)
    for dag in (0, 1):
        for par in (0, 1):
            b = put_spinor(H, F, psi, 1 - par)
            out = F.spinor()
            H.hmc_wilson_dslash(F, out, b, par, dag)
            assert rel(get_spinor(H, F, out, par), O.dslash(L, U, psi, par, dag)) < 1e-14
    b = put_spinor(H, F, psi, 0)
    out = F.spinor()
    H.hmc_mhat(F, out, b, 1)
    assert rel(get_spinor(H, F, out, 0), O.mhat(L, U, k, psi, 1)) < 1e-14
    for prec, tol in ((1, 1e-6), (2, 3e-3), (3, 2e-2)):
        bl = put_spinor(H, F, psi, 1, prec=prec)
        ol = F.spinor(prec=prec)
        H.hmc_wilson_dslash(F, ol, bl, 0, 0, prec)
        assert rel(get_spinor(H, F, ol, 0, prec=prec), O.dslash(L, U, psi, 0, 0)) < tol


@pytest.mark.parametrize("L", SMALL)
def test_two_row_and_full_forms_agree(H, L):
    """The same SU(3) field through both forms (the full form forced by
    fetching the gauge pointer): FP64 results within rounding of each other
    and of the oracle."""
    F = H.Fields(L, 5.6, 0.15)
    U = synth.gauge_field(31, L, eps=0.7)
    put_gauge(H, F, U)
    psi = synth.spinor(32, L)
    b = put_spinor(H, F, psi, 1)
    outs = []
    for two_row in (True, False):
        if not two_row:
            F.pointer(H.FIELD_GAUGE)
        assert H.hmc_links_two_row(F) == two_row
        out = F.spinor()
        H.hmc_wilson_dslash(F, out, b, 0, 1)
        outs.append(get_spinor(H, F, out, 0))
    want = O.dslash(L, U, psi, 0, 1)
    assert rel(outs[0], want) < 1e-14 and rel(outs[1], want) < 1e-14
    assert rel(outs[0], outs[1]) < 1e-14


# Extents used by no other test: the table entries that select the form
# for them leave every other test's lattice alone.
FORM_L = [(6, 4, 4, 8), (8, 6, 4, 6)]


def set_forms(H, path, L, hop, staple, stream):
    ext = " ".join(map(str, L))
    lines = ([f"dslash_links {ext} {p} {hop} 0" for p in range(4)] +
             [f"dslash_stream {ext} {p} {stream} 0" for p in range(4)] + [f"gauge_force_links {ext} 0 {staple} 0"])
    path.write_text("\n".join(lines) + "\n")
    H.hmc_tune_load(str(path))
    for p in range(4):
        assert H.hmc_tune_query(L, H.TUNE_DSLASH_LINKS, p) == (hop, True)
        assert H.hmc_tune_query(L, H.TUNE_DSLASH_STREAM, p) == (stream, True)
    assert H.hmc_tune_query(L, H.TUNE_GAUGE_FORCE_LINKS) == (staple, True)


def permuted_field(seed, L):
    """SU(3) links C V, V near the identity, C the cyclic permutation
    (det 1): |u02| is close to 1 on every link, and about half of them have
    |u02|^2 > 15/16, where the row-0 / column-2 form reads u10, u11 instead
    of solving for them; most wavefronts take both branches."""
    C = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], dtype=complex)
    return C @ synth.gauge_field(seed, L, eps=0.2)


FIELDS = {"haar": lambda L: synth.gauge_field(41, L),
          "weak": lambda L: O.weak_field(L, 42, 0.3),
          "permuted": lambda L: permuted_field(43, L)}


@pytest.mark.parametrize("field", sorted(FIELDS))
@pytest.mark.parametrize("L", FORM_L)
def test_compact_forms_match_oracle(H, tmp_path, L, field):
    from tests.test_gpu_parity import get_momenta, put_momenta
    k, beta = 0.15, 5.6
    U = FIELDS[field](L)
    if field == "permuted":
        assert 0.2 < np.mean(np.abs(U[..., 0, 2]) ** 2 > 15 / 16) < 0.8
    psi = synth.spinor(44, L)
    odd = O.parity_mask(L)
    Xe, Ye = synth.spinor(45, L, odd, 0), synth.spinor(46, L, odd, 0)
    P = synth.hermitian_traceless(47, L)
    want_ds = {(par, dag): O.dslash(L, U, psi, par, dag) for par in (0, 1) for dag in (0, 1)}
    X, Y = Xe.copy(), Ye.copy()
    X[odd] = O.dslash(L, U, Xe, 1)[odd]
    Y[odd] = O.dslash(L, U, Ye, 1, dagger=True)[odd]
    want_ff = P - 0.37 * O.fermion_force(L, U, 0.13 ** 2, X, Y)
    want_gf = P - 0.3 * O.gauge_force(L, U, beta)
    want_plaq = O.plaquette(L, U)
    # (hop form, staple form, streamed hop kernels)
    for hop, staple, stream in ((12, 10, 0), (10, 12, 1), (12, 12, 1), (10, 10, 0)):
        set_forms(H, tmp_path / f"f{hop}_{staple}_{stream}.txt", L, hop, staple, stream)
        F = H.Fields(L, beta, k, flags=H.FIELDS_LOWPREC)
        put_gauge(H, F, U)
        assert H.hmc_links_two_row(F)
        for (par, dag), want in want_ds.items():
            b = put_spinor(H, F, psi, 1 - par)
            out = F.spinor()
            H.hmc_wilson_dslash(F, out, b, par, dag)
            assert rel(get_spinor(H, F, out, par), want) < 1e-14, (hop, stream, par, dag)
        for prec, tol in ((1, 1e-6), (2, 3e-3), (3, 2e-2)):
            bl = put_spinor(H, F, psi, 1, prec=prec)
            ol = F.spinor(prec=prec)
            H.hmc_wilson_dslash(F, ol, bl, 0, 0, prec)
            assert rel(get_spinor(H, F, ol, 0, prec=prec), want_ds[(0, 0)]) < tol, (hop, stream, prec)
        put_momenta(H, F, P)
        H.hmc_fermion_force_bilinear(F, put_spinor(H, F, Xe, 0), put_spinor(H, F, Ye, 0), 0.13, 0.37)
        assert rel(get_momenta(H, F), want_ff) < 1e-13, hop
        put_momenta(H, F, P)
        H.hmc_gauge_force(F, 0.3)
        assert rel(get_momenta(H, F), want_gf) < 1e-13, staple
        assert abs(H.hmc_plaquette(F) - want_plaq) < 1e-13, staple
        del F


@pytest.mark.parametrize("L", SMALL)
def test_exp_update_reads_follow_the_field(H, L):
    """exp(i eps P) U with reunitarisation reads rows 0 and 1 of SU(3) links
    (row 2 rebuilt) and all nine entries of any other link; both against the
    oracle."""
    from tests.test_gpu_parity import get_gauge, put_momenta
    P = synth.hermitian_traceless(51, L, scale=2.0)
    for U, su3 in ((synth.gauge_field(52, L, eps=0.7), True), (u3_field(53, L), False)):
        F = H.Fields(L, 5.6, 0.15)
        put_gauge(H, F, U)
        assert H.hmc_links_two_row(F) == su3
        put_momenta(H, F, P)
        H.hmc_exp_update_reunit(F, 0.1)
        assert rel(get_gauge(H, F), O.update_links(L, U, P, 0.1)) < 1e-14, su3
        assert H.hmc_links_two_row(F)
        del F
