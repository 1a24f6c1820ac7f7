"""GPU: the two link-load forms of the hopping kernels.

On SU(3) fields the kernels read rows 0 and 1 of each link and rebuild row 2
as conj(row0 x row1); on any other field they read all nine entries.  Both
must reproduce the oracle's Wilson operator, and the library must pick the
two-row form only when every stored third row equals the rebuilt one.
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
