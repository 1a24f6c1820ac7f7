"""GPU: the tiled site orders of the one-site-per-work-item Dslash (whole
z-planes, and y-blocks of a few 64-site chunks).

Only the work-item that computes a site changes, not its arithmetic, so
every output equals the linear order's bit for bit; the partial sums of
the norm epilogues cover other site sets, so solves agree with the oracle
to their tolerance instead."""
import numpy as np
import pytest

import oracle as O
from tests import synth
from tests.test_gpu_parity import get_spinor, put_gauge, put_spinor, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# extents that admit the tiled order and that no other test uses (their
# table entries leave the other tests' lattices alone), with the (tiled
# order, workgroups per CU) pairs tried on each: 48 x 16 / 2 = 384 sites
# per z-plane = 6 chunks, so y-blocks of 2 and 3 chunks; 24 x 12 / 2 = 144
# sites per z-plane, not whole chunks, 1152 per t-slice: the walk over the
# chunks of the t-slices
ORDER_L = [(16, 8, 4, 8), (16, 16, 4, 16), (48, 16, 4, 8), (24, 12, 8, 16)]
ORDERS = {(48, 16, 4, 8): ((1, 2), (2, 2), (3, 2), (3, 0))}


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def set_order(H, path, L, order, occ=2):
    ext = " ".join(map(str, L))
    lines = ([f"dslash {ext} {p} 1 0" for p in range(4)] + [f"dslash_order {ext} {p} {order} 0" for p in range(4)] +
             [f"dslash_occupancy {ext} {p} {occ} 0" for p in range(4)])
    path.write_text("\n".join(lines) + "\n")
    H.hmc_tune_load(str(path))
    for p in range(4):
        assert H.hmc_tune_query(L, H.TUNE_DSLASH, p) == (1, True)
        assert H.hmc_tune_query(L, H.TUNE_DSLASH_ORDER, p) == (order, True)
        assert H.hmc_tune_query(L, H.TUNE_DSLASH_OCC, p) == (occ, True)


@pytest.mark.parametrize("L", ORDER_L)
def test_tiled_order_bit_identical_and_oracle(H, tmp_path, L):
    U = synth.gauge_field(61, L, eps=0.5)
    psi = synth.spinor(62, L)
    outs = {}
    orders = ORDERS.get(L, ((1, 2),))
    for order in ((0, 2),) + orders:
        set_order(H, tmp_path / f"o{order[0]}_{order[1]}.txt", L, *order)
        F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
        put_gauge(H, F, U)
        for prec in range(4):
            for par in (0, 1):
                for dag in (0, 1):
                    b = put_spinor(H, F, psi, 1 - par, prec=prec)
                    out = F.spinor(prec=prec)
                    H.hmc_wilson_dslash(F, out, b, par, dag, prec)
                    outs[(order, prec, par, dag)] = out.clone()
                    if prec == 0 and order[0] > 0:
                        want = O.dslash(L, U, psi, par, dag)
                        assert rel(get_spinor(H, F, out, par), want) < 1e-14
        del F
    for key in [k for k in outs if k[0] == (0, 2)]:
        for order in orders:
            assert torch.equal(outs[key], outs[(order,) + key[1:]]), (order, key)


@pytest.mark.parametrize("L", ORDER_L)
def test_tiled_order_solves(H, tmp_path, L):
    k = 0.15
    order = ORDERS.get(L, ((1, 2),))[-1]
    set_order(H, tmp_path / "o.txt", L, *order)
    F = H.Fields(L, 5.6, k, flags=H.FIELDS_LOWPREC)
    U = synth.gauge_field(63, L, eps=0.5)
    put_gauge(H, F, U)
    odd = O.parity_mask(L)
    b = synth.spinor(64, L, odd, 0)
    want, _ = O.cg_mhat(L, U, k, b, tol=1e-12)
    bb = put_spinor(H, F, b, 0)
    for prec in (0, 1, 2):
        x = F.spinor()
        st = H.hmc_cg_solve(F, x, bb, H.cg_params(tol=1e-10, prec=prec, maxiter=20000))
        assert st["status"] == 0 and st["true_rel_res"] <= 1e-10, prec
        assert rel(get_spinor(H, F, x, 0), want) < 1e-8, prec


# (lattice, site walk of the site-blocked staple force): 144 sites per
# parity = two whole chunks and a ragged one (linear walk); one chunk per
# z-plane (tiled, whole planes); six chunks per z-plane (y-blocks of two);
# z-planes not whole chunks (tiled, chunks of the t-slices)
GF_L = [(6, 4, 2, 6), (16, 8, 4, 8), (48, 16, 4, 8), (24, 12, 8, 16)]


@pytest.mark.parametrize("L", GF_L)
def test_staple_force_shapes(H, tmp_path, L):
    """Every staple-force shape and link form against the oracle, and the
    shapes against each other to rounding (the site-blocked shape takes a
    block's own links from LDS, the others from memory: the same values
    through differently scheduled arithmetic).  The plaquette sum walks the
    sites the same way."""
    from tests.test_gpu_parity import get_momenta, put_momenta
    ext = " ".join(map(str, L))
    P0 = synth.hermitian_traceless(81, L)
    for field, forms in (("su3", (10, 12)), ("u3", (18,))):
        U = synth.gauge_field(82, L, eps=0.6)
        if field == "u3":  # det != 1: all nine entries are read
            U = U * np.exp(1j * synth.rng(83).uniform(0.3, 2.5, size=U.shape[:-2]))[..., None, None]
        want = P0 - 0.05 * O.gauge_force(L, U, 5.7)
        want_plaq = O.plaquette(L, U)
        for form in forms:
            got = {}
            for shape in (0, 1, 2):
                path = tmp_path / f"gf_{field}_{form}_{shape}.txt"
                path.write_text(f"gauge_force {ext} 0 {shape} 0\n" +
                                (f"gauge_force_links {ext} 0 {form} 0\n" if form != 18 else ""))
                H.hmc_tune_load(str(path))
                assert H.hmc_tune_query(L, H.TUNE_GAUGE_FORCE) == (shape, True)
                F = H.Fields(L, 5.7, 0.15)
                put_gauge(H, F, U)
                assert H.hmc_links_two_row(F) == (field == "su3")
                put_momenta(H, F, P0)
                H.hmc_gauge_force(F, 0.05)
                got[shape] = get_momenta(H, F)
                assert rel(got[shape], want) < 1e-13, (field, form, shape)
                assert abs(H.hmc_plaquette(F) - want_plaq) < 1e-13, (field, form)
                del F
            assert rel(got[2], got[0]) < 1e-15, (field, form)


@pytest.mark.parametrize("L", GF_L)
def test_fermion_force_walk(H, L):
    """The fermion force in the site-blocked walk (linear with a ragged
    chunk, tiled by whole planes, tiled by y-blocks) against the oracle."""
    from tests.test_gpu_parity import get_momenta, put_momenta
    k = 0.13
    U = synth.gauge_field(91, L, eps=0.6)
    odd = O.parity_mask(L)
    Xe, Ye = synth.spinor(92, L, odd, 0), synth.spinor(93, L, odd, 0)
    P = synth.hermitian_traceless(94, L)
    X, Y = Xe.copy(), Ye.copy()
    X[odd] = O.dslash(L, U, Xe, 1)[odd]
    Y[odd] = O.dslash(L, U, Ye, 1, dagger=True)[odd]
    want = P - 0.37 * O.fermion_force(L, U, k ** 2, X, Y)
    F = H.Fields(L, 5.6, 0.15)
    put_gauge(H, F, U)
    put_momenta(H, F, P)
    H.hmc_fermion_force_bilinear(F, put_spinor(H, F, Xe, 0), put_spinor(H, F, Ye, 0), k, 0.37)
    assert rel(get_momenta(H, F), want) < 1e-13
