"""GPU: solver chunks replayed from HIP-graph recordings give bit for bit the
results of the same launches issued directly (HMC_SOLVER_GRAPHS=0), on
every replay, with other device work and synchronisations in between; the
device-driven reliable updates of mixed precision included."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


@pytest.fixture
def direct():
    """Direct launches (on) or recordings that must succeed (off); the
    library reads the switch per chunk."""
    def set_direct(on):
        os.environ["HMC_SOLVER_GRAPHS"] = "0" if on else "strict"
    yield set_direct
    os.environ.pop("HMC_SOLVER_GRAPHS", None)


def source(H, F, seed, full):
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, H.SOURCE_GAUSS, seed, 0)
    if full:
        return b
    return b[: H.hmc_field_bytes(F.L, H.F64, H.KIND_HALF_SPINOR)].clone()


def solve(H, F, b, prm, full):
    x = F.spinor(full=full)
    st = H.hmc_cg_solve(F, x, b, prm)
    torch.cuda.synchronize()
    return x, st


CASES = [  # lattice, mode, storage, fixed iterations, reliable-update delta (0: default)
    ((8, 6, 6, 10), 0, 0, 37, 0),        # FP64 CG, a length that takes every power of two
    ((8, 6, 6, 10), 0, 0, 0, 0),         # FP64 CG to 1e-10
    ((16, 16, 16, 32), 0, 0, 0, 0),      # the HMC force solve's shape
    ((8, 6, 6, 10), 1, 0, 0, 0),         # FP64 CGLS (Wilson solve)
    ((8, 6, 6, 10), 0, 1, 0, 0),         # mixed FP32 CG with device reliable updates
    ((16, 16, 16, 32), 0, 1, 0, 0),
    ((16, 16, 16, 32), 1, 2, 0, 0),      # mixed FP16 CGLS
    ((8, 8, 8, 8), 1, 3, 0, 0),          # mixed BF16 CGLS
    ((16, 16, 16, 32), 0, 3, 0, 0.01),   # BF16 CG whose updates restart the search direction
]


@pytest.mark.parametrize("L,mode,prec,fixed,delta", CASES)
def test_recorded_chunks_match_direct_launches(H, direct, L, mode, prec, fixed, delta):
    F = H.Fields(L, 5.6, 0.156, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 7, 0.4)
    full = mode == H.CG_WILSON_SOLVE
    b = source(H, F, 3, full)
    prm = H.cg_params(tol=1e-10, mode=mode, prec=prec, fixed_iters=fixed, maxiter=20000, reliable_delta=delta)
    direct(True)
    x0, s0 = solve(H, F, b, prm, full)
    direct(False)
    scratch = F.spinor()
    for rep in range(3):
        x1, s1 = solve(H, F, b, prm, full)
        assert s1["iters"] == s0["iters"] and s1["reliable_updates"] == s0["reliable_updates"], (rep, s0, s1)
        assert torch.equal(x1, x0), rep
        assert s1["true_rel_res"] == s0["true_rel_res"]
        # eager work and a synchronisation between replays
        H.hmc_wilson_dslash(F, scratch, b[: scratch.numel()], 0, 0)
        torch.cuda.synchronize()
    if fixed:
        assert s0["iters"] == fixed
    else:
        assert s0["true_rel_res"] <= 1e-10


def test_recorded_trajectory_matches_direct(H, direct):
    L = (4, 4, 4, 4)
    res = []
    for on in (True, False, False):
        direct(on)
        F = H.Fields(L, 5.6, 0.15)
        H.hmc_weak_field_start(F, 12120785, 0.3)
        r = H.hmc_trajectory(F, 12120785, 0, 1.0, 10, H.cg_params(tol=1e-10))
        c = H.canon_gauge_zeros(L)
        H.hmc_export_gauge(F, c)
        torch.cuda.synchronize()
        res.append((r, c.cpu().numpy()))
    for r, U in res[1:]:
        assert r["dH"] == res[0][0]["dH"] and r["cg_iters_total"] == res[0][0]["cg_iters_total"]
        assert np.array_equal(U, res[0][1])
