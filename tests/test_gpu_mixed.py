"""GPU: robustness of the mixed-precision solves (inner iteration in FP32 /
FP16 / BF16 storage with FP64 reliable updates, after Clark et al. 2010, the
single-precision production mode of Sec. 7).

* Small reliable-update deltas with the 8-bit-mantissa BF16 storage: the
  recursion drifts from the FP64 residual between updates, and keeping the
  search direction across an update then makes the iteration diverge (it
  did, to a non-finite residual, at delta 0.01 and 0.003 on the HMC force
  solve's configuration).  The update restarts the search direction in that
  case; every such solve now converges to the FP64 tolerance and agrees with
  the FP64 solve.
* FP16 storage of a field that spreads from a point source: the per-site
  scales of the spreading front shrink by ~1e-8 per hop and reached the
  float denormals within four operator applications, whose reciprocal
  overflowed (non-finite residual after three iterations at 12^3x24 and
  16^3x32).  Such sites are now stored as zero; the solves converge.
* The iteration limit is exact: the iteration that reaches maxiter asks for
  the last reliable update, which ends the solve with HMC_E_NOCONV after
  exactly maxiter iterations (it ran up to one update cycle past it).
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = (16, 16, 16, 32)  # the HMC force solve's lattice and start
SEED, EPS, KAPPA = 12120785, 0.3, 0.156


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


@pytest.fixture(scope="module")
def setup(H):
    F = H.Fields(L, 5.6, KAPPA, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, SEED, EPS)
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, H.SOURCE_GAUSS, 5, 0)
    be = b[: H.hmc_field_bytes(L, H.F64, H.KIND_HALF_SPINOR)].clone()
    ref = {}
    for mode in (H.CG_NORMAL_MHAT, H.CG_WILSON_SOLVE):
        x = F.spinor(full=mode == H.CG_WILSON_SOLVE)
        st = H.hmc_cg_solve(F, x, be if mode == H.CG_NORMAL_MHAT else b, H.cg_params(tol=1e-12, mode=mode))
        assert st["status"] == 0
        ref[mode] = x.view(torch.float64).clone()
    return F, {H.CG_NORMAL_MHAT: be, H.CG_WILSON_SOLVE: b}, ref


def rel(a, b):
    return ((a - b).norm() / b.norm()).item()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("delta", [0.01, 0.003])
def test_small_delta_low_storage_converges(H, setup, mode, prec, delta):
    F, rhs, ref = setup
    x = F.spinor(full=mode == H.CG_WILSON_SOLVE)
    st = H.hmc_cg_solve(F, x, rhs[mode], H.cg_params(tol=1e-10, mode=mode, prec=prec, reliable_delta=delta,
                                                     maxiter=3000), allow_noconv=True)
    assert st["status"] == 0, st
    assert st["true_rel_res"] <= 1e-10
    assert st["iters"] < 400  # restarted cycles, not a run to the limit
    # both meet |b - A x| <= 1e-10 |b| (the reference 1e-12); the solutions
    # agree to the condition number times that
    assert rel(x.view(torch.float64), ref[mode]) < 1e-7


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("maxiter", [1, 7, 20])
def test_iteration_limit_is_exact(H, setup, mode, prec, maxiter):
    F, rhs, _ = setup
    x = F.spinor(full=mode == H.CG_WILSON_SOLVE)
    st = H.hmc_cg_solve(F, x, rhs[mode], H.cg_params(tol=1e-10, mode=mode, prec=prec, maxiter=maxiter),
                        allow_noconv=True)
    assert st["status"] == H.HMC_E_NOCONV
    assert st["iters"] == maxiter
    assert st["reliable_updates"] >= 1
    # the reported residual is the FP64 one of the last update
    assert 0 < st["true_rel_res"] < 1 and abs(st["true_rel_res"] / st["rel_res"] - 1) < 1e-6


def test_default_delta_keeps_the_search_direction(H, setup):
    """At the default delta (0.01 for FP32 storage) the FP32 recursion
    tracks the FP64 residual: no update restarts the search direction, so
    the mixed solve takes the FP64 solve's iteration count (43 here) with
    about one update per hundredfold decrease of |r|."""
    F, rhs, _ = setup
    x64 = F.spinor()
    s64 = H.hmc_cg_solve(F, x64, rhs[0], H.cg_params(tol=1e-10))
    x = F.spinor()
    st = H.hmc_cg_solve(F, x, rhs[0], H.cg_params(tol=1e-10, prec=H.F32))
    assert st["status"] == 0 and st["iters"] == s64["iters"]
    assert st["reliable_updates"] <= s64["iters"] // 4


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("L", [(12, 12, 12, 24), (16, 16, 16, 32)])
def test_fp16_point_source_converges(H, mode, L):
    F = H.Fields(L, 5.6, 0.156, flags=H.FIELDS_LOWPREC)
    H.hmc_weak_field_start(F, 32, 0.45)
    b = F.spinor(full=True)
    H.hmc_make_source(F, b, H.SOURCE_POINT, 0, 0)
    rhs = b if mode == H.CG_WILSON_SOLVE else b[: H.hmc_field_bytes(L, H.F64, H.KIND_HALF_SPINOR)].clone()
    x = F.spinor(full=mode == H.CG_WILSON_SOLVE)
    st = H.hmc_cg_solve(F, x, rhs, H.cg_params(tol=1e-10, mode=mode, prec=H.F16, maxiter=3000), allow_noconv=True)
    assert st["status"] == 0 and st["true_rel_res"] <= 1e-10, st
    x64 = F.spinor(full=mode == H.CG_WILSON_SOLVE)
    s64 = H.hmc_cg_solve(F, x64, rhs, H.cg_params(tol=1e-12, mode=mode))
    assert s64["status"] == 0
    assert rel(x.view(torch.float64), x64.view(torch.float64)) < 1e-7


def test_fp16_storage_flushes_denormal_sites_and_keeps_nonfinite_ones(H):
    L = (4, 4, 4, 4)
    Vh = 128
    F = H.Fields(L, 5.6, 0.15, flags=H.FIELDS_LOWPREC)
    x = F.spinor()
    v = x.view(torch.float64)
    v.normal_(generator=torch.Generator(device="cuda").manual_seed(5))
    comp = lambda k, s: 2 * (k * Vh + s)  # real part of component k of site s (component-major)
    v[comp(0, 5)] = float("nan")
    for k in range(12):  # site 7: every component 1e-40 (a float denormal)
        v[comp(k, 7)] = 1e-40
        v[comp(k, 7) + 1] = 1e-40
    h = F.spinor(prec=H.F16)
    H.hmc_convert_spinor(F, h, H.F16, x, H.F64)
    back = F.spinor()
    H.hmc_convert_spinor(F, back, H.F64, h, H.F16)
    torch.cuda.synchronize()
    b = back.view(torch.float64)
    assert torch.isnan(b[comp(0, 5)])                      # a non-finite site stays non-finite
    assert all(b[comp(k, 7) + i] == 0 for k in range(12) for i in (0, 1))  # the denormal site is zero
    other = [s for s in range(Vh) if s not in (5, 7)]
    idx = torch.tensor([comp(k, s) + i for s in other for k in range(12) for i in (0, 1)], device="cuda")
    assert torch.isfinite(b[idx]).all()
    assert ((b[idx] - v[idx]).abs() <= 1e-3 * v[idx].abs().max()).all()  # half precision of the site scale
