"""GPU: the kernel-timing facility behind the benchmark's roofline figure.

With every launch sampled, a fused CG solve of n iterations is timed as n
groups of four Dslash launches; the algorithmic bytes per Dslash launch lie
between the plain hop's and the CG-epilogue hop's, and exceed the bytes as
implemented by the compact links' saving; the probe's empty
kernels are timed under "other"; disabled sampling records nothing."""
import os

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
    """The timed launches are those issued directly (a chunk replayed from
    its recording takes no events); HMC_SOLVER_GRAPHS=0 issues all of them
    directly."""
    os.environ["HMC_SOLVER_GRAPHS"] = "0"
    yield
    os.environ.pop("HMC_SOLVER_GRAPHS", None)


def test_cg_iterations_timed_in_groups(H, direct):
    L = (8, 8, 8, 16)   # two-row links by the built-in rule at this volume
    F = H.Fields(L, 5.6, 0.15)
    H.hmc_weak_field_start(F, 5, 0.3)
    Vh = L[0] * L[1] * L[2] * L[3] // 2
    b = F.spinor()
    src = F.spinor(full=True)
    H.hmc_make_source(F, src, 0, 3, 0)
    b.copy_(src[H.hmc_field_bytes(L, H.F64, H.KIND_HALF_SPINOR):])
    x = F.spinor()
    prm = H.cg_params(tol=1e-30, fixed_iters=12)
    H.hmc_cg_solve(F, x, b, prm)  # warm-up
    torch.cuda.synchronize()
    H.hmc_timing_reset()
    H.hmc_timing_enable(1)
    H.hmc_cg_solve(F, x, b, prm)
    torch.cuda.synchronize()
    t = H.hmc_timing_read()
    H.hmc_timing_enable(0)
    ds = t["dslash"]
    # 12 iterations of four hops, plus the set-up and final-residual hops
    assert ds["launches"] >= 4 * 12
    assert ds["calls"] == ds["launches"]  # every launch sampled
    # algorithmic bytes count whole links (144 B); the bytes as implemented
    # count the two stored rows (96 B); spinors 192 B: in + out, + y, + r
    per_site = ds["bytes"] / ds["launches"] / Vh
    assert 8 * 144 + 2 * 192 <= per_site <= 8 * 144 + 4 * 192
    moved = ds["bytes_moved"] / ds["launches"] / Vh
    assert abs((per_site - moved) - 8 * (144 - 96)) < 1e-9
    # the p-update: x read + written, p read + written, r read (5 x 192 B per site)
    cg = t["cg_blas"]
    assert cg["launches"] == 12 and cg["bytes"] == cg["bytes_moved"] == 12 * 5 * 192 * Vh
    assert ds["total_ms"] > 0
    H.hmc_timing_reset()
    H.hmc_timing_enable(0)
    H.hmc_cg_solve(F, x, b, prm)
    torch.cuda.synchronize()
    assert "dslash" not in H.hmc_timing_read()
    # every 5th sample: all launches still counted, a fifth of the groups timed
    H.hmc_timing_reset()
    H.hmc_timing_enable(5)
    H.hmc_cg_solve(F, x, b, prm)
    torch.cuda.synchronize()
    ds5 = H.hmc_timing_read()["dslash"]
    H.hmc_timing_enable(0)
    H.hmc_timing_reset()
    assert ds5["calls"] == ds["calls"] and 0 < ds5["launches"] < ds["launches"]
    # replayed recordings: every launch still counted; every second chunk
    # runs directly with all its launches timed
    os.environ["HMC_SOLVER_GRAPHS"] = "strict"
    H.hmc_timing_reset()
    H.hmc_timing_enable(2)
    H.hmc_cg_solve(F, x, b, prm)
    torch.cuda.synchronize()
    dsg = H.hmc_timing_read()["dslash"]
    H.hmc_timing_enable(0)
    H.hmc_timing_reset()
    assert dsg["calls"] == ds["calls"] and 0 < dsg["launches"] < ds["launches"]


def test_probe(H):
    H.hmc_timing_reset()
    H.hmc_timing_enable(1)
    H.hmc_timing_probe(16)
    torch.cuda.synchronize()
    t = H.hmc_timing_read()["other"]
    H.hmc_timing_enable(0)
    H.hmc_timing_reset()
    assert t["launches"] == 16 and t["total_ms"] > 0 and t["bytes"] == 0
