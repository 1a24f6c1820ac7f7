"""GPU: Creutz's equality <exp(-dH)> = 1 over an equilibrated HMC chain.

It holds for an area-preserving, reversible integrator with the exact
Metropolis step whatever the step size, so a wrong force term, sign or
reunitarisation shows as a mean away from 1.  4^4, beta 5.6, kappa 0.15,
tau 0.5 with 20 steps: 100 trajectories from the weak-field start to
equilibrate, then 400 measured (seeded: the same chain every run)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEED = 424242


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def test_creutz_equality(H):
    L = (4, 4, 4, 4)
    F = H.Fields(L, 5.6, 0.15)
    H.hmc_weak_field_start(F, SEED, 0.3)
    prm = H.cg_params(tol=1e-12)
    for t in range(100):
        H.hmc_trajectory(F, SEED, t, 0.5, 20, prm)
    rs = [H.hmc_trajectory(F, SEED, t, 0.5, 20, prm) for t in range(100, 500)]
    assert all(r["status"] == 0 for r in rs)
    e = np.exp(-np.array([r["dH"] for r in rs]))
    mean, err = e.mean(), e.std(ddof=1) / np.sqrt(len(e))
    assert abs(mean - 1.0) < 4 * err, (mean, err)
    acc = np.mean([r["accepted"] for r in rs])
    assert 0.7 < acc <= 1.0
    # acceptance agrees with <min(1, exp(-dH))>
    assert abs(acc - np.minimum(1.0, e).mean()) < 0.06
