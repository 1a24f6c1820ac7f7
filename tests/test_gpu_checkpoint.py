"""GPU: checkpoint and resume of an HMC chain.  Trajectory k draws its
momenta, pseudofermion noise and Metropolis uniform from the counter-based
generator keyed by (seed, k) (Sec. 1 random number generator), so the chain
state is the gauge field and the next trajectory number: a chain resumed
from a checkpoint repeats the uninterrupted one bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEED, BETA, KAPPA = 12120785, 5.6, 0.15


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def gauge(H, F):
    c = H.canon_gauge_zeros(F.L)
    H.hmc_export_gauge(F, c)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("seed", [4, SEED])
def test_resumed_chain_repeats_the_uninterrupted_one(H, tmp_path, seed):
    # a fine integration (eps 0.01) that accepts on 4^4, so the chain moves
    L, tau, nsteps = (4, 4, 4, 4), 0.2, 20
    prm = H.cg_params(tol=1e-10)
    F = H.Fields(L, BETA, KAPPA)
    H.hmc_weak_field_start(F, seed, 0.3)
    U_start = gauge(H, F)
    full = [H.hmc_trajectory(F, seed, k, tau, nsteps, prm) for k in range(4)]
    U_full = gauge(H, F)
    assert not np.array_equal(U_full, U_start)

    F1 = H.Fields(L, BETA, KAPPA)
    H.hmc_weak_field_start(F1, seed, 0.3)
    for k in range(2):
        H.hmc_trajectory(F1, seed, k, tau, nsteps, prm)
    path = tmp_path / "chain.npz"
    H.save_checkpoint(F1, path, seed, 2)
    del F1

    F2 = H.Fields(L, 1.0, 0.1)  # action taken from the checkpoint
    meta = H.load_checkpoint(F2, path)
    assert meta["next_traj"] == 2 and meta["seed"] == seed and (F2.beta, F2.kappa) == (BETA, KAPPA)
    resumed = [H.hmc_trajectory(F2, meta["seed"], k, tau, nsteps, prm) for k in range(meta["next_traj"], 4)]
    for a, b in zip(full[2:], resumed):
        assert a["dH"] == b["dH"] and a["accepted"] == b["accepted"] and a["cg_iters_total"] == b["cg_iters_total"]
    assert np.array_equal(gauge(H, F2).view(np.uint64), U_full.view(np.uint64))


def test_checkpoint_of_another_lattice_is_refused(H, tmp_path):
    F = H.Fields((4, 4, 4, 4), BETA, KAPPA)
    H.hmc_weak_field_start(F, SEED, 0.3)
    path = tmp_path / "c.npz"
    H.save_checkpoint(F, path, SEED, 0)
    G = H.Fields((4, 4, 4, 6), BETA, KAPPA)
    with pytest.raises(ValueError):
        H.load_checkpoint(G, path)
