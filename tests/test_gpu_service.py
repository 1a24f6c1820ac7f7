"""GPU tests of the solve service (continuous batching of Wilson solves).

Each request solves M x = b on its own weak-field gauge field; the service
result must meet the FP64 true-residual tolerance, agree with the oracle's
FP64 Wilson solve, and be bit-identical to the same request solved alone.
"""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


MIX = [  # L, kappa, gauge seed, eps, source kind, source seed
    ((4, 4, 4, 4), 0.150, 11, 0.2, 1, 3),
    ((8, 6, 6, 10), 0.157, 12, 0.5, 2, 0),
    ((4, 4, 4, 4), 0.155, 13, 0.4, 0, 5),
    ((8, 6, 6, 10), 0.152, 14, 0.3, 1, 6),
    ((4, 4, 4, 4), 0.153, 15, 0.5, 1, 7),
    ((8, 6, 6, 10), 0.150, 16, 0.2, 0, 8),
]


def full_bytes(H, L):
    return H.hmc_field_bytes(L, H.F64, H.KIND_FULL_SPINOR)


def to_canon(H, L, buf):
    F = H.Fields(L, 5.6, 0.15)
    c = H.canon_spinor_zeros(L)
    H.hmc_export_spinor(F, c, buf, -1)
    torch.cuda.synchronize()
    return c.cpu().numpy()


def run_manual(H, reqs, prec, arena=1 << 28, max_batch=16, streams=None, reliable_delta=0.0):
    svc = H.Service(arena, inner_prec=prec, max_batch=max_batch, manual=True, streams=streams,
                    reliable_delta=reliable_delta)
    outs, tickets = [], []
    for (L, k, gs, eps, kind, ss) in reqs:
        out = torch.zeros(full_bytes(H, L), dtype=torch.uint8, device="cuda")
        outs.append(out)
        tickets.append(svc.submit(H.solve_request(L, k, gs, eps, kind, ss, 0, out)))
    rounds = 0
    while svc.step() > 0:
        rounds += 1
        assert rounds < 100000
    res = [svc.poll(t) for t in tickets]
    svc.close()
    return res, outs


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_service_mix_converges_and_matches_alone(H, prec):
    res, outs = run_manual(H, MIX, prec)
    for r in res:
        assert r["status"] == 0 and r["true_rel_res"] <= 1e-10, r
    assert max(r["max_group"] for r in res) == 3  # three requests per volume advanced together
    for i in (0, 1):  # the same request alone: bit-identical solution
        alone, aout = run_manual(H, [MIX[i]], prec)
        assert alone[0]["iters"] == res[i]["iters"]
        assert torch.equal(aout[0], outs[i])


@pytest.mark.parametrize("prec", [2, 3])
def test_service_small_delta_low_storage(H, prec):
    """FP16 / BF16 inner solves with reliable-update delta 0.01, where BF16
    needs the search-direction restarts (the single solve diverged there
    without them): every request of a mix with a 16^3x32 one converges to
    the FP64 tolerance, bit-identical alone and in the mix."""
    reqs = MIX[:3] + [((16, 16, 16, 32), 0.156, 32, 0.45, 2, 0)]
    res, outs = run_manual(H, reqs, prec, arena=1 << 30, reliable_delta=0.01)
    for r in res:
        assert r["status"] == 0 and r["true_rel_res"] <= 1e-10, r
    alone, aout = run_manual(H, [reqs[3]], prec, arena=1 << 30, reliable_delta=0.01)
    assert alone[0]["iters"] == res[3]["iters"] and torch.equal(aout[0], outs[3])


def test_service_matches_oracle(H):
    res, outs = run_manual(H, MIX[:2], 1)
    for (L, k, gs, eps, kind, ss), out in zip(MIX[:2], outs):
        U = O.weak_field(L, gs, eps)
        b = O.source(L, kind, ss, 0)
        want, st = O.wilson_solve(L, U, k, b, tol=1e-12)
        got = to_canon(H, L, out)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-8


# the serving workload's volumes, kappa range and source kinds (Z2, point)
MIX_SERVE = [
    ((8, 8, 8, 8), 0.151, 31, 0.25, 1, 40),
    ((16, 16, 16, 32), 0.156, 32, 0.45, 2, 0),
    ((24, 24, 24, 48), 0.157, 33, 0.5, 1, 41),
    ((8, 8, 8, 8), 0.157, 34, 0.5, 2, 0),
    ((16, 16, 16, 32), 0.150, 35, 0.2, 1, 42),
    ((24, 24, 24, 48), 0.153, 36, 0.3, 2, 0),
]


@pytest.mark.timeout(900)
def test_service_at_serving_volumes(H):
    """Requests of 8^4, 16^3x32 and 24^3x48 in one mix (FP32 inner solves,
    the tuned launch shapes of those volumes, three caller streams): every
    result meets the FP64 true-residual tolerance, is bit-identical to the
    same request solved alone (on the caller's current stream) and agrees
    with the oracle's FP64 Wilson solve (1e-8: both solutions meet
    |b - M x| <= 1e-10 |b|, the oracle's to 1e-12)."""
    streams = [torch.cuda.Stream() for _ in range(3)]
    arena = 6 << 30
    res, outs = run_manual(H, MIX_SERVE, H.F32, arena=arena, streams=streams)
    for r in res:
        assert r["status"] == 0 and r["true_rel_res"] <= 1e-10, r
    assert max(r["max_group"] for r in res) == 2
    for i, req in enumerate(MIX_SERVE):
        alone, aout = run_manual(H, [req], H.F32, arena=arena, streams=[torch.cuda.current_stream()])
        assert alone[0]["iters"] == res[i]["iters"], i
        assert torch.equal(aout[0], outs[i]), i
        del aout
    for (L, k, gs, eps, kind, ss), out in zip(MIX_SERVE, outs):
        U = O.weak_field(L, gs, eps)
        b = O.source(L, kind, ss, 0)
        want, st = O.wilson_solve(L, U, k, b, tol=1e-12, maxiter=50000)
        assert st["status"] == 0
        got = to_canon(H, L, out)
        d = np.linalg.norm(got - want) / np.linalg.norm(want)
        print(f"service {L} kappa {k} source {kind}: |x - x_oracle| / |x_oracle| = {d:.2e}")
        assert d < 1e-8, (L, d)


def test_admission_waits_for_memory(H):
    L = (8, 6, 6, 10)
    need = H.hmc_request_bytes(H.solve_request(L, 0.15, 1, 0.3), H.F32)
    # room for two requests besides the service header (~2.5 MB)
    svc = H.Service(2 * need + (4 << 20), inner_prec=H.F32, max_batch=8, manual=True)
    tickets = [svc.submit(H.solve_request(L, 0.15 + 0.001 * i, 20 + i, 0.3, 1, i)) for i in range(5)]
    rounds = 0
    while svc.step() > 0:
        rounds += 1
    res = [svc.poll(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    assert max(r["max_group"] for r in res) == 2
    starts = sorted(r["t_start"] for r in res)
    assert starts[2] > min(r["t_done"] for r in res[:2]) - 1e-9  # the third started after a slot freed
    svc.close()


def test_request_that_cannot_fit_is_rejected(H):
    svc = H.Service(16 << 20, inner_prec=H.F32, manual=True)
    with pytest.raises(H.HmcError) as e:
        svc.submit(H.solve_request((16, 16, 16, 32), 0.15, 1, 0.3))
    assert e.value.status == H.HMC_E_OOM
    svc.close()


def test_threaded_service(H):
    svc = H.Service(1 << 28, inner_prec=H.F16, max_batch=8)
    tickets = [svc.submit(H.solve_request(L, k, gs, eps, kind, ss)) for (L, k, gs, eps, kind, ss) in MIX]
    res = [svc.wait(t) for t in tickets]
    assert all(r["status"] == 0 and r["true_rel_res"] <= 1e-10 for r in res)
    assert all(r["t_submit"] <= r["t_start"] <= r["t_done"] for r in res)
    svc.close()
