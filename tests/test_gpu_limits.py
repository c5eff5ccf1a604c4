"""Size limits and degenerate shapes against the oracle: the largest minibatch (1024 slots), a
4096^2 object (64-bit offsets), a single scan position, and a minibatch larger than N."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import EPOCH_TOL, MISFIT_TOL, STEP_TOL, amps, host, init_state, rel
from paper_2511_01793_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_01793_amd.emagpie")


def say(*a):
    print(*a, flush=True)


def custom(n, m, pos, seed, photons=1e6):
    """Problem with given positions: synthetic object and probe, Poisson intensities."""
    rng = np.random.default_rng(seed)
    z = synth.make_object(n, rng)
    q = synth.true_probe(m)
    clean = synth.simulate_intensities(q, z, pos)
    s = photons / clean.sum(axis=(1, 2)).mean()
    d = rng.poisson(clean * s).astype(np.float32)
    return z, q * np.sqrt(s), d


def state_after_sweep(rec, n, m, d):
    obj = torch.ones((n, n), dtype=torch.complex64, device="cuda")
    probe = torch.from_numpy(synth.initial_probe(m).astype(np.complex64)).cuda()
    rec.normalize_probe(probe)
    rec.epoch(obj, probe, 11)
    torch.cuda.synchronize()
    return obj, probe


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_largest_minibatch(path):
    # 1024 slots in one minibatch (the limit), every object pixel under ~60 of them
    n, m, N = 128, 32, 1100
    rng = np.random.default_rng(5)
    pos = rng.integers(0, n - m + 1, size=(N, 2)).astype(np.int32)
    _, _, d = custom(n, m, pos, 5)
    say("case: minibatch 1024", path)
    rec = E.Reconstruction(pos, torch.from_numpy(d).cuda(), n, minibatch=1024, levels=2,
                           alpha=0.05, path=path, seed=2)
    obj, probe = state_after_sweep(rec, n, m, d)
    idx = rng.permutation(N)[:1024].astype(np.int32)
    z0, q0 = host(obj), host(probe)
    s = torch.zeros((), dtype=torch.float64, device="cuda")
    rec.step(obj, probe, idx, sampled=s)
    torch.cuda.synchronize()
    q1, z1, info = O.step_minibatch(q0, z0, pos, O.amplitudes(d), idx, alpha=0.05, levels=2)
    assert rel(host(obj), z1) < STEP_TOL and rel(host(probe), q1) < STEP_TOL
    assert abs(float(s.item()) - info["sampled_misfit"]) <= MISFIT_TOL * info["sampled_misfit"]
    rec.close()


def test_large_object_offsets():
    # a 4096^2 object (16.8 M pixels): windows in all four corners and the middle
    n, m = 4096, 64
    pos = np.array([[0, 0], [0, n - m], [n - m, 0], [n - m, n - m], [2000, 3001], [n - m - 1, 7]],
                   dtype=np.int32)
    _, _, d = custom(n, m, pos, 6)
    say("case: 4096^2 object")
    rec = E.Reconstruction(pos, torch.from_numpy(d).cuda(), n, minibatch=3, levels=3, alpha=0.05,
                           path="fused", seed=4)
    obj, probe = state_after_sweep(rec, n, m, d)
    idx = np.array([3, 1, 4], dtype=np.int32)
    z0, q0 = host(obj), host(probe)
    rec.step(obj, probe, idx)
    phi = float(rec.misfit(obj, probe).item())
    torch.cuda.synchronize()
    a = O.amplitudes(d)
    q1, z1, info = O.step_minibatch(q0, z0, pos, a, idx, alpha=0.05, levels=3)
    t = info["touched"]
    zg = host(obj)
    assert rel(zg[t], z1[t]) < STEP_TOL and rel(host(probe), q1) < STEP_TOL
    assert np.array_equal(zg[~t], z0[~t])
    ref = O.misfit(host(probe), zg, pos, a)
    assert abs(phi - ref) <= MISFIT_TOL * ref
    rec.close()


@pytest.mark.parametrize("path", ["fused", "graph", "persistent", "chain"])
def test_single_position_and_minibatch_above_n(path):
    n, m = 80, 32
    pos = np.array([[23, 17]], dtype=np.int32)
    _, _, d = custom(n, m, pos, 7)
    B = 1 if path == "chain" else 4  # B > N = 1 except on the minibatch-1 path
    say("case: N = 1", path)
    rec = E.Reconstruction(pos, torch.from_numpy(d).cuda(), n, minibatch=B, levels=2, alpha=0.05,
                           path=path, seed=8)
    obj, probe = state_after_sweep(rec, n, m, d)
    a = O.amplitudes(d)
    for e in range(2):
        z0, q0 = host(obj), host(probe)
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.epoch(obj, probe, e, sampled=s)
        torch.cuda.synchronize()
        q1, z1, samp = O.run_epoch(q0, z0, pos, a, seed=8, epoch=e, minibatch=B, alpha=0.05,
                                   levels=2)
        assert rel(host(obj), z1) < EPOCH_TOL and rel(host(probe), q1) < EPOCH_TOL
        assert abs(float(s.item()) - samp) <= MISFIT_TOL * samp
    rec.close()
