"""Minibatch sizes that are not multiples of the finalize's slot scan (64 slots per ballot,
256 per step) and ragged last minibatches, in every finalize shape, against the oracle; and
minibatches whose slots the epoch lists in XCD order (B a multiple of the XCD count), where
every launch strategy must still agree bit for bit."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import EPOCH_TOL, MISFIT_TOL, host, rel
from paper_2511_01793_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_01793_amd.emagpie")


def say(*a):
    print(*a, flush=True)


def scattered(n, m, N, seed, photons=1e6):
    """N seeded random windows of a synthetic object, Poisson intensities."""
    rng = np.random.default_rng(seed)
    pos = rng.integers(0, n - m + 1, size=(N, 2)).astype(np.int32)
    z = synth.make_object(n, rng)
    q = synth.true_probe(m)
    clean = synth.simulate_intensities(q, z, pos)
    s = photons / clean.sum(axis=(1, 2)).mean()
    d = rng.poisson(clean * s).astype(np.float32)
    return pos, d


def epoch_from(pos, d, n, m, B, L, shape, seed, state):
    rec = E.Reconstruction(pos, torch.from_numpy(d).cuda(), n, minibatch=B, levels=L, alpha=0.05,
                           path="fused", seed=seed, finalize_shape=shape)
    obj = torch.from_numpy(state[0].astype(np.complex64)).cuda()
    probe = torch.from_numpy(state[1].astype(np.complex64)).cuda()
    s = torch.zeros((), dtype=torch.float64, device="cuda")
    rec.epoch(obj, probe, 4, sampled=s)
    torch.cuda.synchronize()
    rec.close()
    return obj, probe, float(s.item())


@pytest.mark.parametrize("B, N", [(300, 650), (257, 520), (130, 400), (256, 600)])
def test_ragged_minibatches_every_shape(B, N):
    # B = 300: ballots of 64, 64, 64, 64 and 44 over two scan steps; last batch of 50.
    # B = 257: one slot past a scan step; last batch of 6.  B = 130: a ragged third ballot.
    # B = 256: full scan steps, listed in XCD order, and a last batch of 88 (also listed).
    n, m, L = 160, 32, 2
    pos, d = scattered(n, m, N, seed=B)
    rng = np.random.default_rng(B + 1)
    z0 = (0.9 + 0.1 * rng.random((n, n))) * np.exp(0.3j * rng.standard_normal((n, n)))
    q0 = synth.initial_probe(m).astype(np.complex128) * np.sqrt(d.sum(axis=(1, 2)).mean()) / m
    state = (z0, q0)
    say("case: minibatch", B, "of", N)
    runs = [epoch_from(pos, d, n, m, B, L, f, 21, state) for f in range(4)]
    for f in range(1, 4):
        assert torch.equal(runs[f][0], runs[0][0]) and torch.equal(runs[f][1], runs[0][1]), f
        assert runs[f][2] == runs[0][2], f
    q1, z1, samp = O.run_epoch(q0.astype(np.complex64).astype(np.complex128),
                               z0.astype(np.complex64).astype(np.complex128), pos,
                               O.amplitudes(d), seed=21, epoch=4, minibatch=B, alpha=0.05, levels=L)
    assert rel(host(runs[0][0]), z1) < EPOCH_TOL, rel(host(runs[0][0]), z1)
    assert rel(host(runs[0][1]), q1) < EPOCH_TOL, rel(host(runs[0][1]), q1)
    assert abs(runs[0][2] - samp) <= MISFIT_TOL * samp


def test_xcd_listing_every_path_bitwise():
    # B = 32 (a multiple of 8): the epoch lists each minibatch's slots in XCD order; plain,
    # fused, graph and persistent launches of the same sweep agree bit for bit, and with the
    # oracle (which sums in its own order) to the epoch bar
    n, m, L, B, N = 160, 32, 2, 32, 200
    pos, d = scattered(n, m, N, seed=77)
    rng = np.random.default_rng(78)
    z0 = (0.9 + 0.1 * rng.random((n, n))) * np.exp(0.3j * rng.standard_normal((n, n)))
    q0 = synth.initial_probe(m).astype(np.complex128) * np.sqrt(d.sum(axis=(1, 2)).mean()) / m
    say("case: xcd listing, every path")
    out = {}
    for path in ("plain", "fused", "graph", "persistent"):
        rec = E.Reconstruction(pos, torch.from_numpy(d).cuda(), n, minibatch=B, levels=L,
                               alpha=0.05, path=path, seed=5)
        obj = torch.from_numpy(z0.astype(np.complex64)).cuda()
        probe = torch.from_numpy(q0.astype(np.complex64)).cuda()
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.epoch(obj, probe, 3, sampled=s)
        torch.cuda.synchronize()
        out[path] = (obj, probe, float(s.item()))
        rec.close()
    for path in ("fused", "graph", "persistent"):
        assert torch.equal(out[path][0], out["plain"][0]), path
        assert torch.equal(out[path][1], out["plain"][1]), path
        assert out[path][2] == out["plain"][2], path
    q, z, samp = O.run_epoch(q0.astype(np.complex64).astype(np.complex128),
                             z0.astype(np.complex64).astype(np.complex128), pos, O.amplitudes(d),
                             seed=5, epoch=3, minibatch=B, alpha=0.05, levels=L)
    assert rel(host(out["fused"][0]), z) < EPOCH_TOL, rel(host(out["fused"][0]), z)
    assert rel(host(out["fused"][1]), q) < EPOCH_TOL, rel(host(out["fused"][1]), q)
    assert abs(out["fused"][2] - samp) <= MISFIT_TOL * samp
