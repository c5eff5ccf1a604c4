"""Exact-paper sequential mode: minibatch 1 in one workgroup (the chain path) and the stateful
zero-bin phase rule stated after Eq. 3, against the fused path and the oracle."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import EPOCH_TOL, STEP_TOL, amps, host, init_state, make_rec, problem, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_01793_amd.emagpie")


def say(*a):
    print(*a, flush=True)


def small(m, L, side=5, photons=1e6, seed=61):
    n = 3 * m + 4
    step = max(1, (n - m - 2) // (side - 1))
    return problem("tiny", n=n, m=m, scan=("raster", side, step, 1), photons=photons, B=1, L=L,
                   alpha=0.05, seed=seed)


def rec_for(p, **kw):
    d = torch.from_numpy(p.intensities).cuda()
    base = dict(minibatch=1, levels=p.levels, alpha=p.alpha, alpha_z=p.alpha_z, seed=5,
                path="fused")
    base.update(kw)
    return E.Reconstruction(p.positions, d, p.n, **base)


def sweep(p, epochs=2, **kw):
    rec = rec_for(p, **kw)
    obj, probe = init_state(p, rec)
    out = []
    for e in range(epochs):
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.epoch(obj, probe, e, sampled=s)
        out.append(s)
    torch.cuda.synchronize()
    rec.close()
    return obj, probe, [float(x.item()) for x in out]


@pytest.mark.parametrize("m, L", [(32, 1), (32, 2), (64, 2), (64, 3), (128, 1), (128, 3)])
def test_chain_path_equals_fused_path_bitwise(m, L):
    p = small(m, L)
    say("case: chain", m, L)
    of, qf, sf = sweep(p, path="fused")
    oc, qc, sc = sweep(p, path="chain")
    assert torch.equal(of, oc) and torch.equal(qf, qc)
    assert sf == sc


@pytest.mark.parametrize("m, v", [(64, 3), (64, 1), (128, 2)])
def test_chain_path_equals_fused_path_bitwise_other_plans(m, v):
    # plans with two or more per-pixel rounds (64 / 3 loads each round's values one round
    # ahead, beside the in-place writes of the minibatch-1 update)
    p = small(m, 2)
    say("case: chain plan", m, v)
    of, qf, sf = sweep(p, path="fused", fft_plan=v)
    oc, qc, sc = sweep(p, path="chain", fft_plan=v)
    assert torch.equal(of, oc) and torch.equal(qf, qc)
    assert sf == sc


def test_chain_path_epoch_parity_with_the_oracle():
    p = small(32, 2)
    say("case: chain vs oracle")
    rec = rec_for(p, path="chain")
    obj, probe = init_state(p, rec)
    a = amps(p)
    for e in range(2):
        z0, q0 = host(obj), host(probe)
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.epoch(obj, probe, e, sampled=s)
        torch.cuda.synchronize()
        q1, z1, samp = O.run_epoch(q0, z0, p.positions, a, seed=5, epoch=e, minibatch=1,
                                   alpha=p.alpha, levels=2)
        assert rel(host(obj), z1) < EPOCH_TOL and rel(host(probe), q1) < EPOCH_TOL
        assert abs(float(s.item()) - samp) <= 1e-4 * samp
    rec.close()


@pytest.mark.parametrize("m", [64, 128])
def test_phase_memory_off_the_zero_bins_changes_nothing(m):
    # the kernels compiled with the phase memory against those compiled without it
    p = small(m, 2)
    say("case: memory without zero bins", m)
    o1, q1, s1 = sweep(p, path="fused")
    o2, q2, s2 = sweep(p, path="fused", zero_phase_memory=True)
    o3, q3, s3 = sweep(p, path="chain", zero_phase_memory=True)
    assert torch.equal(o1, o2) and torch.equal(q1, q2) and s1 == s2
    assert torch.equal(o1, o3) and torch.equal(q1, q3)


@pytest.mark.parametrize("m", [32, 128])
@pytest.mark.parametrize("path", ["fused", "plain", "chain"])
def test_phase_memory_on_exact_zero_bins_matches_the_oracle(path, m):
    """First visit of pattern k with a random state (no zero bins: the memory takes its
    phases), second visit with a constant exit wave (every bin but DC exactly zero: the
    revised wave carries the first visit's phases there)."""
    p = small(m, 1)
    say("case: phase memory", path, m)
    rng = np.random.default_rng(3)
    k = 7
    Qr = (rng.standard_normal((p.m, p.m)) + 1j * rng.standard_normal((p.m, p.m))).astype(np.complex64)
    zr = (rng.standard_normal((p.n, p.n)) + 1j * rng.standard_normal((p.n, p.n))).astype(np.complex64)
    Qc = np.full((p.m, p.m), 0.6 - 0.2j, dtype=np.complex64)
    zc = np.full((p.n, p.n), 1.0 + 0.1j, dtype=np.complex64)
    a = amps(p)
    mem = np.ones((p.n_pos, p.m, p.m), complex)
    O.step_minibatch(Qr.astype(complex), zr.astype(complex), p.positions, a, [k], alpha=p.alpha,
                     phase_mem=mem)
    q_ref, z_ref, _ = O.step_minibatch(Qc.astype(complex), zc.astype(complex), p.positions, a, [k],
                                       alpha=p.alpha, phase_mem=mem)
    results = {}
    for memory in (True, False):
        rec = rec_for(p, path=path, zero_phase_memory=memory)
        obj, probe = torch.from_numpy(zr).cuda(), torch.from_numpy(Qr).cuda()
        rec.step(obj, probe, [k])
        obj.copy_(torch.from_numpy(zc))
        probe.copy_(torch.from_numpy(Qc))
        rec.step(obj, probe, [k])
        torch.cuda.synchronize()
        results[memory] = (host(obj), host(probe))
        if memory:
            # back to the first-sweep state: the constant visit then equals the memory-less one
            rec.reset_phase_memory()
            o2, p2 = torch.from_numpy(zc).cuda(), torch.from_numpy(Qc).cuda()
            rec.step(o2, p2, [k])
            torch.cuda.synchronize()
            results["reset"] = (host(o2), host(p2))
        rec.close()
    zg, qg = results[True]
    assert rel(zg, z_ref) < STEP_TOL and rel(qg, q_ref) < STEP_TOL, (rel(zg, z_ref), rel(qg, q_ref))
    # the rule matters here: theta = 0 at the zero bins gives a different step
    assert rel(results[False][0], z_ref) > 1e-2
    np.testing.assert_array_equal(results["reset"][0], results[False][0])
    np.testing.assert_array_equal(results["reset"][1], results[False][1])


def test_autotuner_considers_the_chain_path_for_minibatch_one():
    p = small(64, 2)
    say("case: tune b=1")
    rec = rec_for(p, path="auto")
    plan = rec.plan
    assert "chain" in plan["path_ms"] and plan["path"] in plan["path_ms"]
    assert plan["path_ms"][plan["path"]] == min(plan["path_ms"].values())
    rec.close()
