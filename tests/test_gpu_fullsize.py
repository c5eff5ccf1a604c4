"""Parity at the benchmark workloads' full sizes, in the launch configurations the benchmark
times: 512^2 object, 64^2 probe, 1600 positions, minibatch 64, two levels (C2); 1024^2 object,
128^2 probe, 10000 positions, minibatch 256, three levels (C3); 1024^2 object, 256^2 probe, 961
positions, minibatch 32, two levels (C6)."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import MISFIT_TOL, STEP_TOL, amps, host, init_state, make_rec, problem, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def c2():
    return problem("c2")


# (path, FFT plan, finalize shape): the default plan on two launch strategies, and the
# configuration the autotuner picks for this workload (register-resident passes, 16^2 tiles
# in banded order, fused launches)
@pytest.mark.parametrize("path, plan, shape", [("graph", 0, 0), ("persistent", 0, 0),
                                               ("fused", 3, 5)])
def test_c2_minibatch_step_parity(c2, path, plan, shape):
    p = c2
    print("case: c2 step", path, plan, shape, flush=True)
    rec = make_rec(p, path=path, seed=p.seed, fft_plan=plan, finalize_shape=shape)
    obj, probe = init_state(p, rec)
    a = amps(p)
    perm = O.permutation(p.seed, 0, p.n_pos)
    for stage in range(2):
        idx = perm[stage * 64:(stage + 1) * 64]
        z0, q0 = host(obj), host(probe)
        rec.step(obj, probe, idx)
        torch.cuda.synchronize()
        q1, z1, _ = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=2)
        assert rel(host(obj), z1) < STEP_TOL, rel(host(obj), z1)
        assert rel(host(probe), q1) < STEP_TOL, rel(host(probe), q1)
        rec.epoch(obj, probe, 1 + stage)  # move to a mid-reconstruction state
    rec.close()


def test_c2_misfit_parity_and_sampled_misfit(c2):
    p = c2
    print("case: c2 misfit", flush=True)
    rec = make_rec(p, path="graph", seed=p.seed)
    obj, probe = init_state(p, rec)
    a = amps(p)
    s = torch.zeros((), dtype=torch.float64, device="cuda")
    rec.epoch(obj, probe, 0, sampled=s)
    phi = float(rec.misfit(obj, probe).item())
    torch.cuda.synchronize()
    ref = O.misfit(host(probe), host(obj), p.positions, a)
    assert abs(phi - ref) <= MISFIT_TOL * ref
    assert np.isfinite(float(s.item())) and float(s.item()) > phi
    rec.close()


@pytest.fixture(scope="module")
def c3():
    return problem("c3")


# the default plan, and the configuration the autotuner picks for this workload
@pytest.mark.parametrize("path, plan, shape", [("graph", 0, 0), ("fused", 1, 2), ("fused", 1, 10),
                                               ("fused", 0, 8)])
def test_c3_minibatch_step_parity_three_levels(c3, path, plan, shape):
    # 1024^2 object, 128^2 probe, 10000 positions, minibatch 256, three levels; full
    # minibatches from mid-reconstruction states.  At the initial guess (z = 1, smooth
    # zero-phase probe) almost every Fourier bin of the exit wave lies below float32
    # resolution, so its phase -- and R there -- is arbitrary in any finite precision, and
    # with 1e7-photon data the measured amplitudes at those bins are not negligible; the
    # comparison therefore starts after one sweep.
    p = c3
    print("case: c3 step", path, plan, shape, flush=True)
    rec = make_rec(p, path=path, seed=p.seed, fft_plan=plan, finalize_shape=shape)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    a = amps(p)
    perm = O.permutation(p.seed, 3, p.n_pos)
    for stage in range(2):
        idx = perm[stage * 256:(stage + 1) * 256]
        z0, q0 = host(obj), host(probe)
        rec.step(obj, probe, idx)
        torch.cuda.synchronize()
        q1, z1, _ = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=3)
        assert rel(host(obj), z1) < STEP_TOL, rel(host(obj), z1)
        assert rel(host(probe), q1) < STEP_TOL, rel(host(probe), q1)
        rec.epoch(obj, probe, 1 + stage)
    rec.close()


# the full misfit over all 10000 patterns in the XCD order, with the two-workgroups-per-CU
# kernel of each split: plans 0 and 2 (16 x 8) and plan 1 (8 x 16)
@pytest.mark.parametrize("plan", [0, 1, 2])
def test_c3_full_misfit_parity(c3, plan):
    p = c3
    print("case: c3 full misfit", plan, flush=True)
    rec = make_rec(p, path="fused", seed=p.seed, fft_plan=plan, finalize_shape=8)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    phi = float(rec.misfit(obj, probe).item())
    torch.cuda.synchronize()
    ref = O.misfit(host(probe), host(obj), p.positions, amps(p))
    assert abs(phi - ref) <= MISFIT_TOL * ref, (phi, ref)
    rec.close()


@pytest.fixture(scope="module")
def c6():
    return problem("c6")


# 256^2 patterns at full size (1024^2 object, 961 positions, minibatch 32, two levels): full
# minibatches of 32 slots (all 16 strips of a slot on one XCD) from a mid-reconstruction
# state on the fused and graph paths, and the full misfit over all 961 patterns
@pytest.mark.parametrize("path, shape", [("fused", 8), ("graph", 0)])
def test_c6_minibatch_step_and_misfit_parity(c6, path, shape):
    p = c6
    print("case: c6 step", path, shape, flush=True)
    rec = make_rec(p, path=path, seed=p.seed, finalize_shape=shape)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    a = amps(p)
    perm = O.permutation(p.seed, 5, p.n_pos)
    for stage in range(2):
        idx = perm[stage * 32:(stage + 1) * 32]
        z0, q0 = host(obj), host(probe)
        rec.step(obj, probe, idx)
        torch.cuda.synchronize()
        q1, z1, _ = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=p.levels)
        assert rel(host(obj), z1) < STEP_TOL, rel(host(obj), z1)
        assert rel(host(probe), q1) < STEP_TOL, rel(host(probe), q1)
    phi = float(rec.misfit(obj, probe).item())
    torch.cuda.synchronize()
    ref = O.misfit(host(probe), host(obj), p.positions, a)
    assert abs(phi - ref) <= MISFIT_TOL * ref, (phi, ref)
    rec.close()
