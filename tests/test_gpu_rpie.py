"""rPIE comparator (Eq. 2): the same kernels with the joint step of Eq. 6 switched off.

The oracle's step with joint=False is pinned to Eq. 2's written update form on the CPU
(test_reduces_to_rpie_eq2_and_epie); here the HIP path is compared with it element by
element, for one step from identical state and for whole epochs.
"""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import EPOCH_TOL, MISFIT_TOL, STEP_TOL, amps, host, init_state, make_rec, problem, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def small(m=32, n=100, L=1, B=7, side=5, photons=None, seed=21):
    step = max(1, (n - m - 2) // (side - 1))
    return problem("tiny", n=n, m=m, scan=("raster", side, step, 1), photons=photons, B=B, L=L,
                   alpha=0.05, seed=seed)


@pytest.mark.parametrize("m, L", [(32, 1), (64, 1), (64, 2), (128, 1)])
@pytest.mark.parametrize("path", ["plain", "fused"])
def test_rpie_step_parity(m, L, path):
    p = small(m=m, n=m + 3 * (m // 2) + 4, L=L, B=5, photons=1e6)
    say("case: rpie step", p.n, m, L, path)
    rec = make_rec(p, path=path, joint_step=False)
    obj, probe = init_state(p, rec)
    a = amps(p)
    # leave the phase-free initial guess first (ill-conditioned for per-step FP32 parity)
    rec.epoch(obj, probe, 50)
    rng = np.random.default_rng(m + 7 * L)
    for stage in range(2):
        idx = rng.choice(p.n_pos, size=5, replace=False).astype(np.int32)
        z0, q0 = host(obj), host(probe)
        sampled = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.step(obj, probe, idx, sampled=sampled)
        torch.cuda.synchronize()
        q1, z1, info = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=L,
                                        joint=False)
        assert rel(host(obj), z1) < STEP_TOL, (stage, rel(host(obj), z1))
        assert rel(host(probe), q1) < STEP_TOL, (stage, rel(host(probe), q1))
        s = info["sampled_misfit"]
        assert abs(float(sampled.item()) - s) <= MISFIT_TOL * s
        rec.epoch(obj, probe, 60 + stage)
    rec.close()


@pytest.mark.parametrize("path", ["graph", "persistent"])
def test_rpie_sequential_epoch_parity(path):
    # minibatch 1 is the classical sequential PIE sweep (one position per update)
    p = small(m=32, n=100, L=1, B=1)
    say("case: rpie epoch b=1", path)
    rec = make_rec(p, path=path, minibatch=1, seed=17, joint_step=False)
    obj, probe = init_state(p, rec)
    a = amps(p)
    for e in range(2):
        z0, q0 = host(obj), host(probe)
        sampled = torch.zeros((), dtype=torch.float64, device="cuda")
        rec.epoch(obj, probe, e, sampled=sampled)
        torch.cuda.synchronize()
        q1, z1, samp = O.run_epoch(q0, z0, p.positions, a, seed=17, epoch=e, minibatch=1,
                                   alpha=p.alpha, levels=1, joint=False)
        assert rel(host(obj), z1) < EPOCH_TOL, (e, rel(host(obj), z1))
        assert rel(host(probe), q1) < EPOCH_TOL, (e, rel(host(probe), q1))
        assert abs(float(sampled.item()) - samp) <= MISFIT_TOL * samp
    rec.close()


def test_rpie_and_emagpie_differ_only_by_the_joint_step():
    # from the same state, the rPIE result is the pair (z+, Q+) that eMAGPIE's joint step
    # (Eq. 6) combines with the current iterate: aligned_sqrt(z, z+) must give the eMAGPIE result
    p = small(m=32, n=100, L=1, B=7, photons=1e6)
    say("case: rpie vs emagpie")
    ra = make_rec(p, path="fused", joint_step=True)
    rb = make_rec(p, path="fused", joint_step=False)
    obj, probe = init_state(p, ra)
    ra.epoch(obj, probe, 3)
    torch.cuda.synchronize()
    z0, q0 = host(obj), host(probe)
    o2, p2 = obj.clone(), probe.clone()
    idx = np.arange(7, dtype=np.int32)
    ra.step(obj, probe, idx)
    rb.step(o2, p2, idx)
    torch.cuda.synchronize()
    zj, qj = host(obj), host(probe)
    zp, qp = host(o2), host(p2)
    assert rel(zj, zp) > 1e-3
    assert rel(O.aligned_sqrt(z0, zp), zj) < STEP_TOL
    assert rel(O.aligned_sqrt(q0, qp), qj) < STEP_TOL
    ra.close()
    rb.close()
