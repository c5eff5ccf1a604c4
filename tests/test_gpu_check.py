"""Descent-check entry point (surrogate of Eq. 3, Prop. 3.1 agreement and majorisation,
Prop. 3.2 descent) against the oracle, and its step against the ordinary step."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import MISFIT_TOL, amps, host, init_state, make_rec, problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def small(m, L, B, seed=51):
    n = 3 * m + 4
    step = max(1, (n - m - 2) // 4)
    return problem("tiny", n=n, m=m, scan=("raster", 5, step, 1), photons=1e6, B=B, L=L,
                   alpha=0.05, seed=seed)


@pytest.mark.parametrize("m, L, b", [(32, 1, 1), (64, 1, 1), (32, 2, 5), (64, 2, 7), (128, 3, 4),
                                     (128, 1, 1)])
def test_check_step_values_and_properties(m, L, b):
    p = small(m, L, B=max(b, 2))
    print("case: check", m, L, b, flush=True)
    rec = make_rec(p, path="fused", minibatch=max(b, 2))
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 7)
    torch.cuda.synchronize()
    a = amps(p)
    rng = np.random.default_rng(m + L + b)
    for stage in range(3):
        idx = np.sort(rng.choice(p.n_pos, size=b, replace=False)).astype(np.int32)
        z0, q0 = host(obj), host(probe)
        o2, p2 = obj.clone(), probe.clone()
        out = rec.check_step(obj, probe, idx).cpu().numpy()
        rec.step(o2, p2, idx)
        torch.cuda.synchronize()
        # the check path applies exactly the ordinary step
        assert torch.equal(obj, o2) and torch.equal(probe, p2)
        # [0]: sampled misfit before; [1]: surrogate at the new GPU state with the oracle's
        # R frozen at the old state; [2]: sampled misfit at the new GPU state
        _, _, info = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=L)
        z1, q1 = host(obj), host(probe)
        pos = p.positions[idx]
        ref = [info["sampled_misfit"], O.surrogate(q1, z1, pos, info["R"]),
               float(O.misfit_terms(q1, z1, pos, a[idx]).sum())]
        for g, r in zip(out, ref):
            assert abs(g - r) <= MISFIT_TOL * r, (stage, out, ref)
        # majorisation (Prop. 3.1) up to the FP32 rounding of the state
        assert out[2] <= out[1] * (1 + 1e-5), out
        if b == 1 and L == 1:
            assert out[1] <= out[0] * (1 + 1e-5), out  # Prop. 3.2: sampled surrogate descent
        rec.epoch(obj, probe, 20 + stage)
    rec.close()


def test_prop32_descent_at_every_step_of_a_sweep():
    """Prop. 3.2 on the GPU at scale: single-position, single-level steps through a whole
    sweep of a 256^2 object (169 positions, 64^2 probe); every step must lower the sampled
    surrogate, and the misfit after must stay below the surrogate (majorisation)."""
    p = problem("tiny", n=256, m=64, scan=("raster", 13, 15, 1), photons=1e6, B=1, L=1,
                alpha=0.05, seed=71)
    print("case: prop 3.2 sweep", p.n_pos, flush=True)
    rec = make_rec(p, path="fused", minibatch=1, levels=1)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    order = O.permutation(9, 1, p.n_pos)
    outs = torch.stack([rec.check_step(obj, probe, [int(k)]) for k in order]).cpu().numpy()
    before, surr, after = outs[:, 0], outs[:, 1], outs[:, 2]
    assert np.all(surr <= before * (1 + 1e-5)), np.max(surr / before)
    assert np.all(after <= surr * (1 + 1e-5)), np.max(after / surr)
    assert np.mean(surr < before) > 0.95
    rec.close()
