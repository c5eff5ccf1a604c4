"""Adjoint gradient (Sec. 2.1, CR calculus) at full size, and the 16-instance batched workload
at its real size.

* The differentiation workload itself: 256^2 object, 64^2 probe, 20 x 20 raster of 400 positions,
  noiseless 64^2 intensities, in float32 and float64, against the FP64 oracle gradient, and
  against Prop. 3.1's gradient matching (central differences of the quadratic surrogate of
  Eq. 3 with the revised exit waves frozen at the iterate).  400 patterns in one chunk put about
  100 patterns in each of the object scatter's four pattern groups, so its 64-slot ballot scan
  takes several rounds.
* More patterns than one gradient chunk holds, so that later chunks add onto the first
  (m = 128: 256 patterns per chunk; m = 32: 1024).
* The 16 uneven instances (objects 256-1024^2, probes 64^2 / 128^2, 400-4096 positions each):
  a group sweep bitwise equal to the members swept alone, and one member's sweep against the
  oracle.
"""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import (EPOCH_TOL, GRAD32_TOL, GRAD64_TOL, MISFIT_TOL, amps, host, init_state,
                         make_rec, problem, rel)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c4_state():
    """The differentiation workload at a mid-reconstruction state (one sweep from the
    Sec. 4.1 initial guess), with its oracle gradient."""
    p = problem("c4")
    say("case: c4 state", p.n, p.m, p.n_pos)
    rec = make_rec(p, path="fused", seed=p.seed)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    torch.cuda.synchronize()
    z, q = host(obj), host(probe)
    ref = O.gradients(q, z, p.positions, amps(p))
    yield p, rec, obj, probe, ref
    rec.close()


@pytest.mark.parametrize("f64", [False, True])
def test_c4_gradient_against_oracle(c4_state, f64):
    p, rec, obj, probe, (rz, rq, rphi) = c4_state
    say("case: c4 grad", "f64" if f64 else "f32")
    o, q = (obj.to(torch.complex128), probe.to(torch.complex128)) if f64 else (obj, probe)
    gz, gq, phi = rec.grad(o, q)
    torch.cuda.synchronize()
    tol = GRAD64_TOL if f64 else GRAD32_TOL
    assert rel(host(gz), rz) < tol, rel(host(gz), rz)
    assert rel(host(gq), rq) < tol, rel(host(gq), rq)
    assert abs(float(phi.item()) - rphi) <= (1e-12 if f64 else MISFIT_TOL) * rphi
    # pixels no window covers have a zero gradient (the sum of P_k^T over no k)
    covered = np.zeros((p.n, p.n), dtype=bool)
    for r, c in p.positions:
        covered[r:r + p.m, c:c + p.m] = True
    assert np.all(host(gz)[~covered] == 0)


def test_c4_gradient_matches_frozen_surrogate(c4_state):
    # Prop. 3.1: at the iterate the quadratic surrogate (R_k frozen there) and Phi share their
    # gradient.  Central differences of the oracle's surrogate along random directions against
    # the float64 adjoint: Re <grad, v> = d/dt surrogate(x + t v) at t = 0.
    p, rec, obj, probe, _ = c4_state
    say("case: c4 gradient matching")
    o64, q64 = obj.to(torch.complex128), probe.to(torch.complex128)
    gz, gq, _ = rec.grad(o64, q64)
    torch.cuda.synchronize()
    z, q = host(o64), host(q64)
    a = amps(p)
    m = p.m
    R = [O.revised_exit_wave(q, z[r:r + m, c:c + m], a[k]) for k, (r, c) in enumerate(p.positions)]
    rng = np.random.default_rng(44)
    h = 1e-5
    for _ in range(2):
        vz = rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape)
        vq = rng.standard_normal(q.shape) + 1j * rng.standard_normal(q.shape)
        fp = O.surrogate(q + h * vq, z + h * vz, p.positions, R)
        fm = O.surrogate(q - h * vq, z - h * vz, p.positions, R)
        fd = (fp - fm) / (2 * h)
        an = float(np.vdot(host(gz), vz).real + np.vdot(host(gq), vq).real)
        # the surrogate is quadratic: central differences are exact up to rounding
        assert abs(fd - an) <= 1e-8 * abs(an), (fd, an)


@pytest.mark.parametrize("m, n, side, step, f64", [(128, 384, 20, 13, False),
                                                    (32, 256, 34, 6, False),
                                                    (32, 256, 34, 6, True)])
def test_gradient_over_several_chunks(m, n, side, step, f64):
    # 400 patterns at m = 128 (chunks of 256) and 1156 at m = 32 (chunks of 1024): the later
    # chunks' object and probe sums are added onto the first chunk's
    p = problem("tiny", n=n, m=m, scan=("raster", side, step, 1), photons=1e6, B=64, L=2,
                alpha=0.05, seed=61 + m)
    say("case: chunked grad", m, n, p.n_pos, "f64" if f64 else "f32")
    rec = make_rec(p, path="fused", seed=5)
    obj, probe = init_state(p, rec)
    rec.epoch(obj, probe, 0)
    if f64:
        obj, probe = obj.to(torch.complex128), probe.to(torch.complex128)
    gz, gq, phi = rec.grad(obj, probe)
    torch.cuda.synchronize()
    rz, rq, rphi = O.gradients(host(probe), host(obj), p.positions, amps(p))
    tol = GRAD64_TOL if f64 else GRAD32_TOL
    assert rel(host(gz), rz) < tol, rel(host(gz), rz)
    assert rel(host(gq), rq) < tol, rel(host(gq), rq)
    assert abs(float(phi.item()) - rphi) <= (1e-12 if f64 else MISFIT_TOL) * rphi
    # the call overwrites its outputs: a second call gives the same bits
    gz2, gq2, _ = rec.grad(obj, probe)
    torch.cuda.synchronize()
    assert torch.equal(gz, gz2) and torch.equal(gq, gq2)
    rec.close()


# ------------------------------------------------------------------ 16 uneven instances

@pytest.fixture(scope="module")
def c5():
    from paper_2511_01793_amd import synth
    say("case: c5 inputs (16 instances)")
    return synth.make_c5()


def _c5_recs(ps, plan_of):
    recs = []
    for i, p in enumerate(ps):
        v, f = plan_of(p)
        recs.append(make_rec(p, path="graph", seed=p.seed, fft_plan=v, finalize_shape=f))
    return recs


# per probe-size class the plan and finalize shape the benchmark's group leg uses on this
# workload (m = 64: register-pass plan 3, banded 16^2 tiles; m = 128: plan 1, banded 32^2 tiles),
# and the default plans
@pytest.mark.parametrize("plans", [{64: (3, 4), 128: (1, 5)}, {64: (0, 0), 128: (0, 0)}])
def test_c5_group_sweep_equals_members_alone_bitwise(c5, plans):
    import paper_2511_01793_amd.emagpie as E
    ps = c5
    say("case: c5 group vs alone", plans)
    recs = _c5_recs(ps, lambda p: plans[p.m])
    states = [init_state(p, r) for p, r in zip(ps, recs)]
    grp = E.Group(recs)
    sampled = torch.zeros(len(ps), dtype=torch.float64, device="cuda")
    grp.epoch([o for o, _ in states], [q for _, q in states], 0, sampled=sampled)
    torch.cuda.synchronize()
    got = [(o.cpu().numpy(), q.cpu().numpy()) for o, q in states]
    got_s = sampled.cpu().numpy()
    grp.close()
    for i, (p, r) in enumerate(zip(ps, recs)):
        o, q = init_state(p, r)
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        r.epoch(o, q, 0, sampled=s)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), got[i][0]), i
        assert np.array_equal(q.cpu().numpy(), got[i][1]), i
        assert float(s.item()) == got_s[i], i
        r.close()


def test_c5_member_sweep_matches_oracle(c5):
    import paper_2511_01793_amd.emagpie as E
    ps = c5
    j = min(range(len(ps)), key=lambda i: ps[i].n_pos * ps[i].m ** 2)  # the cheapest for the oracle
    say("case: c5 member vs oracle", j, ps[j].n, ps[j].m, ps[j].n_pos)
    recs = _c5_recs(ps, lambda p: (0, 0))
    states = [init_state(p, r) for p, r in zip(ps, recs)]
    grp = E.Group(recs)
    objs, probes = [o for o, _ in states], [q for _, q in states]
    grp.epoch(objs, probes, 0)  # away from the phase-free initial guess
    torch.cuda.synchronize()
    z0, q0 = host(objs[j]), host(probes[j])
    sampled = torch.zeros(len(ps), dtype=torch.float64, device="cuda")
    grp.epoch(objs, probes, 1, sampled=sampled)
    torch.cuda.synchronize()
    p = ps[j]
    q1, z1, samp = O.run_epoch(q0, z0, p.positions, amps(p), seed=p.seed, epoch=1,
                               minibatch=p.minibatch, alpha=p.alpha, levels=p.levels)
    assert rel(host(objs[j]), z1) < EPOCH_TOL, rel(host(objs[j]), z1)
    assert rel(host(probes[j]), q1) < EPOCH_TOL, rel(host(probes[j]), q1)
    assert abs(float(sampled[j].item()) - samp) <= MISFIT_TOL * samp
    grp.close()
    for r in recs:
        r.close()
