"""Kernel plans and the autotuner: every FFT plan and finalize shape against the oracle,
bitwise identities between plans that share a radix split, and tuning with its cache."""
import json

import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import (EPOCH_TOL, GRAD32_TOL, MISFIT_TOL, STEP_TOL, amps, host, init_state,
                         problem, rel)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2511_01793_amd.emagpie")


def say(*a):
    print(*a, flush=True)


def small(m, L=2, B=6, side=5, photons=1e6, seed=31):
    n = 3 * m + 4
    step = max(1, (n - m - 2) // (side - 1))
    return problem("tiny", n=n, m=m, scan=("raster", side, step, 1), photons=photons, B=B, L=L,
                   alpha=0.05, seed=seed)


def rec_for(p, **kw):
    d = torch.from_numpy(p.intensities).cuda()
    base = dict(minibatch=p.minibatch, levels=p.levels, alpha=p.alpha, alpha_z=p.alpha_z, seed=3,
                path="fused")
    base.update(kw)
    return E.Reconstruction(p.positions, d, p.n, **base)


def n_plans(m):
    return E.plan_describe(m)["fft_plans"]


CASES = [(m, v) for m in (32, 64, 128) for v in range({32: 2, 64: 4, 128: 3}[m])]


@pytest.mark.parametrize("m, v", CASES)
def test_every_fft_plan_matches_the_oracle(m, v):
    assert v < n_plans(m)
    L = 3 if m == 128 else 2
    p = small(m, L=L)
    say("case: plan", m, v, L)
    rec = rec_for(p, fft_plan=v)
    assert rec.plan["fft_plan"] == v and rec.plan["tuned"] == "fixed"
    obj, probe = init_state(p, rec)
    a = amps(p)
    rec.epoch(obj, probe, 40)  # leave the phase-free initial guess
    torch.cuda.synchronize()
    idx = np.arange(1, 1 + p.minibatch, dtype=np.int32)
    z0, q0 = host(obj), host(probe)
    sampled = torch.zeros((), dtype=torch.float64, device="cuda")
    rec.step(obj, probe, idx, sampled=sampled)
    phi = rec.misfit(obj, probe)
    torch.cuda.synchronize()
    q1, z1, info = O.step_minibatch(q0, z0, p.positions, a, idx, alpha=p.alpha, levels=L)
    assert rel(host(obj), z1) < STEP_TOL, rel(host(obj), z1)
    assert rel(host(probe), q1) < STEP_TOL, rel(host(probe), q1)
    s = info["sampled_misfit"]
    assert abs(float(sampled.item()) - s) <= MISFIT_TOL * s
    ref = O.misfit(host(probe), host(obj), p.positions, a)
    assert abs(float(phi.item()) - ref) <= MISFIT_TOL * ref
    gz, gq, _ = rec.grad(obj, probe)
    torch.cuda.synchronize()
    rz, rq, _ = O.gradients(host(probe), host(obj), p.positions, a)
    assert rel(host(gz), rz) < GRAD32_TOL and rel(host(gq), rq) < GRAD32_TOL
    rec.close()


def run_epochs(p, epochs=2, **kw):
    rec = rec_for(p, **kw)
    obj, probe = init_state(p, rec)
    for e in range(epochs):
        rec.epoch(obj, probe, e)
    torch.cuda.synchronize()
    plan = rec.plan
    rec.close()
    return obj, probe, plan


@pytest.mark.parametrize("m, va, vb", [(64, 0, 3), (128, 0, 2)])
@pytest.mark.parametrize("path", ["fused", "persistent", "plain"])
def test_plans_with_one_radix_split_are_bitwise_identical(m, va, vb, path):
    da, db = E.plan_describe(m, va), E.plan_describe(m, vb)
    # (64, 3) keeps the tile in registers through each dimension's passes
    # (cross-lane transposes); (128, 2) runs the LDS passes with half the threads
    assert (da["r1"], da["r2"]) == (db["r1"], db["r2"]) and va != vb
    p = small(m, L=2)
    say("case: same split", m, va, vb, path)
    oa, qa, _ = run_epochs(p, fft_plan=va, path=path)
    ob, qb, _ = run_epochs(p, fft_plan=vb, path=path)
    assert torch.equal(oa, ob) and torch.equal(qa, qb)


@pytest.mark.parametrize("m", [32, 64, 128])
def test_finalize_shapes_are_bitwise_identical(m):
    p = small(m, L=2, B=9)
    say("case: finalize shapes", m)
    ref = run_epochs(p, finalize_shape=0)
    for f in range(1, 12):  # 4..7, 8..11: the same tiles in the banded and rows-per-XCD orders
        o, q, plan = run_epochs(p, finalize_shape=f)
        assert plan["finalize_shape"] == f
        assert torch.equal(o, ref[0]) and torch.equal(q, ref[1]), f


def test_autotune_and_cache(tmp_path):
    p = small(64, L=2, B=8, side=7)
    cache = str(tmp_path / "tune.jsonl")
    say("case: autotune")
    rec = rec_for(p, fft_plan=E.TUNE, finalize_shape=E.TUNE, path="auto", tune_cache=cache)
    plan = rec.plan
    assert plan["tuned"] == "timed"
    assert len(plan["fft_us"]) == n_plans(64) and all(t > 0 for t in plan["fft_us"])
    assert len(plan["fin_us"]) == 12 and all(t > 0 for t in plan["fin_us"])
    assert set(plan["path_ms"]) == {"fused", "graph"}
    assert plan["fft_us"][plan["fft_plan"]] == min(plan["fft_us"])
    # the two fastest shapes alone are compared on whole epochs
    assert plan["fin_us"][plan["finalize_shape"]] <= sorted(plan["fin_us"])[1]
    assert plan["path_ms"][plan["path"]] == min(plan["path_ms"].values())
    # the tuned context computes the method: epoch parity with the oracle
    obj, probe = init_state(p, rec)
    a = amps(p)
    for e in range(2):
        z0, q0 = host(obj), host(probe)
        rec.epoch(obj, probe, e)
        torch.cuda.synchronize()
        q1, z1, _ = O.run_epoch(q0, z0, p.positions, a, seed=3, epoch=e, minibatch=8,
                                alpha=p.alpha, levels=2)
        assert rel(host(obj), z1) < EPOCH_TOL and rel(host(probe), q1) < EPOCH_TOL
    phi = float(rec.misfit(obj, probe).item())
    ref = O.misfit(host(probe), host(obj), p.positions, a)
    assert abs(phi - ref) <= MISFIT_TOL * ref
    rec.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert entry["fft_plan"] == plan["fft_plan"] and entry["finalize_shape"] == plan["finalize_shape"]
    # a second context with the same shape reads the cache and times nothing
    rec2 = rec_for(p, fft_plan=E.TUNE, finalize_shape=E.TUNE, path="auto", tune_cache=cache)
    p2 = rec2.plan
    assert p2["tuned"] == "cache" and p2["fft_plan"] == plan["fft_plan"]
    assert p2["finalize_shape"] == plan["finalize_shape"] and p2["path"] == plan["path"]
    o2, q2 = init_state(p, rec2)
    z0, q0 = host(o2), host(q2)
    rec2.epoch(o2, q2, 0)
    torch.cuda.synchronize()
    q1, z1, _ = O.run_epoch(q0, z0, p.positions, a, seed=3, epoch=0, minibatch=8, alpha=p.alpha,
                            levels=2)
    assert rel(host(o2), z1) < EPOCH_TOL and rel(host(q2), q1) < EPOCH_TOL
    rec2.close()
    assert len(open(cache).read().splitlines()) == 1


def test_group_members_with_different_plans_match_individual_runs():
    probs = [small(64, L=2, B=5, seed=41), small(64, L=2, B=7, seed=42), small(32, L=2, B=4, seed=43)]
    plans = [dict(fft_plan=1, finalize_shape=2), dict(fft_plan=3, finalize_shape=1),
             dict(fft_plan=1, finalize_shape=3)]
    say("case: group plans")
    recs = [rec_for(p, **k) for p, k in zip(probs, plans)]
    states = [init_state(p, r) for p, r in zip(probs, recs)]
    solo = []
    for p, k in zip(probs, plans):
        o, q, _ = run_epochs(p, epochs=2, **k)
        solo.append((o, q))
    g = E.Group(recs)
    for e in range(2):
        g.epoch([s[0] for s in states], [s[1] for s in states], e)
    torch.cuda.synchronize()
    for (o, q), (so, sq) in zip(states, solo):
        assert torch.equal(o, so) and torch.equal(q, sq)
    g.close()
    for r in recs:
        r.close()


@pytest.mark.parametrize("path", ["fused", "chain"])
def test_phase_memory_in_the_register_pass_plan(path):
    """Zero-bin phase memory through plan (64, 3), whose projection runs in the column phase
    of the register passes: the first visit of pattern k stores its phases, the second (a
    constant exit wave: every bin but DC exactly zero) takes them back.  Bitwise the LDS plan
    with the same split, and the oracle to the step bar."""
    p = small(64, L=1)
    say("case: phase memory, register passes", path)
    rng = np.random.default_rng(17)
    k = 3
    Qr = (rng.standard_normal((p.m, p.m)) + 1j * rng.standard_normal((p.m, p.m))).astype(np.complex64)
    zr = (rng.standard_normal((p.n, p.n)) + 1j * rng.standard_normal((p.n, p.n))).astype(np.complex64)
    Qc = np.full((p.m, p.m), 0.6 - 0.2j, dtype=np.complex64)
    zc = np.full((p.n, p.n), 1.0 + 0.1j, dtype=np.complex64)
    a = amps(p)
    mem = np.ones((p.n_pos, p.m, p.m), complex)
    O.step_minibatch(Qr.astype(complex), zr.astype(complex), p.positions, a, [k], alpha=p.alpha,
                     levels=p.levels, phase_mem=mem)
    q_ref, z_ref, _ = O.step_minibatch(Qc.astype(complex), zc.astype(complex), p.positions, a, [k],
                                       alpha=p.alpha, levels=p.levels, phase_mem=mem)
    out = {}
    for v in (0, 3):
        rec = rec_for(p, fft_plan=v, path=path, zero_phase_memory=True, minibatch=1)
        obj, probe = torch.from_numpy(zr).cuda(), torch.from_numpy(Qr).cuda()
        rec.step(obj, probe, [k])
        obj.copy_(torch.from_numpy(zc))
        probe.copy_(torch.from_numpy(Qc))
        rec.step(obj, probe, [k])
        torch.cuda.synchronize()
        out[v] = (obj, probe)
        rec.close()
    assert torch.equal(out[3][0], out[0][0]) and torch.equal(out[3][1], out[0][1])
    zg, qg = host(out[3][0]), host(out[3][1])
    assert rel(zg, z_ref) < STEP_TOL and rel(qg, q_ref) < STEP_TOL, (rel(zg, z_ref), rel(qg, q_ref))


@pytest.mark.parametrize("L, joint, update_probe", [(1, True, True), (3, True, True),
                                                    (2, False, True), (2, True, False)])
def test_register_pass_plan_in_every_mode(L, joint, update_probe):
    """Plan (64, 3) against the LDS plan with the same split, bit for bit, for each multigrid
    depth, the rPIE step (no joint step) and the non-blind step (probe fixed); and its
    MAGPIE z+ output (mg_cycle)."""
    p = small(64, L=L)
    say("case: register passes", L, joint, update_probe)
    out = {}
    for v in (0, 3):
        o, q, _ = run_epochs(p, epochs=2, fft_plan=v, joint_step=joint, update_probe=update_probe)
        rec = rec_for(p, fft_plan=v, joint_step=joint, update_probe=update_probe)
        zp = rec.mg_cycle(o.clone(), q.clone(), np.arange(p.minibatch, dtype=np.int32))
        torch.cuda.synchronize()
        out[v] = (o, q, zp)
        rec.close()
    for a, b in zip(out[0], out[3]):
        assert torch.equal(a, b)
