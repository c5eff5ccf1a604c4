"""The C ABI's newer surfaces on the GPU: rectangular objects (Sec. 2.1 takes any n_rows x
n_cols object), device-side error reporting of the persistent epoch, many instances behind one
context, and the measured peaks of the roofline."""
import ctypes

import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import EPOCH_TOL, GRAD32_TOL, MISFIT_TOL, STEP_TOL, host, make_rec, problem, rel
from paper_2511_01793_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def rect_problem(rows=96, cols=200, m=32, step=(21, 19), photons=None, seed=5):
    """A rows x cols crop of the blob object, a raster of windows over all of it (the last
    row and column of windows flush with the far edges), intensities of the forward model."""
    rng = np.random.default_rng(seed)
    obj = synth.make_object(max(rows, cols), rng)[:rows, :cols]
    probe = synth.true_probe(m)
    rr = sorted(set(list(range(0, rows - m + 1, step[0])) + [rows - m]))
    cc = sorted(set(list(range(0, cols - m + 1, step[1])) + [cols - m]))
    pos = np.array([(r, c) for r in rr for c in cc], dtype=np.int32)
    d = synth.simulate_intensities(probe, obj, pos)
    if photons is not None:
        d = rng.poisson(d * (photons / d.sum(axis=(1, 2)).mean())).astype(np.float64)
    return dict(rows=rows, cols=cols, m=m, positions=pos, intensities=d.astype(np.float32),
                probe_init=synth.initial_probe(m).astype(np.complex64),
                object_init=np.ones((rows, cols), dtype=np.complex64))


def rect_rec(p, **kw):
    import paper_2511_01793_amd.emagpie as E
    d = torch.from_numpy(p["intensities"]).cuda()
    args = dict(minibatch=6, levels=2, alpha=0.05, path="fused", seed=9)
    args.update(kw)
    rec = E.Reconstruction(p["positions"], d, (p["rows"], p["cols"]), **args)
    obj = torch.from_numpy(p["object_init"]).cuda()
    probe = torch.from_numpy(p["probe_init"]).cuda()
    rec.normalize_probe(probe)
    return rec, obj, probe


# ------------------------------------------------------------------ rectangular objects

@pytest.mark.parametrize("path, shape, rows, cols", [("fused", 0, 96, 200), ("fused", 5, 96, 200),
                                                     ("plain", 2, 150, 70), ("persistent", 0, 96, 200)])
def test_rectangular_object_step_and_epoch_parity(path, shape, rows, cols):
    p = rect_problem(rows, cols)
    a = O.amplitudes(p["intensities"])
    say("case: rectangular", path, shape, rows, cols, len(p["positions"]))
    rec, obj, probe = rect_rec(p, path=path, finalize_shape=shape)
    rec.epoch(obj, probe, 0)  # away from the phase-free initial guess
    torch.cuda.synchronize()
    perm = O.permutation(9, 1, len(p["positions"]))
    idx = perm[:6]
    z0, q0 = host(obj), host(probe)
    rec.step(obj, probe, idx)
    torch.cuda.synchronize()
    q1, z1, info = O.step_minibatch(q0, z0, p["positions"], a, idx, alpha=0.05, levels=2)
    assert rel(host(obj), z1) < STEP_TOL and rel(host(probe), q1) < STEP_TOL
    # untouched pixels keep their bits
    zt = host(obj)
    assert np.array_equal(zt[~info["touched"]], z0[~info["touched"]])
    z0, q0 = host(obj), host(probe)
    rec.epoch(obj, probe, 2)
    torch.cuda.synchronize()
    q1, z1, _ = O.run_epoch(q0, z0, p["positions"], a, seed=9, epoch=2, minibatch=6, alpha=0.05,
                            levels=2)
    assert rel(host(obj), z1) < EPOCH_TOL and rel(host(probe), q1) < EPOCH_TOL
    phi = float(rec.misfit(obj, probe).item())
    ref = O.misfit(host(probe), host(obj), p["positions"], a)
    assert abs(phi - ref) <= MISFIT_TOL * ref
    rec.close()


def test_rectangular_object_gradient():
    p = rect_problem(80, 224, step=(16, 24))
    say("case: rectangular grad", len(p["positions"]))
    rec, obj, probe = rect_rec(p)
    rec.epoch(obj, probe, 0)
    gz, gq, phi = rec.grad(obj, probe)
    torch.cuda.synchronize()
    rz, rq, rphi = O.gradients(host(probe), host(obj), p["positions"], O.amplitudes(p["intensities"]))
    assert gz.shape == (80, 224)
    assert rel(host(gz), rz) < GRAD32_TOL and rel(host(gq), rq) < GRAD32_TOL
    assert abs(float(phi.item()) - rphi) <= MISFIT_TOL * rphi
    rec.close()



@pytest.mark.parametrize("plan", [0, 1])
def test_rectangular_object_misfit_at_m128(plan):
    """m = 128 on a rectangular object: the two-workgroups-per-CU misfit kernel of each split
    (plan 0: 16 x 8, plan 1: 8 x 16) against the oracle, and the allocation-free misfit
    bitwise equal to the plan-0 context."""
    import paper_2511_01793_amd.emagpie as E
    p = rect_problem(200, 330, m=128, step=(24, 29), photons=1e6, seed=7)
    a = O.amplitudes(p["intensities"])
    say("case: rectangular misfit m=128", plan, len(p["positions"]))
    rec, obj, probe = rect_rec(p, minibatch=8, levels=3, fft_plan=plan)
    rec.epoch(obj, probe, 0)
    phi = float(rec.misfit(obj, probe).item())
    torch.cuda.synchronize()
    ref = O.misfit(host(probe), host(obj), p["positions"], a)
    assert abs(phi - ref) <= MISFIT_TOL * ref
    if plan == 0:
        pos = torch.from_numpy(np.ascontiguousarray(p["positions"])).cuda()
        d = torch.from_numpy(p["intensities"]).cuda()
        out = torch.full((), -1.0, dtype=torch.float64, device="cuda")
        st = E.lib().emagpie_misfit_noalloc(200, 330, 128, len(p["positions"]), pos.data_ptr(),
                                            d.data_ptr(), obj.data_ptr(), probe.data_ptr(),
                                            out.data_ptr(), E._stream())
        assert st == 0, E.last_error()
        torch.cuda.synchronize()
        assert float(out.item()) == phi
    rec.close()


# ------------------------------------------------------------------ device-side errors

def test_persistent_barrier_timeout_is_reported_by_the_next_call():
    # The host makes every grid barrier of a persistent epoch wait for one arrival more than
    # the grid makes, with a short spin bound: each wait gives up after 2000 polls, so the
    # kernel still runs to its end, and it raises the device error flag.  The next call must
    # return E_HIP (and do nothing else); afterwards the context works again, bitwise as the
    # fused path.
    import paper_2511_01793_amd.emagpie as E
    p = problem("tiny", n=100, m=32, scan=("raster", 5, 16, 1), photons=None, B=7, L=2,
                alpha=0.05, seed=11)
    say("case: persistent barrier timeout")
    rec = make_rec(p, path="persistent", seed=3)
    ref = make_rec(p, path="fused", seed=3)
    obj = torch.from_numpy(p.object_init).cuda()
    probe = torch.from_numpy(p.probe_init).cuda()
    rec.normalize_probe(probe)
    rec.debug_barrier(spin_limit=2000, target_skew=1)
    rec.epoch(obj, probe, 0)
    torch.cuda.synchronize()
    with pytest.raises(E.EmagpieError) as ei:
        rec.misfit(obj, probe)
    assert ei.value.name == "E_HIP" and "grid barrier" in str(ei.value)
    assert "grid barrier" in rec.last_error
    # reported once; the barrier counter is re-zeroed before the next persistent epoch
    rec.debug_barrier(0, 0)
    o1 = torch.from_numpy(p.object_init).cuda()
    q1 = torch.from_numpy(p.probe_init).cuda()
    rec.normalize_probe(q1)
    o2, q2 = o1.clone(), q1.clone()
    for e in range(2):
        rec.epoch(o1, q1, e)
        ref.epoch(o2, q2, e)
    torch.cuda.synchronize()
    float(rec.misfit(o1, q1).item())  # no error pending
    assert torch.equal(o1, o2) and torch.equal(q1, q2)
    rec.close()
    ref.close()


# ------------------------------------------------------------------ many instances, one context

def test_many_context_equals_members_alone_bitwise():
    import paper_2511_01793_amd.emagpie as E
    specs = [
        dict(n=100, m=32, scan=("raster", 5, 16, 1), photons=None, B=7, L=2, seed=31),
        dict(n=160, m=64, scan=("raster", 4, 30, 1), photons=1e6, B=5, L=3, seed=32),
        dict(n=130, m=32, scan=("raster", 7, 15, 1), photons=1e5, B=10, L=1, seed=33),
    ]
    ps = [problem("tiny", alpha=0.05, **s) for s in specs]
    say("case: many-context")
    rect = rect_problem(96, 200)
    probs = [dict(positions=p.positions, intensities=torch.from_numpy(p.intensities).cuda(), n=p.n,
                  minibatch=p.minibatch, levels=p.levels, alpha=0.05, path="fused", seed=40 + i)
             for i, p in enumerate(ps)]
    probs.append(dict(positions=rect["positions"], intensities=torch.from_numpy(rect["intensities"]).cuda(),
                      n=(96, 200), minibatch=6, levels=2, alpha=0.05, path="fused", seed=43))
    inits = [(p.object_init, p.probe_init) for p in ps] + [(rect["object_init"], rect["probe_init"])]
    many = E.Many(probs)
    objs, probes = [], []
    for mem, (o0, q0) in zip(many.members, inits):
        o, q = torch.from_numpy(o0).cuda(), torch.from_numpy(q0).cuda()
        mem.normalize_probe(q)
        objs.append(o)
        probes.append(q)
    sampled = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    for e in range(2):
        many.epoch(objs, probes, e, sampled=sampled)
    phis = [float(mem.misfit(o, q).item()) for mem, o, q in zip(many.members, objs, probes)]
    torch.cuda.synchronize()
    # a single-instance call on the many-context itself is an argument error
    st = E.lib().emagpie_epoch(many._ctx, objs[0].data_ptr(), probes[0].data_ptr(), 0, None, None,
                               E._stream())
    assert E.STATUS[st] == "E_ARG" and "emagpie_init_many" in E.last_error(many._ctx)
    for i, (pr, (o0, q0)) in enumerate(zip(probs, inits)):
        args = {k: v for k, v in pr.items() if k not in ("positions", "intensities", "n")}
        rec = E.Reconstruction(pr["positions"], pr["intensities"], pr["n"], **args)
        o, q = torch.from_numpy(o0).cuda(), torch.from_numpy(q0).cuda()
        rec.normalize_probe(q)
        s = torch.zeros((), dtype=torch.float64, device="cuda")
        for e in range(2):
            s.zero_()
            rec.epoch(o, q, e, sampled=s)
        torch.cuda.synchronize()
        assert torch.equal(o, objs[i]) and torch.equal(q, probes[i]), i
        assert float(s.item()) == float(sampled[i].item()), i
        assert float(rec.misfit(o, q).item()) == phis[i], i
        rec.close()
    many.close()


# ------------------------------------------------------------------ measured peaks

def test_measured_peaks_are_plausible():
    import paper_2511_01793_amd.emagpie as E
    say("case: peaks")
    pk = E.measure_peaks(1 << 30, reps=3)
    say(pk)
    # a 1 GiB copy does not fit the 256 MB Infinity Cache, so it runs at HBM speed: well
    # above any PCIe rate and below the 8 TB/s of HBM3E; an FMA rate of the right order for
    # 256 CUs at about 2.4 GHz with 64 FP32 lanes each
    assert 1000.0 < pk["copy_GBs"] < 8000.0
    assert 20.0 < pk["fp32_fma_TFLOPs"] < 170.0
