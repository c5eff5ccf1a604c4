"""emagpie_misfit_noalloc (no context, no workspace; its scratch is a fixed array of the
library's own) against emagpie_misfit on a context with FFT plan 0, through the C ABI: two
calls in a row, the second with a smaller input, bitwise equal; and against the FP64 oracle."""
import ctypes

import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import MISFIT_TOL, host, init_state, make_rec, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def case(m, n, side, photons, seed):
    step = max(1, (n - m - 2) // (side - 1))
    return problem("tiny", n=n, m=m, scan=("raster", side, step, 1), photons=photons, B=8, L=2,
                   alpha=0.05, seed=seed)


def noalloc(p, obj, probe):
    import paper_2511_01793_amd.emagpie as E
    pos = torch.from_numpy(np.ascontiguousarray(p.positions.astype(np.int32))).cuda()
    d = torch.from_numpy(p.intensities).cuda()
    out = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    st = E.lib().emagpie_misfit_noalloc(obj.shape[0], obj.shape[1], p.m, p.n_pos, pos.data_ptr(),
                                        d.data_ptr(), obj.data_ptr(), probe.data_ptr(),
                                        out.data_ptr(), E._stream())
    assert st == 0, E.last_error()
    return out


@pytest.mark.parametrize("m, big, small", [(32, (160, 7), (100, 3)), (64, (300, 6), (140, 2)),
                                           (128, (400, 5), (200, 2))])
def test_noalloc_misfit_equals_context_misfit(m, big, small):
    say("case: noalloc misfit", m, big, small)
    for (n, side), seed in ((big, 71), (small, 72)):  # second call: fewer patterns, smaller object
        p = case(m, n, side, 1e6, seed + m)
        rec = make_rec(p, fft_plan=0)
        obj, probe = init_state(p, rec)
        rec.epoch(obj, probe, 0)  # a mid-reconstruction state
        ref = rec.misfit(obj, probe)
        got = noalloc(p, obj, probe)
        torch.cuda.synchronize()
        say(m, n, p.n_pos, float(got.item()), float(ref.item()))
        assert float(got.item()) == float(ref.item())
        orc = O.misfit(host(probe), host(obj), p.positions, O.amplitudes(p.intensities))
        assert abs(float(got.item()) - orc) <= MISFIT_TOL * orc
        rec.close()


def test_noalloc_rejects_what_it_cannot_hold():
    import paper_2511_01793_amd.emagpie as E
    say("case: noalloc limits")
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    b = buf.data_ptr()
    for args, status in [((100, 100, 32, 65537), "E_SHAPE"), ((100, 100, 48, 10), "E_SHAPE"),
                         ((300, 300, 256, 10), "E_UNSUPPORTED"), ((20, 100, 32, 10), "E_SHAPE"),
                         ((100, 100, 32, 0), "E_SHAPE")]:
        st = E.lib().emagpie_misfit_noalloc(*args, b, b, b, b, b, E._stream())
        assert E.STATUS[st] == status, (args, E.last_error())
    st = E.lib().emagpie_misfit_noalloc(100, 100, 32, 10, None, b, b, b, b, E._stream())
    assert E.STATUS[st] == "E_ARG"
