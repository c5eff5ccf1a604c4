"""The experiment protocol driver on the GPU: histories, stopping rules and metrics against
the oracle on a small synthetic analogue of the paper's noise study."""
import numpy as np
import pytest

from oracle import emagpie_oracle as O
from gpu_helpers import MISFIT_TOL
from paper_2511_01793_amd import synth
from paper_2511_01793_amd.protocol import MovingAverageStop, magnitude_error, reconstruct

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("method", ["rpie", "emagpie"])
def test_protocol_run_is_consistent_with_the_oracle(method):
    p = synth.make_protocol_problem(overlap=0.75, noise_percent=10.0, n=128, m=32, B=1, L=2,
                                    seed=77)
    print("case: protocol", method, p.n_pos, flush=True)
    h = reconstruct(p, method=method, max_epochs=60, floor_factor=0.9, seed=4)
    assert h["stop"] in ("floor", "moving_average", "max_epochs")
    assert h["epochs"] == len(h["residual"]) == len(h["error"]) == len(h["epoch_ms"])
    a = O.amplitudes(p.intensities)
    # the floor: Phi at the ground truth, in the precision the library holds it
    floor_ref = O.misfit(p.probe_true.astype(np.complex64), p.object_true.astype(np.complex64),
                         p.positions, a)
    assert abs(h["floor"] - floor_ref) <= MISFIT_TOL * floor_ref
    # the last residual is Phi of the returned state
    last = O.misfit(h["probe"], h["object"], p.positions, a)
    assert abs(h["residual"][-1] - last) <= MISFIT_TOL * last
    assert h["error"][-1] == pytest.approx(magnitude_error(h["object"], p.object_true), rel=1e-12)
    # the recorded stop agrees with the rules replayed on the residual history
    rule = MovingAverageStop(5, 10)
    fired = [rule.update(r) for r in h["residual"]]
    if h["stop"] == "moving_average":
        assert fired[-1] and not any(fired[:-1])
    else:
        assert not any(fired)
    if h["stop"] == "floor":
        assert h["residual"][-1] < 0.9 * h["floor"]
        assert all(r >= 0.9 * h["floor"] for r in h["residual"][:-1])
    # the reconstruction makes progress from the perturbed initial probe
    assert h["residual"][-1] < 0.5 * h["residual"][0]
