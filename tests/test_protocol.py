"""Host logic of the experiment protocol (Sec. 4.1) and the protocol input generators."""
import math

import numpy as np
import pytest

from paper_2511_01793_amd import synth
from paper_2511_01793_amd.protocol import MovingAverageStop, below_floor, magnitude_error


def brute_force_stop(res, w, p):
    """Stop index (1-based) by the reading: rbar_t for t >= w; a check at t > w fails when
    rbar_t >= min_{w <= s < t} rbar_s; stop after p consecutive failures."""
    r = np.asarray(res, np.float64)
    for t in range(w + p, len(r) + 1):
        ok = True
        for c in range(t - p + 1, t + 1):
            rb = r[c - w:c].mean()
            prev = min(r[s - w:s].mean() for s in range(w, c))
            if rb < prev:
                ok = False
                break
        if ok:
            return t
    return None


def run_rule(res, w, p):
    rule = MovingAverageStop(w, p)
    for t, x in enumerate(res, 1):
        if rule.update(x):
            return t
    return None


def test_strictly_decreasing_never_stops():
    assert run_rule(np.linspace(10, 1, 200), 5, 10) is None


def test_constant_stops_after_window_plus_patience():
    for w, p in [(5, 10), (1, 1), (3, 2), (5, 5)]:
        assert run_rule(np.ones(100), w, p) == w + p


def test_improvement_resets_patience():
    res = [10, 9, 8, 7, 6] + [6] * 9 + [1] + [6] * 30
    # the drop at t = 15 enters every window through t = 19 and leaves at t = 20
    t = run_rule(res, 5, 10)
    assert t == brute_force_stop(res, 5, 10)
    assert t > 15 + 10 - 1


@pytest.mark.parametrize("seed", range(12))
def test_rule_equals_brute_force_on_noisy_curves(seed):
    rng = np.random.default_rng(seed)
    n = 120
    base = 100 * np.exp(-np.arange(n) / rng.uniform(5, 40)) + rng.uniform(0, 5)
    res = base * (1 + rng.uniform(0.0, 0.2) * rng.standard_normal(n))
    for w, p in [(5, 10), (5, 5), (2, 3)]:
        assert run_rule(res, w, p) == brute_force_stop(res, w, p)


def test_rule_rejects_bad_parameters():
    with pytest.raises(ValueError):
        MovingAverageStop(0, 5)
    with pytest.raises(ValueError):
        MovingAverageStop(5, 0)


def test_floor_rule():
    assert below_floor(0.89, 1.0) and not below_floor(0.9, 1.0) and not below_floor(1.2, 1.0)
    assert below_floor(0.5, 1.0, factor=0.6)


def test_magnitude_error_closed_forms():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    # phase-blind: any pixelwise phase leaves the error at zero
    assert magnitude_error(z * np.exp(1j * rng.uniform(0, 6, z.shape)), z) < 1e-12
    # scaled magnitudes: || c|z| - |z| || = |c - 1| ||z||
    assert abs(magnitude_error(1.5 * z, z) - 0.5 * np.linalg.norm(z)) < 1e-9
    assert magnitude_error(np.zeros((3, 3)), np.ones((3, 3))) == pytest.approx(3.0)
    # the scale-aligned form removes a global factor exactly, and is never larger
    assert magnitude_error(2.5 * z, z, align_scale=True) < 1e-9
    w = z + 0.3 * rng.standard_normal(z.shape)
    assert magnitude_error(w, z, align_scale=True) <= magnitude_error(w, z) + 1e-12
    c = np.linspace(0.5, 1.5, 2001)
    brute = min(np.linalg.norm(ci * np.abs(w) - np.abs(z)) for ci in c)
    assert abs(magnitude_error(w, z, align_scale=True) - brute) < 1e-4 * brute


def test_photon_scale_hits_target_noise_percent():
    rng = np.random.default_rng(1)
    clean = rng.gamma(0.5, 2.0, size=(40, 32, 32))
    for pct in (5.0, 10.0, 20.0):
        s = synth.photon_scale_for_noise(clean, pct)
        noisy = rng.poisson(clean * s)
        got = synth.noise_percent(noisy, clean * s)
        assert abs(got - pct) < 0.02 * pct, (pct, got)


def test_overlap_positions_step_and_count():
    rng = np.random.default_rng(2)
    for o, side in [(0.5, 7), (0.75, 13), (0.875, 25)]:
        pos = synth.overlap_positions(512, 128, o, rng, jitter=0)
        assert pos.shape == (side * side, 2)
        step = int(round(128 * (1 - o)))
        assert np.all(np.diff(pos[:side, 1]) == step)
        assert pos.min() >= 0 and pos.max() <= 512 - 128


def test_zone_plate_probe_shape():
    q = synth.zone_plate_probe(128)
    a = np.abs(q)
    assert a.max() == pytest.approx(1.0)
    c = 64
    # radially symmetric about the window centre: transposes and mirrors agree
    sub = a[c - 40:c + 41, c - 40:c + 41]
    assert np.allclose(sub, sub.T, atol=1e-12)
    assert np.allclose(sub, sub[::-1, ::-1], atol=1e-12)
    # most of the window is dim (the ring-structured central disc holds the energy)
    assert (a > 0.1).mean() < 0.5
    edge = np.concatenate([a[0], a[-1], a[:, 0], a[:, -1]])
    assert edge.mean() < 0.05


def test_perturbed_initial_probe_components():
    m = 64
    q = synth.zone_plate_probe(m)
    rng = np.random.default_rng(3)
    # no blur, ramp, aberration or noise: the magnitude of the ground truth, zero phase
    q0 = synth.perturbed_initial_probe(q, rng, sigma_amp=0.0, ramp=0.0, defocus=0.0, astig=0.0,
                                       noise=0.0)
    assert np.allclose(q0, np.abs(q), atol=1e-12)
    # ramp only: the phase of a constant magnitude changes by `ramp` rad edge to edge
    flat = np.ones((m, m), complex)
    q1 = synth.perturbed_initial_probe(flat, np.random.default_rng(4), sigma_amp=0.0, ramp=7.0,
                                       defocus=0.0, astig=0.0, noise=0.0)
    ph = np.angle(q1 * np.conj(q1[m // 2, m // 2]))
    gy, gx = np.gradient(np.unwrap(np.unwrap(ph, axis=0), axis=1))
    slope = math.hypot(gx.mean(), gy.mean()) * (m - 1) / 2.0
    assert abs(slope - 3.5) < 1e-6
    # blur preserves the mean magnitude (transfer function 1 at zero frequency)
    q2 = synth.perturbed_initial_probe(q, rng, ramp=0.0, defocus=0.0, astig=0.0, noise=0.0)
    assert abs(np.abs(q2).sum() - np.abs(q).sum()) < 1e-6 * np.abs(q).sum()
    # full recipe: 1% noise relative to the rms magnitude
    q3 = synth.perturbed_initial_probe(q, np.random.default_rng(5))
    q4 = synth.perturbed_initial_probe(q, np.random.default_rng(5), noise=0.0)
    rms = np.sqrt(np.mean(np.abs(q4) ** 2))
    assert abs(np.sqrt(np.mean(np.abs(q3 - q4) ** 2)) / rms - 0.01) < 0.002
