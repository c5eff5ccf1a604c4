"""Seeded synthetic ptychography workloads (inputs only).

This module builds the inputs that both the HIP path and the FP64 oracle
consume: a ground-truth object and probe, scan positions, and the measured
far-field intensities of the simulated experiment.  It holds none of the
reconstruction method's arithmetic (no revised exit wave, no surrogate step,
no multigrid); the only transform it applies is the forward model that
produces the data, d_k = |F(Q* . P_k z*)|^2 (+ Poisson noise), of Sec. 2.1.

Recipe (the paper's Baboon/Cameraman images, zone-plate probe and beamline
data are not available; these seeded stand-ins take their place):

* object: two independent sums of 20 Gaussian blobs (centre ~ U[0, n)^2,
  width ~ U[n/40, n/10], weight ~ U[-1, 1]), each min-max normalised to
  [0, 1]; |z*| = 0.8 + 0.2 f_A, arg z* = pi (f_phi - 1/2);
* true probe: Gaussian of width sigma (6 px for m = 32, 0.1875 m otherwise)
  times a quadratic defocus phase exp(i rho^2 / sigma^2), centred on the
  window centre ((m-1)/2, (m-1)/2);
* initial probe: a broader (1.5 sigma) zero-phase Gaussian, later scaled by
  the dp_avg rule of Sec. 4.1; initial object z = 1 (Sec. 4.1);
* positions: jittered raster or Fermat spiral, integer top-left corners
  clamped to [0, n - m];
* intensities: computed in float64, stored as float32, unshifted (DC at
  [0, 0]); Poisson configurations first scale the true probe so that the
  mean photon count per pattern equals the target, then draw counts.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "make_object",
    "true_probe",
    "initial_probe",
    "jittered_initial_probe",
    "raster_positions",
    "fermat_positions",
    "simulate_intensities",
    "make_problem",
    "CONFIGS",
    "textured_object",
    "zone_plate_probe",
    "perturbed_initial_probe",
    "overlap_positions",
    "photon_scale_for_noise",
    "make_protocol_problem",
]


def make_object(n: int, rng: np.random.Generator, n_blobs: int = 20) -> np.ndarray:
    """Smooth complex test object, amplitude in [0.8, 1] and phase in [-pi/2, pi/2]."""
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)

    def blob_sum() -> np.ndarray:
        f = np.zeros((n, n))
        for _ in range(n_blobs):
            cy, cx = rng.uniform(0, n, size=2)
            s = rng.uniform(n / 40.0, n / 10.0)
            w = rng.uniform(-1.0, 1.0)
            f += w * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * s * s))
        f -= f.min()
        mx = f.max()
        return f / mx if mx > 0 else f

    fa = blob_sum()
    fp = blob_sum()
    return (0.8 + 0.2 * fa) * np.exp(1j * np.pi * (fp - 0.5))


def probe_sigma(m: int) -> float:
    return 6.0 if m == 32 else 0.1875 * m


def true_probe(m: int, sigma: float | None = None) -> np.ndarray:
    """Defocused Gaussian probe (float64 complex)."""
    s = probe_sigma(m) if sigma is None else sigma
    c = (m - 1) / 2.0
    yy, xx = np.mgrid[0:m, 0:m].astype(np.float64)
    rho2 = (yy - c) ** 2 + (xx - c) ** 2
    return np.exp(-rho2 / (2.0 * s * s)) * np.exp(1j * rho2 / (s * s))


def initial_probe(m: int, sigma: float | None = None) -> np.ndarray:
    """Broader zero-phase Gaussian guess (before the dp_avg scaling)."""
    s = 1.5 * (probe_sigma(m) if sigma is None else sigma)
    c = (m - 1) / 2.0
    yy, xx = np.mgrid[0:m, 0:m].astype(np.float64)
    return np.exp(-((yy - c) ** 2 + (xx - c) ** 2) / (2.0 * s * s)).astype(np.complex128)


def jittered_initial_probe(probe_init: np.ndarray, eps: float, seed: int) -> np.ndarray:
    """The initial probe times (1 + eps g), g complex standard normal per pixel drawn from
    default_rng(seed) (real and imaginary parts each N(0, 1/2)); complex64 like probe_init.
    eps = 0 returns probe_init unchanged.  Seeded variants of one start, for the spread of
    the time to a fixed misfit."""
    if eps == 0.0:
        return probe_init.copy()
    rng = np.random.default_rng(seed)
    shape = probe_init.shape
    g = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)
    return (probe_init.astype(np.complex128) * (1.0 + eps * g)).astype(probe_init.dtype)


def raster_positions(n: int, m: int, side: int, step: int, jitter: int,
                     rng: np.random.Generator) -> np.ndarray:
    """side x side raster, integer jitter in {-J..J}, clamped to [0, n-m]."""
    off = (n - m - (side - 1) * step) // 2
    pos = np.empty((side * side, 2), dtype=np.int64)
    k = 0
    for i in range(side):
        for j in range(side):
            pos[k] = (off + i * step, off + j * step)
            k += 1
    if jitter > 0:
        pos += rng.integers(-jitter, jitter + 1, size=pos.shape)
    return np.clip(pos, 0, n - m).astype(np.int32)


def fermat_positions(n: int, m: int, count: int) -> np.ndarray:
    """Fermat spiral r_i = c sqrt(i), theta_i = i * 137.5078 deg, centred."""
    c = ((n - m) / 2.0 - 1.0) / math.sqrt(count)
    i = np.arange(count, dtype=np.float64)
    r = c * np.sqrt(i)
    th = np.deg2rad(137.5078) * i
    ctr = (n - m) / 2.0
    pos = np.stack([np.rint(ctr + r * np.sin(th)), np.rint(ctr + r * np.cos(th))], axis=1)
    return np.clip(pos, 0, n - m).astype(np.int32)


def simulate_intensities(probe: np.ndarray, obj: np.ndarray, positions: np.ndarray,
                         chunk: int = 512) -> np.ndarray:
    """Noiseless far-field intensities |F(Q . P_k z)|^2 in float64 (forward model, Sec. 2.1)."""
    m = probe.shape[0]
    out = np.empty((positions.shape[0], m, m), dtype=np.float64)
    for s in range(0, positions.shape[0], chunk):
        p = positions[s:s + chunk]
        stack = np.stack([obj[r:r + m, c:c + m] for r, c in p]) * probe
        out[s:s + chunk] = np.abs(np.fft.fft2(stack)) ** 2
    return out


@dataclasses.dataclass
class Problem:
    """One synthetic reconstruction problem; arrays in the dtypes both paths consume."""
    name: str
    n: int
    m: int
    positions: np.ndarray        # (N, 2) int32 (row, col) top-left
    intensities: np.ndarray      # (N, m, m) float32, unshifted
    probe_true: np.ndarray       # (m, m) complex128 (photon-scaled)
    object_true: np.ndarray      # (n, n) complex128
    probe_init: np.ndarray       # (m, m) complex64, NOT yet dp_avg-normalised
    object_init: np.ndarray      # (n, n) complex64, all ones
    minibatch: int
    levels: int
    alpha: float
    alpha_z: float
    epochs: int
    seed: int
    photons: float | None
    noiseless: np.ndarray | None = None   # float64 noiseless intensities (small configs only)

    @property
    def n_pos(self) -> int:
        return int(self.positions.shape[0])


# name -> generator parameters (see module docstring)
CONFIGS = {
    # plain single level: 128^2 object, 32^2 probe, 10x10 raster step 8 jitter 1, noiseless
    "c1": dict(n=128, m=32, scan=("raster", 10, 8, 1), photons=None, B=10, L=1, alpha=0.01, epochs=50, idx=1),
    # two-level multigrid: 512^2 object, 64^2 probe, 40x40 raster step 10 jitter 2, 1e6 photons
    "c2": dict(n=512, m=64, scan=("raster", 40, 10, 2), photons=1e6, B=64, L=2, alpha=0.05, epochs=100, idx=2),
    # batching: 1024^2 object, 128^2 probe, Fermat spiral of 10000, 1e7 photons, 3 levels
    "c3": dict(n=1024, m=128, scan=("fermat", 10000), photons=1e7, B=256, L=3, alpha=0.05, epochs=20, idx=3),
    # differentiation: 256^2 object, 64^2 probe, 20x20 raster step 10, noiseless
    "c4": dict(n=256, m=64, scan=("raster", 20, 10, 0), photons=None, B=400, L=1, alpha=0.05, epochs=0, idx=4),
    # 256^2 patterns (the crop size of the paper's beamline data): 31 x 31 raster, step 24,
    # jitter 2, over a 1024^2 object, 1e8 photons, minibatch 32, 2 levels
    "c6": dict(n=1024, m=256, scan=("raster", 31, 24, 2), photons=1e8, B=32, L=2, alpha=0.05, epochs=0, idx=6),
}


def make_problem(name: str, *, n: int | None = None, m: int | None = None, scan=None,
                 photons: float | None | str = "cfg", B: int | None = None, L: int | None = None,
                 alpha: float | None = None, seed: int | None = None,
                 keep_noiseless: bool = False) -> Problem:
    """Build a named configuration (optionally overriding its parameters)."""
    cfg = dict(CONFIGS[name]) if name in CONFIGS else dict(
        n=64, m=16, scan=("raster", 4, 12, 1), photons=None, B=4, L=1, alpha=0.05, epochs=10, idx=9)
    n = cfg["n"] if n is None else n
    m = cfg["m"] if m is None else m
    scan = cfg["scan"] if scan is None else scan
    photons = cfg["photons"] if photons == "cfg" else photons
    B = cfg["B"] if B is None else B
    L = cfg["L"] if L is None else L
    alpha = cfg["alpha"] if alpha is None else alpha
    seed = 1000 + cfg["idx"] if seed is None else seed
    rng = np.random.default_rng(seed)

    obj = make_object(n, rng)
    probe = true_probe(m)
    if scan[0] == "raster":
        pos = raster_positions(n, m, scan[1], scan[2], scan[3], rng)
    else:
        pos = fermat_positions(n, m, scan[1])
    d = None
    if photons is not None:
        # mean photon count per pattern: by Parseval sum |F psi|^2 = m^2 sum |psi|^2
        energy = np.mean([np.sum(np.abs(probe * obj[r:r + m, c:c + m]) ** 2) for r, c in pos])
        scale = photons / (m * m * energy)
        probe = probe * math.sqrt(scale)
        meas = np.empty((pos.shape[0], m, m), dtype=np.float32)
        for s0 in range(0, pos.shape[0], 512):
            chunk = simulate_intensities(probe, obj, pos[s0:s0 + 512])
            if keep_noiseless:
                d = chunk if d is None else np.concatenate([d, chunk])
            meas[s0:s0 + 512] = rng.poisson(chunk)
    else:
        d = simulate_intensities(probe, obj, pos)
        meas = d.astype(np.float32)
    return Problem(
        name=name, n=n, m=m, positions=pos, intensities=meas,
        probe_true=probe, object_true=obj,
        probe_init=initial_probe(m).astype(np.complex64),
        object_init=np.ones((n, n), dtype=np.complex64),
        minibatch=B, levels=L, alpha=alpha, alpha_z=1.0,
        epochs=cfg["epochs"], seed=seed, photons=photons,
        noiseless=d if keep_noiseless else None,
    )


def noise_percent(noisy: np.ndarray, clean: np.ndarray) -> float:
    """Noise% (amplitude) of Sec. 4.1: 100 sqrt(sum ||d - d~||^2 / sum ||d~||^2)."""
    diff = noisy.astype(np.float64) - clean
    return 100.0 * math.sqrt(float((diff * diff).sum()) / float((clean * clean).sum()))


def make_c5(count: int = 16, seed: int = 1005) -> list:
    """Uneven batched instances: object sides from {256, 384, 512, 768, 1024}, probe sides
    from {64, 128}, 400-4096 jittered raster positions, Poisson photon counts log-uniform
    in [1e5, 1e7], two multigrid levels, minibatch 64; instance j uses seed * 100 + j."""
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed * 100 + j)
        n = int(rng.choice([256, 384, 512, 768, 1024]))
        m = int(rng.choice([64, 128]))
        npos = int(rng.integers(400, 4097))
        side = max(2, int(round(math.sqrt(npos))))
        step = max(1, (n - m - 4) // (side - 1))
        photons = float(10.0 ** rng.uniform(5.0, 7.0))
        p = make_problem(f"c5_{j}", n=n, m=m, scan=("raster", side, step, 1), photons=photons, B=64,
                         L=2, alpha=0.05, seed=seed * 100 + j)
        out.append(p)
    return out


# --------------------------------------------------------------------------
# Stand-ins for the inputs of the paper's synthetic experiments (Sec. 4.1)
# --------------------------------------------------------------------------

def textured_object(n: int, rng: np.random.Generator, n_blobs: int = 400) -> np.ndarray:
    """Object with the value ranges of the paper's test object: |z*| in [0, 1] and arg z* in
    [0, pi/2] (Sec. 4.1), each channel a min-max normalised sum of n_blobs Gaussian blobs of
    width U[n/256, n/24] (finer texture than make_object, standing in for natural images)."""
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)

    def channel() -> np.ndarray:
        f = np.zeros((n, n))
        for _ in range(n_blobs):
            cy, cx = rng.uniform(0, n, size=2)
            s = rng.uniform(n / 256.0, n / 24.0)
            w = rng.uniform(-1.0, 1.0)
            r0, r1 = int(max(0, cy - 5 * s)), int(min(n, cy + 5 * s + 1))
            c0, c1 = int(max(0, cx - 5 * s)), int(min(n, cx + 5 * s + 1))
            f[r0:r1, c0:c1] += w * np.exp(-((yy[r0:r1, c0:c1] - cy) ** 2
                                            + (xx[r0:r1, c0:c1] - cx) ** 2) / (2.0 * s * s))
        f -= f.min()
        mx = f.max()
        return f / mx if mx > 0 else f

    mag = channel()
    ph = channel()
    return mag * np.exp(1j * (np.pi / 2.0) * ph)


def zone_plate_probe(m: int, outer: float = 0.1875, stop: float = 0.4,
                     spot: float = 0.25) -> np.ndarray:
    """Defocused Fresnel-zone-plate illumination (stand-in for the simulated FZP of Sec. 4.1).

    A zone plate with a central stop passes an annulus of spatial frequencies,
    stop * outer * m <= |k| <= outer * m (cycles per window).  Out of focus, each frequency
    picks up the quadratic phase beta |k|^2; beta is chosen so that the geometric shadow of the
    outer zone has radius spot * m pixels.  The result has ring-structured magnitude, very low
    magnitude outside the central disc and concentric phase bands.  Scaled to max |Q| = 1,
    centred on the window centre.
    """
    k = np.fft.fftfreq(m) * m
    ky, kx = np.meshgrid(k, k, indexing="ij")
    rho = np.sqrt(kx * kx + ky * ky)
    r_out = outer * m
    beta = np.pi * spot / r_out
    # annulus with its edges softened over one frequency sample to limit ringing
    pupil = np.clip(np.minimum(r_out + 0.5 - rho, rho - stop * r_out + 0.5), 0.0, 1.0)
    field = np.fft.fftshift(np.fft.ifft2(pupil * np.exp(1j * beta * rho * rho)))
    # fftshift puts the spot centre at pixel m/2; the windows used here are even-sized
    return field / np.abs(field).max()


def perturbed_initial_probe(probe_true: np.ndarray, rng: np.random.Generator, *,
                            sigma_amp: float = 2.0, ramp: float = 7.0, defocus: float = 0.6,
                            astig: float = 0.2, noise: float = 0.01) -> np.ndarray:
    """Initial probe from the ground truth (Sec. 4.1): Fourier-domain Gaussian blur of |Q*|,
    a random linear phase ramp of total size `ramp` rad across the window, defocus and
    astigmatism terms, plus complex noise of relative amplitude `noise`.

    Coordinates x (columns) and y (rows) run over [-1, 1] across the window; the ramp
    (a_x, a_y) = (ramp / 2) (cos b, sin b) with b ~ U[0, 2 pi) changes the phase by `ramp` rad
    from edge to edge along its direction; the noise is circular Gaussian with standard
    deviation noise * rms|Q0|.
    """
    m = probe_true.shape[0]
    k = np.fft.fftfreq(m)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    # transfer function of a spatial Gaussian of standard deviation sigma_amp pixels
    H = np.exp(-2.0 * np.pi ** 2 * sigma_amp ** 2 * (kx * kx + ky * ky))
    mag = np.real(np.fft.ifft2(np.fft.fft2(np.abs(probe_true)) * H))
    mag = np.maximum(mag, 0.0)
    t = np.linspace(-1.0, 1.0, m)
    y, x = np.meshgrid(t, t, indexing="ij")
    b = rng.uniform(0.0, 2.0 * np.pi)
    ax, ay = 0.5 * ramp * np.cos(b), 0.5 * ramp * np.sin(b)
    phase = ax * x + ay * y + defocus * (x * x + y * y) + astig * (x * x - y * y)
    q0 = mag * np.exp(1j * phase)
    rms = math.sqrt(float(np.mean(np.abs(q0) ** 2)))
    q0 = q0 + noise * rms * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / math.sqrt(2.0)
    return q0


def overlap_positions(n: int, m: int, overlap: float, rng: np.random.Generator,
                      jitter: int = 2) -> np.ndarray:
    """Raster whose neighbours are shifted by m (1 - overlap) pixels (the overlap ratio of
    Sec. 2.1: 50% = half a probe width), as many per side as fit in [0, n - m], centred,
    with integer jitter in {-jitter..jitter} against raster artefacts."""
    step = max(1, int(round(m * (1.0 - overlap))))
    side = (n - m) // step + 1
    return raster_positions(n, m, side, step, jitter, rng)


def photon_scale_for_noise(clean: np.ndarray, percent: float) -> float:
    """Factor s such that Poisson counts of s * clean have expected Noise% (Sec. 4.1) equal to
    `percent`: the Poisson variance equals the mean, so E sum n^2 = s sum f and
    Noise%^2 / 100^2 = sum f / (s sum f^2)."""
    c = np.asarray(clean, np.float64)
    return float(c.sum() / ((c * c).sum() * (percent / 100.0) ** 2))


def make_protocol_problem(*, overlap: float, noise_percent: float | None = None, n: int = 512,
                          m: int = 128, alpha: float | None = None, B: int = 1, L: int = 1,
                          seed: int = 2025) -> Problem:
    """Synthetic analogue of the paper's overlap (Sec. 4.2) and noise (Sec. 4.3) studies.

    Object from textured_object, zone-plate probe, overlap raster, the perturbed initial probe
    of Sec. 4.1; noiseless data, or Poisson data at a target Noise%.  alpha defaults to the
    paper's choice (0.05 at 50% overlap and for the noise study, 0.01 at 75% / 87.5%).
    """
    rng = np.random.default_rng(seed)
    obj = textured_object(n, rng)
    probe = zone_plate_probe(m)
    pos = overlap_positions(n, m, overlap, rng)
    clean = simulate_intensities(probe, obj, pos)
    if noise_percent is None:
        meas = clean.astype(np.float32)
    else:
        s = photon_scale_for_noise(clean, noise_percent)
        probe = probe * math.sqrt(s)
        clean = clean * s
        meas = rng.poisson(clean).astype(np.float32)
    if alpha is None:
        alpha = 0.05 if (noise_percent is not None or overlap <= 0.5 + 1e-9) else 0.01
    q0 = perturbed_initial_probe(probe, rng)
    return Problem(
        name=f"protocol_o{overlap:g}_n{noise_percent}", n=n, m=m, positions=pos, intensities=meas,
        probe_true=probe, object_true=obj, probe_init=q0.astype(np.complex64),
        object_init=np.ones((n, n), dtype=np.complex64), minibatch=B, levels=L, alpha=alpha,
        alpha_z=1.0, epochs=0, seed=seed, photons=None, noiseless=clean,
    )
