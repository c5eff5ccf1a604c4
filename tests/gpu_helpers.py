"""Shared set-up for the GPU parity tests (HIP path through the C ABI vs FP64 oracle)."""
from __future__ import annotations

import numpy as np

from oracle import emagpie_oracle as O
from paper_2511_01793_amd import synth

# Parity bars, norm-wise: rel = ||x_gpu - x_orc|| / ||x_orc||.
#   STEP_TOL: one step from identical state.  The FP32 transform error is about
#     eps32 * log2(m^2) ~ 7e-7 of ||Psi||, and a step is two transforms plus O(1)
#     per-pixel operations (observed 3e-7 .. 6e-7).
#   MISFIT_TOL: Phi = sum (|Psi| - a)^2 divides that error by sqrt(Phi / energy),
#     which is >= 1e-3 on every tested state; the FP32 gradient likewise.
#   EPOCH_TOL: several steps compound within an epoch.
#   GRAD64_TOL: the float64 gradient, rounding of FP64 transforms.
STEP_TOL = 1e-5
MISFIT_TOL = 1e-4
EPOCH_TOL = 5e-5
GRAD32_TOL = 1e-4
GRAD64_TOL = 1e-10


def rel(a, b) -> float:
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(name="tiny", **kw):
    return synth.make_problem(name, **kw)


def make_rec(p, path="fused", levels=None, minibatch=None, alpha=None, update_probe=True, seed=3,
             joint_step=True, fft_plan=0, finalize_shape=0):
    import torch
    import paper_2511_01793_amd.emagpie as E
    d = torch.from_numpy(p.intensities).cuda()
    rec = E.Reconstruction(p.positions, d, p.n,
                           minibatch=p.minibatch if minibatch is None else minibatch,
                           levels=p.levels if levels is None else levels,
                           alpha=p.alpha if alpha is None else alpha, alpha_z=p.alpha_z,
                           update_probe=update_probe, joint_step=joint_step, path=path, seed=seed,
                           fft_plan=fft_plan, finalize_shape=finalize_shape)
    return rec


def init_state(p, rec):
    import torch
    obj = torch.from_numpy(p.object_init).cuda()
    probe = torch.from_numpy(p.probe_init).cuda()
    rec.normalize_probe(probe)
    return obj, probe


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def amps(p):
    return O.amplitudes(p.intensities)
