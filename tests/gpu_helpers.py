"""Shared set-up for the GPU parity tests (HIP path through the C ABI vs FP64 oracle)."""
from __future__ import annotations

import numpy as np

from oracle import emagpie_oracle as O
from paper_2511_01793_amd import synth

# Parity bars.  Per step from identical state the spec bar is 1e-5 relative
# (norm-wise, rel = ||x_gpu - x_orc|| / ||x_orc||).  Quantities that compound several
# FP32 steps or divide by a small misfit get the looser bars derived in the design doc.
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
             joint_step=True):
    import torch
    import paper_2511_01793_amd.emagpie as E
    d = torch.from_numpy(p.intensities).cuda()
    rec = E.Reconstruction(p.positions, d, p.n,
                           minibatch=p.minibatch if minibatch is None else minibatch,
                           levels=p.levels if levels is None else levels,
                           alpha=p.alpha if alpha is None else alpha, alpha_z=p.alpha_z,
                           update_probe=update_probe, joint_step=joint_step, path=path, seed=seed)
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
