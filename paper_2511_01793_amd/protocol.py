"""Reconstruction protocol of the paper's numerical experiments (Sec. 4.1).

* quality metrics: the residual Phi of Eq. 1 (evaluated by the library's misfit kernel) and
  the magnitude error || |z| - |z*| ||_2 over the whole object;
* stopping rules: the w-point moving-average rule with patience p, and the noise-floor rule
  that stops once the residual falls below a fraction of the misfit of the ground truth;
* a driver that runs eMAGPIE (joint step of Eq. 6, multigrid object step) or the rPIE
  comparator (Eq. 2: the same kernels, one level, no joint step) epoch by epoch on the GPU;
* the synthetic analogues of the overlap study (Sec. 4.2) and the noise study (Sec. 4.3):
  ``python -m paper_2511_01793_amd.protocol --study overlap|noise``.

Reading of the moving-average rule: the printed condition compares the moving average with
a running minimum that includes the current value, which always holds; the rule is taken to
mean "no new minimum of the moving average", i.e. a check at t fails to improve when
rbar_t >= min over earlier s of rbar_s, and the run stops after p such checks in a row.
Residuals are counted from t = 1 (after the first epoch); rbar_t exists from t = w on and the
first check is at t = w + 1.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

__all__ = ["MovingAverageStop", "below_floor", "magnitude_error", "reconstruct", "study"]


class MovingAverageStop:
    """Moving-average stopping rule (Sec. 4.1) with window w and patience p."""

    def __init__(self, window: int = 5, patience: int = 10):
        if window < 1 or patience < 1:
            raise ValueError("window and patience must be >= 1")
        self.window = int(window)
        self.patience = int(patience)
        self.history: list[float] = []
        self.best = math.inf
        self.stale = 0

    def update(self, residual: float) -> bool:
        """Record r_t; True when the run should stop after this iteration."""
        self.history.append(float(residual))
        t = len(self.history)
        if t < self.window:
            return False
        rbar = sum(self.history[-self.window:]) / self.window
        if t == self.window:
            self.best = rbar
            return False
        if rbar >= self.best:
            self.stale += 1
        else:
            self.best = rbar
            self.stale = 0
        return self.stale >= self.patience


def below_floor(residual: float, floor: float, factor: float = 0.9) -> bool:
    """Noise-floor rule (Sec. 4.3): stop once the residual is below factor x the misfit of
    the ground-truth object and probe on the same (noisy) data."""
    return residual < factor * floor


def magnitude_error(z, z_true, align_scale: bool = False) -> float:
    """|| |z| - |z*| ||_2 over all pixels (the error metric of Sec. 4.1), in float64.

    With align_scale, |z| is first multiplied by the c >= 0 that minimises the norm
    (c = <|z|, |z*|> / <|z|, |z|>): blind reconstructions are determined only up to
    (c z, Q / c), and the plain metric also counts that scale."""
    a = np.abs(np.asarray(z, np.complex128)).ravel()
    b = np.abs(np.asarray(z_true, np.complex128)).ravel()
    if align_scale:
        den = float(a @ a)
        a = a * (float(a @ b) / den if den > 0 else 0.0)
    return float(np.linalg.norm(a - b))


def reconstruct(problem, *, method: str = "emagpie", levels: int | None = None,
                max_epochs: int = 300, window: int = 5, patience: int = 10,
                floor_factor: float | None = None, path: str = "auto", seed: int = 0,
                minibatch: int | None = None, record_error: bool = True) -> dict:
    """Run one method on one problem with the paper's stopping rules; returns the history.

    method "emagpie": joint step on, `levels` multigrid levels (default: the problem's);
    method "rpie": joint step off, one level.  The probe starts from problem.probe_init
    scaled by the dp_avg rule, the object from problem.object_init.  Residuals are the full
    misfit Phi after each epoch; with floor_factor set, the noise floor is Phi at the ground
    truth (object_true, probe_true) on the measured data.
    """
    import torch
    from . import emagpie as E

    if method not in ("emagpie", "rpie"):
        raise ValueError("method must be 'emagpie' or 'rpie'")
    joint = method == "emagpie"
    L = (problem.levels if levels is None else levels) if joint else 1
    d = torch.from_numpy(np.ascontiguousarray(problem.intensities)).cuda()
    rec = E.Reconstruction(problem.positions, d, problem.n,
                           minibatch=problem.minibatch if minibatch is None else minibatch,
                           levels=L, alpha=problem.alpha, alpha_z=problem.alpha_z,
                           update_probe=True, joint_step=joint, path=path, seed=seed)
    try:
        obj = torch.from_numpy(np.ascontiguousarray(problem.object_init, np.complex64)).cuda()
        probe = torch.from_numpy(np.ascontiguousarray(problem.probe_init, np.complex64)).cuda()
        rec.normalize_probe(probe)
        floor = None
        if floor_factor is not None:
            zt = torch.from_numpy(problem.object_true.astype(np.complex64)).cuda()
            qt = torch.from_numpy(problem.probe_true.astype(np.complex64)).cuda()
            floor = float(rec.misfit(zt, qt).item())
        rule = MovingAverageStop(window, patience)
        phi = torch.empty((), dtype=torch.float64, device="cuda")
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        hist = {"method": method, "levels": L, "alpha": problem.alpha, "n_pos": problem.n_pos,
                "residual": [], "error": [], "error_aligned": [], "epoch_ms": [], "floor": floor,
                "stop": "max_epochs"}
        for e in range(max_epochs):
            start.record()
            rec.epoch(obj, probe, e)
            stop.record()
            rec.misfit(obj, probe, out=phi)
            r = float(phi.item())
            hist["epoch_ms"].append(start.elapsed_time(stop))
            hist["residual"].append(r)
            if record_error:
                zh = obj.cpu().numpy()
                hist["error"].append(magnitude_error(zh, problem.object_true))
                hist["error_aligned"].append(magnitude_error(zh, problem.object_true, True))
            if not math.isfinite(r):
                hist["stop"] = "non_finite"
                break
            if floor is not None and below_floor(r, floor, floor_factor):
                hist["stop"] = "floor"
                break
            if rule.update(r):
                hist["stop"] = "moving_average"
                break
        hist["epochs"] = len(hist["residual"])
        hist["object"] = obj.cpu().numpy()
        hist["probe"] = probe.cpu().numpy()
        return hist
    finally:
        rec.close()


def _summary(h: dict, extra: dict) -> dict:
    ms = sorted(h["epoch_ms"])
    return dict(extra, method=h["method"], levels=h["levels"], alpha=h["alpha"], n_pos=h["n_pos"],
                epochs=h["epochs"], stop=h["stop"], residual=h["residual"][-1],
                min_residual=min(h["residual"]), floor=h["floor"],
                error=h["error"][-1] if h["error"] else None,
                error_aligned=h["error_aligned"][-1] if h["error_aligned"] else None,
                median_epoch_ms=ms[len(ms) // 2])


def study(kind: str, *, n: int = 512, m: int = 128, levels: int = 2, minibatch: int = 1,
          max_epochs: int = 300, seed: int = 2025, log=print) -> list[dict]:
    """Synthetic analogue of the overlap study (50 / 75 / 87.5%, noiseless) or the noise
    study (5 / 10 / 20% Poisson noise at 75% overlap, alpha = 0.05, plus the floor rule)."""
    from . import synth

    rows = []
    if kind == "overlap":
        cases = [dict(overlap=o, noise_percent=None) for o in (0.5, 0.75, 0.875)]
    elif kind == "noise":
        cases = [dict(overlap=0.75, noise_percent=p) for p in (5.0, 10.0, 20.0)]
    else:
        raise ValueError("kind must be 'overlap' or 'noise'")
    for c in cases:
        p = synth.make_protocol_problem(n=n, m=m, B=minibatch, L=levels, seed=seed, **c)
        extra = dict(c, noise_measured=(synth.noise_percent(p.intensities, p.noiseless)
                                        if c["noise_percent"] is not None else 0.0))
        for method in ("rpie", "emagpie"):
            t0 = time.time()
            h = reconstruct(p, method=method, max_epochs=max_epochs,
                            floor_factor=0.9 if c["noise_percent"] is not None else None)
            row = _summary(h, extra)
            row["wall_s"] = time.time() - t0
            row["residual_curve"] = h["residual"]
            row["error_curve"] = h["error"]
            rows.append(row)
            log(json.dumps({k: v for k, v in row.items() if not k.endswith("_curve")}))
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--study", choices=["overlap", "noise"], required=True)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--m", type=int, default=128)
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--minibatch", type=int, default=1)
    ap.add_argument("--max-epochs", type=int, default=300)
    ap.add_argument("--seed", type=int, default=2025)
    ap.add_argument("--out", default=None, help="write all rows (with curves) as JSON")
    a = ap.parse_args(argv)
    rows = study(a.study, n=a.n, m=a.m, levels=a.levels, minibatch=a.minibatch,
                 max_epochs=a.max_epochs, seed=a.seed, log=lambda s: print(s, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
