"""Write the oracle misfit trajectories that define the time-to-fixed-misfit targets.

Calls only the FP64 oracle (and the seeded input generators).  For each workload it
runs the oracle from the initial state of Sec. 4.1 (z = 1, probe scaled by dp_avg) for
the workload's epoch count with the library's scan order (SplitMix64 Fisher-Yates,
seed = the workload seed), and records Phi (Eq. 1) after every epoch.  The target is
1.01 x the final value.

A key "NAME/jJ" (J = 1, 2, ...) starts instead from the initial probe times (1 + eps g)
with g complex standard normal per pixel, seeded by JITTER_SEED0 + J and eps = JITTER_EPS
(synth.jittered_initial_probe): seeded variants of the same start, for the spread of the
time to target.

    python tests/golden/make_targets.py [c1] [c2] [c3] [c2/j1] ...

Each key is written as soon as its trajectory is done (the file is locked, re-read and
rewritten), so several keys can be computed by concurrent invocations.
"""
import fcntl
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import emagpie_oracle as O  # noqa: E402
from paper_2511_01793_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "misfit_targets.json")
JITTER_EPS = 1e-2
JITTER_SEED0 = 7000


def parse_key(key: str):
    name, _, var = key.partition("/")
    j = int(var[1:]) if var else 0
    if var and not var.startswith("j"):
        raise ValueError(f"bad key {key!r}: expected NAME or NAME/jJ")
    return name, j


def trajectory(key: str):
    name, j = parse_key(key)
    p = synth.make_problem(name)
    eps = JITTER_EPS if j else 0.0
    probe0 = synth.jittered_initial_probe(p.probe_init, eps, JITTER_SEED0 + j)
    a = O.amplitudes(p.intensities)
    q = O.normalise_probe(probe0, p.intensities)
    z = p.object_init.astype(np.complex128)
    phis = [O.misfit(q, z, p.positions, a)]
    t0 = time.time()
    for e in range(p.epochs):
        q, z, _ = O.run_epoch(q, z, p.positions, a, seed=p.seed, epoch=e, minibatch=p.minibatch,
                              alpha=p.alpha, alpha_z=p.alpha_z, levels=p.levels)
        phis.append(O.misfit(q, z, p.positions, a))
        print(key, e, phis[-1], f"{time.time() - t0:.1f}s", flush=True)
    out = dict(epochs=p.epochs, seed=p.seed, minibatch=p.minibatch, levels=p.levels,
               alpha=p.alpha, misfit=phis, final=phis[-1], target=1.01 * phis[-1])
    if j:
        out.update(jitter_eps=eps, jitter_seed=JITTER_SEED0 + j)
    return out


def store(key: str, value: dict):
    with open(OUT + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as f:
                data = json.load(f)
        data[key] = value
        data["_source"] = ("FP64 oracle (oracle/emagpie_oracle.py) via tests/golden/make_targets.py; "
                           "misfit[e] is Phi of Eq. 1 after e epochs from the Sec. 4.1 initial state "
                           "(keys NAME/jJ: the initial probe jittered by synth.jittered_initial_probe "
                           "with jitter_eps and jitter_seed)")
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1)
        os.replace(OUT + ".tmp", OUT)


def main(keys):
    for k in keys:
        parse_key(k)
    for k in keys:
        store(k, trajectory(k))


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
