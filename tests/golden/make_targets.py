"""Write the oracle misfit trajectories that define the time-to-fixed-misfit targets.

Calls only the FP64 oracle (and the seeded input generators).  For each workload it
runs the oracle from the initial state of Sec. 4.1 (z = 1, probe scaled by dp_avg) for
the workload's epoch count with the library's scan order (SplitMix64 Fisher-Yates,
seed = the workload seed), and records Phi (Eq. 1) after every epoch.  The target is
1.01 x the final value.

    python tests/golden/make_targets.py [c1] [c2]
"""
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


def trajectory(name: str):
    p = synth.make_problem(name)
    a = O.amplitudes(p.intensities)
    q = O.normalise_probe(p.probe_init, p.intensities)
    z = p.object_init.astype(np.complex128)
    phis = [O.misfit(q, z, p.positions, a)]
    t0 = time.time()
    for e in range(p.epochs):
        q, z, _ = O.run_epoch(q, z, p.positions, a, seed=p.seed, epoch=e, minibatch=p.minibatch,
                              alpha=p.alpha, alpha_z=p.alpha_z, levels=p.levels)
        phis.append(O.misfit(q, z, p.positions, a))
        print(name, e, phis[-1], f"{time.time() - t0:.1f}s", flush=True)
    return dict(epochs=p.epochs, seed=p.seed, minibatch=p.minibatch, levels=p.levels,
                alpha=p.alpha, misfit=phis, final=phis[-1], target=1.01 * phis[-1])


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for n in names:
        data[n] = trajectory(n)
    data["_source"] = ("FP64 oracle (oracle/emagpie_oracle.py) via tests/golden/make_targets.py; "
                       "misfit[e] is Phi of Eq. 1 after e epochs from the Sec. 4.1 initial state")
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
