"""CPU-baseline worker: times the FP64 oracle, as it stands, on a window of
steps of a scene stored by the caller.

TEST INFRASTRUCTURE ONLY: run by the benchmark's CPU-baseline leg, one
process per measurement; never by the GPU library or its binding.

    python -m oracle.baseline SCENE.npz STEPS LIBRARY

SCENE.npz holds the scene arrays (pos, vel, mass, ends, k, damping, amp,
phase) and the step parameters (dt, g, ground, ground_k, mu, omega).  Prints
one JSON line: {"seconds": wall time of the step loop alone}.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from oracle import oracle as O


def main(argv):
    path, steps, lib = argv[1], int(argv[2]), argv[3]
    O.use_library(lib)
    z = np.load(path)
    scene = {k: z[k] for k in ("pos", "vel", "mass", "ends", "k", "damping", "amp", "phase")}
    op = O.Params(dt=float(z["dt"]), gravity=tuple(float(x) for x in z["g"]), ground=bool(z["ground"]),
                  ground_k=float(z["ground_k"]), mu=float(z["mu"]), omega=float(z["omega"]))
    sysm = O.System(scene)
    t0 = time.perf_counter()
    sysm.run(op, sysm.x0, sysm.v0, 0, steps)
    print(json.dumps({"seconds": time.perf_counter() - t0}))


if __name__ == "__main__":
    main(sys.argv)
