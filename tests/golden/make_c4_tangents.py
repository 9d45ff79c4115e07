"""Write c4_tangents.json: loss and directional derivatives of the adjoint workload computed by
the oracle in forward mode (dual numbers), for the GPU adjoint test at full size.

Workload: D2Q37, 256 x 256, tau for nu = 0.1, rho = 1, u = 0, T = 1 + 1e-4 N(0, 1) (seed 2307),
LODI-RELAX on all four sides and corners (sigma = 0.25, alpha = Ma = 0 for the fluid at rest,
mach = 0), 2000 steps, loss
= sum over bulk nodes of (P - cs^2)^2 at the final step.  Directions: sigma, alpha (on every side
together) and three seeded random perturbations of the initial temperature (seed 230701).

Run from the repository root: python tests/golden/make_c4_tangents.py  (about 12 minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2307_16766_amd import workloads as W  # noqa: E402

NX = NY = 256
STEPS = 2000
SEED_DIRS = 230701


def main():
    cs2 = O.lattice(37)[0]
    tau = 0.5 + W.NU_D2Q37 / cs2
    bc = ["lodi_relax"] * 4
    fields = W.random_temperature(NX, NY, std=1e-4, seed=2307)
    relax = np.tile(np.array([0.25, 0.0, 1.0, 1.0, 0.0, 0.0]), (4, 1))
    dirs = W.random_directions(3, NX, NY, SEED_DIRS)
    t0 = time.time()
    # run 1: sigma, alpha, T direction 0; run 2: T directions 1 and 2
    dF = np.zeros((3, 4, NY, NX))
    dF[2, 3] = dirs[0]
    loss, d1 = O.tangent_run_fields(37, NX, NY, tau, bc, relax, [1, 0, 0], [0, 1, 0], fields, dF, STEPS)
    dF = np.zeros((3, 4, NY, NX))
    dF[0, 3] = dirs[1]
    dF[1, 3] = dirs[2]
    loss2, d2 = O.tangent_run_fields(37, NX, NY, tau, bc, relax, [0, 0, 0], [0, 0, 0], fields, dF, STEPS)
    out = {
        "workload": "D2Q37 256x256 random temperature (std 1e-4, seed 2307), LODI-RELAX x4 "
                    "(sigma 0.25, alpha 0, mach 0), 2000 steps, pressure loss",
        "nsteps": STEPS, "direction_seed": SEED_DIRS,
        "loss": loss, "loss_second_run": loss2,
        "d_sigma": d1[0], "d_alpha": d1[1], "d_T0": [d1[2], d2[0], d2[1]],
        "oracle_threads": O.num_threads(), "seconds": time.time() - t0,
        "command": "python tests/golden/make_c4_tangents.py",
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_tangents.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
