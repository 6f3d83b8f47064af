"""Write the stored expected values under tests/golden/ (run from the repository root).

    python tests/golden/make_golden.py

Values come from closed forms or from the FP64 oracle only (never from the GPU path):
  manufactured_box.json   discrete eigenvalue of the 7-point operator for the mode
                          sin(pi x) sin(2 pi y) sin(3 pi z) on the open unit box at h = 1/64, and
                          the exact ratio discrete/continuous solution (closed form)
  tiny_channel.json       one projection and a 3-step kinetic-energy gradient on a seeded
                          2x2x2-cube channel of 4^3 cells (oracle), at fixed sample cells
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from bcm_inputs import CHANNEL_BC, uniform_mesh, uniform_random_velocity  # noqa: E402
from oracle import FVMesh, projection as OP  # noqa: E402

SAMPLE = [0, 5, 63, 64, 100, 200, 255, 256, 300, 400, 511]


def tiny_channel_inputs():
    m = uniform_mesh((2, 2, 2), 0.5, 4, CHANNEL_BC)
    u = uniform_random_velocity(m, 41, 0.2, (1.0, 0.0, 0.0))
    alpha = np.random.default_rng(42).uniform(0.0, 1.0, m.n_cells)
    return m, u, alpha, dict(U_in=1.0, dt=0.05, rho=1.0, steps=3)


def main():
    h = 1.0 / 64
    lam = sum(2 * np.cos(k * np.pi * h) - 2 for k in (1, 2, 3)) / h ** 2
    json.dump({"source": "closed form of the 7-point operator's eigenvalue (Poisson equation, "
                         "Sec. 3) for sin(pi x)sin(2 pi y)sin(3 pi z) at h = 1/64",
               "h": h, "lambda_h": lam, "ratio_minus_one": -14 * np.pi ** 2 / lam - 1.0},
              open(os.path.join(HERE, "manufactured_box.json"), "w"), indent=1)
    m, u, alpha, prm = tiny_channel_inputs()
    fv = FVMesh(m)
    r = OP.project(fv, u, alpha, (0, 0, 0), prm["U_in"], prm["dt"], prm["rho"])
    noise = u.reshape(3, -1).copy()
    noise[0] -= prm["U_in"]
    J, ga, gU = OP.multistep_gradient(fv, noise, alpha, (0, 0, 0), prm["U_in"], prm["dt"],
                                      prm["rho"], prm["steps"])
    json.dump({"source": "FP64 oracle (oracle/fv.py, oracle/projection.py), seeded inputs of "
                         "tests/golden/make_golden.py:tiny_channel_inputs",
               "params": prm, "sample": SAMPLE,
               "p": r["p"][SAMPLE].tolist(),
               "u_new": r["u_new"][:, SAMPLE].tolist(),
               "J": J, "g_alpha": ga[SAMPLE].tolist(), "g_U_in": gU},
              open(os.path.join(HERE, "tiny_channel.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
