"""Writes the FP64 oracle trajectory of the headline workload's shape at 8^3
cubes: [-1,1]^3, 8^3 Kuhn cubes x 6 = 3072 tets, interior vertices jittered by
U(-0.1h, 0.1h) (seed 2), eps ~ U[1,4], mu = 1, p = 3, upwind flux, PEC walls,
divergence-free Gaussian pulse e0 = curl(z g) of width 0.2, h0 = 0, classic RK4
at CFL 0.3 for 1000 steps.

Only the oracle and the seeded workload generators are called. The output
(``jittered8_p3_upwind_rk4_1000.npz``) holds dt, the step count, the energy of
the projected initial state and the Cartesian E and H coefficients after the
last step. Run from the repository root:

    python tests/golden/make_jittered8_trajectory.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import OracleDG  # noqa: E402

OUT = os.path.join(HERE, "jittered8_p3_upwind_rk4_1000.npz")
N_CUBES, ORDER, STEPS, CFL = 8, 3, 1000, 0.3


def main():
    w = W.jittered(N_CUBES, ORDER, seed=2, flux="upwind")
    dt = W.cfl_dt(w.verts, w.tets, w.eps, w.mu, w.p, CFL)
    O = OracleDG(w.verts, w.tets, ORDER, eps=w.eps, mu=w.mu, flux="upwind")
    cE = O.project(lambda x: W.gaussian_curl_e(x, 0.2))
    cH = np.zeros_like(cE)
    W0 = O.energy(cE, cH)
    t0 = time.time()
    s = [cE, cH, None, None]
    t = 0.0
    for n in range(STEPS):
        s = O.rk4_step(s, t, dt)
        t += dt
        if (n + 1) % 50 == 0:
            print(f"step {n + 1}/{STEPS}  W={O.energy(s[0], s[1]):.15e}  {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, dt=dt, steps=STEPS, energy0=W0, cE=s[0], cH=s[1])
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
