"""Writes c3_ke_history.json: the kinetic-energy history of the corrected
low-order Taylor-Green run (16^3 elements, P = 3, Re 200, Mach 0.1) with the
Gaussian-initialised forcing network (320 -> 256 -> 256 -> 256 -> 320 tanh,
seed 0, weights rounded to bfloat16) added at every Runge-Kutta stage
(Eq. (4)), over 100 steps of the Eq. (7) time step, computed by the CPU
oracle only.

    python tests/golden/make_c3_ke_history.py      (about four minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle import dg, forcing, mlp, rk  # noqa: E402

DIMS = [320, 256, 256, 256, 320]
NORM = [1.0, 0.0, 0.0, 0.0, synthetic.TGV_ENERGY_LEVEL,
        0.01, 1.0, 1.0, 1.0, 1.0,
        0.0, 0.0, 0.0, 0.0, 0.0,
        1e-3, 1e-3, 1e-3, 1e-3, 1e-3]
STEPS = 100


def main():
    prm = dg.Params(N=16, P=3, Re=200.0)
    layers = synthetic.mlp_init(DIMS, seed=0)
    params = [(mlp.bf16_round(W), b.astype(np.float64)) for W, b in layers]
    norm = forcing.Normalisation(NORM[0:5], NORM[5:10], NORM[10:15], NORM[15:20])
    q0 = dg.tgv_initial_condition(prm)
    dt = dg.stable_dt(q0, prm)
    ke = []
    t0 = time.time()

    def cb(n, q):
        ke.append(dg.kinetic_energy(q, prm))
        if n % 10 == 0:
            print(f"step {n}: KE {ke[-1]:.15e} ({time.time() - t0:.0f} s)", flush=True)

    rk.integrate(q0, dt, STEPS, lambda qq, t: forcing.corrected_rhs(qq, prm, params, norm), callback=cb)
    out = {"what": "kinetic energy after each of 100 RK3 steps, corrected P = 3 TGV (network at every stage)",
           "N": 16, "P": 3, "Re": 200.0, "Mach": 0.1, "dims": DIMS, "norm": NORM, "seed": 0,
           "dt": dt, "ke0": dg.kinetic_energy(q0, prm), "ke": ke,
           "written_by": "tests/golden/make_c3_ke_history.py (CPU oracle only)"}
    with open(os.path.join(HERE, "c3_ke_history.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
