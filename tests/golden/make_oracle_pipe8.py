"""Write the oracle's state of the 8 x 32 x 32 pipe (R = 14, Ha = 5, Re = 10, Rm = 1e-3,
270 magnetic sweeps per step) after 2000 steps from the seeded noise start.

Calls only the FP64 oracle and the seeded workloads; the output is the reference of the
2000-step GPU parity test. Run: python tests/golden/make_oracle_pipe8.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_pipe8x32x32_2000steps.npz")
STEPS = 2000


def main():
    w = W.small_pipe()
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    t0 = time.time()
    for k in range(STEPS // 100):
        o.step(100)
        print(f"step {(k + 1) * 100} ({time.time() - t0:.0f} s)", flush=True)
    bud = o.budgets()
    np.savez_compressed(OUT, rho=o.rho, u=o.u, b=o.b, steps=STEPS, G=o.G.value,
                        budgets=np.array([bud[k] for k in oracle.BUDGET_NAMES]),
                        budget_names=np.array(oracle.BUDGET_NAMES))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
