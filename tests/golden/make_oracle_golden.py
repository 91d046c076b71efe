"""Write the oracle's expected values for the long-run GPU tests (FP64, CPU).

Calls only the oracle (``oracle/``) and the seeded input generator
(``paper_1806_06943_amd.workloads``, geometry and random numbers only):

* ``batched``: the 96-instance static-droplet workload after 5000 steps (the
  step count of that workload): per instance the Laplace-test observables of
  Sec. III B (R_eff, pressure jump, gamma) and both masses;
* ``spinodal``: a 256 x 256 spinodal decomposition with the emulsion couplings
  (3.0, -7.4, 6.4) of Sec. III D after 20000 steps: masses, population momentum
  and the mean domain size (first zero of the radial correlation of
  rho_A - rho_B).

Usage: python tests/golden/make_oracle_golden.py batched|spinodal
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1806_06943_amd import workloads as W  # noqa: E402

BATCHED_STEPS = 5000
SPINODAL = dict(nx=256, ny=256, steps=20000, tau=(1.0, 0.7))


def params(w):
    return O.Params(nx=w.nx, ny=w.ny, G_AB=w.G_AB, G1=w.G1, G2=w.G2, tau=w.tau, g=w.g,
                    walls=w.walls, rho_wall=w.rho_wall)


def batched(path):
    rows = []
    t0 = time.time()
    for n, w in enumerate(W.batched()):
        p = params(w)
        f = O.run(p, O.init(p, w.rhoA, w.rhoB), BATCHED_STEPS)
        L = O.laplace(p, O.fields(p, f))
        m = O.masses(f)
        rows.append((n, w.nx, L["R"], L["dp"], L["gamma"], m[0], m[1]))
        print(f"instance {n} ({w.nx}^2): R {L['R']:.6f} dp {L['dp']:.6e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(path, "w") as fh:
        fh.write("# oracle (FP64) after %d steps of the 96-instance droplet workload;\n"
                 "# written by tests/golden/make_oracle_golden.py batched\n"
                 "# index side R_eff dp gamma mass_A mass_B\n" % BATCHED_STEPS)
        for r in rows:
            fh.write("%d %d %.17g %.17g %.17g %.17g %.17g\n" % r)


def spinodal(path):
    s = SPINODAL
    w = W.spinodal(nx=s["nx"], ny=s["ny"], couplings=W.COUPLINGS_PAPER, tau=s["tau"])
    p = params(w)
    f = O.init(p, w.rhoA, w.rhoB)
    m0 = O.masses(f)
    out = []
    done = 0
    for target in (2000, 5000, 10000, 20000):
        f = O.run(p, f, target - done)
        done = target
        rho = O.density(p, f)
        L = O.domain_size(rho[0] - rho[1])
        m = O.masses(f)
        P = O.raw_momentum(f)
        out.append((target, m[0], m[1], P[0], P[1], L))
        print(f"step {target}: domain size {L:.4f}, mass drift "
              f"{abs(m[0] - m0[0]) / m0[0]:.2e}", flush=True)
    with open(path, "w") as fh:
        fh.write("# oracle (FP64) 256x256 spinodal, couplings (3.0, -7.4, 6.4), tau (1.0, 0.7);\n"
                 "# written by tests/golden/make_oracle_golden.py spinodal\n"
                 "# step mass_A mass_B momentum_x momentum_y domain_size\n")
        for r in out:
            fh.write("%d %.17g %.17g %.17g %.17g %.17g\n" % r)


if __name__ == "__main__":
    which = sys.argv[1]
    dest = os.path.join(HERE, {"batched": "batched_laplace_oracle.txt",
                               "spinodal": "spinodal256_oracle.txt"}[which])
    {"batched": batched, "spinodal": spinodal}[which](dest)
    print("wrote", dest)
