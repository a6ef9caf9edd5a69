"""Write tests/golden/laser_history_8.txt: the oracle's explicit run of the
laser-heating physics (40 seeded bands, 4 x 4 directions per octant, MC
limiter, top face diffuse, other faces thermalizing, Gaussian pulse of
10 ps FWHM centred at 20 ps, dt = 0.5 ps; Algorithm 2 of Sec. 4.1) for
2000 steps on a reduced 8^3 grid with the cell size of the 64^3 case
(31.25 nm, so the same Courant numbers and dt / tau_min).

Calls only oracle/ and the seeded input generators.  Run from the
repository root:  python tests/golden/make_laser_history.py
(about 4 minutes on 8 host cores).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import bte_inputs as I  # noqa: E402
import oracle as O  # noqa: E402

N_CELLS, N_STEPS = 8, 2000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "laser_history_8.txt")


def case():
    cfg = I.cube3d_laser_case(n=N_CELLS, length=N_CELLS * 2e-6 / 64)
    return cfg, O.Case(cfg["geometry"], cfg["material"], P=cfg["P"], limiter=O.LIM_MC)


def run(n_steps):
    cfg, c = case()
    e, hist = O.transient(c, c.zeros(), n_steps, cfg["dt"], 0.0, cfg["pulse"], cfg["hist_weights"])
    T, _, _ = O.moments(c, e)
    return hist, T


def main():
    hist, T = run(N_STEPS)
    with open(OUT, "w") as f:
        f.write("# oracle explicit run, laser physics on 8^3 cells of 31.25 nm, %d steps of 0.5 ps\n" % N_STEPS)
        f.write("# written by tests/golden/make_laser_history.py (oracle only)\n")
        f.write("# section hist: weighted mean top temperature after each step (K)\n")
        f.write("# section T: local temperature of every cell after the last step (K)\n")
        f.write("hist %d\n" % len(hist))
        for x in hist:
            f.write("%.17e\n" % x)
        f.write("T %d\n" % len(T))
        for x in T:
            f.write("%.17e\n" % x)


def load():
    with open(OUT) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    k = 0
    out = {}
    while k < len(lines):
        name, n = lines[k].split()
        n = int(n)
        out[name] = np.array([float(x) for x in lines[k + 1:k + 1 + n]])
        k += 1 + n
    return out["hist"], out["T"]


if __name__ == "__main__":
    main()
