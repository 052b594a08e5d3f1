"""Writes tests/golden/deformed32_1000.npz: the oracle's state after the full
run of the p=3, 32^3 deformed-cube workload (x -> x + 0.08 sin(pi x) sin(pi y)
sin(pi z) per component, eps ~ U[1,4] per element from seed 0, mu = 1, initial
E the sum of the 10 lowest cavity modes with seeded N(0,1) amplitudes, H = 0,
dt = 0.5 CFL of the oracle's own operator, 1000 leapfrog steps with d and b
tracked, Sections 3.4 and 5).

Calls the oracle only.  Run from the repository root:

    python tests/golden/make_deformed32_golden.py

It takes about fifteen minutes on eight host cores.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.geometry import Map  # noqa: E402
from oracle.scheme import Scheme  # noqa: E402

P, N, STEPS, ENERGY_EVERY = 3, 32, 1000, 50
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "deformed32_1000.npz")


def main():
    t0 = time.time()
    S = Scheme(P, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=W.eps_elements(N, 0))
    modes = W.cavity_modes(0)
    field = lambda x: W.eval_modes(modes, x)  # noqa: E731
    e0 = S.project_E(field)
    d0 = S.project_D(field, tol=1e-15)
    dt = 0.5 * S.cfl(iters=300, tol=1e-6)
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, b0=np.zeros(S.n_h))
    print(f"set-up {time.time() - t0:.1f} s, dt = {dt!r}", flush=True)
    e, h, d, b, en = S.step(e0, h, dt, nsteps=STEPS, d=d0, b=b, energy_every=ENERGY_EVERY)
    print(f"{STEPS} steps done after {time.time() - t0:.1f} s", flush=True)
    np.savez(OUT, p=P, N=N, steps=STEPS, dt=dt, energy_every=ENERGY_EVERY, energies=np.array(en),
             e=e, h=h, d=d, b=b)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
