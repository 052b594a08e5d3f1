"""Full-length runs of the workloads against the oracle: the p=3, 32^3
deformed cube over all 1000 steps, and the mixed-precision solves and step at
the full line lengths of 64^3 (p = 3, 4).  Each field is compared by its
relative 2-norm and by an element-wise bound."""
import os

import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, maxrel, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "deformed32_1000.npz")


def test_deformed32_full_run_against_oracle():
    """p=3, 32^3 deformed cube, eps ~ U[1,4], 10 cavity modes, d and b tracked,
    dt = 0.5 CFL (the oracle's), 1000 steps: e, d, h, b after the run match
    the oracle's run (tests/golden/make_deformed32_golden.py) to 1e-12 per
    field, and the leapfrog invariant matches at every 50th step."""
    import torch
    import paper_2302_04979_amd as K
    g = np.load(GOLDEN)
    p, N, steps, dt = int(g["p"]), int(g["N"]), int(g["steps"]), float(g["dt"])
    print(f"\n[case] deformed cube p={p} N={N} {steps} steps dt={dt:.6e}", flush=True)
    _, G = make_pair(p, N, deformed=True)
    Eq = W.eval_modes(W.cavity_modes(0), G.quad_points())
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.project_E(Eq, E[:G.n_e])
    G.project_D(Eq, E[G.n_e:], tol=1e-15)
    G.init_stagger(E, H, dt, flags=K.TRACK_DB)
    en = torch.zeros(steps, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=steps, flags=K.TRACK_DB, energy=en)
    Eh, Hh = to_host(E), to_host(H)
    fields = {"e": Eh[:G.n_e], "d": Eh[G.n_e:], "h": Hh[:G.n_h], "b": Hh[G.n_h:]}
    for k, v in fields.items():
        r, m = rel(v, g[k]), maxrel(v, g[k])
        print(f"{k}: rel {r:.2e}, max {m:.2e}", flush=True)
        assert r < 1e-12 and m < 1e-11, k
    every = int(g["energy_every"])
    en_h = to_host(en)[every - 1::every]
    assert relmax(en_h, g["energies"]) < 1e-12


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("which,transpose", [("K1", False), ("K1t", False), ("K1", True), ("K1t", True)])
def test_mixed_solve_full_line_length(p, which, transpose):
    """At 64^3 (lines of 65-68 entries: every 16-row tile of the FP32 mode
    products, the ragged last one included) the refined mixed solve matches
    the FP64 oracle; without corrections it is FP32-accurate only."""
    import torch
    import paper_2302_04979_amd as K
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    print(f"\n[case] mixed solve p={p} N=64 {which} T={transpose}", flush=True)
    N = 64
    S = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE))
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED)
    n = S.n_e if which == "K1" else S.n_h
    y = W.random_vector(n, 8, 70 + p)
    ref = S.kron_solve(which, y, transpose=transpose)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.set_refinement(0)
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    e0 = rel(to_host(x), ref)
    G.set_refinement(2)
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    xh = to_host(x)
    print(f"rel error: FP32 only {e0:.2e}, refined {rel(xh, ref):.2e} (max {maxrel(xh, ref):.2e})", flush=True)
    assert 1e-9 < e0 < 1e-4
    assert rel(xh, ref) < 1e-13 and maxrel(xh, ref) < 1e-12


def test_mixed_step_full_size_p4():
    """p=4, 64^3 deformed cube with random eps (the mixed-precision
    workload's space): one mixed step from a random state matches the FP64
    oracle's step (the increments compared, to 1e-12)."""
    import torch
    import paper_2302_04979_amd as K
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    p, N, dt = 4, 64, 1e-3
    print(f"\n[case] mixed step p={p} N={N}", flush=True)
    eps = W.eps_elements(N, 0)
    S = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps)
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED)
    G.set_materials(eps=eps)
    e0 = W.random_vector(S.n_e, 9, 31)
    h0 = W.random_vector(S.n_h, 9, 32)
    E, H = to_dev(e0), to_dev(h0)
    G.step(E, H, dt, nsteps=1)
    e, h, _, _, _ = S.step(e0, h0, dt, nsteps=1)
    de, dh = to_host(E) - e0, to_host(H) - h0
    print(f"increments: e {rel(de, e - e0):.2e}, h {rel(dh, h - h0):.2e}", flush=True)
    assert rel(de, e - e0) < 1e-12 and maxrel(de, e - e0) < 1e-11
    assert rel(dh, h - h0) < 1e-12 and maxrel(dh, h - h0) < 1e-11
