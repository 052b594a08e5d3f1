"""Mixed-precision pairing solves (FP32 dense mode products on the matrix
cores, FP64 banded residual refinement) against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from _helpers import rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(p, N, max_batch=1):
    import paper_2302_04979_amd as K
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    eps = W.eps_elements(N, 0)
    S = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps)
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED, max_batch=max_batch)
    G.set_materials(eps=eps)
    return S, G


@pytest.mark.parametrize("p,N", [(2, 7), (3, 5), (3, 17), (4, 6)])
@pytest.mark.parametrize("which", ["K1", "K1t"])
@pytest.mark.parametrize("transpose", [False, True])
def test_mixed_solve_refines_to_fp64(p, N, which, transpose):
    """Without refinement the FP32 solve is accurate to single precision only;
    two FP64-residual corrections bring it to the FP64 oracle."""
    import torch
    print(f"\n[case] mixed solve p={p} N={N} {which} T={transpose}", flush=True)
    S, G = _pair(p, N)
    n = S.n_e if which == "K1" else S.n_h
    y = W.random_vector(n, 6)
    ref = S.kron_solve(which, y, transpose=transpose)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.set_refinement(0)
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    e0 = rel(to_host(x), ref)
    G.set_refinement(1)
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    e1 = rel(to_host(x), ref)
    G.set_refinement(2)
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    e2 = rel(to_host(x), ref)
    print(f"rel error: 0 corrections {e0:.2e}, 1: {e1:.2e}, 2: {e2:.2e}", flush=True)
    assert 1e-9 < e0 < 1e-4      # the first solve really is FP32
    assert e1 < 1e-9
    assert e2 < 1e-13
    # in place
    t = to_dev(y)
    G.op_solve(which, t, t, transpose=transpose)
    assert np.array_equal(to_host(t), to_host(x))


def test_mixed_step_matches_oracle():
    """Deformed cube, random eps, two members with their own dipoles: the
    mixed-precision step matches the FP64 oracle to 1e-12."""
    import math
    import torch
    p, N, dt, nsteps = 3, 6, 0.01, 20
    S, G = _pair(p, N, max_batch=2)
    dip = W.dipoles(2, seed=4, dt=dt)
    dip["t0"] = np.array([8 * dt, 11 * dt])
    dip["sigma"] = np.array([3 * dt, 3 * dt])
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(2))
    E0 = W.random_vector(2 * S.n_e, 51) * 0.1
    H0 = W.random_vector(2 * S.n_h, 52) * 0.1
    E, H = to_dev(E0), to_dev(H0)
    G.step(E, H, dt, nsteps=nsteps, J=J, batch=2)
    Eg, Hg = to_host(E), to_host(H)
    for k in range(2):
        s = S.dipole_source(dip["pos"][k], dip["moment"][k])
        g = lambda t, k=k, s=s: dip["amp"][k] * math.exp(-(t - dip["t0"][k]) ** 2 / (2 * dip["sigma"][k] ** 2)) * s
        e, h, _, _, _ = S.step(E0[k * S.n_e:(k + 1) * S.n_e], H0[k * S.n_h:(k + 1) * S.n_h], dt, nsteps=nsteps,
                               source=g)
        assert relmax(Eg[k * S.n_e:(k + 1) * S.n_e], e) < 1e-12
        assert relmax(Hg[k * S.n_h:(k + 1) * S.n_h], h) < 1e-12


def test_mixed_tracking_energy_conserved():
    """With b, d tracking the leapfrog invariant computed in FP64 stays
    constant to round-off over 50 mixed-precision steps (J = 0)."""
    import torch
    import paper_2302_04979_amd as K
    p, N = 3, 8
    S, G = _pair(p, N)
    xq = G.quad_points()
    Eq = W.eval_modes(W.cavity_modes(0), xq)
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.project_E(Eq, E[:G.n_e])
    G.project_D(Eq, E[G.n_e:], tol=1e-13)
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-6)
    G.init_stagger(E, H, dt, flags=K.TRACK_DB)
    en = torch.zeros(50, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=50, flags=K.TRACK_DB, energy=en)
    v = to_host(en)
    assert np.abs(v / v[0] - 1).max() < 1e-12
