"""GPU parity of the first scheme (Section 3.3: 1-form mass matrices solved by
preconditioned CG) against the FP64 oracle: the 1-form mass applies, the mass
solves, one half step, several leapfrog steps, and the leapfrog invariant.

Tolerances.  The applies are sums of the same products in another order
(1e-13).  The solves stop at |y - M x| <= tol |y| (tol = 1e-14 here); the
oracle's CG goes to 1e-15.  The solution error is then at most
cond(M) * 1e-14 relative; cond(M) of the oracle's dense matrices at N = 3 is
190 / 27 (E / H, p = 2), 6.3e3 / 600 (p = 3) and 2.9e5 / 1.5e4 (p = 4), so the
bound is 1e-10 or below for p <= 3 and 3e-9 for p = 4, where the error
actually left by CG (smallest in the directions of large eigenvalues) stays
well below it.  Solutions and steps are compared at 1e-10 relative, the true
residual at 1e-12, the invariant's drift (the solve error only) at 1e-10."""
import numpy as np
import pytest

import workloads as W
from _helpers import rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-14
CASES = [(2, 1, True, False), (4, 2, True, False), (2, 3, True, False), (3, 5, True, False),
         (3, 8, True, False), (4, 6, True, False), (3, 4, False, False), (3, 5, True, True)]


def _make(p, N, deformed, stored):
    from oracle.geometry import Map
    from oracle.scheme1 import Scheme1
    import paper_2302_04979_amd as K
    eps, mu = W.eps_elements(N, 0), W.eps_elements(N, 1, 1.0, 2.0)
    geo = Map("sine", W.DEFORMED_AMPLITUDE) if deformed else Map("identity")
    S = Scheme1(p, N, geo, eps=eps, mu=mu)
    G = K.Space(p, N, map_kind=1 if deformed else 0, amplitude=W.DEFORMED_AMPLITUDE if deformed else 0.0,
                stored_metric=stored)
    G.set_materials(eps=eps, mu=mu)
    return S, G


@pytest.fixture(scope="module", params=CASES,
                ids=lambda c: f"p{c[0]}N{c[1]}{'def' if c[2] else 'id'}{'-stored' if c[3] else ''}")
def pair(request):
    p, N, deformed, stored = request.param
    print(f"\n[case] scheme 1 p={p} N={N} deformed={deformed} stored={stored}", flush=True)
    return _make(p, N, deformed, stored)


@pytest.mark.parametrize("space", ["E", "H"])
def test_mass1_apply(pair, space):
    S, G = pair
    import torch
    n = S.n_e if space == "E" else S.n_h
    x = W.random_vector(n, 3)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.op_mass1(space, to_dev(x), y)
    assert relmax(to_host(y), S.mass1_apply(space, x)) < 1e-13


@pytest.mark.parametrize("space", ["E", "H"])
def test_mass1_solve(pair, space):
    S, G = pair
    import torch
    n = S.n_e if space == "E" else S.n_h
    y = W.random_vector(n, 5)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    it = G.solve_mass1(space, to_dev(y), x, tol=TOL, max_iter=400)
    xg = to_host(x)
    ref, _ = S.mass1_solve(space, y)
    assert 0 < it < 400
    assert relmax(xg, ref) < 1e-10
    assert np.linalg.norm(y - S.mass1_apply(space, xg)) < 1e-12 * np.linalg.norm(y)
    # a second solve from the solution as the guess stops at once
    it2 = G.solve_mass1(space, to_dev(y), x, tol=1e-10, max_iter=400)
    assert it2 <= 1 and relmax(to_host(x), ref) < 1e-10


def test_half_steps(pair):
    S, G = pair
    import torch
    e = W.random_vector(S.n_e, 6)
    h0 = W.random_vector(S.n_h, 7)
    h = to_dev(h0)
    G.half_step_scheme1("H", to_dev(e), h, -0.3, tol=TOL)
    ref = h0 - 0.3 * S.mass1_solve("H", S.rhs_h(e))[0]
    assert relmax(to_host(h) - h0, ref - h0) < 1e-10
    e0 = W.random_vector(S.n_e, 8)
    eg = to_dev(e0)
    G.half_step_scheme1("E", to_dev(h0), eg, 0.25, tol=TOL)
    ref = e0 + 0.25 * S.mass1_solve("E", S.rhs_e(h0))[0]
    assert relmax(to_host(eg) - e0, ref - e0) < 1e-10


def test_leapfrog_parity_and_invariant(pair):
    S, G = pair
    import torch
    dt, nsteps = 0.1 / S.N, 12
    e0 = W.random_vector(S.n_e, 9)
    # staggered start from h^0 = 0 on both sides
    h_o, _ = S.init_stagger1(e0, np.zeros(S.n_h), dt)
    e_g, h_g = to_dev(e0), torch.zeros(S.n_h, dtype=torch.float64, device="cuda")
    G.half_step_scheme1("H", e_g, h_g, 0.5 * dt, tol=TOL)
    assert relmax(to_host(h_g), h_o) < 1e-10

    def invariant(e, h):
        hh = h.clone()
        G.half_step_scheme1("H", e, hh, -dt, tol=TOL)
        Me = torch.empty_like(e)
        Mh = torch.empty_like(h)
        G.op_mass1("E", e, Me)
        G.op_mass1("H", hh, Mh)
        return 0.5 * float(e @ Me + h @ Mh)

    E0 = invariant(e_g, h_g)
    its = G.step_scheme1(e_g, h_g, dt, nsteps, tol=TOL)
    e_o, h_o, _, _ = S.step1(e0, h_o, dt, nsteps)
    assert relmax(to_host(e_g), e_o) < 1e-10
    assert relmax(to_host(h_g), h_o) < 1e-10
    assert its[0] > 0 and its[1] > 0
    E1 = invariant(e_g, h_g)
    assert abs(E1 / E0 - 1) < 1e-10
    # the oracle's invariant of its own run agrees
    Eo = S.energy1_modified(e_o, h_o, h_o - dt * S.mass1_solve("H", S.rhs_h(e_o))[0])
    assert abs(E1 / Eo - 1) < 1e-10


def test_zero_steps_change_nothing():
    import torch
    import paper_2302_04979_amd as K
    G = K.Space(3, 4, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    e0, h0 = to_dev(W.random_vector(G.n_e, 1)), to_dev(W.random_vector(G.n_h, 2))
    e, h = e0.clone(), h0.clone()
    assert G.step_scheme1(e, h, 0.01, 0) == (0, 0)
    G.step_split(e, h, 0.01, 0, 4)
    G.step(e, h, 0.01, nsteps=0)
    torch.cuda.synchronize()
    assert torch.equal(e, e0) and torch.equal(h, h0)


def test_zero_rhs_and_errors():
    import torch
    import paper_2302_04979_amd as K
    G = K.Space(3, 4, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    n = G.n_h
    x = to_dev(W.random_vector(n, 1))
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert G.solve_mass1("H", y, x, tol=1e-12) == 0
    assert float(x.abs().max()) == 0.0
    with pytest.raises(K.KMXError):
        G.solve_mass1("H", y, x, tol=0.0)
    with pytest.raises(K.KMXError):
        G.solve_mass1("E", to_dev(W.random_vector(G.n_e, 2)), torch.zeros(G.n_e, dtype=torch.float64,
                                                                          device="cuda"), tol=1e-14, max_iter=1)


def test_cfl_scheme1_matches_dense_eigenvalue():
    """Power iteration on the GPU against the largest eigenvalue of the
    oracle's dense operator (p = 2, 3^3 deformed cube)."""
    import scipy.linalg as sla
    S, G = _make(2, 3, True, False)
    M = np.stack([S.mass1_apply("E", c) for c in np.eye(S.n_e)], 1)
    Mt = np.stack([S.mass1_apply("H", c) for c in np.eye(S.n_h)], 1)
    Ch = np.stack([S.rhs_h(c) for c in np.eye(S.n_e)], 1)
    lmax = sla.eigh(Ch.T @ np.linalg.solve(Mt, Ch), M, eigvals_only=True).max()
    ref = 2 / np.sqrt(lmax)
    dt = G.cfl_scheme1(max_iter=5000, tol=1e-12, cg_tol=1e-13)
    assert abs(dt / ref - 1) < 1e-6


def test_full_size_invariant_and_residual():
    """p=3, 64^3 deformed cube, eps ~ U[1,4] (the benchmark's space and PCG
    tolerance): the solve's residual, re-applied with the mass kernel, meets the
    tolerance, and the leapfrog invariant is kept over 10 steps (properties
    that hold at any size; the oracle's CG is too slow at this size)."""
    import torch
    import paper_2302_04979_amd as K
    p, N = 3, 64
    print("\n[case] scheme 1 full size p=3 N=64", flush=True)
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements(N, 0))
    y = to_dev(W.random_vector(G.n_e, 11))
    x = torch.zeros(G.n_e, dtype=torch.float64, device="cuda")
    G.solve_mass1("E", y, x, tol=1e-12, max_iter=400)
    Mx = torch.empty_like(x)
    G.op_mass1("E", x, Mx)
    assert float(torch.linalg.norm(y - Mx) / torch.linalg.norm(y)) < 2e-12
    dt = 0.002
    e = to_dev(W.random_vector(G.n_e, 12))
    h = torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
    G.half_step_scheme1("H", e, h, 0.5 * dt, tol=1e-13)

    def invariant():
        hh = h.clone()
        G.half_step_scheme1("H", e, hh, -dt, tol=1e-13)
        Me, Mh = torch.empty_like(e), torch.empty_like(h)
        G.op_mass1("E", e, Me)
        G.op_mass1("H", hh, Mh)
        return 0.5 * float(e @ Me + h @ Mh)

    E0 = invariant()
    G.step_scheme1(e, h, dt, 10, tol=1e-13)
    assert abs(invariant() / E0 - 1) < 1e-10


@pytest.mark.parametrize("p,N,deformed", [(2, 3, True), (3, 5, True), (3, 4, False)])
def test_project_E1_matches_oracle(p, N, deformed):
    """The L^2_eps projection of ten cavity modes onto X^1_{h,0} (host load
    vector, PCG on the device) against the oracle's projection."""
    import torch
    S, G = _make(p, N, deformed, False)
    modes = W.cavity_modes(0)
    Eq = W.eval_modes(modes, G.quad_points())
    e = torch.zeros(G.n_e, dtype=torch.float64, device="cuda")
    G.project_E1(Eq, e, tol=1e-14)
    ref = S.project_E1(lambda xyz: W.eval_modes(modes, xyz.reshape(-1, 3)).reshape(xyz.shape))
    assert relmax(to_host(e), ref) < 1e-10


def test_graph_captured_fixed_iteration_steps():
    """Steps captured as a HIP graph with fixed CG iteration counts: replays
    from the same state (with eager work and host reads in between) agree to
    rounding (each replay's solves start from the previous replay's solutions,
    the warm start), and match the oracle's steps to the solve tolerance."""
    import torch
    S, G = _make(3, 5, True, False)
    dt, nsteps = 0.02, 4
    e0 = W.random_vector(S.n_e, 21)
    h0, _ = S.init_stagger1(e0, np.zeros(S.n_h), dt)
    e, h = to_dev(e0), to_dev(h0)
    gr = G.graph_scheme1(e, h, dt, nsteps, 60, 40)
    outs = []
    for _ in range(3):
        e.copy_(to_dev(e0))
        h.copy_(to_dev(h0))
        torch.cuda.synchronize()
        gr.launch()
        torch.cuda.synchronize()
        outs.append((to_host(e), to_host(h)))
        G.op_mass1("E", e, torch.empty_like(e))  # eager work between replays
    gr.close()
    for eo, ho in outs[1:]:
        assert relmax(eo, outs[0][0]) < 1e-13 and relmax(ho, outs[0][1]) < 1e-13
    e_o, h_o, _, _ = S.step1(e0, h0, dt, nsteps)
    assert relmax(outs[0][0], e_o) < 1e-10 and relmax(outs[0][1], h_o) < 1e-10
