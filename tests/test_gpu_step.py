"""GPU parity of the whole leapfrog step against the FP64 oracle, plus the
invariants that hold at any size (energy, determinism, batching)."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def _state(S, seed):
    """Consistent d^0, e^0 = K1^{-1} M~ d^0 and a random h^{-1/2}, b^{-1/2}."""
    d0 = W.random_vector(S.n_e, seed, 21)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    h0 = W.random_vector(S.n_h, seed, 22) * 0.1
    b0 = W.random_vector(S.n_h, seed, 23) * 0.1
    return e0, d0, h0, b0


@pytest.mark.parametrize("p,N,deformed,nsteps", [(2, 5, True, 30), (3, 6, True, 25), (4, 4, True, 15),
                                                 (3, 8, False, 20)])
def test_step_matches_oracle(p, N, deformed, nsteps):
    print(f"\n[case] step p={p} N={N} deformed={deformed} nsteps={nsteps}", flush=True)
    S, G = make_pair(p, N, deformed=deformed)
    e0, d0, h0, b0 = _state(S, 1)
    dt = 0.02 / p
    E, H = to_dev(e0), to_dev(h0)
    G.step(E, H, dt, nsteps=nsteps)
    e, h, _, _, _ = S.step(e0, h0, dt, nsteps=nsteps)
    assert relmax(to_host(E), e) < 1e-12
    assert relmax(to_host(H), h) < 1e-12


def test_tracking_and_energy_match_oracle():
    import torch
    S, G = make_pair(3, 5, deformed=True)
    e0, d0, _, _ = _state(S, 2)
    dt = 0.01
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    E = to_dev(np.concatenate([e0, d0]))
    H = to_dev(np.zeros(2 * S.n_h))
    G.init_stagger(E, H, dt, flags=1)
    Hh = to_host(H)
    assert relmax(Hh[:S.n_h], h) < 1e-13 and relmax(Hh[S.n_h:], b) < 1e-13
    nsteps = 40
    en = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=nsteps, flags=1, energy=en)
    e, h, d, b, en_ref = S.step(e0, h, dt, nsteps=nsteps, d=d0, b=b, energy_every=1)
    Eh, Hh = to_host(E), to_host(H)
    for got, ref in ((Eh[:S.n_e], e), (Eh[S.n_e:], d), (Hh[:S.n_h], h), (Hh[S.n_h:], b)):
        assert relmax(got, ref) < 1e-12
    en = to_host(en)
    assert np.abs(en - np.array(en_ref)).max() < 1e-12 * abs(en_ref[0])
    assert np.abs(en / en[0] - 1).max() < 1e-13  # the leapfrog invariant
    both = G.energy(E, H, dt)[0]
    mod, paper = S.energy(e, h, d, b, dt)
    assert abs(both[0] - mod) < 1e-12 * abs(mod) and abs(both[1] - paper) < 1e-12 * abs(paper)


def test_cavity_mode_config_p2_n8():
    """p=2, 8^3 elements, identity map, eps = mu = 1, J = 0, E0 = the (1,1,0)
    mode, dt = 0.5 CFL (oracle CFL), 100 steps: parity, energy, analytic mode."""
    import torch
    S, G = make_pair(2, 8, deformed=False, eps=False)
    dt = 0.5 * S.cfl(iters=3000, tol=1e-11)
    modes = W.mode_110()
    xq = G.quad_points()
    e_gpu = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    G.project_E(W.eval_modes(modes, xq), e_gpu[:G.n_e])
    G.project_D(W.eval_modes(modes, xq), e_gpu[G.n_e:], tol=1e-14)
    e0 = S.project_E(lambda x: W.eval_modes(modes, x))
    d0 = S.project_D(lambda x: W.eval_modes(modes, x))
    E0h = to_host(e_gpu)
    assert relmax(E0h[:G.n_e], e0) < 1e-13
    assert relmax(E0h[G.n_e:], d0) < 1e-11
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.init_stagger(e_gpu, H, dt, flags=1)
    en = torch.zeros(100, dtype=torch.float64, device="cuda")
    G.step(e_gpu, H, dt, nsteps=100, flags=1, energy=en)
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    e, h, d, b, _ = S.step(e0, h, dt, nsteps=100, d=d0, b=b)
    assert relmax(to_host(e_gpu)[:G.n_e], e) < 1e-12
    assert relmax(to_host(H)[:G.n_h], h) < 1e-12
    en = to_host(en)
    assert np.abs(en / en[0] - 1).max() < 1e-13
    # loose analytic check: dispersion dominates at this resolution
    T = 100 * dt
    Eex = W.eval_modes(modes, S.quad_points()) * math.cos(W.mode_omega(modes)[0] * T)
    err = math.sqrt(S.l2_norm_sq_quad(S.field_at_quad("E", e) - Eex) / S.l2_norm_sq_quad(Eex))
    assert err < 0.2  # phase error (omega_h - omega) T is about 0.11 rad alone


def test_point_sources_match_oracle():
    S, G = make_pair(3, 6, deformed=True)
    dt = 0.01
    dip = W.dipoles(3, seed=4, dt=dt)
    src = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"])
    s = [S.dipole_source(dip["pos"][k], dip["moment"][k]) for k in range(3)]

    def s_of_t(t):
        return sum(dip["amp"][k] * math.exp(-(t - dip["t0"][k]) ** 2 / (2 * dip["sigma"][k] ** 2)) * s[k]
                   for k in range(3))

    E = to_dev(np.zeros(S.n_e))
    H = to_dev(np.zeros(S.n_h))
    G.step(E, H, dt, nsteps=60, J=src)
    e, h, _, _, _ = S.step(np.zeros(S.n_e), np.zeros(S.n_h), dt, nsteps=60, source=s_of_t)
    assert np.linalg.norm(e) > 0
    assert relmax(to_host(E), e) < 1e-12 and relmax(to_host(H), h) < 1e-12


def test_batch_members_equal_single_runs_bitwise():
    S, G = make_pair(3, 5, deformed=True, max_batch=3)
    dt = 0.01
    states = [_state(S, 10 + k) for k in range(3)]
    E = to_dev(np.concatenate([s[0] for s in states]))
    H = to_dev(np.concatenate([s[2] for s in states]))
    G.step(E, H, dt, nsteps=12, batch=3)
    Eb, Hb = to_host(E), to_host(H)
    for k, st in enumerate(states):
        E1, H1 = to_dev(st[0]), to_dev(st[2])
        G.step(E1, H1, dt, nsteps=12)
        assert np.array_equal(Eb[k * S.n_e:(k + 1) * S.n_e], to_host(E1))
        assert np.array_equal(Hb[k * S.n_h:(k + 1) * S.n_h], to_host(H1))


def test_batched_per_step_energies():
    """The per-step energies of a batch of tracked runs: each member's series
    equals its single run's bit for bit and the oracle's, for runs of one
    step and of several (a step's energy is summed inside the next step's
    launch, the last one by a launch of its own), and the same run made as
    two calls gives the oracle's series too."""
    import torch
    S, G = make_pair(3, 5, deformed=True, max_batch=3)
    dt = 0.01
    states = [_state(S, 60 + k) for k in range(3)]
    for nsteps in (1, 2, 7):
        print(f"\n[case] batched energies nsteps={nsteps}", flush=True)
        E = to_dev(np.concatenate([np.concatenate([st[0], st[1]]) for st in states]))
        H = to_dev(np.concatenate([np.concatenate([st[2], st[3]]) for st in states]))
        en = torch.full((nsteps, 3), float("nan"), dtype=torch.float64, device="cuda")
        G.step(E, H, dt, nsteps=nsteps, batch=3, flags=1, energy=en)
        en = to_host(en)
        for k, (e0, d0, h0, b0) in enumerate(states):
            E1 = to_dev(np.concatenate([e0, d0]))
            H1 = to_dev(np.concatenate([h0, b0]))
            single = torch.full((nsteps,), float("nan"), dtype=torch.float64, device="cuda")
            G.step(E1, H1, dt, nsteps=nsteps, flags=1, energy=single)
            assert np.array_equal(en[:, k], to_host(single)), (nsteps, k)
            ref = np.array(S.step(e0, h0, dt, nsteps=nsteps, d=d0, b=b0, energy_every=1)[4])
            assert np.abs(en[:, k] - ref).max() < 1e-12 * np.abs(ref).max(), (nsteps, k)
            if nsteps > 1:  # the same run as two calls (the second re-forms K1 e and K~1 h)
                E1 = to_dev(np.concatenate([e0, d0]))
                H1 = to_dev(np.concatenate([h0, b0]))
                first = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
                rest = torch.full((nsteps - 1,), float("nan"), dtype=torch.float64, device="cuda")
                G.step(E1, H1, dt, nsteps=1, flags=1, energy=first)
                G.step(E1, H1, dt, nsteps=nsteps - 1, flags=1, energy=rest)
                two = np.concatenate([to_host(first), to_host(rest)])
                assert np.abs(two - ref).max() < 1e-12 * np.abs(ref).max(), (nsteps, k)


@pytest.mark.parametrize("p,N", [(2, 7), (4, 5), (3, 9)])
def test_per_step_energies_match_oracle_across_degrees(p, N):
    """Per-step energies of a tracked batch of two against the oracle's, at
    degrees whose 1- and 2-form components differ in shape (every position
    of the box of the three 2-form components and the e values around it).
    The random b and h are not each other's Hodge images, so the series
    is not constant: it is compared entry by entry."""
    import torch
    print(f"\n[case] energies p={p} N={N}", flush=True)
    S, G = make_pair(p, N, deformed=True, max_batch=2)
    dt, n = 0.01 / p, 6
    states = [_state(S, 80 + k) for k in range(2)]
    E = to_dev(np.concatenate([np.concatenate([st[0], st[1]]) for st in states]))
    H = to_dev(np.concatenate([np.concatenate([st[2], st[3]]) for st in states]))
    en = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=n, batch=2, flags=1, energy=en)
    en = to_host(en)
    for k, (e0, d0, h0, b0) in enumerate(states):
        ref = np.array(S.step(e0, h0, dt, nsteps=n, d=d0, b=b0, energy_every=1)[4])
        assert np.abs(en[:, k] - ref).max() < 1e-12 * np.abs(ref).max(), k


def test_graph_replays_of_tracked_steps_with_energy_equal_eager():
    """A captured run of tracked steps with per-step energies (a step's
    energy summed inside the next step's launch, the last one by a launch of
    its own) for a batch of two, replayed three times from the same state
    with eager work in between: fields and energies equal the eager run's
    bit for bit on every replay."""
    import torch
    S, G = make_pair(3, 6, deformed=True, max_batch=2)
    dt, n = 0.01, 9
    states = [_state(S, 70 + k) for k in range(2)]
    E0 = to_dev(np.concatenate([np.concatenate([st[0], st[1]]) for st in states]))
    H0 = to_dev(np.concatenate([np.concatenate([st[2], st[3]]) for st in states]))
    E, H = E0.clone(), H0.clone()
    en = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=n, batch=2, flags=1, energy=en)
    Eg, Hg = E0.clone(), H0.clone()
    en_g = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
    gr = G.graph(Eg, Hg, dt, n, batch=2, flags=1, energy=en_g)
    try:
        for rep in range(3):
            print(f"\n[case] graph replay {rep}", flush=True)
            Eg.copy_(E0)
            Hg.copy_(H0)
            en_g.fill_(float("nan"))
            G.set_time(0.0)
            gr.launch()
            torch.cuda.synchronize()
            assert torch.equal(Eg, E) and torch.equal(Hg, H), rep
            assert torch.equal(en_g, en), rep
            # eager work on the same space between the replays
            e2, h2 = E0.clone(), H0.clone()
            G.step(e2, h2, dt, nsteps=2, batch=2, flags=1,
                   energy=torch.zeros((2, 2), dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
    finally:
        gr.close()


def test_run_to_run_bitwise_determinism():
    S, G = make_pair(3, 8, deformed=True)
    e0, _, h0, _ = _state(S, 5)
    outs = []
    for _ in range(2):
        E, H = to_dev(e0), to_dev(h0)
        G.step(E, H, 0.01, nsteps=10)
        outs.append((to_host(E), to_host(H)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_cfl_matches_oracle():
    S, G = make_pair(2, 6, deformed=True)
    c_ref = S.cfl(iters=4000, tol=1e-12)
    c = G.cfl(max_iter=4000, tol=1e-12)
    assert abs(c - c_ref) < 1e-6 * c_ref


def test_deformed_32_config_short_parity_and_long_energy():
    """p=3, 32^3 deformed cube, eps ~ U[1,4], 10 cavity modes: 5-step parity
    with the oracle, and the leapfrog invariant over 1000 steps."""
    import torch
    S, G = make_pair(3, 32, deformed=True)
    modes = W.cavity_modes(0)
    xq = G.quad_points()
    Eq = W.eval_modes(modes, xq)
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    G.project_E(Eq, E[:G.n_e])
    e0 = S.project_E(lambda x: W.eval_modes(modes, x))
    assert relmax(to_host(E)[:G.n_e], e0) < 1e-13
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-6)
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    Es, Hs = E[:G.n_e].clone(), H[:G.n_h].clone()
    G.init_stagger(Es, Hs, dt)
    G.step(Es, Hs, dt, nsteps=5)
    h, _ = S.init_stagger(e0, np.zeros(S.n_h), dt)
    e, h, _, _, _ = S.step(e0, h, dt, nsteps=5)
    assert relmax(to_host(Es), e) < 1e-12 and relmax(to_host(Hs), h) < 1e-12
    # long run with tracking: d^0 by CG on the device
    G.project_D(Eq, E[G.n_e:], tol=1e-14)
    G.init_stagger(E, H, dt, flags=1)
    en = torch.zeros(1000, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=1000, flags=1, energy=en)
    en = to_host(en)
    assert np.isfinite(en).all()
    assert np.abs(en / en[0] - 1).max() < 1e-11


def test_metric_config_one_step_sampled_parity():
    """p=3, 64^3 deformed cube with random eps, the configuration the benchmark
    times: one step from a random state against the oracle."""
    import paper_2302_04979_amd as K
    S, G = make_pair(3, 64, deformed=True)
    e0 = W.random_vector(S.n_e, 7, 31)
    h0 = W.random_vector(S.n_h, 7, 32)
    dt = 1e-3
    e, h, _, _, _ = S.step(e0, h0, dt, nsteps=1)
    # the banded plan and the dense plan the benchmark's tuner picks at this size
    for plan in (K.PLAN_TILED, K.PLAN_TILED_DENSE):
        G.set_plan(plan)
        E, H = to_dev(e0), to_dev(h0)
        G.step(E, H, dt, nsteps=1)
        assert relmax(to_host(E) - e0, e - e0) < 1e-12
        assert relmax(to_host(H) - h0, h - h0) < 1e-12
