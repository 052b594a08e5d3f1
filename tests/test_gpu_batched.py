"""Batched sources under hipGraph: graph replays equal eager steps bitwise,
batch members equal their single-source runs, and the 256-source p=3, 24^3
configuration matches the oracle on sampled members."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_eager_steps():
    import torch
    S, G = make_pair(3, 5, deformed=True, max_batch=3)
    dt, K = 0.01, 7
    dip = W.dipoles(3, seed=6, dt=dt)
    dip["t0"] = np.array([8 * dt] * 3)
    dip["sigma"] = np.array([3 * dt] * 3)
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(3))
    E0 = W.random_vector(3 * S.n_e, 1) * 0.1
    H0 = W.random_vector(3 * S.n_h, 2) * 0.1
    # eager reference, three chunks of K steps
    Ee, He = to_dev(E0), to_dev(H0)
    ref = []
    for c in range(3):
        G.step(Ee, He, dt, nsteps=K, J=J, t_start=c * K * dt, batch=3)
        ref.append((to_host(Ee), to_host(He)))
    # graph: captured once, replayed three times with eager work in between
    Eg, Hg = to_dev(E0), to_dev(H0)
    gr = G.graph(Eg, Hg, dt, K, J=J, batch=3)
    G.set_time(0.0)
    scratch_in = to_dev(W.random_vector(S.n_e, 3))
    scratch_out = torch.zeros(S.n_e, dtype=torch.float64, device="cuda")
    for c in range(3):
        gr.launch()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Eg), ref[c][0]) and np.array_equal(to_host(Hg), ref[c][1])
        G.op_mass("D", scratch_in, scratch_out)  # unrelated eager work between replays
        torch.cuda.synchronize()
    assert abs(G.get_time() - 3 * K * dt) < 1e-14


def _oracle_member(S, dip, k, E0, H0, dt, nsteps, t0=0.0):
    import math
    s = S.dipole_source(dip["pos"][k], dip["moment"][k])
    g = lambda t: dip["amp"][k] * math.exp(-(t - dip["t0"][k]) ** 2 / (2 * dip["sigma"][k] ** 2)) * s
    e, h, _, _, _ = S.step(E0, H0, dt, nsteps=nsteps, t0=t0, source=g)
    return e, h


SEP_CASES = [(2, 5), (3, 6), (3, 9), (4, 4)]


@pytest.mark.parametrize("p,N", SEP_CASES)
def test_separable_plan_matches_oracle(p, N):
    """Identity map, uniform eps = 2.5 and mu = 1.5, two members each driven by
    its own dipole, started at t = 0.03: the separable persistent kernel
    matches the oracle member by member, and the tiled plan on the same
    inputs."""
    import torch
    import paper_2302_04979_amd as K
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    print(f"\n[case] separable p={p} N={N}", flush=True)
    n3 = N ** 3
    S = Scheme(p, N, Map("identity"), eps=np.full(n3, 2.5), mu=np.full(n3, 1.5))
    dt, nsteps, t_start = 0.01, 15, 0.03
    dip = W.dipoles(2, seed=4, dt=dt)
    dip["t0"] = np.array([8 * dt, 11 * dt])
    dip["sigma"] = np.array([3 * dt, 3 * dt])
    E0 = W.random_vector(2 * S.n_e, 21) * 0.1
    H0 = W.random_vector(2 * S.n_h, 22) * 0.1
    out = {}
    for plan in (K.PLAN_SEPARABLE, K.PLAN_SEPARABLE_FUSED, K.PLAN_TILED):
        G = K.Space(p, N, max_batch=2)
        G.set_materials(eps=np.full(n3, 2.5), mu=np.full(n3, 1.5))
        G.set_plan(plan, 256)
        J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(2))
        E, H = to_dev(E0), to_dev(H0)
        G.step(E, H, dt, nsteps=nsteps, J=J, t_start=t_start, batch=2)
        out[plan] = (to_host(E), to_host(H))
    for k in range(2):
        e, h = _oracle_member(S, dip, k, E0[k * S.n_e:(k + 1) * S.n_e], H0[k * S.n_h:(k + 1) * S.n_h], dt, nsteps,
                              t_start)
        for plan in (K.PLAN_SEPARABLE, K.PLAN_SEPARABLE_FUSED):
            Es, Hs = out[plan]
            assert relmax(Es[k * S.n_e:(k + 1) * S.n_e], e) < 1e-12
            assert relmax(Hs[k * S.n_h:(k + 1) * S.n_h], h) < 1e-12
    for plan in (K.PLAN_SEPARABLE, K.PLAN_SEPARABLE_FUSED):
        assert relmax(out[plan][0], out[K.PLAN_TILED][0]) < 1e-13
        assert relmax(out[plan][1], out[K.PLAN_TILED][1]) < 1e-13


def test_separable_thread_counts_agree_at_full_lines():
    """p=3, 24^3 (676 lines per pass, more than any workgroup has threads):
    every workgroup size gives the same bits, and the tiled plan agrees."""
    import paper_2302_04979_amd as K
    p, N, dt = 3, 24, 2e-3
    out = []
    for plan, threads in ((K.PLAN_SEPARABLE, 64), (K.PLAN_SEPARABLE, 256), (K.PLAN_SEPARABLE, 384),
                          (K.PLAN_SEPARABLE, 768), (K.PLAN_TILED, 768), (K.PLAN_SEPARABLE_FUSED, 64),
                          (K.PLAN_SEPARABLE_FUSED, 384), (K.PLAN_SEPARABLE_FUSED, 768)):
        G = K.Space(p, N)
        G.set_plan(plan, threads)
        E = to_dev(W.random_vector(G.n_e, 61))
        H = to_dev(W.random_vector(G.n_h, 62))
        G.step(E, H, dt, nsteps=3)
        out.append((to_host(E), to_host(H)))
    for k in (1, 2, 3):
        assert np.array_equal(out[k][0], out[0][0]) and np.array_equal(out[k][1], out[0][1])
    for k in (6, 7):
        assert np.array_equal(out[k][0], out[5][0]) and np.array_equal(out[k][1], out[5][1])
    for k in (4, 5):
        assert relmax(out[0][0], out[k][0]) < 1e-13 and relmax(out[0][1], out[k][1]) < 1e-13


@pytest.mark.parametrize("fused", [False, True])
def test_separable_plan_tracking_matches_oracle(fused):
    import paper_2302_04979_amd as K
    from oracle.scheme import Scheme
    p, N, dt, nsteps = 3, 7, 0.01, 12
    S = Scheme(p, N)
    G = K.Space(p, N)
    G.set_plan(K.PLAN_SEPARABLE_FUSED if fused else K.PLAN_SEPARABLE, 384)
    e0, h0 = W.random_vector(S.n_e, 31), W.random_vector(S.n_h, 32)
    d0, b0 = W.random_vector(S.n_e, 33), W.random_vector(S.n_h, 34)
    E, H = to_dev(np.concatenate([e0, d0])), to_dev(np.concatenate([h0, b0]))
    G.step(E, H, dt, nsteps=nsteps, flags=K.TRACK_DB)
    e, h, d, b, _ = S.step(e0, h0, dt, nsteps=nsteps, d=d0, b=b0)
    Eg, Hg = to_host(E), to_host(H)
    assert relmax(Eg[:S.n_e], e) < 1e-12 and relmax(Eg[S.n_e:], d) < 1e-12
    assert relmax(Hg[:S.n_h], h) < 1e-12 and relmax(Hg[S.n_h:], b) < 1e-12


def test_separable_plan_refuses_what_it_cannot_run():
    import torch
    import paper_2302_04979_amd as K
    S, G = make_pair(3, 4, deformed=True)
    G.set_plan(K.PLAN_SEPARABLE, 256)
    E = torch.zeros(S.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(S.n_h, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KMXError):
        G.step(E, H, 0.01, nsteps=1)
    G2 = K.Space(3, 4)
    G2.set_materials(eps=W.eps_elements(4, 0))  # non-uniform eps
    G2.set_plan(K.PLAN_SEPARABLE, 256)
    with pytest.raises(K.KMXError):
        G2.step(E, H, 0.01, nsteps=1)
    with pytest.raises(K.KMXError):
        G2.set_plan(K.PLAN_SEPARABLE, 100)  # not a multiple of 64


@pytest.mark.parametrize("fused", [False, True])
def test_separable_graph_replays_equal_eager_steps(fused):
    import torch
    import paper_2302_04979_amd as K
    p, N, B, Kst = 3, 6, 4, 9
    G = K.Space(p, N, max_batch=B)
    G.set_plan(K.PLAN_SEPARABLE_FUSED if fused else K.PLAN_SEPARABLE, 512)
    dt = 0.01
    dip = W.dipoles(B, seed=8, dt=dt)
    dip["t0"] = np.full(B, 10 * dt)
    dip["sigma"] = np.full(B, 4 * dt)
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(B))
    E0 = W.random_vector(B * G.n_e, 41) * 0.1
    H0 = W.random_vector(B * G.n_h, 42) * 0.1
    Ee, He = to_dev(E0), to_dev(H0)
    ref = []
    for c in range(3):
        G.step(Ee, He, dt, nsteps=Kst, J=J, t_start=c * Kst * dt, batch=B)
        ref.append((to_host(Ee), to_host(He)))
    Eg, Hg = to_dev(E0), to_dev(H0)
    gr = G.graph(Eg, Hg, dt, Kst, J=J, batch=B)
    G.set_time(0.0)
    for c in range(3):
        gr.launch()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Eg), ref[c][0]) and np.array_equal(to_host(Hg), ref[c][1])
        torch.zeros(1000, device="cuda").sum().item()  # unrelated eager work between replays


def test_batched_256_sources_p3_n24():
    """256 point dipoles (one per batch member) at seed-uniform positions and
    orientations, identity map, eps = mu = 1, zero initial fields, 400 steps
    in one persistent launch under a captured graph: members equal their own
    single-source runs, and a sampled member matches the oracle over the
    whole run of 400 steps."""
    import time
    import torch
    import paper_2302_04979_amd as K
    from oracle.scheme import Scheme
    p, N, B, nsteps = 3, 24, 256, 400
    G = K.Space(p, N, max_batch=B)
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-7)
    dip = W.dipoles(B, seed=0, dt=dt)
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(B))
    ms = G.tune(B, dt, probe_steps=3, J=J)
    print(f"\ntuning (ms/step): {ms} -> plan {G.plan()}", flush=True)
    assert ms[0] is not None and all(m is not None for m in ms[1:])
    if G.plan()[0] == K.PLAN_TILED:
        G.set_plan(K.PLAN_SEPARABLE, 768)
    kind, threads = G.plan()
    E = torch.zeros(B * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(B * G.n_h, dtype=torch.float64, device="cuda")
    gr = G.graph(E, H, dt, nsteps, J=J, batch=B)
    G.set_time(0.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    gr.launch()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    print(f"batched 256 x 400 steps (plan {kind}, {threads} threads): {el * 1e3:.1f} ms, "
          f"{(G.n_e + G.n_h) * B * nsteps / el:.3e} DOF-updates/s", flush=True)
    Eb = to_host(E)
    assert np.isfinite(Eb).all() and np.abs(Eb).max() > 0
    for k in (0, 97, 255):
        G1 = K.Space(p, N)
        G1.set_plan(kind, threads)
        J1 = G1.source(dip["pos"][k:k + 1], dip["moment"][k:k + 1], dip["t0"][k:k + 1], dip["sigma"][k:k + 1],
                       dip["amp"][k:k + 1])
        E1 = torch.zeros(G1.n_e, dtype=torch.float64, device="cuda")
        H1 = torch.zeros(G1.n_h, dtype=torch.float64, device="cuda")
        G1.step(E1, H1, dt, nsteps=nsteps, J=J1)
        assert np.array_equal(Eb[k * G.n_e:(k + 1) * G.n_e], to_host(E1))
    k, n_or = 97, nsteps
    S = Scheme(p, N)
    e, h = _oracle_member(S, dip, k, np.zeros(S.n_e), np.zeros(S.n_h), dt, n_or)
    G1 = K.Space(p, N)
    G1.set_plan(kind, threads)
    J1 = G1.source(dip["pos"][k:k + 1], dip["moment"][k:k + 1], dip["t0"][k:k + 1], dip["sigma"][k:k + 1],
                   dip["amp"][k:k + 1])
    E1 = torch.zeros(G1.n_e, dtype=torch.float64, device="cuda")
    H1 = torch.zeros(G1.n_h, dtype=torch.float64, device="cuda")
    G1.step(E1, H1, dt, nsteps=n_or, J=J1)
    assert relmax(to_host(E1), e) < 1e-12 and relmax(to_host(H1), h) < 1e-12
