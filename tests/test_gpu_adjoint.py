"""GPU adjoint (permittivity gradient of a probe misfit) against the oracle
adjoint and against finite differences of the GPU forward model."""
import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def _dipole(dt):
    dip = W.dipoles(1, seed=3, dt=dt)
    dip["t0"] = np.array([10 * dt])
    dip["sigma"] = np.array([4 * dt])
    return dip


@pytest.mark.parametrize("p,N,nsteps,ckpt", [(2, 5, 40, 10), (3, 4, 30, 7)])
def test_adjoint_matches_oracle(p, N, nsteps, ckpt):
    import torch
    import paper_2302_04979_amd as K
    from oracle.adjoint import ProbeProblem
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    print(f"\n[case] adjoint p={p} N={N} nsteps={nsteps} ckpt={ckpt}", flush=True)
    dt = 0.01
    dip = _dipole(dt)
    probes = W.probes(6, seed=2)
    eps_true = W.eps_elements(N, 0, purpose="eps_true")
    eps0 = W.eps_elements(N, 0) * 0.5 + 1.0
    S_true = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps_true)
    data = ProbeProblem(S_true, dip, probes, dt, nsteps).forward()
    S = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps0)
    L_ref, g_ref = ProbeProblem(S, dip, probes, dt, nsteps).gradient(data)

    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    prob = K.ProbeMisfitProblem(G, dip, probes, to_dev(data.reshape(-1)), dt, nsteps, checkpoint_every=ckpt)
    # forward probe values match the oracle
    obs = prob.observe(eps_true)
    assert relmax(to_host(obs).reshape(-1), data.reshape(-1)) < 1e-12
    L, g = prob.loss_and_grad(eps0)
    g = to_host(g)
    assert abs(L - L_ref) < 1e-10 * abs(L_ref)
    assert np.abs(g - g_ref).max() < 1e-10 * np.abs(g_ref).max()
    # checkpoint spacing does not change the result (recomputation is bitwise)
    prob2 = K.ProbeMisfitProblem(G, dip, probes, to_dev(data.reshape(-1)), dt, nsteps, checkpoint_every=nsteps)
    L2, g2 = prob2.loss_and_grad(eps0)
    assert L2 == L and np.array_equal(to_host(g2), g)


def test_autograd_function_and_directional_fd():
    import torch
    import paper_2302_04979_amd as K
    p, N, nsteps, dt = 3, 5, 40, 0.01
    dip = _dipole(dt)
    probes = W.probes(8, seed=5)
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    prob0 = K.ProbeMisfitProblem(G, dip, probes, torch.zeros(nsteps * 24, dtype=torch.float64, device="cuda"),
                                 dt, nsteps, checkpoint_every=8)
    data = prob0.observe(W.eps_elements(N, 0, purpose="eps_true")).reshape(-1).clone()
    prob = K.ProbeMisfitProblem(G, dip, probes, data, dt, nsteps, checkpoint_every=8)
    eps = torch.full((N, N, N), 2.0, dtype=torch.float64, requires_grad=True)
    loss = K.probe_misfit(eps, prob)
    loss.backward()
    g = eps.grad.numpy()
    u = W.random_vector(N ** 3, 12).reshape(N, N, N)
    d = 1e-5

    def L(e):
        obs = prob.observe(e).reshape(-1)
        r = to_host(obs) - to_host(data)
        return 0.5 * float(r @ r)

    fd = (L(2.0 + d * u) - L(2.0 - d * u)) / (2 * d)
    assert abs(float(np.sum(g * u)) - fd) < 1e-6 * abs(fd)


def test_adjoint_full_size_directional_fd():
    """p=3, 32^3 deformed cube, eps = 2 start, one dipole, 64 probes, 500 steps,
    checkpoints every 50: directional derivative against central differences
    of the GPU forward model."""
    import torch
    import time
    import paper_2302_04979_amd as K
    p, N, nsteps = 3, 32, 500
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=np.full(N ** 3, 2.0))
    dt = 0.5 * G.cfl(max_iter=200, tol=1e-6)
    dip = W.dipoles(1, seed=0, dt=dt, margin=0.2)
    probes = W.probes(64, seed=0)
    prob0 = K.ProbeMisfitProblem(G, dip, probes, torch.zeros(nsteps * 192, dtype=torch.float64, device="cuda"),
                                 dt, nsteps, checkpoint_every=50)
    data = prob0.observe(W.eps_elements(N, 0, purpose="eps_true")).reshape(-1).clone()
    prob = K.ProbeMisfitProblem(G, dip, probes, data, dt, nsteps, checkpoint_every=50)
    eps0 = np.full((N, N, N), 2.0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    L, g = prob.loss_and_grad(eps0)
    g = to_host(g)
    print(f"\nadjoint gradient p=3 32^3 500 steps: {time.perf_counter() - t:.3f} s, loss {L:.6e}", flush=True)
    u = W.random_vector(N ** 3, 13).reshape(N, N, N)
    d = 1e-4

    def loss_of(e):
        r = to_host(prob.observe(e).reshape(-1)) - to_host(data)
        return 0.5 * float(r @ r)

    fd = (loss_of(eps0 + d * u) - loss_of(eps0 - d * u)) / (2 * d)
    assert abs(float(np.sum(g * u)) - fd) < 1e-6 * abs(fd)
