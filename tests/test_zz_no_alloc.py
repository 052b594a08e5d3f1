"""The allocation-free probe forward run (fixed device working array) against
kmx_probe_forward on the same inputs: two calls in a row, the second on a
smaller space, through the C-ABI."""
import numpy as np
import pytest

import workloads as W
from _helpers import to_host

pytestmark = pytest.mark.gpu


def _run(p, N, nsteps, dt, seed):
    import torch
    import paper_2302_04979_amd as K
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements(N, seed))
    dip = W.dipoles(2, seed=seed, dt=dt)
    dip["t0"] = np.array([6 * dt, 9 * dt])
    dip["sigma"] = np.array([3 * dt, 3 * dt])
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"])
    pr = G.probes(W.probes(5, seed=seed))
    ref = torch.zeros(nsteps * 15, dtype=torch.float64, device="cuda")
    G.probe_forward(pr, J, dt, nsteps, ref)
    out = torch.full((nsteps * 15,), float("nan"), dtype=torch.float64, device="cuda")
    G.probe_forward_noalloc(pr, J, dt, nsteps, out)
    torch.cuda.synchronize()
    return to_host(out), to_host(ref)


def test_noalloc_probe_forward_matches_the_allocating_call():
    print("\n[case] noalloc probe forward p=3 N=6, then p=2 N=4", flush=True)
    out, ref = _run(3, 6, 25, 0.01, 1)
    assert np.abs(ref).max() > 0
    assert np.array_equal(out, ref)
    # the second call on a smaller space: the array still holds the first
    # call's fields, which must not leak into the result
    out, ref = _run(2, 4, 15, 0.02, 2)
    assert np.abs(ref).max() > 0
    assert np.array_equal(out, ref)


def test_noalloc_refuses_what_the_allocating_call_refuses():
    import torch
    import paper_2302_04979_amd as K
    G = K.Space(2, 4)
    pr = G.probes(W.probes(2, seed=3))
    obs = torch.zeros(6, dtype=torch.float64, device="cuda")
    c = G.cfl(max_iter=300, tol=1e-8)
    with pytest.raises(K.KMXError) as ex:
        G.probe_forward_noalloc(pr, None, 2.0 * c, 1, obs)
    assert ex.value.status == 6
