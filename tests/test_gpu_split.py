"""GPU parity of the composed (higher-order symplectic) steps against the
FP64 oracle: order 2 is the leapfrog bit for bit, orders 4 and 6 match the
oracle's compositions to 1e-12 per field (the same operators applied 3 and 9
times per step), under the tiled and tiled-dense plans, with tracking."""
import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_order_two_equals_the_leapfrog_bitwise():
    import torch
    import paper_2302_04979_amd as K
    S, G = make_pair(3, 5)
    print("\n[case] split order 2 vs kmx_step, p=3 N=5", flush=True)
    E0 = to_dev(W.random_vector(2 * G.n_e, 1))
    H0 = to_dev(W.random_vector(2 * G.n_h, 2))
    E1, H1, E2, H2 = E0.clone(), H0.clone(), E0.clone(), H0.clone()
    G.set_plan(K.PLAN_TILED)
    G.step(E1, H1, 0.01, nsteps=5, flags=K.TRACK_DB)
    G.step_split(E2, H2, 0.01, 5, 2, flags=K.TRACK_DB)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(H1, H2)


@pytest.mark.parametrize("order,plan", [(4, "tiled"), (6, "tiled"), (4, "tiled-dense")])
def test_composed_steps_match_oracle(order, plan):
    import paper_2302_04979_amd as K
    from oracle.scheme import composition_weights
    S, G = make_pair(3, 6)
    print(f"\n[case] split order {order} plan {plan}, p=3 N=6 deformed", flush=True)
    G.set_plan(K.PLAN_TILED if plan == "tiled" else K.PLAN_TILED_DENSE)
    d0 = W.random_vector(S.n_e, 3)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    dt, n = 0.004, 4
    c1 = composition_weights(order)[0]
    h_o, b_o = S.init_stagger(e0, np.zeros(S.n_h), c1 * dt, np.zeros(S.n_h))
    e_o, h_o, d_o, b_o = S.step_split(e0, h_o, dt, n, order, d=d0, b=b_o)
    E = to_dev(np.concatenate([e0, d0]))
    H = to_dev(np.zeros(2 * S.n_h))
    G.init_split(E, H, dt, order, flags=K.TRACK_DB)
    G.step_split(E, H, dt, n, order, flags=K.TRACK_DB)
    Eh, Hh = to_host(E), to_host(H)
    assert relmax(Eh[:S.n_e], e_o) < 1e-12
    assert relmax(Eh[S.n_e:], d_o) < 1e-12
    assert relmax(Hh[:S.n_h], h_o) < 1e-12
    assert relmax(Hh[S.n_h:], b_o) < 1e-12


def test_separable_plan_refused_and_bad_order():
    import paper_2302_04979_amd as K
    G = K.Space(2, 4)
    E = to_dev(np.zeros(G.n_e))
    H = to_dev(np.zeros(G.n_h))
    G.set_plan(K.PLAN_SEPARABLE)
    with pytest.raises(K.KMXError):
        G.step_split(E, H, 0.01, 1, 4)
    G.set_plan(K.PLAN_AUTO)
    with pytest.raises(K.KMXError):
        G.step_split(E, H, 0.01, 1, 3)


def test_full_size_composed_steps():
    """p=3, 64^3 deformed cube (the benchmark's space, tiled-dense plan): the
    order-2 composition equals kmx_step bit for bit, and after order-4 steps
    with tracking the Hodge relation K1 e = M~ d still holds (the GPU's
    operator entry points, themselves checked against the oracle)."""
    import torch
    import paper_2302_04979_amd as K
    p, N = 3, 64
    print("\n[case] composed steps full size p=3 N=64", flush=True)
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements(N, 0))
    G.set_plan(K.PLAN_TILED_DENSE)
    E0 = to_dev(W.random_vector(2 * G.n_e, 21))
    H0 = to_dev(W.random_vector(2 * G.n_h, 22))
    E1, H1, E2, H2 = E0.clone(), H0.clone(), E0.clone(), H0.clone()
    G.step(E1, H1, 1e-3, nsteps=2, flags=K.TRACK_DB)
    G.step_split(E2, H2, 1e-3, 2, 2, flags=K.TRACK_DB)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(H1, H2)
    # consistent start: d random, e = K1^{-1} M~ d, h = b = 0
    n_e = G.n_e
    E = torch.zeros(2 * n_e, dtype=torch.float64, device="cuda")
    E[n_e:] = to_dev(W.random_vector(n_e, 23))
    y = torch.empty(n_e, dtype=torch.float64, device="cuda")
    G.op_mass("D", E[n_e:].contiguous(), y)
    e = torch.empty_like(y)
    G.op_solve("K1", y, e)
    E[:n_e] = e
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.init_split(E, H, 2e-3, 4, flags=K.TRACK_DB)
    G.step_split(E, H, 2e-3, 3, 4, flags=K.TRACK_DB)
    Ke, Md = torch.empty_like(y), torch.empty_like(y)
    G.op_pairing("K1", E[:n_e].contiguous(), Ke)
    G.op_mass("D", E[n_e:].contiguous(), Md)
    assert float(torch.linalg.norm(Ke - Md) / torch.linalg.norm(Md)) < 1e-12


def test_full_size_order4_step_matches_oracle():
    """p=3, 64^3 deformed cube with random eps under the dense plan: one
    order-4 composed step (three substeps) from a random state against the
    oracle's composition."""
    import paper_2302_04979_amd as K
    S, G = make_pair(3, 64)
    print("\n[case] composed order 4 vs oracle, p=3 N=64", flush=True)
    G.set_plan(K.PLAN_TILED_DENSE)
    e0 = W.random_vector(S.n_e, 8, 31)
    h0 = W.random_vector(S.n_h, 8, 32)
    dt = 1e-3
    e, h, _, _ = S.step_split(e0, h0, dt, 1, 4)
    E, H = to_dev(e0), to_dev(h0)
    G.step_split(E, H, dt, 1, 4)
    assert relmax(to_host(E) - e0, e - e0) < 1e-12
    assert relmax(to_host(H) - h0, h - h0) < 1e-12
