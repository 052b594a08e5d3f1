"""GPU parity on the curved workload: the quarter coaxial cable of Section 5
as a degree-2 NURBS map, given to the library as Jacobians at the Gauss points
(map kind 2: the metric factors are streamed).  Scheme 2 operators and steps
with tracking and energy, and the first scheme's 1-form masses and half steps,
against the FP64 oracle on the same map."""
import numpy as np
import pytest

import workloads as W
from _helpers import qp_param_points, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(p, N):
    from oracle.geometry import Map
    from oracle.scheme1 import Scheme1
    import paper_2302_04979_amd as K
    eps = W.eps_elements(N, 0)
    S = Scheme1(p, N, Map("annulus"), eps=eps)
    _, DF = W.quarter_annulus_jacobian(qp_param_points(p, N))
    G = K.Space(p, N, map_kind=2, dF_qp=DF.reshape(-1))
    G.set_materials(eps=eps)
    return S, G


@pytest.mark.parametrize("p,N", [(2, 5), (3, 6), (4, 3)])
def test_annulus_operators_and_steps(p, N):
    import torch
    import paper_2302_04979_amd as K
    print(f"\n[case] annulus p={p} N={N}", flush=True)
    S, G = _pair(p, N)
    for space, curl in (("B", True), ("D", True), ("B", False)):
        n_out = S.n_h if space == "B" else S.n_e
        n_in = (S.n_e if space == "B" else S.n_h) if curl else n_out
        x = W.random_vector(n_in, 8)
        y = torch.zeros(n_out, dtype=torch.float64, device="cuda")
        G.op_mass(space, to_dev(x), y, curl=curl)
        assert relmax(to_host(y), S.mass_apply(space, S.curl(x, space == "B") if curl else x)) < 1e-13
    d0 = W.random_vector(S.n_e, 1)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    dt, n = 0.004, 5
    h0, b0 = S.init_stagger(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    E, H = to_dev(np.concatenate([e0, d0])), to_dev(np.concatenate([h0, b0]))
    en = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=n, flags=K.TRACK_DB, energy=en)
    e, h, d, b, en_ref = S.step(e0, h0, dt, nsteps=n, d=d0, b=b0, energy_every=1)
    Eg, Hg = to_host(E), to_host(H)
    assert relmax(Eg[:S.n_e], e) < 1e-12 and relmax(Eg[S.n_e:], d) < 1e-12
    assert relmax(Hg[:S.n_h], h) < 1e-12 and relmax(Hg[S.n_h:], b) < 1e-12
    assert np.abs(to_host(en) - np.array(en_ref)).max() < 1e-12 * abs(en_ref[0])


def test_annulus_first_scheme():
    import torch
    print("\n[case] annulus scheme 1 p=3 N=4", flush=True)
    S, G = _pair(3, 4)
    for space in ("E", "H"):
        n = S.n_e if space == "E" else S.n_h
        x = W.random_vector(n, 3)
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        G.op_mass1(space, to_dev(x), y)
        assert relmax(to_host(y), S.mass1_apply(space, x)) < 1e-13
    e = W.random_vector(S.n_e, 6)
    h = torch.zeros(S.n_h, dtype=torch.float64, device="cuda")
    G.half_step_scheme1("H", to_dev(e), h, 0.01, tol=1e-14)
    assert relmax(to_host(h), 0.01 * S.mass1_solve("H", S.rhs_h(e))[0]) < 1e-10


def test_separable_preconditioner_is_exact_on_the_coax():
    """With uniform material the coax's 1-form masses are Kronecker products
    (orthogonal product map): the preconditioned CG reaches 1e-13 after one
    iteration (the residual test lags one iteration behind, so two are run),
    and the solution matches the oracle's solve."""
    import torch
    from oracle.geometry import Map
    from oracle.scheme1 import Scheme1
    import paper_2302_04979_amd as K
    p, N = 3, 5
    print(f"\n[case] coax exact preconditioner p={p} N={N}", flush=True)
    S = Scheme1(p, N, Map("annulus"))
    _, DF = W.quarter_annulus_jacobian(qp_param_points(p, N))
    G = K.Space(p, N, map_kind=2, dF_qp=DF.reshape(-1))
    for space in ("E", "H"):
        n = S.n_e if space == "E" else S.n_h
        y = W.random_vector(n, 9)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        it = G.solve_mass1(space, to_dev(y), x, tol=1e-13)
        assert it <= 2
        assert relmax(to_host(x), S.mass1_solve(space, y)[0]) < 1e-11
