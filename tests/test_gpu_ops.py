"""GPU parity of each step of the path against the FP64 oracle (one operator
at a time): curls, fused curl + mass applies, pairing applies and Kronecker
solves.  Sizes span several 4^3-element tiles and ragged tails."""
import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [(2, 1, True), (3, 2, True), (2, 3, True), (2, 9, True), (3, 4, False), (3, 5, True), (3, 8, True),
         (4, 6, True)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"p{c[0]}N{c[1]}{'def' if c[2] else 'id'}")
def pair(request):
    p, N, deformed = request.param
    print(f"\n[case] p={p} N={N} deformed={deformed}", flush=True)
    return make_pair(p, N, deformed=deformed)


def test_curls_bitwise(pair):
    S, G = pair
    import torch
    x = W.random_vector(S.n_e, 1)
    y = torch.zeros(S.n_h, dtype=torch.float64, device="cuda")
    G.op_curl(True, to_dev(x), y)
    assert np.array_equal(to_host(y), S.curl_primal(x))
    h = W.random_vector(S.n_h, 2)
    d = torch.zeros(S.n_e, dtype=torch.float64, device="cuda")
    G.op_curl(False, to_dev(h), d)
    assert np.array_equal(to_host(d), S.curl_dual(h))


@pytest.mark.parametrize("space", ["B", "D"])
def test_mass_apply(pair, space):
    S, G = pair
    import torch
    n = S.n_h if space == "B" else S.n_e
    x = W.random_vector(n, 3)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.op_mass(space, to_dev(x), y)
    assert relmax(to_host(y), S.mass_apply(space, x)) < 1e-13


@pytest.mark.parametrize("space", ["B", "D"])
def test_fused_curl_mass_apply(pair, space):
    S, G = pair
    import torch
    n_in, n_out = (S.n_e, S.n_h) if space == "B" else (S.n_h, S.n_e)
    x = W.random_vector(n_in, 4)
    y = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    G.op_mass(space, to_dev(x), y, curl=True)
    ref = S.mass_apply(space, S.curl(x, space == "B"))
    assert relmax(to_host(y), ref) < 1e-13


@pytest.mark.parametrize("which", ["K1", "K1t"])
def test_pairing_apply(pair, which):
    S, G = pair
    import torch
    n = S.n_e if which == "K1" else S.n_h
    x = W.random_vector(n, 5)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.op_pairing(which, to_dev(x), y)
    assert relmax(to_host(y), S.kron_apply(which, x)) < 1e-14


@pytest.mark.parametrize("which", ["K1", "K1t"])
@pytest.mark.parametrize("transpose", [False, True])
def test_kronecker_solve(pair, which, transpose):
    S, G = pair
    import torch
    n = S.n_e if which == "K1" else S.n_h
    y = W.random_vector(n, 6)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    G.op_solve(which, to_dev(y), x, transpose=transpose)
    assert relmax(to_host(x), S.kron_solve(which, y, transpose=transpose)) < 1e-13
    # in place (x and y may alias)
    t = to_dev(y)
    G.op_solve(which, t, t, transpose=transpose)
    assert np.array_equal(to_host(t), to_host(x))


def _qp_param_points(p, N):
    """Parametric Gauss points in the element-major order of the library
    ([ez][ey][ex][iqz][iqy][iqx]), p+1 Gauss-Legendre points per element."""
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    x = (np.arange(N)[:, None] + 0.5 * (g[None, :] + 1.0)) / N  # [e][iq]
    X = np.broadcast_to(x[None, None, :, None, None, :], (N, N, N, p + 1, p + 1, p + 1))
    Y = np.broadcast_to(x[None, :, None, None, :, None], (N, N, N, p + 1, p + 1, p + 1))
    Z = np.broadcast_to(x[:, None, None, :, None, None], (N, N, N, p + 1, p + 1, p + 1))
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


@pytest.mark.parametrize("p,N", [(3, 5), (2, 8)])
def test_metric_modes_agree(p, N):
    """The mass apply with the metric recomputed in-kernel (sine map), streamed
    from memory (same map), and streamed from user Jacobians at the Gauss
    points (map kind 2, DF = I + a (1,1,1)^T grad s^T written out here) agree
    with each other and with the oracle."""
    import torch
    import paper_2302_04979_amd as K
    S, G1 = make_pair(p, N, deformed=True)
    eps = W.eps_elements(N, 0)
    G0 = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, stored_metric=True)
    G0.set_materials(eps=eps)
    xh = _qp_param_points(p, N)
    a = W.DEFORMED_AMPLITUDE
    sx, sy, sz = np.sin(np.pi * xh[:, 0]), np.sin(np.pi * xh[:, 1]), np.sin(np.pi * xh[:, 2])
    cx, cy, cz = np.cos(np.pi * xh[:, 0]), np.cos(np.pi * xh[:, 1]), np.cos(np.pi * xh[:, 2])
    grad = np.pi * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=1)
    DF = np.eye(3)[None] + a * np.ones(3)[None, :, None] * grad[:, None, :]
    G2 = K.Space(p, N, map_kind=2, dF_qp=DF.reshape(-1))
    G2.set_materials(eps=eps)
    for space, curl in (("B", True), ("D", True), ("D", False)):
        n_out = S.n_h if space == "B" else S.n_e
        n_in = (S.n_e if space == "B" else S.n_h) if curl else n_out
        x = W.random_vector(n_in, 8)
        ys = []
        for Gk in (G1, G0, G2):
            y = torch.zeros(n_out, dtype=torch.float64, device="cuda")
            Gk.op_mass(space, to_dev(x), y, curl=curl)
            ys.append(to_host(y))
        ref = S.mass_apply(space, S.curl(x, space == "B") if curl else x)
        for y in ys:
            assert relmax(y, ref) < 1e-13
        assert relmax(ys[0], ys[1]) < 1e-14 and relmax(ys[1], ys[2]) < 1e-14
