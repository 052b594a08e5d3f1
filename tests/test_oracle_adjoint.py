"""Pins of the oracle's adjoint leapfrog and permittivity gradient."""
import numpy as np
import pytest

import workloads as W
from oracle.adjoint import ProbeProblem, curl_T, elem_pairing, step_transpose
from oracle.geometry import Map
from oracle.scheme import Scheme

P_, N_, DT, NSTEPS = 2, 3, 0.01, 40


def _setup(eps):
    S = Scheme(P_, N_, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps)
    dip = W.dipoles(1, seed=3, dt=DT)
    dip["t0"] = np.array([10 * DT])
    dip["sigma"] = np.array([4 * DT])
    probes = W.probes(6, seed=2)
    return ProbeProblem(S, dip, probes, DT, NSTEPS)


def _data():
    return _setup(W.eps_elements(N_, 0, purpose="eps_true")).forward()


def test_curl_transposes():
    S = Scheme(3, 3, Map("sine", W.DEFORMED_AMPLITUDE))
    for primal, (n_in, n_out) in ((True, (S.n_e, S.n_h)), (False, (S.n_h, S.n_e))):
        x, y = W.random_vector(n_in, 1), W.random_vector(n_out, 2)
        assert abs(S.curl(x, primal) @ y - x @ curl_T(S, y, primal)) < 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)


def test_step_transpose_dot_product():
    """<J x, y> = <x, J^T y> for one source-free leapfrog step."""
    S = Scheme(3, 3, Map("sine", W.DEFORMED_AMPLITUDE), eps=W.eps_elements(3, 0))
    e, h = W.random_vector(S.n_e, 5), W.random_vector(S.n_h, 6)
    eb, hb = W.random_vector(S.n_e, 7), W.random_vector(S.n_h, 8)
    e1, h1, _, _, _ = S.step(e, h, 0.02)
    ea, ha = step_transpose(S, eb, hb, 0.02)
    lhs, rhs = e1 @ eb + h1 @ hb, e @ ea + h @ ha
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_elem_pairing_sums_to_mass_form():
    """sum over elements of lam^T M~_e^{(1)} v = lam^T M~^{(1)} v (unit eps)."""
    S = Scheme(2, 3, Map("sine", W.DEFORMED_AMPLITUDE))
    lam, v = W.random_vector(S.n_e, 9), W.random_vector(S.n_e, 10)
    assert abs(elem_pairing(S, lam, v).sum() - lam @ S.mass_apply("D", v)) < 1e-12 * abs(lam @ S.mass_apply("D", v))


def test_gradient_matches_central_differences():
    data = _data()
    eps0 = np.full((N_,) * 3, 2.0)
    L, g = _setup(eps0.copy()).gradient(data)
    pp = _setup(eps0.copy())
    el = np.minimum((pp.dip["pos"][0] * N_).astype(int), N_ - 1)
    idxs = [(0, 0, 0), (2, 1, 0), (el[2], el[1], el[0])]  # includes the dipole's element
    for idx in idxs:
        d = 1e-5 * eps0[idx]
        ep, em = eps0.copy(), eps0.copy()
        ep[idx] += d
        em[idx] -= d
        fd = (_setup(ep).loss(data) - _setup(em).loss(data)) / (2 * d)
        assert abs(g[idx] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (idx, g[idx], fd)


def test_gradient_directional_derivative():
    data = _data()
    eps0 = np.full((N_,) * 3, 2.0)
    _, g = _setup(eps0.copy()).gradient(data)
    u = W.random_vector(N_ ** 3, 11).reshape((N_,) * 3)
    d = 1e-5
    fd = (_setup(eps0 + d * u).loss(data) - _setup(eps0 - d * u).loss(data)) / (2 * d)
    assert abs(np.sum(g * u) - fd) < 1e-6 * abs(fd)
