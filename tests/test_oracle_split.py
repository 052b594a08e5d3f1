"""Pins of the oracle's higher-order symplectic time stepping (compositions of
the leapfrog; the paper names pairing the scheme with higher-order symplectic
integrators as future work, Section 6)."""
import numpy as np
import pytest

import workloads as W
from oracle.geometry import Map
from oracle.scheme import Scheme, composition_weights


@pytest.mark.parametrize("order", [2, 4, 6])
def test_weights_consistent_symmetric_and_triple_jump(order):
    c = np.array(composition_weights(order))
    assert abs(c.sum() - 1.0) < 1e-15
    assert np.array_equal(c, c[::-1])
    assert len(c) == 3 ** (order // 2 - 1)
    if order > 2:
        # the triple jump cancels the leading error term: 2 z1^(2k+1) + z0^(2k+1) = 0
        k = order // 2 - 1
        z1 = c[0] / composition_weights(order - 2)[0]
        z0 = 1 - 2 * z1
        assert abs(2 * z1 ** (2 * k + 1) + z0 ** (2 * k + 1)) < 1e-14


def _small():
    return Scheme(2, 3, Map("sine", W.DEFORMED_AMPLITUDE), eps=W.eps_elements(3, 0))


def test_order_two_is_the_leapfrog():
    S = _small()
    e0 = W.random_vector(S.n_e, 1)
    h0 = W.random_vector(S.n_h, 2)
    e1, h1, _, _, _ = S.step(e0, h0, 0.01, nsteps=7)
    e2, h2, _, _ = S.step_split(e0, h0, 0.01, 7, 2)
    assert np.abs(e1 - e2).max() < 1e-14 * np.abs(e1).max()
    assert np.abs(h1 - h2).max() < 1e-14 * np.abs(h1).max()


def test_orders_against_the_exact_semidiscrete_solution():
    """The semi-discrete system e' = A_e h, h' = -A_h e (A_e = K1^{-1} M~ D~^1,
    A_h = K~1^{-1} M D^1) from e(0) = e0, h(0) = 0 is solved exactly by the
    matrix exponential of its dense generator; the compositions of order
    2, 4, 6 reach it at rates 2, 4, 6 in dt at fixed final time."""
    import scipy.linalg as sla
    S = _small()
    Ae = np.stack([S.half_step_e(c) for c in np.eye(S.n_h)], 1)
    Ah = np.stack([S.half_step_h(c) for c in np.eye(S.n_e)], 1)
    L = np.block([[np.zeros((S.n_e, S.n_e)), Ae], [-Ah, np.zeros((S.n_h, S.n_h))]])
    lmax = np.abs(np.linalg.eigvals(Ae @ Ah)).max()
    e0 = W.random_vector(S.n_e, 3)
    T = 10.0 / np.sqrt(lmax)
    ref = (sla.expm(T * L) @ np.concatenate([e0, np.zeros(S.n_h)]))[:S.n_e]
    for order in (2, 4, 6):
        c1 = composition_weights(order)[0]
        errs = []
        for n in (160, 320):
            dt = T / n
            h, _ = S.init_stagger(e0, np.zeros(S.n_h), c1 * dt)
            e, _, _, _ = S.step_split(e0, h, dt, n, order)
            errs.append(np.linalg.norm(e - ref) / np.linalg.norm(ref))
        rate = np.log2(errs[0] / errs[1])
        assert abs(rate - order) < 0.3, (order, errs)


def test_tracked_forms_keep_the_hodge_relations():
    """b and d follow the same kicks, so K1 e = M~ d stays exact and D^2 b is
    constant."""
    S = _small()
    d0 = W.random_vector(S.n_e, 4)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    c1 = composition_weights(4)[0]
    dt = 0.2 * S.cfl(iters=400, tol=1e-8)
    h, b = S.init_stagger(e0, np.zeros(S.n_h), c1 * dt, np.zeros(S.n_h))
    e, h, d, b2 = S.step_split(e0, h, dt, 20, 4, d=d0, b=b)
    r = S.kron_apply("K1", e) - S.mass_apply("D", d)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(S.mass_apply("D", d))
    assert np.abs(S.div(b2, True) - S.div(b, True)).max() < 1e-13
