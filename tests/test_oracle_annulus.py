"""Pins of the oracle on the curved workload: the quarter coaxial cable
1 < x^2 + y^2 < 2, 0 < z < 1 of Section 5 as a degree-2 NURBS map."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle.geometry import Map, metric_2form
from oracle.scheme import Scheme
from oracle.scheme1 import Scheme1


def test_map_is_the_quarter_annulus():
    """NURBS represent the circle exactly: radius = 1 + (sqrt 2 - 1) u for every
    v, the faces u = 0, 1 are the two cylinders, v = 0, 1 the planes y = 0 and
    x = 0; the Jacobian equals central differences and det DF > 0; the
    input generator's independent formula agrees."""
    m = Map("annulus")
    x = np.random.default_rng([0, 5]).uniform(size=(200, 3))
    F = m.F(x)
    r = np.hypot(F[:, 0], F[:, 1])
    assert np.abs(r - (1 + (np.sqrt(2) - 1) * x[:, 0])).max() < 1e-15
    assert np.abs(F[:, 2] - x[:, 2]).max() == 0.0
    v = np.linspace(0, 1, 7)
    ends = m.F(np.stack([np.zeros(7), v, np.zeros(7)], 1))
    assert np.abs(np.hypot(ends[:, 0], ends[:, 1]) - 1).max() < 1e-15
    assert abs(m.F(np.array([[0.3, 0.0, 0.5]]))[0, 1]) == 0.0
    assert abs(m.F(np.array([[0.3, 1.0, 0.5]]))[0, 0]) < 1e-16
    h = 1e-6
    J = m.DF(x)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (m.F(x + e) - m.F(x - e)) / (2 * h)
        assert np.abs(fd - J[:, :, j]).max() < 1e-8
    assert np.linalg.det(J).min() > 0
    Fw, Jw = W.quarter_annulus_jacobian(x)
    assert np.abs(Fw - F).max() < 1e-15 and np.abs(Jw - J).max() < 1e-14


def test_volume_by_quadrature():
    """sum_q w_q det DF = pi/4 (the quarter annulus of radii 1, sqrt 2, height 1)."""
    S = Scheme(3, 4, Map("annulus"))
    det = np.linalg.det(S.geo.DF(S.quad_points()))
    W3 = S.wq[:, None, None] * S.wq[None, :, None] * S.wq[None, None, :]
    assert abs(np.sum(W3 * det) - np.pi / 4) < 1e-9


@pytest.mark.parametrize("space", ["B", "D"])
def test_mass_on_annulus_equals_element_assembly(space):
    S = Scheme(2, 3, Map("annulus"), eps=W.eps_elements(3, 0))
    pts, _ = A.quad_points_3d(S.axis)
    G = metric_2form(S.geo.DF(pts))
    Mm = A.mass_2form(S.axis, space, G, None if space == "B" else 1.0 / S.eps)
    assert np.linalg.eigvalsh(Mm).min() > 0
    x = W.random_vector(Mm.shape[0], 6)
    assert np.linalg.norm(Mm @ x - S.mass_apply(space, x)) <= 1e-13 * np.linalg.norm(Mm @ x)


def test_leapfrog_invariants_on_annulus():
    """Both schemes keep their leapfrog invariants and the divergences on the
    curved map."""
    S = Scheme(3, 3, Map("annulus"), eps=W.eps_elements(3, 0))
    d0 = W.random_vector(S.n_e, 1)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    dt = 0.005
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    E0 = S.energy(e0, h, d0, b, dt)[0]
    e, h, d, b, en = S.step(e0, h, dt, nsteps=40, d=d0, b=b, energy_every=10)
    assert np.abs(np.array(en) / E0 - 1).max() < 1e-13
    assert np.abs(S.div(d, False) - S.div(d0, False)).max() < 1e-13 * np.abs(d).max()
    S1 = Scheme1(2, 3, Map("annulus"), eps=W.eps_elements(3, 0))
    e0 = W.random_vector(S1.n_e, 2)
    h, _ = S1.init_stagger1(e0, np.zeros(S1.n_h), dt)

    def inv(e, h):
        return S1.energy1_modified(e, h, h - dt * S1.mass1_solve("H", S1.rhs_h(e))[0])

    I0 = inv(e0, h)
    e, h, _, _ = S1.step1(e0, h, dt, 10)
    assert abs(inv(e, h) / I0 - 1) < 1e-12
