"""Pins of the oracle's map-dependent parts against the mathematics of the
pullbacks (Section 2.3) rather than against another formula of the oracle.

A 2-form (vector proxy u) pulls back contravariantly, u o F = DF u^ / det DF,
a 1-form covariantly, E o F = DF^{-T} E^.  Whatever the map, the physical L^2
norms then follow from change of variables, int_Omega |u|^2 dx =
int |u o F|^2 det DF dx^; the oracle's metric factors and mass applies must
reproduce these numbers from the parametric side.  The maps used have
non-symmetric, non-diagonal Jacobians (the sine-deformed cube: DF = I + a 1 grad s^T;
the quarter coax), so a transposed Jacobian anywhere changes the result.
"""
import numpy as np
import pytest

import workloads as W
from oracle.geometry import Map, metric_1form, metric_2form
from oracle.scheme import Scheme
from oracle.scheme1 import Scheme1
from oracle.spaces import comp_tags, split

MAPS = [("sine", W.DEFORMED_AMPLITUDE, 1.0), ("annulus", 0.0, np.pi / 4)]


def _weights(S):
    return S.wq[:, None, None] * S.wq[None, :, None] * S.wq[None, None, :]


def test_sine_map_jacobian_is_the_derivative():
    """DF of x -> x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1) equals central
    differences of F; the map fixes the faces of the cube; det DF = 1 + a 1.grad s
    (a rank-one update of I), whose extremes over the cube are 1 -+ 2 a pi / sqrt 3
    (at x = y = z with cos^2(pi x) = 1/3), so the map is valid for a = 0.08."""
    a = W.DEFORMED_AMPLITUDE
    m = Map("sine", a)
    x = np.random.default_rng([0, 7]).uniform(size=(300, 3))
    J = m.DF(x)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (m.F(x + e) - m.F(x - e)) / (2 * h)
        assert np.abs(fd - J[:, :, j]).max() < 1e-8
    # closed form of the determinant of a rank-one update of the identity
    s_grad = np.pi * np.stack([np.cos(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2]),
                               np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2]),
                               np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])], 1)
    assert np.abs(np.linalg.det(J) - (1 + a * s_grad.sum(1))).max() < 1e-14
    assert np.abs(J - np.swapaxes(J, 1, 2)).max() > 1e-2  # DF is not symmetric
    # faces are fixed: F(x) = x wherever one coordinate is 0 or 1
    f = x.copy()
    f[:, 1] = 1.0
    assert np.abs(m.F(f) - f).max() < 1e-16
    # extremes of det DF over the cube: sampled finely, within the closed form
    bound = 2 * a * np.pi / np.sqrt(3)
    g = np.linspace(0, 1, 61)
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    det = np.linalg.det(m.DF(P))
    assert 1 - bound - 1e-14 <= det.min() < 1 - bound + 1e-3
    assert 1 + bound - 1e-3 < det.max() <= 1 + bound + 1e-14
    t = np.arccos(1 / np.sqrt(3)) / np.pi
    assert abs(np.linalg.det(m.DF(np.array([[t, t, t]])))[0] - (1 + bound)) < 1e-14


@pytest.mark.parametrize("kind,a,vol", MAPS)
def test_constant_2form_pullback_norm(kind, a, vol):
    """For constant physical 2-forms u, v: u^ = det DF DF^{-1} u, and
    sum_q w_q u^.G2 v^ = (u.v) sum_q w_q det DF = (u.v) |Omega| (up to the
    quadrature of the volume)."""
    S = Scheme(3, 3, Map(kind, a))
    xq = S.quad_points()
    DF = S.geo.DF(xq)
    det = np.linalg.det(DF)
    Wq = _weights(S)
    G2 = metric_2form(DF)
    rng = np.random.default_rng([0, 8])
    u, v = rng.standard_normal(3), rng.standard_normal(3)
    uh = det[..., None] * np.linalg.solve(DF, np.broadcast_to(u, DF.shape[:-1])[..., None])[..., 0]
    vh = det[..., None] * np.linalg.solve(DF, np.broadcast_to(v, DF.shape[:-1])[..., None])[..., 0]
    vol_q = np.sum(Wq * det)
    got = np.sum(Wq * np.einsum("...i,...ij,...j->...", uh, G2, vh))
    assert abs(got - (u @ v) * vol_q) < 1e-13 * abs(u @ v) * vol_q + 1e-14
    assert abs(vol_q - vol) < 1e-9


@pytest.mark.parametrize("kind,a,vol", MAPS)
def test_constant_1form_pullback_norm(kind, a, vol):
    """For constant physical 1-forms E, F: E^ = DF^T E, and
    sum_q w_q E^.G1 F^ = (E.F) sum_q w_q det DF."""
    S = Scheme(3, 3, Map(kind, a))
    xq = S.quad_points()
    DF = S.geo.DF(xq)
    det = np.linalg.det(DF)
    Wq = _weights(S)
    G1 = metric_1form(DF)
    rng = np.random.default_rng([0, 9])
    E, F = rng.standard_normal(3), rng.standard_normal(3)
    Eh = np.einsum("...ki,k->...i", DF, E)
    Fh = np.einsum("...ki,k->...i", DF, F)
    vol_q = np.sum(Wq * det)
    got = np.sum(Wq * np.einsum("...i,...ij,...j->...", Eh, G1, Fh))
    assert abs(got - (E @ F) * vol_q) < 1e-13 * abs(E @ F) * vol_q + 1e-14
    assert abs(vol_q - vol) < 1e-9


def _push_2form(S, space, x):
    """Physical vector proxy of a discrete 2-form at the Gauss points,
    u = DF u^ / det DF (contravariant Piola)."""
    V = np.stack(S.interpolate(space, x), axis=-1)
    DF = S.geo.DF(S.quad_points())
    return np.einsum("...ij,...j->...i", DF, V) / np.linalg.det(DF)[..., None]


def _push_1form(S, space, x):
    """Physical vector proxy of a discrete 1-form at the Gauss points,
    E = DF^{-T} E^ (covariant)."""
    V = np.stack(S.interpolate(space, x), axis=-1)
    DF = S.geo.DF(S.quad_points())
    return np.linalg.solve(np.swapaxes(DF, -1, -2), V[..., None])[..., 0]


@pytest.mark.parametrize("kind,a,vol", MAPS)
@pytest.mark.parametrize("space", ["B", "D"])
def test_2form_mass_is_physical_inner_product(kind, a, vol, space):
    """x.M y = int_Omega (1/g) u_x . u_y dx with u the pushed-forward fields and
    g = mu or eps per element, evaluated by change of variables at the same
    Gauss points (the physical integrand is formed explicitly)."""
    eps = W.eps_elements(3, 0)
    S = Scheme(2, 3, Map(kind, a), eps=eps)
    n = S.n_h if space == "B" else S.n_e
    x, y = W.random_vector(n, 1, 60), W.random_vector(n, 1, 61)
    ux, uy = _push_2form(S, space, x), _push_2form(S, space, y)
    det = np.linalg.det(S.geo.DF(S.quad_points()))
    inv_g = 1.0 if space == "B" else S._elem_to_q(1.0 / S.eps)
    phys = np.sum(_weights(S) * det * inv_g * np.sum(ux * uy, -1))
    assert abs(x @ S.mass_apply(space, y) - phys) < 1e-12 * np.sqrt(abs(
        (x @ S.mass_apply(space, x)) * (y @ S.mass_apply(space, y))))


@pytest.mark.parametrize("kind,a,vol", MAPS)
@pytest.mark.parametrize("space", ["E", "H"])
def test_1form_mass_is_physical_inner_product(kind, a, vol, space):
    """Scheme 1: x.M1 y = int_Omega g E_x . E_y dx (g = eps for E, mu for H)
    with E the covariantly pushed-forward 1-forms."""
    eps = W.eps_elements(3, 0)
    S = Scheme1(2, 3, Map(kind, a), eps=eps)
    n = S.n_e if space == "E" else S.n_h
    x, y = W.random_vector(n, 1, 62), W.random_vector(n, 1, 63)
    Ex, Ey = _push_1form(S, space, x), _push_1form(S, space, y)
    det = np.linalg.det(S.geo.DF(S.quad_points()))
    g = S._elem_to_q(S.eps) if space == "E" else 1.0
    phys = np.sum(_weights(S) * det * g * np.sum(Ex * Ey, -1))
    Mx, My = S.mass1_apply(space, x), S.mass1_apply(space, y)
    assert abs(x @ My - phys) < 1e-12 * np.sqrt(abs((x @ Mx) * (y @ My)))


@pytest.mark.parametrize("kind,a,vol", MAPS)
def test_projection_exact_on_discrete_fields_curved(kind, a, vol):
    """e^0 = K1^{-1} l with l_i = int eta^_i . DF^T E0(F) reproduces e when
    E0 is the covariant push-forward DF^{-T} E^_h of a discrete 1-form (the
    pairing of Section 2.4 is map-free, so only the pullback of E0 can be
    wrong)."""
    S = Scheme(3, 3, Map(kind, a))
    e = W.random_vector(S.n_e, 3, 64)
    Eq = _push_1form(S, "E", e)
    Fq = S.geo.F(S.quad_points())

    def field(xyz):
        assert xyz.shape == Fq.shape and np.abs(xyz - Fq).max() == 0.0
        return Eq

    assert np.linalg.norm(S.project_E(field) - e) < 1e-12 * np.linalg.norm(e)


def test_probe_is_covariant_push_forward():
    """probe_E(e, x^) = DF^{-T}(x^) E^_h(x^), E^_h summed from the basis by hand."""
    S = Scheme(2, 3, Map("sine", W.DEFORMED_AMPLITUDE))
    e = W.random_vector(S.n_e, 3, 65)
    pos = np.array([0.23, 0.61, 0.47])
    E = split(S.axis, "E", e)
    Eh = np.zeros(3)
    for c in range(3):
        bx, by, bz = [S.axis.eval(t, np.array([pos[k]]))[0] for k, t in enumerate(comp_tags("E", c))]
        Eh[c] = np.einsum("zyx,z,y,x->", E[c], bz, by, bx)
    DF = S.geo.DF(pos[None])[0]
    # E^ = DF^T E  <=>  E = DF^{-T} E^: check the defining relation, not the solve
    assert np.abs(DF.T @ S.probe_E(e, pos) - Eh).max() < 1e-13 * np.abs(Eh).max()
