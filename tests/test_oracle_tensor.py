"""Pins of the oracle with a degree, a knot vector and an element count per
direction (Section 4.1, eq. (4.2)/(4.3) with p_i and Xi_i; Section 2.3 knot
vectors; Section 3.4 masses): non-uniform bases against their defining
properties, the structured operators against level-0 3D quadrature, the curls
against finite differences of the interpolated fields, the leapfrog against
the isotropic oracle and against a cyclic relabelling of the axes, and the
energy invariant."""
import numpy as np
import pytest

import workloads as W
from oracle.geometry import Map
from oracle.scheme import Scheme
from oracle.splines import Axis
from oracle.tensor import TensorScheme

P_SMALL = (3, 2, 4)
N_SMALL = (3, 4, 2)
RATIO = (1.4, 1.0, 0.7)


def _breaks(n, ratio):
    return tuple(W.graded_breaks(n[a], ratio[a]) for a in range(3))


def _small(geo=True, eps=True, p=P_SMALL, n=N_SMALL, ratio=RATIO):
    return TensorScheme(p, n, _breaks(n, ratio),
                        Map("sine", W.DEFORMED_AMPLITUDE) if geo else None,
                        eps=W.eps_elements_aniso(n, 3) if eps else None)


# ---------------------------------------------------------------------------
# non-uniform univariate bases (Section 2.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 3, 4])
def test_graded_axis_bases(p):
    ax = Axis(5, p, W.graded_breaks(5, 1.6))
    x = np.random.default_rng(0).uniform(0, 1, 200)
    # the whole S_p basis is a partition of unity
    assert np.abs(ax.eval("Pf", x).sum(axis=1) - 1).max() < 1e-14
    # Curry-Schoenberg functions integrate to one (Gauss rule exact for them)
    xg, wg = ax.gauss()
    assert np.abs(wg @ ax.eval("Pd", xg) - 1).max() < 1e-13
    assert np.abs(wg @ ax.eval("Dd", xg) - 1).max() < 1e-13
    # derivatives: Pv' = Pd d and Dv' = Dd d~ (central differences away from knots)
    nodes = ax.nodes()
    xs = np.array([0.5 * (nodes[k] + nodes[k + 1]) + 0.1 * (nodes[k + 1] - nodes[k]) for k in range(5)])
    hstep = 1e-6
    for tag, dtag, D in (("Pv", "Pd", ax.d_primal()), ("Dv", "Dd", ax.d_dual())):
        fd = (ax.eval(tag, xs + hstep) - ax.eval(tag, xs - hstep)) / (2 * hstep)
        assert np.abs(fd - ax.eval(dtag, xs) @ D).max() < 1e-6 * max(1.0, np.abs(fd).max())


def test_uniform_breaks_reproduce_the_uniform_axis():
    a, b = Axis(6, 3), Axis(6, 3, np.arange(1, 6) / 6)
    assert np.allclose(a.xi, b.xi, rtol=0, atol=1e-15)
    assert np.abs(a.G_hat() - b.G_hat()).max() < 1e-14
    assert np.abs(a.M_hat() - b.M_hat()).max() < 1e-14


def test_breaks_are_validated():
    with pytest.raises(ValueError):
        Axis(3, 2, [0.5])
    with pytest.raises(ValueError):
        Axis(3, 2, [0.6, 0.4])


# ---------------------------------------------------------------------------
# structured operators against level 0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["K1", "K1t"])
def test_kronecker_pairing_equals_3d_quadrature(which):
    """Eq. (4.2)/(4.3) with per-direction factors: the Kronecker apply equals
    the matrix of integrals of products of 3D basis functions."""
    S = _small(geo=False, eps=False)
    K = S.pairing_dense(which)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(K.shape[1])
    y = rng.standard_normal(K.shape[0])
    assert np.abs(S.kron_apply(which, x) - K @ x).max() < 1e-13 * np.abs(K @ x).max()
    assert np.abs(S.kron_apply(which, y, transpose=True) - K.T @ y).max() < 1e-13 * np.abs(K.T @ y).max()
    # eq. (4.4)/(4.5): the per-axis LU solves invert the block
    assert np.abs(S.kron_solve(which, K @ x) - x).max() < 1e-10 * np.abs(x).max()
    assert np.abs(S.kron_solve(which, K.T @ y, transpose=True) - y).max() < 1e-10 * np.abs(y).max()


@pytest.mark.parametrize("space", ["B", "D"])
def test_sum_factorised_mass_equals_pointwise_assembly(space):
    S = _small()
    if space == "B":
        S.mu = W.eps_elements_aniso(S.N, 9)
    M = S.mass_dense(space)
    x = np.random.default_rng(2).standard_normal(M.shape[0])
    assert np.abs(S.mass_apply(space, x) - M @ x).max() < 1e-13 * np.abs(M @ x).max()
    # symmetric positive definite
    assert np.abs(M - M.T).max() < 1e-14 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("primal", [True, False])
def test_curl_is_the_curl_of_the_interpolated_field(primal):
    """The 2-form D^1 e (D~^1 h) interpolated at a point equals the curl of the
    interpolated 1-form there, by central differences of the 3D basis."""
    S = _small(geo=False, eps=False)
    src, dst = ("E", "B") if primal else ("H", "D")
    u = np.random.default_rng(3).standard_normal(S.space_size(src))
    w = S.curl(u, primal)
    U = S.split(src, u)
    Wc = S.split(dst, w)
    rng = np.random.default_rng(4)
    pts = rng.uniform(0.05, 0.95, size=(12, 3))
    hstep = 1e-6

    def field(space, coeff, c, x):
        return S.basis_3d(space, c, x) @ coeff[c].ravel()

    for q in pts:
        for c in range(3):
            a1, a2 = (c + 1) % 3, (c + 2) % 3
            e1 = np.zeros(3); e1[a1] = hstep
            e2 = np.zeros(3); e2[a2] = hstep
            d1 = (field(src, U, a2, (q + e1)[None]) - field(src, U, a2, (q - e1)[None])) / (2 * hstep)
            d2 = (field(src, U, a1, (q + e2)[None]) - field(src, U, a1, (q - e2)[None])) / (2 * hstep)
            ref = (d1 - d2)[0]
            got = field(dst, Wc, c, q[None])[0]
            assert abs(got - ref) < 2e-6 * max(1.0, abs(ref))
    # and the divergence of a curl vanishes
    assert np.abs(S.div(w, primal)).max() < 1e-12 * np.abs(w).max()


# ---------------------------------------------------------------------------
# the leapfrog
# ---------------------------------------------------------------------------
def test_isotropic_case_reproduces_the_scheme():
    p, N = 3, 3
    eps = W.eps_elements(N, 0)
    geo = Map("sine", W.DEFORMED_AMPLITUDE)
    S = Scheme(p, N, geo, eps=eps)
    T = TensorScheme((p, p, p), (N, N, N), geo=geo, eps=eps)
    assert (T.n_e, T.n_h) == (S.n_e, S.n_h)
    e0 = W.random_vector(S.n_e, 0, 1)
    h0 = W.random_vector(S.n_h, 0, 2)
    e1, h1 = S.step(e0, h0, 0.01, nsteps=3)[:2]
    e2, h2 = T.step(e0, h0, 0.01, nsteps=3)[:2]
    assert np.abs(e1 - e2).max() < 1e-13 * np.abs(e1).max()
    assert np.abs(h1 - h2).max() < 1e-13 * np.abs(h1).max()


def _rotate_field(S, space, v):
    """Relabel the axes cyclically: direction a of the new mesh is direction
    (a + 1) % 3 of S.  Component c of the new field is component (c + 1) % 3
    of the old one, with its array axes moved accordingly (a cyclic
    relabelling keeps the orientation, so no signs change)."""
    parts = S.split(space, v)
    return np.concatenate([parts[(c + 1) % 3].transpose(2, 0, 1).ravel() for c in range(3)])


def test_cyclic_relabelling_of_the_axes_commutes_with_the_step():
    """The sine map is invariant under cyclic relabelling of the coordinates,
    so the scheme on the relabelled mesh (degrees, knots, element counts and
    permittivities moved with the axes) advances the relabelled fields."""
    pA, nA, rA = P_SMALL, N_SMALL, RATIO
    A = _small(p=pA, n=nA, ratio=rA)
    perm = lambda t: tuple(t[(a + 1) % 3] for a in range(3))
    B = TensorScheme(perm(pA), perm(nA), perm(_breaks(nA, rA)), Map("sine", W.DEFORMED_AMPLITUDE),
                     eps=A.eps.transpose(2, 0, 1))
    e0 = W.random_vector(A.n_e, 5, 1)
    h0 = W.random_vector(A.n_h, 5, 2)
    eA, hA = A.step(e0, h0, 0.01, nsteps=2)[:2]
    eB, hB = B.step(_rotate_field(A, "E", e0), _rotate_field(A, "H", h0), 0.01, nsteps=2)[:2]
    rE, rH = _rotate_field(A, "E", eA), _rotate_field(A, "H", hA)
    assert np.abs(eB - rE).max() < 1e-12 * np.abs(rE).max()
    assert np.abs(hB - rH).max() < 1e-12 * np.abs(rH).max()


def test_modified_energy_is_conserved_on_a_graded_anisotropic_mesh():
    S = _small()
    d0 = W.random_vector(S.n_e, 6, 1)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    dt = 0.5 * S.cfl(iters=300, tol=1e-8)
    b0 = np.zeros(S.n_h)
    h0 = np.zeros(S.n_h)
    E0 = S.energy(e0, h0, d0, b0, dt)[0]
    e, h, d, b, en = S.step(e0, h0, dt, nsteps=60, d=d0, b=b0, energy_every=6)
    assert np.abs(np.array(en) / E0 - 1).max() < 1e-12
    # the tracked d stays the Hodge image of e
    r = S.kron_apply("K1", e) - S.mass_apply("D", d)
    assert np.abs(r).max() < 1e-12 * np.abs(S.kron_apply("K1", e)).max()
