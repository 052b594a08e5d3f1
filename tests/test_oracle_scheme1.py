"""Pins of the oracle's scheme 1 (Section 3.3: mass-matrix Hodge stars)."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assembly as A
from oracle.geometry import Map, metric_1form, metric_2form
from oracle.scheme import Scheme
from oracle.scheme1 import Scheme1
from oracle.spaces import comp_tags, split


def _dense_A1(S):
    """A1 as a dense matrix from dense mass matrices (columns of the mass
    applies) and dense solves: no CG inside."""
    M = np.stack([S.mass1_apply("E", c) for c in np.eye(S.n_e)], 1)
    Mt = np.stack([S.mass1_apply("H", c) for c in np.eye(S.n_h)], 1)
    Ch = np.stack([S.rhs_h(c) for c in np.eye(S.n_e)], 1)
    return np.linalg.solve(M, Ch.T @ np.linalg.solve(Mt, Ch)), M, Mt, Ch


def _deformed(p, N):
    return Scheme1(p, N, Map("sine", W.DEFORMED_AMPLITUDE),
                   eps=W.eps_elements(N, 0), mu=W.eps_elements(N, 1, 1.0, 2.0))


def test_metric_1form_closed_forms():
    """G1 inverts the 2-form factor (the two pullbacks are dual), and for a
    diagonal DF = diag(a, b, c) it is diag(bc/a, ac/b, ab/c)."""
    S = _deformed(3, 2)
    DF = S.geo.DF(S.quad_points())
    G1, G2 = metric_1form(DF), metric_2form(DF)
    I = np.broadcast_to(np.eye(3), G1.shape)
    assert np.abs(np.einsum("...ij,...jk->...ik", G1, G2) - I).max() < 1e-14
    a, b, c = 0.5, 2.0, 3.0
    G = metric_1form(np.diag([a, b, c])[None])[0]
    assert np.abs(G - np.diag([b * c / a, a * c / b, a * b / c])).max() < 1e-14


@pytest.mark.parametrize("p,N", [(2, 3), (3, 2), (3, 3)])
@pytest.mark.parametrize("space", ["E", "H"])
def test_mass1_apply_equals_element_assembly(p, N, space):
    """The sum-factorised 1-form mass equals the element-loop assembly, which is
    symmetric positive definite."""
    S = _deformed(p, N)
    pts, _ = A.quad_points_3d(S.axis)
    G1 = metric_1form(S.geo.DF(pts))
    g = S.eps if space == "E" else S.mu
    Mm = A.mass_1form(S.axis, space, G1, g)
    assert np.abs(Mm - Mm.T).max() < 1e-15 * np.abs(Mm).max() * 10
    assert np.linalg.eigvalsh(Mm).min() > 0
    x = W.random_vector(Mm.shape[0], 6)
    assert np.linalg.norm(Mm @ x - S.mass1_apply(space, x)) <= 1e-13 * np.linalg.norm(Mm @ x)
    # the CG solve reaches the dense solution
    y = W.random_vector(Mm.shape[0], 7)
    xs, it = S.mass1_solve(space, y)
    xd = np.linalg.solve(Mm, y)
    assert np.linalg.norm(xs - xd) <= 1e-12 * np.linalg.cond(Mm) * np.linalg.norm(xd)
    assert it > 0


@pytest.mark.parametrize("p", [2, 3])
def test_identity_mass1_is_kronecker_of_1d_grams(p):
    """Identity map, gamma = 1: each block of M^1 and M~^1 is the Kronecker
    product of the 1D Gram matrices of its component bases."""
    S = Scheme1(p, 3)
    for space in ("E", "H"):
        x = W.random_vector(S.n_e if space == "E" else S.n_h, 7)
        y = S.mass1_apply(space, x)
        X, Y = split(S.axis, space, x), split(S.axis, space, y)
        for c in range(3):
            tx, ty, tz = comp_tags(space, c)
            ref = np.einsum("az,by,cx,zyx->abc", S.axis.gram(tz), S.axis.gram(ty), S.axis.gram(tx), X[c])
            assert np.abs(ref - Y[c]).max() < 1e-14 * np.abs(ref).max() * 10


@pytest.mark.parametrize("p,N", [(2, 3), (3, 3)])
def test_rhs_operators_are_adjoint(p, N):
    """K1^T D~^1 and K~1^T D^1 are transposes of each other (eq. (2.10) with the
    pairing-transpose property), checked on the explicit level-0 matrices."""
    S = Scheme1(p, N)
    K1, K1t = A.pairing_K1(S.axis), A.pairing_K1t(S.axis)
    D1, Dt1 = A.curl_matrix(S.axis, True), A.curl_matrix(S.axis, False)
    Ce = K1.T @ Dt1   # e <- h
    Ch = K1t.T @ D1   # h <- e
    assert np.abs(Ce - Ch.T).max() < 1e-15
    e, h = W.random_vector(S.n_e, 1), W.random_vector(S.n_h, 2)
    assert np.abs(S.rhs_e(h) - Ce @ h).max() < 1e-14 * np.abs(Ce @ h).max()
    assert np.abs(S.rhs_h(e) - Ch @ e).max() < 1e-14 * np.abs(Ch @ e).max()


@pytest.mark.parametrize("p,N", [(2, 3), (3, 2)])
def test_leapfrog_invariant_and_hodge_tracking(p, N):
    """Without sources the leapfrog conserves (1/2)(e^n.M e^n + h^{n-1/2}.M~ h^{n+1/2})
    to round-off; it equals the scheme-2 invariant written with pairings,
    (1/2)(d.K1 e + b.K~1 h - dt (K~1 h).(D^1 e)), when d and b satisfy the
    Hodge relations (3.6), (3.8); and the tracked d, b keep satisfying them."""
    S = _deformed(p, N)
    e0 = W.random_vector(S.n_e, 3)
    _, M, Mt, Ch = _dense_A1(S)
    dt = 0.5 * 2 / np.sqrt(sla.eigh(Ch.T @ np.linalg.solve(Mt, Ch), M, eigvals_only=True).max())
    d0 = S.hodge_d(e0)
    h, b = S.init_stagger1(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    # b^{-1/2} is the Hodge partner of h^{-1/2} (both start from zero)
    assert np.linalg.norm(S.mass1_apply("H", h) - S.kron_apply("K1t", b, transpose=True)) \
        < 1e-12 * np.linalg.norm(S.mass1_apply("H", h))

    def invariant(e, h, d, b):
        h_hi, _ = S.mass1_solve("H", S.rhs_h(e))
        h_hi = h - dt * h_hi
        mass = S.energy1_modified(e, h, h_hi)
        pairing = S.energy(e, h, d, b, dt)[0]
        return mass, pairing

    E0, P0 = invariant(e0, h, d0, b)
    assert abs(P0 - E0) < 1e-12 * E0
    e, h2, d, b2 = S.step1(e0, h, dt, nsteps=40, d=d0, b=b)
    E1, P1 = invariant(e, h2, d, b2)
    assert abs(E1 / E0 - 1) < 1e-12 and abs(P1 / E0 - 1) < 1e-12
    assert abs(S.energy1(e, h2) / E0 - 1) > 1e-8  # the equal-time energy only oscillates
    r = S.mass1_apply("E", e) - S.kron_apply("K1", d, transpose=True)
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(S.mass1_apply("E", e))


def test_divergence_constraints():
    """Gauss laws (Section 3.3): the tracked D^2 b and D~^2 d are constant in
    time (D^2 D^1 = 0, D~^2 D~^1 = 0)."""
    S = _deformed(3, 2)
    e0 = W.random_vector(S.n_e, 4)
    d0, b0 = S.hodge_d(e0), W.random_vector(S.n_h, 5)
    h, b = S.init_stagger1(e0, np.zeros(S.n_h), 0.01, b0)
    _, _, d, b2 = S.step1(e0, h, 0.01, nsteps=20, d=d0, b=b)
    assert np.abs(S.div(b2, True) - S.div(b, True)).max() < 1e-13
    assert np.abs(S.div(d, False) - S.div(d0, False)).max() < 1e-13 * max(1.0, np.abs(d).max())


@pytest.mark.parametrize("p,N", [(2, 3), (3, 3)])
def test_e_operator_spectrum(p, N):
    """A1 = M^{-1} K1^T D~^1 M~^{-1} K~1^T D^1 has real non-negative spectrum
    with null space of dimension n0^3 (the discrete gradients)."""
    S = _deformed(p, N)
    Am = _dense_A1(S)[0]
    x = W.random_vector(S.n_e, 9)
    assert np.linalg.norm(S.apply_A1(x) - Am @ x) < 1e-11 * np.linalg.norm(Am @ x)
    lam = np.linalg.eigvals(Am)
    assert np.sum(np.abs(lam) < 1e-8) == (N + p - 2) ** 3
    assert np.abs(lam.imag).max() < 1e-8 and lam.real.min() > -1e-8


@pytest.mark.parametrize("p,expect", [(2, 2.0), (3, 4.0)])
def test_cavity_eigenvalue_converges(p, expect):
    """The smallest nonzero eigenvalue of A1 tends to 2 pi^2 (Section 5.1),
    triple, at rate about 2(p-1)."""
    errs = []
    for N in (3, 6):
        S = Scheme1(p, N)
        _, M, Mt, Ch = _dense_A1(S)
        lam = sla.eigh(Ch.T @ np.linalg.solve(Mt, Ch), M, eigvals_only=True)
        nz = lam[lam > 1e-6]
        assert np.abs(nz[:3] - nz[0]).max() < 1e-9 * nz[0]
        errs.append(abs(nz[0] - 2 * np.pi ** 2))
    assert np.log2(errs[0] / errs[1]) > expect - 0.3


def test_cfl_power_iteration():
    """cfl1 equals 2/sqrt(lambda_max) of the dense operator."""
    S = Scheme1(2, 3)
    _, M, Mt, Ch = _dense_A1(S)
    lmax = sla.eigh(Ch.T @ np.linalg.solve(Mt, Ch), M, eigvals_only=True).max()
    ref = 2 / np.sqrt(lmax)
    assert abs(S.cfl1(tol=1e-11, iters=3000) - ref) < 1e-5 * ref


def test_cfl_scheme1_exceeds_scheme2():
    """Section 5.2: the mass-solve scheme allows a larger time step, and its
    advantage grows with p (dt ~ p^{-3/2} against p^{-2}); dense eigenvalues."""
    ratios = []
    for p in (2, 3, 4):
        S1, S2 = Scheme1(p, 3), Scheme(p, 3)
        _, M, Mt, Ch = _dense_A1(S1)
        l1 = sla.eigh(Ch.T @ np.linalg.solve(Mt, Ch), M, eigvals_only=True).max()
        l2 = np.abs(np.linalg.eigvals(np.stack([S2.apply_A(c) for c in np.eye(S2.n_e)], 1))).max()
        ratios.append(np.sqrt(l2 / l1))
    assert ratios[0] > 1.0 and ratios[0] < ratios[1] < ratios[2]


def test_projection_is_exact_on_discrete_fields():
    """project_E1 reproduces a field that lies in X^1_{h,0} (deformed map)."""
    S = _deformed(2, 3)
    e = W.random_vector(S.n_e, 13)

    def field(X):
        # the physical field of e at the mapped Gauss points, in the order
        # project_E1 evaluates them
        return S.field_at_quad("E", e)

    assert np.linalg.norm(S.project_E1(field) - e) < 1e-11 * np.linalg.norm(e)


def _cavity_errors1(p, N, T, dt):
    import math
    S = Scheme1(p, N)
    modes = W.mode_110()
    omega = W.mode_omega(modes)[0]
    e = S.project_E1(lambda xyz: W.eval_modes(modes, xyz))
    h, _ = S.init_stagger1(e, np.zeros(S.n_h), dt, tol=1e-14)
    xq = S.quad_points()
    E0, C0 = W.eval_modes(modes, xq), W.curl_modes(modes, xq)
    errE = nrmE = errH = nrmH = 0.0
    for n in range(1, int(round(T / dt)) + 1):
        e, h, _, _ = S.step1(e, h, dt, tol=1e-14)
        Eex = E0 * math.cos(omega * n * dt)
        Hex = -C0 * math.sin(omega * (n - 0.5) * dt) / omega
        errE += S.l2_norm_sq_quad(S.field_at_quad("E", e) - Eex)
        nrmE += S.l2_norm_sq_quad(Eex)
        errH += S.l2_norm_sq_quad(S.field_at_quad("H", h) - Hex)
        nrmH += S.l2_norm_sq_quad(Hex)
    return math.sqrt(errE / nrmE), math.sqrt(errH / nrmH)


def test_cavity_convergence_orders_scheme1():
    """Section 5.1, Fig. 2: the first scheme converges at the same rates as the
    second, h^p for E and h^(p-1) for H in L^2(0,T;L^2) (p = 3, cube cavity,
    first mode)."""
    import math
    p, T, dt = 3, 0.5, 2.5e-3
    errs = [_cavity_errors1(p, N, T, dt) for N in (2, 4)]
    assert math.log2(errs[0][0] / errs[1][0]) > p - 0.3, errs
    assert math.log2(errs[0][1] / errs[1][1]) > p - 1 - 0.3, errs
