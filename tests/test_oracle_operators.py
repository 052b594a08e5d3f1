"""Pins of the oracle's 3D operators: pairing, incidence, mass (Sections 2.4, 3.4, 4)."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle.geometry import Map, metric_2form
from oracle.scheme import Scheme

CASES = [(2, 3), (3, 2), (3, 3), (4, 2)]


def _scheme(p, N, deformed=True, eps=True):
    geo = Map("sine", W.DEFORMED_AMPLITUDE) if deformed else Map("identity")
    return Scheme(p, N, geo, eps=W.eps_elements(N, 0) if eps else None)


@pytest.mark.parametrize("p,N", CASES)
def test_kronecker_structure_of_pairings(p, N):
    """3D-quadrature assembly of K1, K~1 equals the Kronecker blocks (4.2)/(4.3)."""
    S = _scheme(p, N)
    K1, K1t = A.pairing_K1(S.axis), A.pairing_K1t(S.axis)
    I_e, I_h = np.eye(S.n_e), np.eye(S.n_h)
    K1_kron = np.stack([S.kron_apply("K1", c) for c in I_e], 1)
    K1t_kron = np.stack([S.kron_apply("K1t", c) for c in I_h], 1)
    assert np.abs(K1 - K1_kron).max() < 1e-14 * np.abs(K1).max() * 10
    assert np.abs(K1t - K1t_kron).max() < 1e-14 * np.abs(K1t).max() * 10
    # block diagonal: no coupling between components
    o = S.n_e // 3
    assert np.abs(K1[:o, o:]).max() == 0.0


@pytest.mark.parametrize("p,N", CASES)
def test_kronecker_solve_equals_dense_lu(p, N):
    S = _scheme(p, N)
    K1, K1t = A.pairing_K1(S.axis), A.pairing_K1t(S.axis)
    y = W.random_vector(S.n_e, 1)
    z = W.random_vector(S.n_h, 2)
    # both solvers are backward stable: allow a few ulps times the condition number
    tol = 20 * np.finfo(float).eps * max(np.linalg.cond(K1), np.linalg.cond(K1t))
    for x_k, x_d in ((S.kron_solve("K1", y), np.linalg.solve(K1, y)),
                     (S.kron_solve("K1", y, transpose=True), np.linalg.solve(K1.T, y)),
                     (S.kron_solve("K1t", z), np.linalg.solve(K1t, z)),
                     (S.kron_solve("K1t", z, transpose=True), np.linalg.solve(K1t.T, z))):
        assert np.linalg.norm(x_k - x_d) <= tol * np.linalg.norm(x_d)


def test_kronecker_solve_residual_large():
    S = Scheme(4, 16)
    y = W.random_vector(S.n_e, 3)
    x = S.kron_solve("K1", y)
    assert np.linalg.norm(S.kron_apply("K1", x) - y) <= 1e-13 * np.linalg.norm(y)


@pytest.mark.parametrize("p,N", CASES)
def test_curls_integer_and_complex(p, N):
    """D^1, D~^1 are +-1 matrices, D^2 D^1 = 0, D~^2 D~^1 = 0 exactly, and the
    level-1 index-difference curls equal the explicit matrices."""
    S = _scheme(p, N, deformed=False, eps=False)
    for primal in (True, False):
        C = A.curl_matrix(S.axis, primal)
        Dv = A.div_matrix(S.axis, primal)
        assert set(np.unique(C)) <= {-1.0, 0.0, 1.0}
        assert np.count_nonzero(Dv @ C) == 0
        x = W.random_vector(C.shape[1], 4)
        assert np.abs(C @ x - S.curl(x, primal)).max() < 1e-14
        y = W.random_vector(Dv.shape[1], 5)
        assert np.abs(Dv @ y - S.div(y, primal)).max() < 1e-14


@pytest.mark.parametrize("p,N", CASES)
def test_discrete_integration_by_parts(p, N):
    """(2.9) and (2.10) with k = 2: (D^1)^T K~1 = K1^T D~^1 and (D~^1)^T K1 = K~1^T D^1."""
    S = _scheme(p, N, deformed=False, eps=False)
    K1, K1t = A.pairing_K1(S.axis), A.pairing_K1t(S.axis)
    D1, Dt1 = A.curl_matrix(S.axis, True), A.curl_matrix(S.axis, False)
    assert np.abs(D1.T @ K1t - K1.T @ Dt1).max() < 1e-15
    assert np.abs(Dt1.T @ K1 - K1t.T @ D1).max() < 1e-15


@pytest.mark.parametrize("p,N", CASES)
@pytest.mark.parametrize("space", ["B", "D"])
def test_mass_apply_equals_element_assembly(p, N, space):
    S = _scheme(p, N)
    pts, _ = A.quad_points_3d(S.axis)
    G = metric_2form(S.geo.DF(pts))
    inv = None if space == "B" else 1.0 / S.eps
    Mm = A.mass_2form(S.axis, space, G, inv)
    assert np.abs(Mm - Mm.T).max() < 1e-15 * np.abs(Mm).max() * 10
    assert np.linalg.eigvalsh(Mm).min() > 0
    x = W.random_vector(Mm.shape[0], 6)
    assert np.linalg.norm(Mm @ x - S.mass_apply(space, x)) <= 1e-13 * np.linalg.norm(Mm @ x)


@pytest.mark.parametrize("p", [2, 3])
def test_identity_mass_is_kronecker_of_1d_grams(p):
    """Identity map, gamma = 1: each block of M is the Kronecker product of the
    1D Gram matrices of its component bases."""
    S = Scheme(p, 3)
    from oracle.spaces import comp_tags, split
    for space in ("B", "D"):
        x = W.random_vector(S.n_h if space == "B" else S.n_e, 7)
        y = S.mass_apply(space, x)
        X, Y = split(S.axis, space, x), split(S.axis, space, y)
        for c in range(3):
            tx, ty, tz = comp_tags(space, c)
            ref = np.einsum("az,by,cx,zyx->abc", S.axis.gram(tz), S.axis.gram(ty), S.axis.gram(tx), X[c])
            assert np.abs(ref - Y[c]).max() < 1e-14 * np.abs(ref).max() * 10


def test_mass_symmetry_large():
    S = _scheme(3, 6)
    x, y = W.random_vector(S.n_e, 8), W.random_vector(S.n_e, 9)
    a, b = x @ S.mass_apply("D", y), y @ S.mass_apply("D", x)
    assert abs(a - b) <= 1e-13 * abs(a)


@pytest.mark.parametrize("p,N", [(2, 3), (3, 2)])
def test_curl_curl_kernel_is_gradients(p, N):
    """The null space of the e-e leapfrog operator has dimension n0^3 = dim X^0_{h,0}."""
    S = Scheme(p, N)
    Am = np.stack([S.apply_A(c) for c in np.eye(S.n_e)], 1)
    lam = np.linalg.eigvals(Am)
    assert np.sum(np.abs(lam) < 1e-8) == (N + p - 2) ** 3
    assert np.abs(lam.imag).max() < 1e-8 and lam.real.min() > -1e-8


@pytest.mark.parametrize("p,Ns", [(2, (3, 6)), (3, (3, 6))])
def test_cavity_eigenvalue_converges_to_2pi2(p, Ns):
    """The smallest nonzero eigenvalue tends to 2 pi^2 (the cube's first
    curl-curl eigenvalue, omega = sqrt(2) pi, Section 5.1), triple, at the rate
    2(p-1) or faster."""
    errs = []
    for N in Ns:
        S = Scheme(p, N)
        Am = np.stack([S.apply_A(c) for c in np.eye(S.n_e)], 1)
        lam = np.sort(np.linalg.eigvals(Am).real)
        nz = lam[lam > 1e-6]
        assert np.abs(nz[:3] - nz[0]).max() < 1e-9 * nz[0]
        errs.append(nz[0] - 2 * np.pi ** 2)
    assert all(e > 0 for e in errs)
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2 * (p - 1) - 0.3


def test_cfl_power_iteration_and_scaling():
    """Power-iteration CFL equals 2/sqrt(lambda_max) of the dense operator, and
    scales linearly with h at fixed p."""
    S = Scheme(2, 3)
    Am = np.stack([S.apply_A(c) for c in np.eye(S.n_e)], 1)
    lmax = np.abs(np.linalg.eigvals(Am)).max()
    assert abs(S.cfl(tol=1e-11, iters=3000) - 2 / np.sqrt(lmax)) < 1e-5 * 2 / np.sqrt(lmax)
    c4, c8 = Scheme(2, 4).cfl(tol=1e-10, iters=3000), Scheme(2, 8).cfl(tol=1e-10, iters=3000)
    assert abs(c4 / c8 - 2.0) < 0.01
