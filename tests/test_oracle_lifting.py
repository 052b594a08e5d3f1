"""Pins of the oracle's non-homogeneous boundary data (Section 3.5) and of the
coaxial cable's TEM mode (Section 5.1.2)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle.geometry import Map, metric_2form
from oracle.lifting import LiftedScheme
from oracle.spaces import comp_tags, split


def _scheme(p, N, kind="sine"):
    geo = Map("sine", W.DEFORMED_AMPLITUDE) if kind == "sine" else Map(kind)
    return LiftedScheme(p, N, geo, eps=W.eps_elements(N, 0))


def test_full_primal_basis_and_its_derivative():
    """Pf is the whole B-spline basis of S_p(Xi): a partition of unity whose
    derivative is Pd d_full (central differences), and whose interior
    columns are Pv with d_full restricted to them equal to d."""
    from oracle.splines import Axis
    for p in (2, 3, 4):
        ax = Axis(5, p)
        x = np.random.default_rng([0, 30]).uniform(0.001, 0.999, 40)
        Pf = ax.eval("Pf", x)
        assert np.abs(Pf.sum(1) - 1).max() < 1e-14
        assert np.array_equal(Pf[:, 1:-1], ax.eval("Pv", x))
        h = 1e-6
        fd = (ax.eval("Pf", x + h) - ax.eval("Pf", x - h)) / (2 * h)
        assert np.abs(fd - ax.eval("Pd", x) @ ax.d_full()).max() < 1e-7
        assert np.array_equal(ax.d_full()[:, 1:-1], ax.d_primal())


def test_embedding_and_boundary_mask():
    S = _scheme(3, 3)
    e = W.random_vector(S.n_e, 2, 40)
    f = S.embed(e)
    assert np.array_equal(S.interior(f), e)
    mask = S.boundary_mask()
    assert np.count_nonzero(~mask) == S.n_e and np.all(f[mask] == 0)
    # the curl of an interior field lies in X^2_{h,0}: zero on the boundary
    # functions (Pf ends along the component's axis) and D^1 e inside
    U = split(S.axis, "Bf", S.curl_full(f))
    V = split(S.axis, "B", S.curl_primal(e))
    for c in range(3):
        k = 2 - c
        inner = [slice(None)] * 3
        inner[k] = slice(1, -1)
        ends = [slice(None)] * 3
        ends[k] = [0, -1]
        assert np.array_equal(U[c][tuple(inner)], V[c])
        assert np.all(U[c][tuple(ends)] == 0)


@pytest.mark.parametrize("p", [2, 3])
def test_full_operators_equal_level0(p):
    """The whole-space curl, the pairing with the boundary columns and the mass
    with whole-space trial functions equal their level-0 assembly (3D
    quadrature, explicit +-1 matrix, element loop); D^2 D^1 = 0 on X^1_h."""
    N = 2
    S = _scheme(p, N)
    ef = W.random_vector(S.n_full("Ef"), 3, 41)
    bf = W.random_vector(S.n_full("Bf"), 3, 42)
    D = A.curl_matrix_full(S.axis)
    assert np.abs(D @ ef - S.curl_full(ef)).max() < 1e-14 * np.abs(ef).max() * 4
    K = A.pairing_K1_full(S.axis)
    assert np.linalg.norm(K @ ef - S.K1_apply_full(ef)) < 1e-13 * np.linalg.norm(K @ ef)
    pts, _ = A.quad_points_3d(S.axis)
    G = metric_2form(S.geo.DF(pts))
    M = A.mass_2form_trial_full(S.axis, G)
    assert np.linalg.norm(M @ bf - S.mass_apply_trial_full(bf)) < 1e-13 * np.linalg.norm(M @ bf)
    # interior columns: the homogeneous operators
    e0 = W.random_vector(S.n_e, 3, 43)
    assert np.linalg.norm(S.K1_apply_full(S.embed(e0)) - S.kron_apply("K1", e0)) < 1e-13 * np.linalg.norm(e0)
    # divergence of the whole-space curl vanishes: sum_a d_f along a of component a
    U = split(S.axis, "Bf", S.curl_full(ef))
    div = sum(np.diff(U[a], axis=2 - a) for a in range(3))
    assert np.abs(div).max() < 1e-12 * np.abs(ef).max()


@pytest.mark.parametrize("kind", ["sine", "annulus"])
def test_lift_is_exact_on_discrete_traces(kind):
    """The trace fit returns the boundary coefficients of a field of X^1_h from
    its own pulled-back trace, whatever its interior coefficients."""
    S = _scheme(2, 3, kind)
    ef = W.random_vector(S.n_full("Ef"), 4, 44)

    def ehat(P):
        out = np.zeros(P.shape)
        flat = P.reshape(-1, 3)
        F = split(S.axis, "Ef", ef)
        for c in range(3):
            tags = comp_tags("Ef", c)
            B = [S.axis.eval(tags[k], flat[:, k]) for k in range(3)]
            out.reshape(-1, 3)[:, c] = np.einsum("zyx,qz,qy,qx->q", F[c], B[2], B[1], B[0])
        return out

    eb = S.lift_hat(ehat)
    mask = S.boundary_mask()
    assert np.abs(eb[mask] - ef[mask]).max() < 1e-11 * np.abs(ef).max()
    assert np.all(eb[~mask] == 0)


def test_lifted_step_keeps_the_full_space_hodge_relations():
    """With boundary data e_b g(t), the lifted (e, h) leapfrog is the scheme of
    Section 3.5 on the whole spaces: tracking d += dt D~^1 h and
    b_f -= dt D^1_f (e_0 + g e_b) keeps (K1)_f (e_0 + g(t_n) e_b) = M~ d^n and
    K~1 h^{n+1/2} = M_{0,f} b_f^{n+1/2} at every step."""
    p, N, dt, nsteps = 2, 3, 0.01, 12
    S = _scheme(p, N)
    rng = np.random.default_rng([0, 45])
    mask = S.boundary_mask()
    eb = np.where(mask, rng.standard_normal(S.n_full()), 0.0)
    g = lambda t: math.cos(3.0 * t + 0.4)  # noqa: E731
    v_h, v_e = S.lifting_vectors(eb)
    terms = [(v_h, v_e, g)]
    d = W.random_vector(S.n_e, 5, 46)
    e0 = S.kron_solve("K1", S.mass_apply("D", d)) - g(0.0) * v_e
    bf = W.random_vector(S.n_full("Bf"), 5, 47)
    bf = bf + 0.5 * dt * S.curl_full(S.embed(e0) + g(0.0) * eb)  # b_f^{-1/2}
    h = S.kron_solve("K1t", S.mass_apply_trial_full(bf))
    for n in range(nsteps):
        tn = n * dt
        assert np.linalg.norm(S.K1_apply_full(S.embed(e0) + g(tn) * eb) - S.mass_apply("D", d)) < \
            1e-12 * np.linalg.norm(S.mass_apply("D", d))
        bf = bf - dt * S.curl_full(S.embed(e0) + g(tn) * eb)
        e0, h = S.step_lifted(e0, h, dt, 1, terms, t0=tn)
        d = d + dt * S.curl_dual(h)
        lhs = S.kron_apply("K1t", h)
        assert np.linalg.norm(lhs - S.mass_apply_trial_full(bf)) < 1e-12 * np.linalg.norm(lhs)


def _tem_errors(p, N, T, dt):
    """Relative L^2(0,T;L^2) errors of E and H against the TEM mode on the
    quarter coax, Section 5.1.2 (E: full field e_0 + g e_b)."""
    S = LiftedScheme(p, N, Map("annulus"))
    eb = S.lift(lambda x: W.tem_coax_E(x, 0.0))
    g = lambda t: math.cos(math.pi * t)  # noqa: E731
    v_h, v_e = S.lifting_vectors(eb)
    terms = [(v_h, v_e, g)]
    e0, h = S.init_lifted(lambda x: W.tem_coax_E(x, 0.0), terms, dt)
    xq = S.geo.F(S.quad_points())
    nsteps = int(round(T / dt))
    errE = nrmE = errH = nrmH = 0.0
    for n in range(1, nsteps + 1):
        e0, h = S.step_lifted(e0, h, dt, 1, terms, t0=(n - 1) * dt)
        tE, tH = n * dt, (n - 0.5) * dt
        Ed = S.field_full_at_quad(S.embed(e0) + g(tE) * eb)
        Hd = S.field_at_quad("H", h)
        Eex, Hex = W.tem_coax_E(xq, tE), W.tem_coax_H(xq, tH)
        errE += S.l2_norm_sq_quad(Ed - Eex)
        nrmE += S.l2_norm_sq_quad(Eex)
        errH += S.l2_norm_sq_quad(Hd - Hex)
        nrmH += S.l2_norm_sq_quad(Hex)
    return math.sqrt(errE / nrmE), math.sqrt(errH / nrmH)


@pytest.mark.parametrize("p", [2, 3])
def test_tem_convergence_on_the_coax(p):
    """Section 5.1.2, Fig. 3: on the quarter coax with the TEM data on the
    planes y = 0 and x = 0, E converges as h^p and H as h^(p-1)."""
    T, dt = 0.5, 2.5e-3
    Ns = (2, 4) if p == 3 else (3, 6)
    errs = [_tem_errors(p, N, T, dt) for N in Ns]
    r = math.log(Ns[1] / Ns[0])
    rE = math.log(errs[0][0] / errs[1][0]) / r
    rH = math.log(errs[0][1] / errs[1][1]) / r
    assert rE > p - 0.3, errs
    assert rH > p - 1 - 0.3, errs
