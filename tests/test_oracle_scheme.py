"""Pins of the oracle's leapfrog for scheme 2 (Sections 3.4, 4, 5)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import Map
from oracle.scheme import Scheme


def _deformed(p, N, eps=True):
    return Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=W.eps_elements(N, 0) if eps else None)


def _consistent_state(S, seed=0):
    """Random d^0, e^0 = K1^{-1} M~ d^0 (the Hodge (3.11)), h^0 = b^0 = 0."""
    d0 = W.random_vector(S.n_e, seed, 11)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    return d0, e0


@pytest.mark.parametrize("p,N", [(2, 3), (3, 3)])
def test_modified_energy_is_conserved(p, N):
    """With J = 0 the leapfrog conserves 1/2 (d^n.M~ d^n + b^{n-1/2}.M b^{n+1/2})
    to round-off, and the pairing form of it (built from (3.2)) agrees with
    the mass form.  The paper energy (3.2) oscillates (Section 5.1, Fig. 1)."""
    S = _deformed(p, N)
    d0, e0 = _consistent_state(S)
    dt = 0.5 * S.cfl(iters=400, tol=1e-8)
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, np.zeros(S.n_h))
    E0, P0 = S.energy(e0, h, d0, b, dt)
    assert abs(E0 - S.mass_energy(d0, b, b - dt * S.curl_primal(e0))) < 1e-13 * E0
    e, h, d, b, en = S.step(e0, h, dt, nsteps=150, d=d0, b=b, energy_every=5)
    en = np.array(en)
    assert np.abs(en / E0 - 1).max() < 1e-13
    paper = [S.energy(e, h, d, b, dt)[1]]
    assert abs(paper[0] / E0 - 1) > 1e-6  # the plain (3.2) energy is not exactly conserved
    # the tracked d stays consistent with the Hodge K1 e = M~ d
    r = S.kron_apply("K1", e) - S.mass_apply("D", d)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(S.mass_apply("D", d))


def test_divergence_of_b_is_constant():
    """Gauss law for B: D^2 b^{n+1/2} = D^2 b^{-1/2} exactly (D^2 D^1 = 0)."""
    S = _deformed(3, 3)
    d0, e0 = _consistent_state(S, 1)
    b0 = W.random_vector(S.n_h, 1, 12)
    dt = 0.01
    h, b = S.init_stagger(e0, np.zeros(S.n_h), dt, b0)
    div0 = S.div(b, True)
    _, _, d, b, _ = S.step(e0, h, dt, nsteps=40, d=d0, b=b)
    assert np.abs(S.div(b, True) - div0).max() < 1e-14 * max(1.0, np.abs(b).max())
    dd0 = S.div(d0, False)
    assert np.abs(S.div(d, False) - dd0).max() < 1e-13 * max(1.0, np.abs(d).max())


def test_discrete_eigenvector_closed_form():
    """Identity map, constant material: an eigenvector v of A (eigenvalue lambda)
    evolves as e^n = cos(n w dt) v with sin(w dt / 2) = dt sqrt(lambda) / 2."""
    S = Scheme(2, 4)
    Am = np.stack([S.apply_A(c) for c in np.eye(S.n_e)], 1)
    lam, V = np.linalg.eig(Am)
    lam = lam.real
    i = np.argsort(np.where(lam > 1e-6, lam, np.inf))[0]
    v = V[:, i].real
    v /= np.linalg.norm(v)
    dt = 0.5 * 2 / math.sqrt(lam.max())
    w = 2 / dt * math.asin(dt * math.sqrt(lam[i]) / 2)
    h, _ = S.init_stagger(v, np.zeros(S.n_h), dt)
    e = v
    for n in range(1, 61):
        e, h, _, _, _ = S.step(e, h, dt)
        assert np.linalg.norm(e - math.cos(n * w * dt) * v) < 1e-12


def test_time_reversibility():
    S = _deformed(2, 3)
    _, e0 = _consistent_state(S, 2)
    h0 = W.random_vector(S.n_h, 2, 13)
    dt = 0.02
    e, h, _, _, _ = S.step(e0, h0, dt, nsteps=25)
    h_fwd = h - dt * S.half_step_h(e)  # pair e^N with h^{N+1/2}
    e_back, _, _, _, _ = S.step(e, h_fwd, -dt, nsteps=25)
    assert np.linalg.norm(e_back - e0) < 1e-12 * np.linalg.norm(e0)


def test_superposition_in_sources():
    S = _deformed(2, 3)
    dip = W.dipoles(2, seed=0, dt=0.01)
    s = [S.dipole_source(dip["pos"][k], dip["moment"][k]) for k in range(2)]
    g = lambda t: math.exp(-(t - 0.1) ** 2 / (2 * 0.03 ** 2))
    z_e, z_h = np.zeros(S.n_e), np.zeros(S.n_h)
    run = lambda src: S.step(z_e, z_h, 0.01, nsteps=30, source=src)[0]
    e1 = run(lambda t: g(t) * s[0])
    e2 = run(lambda t: g(t) * s[1])
    e12 = run(lambda t: g(t) * (s[0] + s[1]))
    assert np.linalg.norm(e12 - e1 - e2) < 1e-13 * np.linalg.norm(e12)
    assert np.linalg.norm(e1) > 0


def test_dipole_source_is_local_and_tested():
    """s_i = q . eta_i(x0) / eps(x0): nonzero only on the (p)(p-1)^2 dual
    2-form basis functions per component whose support contains x0, and
    s . d equals the pointwise flux q . D_h(x0) / eps(x0) of D_h = sum d_i eta_i."""
    S = _deformed(3, 4)
    pos, q = np.array([0.31, 0.52, 0.77]), np.array([0.3, -0.5, 0.8])
    s = S.dipole_source(pos, q)
    assert np.count_nonzero(s) <= 3 * 3 * 2 * 2
    d = W.random_vector(S.n_e, 5, 14)
    from oracle.spaces import split, comp_tags
    Dh = np.zeros(3)
    Dd = split(S.axis, "D", d)
    for c in range(3):
        bx, by, bz = [S.axis.eval(t, np.array([pos[a]]))[0] for a, t in enumerate(comp_tags("D", c))]
        Dh[c] = np.einsum("zyx,z,y,x->", Dd[c], bz, by, bx)
    DF = S.geo.DF(pos[None])[0]
    Dphys = DF @ Dh / np.linalg.det(DF)
    el = (pos * 4).astype(int)
    assert abs(s @ d - q @ Dphys / S.eps[el[2], el[1], el[0]]) < 1e-12 * abs(s @ d)


def test_projection_is_exact_on_discrete_fields():
    """Identity map: projecting a field that is already in X^1_{h,0} returns it."""
    S = Scheme(3, 3)
    e = W.random_vector(S.n_e, 3, 15)

    def field(xyz):
        from oracle.spaces import split, comp_tags
        E = split(S.axis, "E", e)
        out = np.zeros(xyz.shape)
        pts = xyz.reshape(-1, 3)
        for c in range(3):
            bx, by, bz = [S.axis.eval(t, pts[:, a]) for a, t in enumerate(comp_tags("E", c))]
            out.reshape(-1, 3)[:, c] = np.einsum("zyx,qz,qy,qx->q", E[c], bz, by, bx)
        return out

    assert np.linalg.norm(S.project_E(field) - e) < 1e-12 * np.linalg.norm(e)


def test_probe_matches_interpolation():
    S = _deformed(2, 3)
    e = W.random_vector(S.n_e, 4, 16)
    Fq = S.field_at_quad("E", e)
    xq = S.quad_points()
    i = (3, 5, 7)
    assert np.abs(S.probe_E(e, xq[i]) - Fq[i]).max() < 1e-13


def _cavity_errors(p, N, T, dt):
    S = Scheme(p, N)
    modes = W.mode_110()
    omega = W.mode_omega(modes)[0]
    e = S.project_E(lambda xyz: W.eval_modes(modes, xyz))
    h, _ = S.init_stagger(e, np.zeros(S.n_h), dt)
    xq = S.quad_points()
    E0 = W.eval_modes(modes, xq)
    C0 = W.curl_modes(modes, xq)
    nsteps = int(round(T / dt))
    errE = nrmE = errH = nrmH = 0.0
    for n in range(1, nsteps + 1):
        e, h, _, _, _ = S.step(e, h, dt)
        tE, tH = n * dt, (n - 0.5) * dt
        Eex = E0 * math.cos(omega * tE)
        Hex = -C0 * math.sin(omega * tH) / omega
        Ed = S.field_at_quad("E", e)
        Hd = S.field_at_quad("H", h)
        errE += S.l2_norm_sq_quad(Ed - Eex)
        nrmE += S.l2_norm_sq_quad(Eex)
        errH += S.l2_norm_sq_quad(Hd - Hex)  # after step n the state holds h^{n-1/2}
        nrmH += S.l2_norm_sq_quad(Hex)
    return math.sqrt(errE / nrmE), math.sqrt(errH / nrmH)


@pytest.mark.parametrize("p", [2, 3])
def test_cavity_convergence_orders(p):
    """Relative L^2(0,T;L^2) errors decay as h^p for E and h^(p-1) for H
    (Section 5.1, Fig. 2), cube cavity, first mode."""
    T, dt = 0.5, 2.5e-3
    Ns = (2, 4) if p == 3 else (4, 8)
    errs = [_cavity_errors(p, N, T, dt) for N in Ns]
    rE = math.log2(errs[0][0] / errs[1][0])
    rH = math.log2(errs[0][1] / errs[1][1])
    assert rE > p - 0.3, errs
    assert rH > p - 1 - 0.3, errs
