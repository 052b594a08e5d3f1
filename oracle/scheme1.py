"""Scheme 1 of the oracle: mass-matrix Hodge stars (FP64, plain NumPy).

Test infrastructure only (see ``oracle/__init__``).

What is computed (paper, Section 3.3, eqs. (3.5)-(3.8) and the weak form of
Section 3.3.2): the Hodge stars are imposed with the 1-form mass matrices,

    M^1_eps e = K~2 d,        M~^1_mu h = K2 b,

and by the pairing-transpose property of Section 2.4 (K~2 = K1^T, K2 = K~1^T)
the (e, h) form is

    M^1_eps d_t e  =  K1^T D~^1 h,        M~^1_mu d_t h  = - K~1^T D^1 e,

advanced by the same staggered leapfrog as scheme 2,

    h^{n+1/2} = h^{n-1/2} - dt (M~^1_mu)^{-1} K~1^T D^1 e^n
    e^{n+1}   = e^n + dt (M^1_eps)^{-1} K1^T D~^1 h^{n+1/2},

optionally tracking b and d as in scheme 2 (source-free runs only).

* Mass matrices of 1-forms: entries int eta^_i . G1 eta^_j gamma with the
  covariant-pullback factor G1 = det DF (DF^T DF)^{-1}; gamma = eps for the
  primal space X^1_{h,0}, gamma = mu for the dual space X~^1.  Applied
  sum-factorised like the 2-form masses.
* Mass solves: plain conjugate gradients on the SPD mass apply, run to the
  rounding level (relative residual 1e-15 by default).  The paper solves these
  systems with a direct solver; both give M^{-1} y up to rounding times the
  condition number.
* Energy: the paper's (1/2)(e.M e + h.M~ h) at equal times, and the leapfrog
  invariant (1/2)(e^n.M e^n + h^{n-1/2}.M~ h^{n+1/2}), conserved exactly by the
  scheme without sources.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import metric_1form
from .scheme import Scheme


class Scheme1(Scheme):
    """Scheme 1 on the unit cube mapped by `geo`, degree p, N elements per axis."""

    def __init__(self, *args, **kwargs):
        super().__init__(*args, **kwargs)
        self._metric1 = None

    def metric1(self) -> np.ndarray:
        """w_q * det DF (DF^T DF)^{-1} at the Gauss points, (3, 3, Q, Q, Q)."""
        if self._metric1 is None:
            G = metric_1form(self.geo.DF(self.quad_points()))
            W = self.wq[:, None, None] * self.wq[None, :, None] * self.wq[None, None, :]
            self._metric1 = np.moveaxis(G * W[..., None, None], (-2, -1), (0, 1)).copy()
        return self._metric1

    # ------------------------------------------------------------------
    # 1-form mass matrices and their solves
    # ------------------------------------------------------------------
    def mass1_apply(self, space: str, x: np.ndarray) -> np.ndarray:
        """M^1_eps x (space 'E') or M~^1_mu x (space 'H')."""
        if space not in ("E", "H"):
            raise ValueError(space)
        G = self.metric1()
        g = self.eps if space == "E" else self.mu
        V = self.interpolate(space, x)
        gq = None if g is None else self._elem_to_q(g)
        U = []
        for i in range(3):
            acc = G[i, 0] * V[0] + G[i, 1] * V[1] + G[i, 2] * V[2]
            U.append(acc if gq is None else acc * gq)
        return self.integrate(space, U)

    def mass1_solve(self, space: str, y: np.ndarray, x0: np.ndarray | None = None,
                    tol: float = 1e-15, maxiter: int = 5000):
        """x = M^{-1} y by conjugate gradients; returns (x, iterations)."""
        x = np.zeros_like(y) if x0 is None else np.array(x0, dtype=float, copy=True)
        r = y - self.mass1_apply(space, x) if x0 is not None else y.copy()
        pdir = r.copy()
        rr = r @ r
        stop = (tol * np.linalg.norm(y)) ** 2
        it = 0
        while rr > stop and it < maxiter:
            Ap = self.mass1_apply(space, pdir)
            alpha = rr / (pdir @ Ap)
            x += alpha * pdir
            r -= alpha * Ap
            rr_new = r @ r
            pdir = r + (rr_new / rr) * pdir
            rr = rr_new
            it += 1
        return x, it

    # ------------------------------------------------------------------
    # right-hand sides of the (e, h) form
    # ------------------------------------------------------------------
    def rhs_h(self, e: np.ndarray) -> np.ndarray:
        """K~1^T D^1 e = K2 D^1 e (dual 1-form space)."""
        return self.kron_apply("K1t", self.curl_primal(e), transpose=True)

    def rhs_e(self, h: np.ndarray) -> np.ndarray:
        """K1^T D~^1 h = K~2 D~^1 h (primal 1-form space)."""
        return self.kron_apply("K1", self.curl_dual(h), transpose=True)

    # ------------------------------------------------------------------
    # the leapfrog
    # ------------------------------------------------------------------
    def step1(self, e, h, dt, nsteps=1, d=None, b=None, tol=1e-15):
        """Advance (e^n, h^{n-1/2}) by nsteps; returns (e, h, d, b)."""
        e = np.array(e, dtype=float, copy=True)
        h = np.array(h, dtype=float, copy=True)
        track = d is not None
        if track:
            if b is None:
                raise ValueError("tracking needs both d and b")
            d = np.array(d, dtype=float, copy=True)
            b = np.array(b, dtype=float, copy=True)
        for _ in range(nsteps):
            u = self.curl_primal(e)
            dh, _ = self.mass1_solve("H", self.kron_apply("K1t", u, transpose=True), tol=tol)
            h -= dt * dh
            if track:
                b -= dt * u
            v = self.curl_dual(h)
            de, _ = self.mass1_solve("E", self.kron_apply("K1", v, transpose=True), tol=tol)
            e += dt * de
            if track:
                d += dt * v
        return e, h, d, b

    def init_stagger1(self, e0, h0, dt, b0=None, tol=1e-15):
        """Backward half kick from t = 0: h^{-1/2} = h^0 + dt/2 M~^{-1} K~1^T D^1 e^0
        (and b^{-1/2} = b^0 + dt/2 D^1 e^0)."""
        dh, _ = self.mass1_solve("H", self.rhs_h(e0), tol=tol)
        h = np.array(h0, dtype=float) + 0.5 * dt * dh
        b = None
        if b0 is not None:
            b = np.array(b0, dtype=float) + 0.5 * dt * self.curl_primal(e0)
        return h, b

    def hodge_d(self, e):
        """d with M^1_eps e = K1^T d, i.e. d = K1^{-T} M e (eq. (3.6))."""
        return self.kron_solve("K1", self.mass1_apply("E", e), transpose=True)

    def hodge_b(self, h):
        """b with M~^1_mu h = K~1^T b (eq. (3.8))."""
        return self.kron_solve("K1t", self.mass1_apply("H", h), transpose=True)

    def project_E1(self, efield, tol: float = 1e-15) -> np.ndarray:
        """e^0 = M^{-1} l, l_i = (E0, eta_i)_{L^2_eps} over the primal 1-form
        basis eta_i = DF^{-T} eta^_i: in parametric coordinates
        l_i = int eta^_i . (eps det DF DF^{-1} E0(F(x^))) dx^ (the L^2_eps
        projection of E0 onto X^1_{h,0}, the initial value of the Galerkin
        scheme of Section 3.3.2)."""
        xh = self.quad_points()
        E = efield(self.geo.F(xh))
        DF = self.geo.DF(xh)
        det = np.linalg.det(DF)
        Eh = det[..., None] * np.linalg.solve(DF, E[..., None])[..., 0]
        W = self.wq[:, None, None] * self.wq[None, :, None] * self.wq[None, None, :]
        g = 1.0 if self.eps is None else self._elem_to_q(self.eps)
        l = self.integrate("E", [Eh[..., c] * W * g for c in range(3)])
        return self.mass1_solve("E", l, tol=tol)[0]

    # ------------------------------------------------------------------
    # energies
    # ------------------------------------------------------------------
    def energy1(self, e, h) -> float:
        """The paper's (1/2)(e.M^1_eps e + h.M~^1_mu h) at one time level."""
        return 0.5 * (e @ self.mass1_apply("E", e) + h @ self.mass1_apply("H", h))

    def energy1_modified(self, e, h_lo, h_hi) -> float:
        """(1/2)(e^n.M e^n + h^{n-1/2}.M~ h^{n+1/2}), the leapfrog invariant."""
        return 0.5 * (e @ self.mass1_apply("E", e) + h_lo @ self.mass1_apply("H", h_hi))

    # ------------------------------------------------------------------
    # CFL
    # ------------------------------------------------------------------
    def apply_A1(self, e, tol=1e-15):
        """A1 e = M^{-1} K1^T D~^1 M~^{-1} K~1^T D^1 e (the e-e leapfrog operator)."""
        dh, _ = self.mass1_solve("H", self.rhs_h(e), tol=tol)
        de, _ = self.mass1_solve("E", self.rhs_e(dh), tol=tol)
        return de

    def cfl1(self, iters: int = 2000, tol: float = 1e-10, seed: int = 0) -> float:
        """dt_max = 2 / sqrt(lambda_max(A1)) by power iteration (seeded)."""
        x = np.random.default_rng([seed, 98]).standard_normal(self.n_e)
        x /= np.linalg.norm(x)
        lam = 0.0
        for _ in range(iters):
            y = self.apply_A1(x, tol=1e-13)
            lam_new = np.linalg.norm(y)
            x = y / lam_new
            if abs(lam_new - lam) <= tol * lam_new:
                lam = lam_new
                break
            lam = lam_new
        return 2.0 / math.sqrt(lam)
