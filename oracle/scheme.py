"""Level 1 of the oracle: the structured scheme-2 leapfrog (FP64, plain NumPy).

Test infrastructure only (see ``oracle/__init__``).

What is computed (paper, Section 3.4 and Section 4):

  semi-discrete scheme (3.10)-(3.13)
      d_t d = D~^1 h - j,   K1 e = M~^2_{1/eps} d,
      d_t b = - D^1 e,      K~1 h = M^2_{1/mu} b,
  in the equivalent Petrov-Galerkin (e, h) form of Section 3.4.2
      K~1 d_t h = - M^2_{1/mu} D^1 e,   K1 d_t e = M~^2_{1/eps} D~^1 h - s,
  with s = M~ j the tested source, advanced by the staggered leapfrog
      h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M D^1 e^n
      e^{n+1}   = e^n + dt K1^{-1} (M~ D~^1 h^{n+1/2} - s(t_{n+1/2})),
  optionally tracking b and d with b^{n+1/2} = b^{n-1/2} - dt D^1 e^n and
  d^{n+1} = d^n + dt D~^1 h^{n+1/2} (source-free runs only).

* Pairing solves: K1 and K~1 are block diagonal with Kronecker blocks
  (4.2)/(4.3); each block is inverted one axis at a time with the LU factors of
  the 1D matrices G^, M^ (eq. (4.4) and the vec identity before (4.5)).
* Mass applies: y = B^T W G B x with B the collocation of the basis at the
  Gauss points, applied as three mode products with dense 1D collocation
  matrices (sum factorisation), G the 2-form metric factor.
* Curls: the +-1 incidence matrices applied as index differences.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .geometry import Map, metric_2form
from .spaces import SPACE_TAGS, comp_shape, comp_tags, join, space_size, split
from .splines import Axis

# 1D factor of block c of each pairing matrix along axis a
#   K1  block c = (x) over axes of: M^ along axis c, G^ across   (eq. (4.2))
#   K~1 block c = (x) over axes of: G^T along axis c, M^T across (eq. (4.3))
_K_FACTOR = {
    "K1": lambda c, a: ("M", False) if a == c else ("G", False),
    "K1t": lambda c, a: ("G", True) if a == c else ("M", True),
}
_K_SPACES = {"K1": ("E", "D"), "K1t": ("H", "B")}  # (column space, row space)


def composition_weights(order: int):
    """Step weights c_1..c_m of the symmetric composition of the leapfrog
    (kick-drift-kick) that has the given even order: order 2 is the leapfrog,
    order 2k+2 composes three order-2k methods with the triple-jump weights
    z1 = 1 / (2 - 2^(1/(2k+1))), z0 = 1 - 2 z1 (Yoshida 1990; the paper names
    pairing the scheme with higher-order symplectic integrators as future
    work, Section 6)."""
    if order not in (2, 4, 6):
        raise ValueError("order must be 2, 4 or 6")
    c = [1.0]
    for k in range(1, order // 2):
        z1 = 1.0 / (2.0 - 2.0 ** (1.0 / (2 * k + 1)))
        z0 = 1.0 - 2.0 * z1
        c = [w * z for z in (z1, z0, z1) for w in c]
    return c


def _mode(X: np.ndarray, C: np.ndarray, ax: int) -> np.ndarray:
    """Apply matrix C along parametric axis ax (0 = x, the last array axis)."""
    k = 2 - ax
    return np.moveaxis(np.tensordot(C, X, axes=([1], [k])), 0, k)


class Scheme:
    """Scheme 2 on the unit cube mapped by `geo`, degree p, N elements per axis."""

    def __init__(self, p: int, n_elem: int, geo: Map | None = None,
                 eps: np.ndarray | None = None, mu: np.ndarray | None = None):
        self.p, self.N = p, n_elem
        self.axis = Axis(n_elem, p)
        self.geo = geo if geo is not None else Map("identity")
        self.nq = p + 1
        self.xq, self.wq = self.axis.gauss()
        self.Q = self.xq.size
        self.eps = None if eps is None else np.asarray(eps, float).reshape(n_elem, n_elem, n_elem)
        self.mu = None if mu is None else np.asarray(mu, float).reshape(n_elem, n_elem, n_elem)
        self.n_e = space_size(self.axis, "E")
        self.n_h = space_size(self.axis, "H")
        # 1D pairing matrices and their LU factors (Section 4.2)
        self.G = self.axis.G_hat()
        self.M = self.axis.M_hat()
        self._lu = {("G", False): sla.lu_factor(self.G), ("G", True): sla.lu_factor(self.G.T),
                    ("M", False): sla.lu_factor(self.M), ("M", True): sla.lu_factor(self.M.T)}
        self._mat = {("G", False): self.G, ("G", True): self.G.T,
                     ("M", False): self.M, ("M", True): self.M.T}
        # collocation matrices at the Gauss points
        self.C = {t: self.axis.eval(t, self.xq) for t in ("Pv", "Pd", "Dv", "Dd")}
        self._metric = None

    # ------------------------------------------------------------------
    # geometry at the Gauss points
    # ------------------------------------------------------------------
    def quad_points(self) -> np.ndarray:
        """Parametric Gauss points, array (Q, Q, Q, 3) indexed [qz, qy, qx]."""
        Z, Y, X = np.meshgrid(self.xq, self.xq, self.xq, indexing="ij")
        return np.stack([X, Y, Z], axis=-1)

    def metric(self) -> np.ndarray:
        """w_q * DF^T DF / det DF at the Gauss points, (3, 3, Q, Q, Q)."""
        if self._metric is None:
            xh = self.quad_points()
            G = metric_2form(self.geo.DF(xh))  # (Q,Q,Q,3,3)
            W = self.wq[:, None, None] * self.wq[None, :, None] * self.wq[None, None, :]
            self._metric = np.moveaxis(G * W[..., None, None], (-2, -1), (0, 1)).copy()
        return self._metric

    def _elem_to_q(self, v: np.ndarray) -> np.ndarray:
        r = self.nq
        return np.repeat(np.repeat(np.repeat(v, r, axis=0), r, axis=1), r, axis=2)

    # ------------------------------------------------------------------
    # curls (Section 2.4): component c = d_{c+1} u_{c+2} - d_{c+2} u_{c+1}
    # ------------------------------------------------------------------
    @staticmethod
    def _diff_primal(v: np.ndarray, ax: int) -> np.ndarray:
        """(d v)[k] = v[k] - v[k-1], k = 0..n0 (zero outside 0..n0-1)."""
        k = 2 - ax
        pad = [(0, 0)] * 3
        pad[k] = (1, 1)
        w = np.pad(v, pad)
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[k] = slice(1, None)
        lo[k] = slice(0, -1)
        return w[tuple(hi)] - w[tuple(lo)]

    @staticmethod
    def _diff_dual(v: np.ndarray, ax: int) -> np.ndarray:
        """(d~ v)[r] = v[r+1] - v[r], r = 0..n1-2."""
        k = 2 - ax
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[k] = slice(1, None)
        lo[k] = slice(0, -1)
        return v[tuple(hi)] - v[tuple(lo)]

    def curl(self, u: np.ndarray, primal: bool) -> np.ndarray:
        src = "E" if primal else "H"
        diff = self._diff_primal if primal else self._diff_dual
        U = split(self.axis, src, u)
        out = []
        for c in range(3):
            a1, a2 = (c + 1) % 3, (c + 2) % 3
            out.append(diff(U[a2], a1) - diff(U[a1], a2))
        return join(out)

    def div(self, u: np.ndarray, primal: bool) -> np.ndarray:
        """D^2 b (primal) or D~^2 d (dual): sum_a d_a u_a, a 2-form -> 3-form."""
        src = "B" if primal else "D"
        diff = self._diff_primal if primal else self._diff_dual
        U = split(self.axis, src, u)
        return (diff(U[0], 0) + diff(U[1], 1) + diff(U[2], 2)).ravel()

    def curl_primal(self, e):
        """D^1 e, X^1_{h,0} -> X^2_{h,0}."""
        return self.curl(e, True)

    def curl_dual(self, h):
        """D~^1 h, X~^1 -> X~^2."""
        return self.curl(h, False)

    # ------------------------------------------------------------------
    # pairing matrices: Kronecker apply and solve (eq. (4.2)-(4.5))
    # ------------------------------------------------------------------
    def kron_apply(self, which: str, x: np.ndarray, transpose: bool = False) -> np.ndarray:
        col, row = _K_SPACES[which]
        if transpose:
            col, row = row, col
        X = split(self.axis, col, x)
        out = []
        for c in range(3):
            Y = X[c]
            for a in range(3):
                name, tr = _K_FACTOR[which](c, a)
                A = self._mat[(name, tr != transpose)]
                Y = _mode(Y, A, a)
            out.append(Y)
        return join(out)

    def kron_solve(self, which: str, y: np.ndarray, transpose: bool = False) -> np.ndarray:
        """x = K^{-1} y (or K^{-T} y), one 1D LU solve per axis and block."""
        col, row = _K_SPACES[which]
        if transpose:
            col, row = row, col
        Y = split(self.axis, row, y)
        out = []
        for c in range(3):
            X = Y[c]
            for a in range(3):
                name, tr = _K_FACTOR[which](c, a)
                lu = self._lu[(name, tr != transpose)]
                k = 2 - a
                Xm = np.moveaxis(X, k, 0)
                sh = Xm.shape
                Xm = sla.lu_solve(lu, Xm.reshape(sh[0], -1)).reshape(sh)
                X = np.moveaxis(Xm, 0, k)
            out.append(X)
        return join(out)

    # ------------------------------------------------------------------
    # mass applies (Section 3.4), sum-factorised
    # ------------------------------------------------------------------
    def interpolate(self, space: str, x: np.ndarray):
        """Parametric vector proxy of a field of `space` at the Gauss points:
        list of 3 arrays (Q, Q, Q)."""
        X = split(self.axis, space, x)
        vals = []
        for c in range(3):
            V = X[c]
            for a, t in enumerate(comp_tags(space, c)):
                V = _mode(V, self.C[t], a)
            vals.append(V)
        return vals

    def integrate(self, space: str, F) -> np.ndarray:
        """Load vector int w^_i . F over the Gauss points (F already weighted)."""
        out = []
        for c in range(3):
            V = F[c]
            for a, t in enumerate(comp_tags(space, c)):
                V = _mode(V, self.C[t].T, a)
            out.append(V)
        return join(out)

    def mass_apply(self, space: str, x: np.ndarray) -> np.ndarray:
        """M^2_{1/mu} x (space 'B') or M~^2_{1/eps} x (space 'D')."""
        G = self.metric()
        g = self.mu if space == "B" else self.eps
        V = self.interpolate(space, x)
        inv = None if g is None else self._elem_to_q(1.0 / g)
        U = []
        for i in range(3):
            acc = G[i, 0] * V[0] + G[i, 1] * V[1] + G[i, 2] * V[2]
            U.append(acc if inv is None else acc * inv)
        return self.integrate(space, U)

    # ------------------------------------------------------------------
    # the leapfrog (e, h) step
    # ------------------------------------------------------------------
    def half_step_h(self, e):
        """K~1^{-1} M^2_{1/mu} D^1 e."""
        return self.kron_solve("K1t", self.mass_apply("B", self.curl_primal(e)))

    def half_step_e(self, h, s=None):
        """K1^{-1} (M~^2_{1/eps} D~^1 h - s)."""
        y = self.mass_apply("D", self.curl_dual(h))
        if s is not None:
            y = y - s
        return self.kron_solve("K1", y)

    def step(self, e, h, dt, nsteps=1, t0=0.0, source=None, d=None, b=None,
             energy_every: int = 0):
        """Advance (e^n, h^{n-1/2}) by nsteps; returns (e, h, d, b, energies).

        source: None or a callable t -> tested source vector s(t) in X~^2 dual.
        d, b: optional tracked 2-forms (d^n, b^{n-1/2}); source must be None.
        energies: modified energy after every `energy_every` steps (needs d, b).
        """
        e = np.array(e, dtype=float, copy=True)
        h = np.array(h, dtype=float, copy=True)
        track = d is not None
        if track:
            if b is None or source is not None:
                raise ValueError("tracking needs both d and b and no source")
            d = np.array(d, dtype=float, copy=True)
            b = np.array(b, dtype=float, copy=True)
        energies = []
        for n in range(nsteps):
            t_half = t0 + (n + 0.5) * dt
            u = self.curl_primal(e)
            h -= dt * self.kron_solve("K1t", self.mass_apply("B", u))
            if track:
                b -= dt * u
            v = self.curl_dual(h)
            y = self.mass_apply("D", v)
            if source is not None:
                y = y - source(t_half)
            e += dt * self.kron_solve("K1", y)
            if track:
                d += dt * v
                if energy_every and (n + 1) % energy_every == 0:
                    energies.append(self.energy(e, h, d, b, dt)[0])
        return e, h, d, b, energies

    def step_split(self, e, h, dt, nsteps, order, d=None, b=None):
        """Advance (e^n, h^) by nsteps of the symmetric composition of the
        leapfrog of the given order (2, 4, 6; `composition_weights`), source
        free.  h^ is h with the first half kick of the next step taken back,
        h^ = h + (c_1 dt / 2) K~1^{-1} M D^1 e (`init_stagger` with c_1 dt).
        One step runs m substeps: h^ -= a_j dt K~1^{-1} M D^1 e, then
        e += c_j dt K1^{-1} M~ D~^1 h^, with a_1 = c_1 (the last half kick of
        the previous step merged with the first of this one, c_m = c_1) and
        a_j = (c_{j-1} + c_j) / 2.  Tracked b and d follow the same kicks."""
        c = composition_weights(order)
        a = [c[0]] + [0.5 * (c[j - 1] + c[j]) for j in range(1, len(c))]
        e = np.array(e, dtype=float, copy=True)
        h = np.array(h, dtype=float, copy=True)
        track = d is not None
        if track:
            d = np.array(d, dtype=float, copy=True)
            b = np.array(b, dtype=float, copy=True)
        for _ in range(nsteps):
            for aj, cj in zip(a, c):
                u = self.curl_primal(e)
                h -= aj * dt * self.kron_solve("K1t", self.mass_apply("B", u))
                if track:
                    b -= aj * dt * u
                v = self.curl_dual(h)
                e += cj * dt * self.kron_solve("K1", self.mass_apply("D", v))
                if track:
                    d += cj * dt * v
        return e, h, d, b

    def init_stagger(self, e0, h0, dt, b0=None):
        """Backward half kick from t = 0: h^{-1/2} = h^0 + dt/2 K~1^{-1} M D^1 e^0
        (and b^{-1/2} = b^0 + dt/2 D^1 e^0)."""
        h = np.array(h0, dtype=float) + 0.5 * dt * self.half_step_h(e0)
        b = None
        if b0 is not None:
            b = np.array(b0, dtype=float) + 0.5 * dt * self.curl_primal(e0)
        return h, b

    # ------------------------------------------------------------------
    # energies (eq. (3.2)) and the leapfrog invariant
    # ------------------------------------------------------------------
    def energy(self, e, h, d, b, dt):
        """State (e^n, d^n, h^{n-1/2}, b^{n-1/2}).

        Returns (modified, paper):
          paper    = 1/2 (e^T K~2 d + h^T K2 b) = 1/2 (d.K1 e + b.K~1 h)   (3.2)
          modified = 1/2 (d^n.M~ d^n + b^{n-1/2}.M b^{n+1/2}), exactly conserved by
                     the leapfrog with J = 0; written with pairing matrices as
                     1/2 (d.K1 e + b.K~1 h - dt (K~1 h).(D^1 e)).
        """
        v = self.kron_apply("K1", e)
        u = self.kron_apply("K1t", h)
        w = self.curl_primal(e)
        paper = 0.5 * (v @ d + u @ b)
        modified = paper - 0.5 * dt * (u @ w)
        return modified, paper

    def mass_energy(self, d, b_lo, b_hi):
        """1/2 (d.M~ d + b_lo.M b_hi), the modified energy through mass matrices."""
        return 0.5 * (d @ self.mass_apply("D", d) + b_lo @ self.mass_apply("B", b_hi))

    # ------------------------------------------------------------------
    # set-up: projection, CFL, sources, probes
    # ------------------------------------------------------------------
    def load_E(self, efield) -> np.ndarray:
        """l_i = int_Omega eta_i . E0 dx = int eta^_i . (DF^T E0(F(x^))) dx^, eta_i in X~^2."""
        xh = self.quad_points()
        E = efield(self.geo.F(xh))  # (Q,Q,Q,3) physical field at mapped points
        DF = self.geo.DF(xh)
        Eh = np.einsum("...ki,...k->...i", DF, E)  # DF^T E
        W = self.wq[:, None, None] * self.wq[None, :, None] * self.wq[None, None, :]
        return self.integrate("D", [Eh[..., c] * W for c in range(3)])

    def project_E(self, efield) -> np.ndarray:
        """e^0 = K1^{-1} l (the L^2_{1/eps} projection of D0 = eps E0 onto X~^2,
        followed by the Hodge (3.11); no mass solve is needed)."""
        return self.kron_solve("K1", self.load_E(efield))

    def project_D(self, efield, tol: float = 1e-15, maxiter: int = 5000) -> np.ndarray:
        """d^0 = M~^{-1} l by conjugate gradients on the mass apply."""
        l = self.load_E(efield)
        return self.cg_mass("D", l, tol=tol, maxiter=maxiter)

    def cg_mass(self, space, rhs, tol=1e-15, maxiter=5000):
        x = np.zeros_like(rhs)
        r = rhs.copy()
        pdir = r.copy()
        rr = r @ r
        stop = (tol * np.linalg.norm(rhs)) ** 2
        for _ in range(maxiter):
            if rr <= stop:
                break
            Ap = self.mass_apply(space, pdir)
            alpha = rr / (pdir @ Ap)
            x += alpha * pdir
            r -= alpha * Ap
            rr_new = r @ r
            pdir = r + (rr_new / rr) * pdir
            rr = rr_new
        return x

    def apply_A(self, e):
        """A e = K1^{-1} M~ D~^1 K~1^{-1} M D^1 e (the e-e leapfrog operator)."""
        return self.half_step_e(self.half_step_h(e))

    def cfl(self, iters: int = 2000, tol: float = 1e-10, seed: int = 0) -> float:
        """dt_max = 2 / sqrt(lambda_max(A)) by power iteration (seeded)."""
        x = np.random.default_rng([seed, 99]).standard_normal(self.n_e)
        x /= np.linalg.norm(x)
        lam = 0.0
        for _ in range(iters):
            y = self.apply_A(x)
            lam_new = np.linalg.norm(y)
            x = y / lam_new
            if abs(lam_new - lam) <= tol * lam_new:
                lam = lam_new
                break
            lam = lam_new
        return 2.0 / math.sqrt(lam)

    def _point_tags(self, space, c, xh):
        return [self.axis.eval(t, np.array([xh[a]]))[0] for a, t in enumerate(comp_tags(space, c))]

    def dipole_source(self, pos, moment) -> np.ndarray:
        """Tested point dipole s_i = (1/eps(x0)) q . eta_i(x0), eta_i = DF eta^_i / det DF
        the physical dual 2-form basis at parametric position pos."""
        xh = np.asarray(pos, float)
        DF = self.geo.DF(xh[None])[0]
        det = np.linalg.det(DF)
        el = np.minimum((xh * self.N).astype(int), self.N - 1)
        inv_eps = 1.0 if self.eps is None else 1.0 / self.eps[el[2], el[1], el[0]]
        out = []
        for c in range(3):
            bx, by, bz = self._point_tags("D", c, xh)
            coef = inv_eps * (np.asarray(moment, float) @ DF[:, c]) / det
            out.append(coef * bz[:, None, None] * by[None, :, None] * bx[None, None, :])
        return join(out)

    def probe_E(self, e, pos) -> np.ndarray:
        """Physical E_h = DF^{-T} E^_h at parametric point pos."""
        xh = np.asarray(pos, float)
        E = split(self.axis, "E", e)
        Eh = np.zeros(3)
        for c in range(3):
            bx, by, bz = self._point_tags("E", c, xh)
            Eh[c] = np.einsum("zyx,z,y,x->", E[c], bz, by, bx)
        DF = self.geo.DF(xh[None])[0]
        return np.linalg.solve(DF.T, Eh)

    def field_at_quad(self, space, x):
        """Physical field of a 1-form ('E' or 'H') at the Gauss points, (Q,Q,Q,3)."""
        V = np.stack(self.interpolate(space, x), axis=-1)
        DF = self.geo.DF(self.quad_points())
        return np.linalg.solve(np.swapaxes(DF, -1, -2), V[..., None])[..., 0]

    def l2_norm_sq_quad(self, F):
        """int |F|^2 dx over the physical domain from values at the Gauss points."""
        W = self.wq[:, None, None] * self.wq[None, :, None] * self.wq[None, None, :]
        det = np.linalg.det(self.geo.DF(self.quad_points()))
        return float(np.sum(W * det * np.sum(F * F, axis=-1)))
