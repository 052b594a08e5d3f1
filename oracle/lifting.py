"""Non-homogeneous tangential boundary data for the electric field (oracle,
FP64).

Test infrastructure only (see ``oracle/__init__``).

What is computed (paper, Section 3.5, with the separable-in-time data of the
coaxial cable test, Section 5.1.2):

* The electric field is split as E_h = E_{h,0} + E_{h,b}: E_{h,0} in X^1_{h,0}
  (the unknowns e of the scheme) and a lifting E_{h,b} in the whole X^1_h,
  carried by the basis functions with a non-vanishing tangential trace.
* Trace projection (the paper asks for a projection of the boundary data on
  the trace space without fixing it; reading): the boundary coefficients e_b
  minimise the sum over the six faces of the parametric L^2 distance between
  the tangential components of the pulled-back data E^ = DF^T E o F and those
  of the trace of the lifting, one least-squares problem for all faces, so a
  coefficient shared by two faces (an edge) is fitted to both.  It returns
  the boundary coefficients of any field of X^1_h from its own trace.
* Second scheme with the lifting: (K1)_0 e_0 = M~ d - (K1)_b e_b, D^1 acting
  from X^1_h to X^2_h and the Hodge K~1 h = M^2_{1/mu} b with b in the whole
  X^2_h (the mass matrix takes trial functions in X^2_h, test functions in
  X^2_{h,0}).  For data E_b(x, t) = sum_j g_j(t) E_b^j(x) the lifting is
  e_b(t) = sum_j g_j(t) e_b^j, and the (e, h) leapfrog becomes
      h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M D^1 e_0^n - dt sum_j g_j(t_n) v_h^j
      e_0^{n+1} = e_0^n + dt K1^{-1} M~ D~^1 h^{n+1/2}
                  - sum_j (g_j(t_{n+1}) - g_j(t_n)) v_e^j
  with v_h^j = K~1^{-1} M_{0,f} D^1_f e_b^j and v_e^j = (K1)_0^{-1} (K1)_b e_b^j
  formed once: the first from Faraday on the whole space, b^{n+1/2} =
  b^{n-1/2} - dt D^1_f (e_0^n + e_b(t_n)), the second from the Hodge of the
  full field at t_{n+1} and t_n with d^{n+1} = d^n + dt D~^1 h^{n+1/2}.
"""
from __future__ import annotations

import numpy as np

from .scheme import Scheme, _mode
from .spaces import comp_tags, join, split

FULL = {"E": "Ef", "B": "Bf"}


class LiftedScheme(Scheme):
    """Scheme 2 with non-homogeneous tangential data for E (Section 3.5)."""

    def __init__(self, *args, **kwargs):
        super().__init__(*args, **kwargs)
        self.C["Pf"] = self.axis.eval("Pf", self.xq)
        # Dd-by-Pf pairing of the axis, the across factor of (K1)_f
        x, w = self.axis.gauss()
        self.G_full = self.axis.eval("Dd", x).T @ (w[:, None] * self.axis.eval("Pf", x))

    # ------------------------------------------------------------------
    # the whole space X^1_h: interior embedding and boundary coefficients
    # ------------------------------------------------------------------
    def n_full(self, space="Ef") -> int:
        return sum(int(np.prod(self._shape(space, c))) for c in range(3))

    def _shape(self, space, c):
        tx, ty, tz = comp_tags(space, c)
        d = self.axis.dims
        return (d[tz], d[ty], d[tx])

    def embed(self, e0: np.ndarray) -> np.ndarray:
        """The field of X^1_{h,0} as a vector of X^1_h (boundary coefficients 0)."""
        E = split(self.axis, "E", e0)
        out = []
        for c in range(3):
            F = np.zeros(self._shape("Ef", c))
            sl = [slice(1, -1)] * 3
            sl[2 - c] = slice(None)  # along c the Pd index is the same
            F[tuple(sl)] = E[c]
            out.append(F)
        return join(out)

    def interior(self, e_full: np.ndarray) -> np.ndarray:
        """The coefficients of X^1_{h,0} inside a vector of X^1_h."""
        F = split(self.axis, "Ef", e_full)
        out = []
        for c in range(3):
            sl = [slice(1, -1)] * 3
            sl[2 - c] = slice(None)
            out.append(F[c][tuple(sl)])
        return join(out)

    def boundary_mask(self) -> np.ndarray:
        """True at the coefficients of X^1_h that are not in X^1_{h,0}."""
        return self.embed(np.ones(self.n_e)) == 0.0

    # ------------------------------------------------------------------
    # operators on the whole spaces
    # ------------------------------------------------------------------
    def curl_full(self, e_full: np.ndarray) -> np.ndarray:
        """D^1 from X^1_h to X^2_h: component c = d_{c+1} u_{c+2} - d_{c+2} u_{c+1}
        with the full incidence (d_f v)[k] = v[k+1] - v[k] along a Pf axis."""
        U = split(self.axis, "Ef", e_full)

        def d_full(v, ax):
            k = 2 - ax
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            hi[k] = slice(1, None)
            lo[k] = slice(0, -1)
            return v[tuple(hi)] - v[tuple(lo)]

        out = []
        for c in range(3):
            a1, a2 = (c + 1) % 3, (c + 2) % 3
            out.append(d_full(U[a2], a1) - d_full(U[a1], a2))
        return join(out)

    def mass_apply_trial_full(self, b_full: np.ndarray) -> np.ndarray:
        """M^2_{1/mu} b for b in X^2_h, tested with X^2_{h,0} (sum factorised)."""
        G = self.metric()
        X = split(self.axis, "Bf", b_full)
        V = []
        for c in range(3):
            v = X[c]
            for a, t in enumerate(comp_tags("Bf", c)):
                v = _mode(v, self.C[t], a)
            V.append(v)
        inv = None if self.mu is None else self._elem_to_q(1.0 / self.mu)
        U = []
        for i in range(3):
            acc = G[i, 0] * V[0] + G[i, 1] * V[1] + G[i, 2] * V[2]
            U.append(acc if inv is None else acc * inv)
        return self.integrate("B", U)

    def K1_apply_full(self, e_full: np.ndarray) -> np.ndarray:
        """(K1)_f e = [(K1)_0 (K1)_b] e for e in X^1_h: block c is M^ along c and
        the Dd-by-Pf pairing across (the Kronecker form of eq. (4.2) with the
        boundary columns kept)."""
        X = split(self.axis, "Ef", e_full)
        out = []
        for c in range(3):
            Y = X[c]
            for a in range(3):
                Y = _mode(Y, self.M if a == c else self.G_full, a)
            out.append(Y)
        return join(out)

    # ------------------------------------------------------------------
    # trace projection (the lifting)
    # ------------------------------------------------------------------
    def face_points(self, a: int, s: int) -> np.ndarray:
        """Parametric Gauss points of face x^_a = s: (Q, Q, 3) indexed by the
        two other axes in increasing order."""
        b1, b2 = [k for k in range(3) if k != a]
        P = np.zeros((self.Q, self.Q, 3))
        P[..., a] = float(s)
        P[..., b1] = self.xq[:, None]
        P[..., b2] = self.xq[None, :]
        return P

    def trace_rows(self, a: int, s: int, c: int):
        """Values of the tangential component c of every basis function of X^1_h
        at the Gauss points of face x^_a = s: (Q*Q, n_full)."""
        n_full = self.n_full()
        offs = np.cumsum([0] + [int(np.prod(self._shape("Ef", k))) for k in range(3)])
        P = self.face_points(a, s).reshape(-1, 3)
        tags = comp_tags("Ef", c)
        B = [self.axis.eval(tags[k], P[:, k]) for k in range(3)]  # x, y, z
        rows = np.einsum("qz,qy,qx->qzyx", B[2], B[1], B[0]).reshape(P.shape[0], -1)
        out = np.zeros((P.shape[0], n_full))
        out[:, offs[c]:offs[c + 1]] = rows
        return out

    def lift(self, efield) -> np.ndarray:
        """Boundary coefficients e_b (a vector of X^1_h, zero in the interior)
        of the physical field efield(xyz) -> (..., 3): the least-squares fit of
        the tangential components of E^ = DF^T E o F on the six faces."""
        def ehat(P):
            E = efield(self.geo.F(P))
            return np.einsum("...ki,...k->...i", self.geo.DF(P), E)
        return self.lift_hat(ehat)

    def lift_hat(self, ehat) -> np.ndarray:
        """The same fit from the pulled-back field ehat(x^) -> (..., 3) given at
        parametric points."""
        mask = self.boundary_mask()
        wq = self.wq
        W2 = (wq[:, None] * wq[None, :]).ravel()
        A_rows, rhs = [], []
        for a in range(3):
            for s in (0, 1):
                Eh = ehat(self.face_points(a, s)).reshape(-1, 3)
                for c in range(3):
                    if c == a:
                        continue
                    R = self.trace_rows(a, s, c)[:, mask]
                    A_rows.append(np.sqrt(W2)[:, None] * R)
                    rhs.append(np.sqrt(W2) * Eh[:, c])
        A = np.vstack(A_rows)
        y = np.concatenate(rhs)
        x, *_ = np.linalg.lstsq(A, y, rcond=None)
        e_b = np.zeros(self.n_full())
        e_b[mask] = x
        return e_b

    # ------------------------------------------------------------------
    # the leapfrog with the lifting
    # ------------------------------------------------------------------
    def lifting_vectors(self, e_b: np.ndarray):
        """(v_h, v_e) = (K~1^{-1} M_{0,f} D^1_f e_b, (K1)_0^{-1} (K1)_b e_b)."""
        v_h = self.kron_solve("K1t", self.mass_apply_trial_full(self.curl_full(e_b)))
        v_e = self.kron_solve("K1", self.K1_apply_full(e_b))
        return v_h, v_e

    def init_lifted(self, efield0, terms, dt, d_tol=1e-15):
        """Initial state from the exact field at t = 0 (Section 5.1.2: D
        projected onto the 2-forms, H^0 = 0 here): d^0 = M~^{-1} l,
        e_0^0 = K1^{-1} l - sum_j g_j(0) v_e^j (the Hodge with the lifting),
        and the backward half kick h^{-1/2} = (dt/2) (K~1^{-1} M D^1 e_0^0 +
        sum_j g_j(0) v_h^j).  terms: list of (v_h, v_e, g)."""
        e0 = self.project_E(efield0)
        for _, v_e, g in terms:
            e0 = e0 - g(0.0) * v_e
        h = 0.5 * dt * self.half_step_h(e0)
        for v_h, _, g in terms:
            h = h + 0.5 * dt * g(0.0) * v_h
        return e0, h

    def step_lifted(self, e0, h, dt, nsteps, terms, t0=0.0):
        """nsteps of the lifted leapfrog from (e_0^n, h^{n-1/2}) at t0."""
        e0 = np.array(e0, dtype=float, copy=True)
        h = np.array(h, dtype=float, copy=True)
        for n in range(nsteps):
            tn, tn1 = t0 + n * dt, t0 + (n + 1) * dt
            h -= dt * self.half_step_h(e0)
            for v_h, _, g in terms:
                h -= dt * g(tn) * v_h
            e0 += dt * self.half_step_e(h)
            for _, v_e, g in terms:
                e0 -= (g(tn1) - g(tn)) * v_e
        return e0, h

    def field_full_at_quad(self, e_full: np.ndarray) -> np.ndarray:
        """Physical E = DF^{-T} E^ of a field of X^1_h at the Gauss points."""
        X = split(self.axis, "Ef", e_full)
        V = []
        for c in range(3):
            v = X[c]
            for a, t in enumerate(comp_tags("Ef", c)):
                v = _mode(v, self.C[t], a)
            V.append(v)
        V = np.stack(V, axis=-1)
        DF = self.geo.DF(self.quad_points())
        return np.linalg.solve(np.swapaxes(DF, -1, -2), V[..., None])[..., 0]
