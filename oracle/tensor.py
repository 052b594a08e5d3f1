"""Scheme 2 with a degree, a knot vector and an element count per direction
(oracle, FP64, plain NumPy).

Test infrastructure only (see ``oracle/__init__``).

Section 4.1 lifts the assumption of one degree p and one knot vector Xi for
the three directions: with p_i and Xi_i per direction i the pairing blocks keep
their Kronecker form (4.2)/(4.3), each 1D factor G^i or M^i built from the
bases of direction i, and every solve is still one 1D LU solve per axis
(eq. (4.4), (4.5)).  The remark after (4.5) on reordering directions concerns
only the sizes of the solves; the result does not depend on it.  Nothing else
in the scheme changes: the spaces are tensor products of the per-direction
univariate spaces (Section 2.3), the curls are the same +-1 index differences
(Section 2.4) and the mass applies the same integrals (Section 3.4), now over
per-direction Gauss rules with p_i + 1 points per element.

The structure follows ``scheme.Scheme`` (same unknown layout, same leapfrog and
energies) with every axis-dependent quantity indexed by direction; the
isotropic case reproduces ``Scheme``.  Level-0 counterparts (3D quadrature of
3D basis functions, no Kronecker factorisation or sum factorisation) are here
too, for the tests: ``pairing_dense``, ``mass_dense``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .geometry import Map, metric_2form
from .spaces import SPACE_TAGS
from .splines import Axis

# 1D factor of block c of each pairing matrix along axis a (eq. (4.2), (4.3))
_K_FACTOR = {
    "K1": lambda c, a: ("M", False) if a == c else ("G", False),
    "K1t": lambda c, a: ("G", True) if a == c else ("M", True),
}
_K_SPACES = {"K1": ("E", "D"), "K1t": ("H", "B")}  # (column space, row space)


def _mode(X: np.ndarray, C: np.ndarray, ax: int) -> np.ndarray:
    """Apply matrix C along parametric axis ax (0 = x, the last array axis)."""
    k = 2 - ax
    return np.moveaxis(np.tensordot(C, X, axes=([1], [k])), 0, k)


def _tags(space: str, c: int):
    f = SPACE_TAGS[space]
    return tuple(f(c, a) for a in range(3))


class TensorScheme:
    """Scheme 2 on the unit cube mapped by `geo`; direction a (0 = x) has
    degree p[a], n_elem[a] elements and interior breakpoints breaks[a] (None:
    uniform)."""

    def __init__(self, p, n_elem, breaks=(None, None, None), geo: Map | None = None,
                 eps: np.ndarray | None = None, mu: np.ndarray | None = None):
        self.p = tuple(int(v) for v in p)
        self.N = tuple(int(v) for v in n_elem)
        self.axes = tuple(Axis(self.N[a], self.p[a], breaks[a]) for a in range(3))
        self.geo = geo if geo is not None else Map("identity")
        shape = (self.N[2], self.N[1], self.N[0])
        self.eps = None if eps is None else np.asarray(eps, float).reshape(shape)
        self.mu = None if mu is None else np.asarray(mu, float).reshape(shape)
        self.nq = tuple(pa + 1 for pa in self.p)
        gw = [ax.gauss() for ax in self.axes]
        self.xq = [g[0] for g in gw]
        self.wq = [g[1] for g in gw]
        self.n_e = self.space_size("E")
        self.n_h = self.space_size("H")
        # per direction: 1D pairing matrices (Section 4.1) and their LU factors
        self.G = [ax.G_hat() for ax in self.axes]
        self.M = [ax.M_hat() for ax in self.axes]
        self._mat, self._lu = [], []
        for a in range(3):
            mats = {("G", False): self.G[a], ("G", True): self.G[a].T,
                    ("M", False): self.M[a], ("M", True): self.M[a].T}
            self._mat.append(mats)
            self._lu.append({k: sla.lu_factor(v) for k, v in mats.items()})
        # per direction: collocation matrices at the Gauss points
        self.C = [{t: self.axes[a].eval(t, self.xq[a]) for t in ("Pv", "Pd", "Dv", "Dd")} for a in range(3)]
        self._metric = None

    # ------------------------------------------------------------------
    # unknown layout: components one after the other, x fastest inside
    # ------------------------------------------------------------------
    def comp_shape(self, space: str, c: int):
        """(n_z, n_y, n_x) of component c: direction a contributes the
        dimension of its univariate space of the component's tag."""
        t = _tags(space, c)
        return tuple(self.axes[a].dims[t[a]] for a in (2, 1, 0))

    def space_size(self, space: str) -> int:
        return sum(int(np.prod(self.comp_shape(space, c))) for c in range(3))

    def split(self, space: str, v: np.ndarray):
        out, o = [], 0
        for c in range(3):
            sh = self.comp_shape(space, c)
            n = int(np.prod(sh))
            out.append(np.asarray(v)[o:o + n].reshape(sh))
            o += n
        if o != np.asarray(v).size:
            raise ValueError(f"vector of length {np.asarray(v).size} is not in space {space}")
        return out

    @staticmethod
    def join(parts) -> np.ndarray:
        return np.concatenate([np.asarray(x).ravel() for x in parts])

    # ------------------------------------------------------------------
    # geometry at the Gauss points
    # ------------------------------------------------------------------
    def quad_points(self) -> np.ndarray:
        """Parametric Gauss points (Qz, Qy, Qx, 3), x first in the last axis."""
        Z, Y, X = np.meshgrid(self.xq[2], self.xq[1], self.xq[0], indexing="ij")
        return np.stack([X, Y, Z], axis=-1)

    def weights(self) -> np.ndarray:
        return self.wq[2][:, None, None] * self.wq[1][None, :, None] * self.wq[0][None, None, :]

    def metric(self) -> np.ndarray:
        """w_q DF^T DF / det DF at the Gauss points, (3, 3, Qz, Qy, Qx)."""
        if self._metric is None:
            G = metric_2form(self.geo.DF(self.quad_points()))
            self._metric = np.moveaxis(G * self.weights()[..., None, None], (-2, -1), (0, 1)).copy()
        return self._metric

    def _elem_to_q(self, v: np.ndarray) -> np.ndarray:
        """Per-element values (Nz, Ny, Nx) repeated onto the Gauss points."""
        return np.repeat(np.repeat(np.repeat(v, self.nq[2], axis=0), self.nq[1], axis=1), self.nq[0], axis=2)

    # ------------------------------------------------------------------
    # curls (Section 2.4): component c = d_{c+1} u_{c+2} - d_{c+2} u_{c+1}
    # ------------------------------------------------------------------
    @staticmethod
    def _diff(v: np.ndarray, ax: int, primal: bool) -> np.ndarray:
        """primal: (d v)[k] = v[k] - v[k-1], k = 0..n (zero outside);
        dual: (d~ v)[r] = v[r+1] - v[r]."""
        k = 2 - ax
        if primal:
            pad = [(0, 0)] * 3
            pad[k] = (1, 1)
            v = np.pad(v, pad)
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[k] = slice(1, None)
        lo[k] = slice(0, -1)
        return v[tuple(hi)] - v[tuple(lo)]

    def curl(self, u: np.ndarray, primal: bool) -> np.ndarray:
        U = self.split("E" if primal else "H", u)
        out = []
        for c in range(3):
            a1, a2 = (c + 1) % 3, (c + 2) % 3
            out.append(self._diff(U[a2], a1, primal) - self._diff(U[a1], a2, primal))
        return self.join(out)

    def div(self, u: np.ndarray, primal: bool) -> np.ndarray:
        U = self.split("B" if primal else "D", u)
        return (self._diff(U[0], 0, primal) + self._diff(U[1], 1, primal) + self._diff(U[2], 2, primal)).ravel()

    def curl_primal(self, e):
        return self.curl(e, True)

    def curl_dual(self, h):
        return self.curl(h, False)

    # ------------------------------------------------------------------
    # pairing matrices: Kronecker apply and solve with per-direction factors
    # ------------------------------------------------------------------
    def kron_apply(self, which: str, x: np.ndarray, transpose: bool = False) -> np.ndarray:
        col, row = _K_SPACES[which]
        if transpose:
            col, row = row, col
        X = self.split(col, x)
        out = []
        for c in range(3):
            Y = X[c]
            for a in range(3):
                name, tr = _K_FACTOR[which](c, a)
                Y = _mode(Y, self._mat[a][(name, tr != transpose)], a)
            out.append(Y)
        return self.join(out)

    def kron_solve(self, which: str, y: np.ndarray, transpose: bool = False) -> np.ndarray:
        col, row = _K_SPACES[which]
        if transpose:
            col, row = row, col
        Y = self.split(row, y)
        out = []
        for c in range(3):
            X = Y[c]
            for a in range(3):
                name, tr = _K_FACTOR[which](c, a)
                k = 2 - a
                Xm = np.moveaxis(X, k, 0)
                sh = Xm.shape
                Xm = sla.lu_solve(self._lu[a][(name, tr != transpose)], Xm.reshape(sh[0], -1)).reshape(sh)
                X = np.moveaxis(Xm, 0, k)
            out.append(X)
        return self.join(out)

    # ------------------------------------------------------------------
    # mass applies (Section 3.4), sum-factorised over per-direction rules
    # ------------------------------------------------------------------
    def interpolate(self, space: str, x: np.ndarray):
        X = self.split(space, x)
        vals = []
        for c in range(3):
            V = X[c]
            for a, t in enumerate(_tags(space, c)):
                V = _mode(V, self.C[a][t], a)
            vals.append(V)
        return vals

    def integrate(self, space: str, F) -> np.ndarray:
        out = []
        for c in range(3):
            V = F[c]
            for a, t in enumerate(_tags(space, c)):
                V = _mode(V, self.C[a][t].T, a)
            out.append(V)
        return self.join(out)

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
    # the leapfrog (e, h) step and its energies (as in scheme.Scheme)
    # ------------------------------------------------------------------
    def step(self, e, h, dt, nsteps=1, d=None, b=None, energy_every: int = 0):
        """Advance (e^n, h^{n-1/2}) by nsteps, source free; returns
        (e, h, d, b, energies) with d, b tracked when given."""
        e = np.array(e, dtype=float, copy=True)
        h = np.array(h, dtype=float, copy=True)
        track = d is not None
        if track:
            d = np.array(d, dtype=float, copy=True)
            b = np.array(b, dtype=float, copy=True)
        energies = []
        for n in range(nsteps):
            u = self.curl_primal(e)
            h -= dt * self.kron_solve("K1t", self.mass_apply("B", u))
            if track:
                b -= dt * u
            v = self.curl_dual(h)
            e += dt * self.kron_solve("K1", self.mass_apply("D", v))
            if track:
                d += dt * v
                if energy_every and (n + 1) % energy_every == 0:
                    energies.append(self.energy(e, h, d, b, dt)[0])
        return e, h, d, b, energies

    def energy(self, e, h, d, b, dt):
        """(modified, paper) energies of the state (e^n, d^n, h^{n-1/2},
        b^{n-1/2}), as ``scheme.Scheme.energy``."""
        v = self.kron_apply("K1", e)
        u = self.kron_apply("K1t", h)
        w = self.curl_primal(e)
        paper = 0.5 * (v @ d + u @ b)
        return paper - 0.5 * dt * (u @ w), paper

    def cfl(self, iters: int = 2000, tol: float = 1e-10, seed: int = 0) -> float:
        """Largest stable dt = 2 / sqrt(lambda_max) of the e-update operator
        K1^{-1} M~ D~^1 K~1^{-1} M D^1, by power iteration."""
        rng = np.random.default_rng(seed)
        x = rng.standard_normal(self.n_e)
        lam = 0.0
        for _ in range(iters):
            y = self.kron_solve("K1", self.mass_apply("D", self.curl_dual(
                self.kron_solve("K1t", self.mass_apply("B", self.curl_primal(x))))))
            lam_new = float(np.linalg.norm(y) / np.linalg.norm(x))
            x = y / np.linalg.norm(y)
            if abs(lam_new - lam) <= tol * lam_new:
                lam = lam_new
                break
            lam = lam_new
        return 2.0 / np.sqrt(lam)

    # ------------------------------------------------------------------
    # level 0 (tests only): 3D quadrature of 3D basis functions
    # ------------------------------------------------------------------
    def basis_3d(self, space: str, c: int, pts: np.ndarray) -> np.ndarray:
        """Values of every basis function of component c at 3D points (npts, 3),
        each the product of its three 1D factors evaluated at the point."""
        t = _tags(space, c)
        B = [self.axes[a].eval(t[a], pts[:, a]) for a in range(3)]
        out = np.empty((pts.shape[0], B[2].shape[1], B[1].shape[1], B[0].shape[1]))
        for q in range(pts.shape[0]):
            out[q] = B[2][q][:, None, None] * B[1][q][None, :, None] * B[0][q][None, None, :]
        return out.reshape(pts.shape[0], -1)

    def _pts_weights(self):
        P = self.quad_points().reshape(-1, 3)
        return P, self.weights().ravel()

    def pairing_dense(self, which: str) -> np.ndarray:
        """K1 (rows X~^2, columns X^1_{h,0}) or K~1 (rows X^2_{h,0}, columns
        X~^1): entries the integrals of products of 3D basis functions."""
        col, row = _K_SPACES[which]
        pts, w = self._pts_weights()
        K = np.zeros((self.space_size(row), self.space_size(col)))
        ro = np.cumsum([0] + [int(np.prod(self.comp_shape(row, c))) for c in range(3)])
        co = np.cumsum([0] + [int(np.prod(self.comp_shape(col, c))) for c in range(3)])
        for c in range(3):
            R = self.basis_3d(row, c, pts)
            Cm = self.basis_3d(col, c, pts)
            K[ro[c]:ro[c + 1], co[c]:co[c + 1]] = R.T @ (w[:, None] * Cm)
        return K

    def mass_dense(self, space: str) -> np.ndarray:
        """The 2-form mass matrix: entries sum_q w_q u_i(q)^T G(q) u_j(q) / gamma
        with G = DF^T DF / det DF evaluated point by point."""
        pts, w = self._pts_weights()
        G = metric_2form(self.geo.DF(pts))  # (npts, 3, 3)
        g = self.mu if space == "B" else self.eps
        scale = w.copy()
        if g is not None:
            scale = scale / self._elem_to_q(g).ravel()
        B = [self.basis_3d(space, c, pts) for c in range(3)]
        n = self.space_size(space)
        o = np.cumsum([0] + [b.shape[1] for b in B])
        M = np.zeros((n, n))
        for i in range(3):
            for j in range(3):
                M[o[i]:o[i + 1], o[j]:o[j + 1]] = B[i].T @ ((scale * G[:, i, j])[:, None] * B[j])
        return M
