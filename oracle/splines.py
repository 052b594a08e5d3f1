"""Univariate spline spaces of the primal and dual complexes (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

Section 2.3 of the paper: a p-open knot vector Xi with maximal regularity, its
trimmed versions Xi' (first and last knot removed) and Xi'' (two removed), the
primal spaces S_p(Xi) (boundary functions removed, Section 4 start) and
S_{p-1}(Xi'), and the dual spaces S_{p-1}(Xi') and S_{p-2}(Xi'').
Section 4.1: derivative spaces use scaled Curry-Schoenberg bases (unit
integral) so that the exterior derivative is a +-1 incidence matrix; value
spaces use standard B-splines.

The four 1D bases, by tag:
  Pv  primal value       S_p(Xi) without its two boundary functions   dim n0 = N+p-2
  Pd  primal derivative  Curry-Schoenberg basis of S_{p-1}(Xi')       dim n1 = N+p-1
  Dv  dual value         standard B-splines of S_{p-1}(Xi')            dim n1
  Dd  dual derivative    Curry-Schoenberg basis of S_{p-2}(Xi'')       dim n0
  Pf  primal value, full S_p(Xi) with its boundary functions           dim n0+2
      (only for non-homogeneous boundary data, Section 3.5)
"""
from __future__ import annotations

import numpy as np

TAGS = ("Pv", "Pd", "Dv", "Dd")


def open_knots(n_elem: int, p: int) -> np.ndarray:
    """p-open uniform knot vector on [0, 1] with n_elem elements (Section 2.3)."""
    inner = np.arange(1, n_elem) / n_elem
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def bspline_basis(knots: np.ndarray, deg: int, x) -> np.ndarray:
    """All B-splines of degree `deg` on `knots` evaluated at points x.

    Plain Cox-de Boor recursion (0/0 := 0).  Degree-0 functions are the
    indicators of [t_i, t_{i+1}) (right-continuous); the right end point of the
    domain is assigned to the last non-empty span.  Returns (len(x), m) with
    m = len(knots) - deg - 1.
    """
    x = np.atleast_1d(np.asarray(x, dtype=float))
    t = np.asarray(knots, dtype=float)
    m0 = len(t) - 1
    B = np.zeros((x.size, m0))
    for i in range(m0):
        if t[i] < t[i + 1]:
            B[:, i] = ((x >= t[i]) & (x < t[i + 1])).astype(float)
    last = max(i for i in range(m0) if t[i] < t[i + 1])
    B[x == t[-1], last] = 1.0
    for k in range(1, deg + 1):
        Bn = np.zeros((x.size, m0 - k))
        for i in range(m0 - k):
            acc = np.zeros(x.size)
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                acc += (x - t[i]) / d1 * B[:, i]
            if d2 > 0:
                acc += (t[i + k + 1] - x) / d2 * B[:, i + 1]
            Bn[:, i] = acc
        B = Bn
    return B


def open_knots_from_breaks(breaks: np.ndarray, p: int) -> np.ndarray:
    """p-open knot vector on [0, 1] whose interior knots are the given
    breakpoints, each simple (maximal regularity; Section 2.3 with a general
    knot vector Xi, Section 4.1 with one per direction)."""
    return np.concatenate([np.zeros(p + 1), np.asarray(breaks, float), np.ones(p + 1)])


class Axis:
    """The four 1D bases on one parametric axis with N elements and degree p.

    breaks: None for N uniform elements, else the N - 1 interior breakpoints
    (strictly increasing inside (0, 1)) of a non-uniform knot vector."""

    def __init__(self, n_elem: int, p: int, breaks=None):
        if p < 2:
            raise ValueError("the dual complex needs p >= 2 (Section 2.3, p > 1)")
        if n_elem < 1:
            raise ValueError("need at least one element")
        self.N = n_elem
        self.p = p
        self.breaks = None
        if breaks is None:
            self.xi = open_knots(n_elem, p)
        else:
            b = np.asarray(breaks, dtype=float)
            if b.shape != (n_elem - 1,) or not np.all(np.diff(np.concatenate([[0.0], b, [1.0]])) > 0):
                raise ValueError("breaks must be N - 1 increasing points inside (0, 1)")
            self.breaks = b
            self.xi = open_knots_from_breaks(b, p)
        self.xi1 = self.xi[1:-1]
        self.xi2 = self.xi[2:-2]
        self.n0 = n_elem + p - 2
        self.n1 = n_elem + p - 1
        self.dims = {"Pv": self.n0, "Pd": self.n1, "Dv": self.n1, "Dd": self.n0, "Pf": self.n0 + 2}

    # ---- bases ----------------------------------------------------------
    def eval(self, tag: str, x) -> np.ndarray:
        """Values of every function of basis `tag` at points x: (len(x), dim)."""
        p = self.p
        if tag == "Pv":
            return bspline_basis(self.xi, p, x)[:, 1:-1]
        if tag == "Pf":
            return bspline_basis(self.xi, p, x)
        if tag == "Pd":
            B = bspline_basis(self.xi1, p - 1, x)
            j = np.arange(B.shape[1])
            return B * (p / (self.xi1[j + p] - self.xi1[j]))
        if tag == "Dv":
            return bspline_basis(self.xi1, p - 1, x)
        if tag == "Dd":
            B = bspline_basis(self.xi2, p - 2, x)
            j = np.arange(B.shape[1])
            return B * ((p - 1) / (self.xi2[j + p - 1] - self.xi2[j]))
        raise KeyError(tag)

    # ---- quadrature -----------------------------------------------------
    def gauss(self, nq: int | None = None):
        """Gauss-Legendre points and weights, nq per element (default p+1),
        ordered element by element: arrays of length N*nq."""
        nq = self.p + 1 if nq is None else nq
        g, w = np.polynomial.legendre.leggauss(nq)
        if self.breaks is None:
            h = 1.0 / self.N
            x = np.concatenate([(e + 0.5 * (g + 1.0)) * h for e in range(self.N)])
            wt = np.concatenate([0.5 * w * h for _ in range(self.N)])
            return x, wt
        nodes = np.concatenate([[0.0], self.breaks, [1.0]])
        lo, hi = nodes[:-1], nodes[1:]
        x = np.concatenate([lo[e] + 0.5 * (g + 1.0) * (hi[e] - lo[e]) for e in range(self.N)])
        wt = np.concatenate([0.5 * w * (hi[e] - lo[e]) for e in range(self.N)])
        return x, wt

    def nodes(self) -> np.ndarray:
        """The N + 1 element boundaries."""
        if self.breaks is None:
            return np.arange(self.N + 1) / self.N
        return np.concatenate([[0.0], self.breaks, [1.0]])

    # ---- incidence matrices (Section 2.4, +-1 with Curry-Schoenberg bases) --
    def d_primal(self) -> np.ndarray:
        """n1 x n0 matrix d with Pv' = Pd d: d[c, c] = +1, d[c+1, c] = -1."""
        d = np.zeros((self.n1, self.n0))
        for c in range(self.n0):
            d[c, c] = 1.0
            d[c + 1, c] = -1.0
        return d

    def d_full(self) -> np.ndarray:
        """n1 x (n0+2) matrix with Pf' = Pd d_full: the derivative of the full
        primal basis, d_full[k, k+1] = +1, d_full[k, k] = -1 (it equals d on
        the interior columns)."""
        d = np.zeros((self.n1, self.n0 + 2))
        for k in range(self.n1):
            d[k, k] = -1.0
            d[k, k + 1] = 1.0
        return d

    def d_dual(self) -> np.ndarray:
        """n0 x n1 matrix d~ with Dv' = Dd d~: d~[j-1, j] = +1, d~[j, j] = -1."""
        d = np.zeros((self.n0, self.n1))
        for j in range(self.n1):
            if j >= 1:
                d[j - 1, j] = 1.0
            if j < self.n0:
                d[j, j] = -1.0
        return d

    # ---- 1D pairing matrices (Section 4.1) -------------------------------
    def G_hat(self) -> np.ndarray:
        """G^ = int Dd^T Pv: dual S_{p-2}(Xi'') rows, primal S_p(Xi) columns."""
        x, w = self.gauss()
        return self.eval("Dd", x).T @ (w[:, None] * self.eval("Pv", x))

    def M_hat(self) -> np.ndarray:
        """M^ = int Dv^T Pd: dual S_{p-1}(Xi') rows, primal S_{p-1}(Xi') columns."""
        x, w = self.gauss()
        return self.eval("Dv", x).T @ (w[:, None] * self.eval("Pd", x))

    def gram(self, tag: str) -> np.ndarray:
        """Symmetric 1D mass (Gram) matrix of one basis (identity-map masses)."""
        x, w = self.gauss()
        B = self.eval(tag, x)
        return B.T @ (w[:, None] * B)


def cardinal_bspline(deg: int, x) -> np.ndarray:
    """Centred cardinal B-spline of degree `deg` (support [-(deg+1)/2, (deg+1)/2]),
    by the truncated-power closed form
    M(x) = 1/deg! * sum_k (-1)^k C(deg+1, k) (x + (deg+1)/2 - k)_+^deg.
    Used only to pin the interior rows of G^ and M^."""
    from math import comb, factorial
    x = np.asarray(x, dtype=float)
    n = deg + 1
    s = np.zeros_like(x)
    for k in range(n + 1):
        u = x + n / 2.0 - k
        s += (-1) ** k * comb(n, k) * np.where(u > 0, u, 0.0) ** deg
    return s / factorial(deg)
