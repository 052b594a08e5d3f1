"""Maps of the parametric unit cube and the 2-form metric factor (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

Section 2.3: the physical domain is the image of (0,1)^3 under a map F, and the
discrete forms are pullbacks of parametric ones.  For 2-forms (vector proxies)
the pullback is the contravariant Piola map u = DF u^ / det DF, so the weighted
L^2 product of two 2-forms becomes, in parametric coordinates,

    (u, v)_{L^2_{1/gamma}} = int u^ . G v^ dx^,   G = DF^T DF / (gamma det DF).

The paper only refers to the pullbacks; this factor is derived here.  For a
1-form the pullback is covariant (E = DF^{-T} E^), used for probes and for the
initial projection; it gives the 1-form factor of the mass matrices of scheme
1 (Section 3.3),

    (E, E')_{L^2_gamma} = int E^ . G1 E'^ dx^,   G1 = gamma det DF (DF^T DF)^{-1}.
"""
from __future__ import annotations

import numpy as np


class Map:
    """kind 'identity', 'sine': F(x) = x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1),
    or 'annulus': the quarter coaxial cable 1 < x^2 + y^2 < 2, 0 < z < 1 of
    Section 5, as a degree-2 NURBS map (radial x^, angular y^, axial z^):
    F = (r(x^) cos t, r(x^) sin t, z^) with r = 1 + (sqrt 2 - 1) x^ and the
    angle t(y^) of the rational quadratic quarter circle."""

    def __init__(self, kind: str = "identity", amplitude: float = 0.0):
        if kind not in ("identity", "sine", "annulus"):
            raise ValueError(kind)
        self.kind = kind
        self.a = float(amplitude) if kind == "sine" else 0.0

    @staticmethod
    def _quarter_circle(v):
        """Point and derivative of the quarter unit circle as a rational
        quadratic Bezier curve: control points (1,0), (1,1), (0,1), weights
        1, 1/sqrt 2, 1 (homogeneous coordinates, then projected)."""
        w1 = np.sqrt(0.5)
        Pw = np.array([[1.0, 0.0, 1.0], [w1, w1, w1], [0.0, 1.0, 1.0]])  # (w x, w y, w)
        B = np.stack([(1 - v) ** 2, 2 * v * (1 - v), v ** 2], axis=-1)
        dB = np.stack([-2 * (1 - v), 2 - 4 * v, 2 * v], axis=-1)
        H, dH = B @ Pw, dB @ Pw
        pt = H[..., :2] / H[..., 2:3]
        dpt = (dH[..., :2] * H[..., 2:3] - H[..., :2] * dH[..., 2:3]) / H[..., 2:3] ** 2
        return pt, dpt

    def F(self, xh: np.ndarray) -> np.ndarray:
        xh = np.asarray(xh, dtype=float)
        if self.kind == "identity":
            return xh.copy()
        if self.kind == "annulus":
            pt, _ = self._quarter_circle(xh[..., 1])
            r = 1.0 + (np.sqrt(2.0) - 1.0) * xh[..., 0]
            return np.stack([r * pt[..., 0], r * pt[..., 1], xh[..., 2]], axis=-1)
        s = np.sin(np.pi * xh[..., 0]) * np.sin(np.pi * xh[..., 1]) * np.sin(np.pi * xh[..., 2])
        return xh + self.a * s[..., None]

    def DF(self, xh: np.ndarray) -> np.ndarray:
        """Jacobian matrices, shape (..., 3, 3), DF[i, j] = dF_i / dx^_j."""
        xh = np.asarray(xh, dtype=float)
        J = np.zeros(xh.shape[:-1] + (3, 3))
        for i in range(3):
            J[..., i, i] = 1.0
        if self.kind == "identity":
            return J
        if self.kind == "annulus":
            pt, dpt = self._quarter_circle(xh[..., 1])
            r, dr = 1.0 + (np.sqrt(2.0) - 1.0) * xh[..., 0], np.sqrt(2.0) - 1.0
            J[..., 0, 0], J[..., 1, 0] = dr * pt[..., 0], dr * pt[..., 1]
            J[..., 0, 1], J[..., 1, 1] = r * dpt[..., 0], r * dpt[..., 1]
            return J
        x, y, z = xh[..., 0], xh[..., 1], xh[..., 2]
        pi = np.pi
        grad = np.stack([pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * z),
                         pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * z),
                         pi * np.sin(pi * x) * np.sin(pi * y) * np.cos(pi * z)], axis=-1)
        for i in range(3):
            for j in range(3):
                J[..., i, j] += self.a * grad[..., j]
        return J


def metric_2form(DF: np.ndarray) -> np.ndarray:
    """DF^T DF / det DF at each point (gamma = 1), shape (..., 3, 3)."""
    det = np.linalg.det(DF)
    if np.any(det <= 0):
        raise ValueError("map is not orientation preserving (det DF <= 0)")
    return np.einsum("...ki,...kj->...ij", DF, DF) / det[..., None, None]


def metric_1form(DF: np.ndarray) -> np.ndarray:
    """det DF (DF^T DF)^{-1} at each point (gamma = 1), shape (..., 3, 3)."""
    det = np.linalg.det(DF)
    if np.any(det <= 0):
        raise ValueError("map is not orientation preserving (det DF <= 0)")
    return det[..., None, None] * np.linalg.inv(np.einsum("...ki,...kj->...ij", DF, DF))
