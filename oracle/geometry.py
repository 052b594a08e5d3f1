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
    """kind 'identity' or 'sine': F(x) = x + a sin(pi x) sin(pi y) sin(pi z) (1,1,1)."""

    def __init__(self, kind: str = "identity", amplitude: float = 0.0):
        if kind not in ("identity", "sine"):
            raise ValueError(kind)
        self.kind = kind
        self.a = float(amplitude) if kind == "sine" else 0.0

    def F(self, xh: np.ndarray) -> np.ndarray:
        xh = np.asarray(xh, dtype=float)
        if self.kind == "identity":
            return xh.copy()
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
