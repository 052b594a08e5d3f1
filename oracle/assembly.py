"""Level 0 of the oracle: the plain definitions, assembled explicitly (FP64).

Test infrastructure only (see ``oracle/__init__``).  Meant for tiny meshes
(N <= 4..6): every matrix is dense.

* Pairing matrices K1 (rows: dual 2-forms X~^2, columns: primal 1-forms
  X^1_{h,0}) and K~1 (rows: primal 2-forms X^2_{h,0}, columns: dual 1-forms
  X~^1), entries = integral of the wedge product of two basis forms (Section
  2.4).  In parametric coordinates the wedge of a 2-form and a 1-form is the dot
  product of their vector proxies, so each entry is a 3D integral of a product
  of tensor-product splines, computed here by 3D Gauss quadrature of the 3D
  basis functions - not from the Kronecker factorisation (4.2)/(4.3), which the
  tests check against this.
* Mass matrices M^2_{1/mu} (primal 2-forms) and M~^2_{1/eps} (dual 2-forms),
  Section 3.4: entries int w^_i . G w^_j with the 2-form metric factor G; and
  for scheme 1 (Section 3.3) M^1_eps (primal 1-forms) and M~^1_mu (dual
  1-forms) with the 1-form factor G1 and the material as a factor.
* Incidence matrices D^1 (primal curl, e -> b) and D~^1 (dual curl,
  h -> d-space) as explicit +-1 matrices (Section 2.4).
"""
from __future__ import annotations

import numpy as np

from .spaces import comp_shape, comp_tags, space_size
from .splines import Axis


def quad_points_3d(axis: Axis):
    """All 3D Gauss points (x fastest) with their weights: (Q^3, 3), (Q^3,)."""
    x, w = axis.gauss()
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    WZ, WY, WX = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts, (WX * WY * WZ).ravel()


def basis_3d(axis: Axis, space: str, c: int, pts: np.ndarray) -> np.ndarray:
    """Values of every basis function of component c at 3D points: (npts, ndofs_c).
    Column index = (iz * n_y + iy) * n_x + ix."""
    tx, ty, tz = comp_tags(space, c)
    Bx = axis.eval(tx, pts[:, 0])
    By = axis.eval(ty, pts[:, 1])
    Bz = axis.eval(tz, pts[:, 2])
    npts = pts.shape[0]
    out = np.empty((npts, Bz.shape[1], By.shape[1], Bx.shape[1]))
    for q in range(npts):  # tensor-product basis function = product of 1D values
        out[q] = Bz[q][:, None, None] * By[q][None, :, None] * Bx[q][None, None, :]
    return out.reshape(npts, -1)


def _offsets(axis: Axis, space: str):
    o = [0]
    for c in range(3):
        o.append(o[-1] + int(np.prod(comp_shape(axis, space, c))))
    return o


def pairing_K1(axis: Axis) -> np.ndarray:
    """K1: eta~^T K1 omega = int eta~ ^ omega, eta~ in X~^2 (rows), omega in X^1_{h,0}."""
    pts, w = quad_points_3d(axis)
    n = space_size(axis, "D")
    K = np.zeros((n, space_size(axis, "E")))
    od, oe = _offsets(axis, "D"), _offsets(axis, "E")
    for c in range(3):
        Pd = basis_3d(axis, "D", c, pts)
        Pe = basis_3d(axis, "E", c, pts)
        K[od[c]:od[c + 1], oe[c]:oe[c + 1]] = Pd.T @ (w[:, None] * Pe)
    return K


def pairing_K1t(axis: Axis) -> np.ndarray:
    """K~1: rows index primal 2-forms X^2_{h,0}, columns dual 1-forms X~^1."""
    pts, w = quad_points_3d(axis)
    K = np.zeros((space_size(axis, "B"), space_size(axis, "H")))
    ob, oh = _offsets(axis, "B"), _offsets(axis, "H")
    for c in range(3):
        Pb = basis_3d(axis, "B", c, pts)
        Ph = basis_3d(axis, "H", c, pts)
        K[ob[c]:ob[c + 1], oh[c]:oh[c + 1]] = Pb.T @ (w[:, None] * Ph)
    return K


def mass_2form(axis: Axis, space: str, G: np.ndarray, inv_gamma_elem: np.ndarray | None):
    """Mass matrix of the 2-form space `space` ('B' or 'D') by an element loop.

    G: metric factor DF^T DF / det DF at the 3D Gauss points, shape (Q^3, 3, 3)
    in the order of ``quad_points_3d``; inv_gamma_elem: (N, N, N) [ez, ey, ex]
    or None for gamma = 1.
    """
    N, nq = axis.N, axis.p + 1
    pts, w = quad_points_3d(axis)
    Q = N * nq
    n = space_size(axis, space)
    o = _offsets(axis, space)
    M = np.zeros((n, n))
    qidx = np.arange(Q ** 3).reshape(Q, Q, Q)  # [qz, qy, qx]
    for ez in range(N):
        for ey in range(N):
            for ex in range(N):
                q = qidx[ez * nq:(ez + 1) * nq, ey * nq:(ey + 1) * nq,
                         ex * nq:(ex + 1) * nq].ravel()
                g = 1.0 if inv_gamma_elem is None else inv_gamma_elem[ez, ey, ex]
                Phi = [basis_3d(axis, space, c, pts[q]) for c in range(3)]
                for ci in range(3):
                    for cj in range(3):
                        Wij = w[q] * G[q, ci, cj] * g
                        M[o[ci]:o[ci + 1], o[cj]:o[cj + 1]] += Phi[ci].T @ (Wij[:, None] * Phi[cj])
    return M


def mass_1form(axis: Axis, space: str, G1: np.ndarray, gamma_elem: np.ndarray | None):
    """Mass matrix of the 1-form space `space` ('E' with gamma = eps, 'H' with
    gamma = mu) by the same element loop: G1 = det DF (DF^T DF)^{-1} at the
    Gauss points, the material multiplying (not dividing) the integrand."""
    return mass_2form(axis, space, G1, gamma_elem)


def curl_matrix(axis: Axis, primal: bool) -> np.ndarray:
    """D^1 (primal=True, X^1_{h,0} -> X^2_{h,0}) or D~^1 (X~^1 -> X~^2).

    Component c of the curl is d_{c+1} u_{c+2} - d_{c+2} u_{c+1} (indices mod 3),
    where d_a applies the 1D incidence matrix (d or d~) along axis a.
    """
    src, dst = ("E", "B") if primal else ("H", "D")
    d1 = axis.d_primal() if primal else axis.d_dual()
    os_, od = _offsets(axis, src), _offsets(axis, dst)
    D = np.zeros((od[3], os_[3]))
    for c in range(3):
        sh_dst = comp_shape(axis, dst, c)
        for sign, a, s in ((+1.0, (c + 1) % 3, (c + 2) % 3), (-1.0, (c + 2) % 3, (c + 1) % 3)):
            sh_src = comp_shape(axis, src, s)
            # along axis a the 1D matrix d1 maps the source index to the destination index
            for iz in range(sh_dst[0]):
                for iy in range(sh_dst[1]):
                    for ix in range(sh_dst[2]):
                        row = od[c] + (iz * sh_dst[1] + iy) * sh_dst[2] + ix
                        dst_idx = [ix, iy, iz]
                        for k in range(d1.shape[1]):
                            coef = d1[dst_idx[a], k]
                            if coef == 0.0:
                                continue
                            src_idx = list(dst_idx)
                            src_idx[a] = k
                            jx, jy, jz = src_idx
                            col = os_[s] + (jz * sh_src[1] + jy) * sh_src[2] + jx
                            D[row, col] += sign * coef
    return D


def div_matrix(axis: Axis, primal: bool) -> np.ndarray:
    """D^2 (X^2_{h,0} -> X^3) or D~^2 (X~^2 -> X~^3): sum over a of d_a u_a."""
    src = "B" if primal else "D"
    d1 = axis.d_primal() if primal else axis.d_dual()
    m = d1.shape[0]
    os_ = _offsets(axis, src)
    D = np.zeros((m ** 3, os_[3]))
    for a in range(3):
        sh = comp_shape(axis, src, a)
        for iz in range(m):
            for iy in range(m):
                for ix in range(m):
                    row = (iz * m + iy) * m + ix
                    idx = [ix, iy, iz]
                    for k in range(d1.shape[1]):
                        coef = d1[idx[a], k]
                        if coef == 0.0:
                            continue
                        j = list(idx)
                        j[a] = k
                        D[row, os_[a] + (j[2] * sh[1] + j[1]) * sh[2] + j[0]] += coef
    return D


# ---------------------------------------------------------------------------
# whole primal spaces (non-homogeneous boundary data, Section 3.5)
# ---------------------------------------------------------------------------
def pairing_K1_full(axis: Axis) -> np.ndarray:
    """The pairing of X~^2 (rows) with the whole X^1_h (columns), by 3D
    quadrature: [(K1)_0 (K1)_b] up to the ordering of the columns."""
    pts, w = quad_points_3d(axis)
    K = np.zeros((space_size(axis, "D"), space_size(axis, "Ef")))
    od, oe = _offsets(axis, "D"), _offsets(axis, "Ef")
    for c in range(3):
        Pd = basis_3d(axis, "D", c, pts)
        Pe = basis_3d(axis, "Ef", c, pts)
        K[od[c]:od[c + 1], oe[c]:oe[c + 1]] = Pd.T @ (w[:, None] * Pe)
    return K


def mass_2form_trial_full(axis: Axis, G: np.ndarray, inv_mu_elem: np.ndarray | None = None):
    """M^2_{1/mu} with test functions in X^2_{h,0} (rows) and trial functions
    in the whole X^2_h (columns), by the element loop of ``mass_2form``."""
    N, nq = axis.N, axis.p + 1
    pts, w = quad_points_3d(axis)
    Q = N * nq
    ot, of = _offsets(axis, "B"), _offsets(axis, "Bf")
    M = np.zeros((ot[3], of[3]))
    qidx = np.arange(Q ** 3).reshape(Q, Q, Q)
    for ez in range(N):
        for ey in range(N):
            for ex in range(N):
                q = qidx[ez * nq:(ez + 1) * nq, ey * nq:(ey + 1) * nq, ex * nq:(ex + 1) * nq].ravel()
                g = 1.0 if inv_mu_elem is None else inv_mu_elem[ez, ey, ex]
                Pt = [basis_3d(axis, "B", c, pts[q]) for c in range(3)]
                Pf = [basis_3d(axis, "Bf", c, pts[q]) for c in range(3)]
                for ci in range(3):
                    for cj in range(3):
                        Wij = w[q] * G[q, ci, cj] * g
                        M[ot[ci]:ot[ci + 1], of[cj]:of[cj + 1]] += Pt[ci].T @ (Wij[:, None] * Pf[cj])
    return M


def curl_matrix_full(axis: Axis) -> np.ndarray:
    """D^1 from the whole X^1_h to the whole X^2_h: the +-1 matrix with the
    full primal incidence d_full (Pf' = Pd d_full) along each axis."""
    d1 = axis.d_full()
    os_, od = _offsets(axis, "Ef"), _offsets(axis, "Bf")
    D = np.zeros((od[3], os_[3]))
    for c in range(3):
        sh_dst = comp_shape(axis, "Bf", c)
        for sign, a, s in ((+1.0, (c + 1) % 3, (c + 2) % 3), (-1.0, (c + 2) % 3, (c + 1) % 3)):
            sh_src = comp_shape(axis, "Ef", s)
            for iz in range(sh_dst[0]):
                for iy in range(sh_dst[1]):
                    for ix in range(sh_dst[2]):
                        row = od[c] + (iz * sh_dst[1] + iy) * sh_dst[2] + ix
                        dst_idx = [ix, iy, iz]
                        for k in range(d1.shape[1]):
                            coef = d1[dst_idx[a], k]
                            if coef == 0.0:
                                continue
                            src_idx = list(dst_idx)
                            src_idx[a] = k
                            jx, jy, jz = src_idx
                            D[row, os_[s] + (jz * sh_src[1] + jy) * sh_src[2] + jx] += sign * coef
    return D

