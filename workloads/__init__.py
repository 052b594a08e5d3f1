"""Seeded synthetic inputs for the spline Maxwell leapfrog workloads.

This module is shared by the FP64 oracle and by the HIP path.  It only draws
random numbers and evaluates the analytic *input* fields (cavity modes, the
deformed-cube parameters, dipole and probe placements); it holds none of the
discretisation's arithmetic (no bases, quadrature, Hodge or pairing matrices).

Workloads follow the numerical experiments of the paper (Section 5: the unit
cube cavity with its first curl-curl eigenfunction, whose angular frequency is
sqrt(2)*pi) and extend them to a deformed cube with random per-element
permittivity, point-dipole sources and point probes.

Random streams: ``numpy.random.default_rng([seed, purpose_id])``, one stream
per purpose, base seed 0.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

PURPOSE = {
    "eps": 1,
    "modes": 2,
    "dipoles": 3,
    "probes": 4,
    "fd": 5,
    "field": 6,
    "eps_true": 7,
    "mu": 8,
}

#: amplitude of the deformed-cube map x -> x + a*sin(pi x)sin(pi y)sin(pi z)
DEFORMED_AMPLITUDE = 0.08


def rng(seed: int, purpose: str) -> np.random.Generator:
    """Independent generator for one purpose of one seeded workload."""
    return np.random.default_rng([int(seed), PURPOSE[purpose]])


def eps_elements(n_elem: int, seed: int = 0, lo: float = 1.0, hi: float = 4.0,
                 purpose: str = "eps") -> np.ndarray:
    """Per-element permittivity, uniform in [lo, hi], shape (N, N, N) indexed
    [ez, ey, ex] (x fastest when flattened)."""
    return rng(seed, purpose).uniform(lo, hi, size=(n_elem, n_elem, n_elem))


def eps_elements_aniso(n_elem, seed: int = 0, lo: float = 1.0, hi: float = 4.0,
                       purpose: str = "eps") -> np.ndarray:
    """Per-element permittivity on an (Nx, Ny, Nz) mesh, uniform in [lo, hi],
    shape (Nz, Ny, Nx) indexed [ez, ey, ex]."""
    nx, ny, nz = (int(v) for v in n_elem)
    return rng(seed, purpose).uniform(lo, hi, size=(nz, ny, nx))


def graded_breaks(n_elem: int, ratio: float):
    """Interior breakpoints of a geometrically graded mesh of [0, 1]: element
    sizes proportional to ratio^k, k = 0..N-1 (ratio 1: uniform).  None for one
    element."""
    if n_elem < 2:
        return None
    w = np.asarray(ratio, float) ** np.arange(n_elem)
    return np.cumsum(w)[:-1] / w.sum()


# The anisotropic workload of the per-direction path: degrees (p_x, p_y, p_z),
# elements (N_x, N_y, N_z) and the grading ratio of each direction (the finest
# direction first, as the remark after eq. (4.5) recommends).
ANISO_SMALL = {"p": (3, 2, 4), "n": (6, 5, 3), "ratio": (1.3, 1.0, 0.8)}
ANISO_FULL = {"p": (3, 3, 2), "n": (64, 48, 32), "ratio": (1.02, 1.0, 0.97)}


def random_vector(n: int, seed: int = 0, salt: int = 0) -> np.ndarray:
    """Standard-normal coefficient vector (operator tests)."""
    g = np.random.default_rng([int(seed), PURPOSE["field"], int(salt)])
    return g.standard_normal(n)


# --------------------------------------------------------------------------
# PEC cavity modes of the unit cube
# --------------------------------------------------------------------------
def _mode_indices(count: int):
    """The `count` lowest (l, m, n) with at most one zero index, ordered by
    l^2+m^2+n^2 and then lexicographically."""
    cand = []
    top = int(math.ceil(math.sqrt(count))) + 3
    for lmn in itertools.product(range(top + 1), repeat=3):
        if sum(1 for v in lmn if v == 0) > 1:
            continue
        cand.append((lmn[0] ** 2 + lmn[1] ** 2 + lmn[2] ** 2, lmn))
    cand.sort()
    return [lmn for _, lmn in cand[:count]]


def cavity_modes(seed: int = 0, count: int = 10):
    """Random smooth initial field: `count` PEC cavity modes.

    Each mode is (l, m, n, a, amp): E = amp * (a_x cos(l pi x) sin(m pi y) sin(n pi z),
    a_y sin(l pi x) cos(m pi y) sin(n pi z), a_z sin(l pi x) sin(m pi y) cos(n pi z))
    with a a unit vector orthogonal to (l, m, n) (divergence free) and amp ~ N(0, 1).
    When one index is zero only the component along that axis survives, so a
    is that unit axis vector.
    """
    g = rng(seed, "modes")
    modes = []
    for lmn in _mode_indices(count):
        k = np.array(lmn, dtype=float)
        if (k == 0).any():
            a = (k == 0).astype(float)
            _ = g.standard_normal(3)  # keep the stream layout uniform
        else:
            v = g.standard_normal(3)
            v -= k * (v @ k) / (k @ k)
            a = v / np.linalg.norm(v)
        amp = g.standard_normal()
        modes.append((int(lmn[0]), int(lmn[1]), int(lmn[2]), a, float(amp)))
    return modes


def mode_110():
    """The lowest cavity mode E = (0, 0, sin(pi x) sin(pi y)), omega = sqrt(2) pi."""
    return [(1, 1, 0, np.array([0.0, 0.0, 1.0]), 1.0)]


def eval_modes(modes, xyz: np.ndarray) -> np.ndarray:
    """Electric field of a sum of cavity modes at physical points xyz (n, 3)."""
    xyz = np.asarray(xyz, dtype=float)
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    out = np.zeros(xyz.shape, dtype=float)
    pi = math.pi
    for l, m, n, a, amp in modes:
        sx, cx = np.sin(l * pi * x), np.cos(l * pi * x)
        sy, cy = np.sin(m * pi * y), np.cos(m * pi * y)
        sz, cz = np.sin(n * pi * z), np.cos(n * pi * z)
        out[..., 0] += amp * a[0] * cx * sy * sz
        out[..., 1] += amp * a[1] * sx * cy * sz
        out[..., 2] += amp * a[2] * sx * sy * cz
    return out


def curl_modes(modes, xyz: np.ndarray) -> np.ndarray:
    """curl E of a sum of cavity modes at physical points (for the exact H)."""
    xyz = np.asarray(xyz, dtype=float)
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    out = np.zeros(xyz.shape, dtype=float)
    pi = math.pi
    for l, m, n, a, amp in modes:
        kx, ky, kz = l * pi, m * pi, n * pi
        sx, cx = np.sin(kx * x), np.cos(kx * x)
        sy, cy = np.sin(ky * y), np.cos(ky * y)
        sz, cz = np.sin(kz * z), np.cos(kz * z)
        # E = (A cx sy sz, B sx cy sz, C sx sy cz)
        A, B, C = amp * a[0], amp * a[1], amp * a[2]
        dEz_dy = C * sx * ky * cy * cz
        dEy_dz = B * sx * cy * kz * cz
        dEx_dz = A * cx * sy * kz * cz
        dEz_dx = C * kx * cx * sy * cz
        dEy_dx = B * kx * cx * cy * sz
        dEx_dy = A * cx * ky * cy * sz
        out[..., 0] += dEz_dy - dEy_dz
        out[..., 1] += dEx_dz - dEz_dx
        out[..., 2] += dEy_dx - dEx_dy
    return out


def mode_omega(modes) -> np.ndarray:
    """Angular frequency pi*sqrt(l^2+m^2+n^2) of each mode (eps = mu = 1)."""
    return np.array([math.pi * math.sqrt(l * l + m * m + n * n) for l, m, n, _, _ in modes])


# --------------------------------------------------------------------------
# Point dipoles and probes
# --------------------------------------------------------------------------
def dipoles(count: int, seed: int = 0, dt: float = 1.0, sigma_steps: float = 20.0,
            t0_sigmas: float = 5.0, margin: float = 0.0):
    """`count` point dipoles: parametric positions U(margin, 1-margin)^3,
    unit moments uniform on the sphere, Gaussian-in-time profile
    amp*exp(-(t-t0)^2/(2 sigma^2)) with sigma = sigma_steps*dt, t0 = t0_sigmas*sigma.

    Returns dict of arrays: pos (n,3), moment (n,3), t0 (n,), sigma (n,), amp (n,).
    """
    g = rng(seed, "dipoles")
    pos = g.uniform(margin, 1.0 - margin, size=(count, 3))
    v = g.standard_normal((count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    sigma = np.full(count, sigma_steps * dt)
    return {"pos": pos, "moment": v, "t0": t0_sigmas * sigma, "sigma": sigma,
            "amp": np.ones(count)}


def probes(count: int, seed: int = 0, margin: float = 0.0) -> np.ndarray:
    """`count` probe points in parametric coordinates, U(margin, 1-margin)^3."""
    return rng(seed, "probes").uniform(margin, 1.0 - margin, size=(count, 3))


# --------------------------------------------------------------------------
# Quarter of a coaxial cable: 1 < x^2 + y^2 < 2, 0 < z < 1 (Section 5), as a
# degree-2 NURBS map of the unit cube (geometry input of the curved workload)
# --------------------------------------------------------------------------
def quarter_annulus_jacobian(xh: np.ndarray):
    """Map x^ = (u, v, w) -> (rho(u) C(v), w) with rho(u) = 1 + (sqrt(2) - 1) u
    (radius from 1 to sqrt(2)) and C the quarter unit circle from (1, 0) to
    (0, 1) as a rational quadratic Bezier curve (control points (1,0), (1,1),
    (0,1), weights 1, 1/sqrt(2), 1).  Returns the mapped points (..., 3) and
    the Jacobians DF[i, j] = dF_i / dx^_j (..., 3, 3)."""
    xh = np.asarray(xh, dtype=float)
    u, v, w = xh[..., 0], xh[..., 1], xh[..., 2]
    wt = 1.0 / math.sqrt(2.0)
    b0, b1, b2 = (1 - v) ** 2, 2 * v * (1 - v) * wt, v ** 2
    db0, db1, db2 = -2 * (1 - v), 2 * wt * (1 - 2 * v), 2 * v
    den = b0 + b1 + b2
    dden = db0 + db1 + db2
    cx, cy = (b0 + b1) / den, (b1 + b2) / den
    dcx = ((db0 + db1) * den - (b0 + b1) * dden) / den ** 2
    dcy = ((db1 + db2) * den - (b1 + b2) * dden) / den ** 2
    rho = 1.0 + (math.sqrt(2.0) - 1.0) * u
    drho = math.sqrt(2.0) - 1.0
    F = np.stack([rho * cx, rho * cy, w], axis=-1)
    J = np.zeros(xh.shape[:-1] + (3, 3))
    J[..., 0, 0], J[..., 0, 1] = drho * cx, rho * dcx
    J[..., 1, 0], J[..., 1, 1] = drho * cy, rho * dcy
    J[..., 2, 2] = 1.0
    return F, J


# --------------------------------------------------------------------------
# TEM standing wave of the quarter coaxial cable (Section 5.1.2)
# --------------------------------------------------------------------------
def tem_coax_E(xyz: np.ndarray, t: float = 0.0) -> np.ndarray:
    """E = (1/r) sin(pi z) cos(pi t) r^ (eps = mu = 1): the TEM mode between
    the cylinders r = 1, sqrt 2 with the shorting planes z = 0, 1; its
    tangential trace vanishes on those four faces and not on the planes y = 0
    and x = 0 (the Dirichlet data there)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r2 = x * x + y * y
    f = np.sin(np.pi * z) * np.cos(np.pi * t) / r2
    return np.stack([f * x, f * y, np.zeros_like(z)], axis=-1)


def tem_coax_H(xyz: np.ndarray, t: float = 0.0) -> np.ndarray:
    """H = -(1/r) cos(pi z) sin(pi t) phi^, the magnetic field of the same mode."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r2 = x * x + y * y
    f = -np.cos(np.pi * z) * np.sin(np.pi * t) / r2
    return np.stack([-f * y, f * x, np.zeros_like(z)], axis=-1)


def face_gauss_points(p: int, n_elem: int) -> np.ndarray:
    """Parametric Gauss points of the six faces of the unit cube (p + 1
    Gauss-Legendre points per element and axis), shape (6, Q, Q, 3): face
    f = 2 a + s is x^_a = s, indexed [i_v][i_u] over its two other axes u < v
    (u fastest)."""
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    x = ((np.arange(n_elem)[:, None] + 0.5 * (g[None, :] + 1.0)) / n_elem).ravel()
    Q = x.size
    out = np.zeros((6, Q, Q, 3))
    for a in range(3):
        u, v = [k for k in range(3) if k != a]
        for s in range(2):
            f = out[2 * a + s]
            f[..., a] = float(s)
            f[..., u] = x[None, :]
            f[..., v] = x[:, None]
    return out

