"""Pins of the oracle's univariate spline layer (Section 2.3, Section 4.1)."""
import os

import numpy as np
import pytest

from oracle.splines import Axis, bspline_basis, cardinal_bspline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cardinal_rows.txt")


def _off_knot_points(N, n=40, seed=0):
    x = np.random.default_rng(seed).uniform(0, 1, n)
    # keep away from knots so finite differences see one polynomial piece
    frac = (x * N) % 1.0
    return x[(frac > 0.05) & (frac < 0.95)]


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("N", [1, 3, 8])
def test_partition_of_unity_and_dims(p, N):
    ax = Axis(N, p)
    x = np.linspace(0, 1, 57)
    assert np.abs(bspline_basis(ax.xi, p, x).sum(1) - 1).max() < 1e-14
    assert np.abs(bspline_basis(ax.xi1, p - 1, x).sum(1) - 1).max() < 1e-14
    assert ax.eval("Pv", x).shape[1] == N + p - 2
    assert ax.eval("Pd", x).shape[1] == N + p - 1
    assert ax.eval("Dv", x).shape[1] == N + p - 1
    assert ax.eval("Dd", x).shape[1] == N + p - 2
    # the homogeneous primal space vanishes on the boundary
    assert np.abs(ax.eval("Pv", np.array([0.0, 1.0]))).max() == 0.0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_curry_schoenberg_unit_integral(p):
    ax = Axis(6, p)
    x, w = ax.gauss()
    for tag in ("Pd", "Dd"):
        integ = w @ ax.eval(tag, x)
        assert np.abs(integ - 1).max() < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4])
def test_incidence_matrices_are_derivatives(p):
    """Pv' = Pd d and Dv' = Dd d~ (derivative identities, checked by central
    differences), d and d~ pure +-1 and d~ = -d^T."""
    N = 5
    ax = Axis(N, p)
    x = _off_knot_points(N)
    h = 1e-6
    d, dt = ax.d_primal(), ax.d_dual()
    for vtag, dtag, D in (("Pv", "Pd", d), ("Dv", "Dd", dt)):
        fd = (ax.eval(vtag, x + h) - ax.eval(vtag, x - h)) / (2 * h)
        assert np.abs(fd - ax.eval(dtag, x) @ D).max() < 1e-7
    assert set(np.unique(d)) <= {-1.0, 0.0, 1.0}
    assert np.array_equal(dt, -d.T)


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("N", [2, 5, 16])
def test_1d_integration_by_parts(p, N):
    """M^ d = d G^ (1D integration by parts with homogeneous primal functions)."""
    ax = Axis(N, p)
    assert np.abs(ax.M_hat() @ ax.d_primal() - ax.d_primal() @ ax.G_hat()).max() < 1e-14


def _golden_rows():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t) for t in line.split()]
            rows[v[0]] = np.array(v[2:], dtype=float) / v[1]
    return rows


@pytest.mark.parametrize("p", [2, 3, 4])
def test_interior_rows_are_cardinal_splines(p):
    ref = _golden_rows()[p]
    # the closed form of the centred cardinal B-spline gives the same samples
    assert np.abs(cardinal_bspline(2 * p - 1, np.arange(-p + 1, p)) - ref).max() < 1e-15
    ax = Axis(20, p)
    G, M = ax.G_hat(), ax.M_hat()
    for A in (G, M):
        i = A.shape[0] // 2
        row = A[i, i - p + 1:i + p]
        assert np.abs(row - ref).max() < 1e-14
        # nothing outside the band of half-width p-1
        assert np.abs(A[i, :i - p + 1]).max(initial=0) == 0 and np.abs(A[i, i + p:]).max(initial=0) == 0


@pytest.mark.parametrize("p,cmax", [(2, 3.2), (3, 8.5), (4, 23.0)])
def test_pairing_conditioning_is_mesh_independent(p, cmax):
    """G^ and M^ stay well conditioned under refinement (inf-sup stable pairing)."""
    c = [np.linalg.cond(Axis(N, p).G_hat()) for N in (8, 16, 32)]
    assert max(c) < cmax and abs(c[-1] - c[0]) / c[0] < 0.05
