"""Per-direction degrees, knot vectors and element counts on the device
(Section 4.1: per-direction factors of eqs. (4.2)/(4.3), eqs. (4.4)-(4.5)
solves; Section 3.4 masses over per-direction Gauss rules) against the
oracle's TensorScheme on the same seeded inputs: curls bit for bit, mass
applies, pairing applies and solves (dense inverses on the matrix cores and
banded LU), and leapfrog runs with and without b/d tracking; batch members
equal single runs; a full-size anisotropic graded step; the calls it
refuses."""
import numpy as np
import pytest

import workloads as W
from _helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def _breaks(cfg):
    return tuple(W.graded_breaks(cfg["n"][a], cfg["ratio"][a]) for a in range(3))


def _pair(cfg, seed=3, max_batch=1, deformed=True, solver="dense"):
    import paper_2302_04979_amd as K
    from oracle.geometry import Map
    from oracle.tensor import TensorScheme
    eps = W.eps_elements_aniso(cfg["n"], seed)
    mu = W.eps_elements_aniso(cfg["n"], seed + 1, lo=1.0, hi=2.0, purpose="mu")
    geo = Map("sine", W.DEFORMED_AMPLITUDE) if deformed else None
    S = TensorScheme(cfg["p"], cfg["n"], _breaks(cfg), geo, eps=eps, mu=mu)
    G = K.TSpace(cfg["p"], cfg["n"], _breaks(cfg), map_kind=1 if deformed else 0,
                 amplitude=W.DEFORMED_AMPLITUDE if deformed else 0.0, max_batch=max_batch)
    G.set_materials(eps=eps, mu=mu)
    G.set_solver(solver == "dense")
    assert (G.n_e, G.n_h) == (S.n_e, S.n_h)
    return S, G


CASES = [
    W.ANISO_SMALL,
    {"p": (2, 4, 3), "n": (9, 2, 5), "ratio": (0.75, 1.5, 1.0)},
    {"p": (4, 3, 2), "n": (1, 7, 4), "ratio": (1.0, 1.2, 1.4)},
]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("solver", ["dense", "banded"])
@pytest.mark.parametrize("k", range(len(CASES)))
def test_operators_match_oracle(k, solver):
    import torch
    cfg = CASES[k]
    print(f"\n[case] per-direction operators {cfg} {solver}", flush=True)
    S, G = _pair(cfg, solver=solver)
    e = W.random_vector(S.n_e, k, 1)
    h = W.random_vector(S.n_h, k, 2)
    # curls: the same index differences, bit for bit
    y = torch.zeros(S.n_h, dtype=torch.float64, device="cuda")
    G.op_curl(True, to_dev(e), y)
    assert np.array_equal(to_host(y), S.curl_primal(e))
    z = torch.zeros(S.n_e, dtype=torch.float64, device="cuda")
    G.op_curl(False, to_dev(h), z)
    assert np.array_equal(to_host(z), S.curl_dual(h))
    # mass applies (sum factorisation, other summation order)
    for which, x in (("B", h), ("D", e)):
        out = torch.zeros(x.size, dtype=torch.float64, device="cuda")
        G.op_mass(which, to_dev(x), out)
        ref = S.mass_apply(which, x)
        assert np.abs(to_host(out) - ref).max() < 1e-13 * np.abs(ref).max(), which
    # pairing applies and solves, both blocks, K^{-1} and K^{-T}
    for which, x in (("K1", e), ("K1t", h)):
        out = torch.zeros(x.size, dtype=torch.float64, device="cuda")
        G.op_pairing(which, to_dev(x), out)
        ref = S.kron_apply(which, x)
        assert np.abs(to_host(out) - ref).max() < 1e-13 * np.abs(ref).max(), which
        for tr in (False, True):
            G.op_solve(which, to_dev(x), out, transpose=tr)
            ref = S.kron_solve(which, x, transpose=tr)
            assert np.abs(to_host(out) - ref).max() < 1e-11 * np.abs(ref).max(), (which, tr)


@pytest.mark.parametrize("solver", ["dense", "banded"])
@pytest.mark.parametrize("k", range(len(CASES)))
def test_leapfrog_matches_oracle(k, solver):
    import paper_2302_04979_amd as K
    cfg = CASES[k]
    print(f"\n[case] per-direction leapfrog {cfg} {solver}", flush=True)
    S, G = _pair(cfg, seed=10 + k, solver=solver)
    e0 = W.random_vector(S.n_e, 20 + k, 1)
    h0 = W.random_vector(S.n_h, 20 + k, 2)
    d0 = W.random_vector(S.n_e, 20 + k, 3)
    b0 = W.random_vector(S.n_h, 20 + k, 4)
    dt, n = 2e-3, 6
    E, H = to_dev(e0), to_dev(h0)
    G.step(E, H, dt, nsteps=n)
    e, h = S.step(e0, h0, dt, nsteps=n)[:2]
    assert _rel(to_host(E), e) < 1e-12 and _rel(to_host(H), h) < 1e-12
    assert np.abs(to_host(E) - e).max() < 1e-11 * np.abs(e).max()
    # tracking d and b
    E2, H2 = to_dev(np.concatenate([e0, d0])), to_dev(np.concatenate([h0, b0]))
    G.step(E2, H2, dt, nsteps=n, flags=K.TRACK_DB)
    e, h, d, b, _ = S.step(e0, h0, dt, nsteps=n, d=d0, b=b0)
    Eh, Hh = to_host(E2), to_host(H2)
    assert _rel(Eh[:S.n_e], e) < 1e-12 and _rel(Hh[:S.n_h], h) < 1e-12
    assert _rel(Eh[S.n_e:], d) < 1e-12 and _rel(Hh[S.n_h:], b) < 1e-12


def test_energy_of_the_device_run_is_conserved():
    """The oracle's invariant 1/2 (d.K1 e + b.K~1 h - dt (K~1 h).(D^1 e))
    evaluated on the device's tracked states stays constant."""
    import paper_2302_04979_amd as K
    S, G = _pair(W.ANISO_SMALL, seed=40)
    d0 = W.random_vector(S.n_e, 41, 1)
    e0 = S.kron_solve("K1", S.mass_apply("D", d0))
    dt = 0.5 * S.cfl(iters=300, tol=1e-8)
    z = np.zeros(S.n_h)
    E, H = to_dev(np.concatenate([e0, d0])), to_dev(np.concatenate([z, z]))
    E0 = S.energy(e0, z, d0, z, dt)[0]
    for _ in range(5):
        G.step(E, H, dt, nsteps=20, flags=K.TRACK_DB)
        Eh, Hh = to_host(E), to_host(H)
        En = S.energy(Eh[:S.n_e], Hh[:S.n_h], Eh[S.n_e:], Hh[S.n_h:], dt)[0]
        assert abs(En / E0 - 1) < 1e-12


def test_batch_members_equal_single_runs():
    S, G = _pair(W.ANISO_SMALL, seed=50, max_batch=3)
    e = [W.random_vector(S.n_e, 51, m) for m in range(3)]
    h = [W.random_vector(S.n_h, 52, m) for m in range(3)]
    E, H = to_dev(np.concatenate(e)), to_dev(np.concatenate(h))
    G.step(E, H, 1e-3, nsteps=4, batch=3)
    for m in range(3):
        Em, Hm = to_dev(e[m]), to_dev(h[m])
        G.step(Em, Hm, 1e-3, nsteps=4)
        assert np.array_equal(to_host(E)[m * S.n_e:(m + 1) * S.n_e], to_host(Em))
        assert np.array_equal(to_host(H)[m * S.n_h:(m + 1) * S.n_h], to_host(Hm))


def test_full_size_graded_anisotropic_step_matches_oracle():
    """The measured workload (degrees (3, 3, 2), 64 x 48 x 32 graded
    elements, deformed cube, eps and mu per element): one step against the
    oracle, every entry, with the dense (default) and the banded solves."""
    cfg = W.ANISO_FULL
    print(f"\n[case] per-direction full size {cfg}", flush=True)
    S, G = _pair(cfg, seed=60)
    e0 = W.random_vector(S.n_e, 61, 1)
    h0 = W.random_vector(S.n_h, 61, 2)
    e, h = S.step(e0, h0, 1e-3, nsteps=1)[:2]
    for dense in (True, False):
        G.set_solver(dense)
        E, H = to_dev(e0), to_dev(h0)
        G.step(E, H, 1e-3, nsteps=1)
        assert np.abs(to_host(E) - e).max() < 1e-12 * np.abs(e).max(), dense
        assert np.abs(to_host(H) - h).max() < 1e-12 * np.abs(h).max(), dense


def test_refusals():
    import torch
    import paper_2302_04979_amd as K
    G = K.TSpace((2, 3, 2), (3, 3, 3), max_batch=1)
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KMXError) as ex:
        G.step(E, H, 0.01, nsteps=1, batch=2)
    assert ex.value.status == 1
    with pytest.raises(K.KMXError) as ex:
        G.set_materials(eps=-np.ones(27))
    assert ex.value.status == 3
    with pytest.raises(K.KMXError) as ex:
        K.TSpace((2, 3, 2), (3, 3, 3), map_kind=1, amplitude=5.0)  # folds the cube: det DF < 0
    assert ex.value.status == 2
    assert K.load_library().kmx_tspace_set_solver(G._h, 2) == 1
