"""Tiled plan variants: dense FP64 mode-product solves (matrix cores) and the
four-wave mass kernel, against the FP64 oracle and the default tiled plan."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p,N", [(2, 7), (3, 6), (3, 9), (4, 5)])
def test_dense_plan_matches_oracle(p, N):
    """Deformed cube, random eps, two members with their own dipoles: the
    dense-solve plan matches the oracle (1e-12) and the banded plan (1e-13)."""
    import paper_2302_04979_amd as K
    print(f"\n[case] dense plan p={p} N={N}", flush=True)
    S, G = make_pair(p, N, deformed=True, max_batch=2)
    dt, nsteps = 0.01, 15
    dip = W.dipoles(2, seed=9, dt=dt)
    dip["t0"] = np.array([6 * dt, 9 * dt])
    dip["sigma"] = np.array([3 * dt, 3 * dt])
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=np.arange(2))
    E0 = W.random_vector(2 * S.n_e, 71) * 0.1
    H0 = W.random_vector(2 * S.n_h, 72) * 0.1
    out = {}
    for plan in (K.PLAN_TILED_DENSE, K.PLAN_TILED, K.PLAN_TILED_W4):
        G.set_plan(plan)
        E, H = to_dev(E0), to_dev(H0)
        G.step(E, H, dt, nsteps=nsteps, J=J, t_start=0.02, batch=2)
        out[plan] = (to_host(E), to_host(H))
    Ed, Hd = out[K.PLAN_TILED_DENSE]
    for k in range(2):
        s = S.dipole_source(dip["pos"][k], dip["moment"][k])
        g = lambda t, k=k, s=s: dip["amp"][k] * math.exp(-(t - dip["t0"][k]) ** 2 / (2 * dip["sigma"][k] ** 2)) * s
        e, h, _, _, _ = S.step(E0[k * S.n_e:(k + 1) * S.n_e], H0[k * S.n_h:(k + 1) * S.n_h], dt, nsteps=nsteps,
                               t0=0.02, source=g)
        assert relmax(Ed[k * S.n_e:(k + 1) * S.n_e], e) < 1e-12
        assert relmax(Hd[k * S.n_h:(k + 1) * S.n_h], h) < 1e-12
    assert relmax(Ed, out[K.PLAN_TILED][0]) < 1e-13 and relmax(Hd, out[K.PLAN_TILED][1]) < 1e-13
    # the four-wave mass kernel variant performs the same operations: same bits
    assert np.array_equal(out[K.PLAN_TILED_W4][0], out[K.PLAN_TILED][0])
    assert np.array_equal(out[K.PLAN_TILED_W4][1], out[K.PLAN_TILED][1])


def test_dense_plan_tracking_and_energy():
    """b/d tracking and the invariant under the dense-solve plan (64^3 lines of
    65-66 entries are covered by the p=3, N=20 case: several 16-row tiles and
    a ragged tail)."""
    import torch
    import paper_2302_04979_amd as K
    from oracle.scheme import Scheme
    p, N, dt, nsteps = 3, 20, 2e-3, 6
    S, G = make_pair(p, N, deformed=True)
    G.set_plan(K.PLAN_TILED_DENSE)
    e0, h0 = W.random_vector(S.n_e, 81), W.random_vector(S.n_h, 82)
    d0, b0 = W.random_vector(S.n_e, 83), W.random_vector(S.n_h, 84)
    E, H = to_dev(np.concatenate([e0, d0])), to_dev(np.concatenate([h0, b0]))
    en = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    G.step(E, H, dt, nsteps=nsteps, flags=K.TRACK_DB, energy=en)
    e, h, d, b, en_ref = S.step(e0, h0, dt, nsteps=nsteps, d=d0, b=b0, energy_every=1)
    Eg, Hg = to_host(E), to_host(H)
    assert relmax(Eg[:S.n_e], e) < 1e-12 and relmax(Eg[S.n_e:], d) < 1e-12
    assert relmax(Hg[:S.n_h], h) < 1e-12 and relmax(Hg[S.n_h:], b) < 1e-12
    assert np.abs(to_host(en) - np.array(en_ref)).max() < 1e-12 * abs(en_ref[0])


def test_dense_plan_full_size_one_step():
    """p=3, 64^3 (lines of 65 and 66 entries, the metric workload's shape):
    one step of the dense-solve plan equals the banded plan to 1e-13."""
    import paper_2302_04979_amd as K
    p, N, dt = 3, 64, 1e-3
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements(N, 0))
    E0 = W.random_vector(G.n_e, 91)
    H0 = W.random_vector(G.n_h, 92)
    res = []
    for plan in (K.PLAN_TILED, K.PLAN_TILED_DENSE):
        G.set_plan(plan)
        E, H = to_dev(E0), to_dev(H0)
        G.step(E, H, dt, nsteps=1)
        res.append((to_host(E), to_host(H)))
    assert relmax(res[1][0] - E0, res[0][0] - E0) < 1e-12 and relmax(res[1][1] - H0, res[0][1] - H0) < 1e-12
