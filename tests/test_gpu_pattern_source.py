"""The second source form: a dense time-independent pattern P in the dual
2-form space times a sampled time series g, s(t) = g(t) P, against the
oracle's leapfrog driven by the same s(t) (Section 3.4: the source enters the
e update as K1^{-1}(M~ D~^1 h - s(t_{n+1/2}))), on the tiled, tiled-dense and
mixed-precision paths; graph replays equal eager steps; one pattern per batch
member; the calls it refuses."""

import numpy as np
import pytest

import workloads as W
from _helpers import make_pair, rel, relmax, to_dev, to_host

pytestmark = pytest.mark.gpu

T0, DTS, NS = 0.005, 0.01, 21  # samples at T0 + k DTS


def _series(seed):
    k = np.arange(NS)
    return np.sin(3.0 * (T0 + k * DTS) + seed) * np.exp(-((k - 8.0) / 6.0) ** 2)


def _g(series):
    """Linear interpolation of the samples, zero outside their span (the
    reading stated for the library's pattern source)."""
    def g(t):
        u = (t - T0) / DTS
        if u < 0.0 or u > NS - 1:
            return 0.0
        k = min(int(u), NS - 2)
        f = u - k
        return series[k] + f * (series[k + 1] - series[k])
    return g


def _pattern(n, seed):
    return W.random_vector(n, seed, 61) * 0.5


@pytest.mark.parametrize("plan", ["tiled", "tiled-dense", "mixed"])
def test_pattern_source_matches_oracle(plan):
    import paper_2302_04979_amd as K
    print(f"\n[case] pattern source, plan {plan}", flush=True)
    p, N, dt, nsteps, t_start = 2, 5, 0.01, 16, 0.02
    S, G = make_pair(p, N, deformed=True)
    if plan == "mixed":
        G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED)
        G.set_materials(eps=W.eps_elements(N, 0))
    elif plan == "tiled-dense":
        G.set_plan(K.PLAN_TILED_DENSE)
    else:
        G.set_plan(K.PLAN_TILED)
    P = _pattern(S.n_e, 1)
    ser = _series(0.3)
    src = G.source_pattern(P, ser, T0, DTS)
    g = _g(ser)
    e0 = W.random_vector(S.n_e, 2, 62) * 0.1
    h0 = W.random_vector(S.n_h, 2, 63) * 0.1
    E, H = to_dev(e0), to_dev(h0)
    G.step(E, H, dt, nsteps=nsteps, J=src, t_start=t_start)
    e, h = S.step(e0, h0, dt, nsteps=nsteps, t0=t_start, source=lambda t: g(t) * P)[:2]
    # the source must have acted: the run differs from the source-free one
    e_free = S.step(e0, h0, dt, nsteps=nsteps, t0=t_start)[0]
    assert rel(e, e_free) > 1e-3
    Eh, Hh = to_host(E), to_host(H)
    assert relmax(Eh, e) < 1e-12 and relmax(Hh, h) < 1e-12
    assert np.abs(Eh - e).max() < 1e-12 * np.abs(e).max()


def test_pattern_source_graph_replays_equal_eager_steps():
    import torch
    p, N, dt, nsteps = 2, 4, 0.01, 6
    S, G = make_pair(p, N, deformed=True)
    src = G.source_pattern(_pattern(S.n_e, 3), _series(1.1), T0, DTS)
    e0 = to_dev(W.random_vector(S.n_e, 4, 64))
    h0 = to_dev(W.random_vector(S.n_h, 4, 65))
    # eager steps in the graph's chunks: the source time of the second chunk
    # is nsteps dt plus the step's offset, as the device clock forms it
    E, H = e0.clone(), h0.clone()
    G.step(E, H, dt, nsteps=nsteps, J=src, t_start=0.0)
    G.step(E, H, dt, nsteps=nsteps, J=src, t_start=nsteps * dt)
    Eg, Hg = e0.clone(), h0.clone()
    gr = G.graph(Eg, Hg, dt, nsteps, J=src)
    G.set_time(0.0)
    gr.launch()
    torch.cuda.synchronize()
    gr.launch()  # the device clock has moved by nsteps dt
    torch.cuda.synchronize()
    gr.close()
    assert torch.equal(Eg, E) and torch.equal(Hg, H)


def test_one_pattern_per_member():
    import paper_2302_04979_amd as K
    p, N, dt, nsteps = 2, 4, 0.01, 8
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, max_batch=2)
    G.set_materials(eps=W.eps_elements(N, 0))
    pats = [_pattern(G.n_e, 10 + k) for k in range(2)]
    ser = _series(0.7)
    both = G.source_pattern(np.stack(pats), ser, T0, DTS)
    e0 = [W.random_vector(G.n_e, 5, k) * 0.1 for k in range(2)]
    h0 = [W.random_vector(G.n_h, 6, k) * 0.1 for k in range(2)]
    E, H = to_dev(np.concatenate(e0)), to_dev(np.concatenate(h0))
    G.step(E, H, dt, nsteps=nsteps, J=both, batch=2)
    for k in range(2):
        one = G.source_pattern(pats[k], ser, T0, DTS)
        Ek, Hk = to_dev(e0[k]), to_dev(h0[k])
        G.step(Ek, Hk, dt, nsteps=nsteps, J=one)
        assert np.array_equal(to_host(E)[k * G.n_e:(k + 1) * G.n_e], to_host(Ek))
        assert np.array_equal(to_host(H)[k * G.n_h:(k + 1) * G.n_h], to_host(Hk))


def test_pattern_source_refusals():
    import torch
    import paper_2302_04979_amd as K
    G = K.Space(2, 4, max_batch=2)
    P = _pattern(G.n_e, 7)
    with pytest.raises(K.KMXError) as ex:
        G.source_pattern(P, _series(0.0)[:1], T0, DTS)
    assert ex.value.status == 1
    with pytest.raises(K.KMXError) as ex:
        G.source_pattern(np.stack([P, P, P]), _series(0.0), T0, DTS)
    assert ex.value.status == 1
    with pytest.raises(K.KMXError) as ex:
        G.source_pattern(P, _series(0.0), T0, 0.0)
    assert ex.value.status == 1
    src = G.source_pattern(P, _series(0.0), T0, DTS)
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.set_plan(K.PLAN_SEPARABLE)
    with pytest.raises(K.KMXError) as ex:
        G.step(E, H, 0.01, nsteps=1, J=src, batch=2)
    assert ex.value.status == 7
    G.set_plan(K.PLAN_AUTO)
    G.step(E, H, 0.01, nsteps=3, J=src, t_start=T0, batch=2)  # the automatic plan takes the tiled one
    assert float(torch.linalg.norm(E)) > 0
    pr = G.probes(W.probes(2, seed=8))
    data = torch.zeros(3 * 6, dtype=torch.float64, device="cuda")
    grad = torch.zeros(4 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KMXError) as ex:
        G.adjoint(pr, src, data, 0.01, 3, 1, grad)
    assert ex.value.status == 7
