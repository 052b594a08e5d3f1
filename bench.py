#!/usr/bin/env python3
"""Benchmark of the scheme-2 spline Maxwell leapfrog on one MI355X.

Workload: degree p=3, 64^3 elements, the deformed cube
x -> x + 0.08 sin(pi x) sin(pi y) sin(pi z) on every component, per-element
eps ~ U[1,4] (seed 0), mu = 1, initial E = sum of the 10 lowest cavity modes
with N(0,1) amplitudes (seed 0), H = 0, dt = 0.5 CFL, FP64.

A timed step is one pass of the whole hot path: fused curl + Hodge mass apply
M^2_{1/mu} D^1 e, Kronecker solve with K~1, h update; fused dual curl + mass
apply M~^2_{1/eps} D~^1 h, Kronecker solve with K1, e update; tracking of b
and d; the leapfrog energy invariant.  Inputs are resident in HBM before the
timed region.  value = DOF-updates/s = (dim e + dim h) * steps / seconds.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per leapfrog step at p=3, 64^3 (mixed vs FP64) + adjoint grad time"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def mass_flops(p, N, space):
    """Floating-point operations of one fused curl + mass apply as the kernel
    performs them (FMA = 2): per 4^3-element tile, the x/y contractions of the
    coefficient window and their transposes, and per Gauss point the z
    contraction, the z integral, and the metric applied as a rank-2 update of
    the identity (grad s, 1/det DF by a refined reciprocal, the two dot
    products and the update: about 20 FMA-equivalents); times the tiles."""
    T, nq = 4, p + 1
    Q = T * nq
    K = {"Pv": p + 1, "Pd": p, "Dv": p, "Dd": p - 1}
    along, across = {"B": ("Pv", "Pd"), "D": ("Dv", "Dd"), "E": ("Pd", "Pv"), "H": ("Dd", "Dv")}[space]
    fma_xy = 0
    kz_sum = 0
    for c in range(3):
        tags = [along if a == c else across for a in range(3)]
        kx, ky, kz = (K[t] for t in tags)
        wx, wy, wz = (T + k - 1 for k in (kx, ky, kz))
        fma_xy += 2 * (wz * Q * wx * ky + wz * Q * Q * kx)  # forward and transposed
        kz_sum += kz
    per_qp = 2 * kz_sum + 20
    tiles = ((N + T - 1) // T) ** 3
    return 2.0 * tiles * (fma_xy + per_qp * Q ** 3)


def measured_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/hbm_traffic.json, FETCH_SIZE + WRITE_SIZE scaled by the copy
    calibration), or None when that file is missing or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        src = os.path.join(ROOT, "paper_2302_04979_amd", "csrc", t["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
                return None
        return t["kernels"][kernel_key]["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(p, N, steps, eps):
    """The FP64 oracle on the host cores: `steps` leapfrog steps of the same
    workload from a seeded random state (the step cost does not depend on the
    data), timed after its one-off set-up."""
    import numpy as np
    import workloads as W
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    S = Scheme(p, N, Map("sine", W.DEFORMED_AMPLITUDE), eps=eps)
    S.metric()
    e = W.random_vector(S.n_e, 0, 41)
    h = W.random_vector(S.n_h, 0, 42)
    S.step(e, h, 1e-3, nsteps=1)  # warm caches and BLAS threads
    t0 = time.perf_counter()
    S.step(e, h, 1e-3, nsteps=steps)
    dt = time.perf_counter() - t0
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            S.step(e, h, 1e-3, nsteps=2)
            single = (S.n_e + S.n_h) * 2 / (time.perf_counter() - t1)
    except Exception:
        pass
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": (S.n_e + S.n_h) * steps / dt, "unit": "DOF-updates/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle leapfrog steps of the same p={p}, {N}^3 deformed-cube workload "
                      f"from a seeded random state ({dt:.1f} s of CPU work, set-up excluded)",
            "value_single_thread": single, "host_cpu": model, "nproc": os.cpu_count()}


def adjoint_timing(K, W, torch):
    """Wall time of one loss + gradient evaluation (forward with checkpoints,
    recomputation, reverse sweep) on the differentiation workload."""
    import numpy as np
    p, N, nsteps = 3, 32, 500
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=np.full(N ** 3, 2.0))
    dt = 0.5 * G.cfl(max_iter=200, tol=1e-6)
    dip = W.dipoles(1, seed=0, dt=dt, margin=0.2)
    probes = W.probes(64, seed=0)
    zero = torch.zeros(nsteps * 192, dtype=torch.float64, device="cuda")
    prob = K.ProbeMisfitProblem(G, dip, probes, zero, dt, nsteps, checkpoint_every=50)
    data = prob.observe(W.eps_elements(N, 0, purpose="eps_true")).reshape(-1).clone()
    prob = K.ProbeMisfitProblem(G, dip, probes, data, dt, nsteps, checkpoint_every=50)
    eps0 = np.full(N ** 3, 2.0)
    prob.loss_and_grad(eps0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        prob.loss_and_grad(eps0)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _state(K, W, torch, G, N):
    """e^0, d^0 from the 10 seeded cavity modes, h = b = 0, staggered to -dt/2."""
    xq = G.quad_points()
    Eq = W.eval_modes(W.cavity_modes(0), xq)
    del xq
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device="cuda")
    G.project_E(Eq, E[:G.n_e])
    G.project_D(Eq, E[G.n_e:], tol=1e-13)
    return E, H


def _rel(a, b):
    return float(torch_norm(a - b) / torch_norm(b))


def torch_norm(x):
    return x.double().norm()


def mixed_vs_fp64(K, W, torch, p, N, steps, eps, dt=None, E0=None, H0=None, G64=None):
    """The same run (deformed cube, eps, tracking + energy) with FP64 and with
    mixed-precision solves from the same state: ms per step of each and the
    relative difference of every field and of the energy after `steps`."""
    dev = "cuda"
    if G64 is None:
        G64 = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
        G64.set_materials(eps=eps)
    Gm = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED)
    Gm.set_materials(eps=eps)
    if E0 is None:
        E0, H0 = _state(K, W, torch, G64, N)
        dt = 0.5 * G64.cfl(max_iter=300, tol=1e-6)
        G64.init_stagger(E0, H0, dt, flags=K.TRACK_DB)
    stream = torch.cuda.current_stream()
    res = {}
    for name, G in (("fp64", G64), ("mixed", Gm)):
        E, H = E0.clone(), H0.clone()
        en = torch.zeros(steps, dtype=torch.float64, device=dev)
        G.step(E, H, dt, nsteps=2, flags=K.TRACK_DB, energy=en)  # warm-up on a scratch copy
        E, H = E0.clone(), H0.clone()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        G.step(E, H, dt, nsteps=steps, flags=K.TRACK_DB, energy=en)
        ev1.record(stream)
        torch.cuda.synchronize()
        res[name] = (ev0.elapsed_time(ev1) / steps, E, H, en)
    ne, nh = G64.n_e, G64.n_h
    E64, H64, en64 = res["fp64"][1], res["fp64"][2], res["fp64"][3]
    Em, Hm, enm = res["mixed"][1], res["mixed"][2], res["mixed"][3]
    dofs = ne + nh
    return {"workload": f"p={p}, {N}^3 deformed cube (a=0.08), eps~U[1,4], 10 cavity modes, dt=0.5 CFL, "
                        f"b/d tracking + energy, {steps} steps",
            "ms_per_step_fp64": res["fp64"][0], "ms_per_step_mixed": res["mixed"][0],
            "value_fp64": dofs / (res["fp64"][0] * 1e-3), "value_mixed": dofs / (res["mixed"][0] * 1e-3),
            "speedup_mixed_over_fp64": res["fp64"][0] / res["mixed"][0],
            "refinement_corrections": 2,
            "rel_err_vs_fp64": {"e": _rel(Em[:ne], E64[:ne]), "d": _rel(Em[ne:], E64[ne:]),
                                "h": _rel(Hm[:nh], H64[:nh]), "b": _rel(Hm[nh:], H64[nh:]),
                                "energy": float((enm[-1] - en64[-1]).abs() / en64[-1].abs())},
            "energy_rel_drift_mixed": float(((enm / enm[0]) - 1).abs().max())}


def scheme1_timing(K, W, torch, G, e0, dt2, ms_step2, steps=20, tol=1e-12):
    """The first scheme (1-form mass solves by PCG) on the same space and
    initial e as the headline run: its CFL next to scheme 2's, ms per step at
    dt = 0.5 CFL with the solves to |r| <= tol |y|, CG iterations per solve, the
    1-form mass kernel's launch time and FLOP rate, and the per-step and
    per-simulated-time ratios to scheme 2."""
    p, N = G.p, G.N
    cfl1 = G.cfl_scheme1(max_iter=300, tol=1e-6, cg_tol=1e-10)
    dt1 = 0.5 * cfl1
    e = e0.clone()
    h = torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
    G.half_step_scheme1("H", e, h, 0.5 * dt1, tol=tol)
    G.step_scheme1(e, h, dt1, 3, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = G.step_scheme1(e, h, dt1, steps, tol=tol)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / steps
    # the same steps captured as one HIP graph with fixed iteration counts (the
    # tolerance-driven counts, rounded up, plus one)
    it_e, it_h = int(math.ceil(its[0] / steps)) + 1, int(math.ceil(its[1] / steps)) + 1
    gsteps = 10
    gr = G.graph_scheme1(e, h, dt1, gsteps, it_e, it_h)
    gr.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr.launch()
    torch.cuda.synchronize()
    ms1_graph = (time.perf_counter() - t0) * 1e3 / gsteps
    gr.close()
    G.profile_begin(capacity=4096)
    G.step_scheme1(e, h, dt1, 4, tol=tol)
    prof = G.profile_end()
    m = prof["mass_1form"]
    avg = m[0] / m[1] * 1e-3
    flops = 0.5 * (mass_flops(p, N, "E") + mass_flops(p, N, "H"))
    share = {k: round(v[0] / sum(x[0] for x in prof.values()), 3) for k, v in prof.items() if v[1]}
    cfl2 = 2.0 * dt2
    te, th = measured_traffic("mass_E"), measured_traffic("mass_H")
    return {"workload": f"first scheme (1-form mass solves), same space, e^0 and eps as the headline, mu = 1, "
                        f"dt = 0.5 CFL1, PCG to |r| <= {tol:g} |y|, warm-started",
            "ms_per_step": ms1, "steps": steps, "dt": dt1,
            "graph_fixed_iterations": {"iters_e": it_e, "iters_h": it_h, "ms_per_step": ms1_graph,
                                       "per_step_ratio_vs_scheme2": ms1_graph / ms_step2},
            "cg_iters_per_solve": {"e": its[0] / steps, "h": its[1] / steps},
            "cfl": cfl1, "cfl_scheme2": cfl2, "cfl_ratio": cfl1 / cfl2,
            "per_step_ratio_vs_scheme2": ms1 / ms_step2,
            "per_simulated_time_ratio_vs_scheme2": (ms1 / dt1) / (ms_step2 / dt2),
            "mass_1form_kernel": {"avg_launch_us": round(avg * 1e6, 2),
                                  "tflops": round(flops / avg / 1e12, 2),
                                  "frac_fp64_peak": round(flops / avg / 1e12 / FP64_PEAK_TFLOPS, 4),
                                  "traffic": None if te is None or th is None else 0.5 * (te + th)},
            "time_share": share}


def schemes_vs_degree(K, W, torch, N=32, degrees=(2, 3, 4), steps=10, tol=1e-12):
    """Both schemes on the deformed cube (eps ~ U[1,4], mu = 1) at N^3 for
    p = 2, 3, 4: the CFL limits of each (power iteration on the device), the
    time per step of each (scheme 2: the plain step under the tuner's plan;
    scheme 1: PCG to tol), and the ratios per step and per unit of simulated
    time (Section 5.2: the CFL of the mass-solve scheme decays more slowly in
    p, its steps cost far more)."""
    out = {"workload": f"deformed cube (a=0.08), {N}^3, eps~U[1,4], mu=1, random e^0, h^0 = 0; "
                       f"scheme 1 PCG to |r| <= {tol:g} |y|", "p": {}}
    for p in degrees:
        G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
        G.set_materials(eps=W.eps_elements(N, 0))
        cfl2 = G.cfl(max_iter=300, tol=1e-6)
        cfl1 = G.cfl_scheme1(max_iter=300, tol=1e-6, cg_tol=1e-10)
        e0 = torch.tensor(W.random_vector(G.n_e, 0, 51), dtype=torch.float64, device="cuda")
        G.tune(1, 0.5 * cfl2, probe_steps=5)
        e, h = e0.clone(), torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
        G.init_stagger(e, h, 0.5 * cfl2)
        G.step(e, h, 0.5 * cfl2, nsteps=5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.step(e, h, 0.5 * cfl2, nsteps=10 * steps)
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t0) * 1e3 / (10 * steps)
        e, h = e0.clone(), torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
        G.half_step_scheme1("H", e, h, 0.25 * cfl1, tol=tol)
        G.step_scheme1(e, h, 0.5 * cfl1, 2, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = G.step_scheme1(e, h, 0.5 * cfl1, steps, tol=tol)
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t0) * 1e3 / steps
        out["p"][str(p)] = {"cfl_scheme2": cfl2, "cfl_scheme1": cfl1, "cfl_ratio": cfl1 / cfl2,
                            "ms_per_step_scheme2": ms2, "ms_per_step_scheme1": ms1,
                            "cg_iters_per_solve": {"e": its[0] / steps, "h": its[1] / steps},
                            "per_step_ratio": ms1 / ms2, "per_simulated_time_ratio": (ms1 / cfl1) / (ms2 / cfl2)}
        G.close()
    return out


def convergence_both_schemes(K, W, torch, p=3, Ns=(4, 8, 16), T=0.5, dt=1e-3, n_probe=2000):
    """Section 5.1, Fig. 2 on the device: the cube cavity's first mode
    E = (0, 0, sin(pi x) sin(pi y)) cos(sqrt(2) pi t), eps = mu = 1, from each
    scheme's own projection of E(0) (scheme 2: K1^{-1} l; scheme 1: the L^2
    projection), h = 0, leapfrog with dt = 1e-3 to T = 0.5 (time error ~1e-6,
    below the spatial one); relative RMS error of E(T) at seeded probe points
    and the observed rate between consecutive meshes."""
    import numpy as np
    modes = W.mode_110()
    omega = float(W.mode_omega(modes)[0])
    pos = np.random.default_rng([0, 71]).uniform(0.02, 0.98, size=(n_probe, 3))
    exact = W.eval_modes(modes, pos) * np.cos(omega * T)
    nsteps = int(round(T / dt))
    out = {"workload": f"cube cavity, first mode, p={p}, eps=mu=1, dt={dt:g}, T={T:g}, "
                       f"RMS error of E(T) at {n_probe} seeded points", "N": list(Ns),
           "scheme2": [], "scheme1": []}
    for N in Ns:
        G = K.Space(p, N)
        Eq = W.eval_modes(modes, G.quad_points())
        pr = G.probes(pos)
        val = torch.zeros(3 * n_probe, dtype=torch.float64, device="cuda")
        for name in ("scheme2", "scheme1"):
            e = torch.zeros(G.n_e, dtype=torch.float64, device="cuda")
            h = torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
            if name == "scheme2":
                G.project_E(Eq, e)
                G.init_stagger(e, h, dt)
                G.step(e, h, dt, nsteps=nsteps)
            else:
                G.project_E1(Eq, e, tol=1e-13)
                G.half_step_scheme1("H", e, h, 0.5 * dt, tol=1e-13)
                G.step_scheme1(e, h, dt, nsteps, tol=1e-13)
            G.probe_eval(pr, e, val)
            got = val.cpu().numpy().reshape(n_probe, 3)
            out[name].append(float(np.sqrt(np.sum((got - exact) ** 2) / np.sum(exact ** 2))))
        pr.close()
        G.close()
    for name in ("scheme2", "scheme1"):
        err = out[name]
        out[name + "_rates"] = [float(np.log2(err[i] / err[i + 1])) for i in range(len(err) - 1)]
    return out


def _coax_space(K, W, p, N):
    import numpy as np
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    x = (np.arange(N)[:, None] + 0.5 * (g[None, :] + 1.0)) / N
    sh = (N, N, N, p + 1, p + 1, p + 1)
    X = np.broadcast_to(x[None, None, :, None, None, :], sh)
    Y = np.broadcast_to(x[None, :, None, None, :, None], sh)
    Z = np.broadcast_to(x[:, None, None, :, None, None], sh)
    _, DF = W.quarter_annulus_jacobian(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    return K.Space(p, N, map_kind=2, dF_qp=DF.reshape(-1))


def coax_schemes(K, W, torch, p=4, N=16, steps=20, tol=1e-12, random_eps=False):
    """Both schemes on the quarter coax, p = 4 and 16^3 elements (the paper's
    finest coax mesh, where it quotes its per-step and total-time ratios,
    Section 6): CFL limits, ms per step (scheme 2: plain step under the tuner's
    plan; scheme 1: PCG to tol) and the ratios; eps = mu = 1, or eps ~ U[1,4]
    per element.  With uniform material the coax's 1-form masses are exact
    Kronecker products (orthogonal product map), which the separable
    preconditioner inverts in one iteration."""
    G = _coax_space(K, W, p, N)
    if random_eps:
        G.set_materials(eps=W.eps_elements(N, 0))
    cfl2 = G.cfl(max_iter=300, tol=1e-6)
    cfl1 = G.cfl_scheme1(max_iter=300, tol=1e-6, cg_tol=1e-10)
    G.tune(1, 0.5 * cfl2, probe_steps=5)
    e0 = torch.tensor(W.random_vector(G.n_e, 0, 81), dtype=torch.float64, device="cuda")
    e, h = e0.clone(), torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
    G.init_stagger(e, h, 0.5 * cfl2)
    G.step(e, h, 0.5 * cfl2, nsteps=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.step(e, h, 0.5 * cfl2, nsteps=20 * steps)
    torch.cuda.synchronize()
    ms2 = (time.perf_counter() - t0) * 1e3 / (20 * steps)
    e, h = e0.clone(), torch.zeros(G.n_h, dtype=torch.float64, device="cuda")
    G.half_step_scheme1("H", e, h, 0.25 * cfl1, tol=tol)
    G.step_scheme1(e, h, 0.5 * cfl1, 2, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = G.step_scheme1(e, h, 0.5 * cfl1, steps, tol=tol)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / steps
    G.close()
    mat = "eps~U[1,4], mu=1" if random_eps else "eps=mu=1"
    return {"workload": f"quarter coax (NURBS map), p={p}, {N}^3, {mat}, random e^0; scheme 1 PCG to {tol:g}",
            "cfl_scheme2": cfl2, "cfl_scheme1": cfl1, "cfl_ratio": cfl1 / cfl2,
            "ms_per_step_scheme2": ms2, "ms_per_step_scheme1": ms1,
            "cg_iters_per_solve": {"e": its[0] / steps, "h": its[1] / steps},
            "per_step_ratio": ms1 / ms2, "per_simulated_time_ratio": (ms1 / cfl1) / (ms2 / cfl2)}


def coax_timing(K, W, torch, p=3, N=32, steps=100):
    """The curved workload: the quarter coaxial cable (Section 5) as a
    degree-2 NURBS map given by its Jacobians at the Gauss points (the metric
    factor streamed from HBM), eps ~ U[1,4], PEC walls, random e^0 with a
    consistent d^0, dt = 0.5 CFL, tracking and energy; ms per step under the
    tuner's plan and the streamed mass kernel's HBM rate."""
    import numpy as np
    G = _coax_space(K, W, p, N)
    G.set_materials(eps=W.eps_elements(N, 0))
    dev = torch.device("cuda")
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device=dev)
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device=dev)
    E[G.n_e:] = torch.tensor(W.random_vector(G.n_e, 0, 61), dtype=torch.float64, device=dev)
    y = torch.empty(G.n_e, dtype=torch.float64, device=dev)
    G.op_mass("D", E[G.n_e:].contiguous(), y)
    e = torch.empty_like(y)
    G.op_solve("K1", y, e)
    E[:G.n_e] = e
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-6)
    G.init_stagger(E, H, dt, flags=K.TRACK_DB)
    G.tune(1, dt, probe_steps=5)
    en = torch.zeros(steps, dtype=torch.float64, device=dev)
    G.step(E, H, dt, nsteps=10, flags=K.TRACK_DB, energy=en)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.step(E, H, dt, nsteps=steps, flags=K.TRACK_DB, energy=en)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    e_n = en.cpu().numpy()
    G.profile_begin(capacity=16 * 20 + 64)
    G.step(E, H, dt, nsteps=20, flags=K.TRACK_DB, energy=en[:20])
    prof = G.profile_end()
    avg = (prof["mass_B"][0] + prof["mass_D"][0]) / (prof["mass_B"][1] + prof["mass_D"][1]) * 1e-3
    bytes_mass = 8.0 * (6 * G.n_qp + N ** 3 + G.n_e + G.n_h)
    out = {"workload": f"quarter coax (1 < x^2+y^2 < 2, 0 < z < 1) as a degree-2 NURBS map, p={p}, {N}^3, "
                       "eps~U[1,4], PEC, random consistent (e, d), dt = 0.5 CFL, tracking + energy, metric streamed",
           "ms_per_step": ms, "value": (G.n_e + G.n_h) / (ms * 1e-3), "unit": "DOF-updates/s", "dt": dt,
           "plan": K.PLAN_NAMES[G.plan()[0]], "energy_rel_drift": float(np.abs(e_n / e_n[0] - 1).max()),
           "mass_kernel": {"avg_launch_us": round(avg * 1e6, 2), "algorithmic_bytes_per_launch": int(bytes_mass),
                           "GB_s": round(bytes_mass / avg / 1e9, 1),
                           "frac_hbm_peak": round(bytes_mass / avg / 1e9 / HBM_PEAK_GBS, 4)}}
    G.close()
    return out


def coax_tem_timing(K, W, torch, p=3, N=32, steps=100):
    """The quarter coax with non-homogeneous tangential data (Section 3.5):
    the TEM standing wave E = (1/r) sin(pi z) cos(pi t) r^ (Section 5.1.2),
    eps = mu = 1, its tangential trace on the planes y = 0 and x = 0 fitted
    by the library's trace fit, the lifting g(t) = cos(pi t) added at every
    step, e^0 projected with the lifting; ms per step with and without the
    lifting (the same plan) and the trace fit's set-up time."""
    import math
    G = _coax_space(K, W, p, N)
    P = W.face_gauss_points(p, N)
    F, J = W.quarter_annulus_jacobian(P)
    import numpy as np
    Eh = np.einsum("...ki,...k->...i", J, W.tem_coax_E(F, 0.0))
    t0 = time.perf_counter()
    eb = G.lift_boundary(Eh)
    G.set_lifting(eb, [1.0], [math.pi], [0.0])
    t_setup = time.perf_counter() - t0
    dev = torch.device("cuda")
    E = torch.zeros(G.n_e, dtype=torch.float64, device=dev)
    H = torch.zeros(G.n_h, dtype=torch.float64, device=dev)
    Fq, _ = W.quarter_annulus_jacobian(G.quad_points())  # map kind 2: parametric points returned
    G.project_E(W.tem_coax_E(Fq, 0.0), E)
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-6)
    G.init_stagger(E, H, dt)
    G.tune(1, dt, probe_steps=5)
    G.step(E, H, dt, nsteps=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.step(E, H, dt, nsteps=steps, t_start=10 * dt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    finite = bool(torch.isfinite(E).all() and torch.isfinite(H).all())
    G.set_lifting([], [], [], [])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.step(E, H, dt, nsteps=steps)
    torch.cuda.synchronize()
    ms0 = (time.perf_counter() - t0) * 1e3 / steps
    out = {"workload": f"quarter coax, p={p}, {N}^3, eps=mu=1, TEM data on y = 0 and x = 0 lifted, "
                       "dt = 0.5 CFL, no tracking",
           "ms_per_step_lifted": ms, "ms_per_step_without_lifting": ms0,
           "value": (G.n_e + G.n_h) / (ms * 1e-3), "unit": "DOF-updates/s", "plan": K.PLAN_NAMES[G.plan()[0]],
           "trace_fit_and_lifting_setup_s": t_setup, "fields_finite": finite}
    G.close()
    return out


def time_order_comparison(K, W, torch, G, e0, dt, steps=100):
    """Time-discretisation error of the leapfrog and of its order-4 and
    order-6 symmetric compositions on the headline space: from (e0, h = 0) to
    T = steps * dt, against the order-6 composition with dt / 4 as reference;
    the leapfrog also at dt / 3 (the order-4 step's cost).  The order-6 step is
    run at dt / 2 (its largest weight, 2.30, exceeds the leapfrog's stability
    limit at dt = 0.5 CFL).  Costs are ms per step of the plain composed step."""
    dev = torch.device("cuda")

    def run(order, sub, n):
        e = e0.clone()
        h = torch.zeros(G.n_h, dtype=torch.float64, device=dev)
        G.init_split(e, h, dt / sub, order)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.step_split(e, h, dt / sub, n * sub, order)
        torch.cuda.synchronize()
        return e, (time.perf_counter() - t0) * 1e3 / (n * sub)

    ref, _ = run(6, 4, steps)
    out = {"workload": f"headline space and e^0 (projected cavity modes, h^0 = 0), T = {steps} dt, dt = 0.5 CFL; "
                       "reference: order-6 composition with dt/4", "T": steps * dt, "errors": {}, "ms_per_step": {}}
    for name, order, sub in (("leapfrog_dt", 2, 1), ("leapfrog_dt/3", 2, 3), ("order4_dt", 4, 1),
                             ("order6_dt/2", 6, 2)):
        e, ms = run(order, sub, steps)
        out["errors"][name] = float(torch.linalg.norm(e - ref) / torch.linalg.norm(ref))
        out["ms_per_step"][name] = ms
    return out


def profile_run(K, W, torch, p, N, steps):
    """A short run for the profiler: a device copy of known size (512 MiB read,
    512 MiB written: the reference for the HBM byte counters), then `steps`
    steps of the metric workload's kernels from a seeded random state under
    each of the three tiled plans, then two steps of the first scheme, two
    steps with mixed-precision solves, and 10 steps of the batched separable
    plan (256 members, 24^3)."""
    import numpy as np
    n = 64 * 1024 * 1024  # doubles: 512 MiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements(N, 0))
    E = torch.tensor(W.random_vector(2 * G.n_e, 0, 41), dtype=torch.float64, device="cuda")
    H = torch.tensor(W.random_vector(2 * G.n_h, 0, 42), dtype=torch.float64, device="cuda")
    en = torch.zeros(steps, dtype=torch.float64, device="cuda")
    # the tiled plan, the tiled plan with the four-wave mass kernel, and the
    # tiled plan with dense solves
    for plan in (K.PLAN_TILED, K.PLAN_TILED_W4, K.PLAN_TILED_DENSE):
        G.set_plan(plan)
        G.step(E, H, 1e-3, nsteps=steps, flags=K.TRACK_DB, energy=en)
    # two steps of the first scheme (1-form mass kernels, PCG)
    G.step_scheme1(E[:G.n_e], H[:G.n_h], 1e-3, 2, tol=1e-10)
    torch.cuda.synchronize()
    del G
    # two steps with mixed-precision solves (FP32 mode products + FP64 refinement)
    Gm = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, precision=K.MIXED)
    Gm.set_materials(eps=W.eps_elements(N, 0))
    Gm.step(E, H, 1e-3, nsteps=2, flags=K.TRACK_DB, energy=en[:2])
    torch.cuda.synchronize()
    del Gm, E, H
    # the batched separable plan: p=3, 24^3, 256 members, 10 steps
    B, Nb = 256, 24
    Gb = K.Space(p, Nb, max_batch=B)
    Gb.set_plan(K.PLAN_SEPARABLE, 768)
    Eb = torch.tensor(np.tile(W.random_vector(Gb.n_e, 0, 43), B), dtype=torch.float64, device="cuda")
    Hb = torch.zeros(B * Gb.n_h, dtype=torch.float64, device="cuda")
    Gb.step(Eb, Hb, 1e-3, nsteps=10, batch=B)
    torch.cuda.synchronize()
    del Gb, Eb, Hb
    # two steps of the per-direction workload (degrees (3, 3, 2), 64 x 48 x 32 graded)
    cfg = W.ANISO_FULL
    br = tuple(W.graded_breaks(cfg["n"][a], cfg["ratio"][a]) for a in range(3))
    Ga = K.TSpace(cfg["p"], cfg["n"], br, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    Ga.set_materials(eps=W.eps_elements_aniso(cfg["n"], 60))
    Ea = torch.tensor(W.random_vector(2 * Ga.n_e, 62, 1), dtype=torch.float64, device="cuda")
    Ha = torch.tensor(W.random_vector(2 * Ga.n_h, 62, 2), dtype=torch.float64, device="cuda")
    Ga.step(Ea, Ha, 1e-4, nsteps=2, flags=K.TRACK_DB)
    torch.cuda.synchronize()
    return {"profile_run": {"copy_bytes_each_way": n * 8, "copies": 3, "steps": steps, "p": p, "N": N,
                            "mixed_steps": 2, "batched": {"members": B, "N": Nb, "steps": 10},
                            "aniso_steps": 2}}


def aniso_support(p, space, c, a):
    """Functions of component c nonzero on one element along direction a: the
    2-form space B has the degree-p value basis (p + 1) along c and the
    derivative basis (p) across; D has p along c and p - 1 across."""
    if space == "B":
        return p[a] + 1 if a == c else p[a]
    return p[a] if a == c else p[a] - 1


def aniso_window(p, space):
    """Doubles of one element's window of all three components."""
    return sum(aniso_support(p, space, c, 0) * aniso_support(p, space, c, 1) * aniso_support(p, space, c, 2)
               for c in range(3))


def aniso_flops_per_element(p, space):
    """FLOPs of the per-element mass kernel for one element: per component the
    three interpolation passes and the three integration passes (2 flops per
    multiply-add), plus 18 flops per Gauss point for u = (1/gamma) G v."""
    nq = [pa + 1 for pa in p]
    tot = 0
    for c in range(3):
        Kx, Ky, Kz = (aniso_support(p, space, c, a) for a in range(3))
        fwd = Kz * Ky * nq[0] * Kx + Kz * nq[1] * nq[0] * Ky + nq[2] * nq[1] * nq[0] * Kz
        tot += 2 * 2 * fwd
    return tot + 18 * nq[0] * nq[1] * nq[2]


def aniso_timing(K, W, torch, steps=50, reps=20):
    """Per-direction degrees, knot vectors and element counts (Section 4.1):
    degrees (3, 3, 2), 64 x 48 x 32 geometrically graded elements (size ratios
    1.02, 1, 0.97 between neighbours), the deformed cube, eps in [1, 4] and mu
    in [1, 2] per element, b/d tracking, dt = 1e-4; `steps` eager steps, then
    `reps` mass applies of each 2-form space timed alone."""
    cfg = W.ANISO_FULL
    br = tuple(W.graded_breaks(cfg["n"][a], cfg["ratio"][a]) for a in range(3))
    G = K.TSpace(cfg["p"], cfg["n"], br, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    G.set_materials(eps=W.eps_elements_aniso(cfg["n"], 60), mu=W.eps_elements_aniso(cfg["n"], 61, 1.0, 2.0, "mu"))
    dt = 1e-4
    E = torch.tensor(W.random_vector(2 * G.n_e, 62, 1), dtype=torch.float64, device="cuda")
    H = torch.tensor(W.random_vector(2 * G.n_h, 62, 2), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    G.step(E, H, dt, nsteps=3, flags=K.TRACK_DB)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    G.step(E, H, dt, nsteps=steps, flags=K.TRACK_DB)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    # the same steps with the banded LU solves instead of the dense inverses
    G.set_solver(False)
    G.step(E, H, dt, nsteps=3, flags=K.TRACK_DB)
    torch.cuda.synchronize()
    ev0.record(stream)
    G.step(E, H, dt, nsteps=steps, flags=K.TRACK_DB)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_banded = ev0.elapsed_time(ev1) / steps
    G.set_solver(True)
    n_e, n_h = G.n_e, G.n_h
    nel = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    npts = (cfg["p"][0] + 1) * (cfg["p"][1] + 1) * (cfg["p"][2] + 1)
    mass = {}
    for which, n in (("B", G.n_h), ("D", G.n_e)):
        x = torch.tensor(W.random_vector(n, 63, 0), dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        G.op_mass(which, x, y)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            G.op_mass(which, x, y)
        ev1.record(stream)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) / reps * 1e3
        # algorithmic bytes of one apply (element kernel + gather): the metric
        # (6 doubles per point), 1/gamma per element, the input field, the
        # per-element windows written and read back once, the output field
        win = aniso_window(cfg["p"], which)
        flops = aniso_flops_per_element(cfg["p"], which) * nel
        bytes_ = 8.0 * (6 * npts * nel + nel + 2 * n + 2 * win * nel)
        mass[which] = {"us_per_apply": round(us, 2), "algorithmic_bytes": int(bytes_),
                       "GBps": round(bytes_ / (us * 1e-6) / 1e9, 1), "flops": int(flops),
                       "TFLOPs": round(flops / (us * 1e-6) / 1e12, 2)}
    del G, E, H
    # the same path on the single-degree headline space (p = 3 in every
    # direction, 64^3 uniform, deformed cube, eps ~ U[1,4]), plain steps,
    # beside the tuned single-degree path's plain step
    Gi = K.TSpace((3, 3, 3), (64, 64, 64), map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    Gi.set_materials(eps=W.eps_elements(64, 0))
    Ei = torch.tensor(W.random_vector(Gi.n_e, 64, 1), dtype=torch.float64, device="cuda")
    Hi = torch.tensor(W.random_vector(Gi.n_h, 64, 2), dtype=torch.float64, device="cuda")
    Gi.step(Ei, Hi, dt, nsteps=3)
    torch.cuda.synchronize()
    ev0.record(stream)
    Gi.step(Ei, Hi, dt, nsteps=steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_iso = ev0.elapsed_time(ev1) / steps
    del Gi, Ei, Hi
    return {"workload": "p=(3,3,2), 64x48x32 graded elements, deformed cube, eps/mu per element, tracking",
            "isotropic_64_plain_ms_per_step": round(ms_iso, 4),
            "n_e": n_e, "n_h": n_h, "ms_per_step": round(ms, 4), "ms_per_step_banded_solves": round(ms_banded, 4),
            "value": (n_e + n_h) / (ms * 1e-3), "unit": "DOF-updates/s", "mass_apply": mass}


def batched_timing(K, W, torch, steps=400):
    """Batched form: p=3, 24^3 elements, identity map, eps = mu = 1, zero
    initial fields, 256 members each driven by its own Gaussian point dipole
    (seed 0), dt = 0.5 CFL, `steps` steps captured as one graph (one
    persistent launch).  The plan is chosen by the library's tuner."""
    p, N, B = 3, 24, 256
    G = K.Space(p, N, max_batch=B)
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-7)
    dip = W.dipoles(B, seed=0, dt=dt)
    J = G.source(dip["pos"], dip["moment"], dip["t0"], dip["sigma"], dip["amp"], batch_of=list(range(B)))
    tune_ms = G.tune(B, dt, probe_steps=5, J=J)
    plan = G.plan()
    E = torch.zeros(B * G.n_e, dtype=torch.float64, device="cuda")
    H = torch.zeros(B * G.n_h, dtype=torch.float64, device="cuda")
    gr = G.graph(E, H, dt, steps, J=J, batch=B)
    stream = torch.cuda.current_stream()
    G.set_time(0.0)
    gr.launch()  # warm-up pass
    E.zero_()
    H.zero_()
    G.set_time(0.0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    gr.launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    dofs = (G.n_e + G.n_h) * B
    out = {"workload": f"batched sources: p={p}, {N}^3, identity map, eps=mu=1, {B} Gaussian point dipoles "
                       f"(one per member), zero initial fields, dt=0.5 CFL, {steps} steps in one graph launch, FP64",
           "dofs_e_plus_h": dofs, "ms_per_step": ms / steps, "value": dofs * steps / (ms * 1e-3),
           "unit": "DOF-updates/s", "plan": {"kind": K.PLAN_NAMES[plan[0]],
                                             "threads": plan[1]},
           "tuner_ms_per_step": dict(zip(K.TUNE_LABELS, tune_ms))}
    if plan[0] in (K.PLAN_SEPARABLE, K.PLAN_SEPARABLE_FUSED):
        # kernel duration with HIP events on the launch stream (eager call, same launch)
        G.profile_begin(capacity=8)
        G.step(E, H, dt, nsteps=steps, J=J, batch=B)
        prof = G.profile_end()
        k_s = prof["separable"][0] * 1e-3 / steps
        # algorithmic bytes per step: e and h each read twice (curl input, own
        # update) and written once
        bytes_step = 3.0 * 8.0 * dofs
        bw = bytes_step / k_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(bw, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(bw / HBM_PEAK_GBS, 4), "kernel": "sep_kernel (persistent, one launch)",
                           "avg_launch_ms": round(prof["separable"][0] / max(prof["separable"][1], 1), 3),
                           "algorithmic_bytes_per_step": int(bytes_step)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--only-mixed", action="store_true")
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--only-batched", action="store_true")
    ap.add_argument("--no-scheme1", action="store_true")
    ap.add_argument("--only-scheme1", action="store_true")
    ap.add_argument("--no-time-order", action="store_true")
    ap.add_argument("--no-coax", action="store_true")
    ap.add_argument("--no-aniso", action="store_true")
    ap.add_argument("--only-aniso", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only: the scheme-2 leapfrog here is a single-GPU build "
              f"(requested --gpus {args.gpus}, WORLD_SIZE={world}); the multi-GPU slab decomposition "
              f"is a design, not an implementation.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2302_04979_amd as K
    import workloads as W

    p, N = args.p, args.n
    torch.cuda.set_device(0)
    if args.profile_run:
        print(json.dumps(profile_run(K, W, torch, p, N, 10)), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_timing(K, W, torch)}), flush=True)
        return
    if args.only_aniso:
        print(json.dumps({"aniso": aniso_timing(K, W, torch)}), flush=True)
        return
    if args.only_mixed:
        print(json.dumps({"mixed": mixed_vs_fp64(K, W, torch, p, N, args.steps, W.eps_elements(N, 0)),
                          "p4": mixed_vs_fp64(K, W, torch, 4, 64, 500, W.eps_elements(64, 0))}), flush=True)
        return
    log(f"set-up p={p} N={N}")
    G = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE)
    eps = W.eps_elements(N, 0)
    G.set_materials(eps=eps)
    xq = G.quad_points()
    Eq = W.eval_modes(W.cavity_modes(0), xq)
    del xq
    dev = torch.device("cuda")
    E = torch.zeros(2 * G.n_e, dtype=torch.float64, device=dev)
    H = torch.zeros(2 * G.n_h, dtype=torch.float64, device=dev)
    G.project_E(Eq, E[:G.n_e])
    G.project_D(Eq, E[G.n_e:], tol=1e-13)
    del Eq
    e_proj = E[:G.n_e].clone()
    dt = 0.5 * G.cfl(max_iter=300, tol=1e-6)
    log(f"dt = {dt:.6e}")
    flags = K.TRACK_DB
    if args.only_scheme1:
        # scheme 2 on the same state for the ratio (plain step, eager), then scheme 1
        e2, h2 = E[:G.n_e].clone(), torch.zeros(G.n_h, dtype=torch.float64, device=dev)
        G.init_stagger(e2, h2, dt)
        G.step(e2, h2, dt, nsteps=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.step(e2, h2, dt, nsteps=args.steps)
        torch.cuda.synchronize()
        ms2 = (time.perf_counter() - t0) * 1e3 / args.steps
        print(json.dumps({"scheme2_ms_per_step_plain": ms2,
                          "scheme1": scheme1_timing(K, W, torch, G, E[:G.n_e].clone(), dt, ms2)}), flush=True)
        return
    G.init_stagger(E, H, dt, flags=flags)
    # the library's tuner picks the plan (tiled with banded or dense solves here)
    tune_ms = G.tune(1, dt, probe_steps=10)
    plan = G.plan()
    log(f"plan {K.PLAN_NAMES[plan[0]]}: {dict(zip(K.TUNE_LABELS, tune_ms))}")
    en_w = torch.zeros(max(args.warmup, 1), dtype=torch.float64, device=dev)
    en = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    en_p = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    if args.warmup:
        G.step(E, H, dt, nsteps=args.warmup, flags=flags, energy=en_w)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    E_start, H_start = E.clone(), H.clone()
    # ---- timed region ----
    log(f"timing {args.steps} steps")
    t_start = args.warmup * dt
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    G.step(E, H, dt, nsteps=args.steps, t_start=t_start, flags=flags, energy=en)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_eager = ev0.elapsed_time(ev1)
    # the same steps from the same state, captured once as a HIP graph and replayed
    Eg, Hg = E_start.clone(), H_start.clone()
    en_g = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    gr = G.graph(Eg, Hg, dt, args.steps, flags=flags, energy=en_g)
    G.set_time(t_start)
    gr.launch()  # first replay (warm)
    Eg.copy_(E_start)
    Hg.copy_(H_start)
    G.set_time(t_start)
    torch.cuda.synchronize()
    ev0.record(stream)
    gr.launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_graph = ev0.elapsed_time(ev1)
    graph_equal = bool(torch.equal(Eg, E) and torch.equal(Hg, H))
    gr.close()
    del Eg, Hg
    launch = "graph" if ms_graph < ms_eager else "eager"
    ms = min(ms_graph, ms_eager)
    ms_per_step = ms / args.steps
    dofs = G.n_e + G.n_h
    value = dofs * args.steps / (ms * 1e-3)
    energies = (en_g if launch == "graph" else en).cpu().numpy()
    drift = float(np.abs(energies / energies[0] - 1.0).max())

    # ---- per-kernel durations, HIP events on the launch stream ----
    G.profile_begin(capacity=16 * args.steps + 64)
    G.step(E, H, dt, nsteps=args.steps, t_start=t_start + args.steps * dt, flags=flags, energy=en_p)
    prof = G.profile_end()
    torch.cuda.synchronize()
    # the plain step (no b/d tracking, no energy) for reference
    e_only, h_only = E[:G.n_e].clone(), H[:G.n_h].clone()
    ev0.record(stream)
    G.step(e_only, h_only, dt, nsteps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / args.steps

    # dominant kernel: the fused curl + mass apply (two launches per step),
    # timed in a pass of its own where only its launches are bracketed by
    # events (the other kernels of the step run back to back)
    G.profile_begin(capacity=4 * args.steps + 64)
    G.profile_select(["mass_B", "mass_D"])
    G.step(E, H, dt, nsteps=args.steps, t_start=t_start + 2 * args.steps * dt, flags=flags, energy=en_p)
    prof_m = G.profile_end()
    ms_mass = prof_m["mass_B"][0] + prof_m["mass_D"][0]
    n_mass = prof_m["mass_B"][1] + prof_m["mass_D"][1]
    avg_mass_s = ms_mass / n_mass * 1e-3
    flops = 0.5 * (mass_flops(p, N, "B") + mass_flops(p, N, "D"))
    achieved = flops / avg_mass_s / 1e12
    sfx = "_w4" if plan[0] == K.PLAN_TILED_W4 else ""
    tb, td = measured_traffic("mass_B" + sfx), measured_traffic("mass_D" + sfx)
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": None if tb is None or td is None else 0.5 * (tb + td),
                "kernel": "mass_kernel (fused curl + 2-form Hodge apply, metric recomputed per Gauss point)",
                "avg_launch_us": round(avg_mass_s * 1e6, 2),
                "algorithmic_flops_per_launch": int(flops)}

    # the same step with the metric streamed from HBM (6 doubles per Gauss point)
    log("stored-metric variant")
    Gs = K.Space(p, N, map_kind=1, amplitude=W.DEFORMED_AMPLITUDE, stored_metric=True)
    Gs.set_materials(eps=eps)
    Es, Hs = E.clone(), H.clone()
    en_s = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    Gs.step(Es, Hs, dt, nsteps=args.warmup, flags=flags, energy=en_w)
    torch.cuda.synchronize()
    ev0.record(stream)
    Gs.step(Es, Hs, dt, nsteps=args.steps, flags=flags, energy=en_s)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_stored = ev0.elapsed_time(ev1) / args.steps
    Gs.profile_begin(capacity=16 * args.steps + 64)
    Gs.step(Es, Hs, dt, nsteps=args.steps, flags=flags, energy=en_s)
    prof_s = Gs.profile_end()
    avg_stored_s = (prof_s["mass_B"][0] + prof_s["mass_D"][0]) / (prof_s["mass_B"][1] + prof_s["mass_D"][1]) * 1e-3
    n_qp = G.n_qp
    # algorithmic bytes of one stored-metric mass apply: metric (6 doubles per
    # Gauss point), per-element 1/gamma, the input 1-form and the output 2-form
    bytes_mass = 8.0 * (6 * n_qp + N ** 3 + G.n_e + G.n_h)
    bw = bytes_mass / avg_stored_s / 1e9
    stored = {"ms_per_step": ms_stored, "value": dofs / (ms_stored * 1e-3),
              "roofline": {"bound": "hbm", "achieved": round(bw, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(bw / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_stored_s * 1e6, 2),
                           "algorithmic_bytes_per_launch": int(bytes_mass)}}
    del Gs, Es, Hs
    breakdown = {k: {"ms_per_launch": round(v[0] / v[1], 4) if v[1] else None, "launches": v[1]}
                 for k, v in prof.items()}

    # adjoint gradient: p=3, 32^3 deformed cube, eps = 2, one dipole, 64 probes,
    # 500 steps, checkpoints every 50 (the differentiation workload)
    adjoint_s = None
    if not args.no_adjoint:
        log("adjoint gradient")
        adjoint_s = adjoint_timing(K, W, torch)

    batched = None
    if not args.no_batched:
        log("batched form")
        batched = batched_timing(K, W, torch)

    mixed = None
    if not args.no_mixed:
        log("mixed precision, metric workload")
        mixed = mixed_vs_fp64(K, W, torch, p, N, args.steps, eps, dt, E_start, H_start, G)
        del E_start, H_start
        log("mixed precision, p=4 64^3, 500 steps")
        mixed["p4_n64_500_steps"] = mixed_vs_fp64(K, W, torch, 4, 64, 500, W.eps_elements(64, 0))

    def guarded(name, fn, *a, **kw):
        """An auxiliary measurement: its failure is recorded in the JSON line
        instead of ending the run (the headline figure above is complete)."""
        try:
            return fn(*a, **kw)
        except Exception as ex:  # noqa: BLE001 - reported, not hidden
            log(f"{name} failed: {ex}")
            return {"error": f"{type(ex).__name__}: {ex}"}

    time_order = None
    if not args.no_time_order:
        log("higher-order time stepping")
        time_order = guarded("time_order", time_order_comparison, K, W, torch, G, e_proj, dt)

    coax = None
    if not args.no_coax:
        log("curved workload (quarter coax)")
        coax = guarded("coax", coax_timing, K, W, torch)
        log("quarter coax with the TEM data lifted")
        coax["tem_lifted"] = guarded("coax_tem", coax_tem_timing, K, W, torch)

    aniso = None
    if not args.no_aniso:
        log("per-direction degrees, knots and element counts")
        aniso = guarded("aniso", aniso_timing, K, W, torch)

    scheme1 = None
    if not args.no_scheme1:
        log("first scheme")
        scheme1 = guarded("scheme1", scheme1_timing, K, W, torch, G, e_only, dt, ms_per_step)
        log("both schemes against the degree, 32^3")
        scheme1["vs_degree"] = guarded("vs_degree", schemes_vs_degree, K, W, torch)
        log("cavity convergence of both schemes")
        scheme1["convergence"] = guarded("convergence", convergence_both_schemes, K, W, torch)
        log("both schemes on the quarter coax, p=4, 16^3")
        scheme1["coax_p4_n16"] = guarded("coax_p4_n16", coax_schemes, K, W, torch)
        scheme1["coax_p4_n16_random_eps"] = guarded("coax_p4_n16_random_eps", coax_schemes, K, W, torch,
                                                    random_eps=True)

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        cpu = cpu_baseline(p, N, args.cpu_steps, eps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scheme-2 leapfrog, deformed cube (a=0.08), p={p}, {N}^3 elements, "
                               f"eps~U[1,4], 10 cavity modes, dt=0.5 CFL, FP64, b/d tracking + energy",
                   "dofs_e_plus_h": dofs, "dt": dt, "parallelism": "single GPU",
                   "plan": K.PLAN_NAMES[plan[0]], "launch": launch,
                   "ms_per_step_eager": ms_eager / args.steps, "ms_per_step_graph": ms_graph / args.steps,
                   "graph_result_equals_eager": graph_equal,
                   "tuner_ms_per_step": {k: v for k, v in zip(K.TUNE_LABELS, tune_ms) if v is not None}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ms_per_step_plain": ms_plain,
        "value_plain": dofs / (ms_plain * 1e-3),
        "energy_rel_drift": drift,
        "kernels": breakdown,
        "stored_metric": stored,
        "mixed": mixed,
        "adjoint_grad_s": adjoint_s,
        "batched": batched,
        "scheme1": scheme1,
        "time_order": time_order,
        "coax": coax,
        "aniso": aniso,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
