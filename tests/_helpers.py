"""Shared helpers for the GPU parity tests (oracle on the host, HIP path on cuda:0)."""
import numpy as np

import workloads as W


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def make_pair(p, N, deformed=True, eps=True, max_batch=1, eps_seed=0):
    """Oracle Scheme and GPU Space on the same problem."""
    from oracle.geometry import Map
    from oracle.scheme import Scheme
    import paper_2302_04979_amd as K
    e = W.eps_elements(N, eps_seed) if eps else None
    geo = Map("sine", W.DEFORMED_AMPLITUDE) if deformed else Map("identity")
    S = Scheme(p, N, geo, eps=e)
    G = K.Space(p, N, map_kind=1 if deformed else 0, amplitude=W.DEFORMED_AMPLITUDE if deformed else 0.0,
                max_batch=max_batch)
    if eps:
        G.set_materials(eps=e)
    return S, G


def to_dev(x):
    import torch
    return torch.tensor(np.asarray(x, dtype=float), dtype=torch.float64, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(float)


def qp_param_points(p, N):
    """Parametric Gauss points in the element-major order of the library
    ([ez][ey][ex][iqz][iqy][iqx]), p+1 Gauss-Legendre points per element."""
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    x = (np.arange(N)[:, None] + 0.5 * (g[None, :] + 1.0)) / N  # [e][iq]
    X = np.broadcast_to(x[None, None, :, None, None, :], (N, N, N, p + 1, p + 1, p + 1))
    Y = np.broadcast_to(x[None, :, None, None, :, None], (N, N, N, p + 1, p + 1, p + 1))
    Z = np.broadcast_to(x[:, None, None, :, None, None], (N, N, N, p + 1, p + 1, p + 1))
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def relmax(a, b):
    """The larger of the relative 2-norm error and the element-wise error
    (max |a - b| over max |b|): a parity bound on both."""
    return max(rel(a, b), maxrel(a, b))


def maxrel(a, b):
    """Element-wise bound: max |a - b| over max |b|."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0
