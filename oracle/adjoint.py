"""Probe-misfit loss and its gradient with respect to per-element permittivity,
by the discrete adjoint of the (e, h) leapfrog (oracle, FP64, plain NumPy).

Test infrastructure only (see ``oracle/__init__``).

The paper has no adjoint; this is the exact reverse-mode derivative of the
time-discrete scheme it defines (Section 3.4.2 form, see ``oracle.scheme``):

  forward, from e^0 = 0, h^{-1/2} = 0:
      h^{n+1/2} = h^{n-1/2} - dt K~1^{-1} M D^1 e^n
      e^{n+1}   = e^n + dt K1^{-1} (M~_eps D~^1 h^{n+1/2} - s_eps(t_{n+1/2}))
  loss  L = 1/2 sum_{n=1}^{N} sum_k |E_h(x_k, t_n) - y_k^n|^2,  E_h(x_k) = P_k e.

  reverse, with ebar = dL/de, hbar = dL/dh (all states stored):
      ebar^N = P^T r^N, hbar = 0
      for n = N-1 .. 0:
          lam   = K1^{-T} ebar^{n+1}
          hbar += dt D~^{1T} M~ lam
          g_e  += dt [ -(1/eps_e^2) lam^T M~_e^{(1)} D~^1 h^{n+1/2} ]      every element e
          g_e0 += dt (lam . s(t_{n+1/2})) / eps_e0                          dipole element
          ebar^n = ebar^{n+1} - dt D^{1T} M K~1^{-T} hbar  (+ P^T r^n for n >= 1)

M~_e^{(1)} is the element's contribution to M~ with 1/eps = 1; lam^T M~_e^{(1)} v
is the sum over the element's Gauss points of Lam(q) . G(q) V(q) with Lam, V the
interpolated fields and G the 2-form metric factor (weights included).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .scheme import Scheme
from .spaces import comp_tags, join, split


def _diffT_primal(u: np.ndarray, ax: int) -> np.ndarray:
    """Transpose of (d v)[k] = v[k] - v[k-1]: (d^T u)[c] = u[c] - u[c+1]."""
    k = 2 - ax
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[k] = slice(0, -1)
    hi[k] = slice(1, None)
    return u[tuple(lo)] - u[tuple(hi)]


def _diffT_dual(u: np.ndarray, ax: int) -> np.ndarray:
    """Transpose of (d~ v)[r] = v[r+1] - v[r]: (d~^T u)[j] = u[j-1] - u[j] (zero outside)."""
    k = 2 - ax
    pad = [(0, 0)] * 3
    pad[k] = (1, 1)
    w = np.pad(u, pad)
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[k] = slice(0, -1)
    hi[k] = slice(1, None)
    return w[tuple(lo)] - w[tuple(hi)]


def curl_T(S: Scheme, y: np.ndarray, primal: bool) -> np.ndarray:
    """(D^1)^T y (primal: X^2_{h,0} -> X^1_{h,0}) or (D~^1)^T y (X~^2 -> X~^1)."""
    src, dst = ("B", "E") if primal else ("D", "H")
    diffT = _diffT_primal if primal else _diffT_dual
    Y = split(S.axis, src, y)
    out = [None, None, None]
    for c in range(3):
        a1, a2 = (c + 1) % 3, (c + 2) % 3
        # y_c = d_{a1} u_{a2} - d_{a2} u_{a1}
        t2 = diffT(Y[c], a1)
        t1 = -diffT(Y[c], a2)
        out[a2] = t2 if out[a2] is None else out[a2] + t2
        out[a1] = t1 if out[a1] is None else out[a1] + t1
    return join(out)


def probe_matrix(S: Scheme, pos: np.ndarray) -> sp.csr_matrix:
    """Sparse P (3 n_probes x n_e): rows (k, c) give the physical component c of
    E_h = DF^{-T} E^_h at parametric point pos[k]."""
    rows, cols, vals = [], [], []
    offs = np.cumsum([0] + [int(np.prod(x.shape)) for x in split(S.axis, "E", np.zeros(S.n_e))])
    for k, xh in enumerate(np.asarray(pos, float)):
        DF = S.geo.DF(xh[None])[0]
        Minv_T = np.linalg.inv(DF).T  # physical = DF^{-T} parametric
        for j in range(3):
            bx, by, bz = [S.axis.eval(t, np.array([xh[a]]))[0] for a, t in enumerate(comp_tags("E", j))]
            w3 = (bz[:, None, None] * by[None, :, None] * bx[None, None, :]).ravel()
            nz = np.nonzero(w3)[0]
            for c in range(3):
                rows.extend([3 * k + c] * nz.size)
                cols.extend((offs[j] + nz).tolist())
                vals.extend((Minv_T[c, j] * w3[nz]).tolist())
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * len(pos), S.n_e))


def elem_pairing(S: Scheme, lam: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Per element: sum over its Gauss points of Lam . G V (G = w DF^T DF / det DF),
    for two fields of the dual 2-form space; array (N, N, N) [ez, ey, ex]."""
    L = S.interpolate("D", lam)
    V = S.interpolate("D", v)
    G = S.metric()
    tot = np.zeros_like(L[0])
    for i in range(3):
        for j in range(3):
            tot += L[i] * G[i, j] * V[j]
    N, nq = S.N, S.nq
    return tot.reshape(N, nq, N, nq, N, nq).sum(axis=(1, 3, 5))


class ProbeProblem:
    """Zero initial fields, point dipoles, probes; loss and gradient in eps."""

    def __init__(self, S: Scheme, dip: dict, probes: np.ndarray, dt: float, nsteps: int):
        self.S, self.dip, self.dt, self.nsteps = S, dip, dt, nsteps
        self.P = probe_matrix(S, probes)
        self.n_probes = len(probes)

    def _sources(self):
        S, dip = self.S, self.dip
        return [S.dipole_source(dip["pos"][k], dip["moment"][k]) for k in range(len(dip["pos"]))]

    def _g(self, k, t):
        d = self.dip
        return d["amp"][k] * np.exp(-(t - d["t0"][k]) ** 2 / (2 * d["sigma"][k] ** 2))

    def forward(self, record_states: bool = False):
        """Probe values P e^n for n = 1..N, shape (N, n_probes, 3); optionally
        the states (e^n for n = 0..N, h^{n+1/2} for n = 0..N-1)."""
        S, dt = self.S, self.dt
        s = self._sources()
        e = np.zeros(S.n_e)
        h = np.zeros(S.n_h)
        es, hs, obs = [e.copy()], [], []
        for n in range(self.nsteps):
            t = (n + 0.5) * dt
            src = sum(self._g(k, t) * s[k] for k in range(len(s)))
            e, h, _, _, _ = S.step(e, h, dt, nsteps=1, t0=n * dt, source=lambda tt, src=src: src)
            obs.append((self.P @ e).reshape(self.n_probes, 3))
            if record_states:
                es.append(e.copy())
                hs.append(h.copy())
        obs = np.array(obs)
        return (obs, es, hs) if record_states else obs

    def loss(self, data: np.ndarray) -> float:
        r = self.forward() - data
        return 0.5 * float(np.sum(r * r))

    def gradient(self, data: np.ndarray):
        """(loss, dL/deps (N, N, N)) by the reverse sweep over stored states."""
        S, dt = self.S, self.dt
        obs, es, hs = self.forward(record_states=True)
        res = obs - data
        loss = 0.5 * float(np.sum(res * res))
        s = self._sources()
        eps = S.eps if S.eps is not None else np.ones((S.N,) * 3)
        grad = np.zeros((S.N,) * 3)
        N = self.nsteps
        ebar = self.P.T @ res[N - 1].ravel()
        hbar = np.zeros(S.n_h)
        for n in range(N - 1, -1, -1):
            t = (n + 0.5) * dt
            lam = S.kron_solve("K1", ebar, transpose=True)
            hbar = hbar + dt * curl_T(S, S.mass_apply("D", lam), primal=False)
            v = S.curl_dual(hs[n])
            grad -= dt * elem_pairing(S, lam, v) / eps ** 2
            for k in range(len(s)):
                el = np.minimum((np.asarray(self.dip["pos"][k]) * S.N).astype(int), S.N - 1)
                grad[el[2], el[1], el[0]] += dt * self._g(k, t) * (lam @ s[k]) / eps[el[2], el[1], el[0]]
            ebar = ebar - dt * curl_T(S, S.mass_apply("B", S.kron_solve("K1t", hbar, transpose=True)), primal=True)
            if n >= 1:
                ebar = ebar + self.P.T @ res[n - 1].ravel()
        return loss, grad


def step_transpose(S: Scheme, ebar: np.ndarray, hbar: np.ndarray, dt: float):
    """Adjoint of one source-free (e, h) step at fixed eps: returns
    (ebar_prev, hbar_prev) such that <J x, y> = <x, J^T y>."""
    lam = S.kron_solve("K1", ebar, transpose=True)
    hbar = hbar + dt * curl_T(S, S.mass_apply("D", lam), primal=False)
    ebar = ebar - dt * curl_T(S, S.mass_apply("B", S.kron_solve("K1t", hbar, transpose=True)), primal=True)
    return ebar, hbar
