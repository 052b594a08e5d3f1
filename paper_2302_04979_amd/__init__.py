"""kronmaxwell: MI355X-native explicit leapfrog for the spline geometric Maxwell
scheme with Kronecker-structured pairing solves (scheme 2 of Kapidani &
Vazquez, Section 3.4 and Section 4).

Thin Python binding over the C-ABI library ``libkronmaxwell.so`` (declared in
``include/kronmaxwell.h``).  Every function here only marshals arguments:
device vectors are torch float64 CUDA tensors passed as raw pointers, on the
caller's current stream.  All arithmetic of the time step runs in the HIP
kernels of the library; there is no fallback path: if the library is missing
an ImportError-like RuntimeError is raised on first use.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Space", "TSpace", "Source", "load_library", "EXPORTS", "TRACK_DB", "KMXError"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkronmaxwell.so")
TRACK_DB = 1
STORED_METRIC = 16
FP64, MIXED = 0, 1
PLAN_AUTO, PLAN_TILED, PLAN_SEPARABLE, PLAN_SEPARABLE_FUSED, PLAN_TILED_DENSE, PLAN_TILED_W4 = -1, 0, 1, 2, 3, 4
TUNE_CANDIDATES = 8
TUNE_LABELS = ("tiled", "tiled-w4", "tiled-dense", "separable/384", "separable/512", "separable/768",
               "separable-fused/512", "separable-fused/768")
PLAN_NAMES = {PLAN_AUTO: "auto", PLAN_TILED: "tiled", PLAN_SEPARABLE: "separable",
              PLAN_SEPARABLE_FUSED: "separable-fused", PLAN_TILED_DENSE: "tiled-dense", PLAN_TILED_W4: "tiled-w4"}

# every symbol declared in include/kronmaxwell.h
EXPORTS = (
    "kmx_create_space", "kmx_destroy_space", "kmx_set_materials", "kmx_sizes", "kmx_quad_points",
    "kmx_project_E", "kmx_project_D", "kmx_cfl", "kmx_create_source", "kmx_destroy_source",
    "kmx_create_source_pattern",
    "kmx_init_stagger", "kmx_step", "kmx_energy", "kmx_op_curl", "kmx_op_mass", "kmx_op_solve",
    "kmx_op_pairing", "kmx_profile_begin", "kmx_profile_end", "kmx_create_probes", "kmx_destroy_probes",
    "kmx_probe_eval", "kmx_probe_forward", "kmx_adjoint", "kmx_set_plan", "kmx_get_plan", "kmx_tune",
    "kmx_set_refinement",
    "kmx_graph_create", "kmx_graph_launch",
    "kmx_graph_destroy", "kmx_set_time", "kmx_get_time", "kmx_last_error",
    "kmx_op_mass1", "kmx_solve_mass1", "kmx_half_step_scheme1", "kmx_step_scheme1", "kmx_cfl_scheme1",
    "kmx_init_split", "kmx_step_split", "kmx_project_E1", "kmx_graph_create_scheme1",
    "kmx_probe_forward_noalloc", "kmx_profile_select", "kmx_sizes_full", "kmx_lift_boundary",
    "kmx_set_lifting",
    "kmx_create_tspace", "kmx_destroy_tspace", "kmx_tspace_sizes", "kmx_tspace_set_materials",
    "kmx_tspace_op_curl", "kmx_tspace_op_mass", "kmx_tspace_op_solve", "kmx_tspace_op_pairing",
    "kmx_tspace_step", "kmx_tspace_set_solver",
)
PROFILE_KINDS = ("mass_B", "mass_D", "solve_xy", "solve_z", "curl", "energy", "gather", "separable",
                 "mode_fp32", "dense_fp64", "mass_1form", "cg_vector")

_STATUS = {0: "KMX_OK", 1: "KMX_E_ARG", 2: "KMX_E_GEOMETRY", 3: "KMX_E_MATERIAL", 4: "KMX_E_DEVICE",
           5: "KMX_E_OOM", 6: "KMX_E_UNSTABLE", 7: "KMX_E_STATE"}


class KMXError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Map(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("amplitude", ctypes.c_double), ("dF_qp", ctypes.c_void_p)]


_lib = None


def load_library():
    """Load libkronmaxwell.so (built in-tree by ``paper_2302_04979_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_04979_amd.build`")
    # torch ships its own HIP runtime; load it first so that the library binds
    # to that same runtime instance (one device context, shared streams and
    # allocations) instead of mapping a second copy from the ROCm install.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, i64p = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)
    sig = {
        "kmx_create_space": ([i, i, ctypes.POINTER(_Map), i, i, ctypes.POINTER(vp)], i),
        "kmx_destroy_space": ([vp], None),
        "kmx_set_materials": ([vp, vp, vp], i),
        "kmx_sizes": ([vp, i64p, i64p, i64p], i),
        "kmx_quad_points": ([vp, vp], i),
        "kmx_project_E": ([vp, vp, vp, vp], i),
        "kmx_project_D": ([vp, vp, vp, d, vp], i),
        "kmx_cfl": ([vp, i, d, ctypes.POINTER(d)], i),
        "kmx_create_source": ([vp, i, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)], i),
        "kmx_create_source_pattern": ([vp, i, vp, i, d, d, vp, ctypes.POINTER(vp)], i),
        "kmx_destroy_source": ([vp], None),
        "kmx_init_stagger": ([vp, vp, vp, d, i, i, vp], i),
        "kmx_step": ([vp, vp, vp, vp, d, d, i, i, i, vp, vp], i),
        "kmx_energy": ([vp, vp, vp, d, i, vp, vp], i),
        "kmx_op_curl": ([vp, i, vp, vp, vp], i),
        "kmx_op_mass": ([vp, i, i, vp, vp, vp], i),
        "kmx_op_solve": ([vp, i, i, vp, vp, vp], i),
        "kmx_op_pairing": ([vp, i, vp, vp, vp], i),
        "kmx_profile_begin": ([vp, i], i),
        "kmx_profile_select": ([vp, ctypes.c_uint], i),
        "kmx_profile_end": ([vp, vp, vp], i),
        "kmx_create_probes": ([vp, i, vp, ctypes.POINTER(vp)], i),
        "kmx_destroy_probes": ([vp], None),
        "kmx_probe_eval": ([vp, vp, vp, vp, vp], i),
        "kmx_probe_forward": ([vp, vp, vp, d, i, vp, vp], i),
        "kmx_probe_forward_noalloc": ([vp, vp, vp, d, i, vp, vp], i),
        "kmx_adjoint": ([vp, vp, vp, vp, d, i, i, ctypes.POINTER(d), vp, vp], i),
        "kmx_set_plan": ([vp, i, i], i),
        "kmx_set_refinement": ([vp, i], i),
        "kmx_get_plan": ([vp, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "kmx_tune": ([vp, i, i, vp, d, vp, vp], i),
        "kmx_graph_create": ([vp, vp, vp, vp, d, i, i, i, vp, ctypes.POINTER(vp)], i),
        "kmx_graph_launch": ([vp, vp], i),
        "kmx_graph_destroy": ([vp], None),
        "kmx_set_time": ([vp, d, vp], i),
        "kmx_get_time": ([vp, ctypes.POINTER(d), vp], i),
        "kmx_last_error": ([], ctypes.c_char_p),
        "kmx_op_mass1": ([vp, i, vp, vp, vp], i),
        "kmx_solve_mass1": ([vp, i, vp, vp, d, i, ctypes.POINTER(i), vp], i),
        "kmx_half_step_scheme1": ([vp, i, vp, vp, d, d, i, ctypes.POINTER(i), vp], i),
        "kmx_step_scheme1": ([vp, vp, vp, d, i, d, i, vp, vp], i),
        "kmx_cfl_scheme1": ([vp, i, d, d, ctypes.POINTER(d)], i),
        "kmx_init_split": ([vp, vp, vp, d, i, i, i, vp], i),
        "kmx_project_E1": ([vp, vp, vp, d, vp], i),
        "kmx_graph_create_scheme1": ([vp, vp, vp, d, i, i, i, ctypes.POINTER(vp)], i),
        "kmx_step_split": ([vp, vp, vp, d, i, i, i, i, vp], i),
        "kmx_sizes_full": ([vp, i64p], i),
        "kmx_lift_boundary": ([vp, vp, vp, ctypes.POINTER(i)], i),
        "kmx_set_lifting": ([vp, i, vp, vp, vp, vp], i),
        "kmx_create_tspace": ([vp, vp, vp, vp, vp, ctypes.POINTER(_Map), i, ctypes.POINTER(vp)], i),
        "kmx_destroy_tspace": ([vp], None),
        "kmx_tspace_sizes": ([vp, i64p, i64p], i),
        "kmx_tspace_set_materials": ([vp, vp, vp], i),
        "kmx_tspace_op_curl": ([vp, i, vp, vp, vp], i),
        "kmx_tspace_op_mass": ([vp, i, vp, vp, vp], i),
        "kmx_tspace_op_solve": ([vp, i, i, vp, vp, vp], i),
        "kmx_tspace_op_pairing": ([vp, i, vp, vp, vp], i),
        "kmx_tspace_step": ([vp, vp, vp, d, i, i, i, vp], i),
        "kmx_tspace_set_solver": ([vp, i], i),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise KMXError(st, load_library().kmx_last_error().decode())


def _dptr(t, n=None, name="tensor"):
    """Raw device pointer of a contiguous float64 CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} entries, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a, n=None, dtype=np.float64, name="array"):
    a = np.ascontiguousarray(a, dtype=dtype)
    if n is not None and a.size != n:
        raise ValueError(f"{name} has {a.size} entries, needs {n}")
    return a, ctypes.c_void_p(a.ctypes.data)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Source:
    """Point dipoles (see kmx_create_source), or with `pattern` a dense pattern
    times a sampled time series (kmx_create_source_pattern)."""

    def __init__(self, space: "Space", pos=None, moment=None, t0=None, sigma=None, amp=None, batch_of=None,
                 pattern=None, series=None, series_t0=0.0, series_dt=None):
        L = load_library()
        if pattern is not None:
            pat = np.ascontiguousarray(np.asarray(pattern, dtype=np.float64).reshape(-1, space.n_e))
            ser = np.ascontiguousarray(np.asarray(series, dtype=np.float64).ravel())
            h = ctypes.c_void_p()
            _check(L.kmx_create_source_pattern(space._h, int(pat.shape[0]), ctypes.c_void_p(pat.ctypes.data),
                                               int(ser.size), float(series_t0), float(series_dt),
                                               ctypes.c_void_p(ser.ctypes.data), ctypes.byref(h)))
            self._h = h
            self.space = space
            self.n = 0
            return
        n = int(np.asarray(pos).shape[0])
        self._keep = [_hptr(pos, 3 * n), _hptr(moment, 3 * n), _hptr(t0, n), _hptr(sigma, n), _hptr(amp, n)]
        bo = None if batch_of is None else _hptr(batch_of, n, np.int32)
        h = ctypes.c_void_p()
        _check(L.kmx_create_source(space._h, n, *[k[1] for k in self._keep],
                                   None if bo is None else bo[1], ctypes.byref(h)))
        self._h = h
        self.space = space
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            load_library().kmx_destroy_source(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured chunk of leapfrog steps (kmx_graph_create); launch() replays it."""

    def __init__(self, space: "Space", E, H, dt, nsteps, J=None, batch=1, flags=0, energy=None):
        k = 1 + (flags & TRACK_DB)
        en = None if energy is None else _dptr(energy, nsteps * batch, "energy")
        h = ctypes.c_void_p()
        _check(load_library().kmx_graph_create(space._h, _dptr(E, batch * k * space.n_e, "E"),
                                               _dptr(H, batch * k * space.n_h, "H"), None if J is None else J._h,
                                               float(dt), int(nsteps), int(batch), int(flags), en, ctypes.byref(h)))
        self._h = h
        self._keep = (E, H, J, energy)  # bound at capture
        self.space = space
        self.nsteps = nsteps

    def launch(self):
        _check(load_library().kmx_graph_launch(self._h, _stream()))

    def close(self):
        if getattr(self, "_h", None):
            load_library().kmx_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Probes:
    """Point probes of the physical electric field (kmx_create_probes)."""

    def __init__(self, space: "Space", pos):
        n = int(np.asarray(pos).shape[0])
        self._pos = _hptr(pos, 3 * n)
        h = ctypes.c_void_p()
        _check(load_library().kmx_create_probes(space._h, n, self._pos[1], ctypes.byref(h)))
        self._h = h
        self.space = space
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            load_library().kmx_destroy_probes(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GraphScheme1(Graph):
    """nsteps first-scheme steps with fixed CG iteration counts, captured as a
    HIP graph (kmx_graph_create_scheme1); launch() replays it."""

    def __init__(self, space: "Space", e, h, dt, nsteps, iters_e, iters_h):
        g = ctypes.c_void_p()
        _check(load_library().kmx_graph_create_scheme1(space._h, _dptr(e, space.n_e, "e"),
                                                       _dptr(h, space.n_h, "h"), float(dt), int(nsteps),
                                                       int(iters_e), int(iters_h), ctypes.byref(g)))
        self._h = g
        self._keep = (e, h)  # bound at capture
        self.space = space
        self.nsteps = nsteps


class TSpace:
    """Spaces with a degree, a knot vector and an element count per direction
    (kmx_create_tspace): p and n_elem are (x, y, z) triples, breaks the
    interior breakpoints of each direction (None: uniform)."""

    def __init__(self, p, n_elem, breaks=(None, None, None), map_kind: int = 0, amplitude: float = 0.0,
                 max_batch: int = 1):
        L = load_library()
        self.p = tuple(int(v) for v in p)
        self.N = tuple(int(v) for v in n_elem)
        pa = (ctypes.c_int * 3)(*self.p)
        na = (ctypes.c_int * 3)(*self.N)
        self._breaks = []
        ptrs = []
        for a in range(3):
            if breaks[a] is None:
                ptrs.append(None)
            else:
                arr, ptr = _hptr(breaks[a], self.N[a] - 1, name="breaks")
                self._breaks.append(arr)
                ptrs.append(ptr)
        m = _Map(int(map_kind), float(amplitude), None)
        h = ctypes.c_void_p()
        _check(L.kmx_create_tspace(pa, na, ptrs[0], ptrs[1], ptrs[2], ctypes.byref(m), int(max_batch),
                                   ctypes.byref(h)))
        self._h = h
        self.max_batch = max_batch
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(L.kmx_tspace_sizes(h, ctypes.byref(a), ctypes.byref(b)))
        self.n_e, self.n_h = a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().kmx_destroy_tspace(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_materials(self, eps=None, mu=None):
        n = self.N[0] * self.N[1] * self.N[2]
        e = None if eps is None else _hptr(np.asarray(eps).ravel(), n, name="eps")
        m = None if mu is None else _hptr(np.asarray(mu).ravel(), n, name="mu")
        _check(load_library().kmx_tspace_set_materials(self._h, None if e is None else e[1],
                                                       None if m is None else m[1]))

    def set_solver(self, dense: bool):
        """Dense inverse factors on the matrix cores (True) or banded LU (False)."""
        _check(load_library().kmx_tspace_set_solver(self._h, int(bool(dense))))

    def op_curl(self, primal: bool, x, y):
        n_in, n_out = (self.n_e, self.n_h) if primal else (self.n_h, self.n_e)
        _check(load_library().kmx_tspace_op_curl(self._h, 0 if primal else 1, _dptr(x, n_in, "x"),
                                                 _dptr(y, n_out, "y"), _stream()))

    def op_mass(self, which: str, x, y):
        """which 'B' (M^2_{1/mu}) or 'D' (M~^2_{1/eps})."""
        w = 0 if which == "B" else 1
        n = self.n_h if w == 0 else self.n_e
        _check(load_library().kmx_tspace_op_mass(self._h, w, _dptr(x, n, "x"), _dptr(y, n, "y"), _stream()))

    def op_solve(self, which: str, y, x, transpose=False):
        """which 'K1' or 'K1t': x = K^{-1} y (or K^{-T} y)."""
        w = 1 if which == "K1" else 0
        n = self.n_e if w else self.n_h
        _check(load_library().kmx_tspace_op_solve(self._h, w, int(bool(transpose)), _dptr(y, n, "y"),
                                                  _dptr(x, n, "x"), _stream()))

    def op_pairing(self, which: str, x, y):
        """y = K x, which 'K1' or 'K1t'."""
        w = 1 if which == "K1" else 0
        n = self.n_e if w else self.n_h
        _check(load_library().kmx_tspace_op_pairing(self._h, w, _dptr(x, n, "x"), _dptr(y, n, "y"), _stream()))

    def step(self, E, H, dt, nsteps=1, batch=1, flags=0):
        k = 1 + (flags & TRACK_DB)
        _check(load_library().kmx_tspace_step(self._h, _dptr(E, batch * k * self.n_e, "E"),
                                              _dptr(H, batch * k * self.n_h, "H"), float(dt), int(nsteps),
                                              int(batch), int(flags), _stream()))


class Space:
    """Discrete spaces, operators and scratch of one problem (kmx_create_space)."""

    def __init__(self, p: int, n_elem: int, map_kind: int = 0, amplitude: float = 0.0, dF_qp=None,
                 precision: int = 0, max_batch: int = 1, stored_metric: bool = False):
        L = load_library()
        if stored_metric:
            precision |= STORED_METRIC
        self._dF = None
        m = _Map(int(map_kind), float(amplitude), None)
        if dF_qp is not None:
            self._dF, ptr = _hptr(dF_qp)
            m.dF_qp = ptr
        h = ctypes.c_void_p()
        _check(L.kmx_create_space(int(p), int(n_elem), ctypes.byref(m), int(precision), int(max_batch),
                                  ctypes.byref(h)))
        self._h = h
        self.p, self.N, self.max_batch = p, n_elem, max_batch
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.kmx_sizes(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        self.n_e, self.n_h, self.n_qp = a.value, b.value, c.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().kmx_destroy_space(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- set-up -------------------------------------------------------
    def set_materials(self, eps=None, mu=None):
        n3 = self.N ** 3
        e = None if eps is None else _hptr(np.asarray(eps).ravel(), n3, name="eps")
        m = None if mu is None else _hptr(np.asarray(mu).ravel(), n3, name="mu")
        _check(load_library().kmx_set_materials(self._h, None if e is None else e[1], None if m is None else m[1]))

    def quad_points(self) -> np.ndarray:
        out = np.empty((self.n_qp, 3))
        _check(load_library().kmx_quad_points(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def project_E(self, E_qp, e):
        a, ptr = _hptr(E_qp, 3 * self.n_qp, name="E_qp")
        _check(load_library().kmx_project_E(self._h, ptr, _dptr(e, self.n_e, "e"), _stream()))

    def project_D(self, E_qp, d, tol=1e-13):
        a, ptr = _hptr(E_qp, 3 * self.n_qp, name="E_qp")
        _check(load_library().kmx_project_D(self._h, ptr, _dptr(d, self.n_e, "d"), float(tol), _stream()))

    def cfl(self, max_iter=2000, tol=1e-10) -> float:
        out = ctypes.c_double()
        _check(load_library().kmx_cfl(self._h, int(max_iter), float(tol), ctypes.byref(out)))
        return out.value

    def source_pattern(self, pattern, series, t0, dt_sample) -> Source:
        """s(t) = g(t) P: pattern (npat x n_e, host), g sampled at t0 + k dt_sample."""
        return Source(self, pattern=pattern, series=series, series_t0=t0, series_dt=dt_sample)

    def source(self, pos, moment, t0, sigma, amp, batch_of=None) -> Source:
        return Source(self, pos, moment, t0, sigma, amp, batch_of)

    # ---- time stepping ------------------------------------------------
    def init_stagger(self, E, H, dt, batch=1, flags=0):
        k = 1 + (flags & TRACK_DB)
        _check(load_library().kmx_init_stagger(self._h, _dptr(E, batch * k * self.n_e, "E"),
                                               _dptr(H, batch * k * self.n_h, "H"), float(dt), int(batch),
                                               int(flags), _stream()))

    def step(self, E, H, dt, nsteps=1, J: Source | None = None, t_start=0.0, batch=1, flags=0, energy=None):
        k = 1 + (flags & TRACK_DB)
        en = None if energy is None else _dptr(energy, nsteps * batch, "energy")
        _check(load_library().kmx_step(self._h, _dptr(E, batch * k * self.n_e, "E"),
                                       _dptr(H, batch * k * self.n_h, "H"), None if J is None else J._h,
                                       float(t_start), float(dt), int(nsteps), int(batch), int(flags), en,
                                       _stream()))

    def init_split(self, E, H, dt, order, batch=1, flags=0):
        """Staggered start of a composed run of the given order (2, 4, 6)."""
        k = 1 + (flags & TRACK_DB)
        _check(load_library().kmx_init_split(self._h, _dptr(E, batch * k * self.n_e, "E"),
                                             _dptr(H, batch * k * self.n_h, "H"), float(dt), int(order),
                                             int(batch), int(flags), _stream()))

    def step_split(self, E, H, dt, nsteps, order, batch=1, flags=0):
        """nsteps symmetric-composition steps of order 2, 4 or 6 (source free)."""
        k = 1 + (flags & TRACK_DB)
        _check(load_library().kmx_step_split(self._h, _dptr(E, batch * k * self.n_e, "E"),
                                             _dptr(H, batch * k * self.n_h, "H"), float(dt), int(nsteps),
                                             int(order), int(batch), int(flags), _stream()))

    def energy(self, E, H, dt, batch=1) -> np.ndarray:
        out = np.empty(2 * batch)
        _check(load_library().kmx_energy(self._h, _dptr(E, batch * 2 * self.n_e, "E"),
                                         _dptr(H, batch * 2 * self.n_h, "H"), float(dt), int(batch),
                                         ctypes.c_void_p(out.ctypes.data), _stream()))
        return out.reshape(batch, 2)

    # ---- single operators ---------------------------------------------
    def op_curl(self, primal: bool, x, y):
        n_in, n_out = (self.n_e, self.n_h) if primal else (self.n_h, self.n_e)
        _check(load_library().kmx_op_curl(self._h, 0 if primal else 1, _dptr(x, n_in, "x"), _dptr(y, n_out, "y"),
                                          _stream()))

    def op_mass(self, which: str, x, y, curl=False):
        """which 'B' (M^2_{1/mu}) or 'D' (M~^2_{1/eps}); curl=True applies M D."""
        w = 0 if which == "B" else 1
        n_out = self.n_h if w == 0 else self.n_e
        n_in = (self.n_e if w == 0 else self.n_h) if curl else n_out
        _check(load_library().kmx_op_mass(self._h, w, int(bool(curl)), _dptr(x, n_in, "x"), _dptr(y, n_out, "y"),
                                          _stream()))

    def op_solve(self, which: str, y, x, transpose=False):
        """which 'K1' or 'K1t': x = K^{-1} y (or K^{-T} y)."""
        w = 1 if which == "K1" else 0
        n = self.n_e if w else self.n_h
        _check(load_library().kmx_op_solve(self._h, w, int(bool(transpose)), _dptr(y, n, "y"), _dptr(x, n, "x"),
                                           _stream()))

    # ---- the first scheme (1-form mass solves) ---------------------------
    def op_mass1(self, which: str, x, y):
        """which 'E' (M^1_eps on X^1_{h,0}) or 'H' (M~^1_mu on X~^1)."""
        w = 0 if which == "E" else 1
        n = self.n_e if w == 0 else self.n_h
        _check(load_library().kmx_op_mass1(self._h, w, _dptr(x, n, "x"), _dptr(y, n, "y"), _stream()))

    def solve_mass1(self, which: str, y, x, tol=1e-13, max_iter=500) -> int:
        """x = M^{-1} y from the guess in x; returns the CG iterations."""
        w = 0 if which == "E" else 1
        n = self.n_e if w == 0 else self.n_h
        it = ctypes.c_int(0)
        _check(load_library().kmx_solve_mass1(self._h, w, _dptr(y, n, "y"), _dptr(x, n, "x"), float(tol),
                                              int(max_iter), ctypes.byref(it), _stream()))
        return it.value

    def half_step_scheme1(self, which: str, x, out, alpha, tol=1e-13, max_iter=500) -> int:
        """which 'H': out += alpha M~^{-1} K~1^T D^1 x; which 'E': out += alpha M^{-1} K1^T D~^1 x."""
        w = 0 if which == "E" else 1
        n_x, n_o = (self.n_h, self.n_e) if w == 0 else (self.n_e, self.n_h)
        it = ctypes.c_int(0)
        _check(load_library().kmx_half_step_scheme1(self._h, w, _dptr(x, n_x, "x"), _dptr(out, n_o, "out"),
                                                    float(alpha), float(tol), int(max_iter), ctypes.byref(it),
                                                    _stream()))
        return it.value

    def step_scheme1(self, e, h, dt, nsteps=1, tol=1e-13, max_iter=500):
        """nsteps leapfrog steps of the first scheme; returns the summed CG
        iterations (e solves, h solves)."""
        it = (ctypes.c_int * 2)()
        _check(load_library().kmx_step_scheme1(self._h, _dptr(e, self.n_e, "e"), _dptr(h, self.n_h, "h"),
                                               float(dt), int(nsteps), float(tol), int(max_iter),
                                               ctypes.cast(it, ctypes.c_void_p), _stream()))
        return int(it[0]), int(it[1])

    def project_E1(self, E_qp, e, tol=1e-13):
        """e^0 = L^2_eps projection of E0 (physical field at the quadrature
        points, (n_qp, 3) host array) onto X^1_{h,0}."""
        keep, ptr = _hptr(E_qp, 3 * self.n_qp)
        _check(load_library().kmx_project_E1(self._h, ptr, _dptr(e, self.n_e, "e"), float(tol), _stream()))

    def graph_scheme1(self, e, h, dt, nsteps, iters_e, iters_h) -> GraphScheme1:
        """Capture nsteps first-scheme steps with fixed CG iteration counts."""
        return GraphScheme1(self, e, h, dt, nsteps, iters_e, iters_h)

    def cfl_scheme1(self, max_iter=2000, tol=1e-10, cg_tol=1e-12) -> float:
        out = ctypes.c_double()
        _check(load_library().kmx_cfl_scheme1(self._h, int(max_iter), float(tol), float(cg_tol),
                                              ctypes.byref(out)))
        return out.value

    def set_refinement(self, steps: int):
        """Number of FP64-residual corrections of mixed-precision solves."""
        _check(load_library().kmx_set_refinement(self._h, int(steps)))

    # ---- execution plans --------------------------------------------------
    def set_plan(self, kind: int, threads: int = 768):
        _check(load_library().kmx_set_plan(self._h, int(kind), int(threads)))

    def plan(self):
        k, t = ctypes.c_int(), ctypes.c_int()
        _check(load_library().kmx_get_plan(self._h, ctypes.byref(k), ctypes.byref(t)))
        return k.value, t.value

    def tune(self, batch: int, dt: float, probe_steps: int = 5, J: "Source | None" = None):
        """Time the candidate plans and keep the fastest; returns the mean ms
        per step of each candidate (None where it does not apply)."""
        ms = np.zeros(TUNE_CANDIDATES)
        _check(load_library().kmx_tune(self._h, int(batch), int(probe_steps), None if J is None else J._h,
                                       float(dt), ctypes.c_void_p(ms.ctypes.data), _stream()))
        return [None if m < 0 else float(m) for m in ms]

    # ---- graph-captured stepping --------------------------------------------
    def graph(self, E, H, dt, nsteps, J=None, batch=1, flags=0, energy=None) -> Graph:
        return Graph(self, E, H, dt, nsteps, J, batch, flags, energy)

    def set_time(self, t):
        _check(load_library().kmx_set_time(self._h, float(t), _stream()))

    def get_time(self) -> float:
        t = ctypes.c_double()
        _check(load_library().kmx_get_time(self._h, ctypes.byref(t), _stream()))
        return t.value

    # ---- probes and the adjoint ------------------------------------------
    def probes(self, pos) -> Probes:
        return Probes(self, pos)

    def probe_eval(self, pr: Probes, e, out):
        _check(load_library().kmx_probe_eval(self._h, pr._h, _dptr(e, self.n_e, "e"),
                                             _dptr(out, 3 * pr.n, "out"), _stream()))

    def probe_forward(self, pr: Probes, J: "Source | None", dt, nsteps, obs):
        _check(load_library().kmx_probe_forward(self._h, pr._h, None if J is None else J._h, float(dt), int(nsteps),
                                                _dptr(obs, nsteps * 3 * pr.n, "obs"), _stream()))

    def probe_forward_noalloc(self, pr: Probes, J: "Source | None", dt, nsteps, obs):
        _check(load_library().kmx_probe_forward_noalloc(self._h, pr._h, None if J is None else J._h, float(dt),
                                                        int(nsteps), _dptr(obs, nsteps * 3 * pr.n, "obs"),
                                                        _stream()))

    def adjoint(self, pr: Probes, J: "Source | None", data, dt, nsteps, checkpoint_every, grad) -> float:
        loss = ctypes.c_double()
        _check(load_library().kmx_adjoint(self._h, pr._h, None if J is None else J._h,
                                          _dptr(data, nsteps * 3 * pr.n, "data"), float(dt), int(nsteps),
                                          int(checkpoint_every), ctypes.byref(loss),
                                          _dptr(grad, self.N ** 3, "grad"), _stream()))
        return loss.value

    def profile_begin(self, capacity=100000):
        _check(load_library().kmx_profile_begin(self._h, int(capacity)))

    def profile_select(self, kinds):
        """Bracket only the named kernel kinds (names of PROFILE_KINDS)."""
        mask = 0
        for k in kinds:
            mask |= 1 << PROFILE_KINDS.index(k)
        _check(load_library().kmx_profile_select(self._h, mask))

    def profile_end(self) -> dict:
        """{kind: (total_ms, launches)} for the launches since profile_begin."""
        ms = np.zeros(len(PROFILE_KINDS))
        cnt = np.zeros(len(PROFILE_KINDS), dtype=np.int32)
        _check(load_library().kmx_profile_end(self._h, ctypes.c_void_p(ms.ctypes.data),
                                              ctypes.c_void_p(cnt.ctypes.data)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_KINDS)}

    # ---- non-homogeneous tangential data (Section 3.5) ---------------------
    @property
    def n_ef(self) -> int:
        out = ctypes.c_int64()
        _check(load_library().kmx_sizes_full(self._h, ctypes.byref(out)))
        return out.value

    def lift_boundary(self, Eh_faces) -> np.ndarray:
        """Boundary coefficients (a vector of X^1_h) fitted to the pulled-back
        tangential data at the face Gauss points (kmx_lift_boundary layout)."""
        q = self.N * (self.p + 1)
        a, ptr = _hptr(Eh_faces, 6 * q * q * 3, name="Eh_faces")
        out = np.zeros(self.n_ef)
        it = ctypes.c_int()
        _check(load_library().kmx_lift_boundary(self._h, ptr, ctypes.c_void_p(out.ctypes.data), ctypes.byref(it)))
        return out

    def set_lifting(self, eb_full, amp, omega, phase):
        """Lifting terms sum_j amp_j cos(omega_j t + phase_j) E_b^j (eb_full: one
        vector of X^1_h per term); no terms removes it."""
        eb = np.ascontiguousarray(np.asarray(eb_full, dtype=np.float64).reshape(-1))
        n = len(np.atleast_1d(amp))
        if n and eb.size != n * self.n_ef:
            raise ValueError(f"eb_full has {eb.size} entries, needs {n} x {self.n_ef}")
        arrs = [np.ascontiguousarray(np.atleast_1d(np.asarray(v, dtype=np.float64))) for v in (amp, omega, phase)]
        ptr = lambda x: ctypes.c_void_p(x.ctypes.data) if x.size else None  # noqa: E731
        _check(load_library().kmx_set_lifting(self._h, int(n), ptr(eb), *(ptr(x) for x in arrs)))

    def op_pairing(self, which: str, x, y):
        w = 1 if which == "K1" else 0
        n = self.n_e if w else self.n_h
        _check(load_library().kmx_op_pairing(self._h, w, _dptr(x, n, "x"), _dptr(y, n, "y"), _stream()))


class ProbeMisfitProblem:
    """Probe-misfit inverse problem in the per-element permittivity: zero initial
    fields, point dipoles (dict of arrays pos, moment, t0, sigma, amp), probes at
    parametric points, observed data (device tensor, nsteps x n_probes x 3)."""

    def __init__(self, space: Space, dipoles: dict, probe_pos, data, dt, nsteps, checkpoint_every=50, mu=None):
        self.space, self.dip, self.data = space, dipoles, data
        self.dt, self.nsteps, self.ckpt = float(dt), int(nsteps), int(checkpoint_every)
        self.mu = mu
        self.probes = space.probes(probe_pos)

    def _source(self):
        d = self.dip
        return self.space.source(d["pos"], d["moment"], d["t0"], d["sigma"], d["amp"])

    def loss_and_grad(self, eps):
        """(loss, dL/deps as a device tensor of shape (N, N, N))."""
        import torch
        N = self.space.N
        self.space.set_materials(eps=np.asarray(eps, dtype=float).reshape(-1), mu=self.mu)
        J = self._source()
        grad = torch.zeros(N ** 3, dtype=torch.float64, device="cuda")
        loss = self.space.adjoint(self.probes, J, self.data, self.dt, self.nsteps, self.ckpt, grad)
        return loss, grad.reshape(N, N, N)

    def observe(self, eps):
        """Probe values of a forward run with the given eps (device tensor)."""
        import torch
        self.space.set_materials(eps=np.asarray(eps, dtype=float).reshape(-1), mu=self.mu)
        obs = torch.zeros(self.nsteps, self.probes.n, 3, dtype=torch.float64, device="cuda")
        self.space.probe_forward(self.probes, self._source(), self.dt, self.nsteps, obs)
        return obs


def _misfit_function():
    import torch

    class ProbeMisfit(torch.autograd.Function):
        """loss = ProbeMisfit.apply(eps, problem): forward and adjoint run on the
        device through kmx_adjoint (checkpointed); backward returns dL/deps."""

        @staticmethod
        def forward(ctx, eps, problem):
            loss, grad = problem.loss_and_grad(eps.detach().cpu().numpy())
            ctx.save_for_backward(grad.to(eps.device))
            return torch.tensor(loss, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, grad_out):
            (grad,) = ctx.saved_tensors
            return grad_out * grad, None

    return ProbeMisfit


def probe_misfit(eps, problem: ProbeMisfitProblem):
    """Differentiable probe misfit (torch.autograd.Function over the adjoint)."""
    return _misfit_function().apply(eps, problem)
