"""Tensor-product spline spaces of 1- and 2-forms (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

Section 2.3 and Section 4.1 (the component spaces listed for K1 and K~1): the
unknowns are

  e in X^1_{h,0} (primal 1-form)   component c: derivative basis Pd along axis c, Pv across
  b in X^2_{h,0} (primal 2-form)   component c: Pv along axis c, Pd across
  h in X~^1      (dual 1-form)     component c: Dd along axis c, Dv across
  d in X~^2      (dual 2-form)     component c: Dv along axis c, Dd across
and, for non-homogeneous boundary data (Section 3.5), the whole primal spaces
  X^1_h ('Ef')                     component c: Pd along axis c, Pf across
  X^2_h ('Bf')                     component c: Pf along axis c, Pd across

A vector stores its three components one after the other; inside a component
the x index runs fastest (the vec convention of Section 4.2), i.e. a component
is a C-ordered array of shape (n_z, n_y, n_x).
"""
from __future__ import annotations

import numpy as np

from .splines import Axis

SPACE_TAGS = {
    "E": lambda c, a: "Pd" if a == c else "Pv",
    "B": lambda c, a: "Pv" if a == c else "Pd",
    "H": lambda c, a: "Dd" if a == c else "Dv",
    "D": lambda c, a: "Dv" if a == c else "Dd",
    # the whole primal spaces X^1_h and X^2_h, boundary functions kept
    # (non-homogeneous boundary data, Section 3.5)
    "Ef": lambda c, a: "Pd" if a == c else "Pf",
    "Bf": lambda c, a: "Pf" if a == c else "Pd",
}


def comp_tags(space: str, c: int):
    """(tag_x, tag_y, tag_z) of component c."""
    f = SPACE_TAGS[space]
    return tuple(f(c, a) for a in range(3))


def comp_shape(axis: Axis, space: str, c: int):
    """Array shape (n_z, n_y, n_x) of component c."""
    tx, ty, tz = comp_tags(space, c)
    return (axis.dims[tz], axis.dims[ty], axis.dims[tx])


def space_size(axis: Axis, space: str) -> int:
    return sum(int(np.prod(comp_shape(axis, space, c))) for c in range(3))


def split(axis: Axis, space: str, v: np.ndarray):
    """View a flat vector as its three component arrays."""
    out, o = [], 0
    for c in range(3):
        sh = comp_shape(axis, space, c)
        n = int(np.prod(sh))
        out.append(v[o:o + n].reshape(sh))
        o += n
    if o != v.size:
        raise ValueError(f"vector of length {v.size} is not in space {space}")
    return out


def join(parts) -> np.ndarray:
    return np.concatenate([np.asarray(x).ravel() for x in parts])
