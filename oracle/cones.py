"""Euclidean projections onto the cones of the paper's cone programs.

The cone ``K`` of eq. (1) is, for the deconvolution (eq. 6) and lasso (eq. 5)
examples, a product of one nonnegative orthant and second-order cones.  Both are
self-dual, so the dual cone ``K*`` used by the embedding equals ``K``.

Closed forms (textbook, Boyd & Vandenberghe; Parikh & Boyd):

* nonnegative orthant: ``max(v, 0)`` elementwise;
* second-order cone ``{(t, z) : ||z||_2 <= t}``: ``(t, z)`` if ``||z|| <= t``;
  ``0`` if ``||z|| <= -t``; otherwise ``((t + ||z||)/2) * (1, z/||z||)``.
"""
from __future__ import annotations

import numpy as np


def proj_nonneg(v: np.ndarray) -> np.ndarray:
    return np.maximum(v, 0.0)


def proj_soc(v: np.ndarray) -> np.ndarray:
    """Project ``v = (t, z)`` onto the second-order cone of dimension ``len(v)``."""
    v = np.asarray(v, dtype=np.float64)
    t = v[0]
    z = v[1:]
    nz = float(np.linalg.norm(z)) if z.size else 0.0
    if nz <= t:
        return v.copy()
    if nz <= -t:
        return np.zeros_like(v)
    a = 0.5 * (t + nz)
    out = np.empty_like(v)
    out[0] = a
    out[1:] = (a / nz) * z
    return out


def proj_cone(y: np.ndarray, l: int, q) -> np.ndarray:
    """Project onto ``R_+^l x SOC(q[0]) x SOC(q[1]) x ...`` (rows in that order)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    out[:l] = proj_nonneg(y[:l])
    off = l
    for qi in q:
        out[off:off + qi] = proj_soc(y[off:off + qi])
        off += qi
    if off != y.shape[0]:
        raise ValueError("cone sizes do not cover the vector")
    return out


def in_cone(y: np.ndarray, l: int, q, tol: float = 0.0) -> bool:
    """Membership test with an absolute slack ``tol``."""
    if np.any(y[:l] < -tol):
        return False
    off = l
    for qi in q:
        seg = y[off:off + qi]
        if np.linalg.norm(seg[1:]) > seg[0] + tol:
            return False
        off += qi
    return True
