"""Regularized least squares (Section V-A, eqs. (4)-(5)): the closed form.

``minimize (1/2)||A x - b||^2 + (lam/2)||x||^2`` has the solution
``x* = (lam I + A^T A)^{-1} A^T b``, the linear system the paper solves by
conjugate gradients.  (The paper prints the regulariser as ``lam ||x||^2``
next to this closed form; the closed form is taken as authoritative, i.e. the
regulariser is ``(lam/2)||x||^2``.)  The oracle computes ``x*`` by a direct
factorisation in float64: dense Cholesky of ``lam I + A^T A`` for a dense
``A``; for the full convolution ``A x = c * x``, a banded Cholesky of
``lam I + C^T C`` (``C^T C`` is banded Toeplitz).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .program import gram_toeplitz_solver


def regls_rhs(data: dict) -> np.ndarray:
    """``A^T b`` (dense product, or the valid correlation of ``b`` with ``c``)."""
    if data["kind"] == "dense":
        return np.asarray(data["A"]).T @ np.asarray(data["b"])
    return np.correlate(np.asarray(data["b"]), np.asarray(data["c"]), mode="valid")


def regls_apply_normal(data: dict, x: np.ndarray) -> np.ndarray:
    """``(lam I + A^T A) x``."""
    lam = float(data["lam"])
    if data["kind"] == "dense":
        A = np.asarray(data["A"])
        return lam * x + A.T @ (A @ x)
    c = np.asarray(data["c"])
    return lam * x + np.correlate(np.convolve(c, x), c, mode="valid")


def regls_solution(data: dict) -> np.ndarray:
    """The closed form ``(lam I + A^T A)^{-1} A^T b`` (eq. (5))."""
    lam = float(data["lam"])
    rhs = regls_rhs(data)
    if data["kind"] == "dense":
        A = np.asarray(data["A"])
        cf = sla.cho_factor(lam * np.eye(A.shape[1]) + A.T @ A, lower=False, check_finite=False)
        return sla.cho_solve(cf, rhs, check_finite=False)
    c = np.asarray(data["c"])
    n = rhs.shape[0]
    return gram_toeplitz_solver(c, n, lam, 1.0)(rhs)


def regls_objective(data: dict, x: np.ndarray) -> float:
    """``(1/2)||A x - b||^2 + (lam/2)||x||^2``."""
    lam = float(data["lam"])
    if data["kind"] == "dense":
        r = np.asarray(data["A"]) @ x - np.asarray(data["b"])
    else:
        r = np.convolve(np.asarray(data["c"]), x) - np.asarray(data["b"])
    return float(0.5 * (r @ r) + 0.5 * lam * (x @ x))
