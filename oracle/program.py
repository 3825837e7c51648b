"""Cone programs of the paper's examples, written out explicitly (float64).

Standard form (eq. (1), Section II-A) in the sign convention
``minimize c^T x  s.t.  A x + s = b,  s in K`` -- the paper's ``A x + b in K``
with ``A -> -A``.  ``K`` is ``R_+^l x SOC(q_1) x ...`` with rows in that order.

Each constructor returns a :class:`ConeProgram` that can apply ``A`` and ``A^T``
(through library primitives: ``numpy.convolve``/``correlate`` and dense matrix
products), build ``A`` explicitly for small sizes, and factor
``K = I + A^T A`` directly.  The factorisation uses the block-diagonal form of
``K`` that each canonical form has (stated per constructor and checked against
the explicit ``I + A^T A`` in the tests).
"""
from __future__ import annotations

from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla


class Factor:
    """Direct solver for ``K v = r`` with ``K = I + A^T A``."""

    def __init__(self, solve: Callable[[np.ndarray], np.ndarray], kind: str):
        self._solve = solve
        self.kind = kind

    def solve(self, r: np.ndarray) -> np.ndarray:
        return self._solve(np.asarray(r, dtype=np.float64))


class ConeProgram:
    """``minimize c^T x s.t. A x + s = b, s in R_+^l x SOC(q...)``."""

    def __init__(self, n: int, m: int, b: np.ndarray, c: np.ndarray, l: int, q: Sequence[int],
                 apply: Callable, apply_T: Callable, explicit: Callable,
                 factor: Callable, family: str, data: Optional[dict] = None,
                 blocks: Sequence[tuple] = (), apply_sq: Optional[Callable] = None,
                 scaled_factor: Optional[Callable] = None):
        self.n, self.m = int(n), int(m)
        self.b = np.asarray(b, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        self.l = int(l)
        self.q: List[int] = [int(v) for v in q]
        self._apply, self._apply_T = apply, apply_T
        self._explicit, self._factor = explicit, factor
        self.family = family
        self.data = data or {}
        # (row0, rows, col0, cols) of every nonzero block of A, the product of
        # A's entrywise square with a vector, and the factorisation of
        # I + (D A E)^T (D A E) for diagonal scalings constant on the blocks
        self.blocks = [tuple(int(v) for v in bl) for bl in blocks]
        self._apply_sq, self._scaled_factor = apply_sq, scaled_factor
        if self.b.shape != (self.m,) or self.c.shape != (self.n,):
            raise ValueError("b/c shape mismatch")
        if self.l + sum(self.q) != self.m:
            raise ValueError("cone sizes must cover all m rows")

    def A(self, x: np.ndarray) -> np.ndarray:
        return self._apply(np.asarray(x, dtype=np.float64))

    def AT(self, y: np.ndarray) -> np.ndarray:
        return self._apply_T(np.asarray(y, dtype=np.float64))

    def explicit(self) -> np.ndarray:
        """Dense ``m x n`` matrix ``A`` (small sizes only)."""
        return self._explicit()

    def factor(self) -> Factor:
        return self._factor()

    def A_sq(self, x: np.ndarray) -> np.ndarray:
        """``(A o A) x``: ``A`` with every entry squared, applied to ``x``."""
        return self._apply_sq(np.asarray(x, dtype=np.float64))

    def scaled_factor(self, D: np.ndarray, E: np.ndarray) -> Factor:
        """Factorisation of ``I + (D A E)^T (D A E)`` for diagonal ``D`` (rows) and
        ``E`` (columns) that are constant on each block of ``A``."""
        return self._scaled_factor(np.asarray(D, dtype=np.float64), np.asarray(E, dtype=np.float64))


def _require_constant(v: np.ndarray, ranges) -> None:
    for lo, hi in ranges:
        if hi > lo and np.any(v[lo:hi] != v[lo]):
            raise ValueError("scaling is not constant on a block of the operator")


def _dense_factor(M: np.ndarray) -> Factor:
    """Cholesky of the SPD matrix ``M``."""
    cf = sla.cho_factor(M, lower=False, check_finite=False)
    return Factor(lambda r: sla.cho_solve(cf, r, check_finite=False), "dense")


def dense_program(A: np.ndarray, b: np.ndarray, c: np.ndarray, l: int,
                  q: Sequence[int] = ()) -> ConeProgram:
    """A generic cone program with an explicit dense ``A`` (used for small LPs/SOCPs)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape

    def factor():
        return _dense_factor(np.eye(n) + A.T @ A)

    def scaled_factor(D, E):
        As = D[:, None] * A * E[None, :]
        return _dense_factor(np.eye(n) + As.T @ As)

    A2 = A * A
    return ConeProgram(n, m, b, c, l, q, lambda x: A @ x, lambda y: A.T @ y,
                       lambda: A.copy(), factor, "dense", {"A": A},
                       blocks=[(0, m, 0, n)], apply_sq=lambda x: A2 @ x,
                       scaled_factor=scaled_factor)


def conv_matrix(c: np.ndarray, n: int) -> np.ndarray:
    """Explicit ``(n+k-1) x n`` full-convolution matrix: column j is c shifted by j."""
    k = c.shape[0]
    C = np.zeros((n + k - 1, n))
    for j in range(n):
        C[j:j + k, j] = c
    return C


def autocorrelation(c: np.ndarray) -> np.ndarray:
    """``r_d = sum_j c_j c_{j+d}`` for lags ``d = 0..k-1``."""
    k = c.shape[0]
    return np.array([np.dot(c[:k - d], c[d:]) for d in range(k)])


def gram_toeplitz_solver(c: np.ndarray, n: int, diag: float, w: float) -> Callable:
    """Solver for ``(diag I + w C^T C) v = r`` with ``C`` the full convolution by
    ``c`` on ``n`` inputs.  ``C^T C`` is the symmetric Toeplitz matrix of the
    kernel autocorrelation (no boundary terms: the convolution is full), so the
    matrix is factored by a banded Cholesky of half-bandwidth ``k - 1``."""
    k = c.shape[0]
    ac = autocorrelation(c)
    kd = min(k - 1, n - 1)
    ab = np.zeros((kd + 1, n))          # upper banded storage
    for d in range(kd + 1):
        ab[kd - d, d:] = w * ac[d]
    ab[kd, :] += diag
    cb = sla.cholesky_banded(ab, lower=False, check_finite=False)
    return lambda r: sla.cho_solve_banded((cb, False), r, check_finite=False)


def deconv_program(c: np.ndarray, b_obs: np.ndarray) -> ConeProgram:
    """Nonnegative deconvolution (Section V-C, eq. 6) as a cone program.

    ``minimize ||c * x - b||_2 s.t. x >= 0`` with full convolution (``b`` has
    ``n + k - 1`` entries, as ``c in R^n, b in R^{2n-1}`` in the paper).
    Variables ``(x, t)``; rows ``[x >= 0 (n) | SOC(t, c*x - b) (n+k)]``:

        A = [[-I, 0], [0, -1], [-C, 0]],  b = [0, 0, -b_obs],  c = [0, 1].

    With ``n`` the signal length and a length-``n`` kernel this gives ``n+1``
    variables and ``3n`` constraints, the counts of Table III.
    ``I + A^T A = blockdiag(2I + C^T C, 2)`` where ``C^T C`` is the symmetric
    Toeplitz matrix of the kernel autocorrelation (no boundary terms, because the
    convolution is full); it is factored as a banded Cholesky of half-bandwidth
    ``k-1``.
    """
    c = np.asarray(c, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    k = c.shape[0]
    n = b_obs.shape[0] - k + 1
    if n < 1:
        raise ValueError("observation shorter than kernel")
    nv = n + 1
    m = n + 1 + (n + k - 1)
    b = np.concatenate([np.zeros(n + 1), -b_obs])
    cc = np.zeros(nv)
    cc[n] = 1.0

    def apply(z):
        x, t = z[:n], z[n]
        return np.concatenate([-x, [-t], -np.convolve(c, x)])

    def apply_T(y):
        out = np.empty(nv)
        out[:n] = -y[:n] - np.correlate(y[n + 1:], c, mode="valid")
        out[n] = -y[n]
        return out

    def explicit():
        A = np.zeros((m, nv))
        A[:n, :n] = -np.eye(n)
        A[n, n] = -1.0
        A[n + 1:, :n] = -conv_matrix(c, n)
        return A

    def banded(p, q, r):
        # I + A^T A for A = [[-p I, 0], [0, -q], [-r C, 0]]:
        # blockdiag((1 + p^2) I + r^2 C^T C, 1 + q^2)
        gram = gram_toeplitz_solver(c, n, 1.0 + p * p, r * r)
        tt = 1.0 + q * q

        def solve(rhs):
            out = np.empty(nv)
            out[:n] = gram(rhs[:n])
            out[n] = rhs[n] / tt
            return out
        return Factor(solve, "banded")

    def scaled_factor(D, E):
        _require_constant(D, [(0, n), (n, m)])
        _require_constant(E, [(0, n), (n, nv)])
        return banded(D[0] * E[0], D[n] * E[n], D[n + 1] * E[0])

    c2 = c * c

    def apply_sq(z):
        return np.concatenate([z[:n], [z[n]], np.convolve(c2, z[:n])])

    return ConeProgram(nv, m, b, cc, n, [n + k], apply, apply_T, explicit,
                       lambda: banded(1.0, 1.0, 1.0), "deconv",
                       {"c": c, "b_obs": b_obs, "n": n, "k": k},
                       blocks=[(0, n, 0, n), (n, 1, n, 1), (n + 1, n + k - 1, 0, n)],
                       apply_sq=apply_sq, scaled_factor=scaled_factor)


def lasso_program(A: np.ndarray, b_obs: np.ndarray, lam: float) -> ConeProgram:
    """Lasso (Section V-B, eq. 5) as a cone program.

    ``minimize (1/2)||A x - b||^2 + lam ||x||_1``.  Variables ``(x, t, u)`` with
    ``|x| <= t`` (``2n`` nonnegative rows ``t - x``, ``t + x``) and
    ``||A x - b||^2 <= u`` written as the second-order cone
    ``(u + 1, 2(A x - b), u - 1)`` of size ``m + 2``; objective
    ``lam 1^T t + u/2``.  For ``A`` of size ``m x n`` this gives ``2n + 1``
    variables, ``2n + m + 2`` constraints and ``4n + mn + 2`` nonzeros, the
    counts of Table II.  ``I + A_c^T A_c = blockdiag(3I + 4 A^T A, 3I, 3)``.
    """
    A = np.asarray(A, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    m0, n0 = A.shape
    nv = 2 * n0 + 1
    m = 2 * n0 + m0 + 2
    b = np.concatenate([np.zeros(2 * n0), [1.0], -2.0 * b_obs, [-1.0]])
    cc = np.concatenate([np.zeros(n0), np.full(n0, float(lam)), [0.5]])
    i_mid = 2 * n0 + 1

    def apply(z):
        x, t, u = z[:n0], z[n0:2 * n0], z[2 * n0]
        return np.concatenate([x - t, -x - t, [-u], -2.0 * (A @ x), [-u]])

    def apply_T(y):
        y1, y2 = y[:n0], y[n0:2 * n0]
        out = np.empty(nv)
        out[:n0] = y1 - y2 - 2.0 * (A.T @ y[i_mid:i_mid + m0])
        out[n0:2 * n0] = -y1 - y2
        out[2 * n0] = -y[2 * n0] - y[m - 1]
        return out

    def explicit():
        Ac = np.zeros((m, nv))
        I = np.eye(n0)
        Ac[:n0, :n0] = I
        Ac[:n0, n0:2 * n0] = -I
        Ac[n0:2 * n0, :n0] = -I
        Ac[n0:2 * n0, n0:2 * n0] = -I
        Ac[2 * n0, 2 * n0] = -1.0
        Ac[i_mid:i_mid + m0, :n0] = -2.0 * A
        Ac[m - 1, 2 * n0] = -1.0
        return Ac

    def blockdiag(dx, dt, du, r):
        # I + A^T A when the x, t and u columns carry the row-group weights
        # dx = sum of squared x coefficients in the nonnegative rows (and dt, du
        # likewise) and the dense block is -r A: blockdiag((1 + dx) I + r^2 A^T A,
        # (1 + dt) I, 1 + du); the x-t cross terms of the rows t - x and t + x cancel.
        cf = sla.cho_factor((1.0 + dx) * np.eye(n0) + r * r * (A.T @ A), lower=False,
                            check_finite=False)

        def solve(rhs):
            out = np.empty(nv)
            out[:n0] = sla.cho_solve(cf, rhs[:n0], check_finite=False)
            out[n0:2 * n0] = rhs[n0:2 * n0] / (1.0 + dt)
            out[2 * n0] = rhs[2 * n0] / (1.0 + du)
            return out
        return Factor(solve, "lasso-blockdiag")

    def scaled_factor(D, E):
        _require_constant(D, [(0, n0), (n0, 2 * n0), (2 * n0, m)])
        _require_constant(E, [(0, n0), (n0, 2 * n0), (2 * n0, nv)])
        d1, d2, d3 = D[0], D[n0], D[2 * n0]
        ex, et, eu = E[0], E[n0], E[2 * n0]
        if d1 != d2:
            raise ValueError("rows t - x and t + x must carry the same scale")
        return blockdiag(2.0 * (d1 * ex) ** 2, 2.0 * (d1 * et) ** 2, 2.0 * (d3 * eu) ** 2,
                         2.0 * d3 * ex)

    A2 = A * A

    def apply_sq(z):
        x, t, u = z[:n0], z[n0:2 * n0], z[2 * n0]
        return np.concatenate([x + t, x + t, [u], 4.0 * (A2 @ x), [u]])

    return ConeProgram(nv, m, b, cc, 2 * n0, [m0 + 2], apply, apply_T, explicit,
                       lambda: blockdiag(2.0, 2.0, 2.0, 2.0), "lasso",
                       {"A": A, "b_obs": b_obs, "lam": float(lam), "n": n0, "m": m0},
                       blocks=[(0, n0, 0, n0), (0, n0, n0, n0), (n0, n0, 0, n0), (n0, n0, n0, n0),
                               (2 * n0, 1, 2 * n0, 1), (i_mid, m0, 0, n0), (m - 1, 1, 2 * n0, 1)],
                       apply_sq=apply_sq, scaled_factor=scaled_factor)


def conv_lasso_program(c: np.ndarray, b_obs: np.ndarray, lam: float) -> ConeProgram:
    """Lasso with a convolution operator (Section V-B, the convolution column
    of Table II): ``minimize (1/2)||c * x - b||^2 + lam ||x||_1`` in the cone form
    of :func:`lasso_program` with the dense block replaced by the full
    convolution ``C`` (``n + k - 1`` rows).  ``2n + 1`` variables,
    ``2n + (n + k - 1) + 2`` constraints and ``4n + kn + 2`` nonzeros;
    ``I + A_c^T A_c = blockdiag(3I + 4 C^T C, 3I, 3)`` with ``C^T C`` banded
    Toeplitz (banded Cholesky).
    """
    c = np.asarray(c, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    k = c.shape[0]
    n0 = b_obs.shape[0] - k + 1
    if n0 < 1:
        raise ValueError("observation shorter than kernel")
    m0 = n0 + k - 1
    nv = 2 * n0 + 1
    m = 2 * n0 + m0 + 2
    b = np.concatenate([np.zeros(2 * n0), [1.0], -2.0 * b_obs, [-1.0]])
    cc = np.concatenate([np.zeros(n0), np.full(n0, float(lam)), [0.5]])
    i_mid = 2 * n0 + 1

    def apply(z):
        x, t, u = z[:n0], z[n0:2 * n0], z[2 * n0]
        return np.concatenate([x - t, -x - t, [-u], -2.0 * np.convolve(c, x), [-u]])

    def apply_T(y):
        y1, y2 = y[:n0], y[n0:2 * n0]
        out = np.empty(nv)
        out[:n0] = y1 - y2 - 2.0 * np.correlate(y[i_mid:i_mid + m0], c, mode="valid")
        out[n0:2 * n0] = -y1 - y2
        out[2 * n0] = -y[2 * n0] - y[m - 1]
        return out

    def explicit():
        Ac = np.zeros((m, nv))
        I = np.eye(n0)
        Ac[:n0, :n0] = I
        Ac[:n0, n0:2 * n0] = -I
        Ac[n0:2 * n0, :n0] = -I
        Ac[n0:2 * n0, n0:2 * n0] = -I
        Ac[2 * n0, 2 * n0] = -1.0
        Ac[i_mid:i_mid + m0, :n0] = -2.0 * conv_matrix(c, n0)
        Ac[m - 1, 2 * n0] = -1.0
        return Ac

    def blockdiag(dx, dt, du, r):
        # as in lasso_program, with the Gram block r^2 C^T C banded Toeplitz
        gram = gram_toeplitz_solver(c, n0, 1.0 + dx, r * r)

        def solve(rhs):
            out = np.empty(nv)
            out[:n0] = gram(rhs[:n0])
            out[n0:2 * n0] = rhs[n0:2 * n0] / (1.0 + dt)
            out[2 * n0] = rhs[2 * n0] / (1.0 + du)
            return out
        return Factor(solve, "conv-lasso-banded")

    def scaled_factor(D, E):
        _require_constant(D, [(0, n0), (n0, 2 * n0), (2 * n0, m)])
        _require_constant(E, [(0, n0), (n0, 2 * n0), (2 * n0, nv)])
        d1, d2, d3 = D[0], D[n0], D[2 * n0]
        ex, et, eu = E[0], E[n0], E[2 * n0]
        if d1 != d2:
            raise ValueError("rows t - x and t + x must carry the same scale")
        return blockdiag(2.0 * (d1 * ex) ** 2, 2.0 * (d1 * et) ** 2, 2.0 * (d3 * eu) ** 2,
                         2.0 * d3 * ex)

    c2 = c * c

    def apply_sq(z):
        x, t, u = z[:n0], z[n0:2 * n0], z[2 * n0]
        return np.concatenate([x + t, x + t, [u], 4.0 * np.convolve(c2, x), [u]])

    return ConeProgram(nv, m, b, cc, 2 * n0, [m0 + 2], apply, apply_T, explicit,
                       lambda: blockdiag(2.0, 2.0, 2.0, 2.0), "lasso_conv",
                       {"c": c, "b_obs": b_obs, "lam": float(lam), "n": n0, "m": m0, "k": k},
                       blocks=[(0, n0, 0, n0), (0, n0, n0, n0), (n0, n0, 0, n0), (n0, n0, n0, n0),
                               (2 * n0, 1, 2 * n0, 1), (i_mid, m0, 0, n0), (m - 1, 1, 2 * n0, 1)],
                       apply_sq=apply_sq, scaled_factor=scaled_factor)
