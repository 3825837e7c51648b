"""Regularized least squares by matrix-free conjugate gradients (Section V-A).

``minimize (1/2)||A x - b||^2 + (lam/2)||x||^2`` has the solution
``x* = (lam I + A^T A)^{-1} A^T b`` (eq. (5)); the paper solves this system by
CG until ``||(lam I + A^T A) x - A^T b|| <= tol ||A^T b||``.  With
``A' = A / sqrt(lam)`` the system is ``(I + A'^T A') x = A'^T (b / sqrt(lam))``
-- the library's CG on ``I + A^T A`` (``cgs_solver_normal_solve``) with the
operator scaled at upload, and the same relative stop test.  The right-hand
side is one adjoint apply of the library; every product, dot and update runs
in its kernels.  ``A`` is a dense matrix or a full convolution.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from ._lib import FP64, Operator, Settings, Solver


class RegLS:
    """The operator and solver state of one regularized least-squares problem."""

    def __init__(self, lam: float, A=None, taps=None, n: Optional[int] = None,
                 precision: int = FP64, stream=None):
        if (A is None) == (taps is None):
            raise ValueError("give exactly one of A (dense) or taps (convolution)")
        if not lam > 0.0:
            raise ValueError("lam must be positive")
        self.lam = float(lam)
        s = 1.0 / math.sqrt(self.lam)
        if A is not None:
            A = np.asarray(A, dtype=np.float64)
            m, n = A.shape
            op = Operator(m, n)
            op.add_dense(0, 0, A, s)
        else:
            taps = np.asarray(taps, dtype=np.float64)
            if n is None:
                raise ValueError("n (signal length) is needed for a convolution")
            m = n + taps.shape[0] - 1
            op = Operator(m, n)
            op.add_conv(0, 0, taps, n, s)
        self.m, self.n = m, n
        self.op = op
        # the cone part is never used by the CG entry points: all rows nonnegative
        st = Settings.make(precision=precision, normalize=0)
        self.solver = Solver(op, m, [], st, stream=stream)

    def solve(self, b, tol: float = 1e-8, max_iters: int = 10000, x0=None):
        """Returns ``(x, cg_iterations)``."""
        b = np.asarray(b, dtype=np.float64)
        if b.shape != (self.m,):
            raise ValueError("b must have %d entries" % self.m)
        rhs = self.solver.apply(b / math.sqrt(self.lam), transpose=True)   # A^T b / lam
        return self.solver.normal_solve(rhs, z0=x0, tol=tol, max_iters=max_iters)

    def close(self) -> None:
        self.solver.close()
