"""Canonical cone forms of the paper's examples as structured-operator descriptions.

Sign convention: ``minimize c^T z s.t. A z + s = b, s in K`` (eq. (1) with
``A -> -A``), ``K = R_+^l x SOC(q...)``.  The operator is never formed as a
matrix: convolution and dense data enter as blocks (Sections III-A, IV).

* Nonnegative deconvolution (Section V-C, eq. 6), variables ``(x, t)``::

      A = [[-I, 0], [0, -1], [-C, 0]],  b = [0, 0, -b_obs],  c = [0, 1]
      K = R_+^n x SOC(n + k)          (rows: x >= 0 | ||C x - b_obs|| <= t)

* Lasso (Section V-B, eq. 5), variables ``(x, t, u)``::

      rows [t - x >= 0 | t + x >= 0 | SOC(u + 1, 2(A x - b_obs), u - 1)]
      A = [[I, -I, 0], [-I, -I, 0], [0, 0, -1], [-2A, 0, 0], [0, 0, -1]]
      b = [0, 0, 1, -2 b_obs, -1],  c = [0, lam 1, 1/2]

* Lasso with a convolution operator (Table II, convolution column): the same
  layout with the dense block ``-2A`` replaced by the full convolution ``-2C``.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from ._lib import Operator


@dataclasses.dataclass
class ConeProblem:
    op: Operator
    l: int
    q: List[int]
    b: np.ndarray
    c: np.ndarray
    n_signal: int        # length of the natural variable x inside z


def _is_device_tensor(a) -> bool:
    try:
        import torch
    except ImportError:   # pragma: no cover
        return False
    return isinstance(a, torch.Tensor) and a.is_cuda


def deconv_problem(taps, b_obs) -> ConeProblem:
    taps = np.asarray(taps, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    k = taps.shape[0]
    n = b_obs.shape[0] - k + 1
    if n < 1:
        raise ValueError("observation shorter than the kernel")
    m = n + 1 + (n + k - 1)
    op = Operator(m, n + 1)
    op.add_identity(0, 0, n, -1.0)            # s = x
    op.add_identity(n, n, 1, -1.0)            # s = t
    op.add_conv(n + 1, 0, taps, n, -1.0)      # s = C x - b_obs
    b = np.concatenate([np.zeros(n + 1), -b_obs])
    c = np.zeros(n + 1)
    c[n] = 1.0
    return ConeProblem(op, n, [n + k], b, c, n)


def lasso_problem(A, b_obs, lam: float) -> ConeProblem:
    # (a torch tensor on the GPU is passed through: the operator borrows it)
    if not _is_device_tensor(A):
        A = np.asarray(A, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    m0, n0 = A.shape
    nv = 2 * n0 + 1
    m = 2 * n0 + m0 + 2
    op = Operator(m, nv)
    op.add_identity(0, 0, n0, 1.0)            # t - x >= 0
    op.add_identity(0, n0, n0, -1.0)
    op.add_identity(n0, 0, n0, -1.0)          # t + x >= 0
    op.add_identity(n0, n0, n0, -1.0)
    op.add_identity(2 * n0, 2 * n0, 1, -1.0)  # u + 1
    op.add_dense(2 * n0 + 1, 0, A, -2.0)      # 2(A x - b)
    op.add_identity(m - 1, 2 * n0, 1, -1.0)   # u - 1
    b = np.concatenate([np.zeros(2 * n0), [1.0], -2.0 * b_obs, [-1.0]])
    c = np.concatenate([np.zeros(n0), np.full(n0, float(lam)), [0.5]])
    return ConeProblem(op, 2 * n0, [m0 + 2], b, c, n0)


def conv_lasso_problem(taps, b_obs, lam: float) -> ConeProblem:
    taps = np.asarray(taps, dtype=np.float64)
    b_obs = np.asarray(b_obs, dtype=np.float64)
    k = taps.shape[0]
    n0 = b_obs.shape[0] - k + 1
    if n0 < 1:
        raise ValueError("observation shorter than the kernel")
    m0 = n0 + k - 1
    nv = 2 * n0 + 1
    m = 2 * n0 + m0 + 2
    op = Operator(m, nv)
    op.add_identity(0, 0, n0, 1.0)            # t - x >= 0
    op.add_identity(0, n0, n0, -1.0)
    op.add_identity(n0, 0, n0, -1.0)          # t + x >= 0
    op.add_identity(n0, n0, n0, -1.0)
    op.add_identity(2 * n0, 2 * n0, 1, -1.0)  # u + 1
    op.add_conv(2 * n0 + 1, 0, taps, n0, -2.0)   # 2(c * x - b)
    op.add_identity(m - 1, 2 * n0, 1, -1.0)   # u - 1
    b = np.concatenate([np.zeros(2 * n0), [1.0], -2.0 * b_obs, [-1.0]])
    c = np.concatenate([np.zeros(n0), np.full(n0, float(lam)), [0.5]])
    return ConeProblem(op, 2 * n0, [m0 + 2], b, c, n0)
