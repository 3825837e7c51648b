"""Diagonal equilibration of a cone program (test infrastructure).

The paper notes that operator applications alone suffice to precondition a
problem (Section III, computation graphs); it does not fix a scheme.  The
reading taken here, and mirrored by the HIP library, is SCS's data
normalisation restricted to scalings that are constant on the operator's blocks,
in two levels: ``passes = 0`` leaves ``D = E = I`` and only scales ``b`` and
``c`` (the operator, and so the conditioning of ``I + A^T A`` that conjugate
gradients see, is unchanged); ``passes = 20`` also balances the blocks:

* Groups.  Rows are partitioned into the coarsest contiguous groups such that
  every nonzero block of ``A`` and every second-order cone lies inside one
  group (intervals that share a row are merged; rows that no block or cone
  touches form groups of their own).  Columns likewise, from the blocks.  A
  single scale per second-order cone keeps the cone invariant.
* Ruiz passes.  With ``F[g, h]`` the sum of squares of the entries of ``A`` in
  row group ``g`` and column group ``h`` (``1_g^T (A o A) 1_h``), each pass sets
  ``D_g <- D_g / sqrt(rho_g)`` with ``rho_g`` the root-mean-square row norm of
  ``D A E`` over group ``g``, then ``E_h <- E_h / sqrt(gamma_h)`` with the
  column norms of the row-scaled matrix; the norms are clipped to
  ``[1e-4, 1e4]``, and a group with zero norm keeps its scale.
* Data scaling.  ``b^ = sigma_b D b`` and ``c^ = sigma_c E c`` with
  ``sigma_b = mean row norm / max(||D b||, 1e-4)`` and
  ``sigma_c = mean column norm / max(||E c||, 1e-4)`` (means weighted by the
  group sizes, norms of the scaled ``A``).

The scaled problem ``min c^T x s.t. A^ x^ + s^ = b^`` with ``A^ = D A E`` has
the solutions ``x = E x^ / sigma_b``, ``y = D y^ / sigma_c``,
``s = s^ / (D sigma_b)``; the termination test is applied to those unscaled
points, so the criteria keep their plain meaning.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

from .program import ConeProgram

PASSES = 20
NORM_MIN, NORM_MAX = 1e-4, 1e4
DATA_MIN = 1e-4


@dataclasses.dataclass
class Scaling:
    D: np.ndarray          # per row
    E: np.ndarray          # per column
    sigma_b: float
    sigma_c: float
    row_groups: np.ndarray  # group index of every row
    col_groups: np.ndarray  # group index of every column

    def unscale(self, ux, uy, tau, vs):
        """Unscaled ``(x, y, s)`` of an iterate of the scaled problem."""
        x = self.E * ux / (tau * self.sigma_b)
        y = self.D * uy / (tau * self.sigma_c)
        s = vs / (self.D * tau * self.sigma_b)
        return x, y, s


def partition(length: int, intervals: Sequence[Tuple[int, int]]) -> np.ndarray:
    """Group index of every position: overlapping ``[lo, hi)`` intervals merge,
    positions covered by none form runs of their own."""
    ivs = sorted((lo, hi) for lo, hi in intervals if hi > lo)
    merged: List[List[int]] = []
    for lo, hi in ivs:
        if merged and lo < merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], hi)
        else:
            merged.append([lo, hi])
    group = np.empty(length, dtype=np.int64)
    g, pos = 0, 0
    for lo, hi in merged:
        if lo > pos:
            group[pos:lo] = g
            g += 1
        group[lo:hi] = g
        g += 1
        pos = hi
    if pos < length:
        group[pos:] = g
    return group


def groups(prog: ConeProgram) -> Tuple[np.ndarray, np.ndarray]:
    rows = [(r0, r0 + nr) for r0, nr, _, _ in prog.blocks]
    start = prog.l
    for qq in prog.q:
        rows.append((start, start + qq))
        start += qq
    cols = [(c0, c0 + nc) for _, _, c0, nc in prog.blocks]
    return partition(prog.m, rows), partition(prog.n, cols)


def group_norms(prog: ConeProgram, rg: np.ndarray, cg: np.ndarray) -> np.ndarray:
    """``F[g, h] = 1_g^T (A o A) 1_h``."""
    p, r = int(rg.max()) + 1, int(cg.max()) + 1
    F = np.zeros((p, r))
    for h in range(r):
        col = prog.A_sq((cg == h).astype(np.float64))
        F[:, h] = np.bincount(rg, weights=col, minlength=p)
    return F


def equilibrate(prog: ConeProgram, passes: int = PASSES) -> Scaling:
    rg, cg = groups(prog)
    F = group_norms(prog, rg, cg)
    R = np.bincount(rg).astype(np.float64)
    C = np.bincount(cg).astype(np.float64)
    D = np.ones(F.shape[0])
    E = np.ones(F.shape[1])

    def row_rms():
        return np.sqrt(D * D * (F @ (E * E)) / R)

    def col_rms():
        return np.sqrt(E * E * (F.T @ (D * D)) / C)

    for _ in range(passes):
        rho = row_rms()
        D = np.where(rho > 0, D / np.sqrt(np.clip(rho, NORM_MIN, NORM_MAX)), D)
        gam = col_rms()
        E = np.where(gam > 0, E / np.sqrt(np.clip(gam, NORM_MIN, NORM_MAX)), E)
    mean_row = float(R @ row_rms()) / prog.m
    mean_col = float(C @ col_rms()) / prog.n
    Dv, Ev = D[rg], E[cg]
    sb = mean_row / max(float(np.linalg.norm(Dv * prog.b)), DATA_MIN)
    sc = mean_col / max(float(np.linalg.norm(Ev * prog.c)), DATA_MIN)
    return Scaling(Dv, Ev, sb, sc, rg, cg)


def identity_scaling(prog: ConeProgram) -> Scaling:
    rg, cg = groups(prog)
    return Scaling(np.ones(prog.m), np.ones(prog.n), 1.0, 1.0, rg, cg)


def scaled_program(prog: ConeProgram, s: Scaling) -> ConeProgram:
    """The program ``min c^T x s.t. (D A E) x + s = b^`` of the scaled data."""
    D, E = s.D, s.E

    def apply(x):
        return D * prog.A(E * x)

    def apply_T(y):
        return E * prog.AT(D * y)

    def explicit():
        return D[:, None] * prog.explicit() * E[None, :]

    def apply_sq(x):
        return D * D * prog.A_sq(E * E * x)

    return ConeProgram(prog.n, prog.m, s.sigma_b * D * prog.b, s.sigma_c * E * prog.c,
                       prog.l, prog.q, apply, apply_T, explicit,
                       lambda: prog.scaled_factor(D, E), prog.family,
                       dict(prog.data, scaling=s), blocks=prog.blocks, apply_sq=apply_sq)
