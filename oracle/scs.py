"""Homogeneous self-dual embedding ADMM ("SCS"), plain FP64.

The paper implements SCS as a computation graph (Sections II-D, V-B): the
iteration alternates a projection onto a linear subspace, done by solving a
linear system in ``I + A^T A``, with a projection onto a convex cone.  The
paper only cites the method (O'Donoghue, Chu, Parikh, Boyd); the steps below are
its published mathematics, written out in the order they are applied.  Here the
subspace step is solved exactly with the direct factorisation of
``K = I + A^T A`` (the "direct" variant of Section II-D); the GPU path solves the
same system with conjugate gradients (the "indirect" variant).

Embedding.  For ``min c^T x s.t. A x + s = b, s in K`` with ``u = (x, y, tau)``
and ``v = (r, s, kappa)``::

    Q = [[ 0,   A^T,  c],
         [-A,    0,   b],
         [-c^T, -b^T, 0]],      v = Q u,  u in R^n x K* x R_+,  v in {0}^n x K x R_+.

Iteration (relaxation ``alpha``)::

    u~ = (I + Q)^{-1} (u + v)
    u_bar = alpha u~ + (1 - alpha) u
    u  <- Pi(u_bar - v)                      # x free, y onto K*, tau onto R_+
    v  <- v - u_bar + u

``(I + Q)^{-1} w``: with ``M = [[I, A^T], [-A, I]]``, ``h = (c, b)`` and
``g = M^{-1} h`` (computed once), ``eta = 1 + h^T g`` (> 1 since ``M + M^T = 2I``):
``z = M^{-1} w_xy`` (``z_x = K^{-1}(w_x - A^T w_y)``, ``z_y = w_y + A z_x``),
``u~_tau = (w_tau + c^T z_x + b^T z_y) / eta``, ``u~_xy = z - u~_tau g``.

Readings where the paper is silent: the iteration runs on the scaled data of
``oracle.equil`` -- ``normalize=1`` (the default) scales ``b`` and ``c`` only,
``normalize=2`` also balances the operator's blocks, ``normalize=0`` keeps the
data as given -- ``alpha = 1.5``, start ``u = v = (0, 0, 1)``; ``v_x`` stays
0 and is not stored (the ``y``-block of ``v`` is ``s``).  Termination, on the
unscaled point, uses the relative 2-norm criteria
``res_pri = ||A x + s - b|| / (1 + ||b||)``,
``res_dual = ||A^T y + c|| / (1 + ||c||)``,
``gap = |c^T x + b^T y| / (1 + |c^T x| + |b^T y|)`` at ``(x, y, s) = (u_x, u_y,
v_s)/tau``; when ``tau < kappa`` the infeasibility / unboundedness certificates
``-b^T u_y > 0, ||A^T u_y|| <= eps (-b^T u_y)`` and
``-c^T u_x > 0, ||A u_x + v_s|| <= eps (-c^T u_x)`` are tested instead.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Optional

import numpy as np

from .cones import proj_cone
from .equil import PASSES, Scaling, equilibrate, identity_scaling, scaled_program
from .program import ConeProgram, Factor


@dataclasses.dataclass
class ScsResult:
    status: str           # "solved" | "infeasible" | "unbounded" | "max_iters"
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    tau: float
    kappa: float
    iters: int
    pobj: float
    dobj: float
    res_pri: float
    res_dual: float
    gap: float
    setup_s: float
    solve_s: float
    u: Optional[tuple] = None   # final (u_x, u_y, tau, v_s, kappa) of the scaled problem
    scaling: Optional[Scaling] = None


def embedding_vector(prog: ConeProgram, fac: Factor):
    """``g = M^{-1} (c, b)`` and ``eta = 1 + c^T g_x + b^T g_y``."""
    gx = fac.solve(prog.c - prog.AT(prog.b))
    gy = prog.b + prog.A(gx)
    eta = 1.0 + float(prog.c @ gx) + float(prog.b @ gy)
    return gx, gy, eta


def hsde_subspace_step(prog: ConeProgram, fac: Factor, gx, gy, eta, wx, wy, wtau):
    """Exact ``u~ = (I + Q)^{-1} w``; returns ``(u~_x, u~_y, u~_tau)``."""
    zx = fac.solve(wx - prog.AT(wy))
    zy = wy + prog.A(zx)
    ut = (wtau + float(prog.c @ zx) + float(prog.b @ zy)) / eta
    return zx - ut * gx, zy - ut * gy, ut


def residuals(prog: ConeProgram, ux, uy, tau, vs):
    """Relative primal/dual residuals and gap at ``(u_x, u_y, v_s) / tau``."""
    x, y, s = ux / tau, uy / tau, vs / tau
    cx = float(prog.c @ x)
    by = float(prog.b @ y)
    rp = float(np.linalg.norm(prog.A(x) + s - prog.b)) / (1.0 + float(np.linalg.norm(prog.b)))
    rd = float(np.linalg.norm(prog.AT(y) + prog.c)) / (1.0 + float(np.linalg.norm(prog.c)))
    gap = abs(cx + by) / (1.0 + abs(cx) + abs(by))
    return rp, rd, gap, cx, -by


def prepare(prog: ConeProgram, normalize: int = 1):
    """``(working program, scaling)``: the scaled program (``normalize`` 1: data
    only, 2: blocks and data), or ``prog`` itself (0)."""
    normalize = int(normalize)
    if normalize not in (0, 1, 2):
        raise ValueError("normalize must be 0, 1 or 2")
    if normalize:
        scl = equilibrate(prog, passes=PASSES if normalize == 2 else 0)
        return scaled_program(prog, scl), scl
    return prog, identity_scaling(prog)


def scs_solve(prog: ConeProgram, eps: float = 1e-8, alpha: float = 1.5,
              max_iters: int = 100_000, check_every: int = 1,
              fac: Optional[Factor] = None, warm: Optional[tuple] = None,
              callback: Optional[Callable] = None,
              time_limit_s: Optional[float] = None, normalize: int = 1) -> ScsResult:
    """Run the HSDE ADMM iteration to the relative tolerance ``eps``.

    ``fac`` factors ``I + A^T A`` of the working (scaled) program.
    ``warm`` = ``(u_x, u_y, tau, v_s, kappa)`` resumes from a saved state and
    ``callback(it, ux, uy, tau, vs, kappa)`` sees every iterate, both in the
    variables of the working program.
    """
    t0 = time.perf_counter()
    orig = prog
    prog, scl = prepare(orig, normalize)
    if fac is None:
        fac = prog.factor()
    gx, gy, eta = embedding_vector(prog, fac)
    t1 = time.perf_counter()
    n, m = prog.n, prog.m
    if warm is None:
        ux, uy, tau = np.zeros(n), np.zeros(m), 1.0
        vs, kappa = np.zeros(m), 1.0
    else:
        ux, uy, tau, vs, kappa = (np.array(warm[0], dtype=np.float64),
                                  np.array(warm[1], dtype=np.float64), float(warm[2]),
                                  np.array(warm[3], dtype=np.float64), float(warm[4]))
    status = "max_iters"
    it = 0
    rp = rd = gap = np.inf
    pobj = dobj = np.nan
    for it in range(1, max_iters + 1):
        # subspace projection of w = u + v (v_x = 0)
        utx, uty, utt = hsde_subspace_step(prog, fac, gx, gy, eta, ux, uy + vs, tau + kappa)
        # over-relaxation
        bx = alpha * utx + (1.0 - alpha) * ux
        by = alpha * uty + (1.0 - alpha) * uy
        bt = alpha * utt + (1.0 - alpha) * tau
        # cone projection of u_bar - v
        uy_new = proj_cone(by - vs, prog.l, prog.q)
        tau_new = max(bt - kappa, 0.0)
        # dual update v <- v - u_bar + u
        vs = vs - by + uy_new
        kappa = kappa - bt + tau_new
        ux, uy, tau = bx, uy_new, tau_new
        if callback is not None:
            callback(it, ux, uy, tau, vs, kappa)
        if it % check_every == 0 or it == max_iters:
            # the point of the original problem (a positive multiple of it for rays)
            rx, ry, rs = scl.unscale(ux, uy, 1.0, vs)
            if tau > 0.0:
                rp, rd, gap, pobj, dobj = residuals(orig, rx, ry, tau, rs)
                if rp <= eps and rd <= eps and gap <= eps:
                    status = "solved"
                    break
            if tau < kappa:
                bty = float(orig.b @ ry)
                if bty < 0.0 and np.linalg.norm(orig.AT(ry)) <= eps * (-bty):
                    status = "infeasible"
                    break
                ctx = float(orig.c @ rx)
                if ctx < 0.0 and np.linalg.norm(orig.A(rx) + rs) <= eps * (-ctx):
                    status = "unbounded"
                    break
            if time_limit_s is not None and time.perf_counter() - t1 > time_limit_s:
                break
    t2 = time.perf_counter()
    rx, ry, rs = scl.unscale(ux, uy, 1.0, vs)
    if status == "infeasible":
        scale = -float(orig.b @ ry)
        x, y, s = np.full(n, np.nan), ry / scale, np.full(m, np.nan)
    elif status == "unbounded":
        scale = -float(orig.c @ rx)
        x, y, s = rx / scale, np.full(m, np.nan), rs / scale
    else:
        x, y, s = rx / tau, ry / tau, rs / tau
    return ScsResult(status, x, y, s, tau, kappa, it, pobj, dobj, rp, rd, gap,
                     t1 - t0, t2 - t1, (ux, uy, tau, vs, kappa), scl)
