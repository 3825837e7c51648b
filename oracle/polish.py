"""Active-set polish and KKT certificates for the deconvolution and lasso examples.

The iterative method returns an approximate optimum.  The exact optimum has a
plain definition (the unique minimiser of eq. 6, resp. eq. 5), computed here by
active-set methods and accepted only if the full Karush-Kuhn-Tucker conditions
of the original problem hold to a tight tolerance:

* lasso: the iterate's support and signs define a smaller unconstrained least
  squares problem; textbook active-set steps fix wrong signs and add violated
  coordinates until the subgradient conditions hold;
* deconvolution: Lawson-Hanson nonnegative least squares on the explicit
  convolution matrix (small sizes only).

Natural objectives (evaluated in float64 from a returned primal point):

* deconvolution (eq. 6): ``||c * max(x, 0) - b||_2`` (the clip removes the
  tolerance-level infeasibility of an iterate);
* lasso (eq. 5): ``(1/2)||A x - b||^2 + lam ||x||_1``.
"""
from __future__ import annotations

from typing import Dict

import numpy as np
from scipy.optimize import nnls

from .program import conv_matrix


def deconv_objective(c: np.ndarray, b_obs: np.ndarray, x: np.ndarray) -> float:
    return float(np.linalg.norm(np.convolve(c, np.maximum(x, 0.0)) - b_obs))


def lasso_objective(A: np.ndarray, b_obs: np.ndarray, lam: float, x: np.ndarray) -> float:
    r = A @ x - b_obs
    return float(0.5 * (r @ r) + lam * np.sum(np.abs(x)))


def polish_deconv(c: np.ndarray, b_obs: np.ndarray, x0=None, tol: float = 1e-9,
                  max_n: int = 6000) -> Dict[str, object]:
    """Exact nonnegative least squares for ``min ||c*x - b|| s.t. x >= 0``.

    The blur operator is so ill-conditioned that a support taken from an
    iterate does not pin the optimum, so the reference is the Lawson-Hanson
    active-set algorithm run from scratch on the explicit convolution matrix
    (``scipy.optimize.nnls``), followed by the KKT check: ``x >= 0``,
    ``grad = C^T (C x - b) >= 0`` and ``x_i grad_i = 0``, relative to
    ``||C^T b||_inf``.  Only sizes with ``n <= max_n`` are attempted.
    """
    c = np.asarray(c, dtype=np.float64)
    k = c.shape[0]
    n = b_obs.shape[0] - k + 1
    if n > max_n:
        return {"x": None, "obj": None, "kkt_ok": False, "kkt_err": np.inf, "support": None}
    C = conv_matrix(c, n)
    x, _ = nnls(C, b_obs, maxiter=50 * n)
    grad = C.T @ (C @ x - b_obs)
    scale = max(float(np.max(np.abs(C.T @ b_obs))), 1e-300)
    P = x > 0.0
    err_in = float(np.max(np.abs(grad[P]))) if np.any(P) else 0.0
    err_out = float(np.max(-grad[~P])) if np.any(~P) else 0.0
    err = max(err_in, err_out, 0.0) / scale
    return {"x": x, "obj": deconv_objective(c, b_obs, x), "kkt_ok": bool(err <= tol),
            "kkt_err": err, "support": int(np.count_nonzero(P))}


def polish_lasso(A: np.ndarray, b_obs: np.ndarray, lam: float, x0: np.ndarray,
                 tol: float = 1e-9, max_rounds: int = 50,
                 rel_thresh: float = 1e-4) -> Dict[str, object]:
    """Active-set polish of the lasso from the iterate ``x0``.

    KKT (subgradient) conditions: ``A_j^T (b - A x) = lam sign(x_j)`` on the
    support and ``|A_j^T (b - A x)| <= lam`` off it; checked relative to ``lam``.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    xmax = float(np.max(np.abs(x0))) if x0.size else 0.0
    S = np.flatnonzero(np.abs(x0) > rel_thresh * max(xmax, 1e-300))
    sig = np.sign(x0[S])
    x = np.zeros(n)
    ok = False
    err = np.inf
    for rounds in range(1, max_rounds + 1):
        x = np.zeros(n)
        if S.size:
            AS = A[:, S]
            x[S] = np.linalg.solve(AS.T @ AS, AS.T @ b_obs - lam * sig)
        wrong = np.sign(x[S]) != sig
        if np.any(wrong):
            keep = ~wrong
            S, sig = S[keep], sig[keep]
            continue
        corr = A.T @ (b_obs - A @ x)
        err_in = float(np.max(np.abs(corr[S] - lam * sig))) if S.size else 0.0
        comp = np.setdiff1d(np.arange(n), S)
        over = np.abs(corr[comp]) - lam
        err_out = float(np.max(over)) if comp.size else 0.0
        err = max(err_in, err_out, 0.0) / lam
        if err <= tol:
            ok = True
            break
        bad = over > tol * lam
        if not np.any(bad):
            break
        idx = comp[bad]
        order = np.argsort(-over[bad])
        add = idx[order[: max(1, idx.size // 4 + 1)]]
        S_new = np.concatenate([S, add])
        sig_new = np.concatenate([sig, np.sign(corr[add])])
        o = np.argsort(S_new)
        S, sig = S_new[o], sig_new[o]
    return {"x": x, "obj": lasso_objective(A, b_obs, lam, x), "kkt_ok": ok, "kkt_err": err,
            "rounds": rounds, "support": int(S.size)}
