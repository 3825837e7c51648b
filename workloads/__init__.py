"""Seeded synthetic problem data for the paper's workloads (Section V).

This module only *draws* problem data: convolution kernels, sparse ground-truth
signals, dense measurement matrices, noisy observations and request traces.  It
holds none of the solver's arithmetic (no canonicalisation, no projection, no
iteration), so both the FP64 oracle and the GPU path may use it as their common
source of inputs.

Readings of the paper's instance recipes (Section V-A/B/C):

* Gaussian kernel: ``c_j ∝ exp(-(j-(k-1)/2)^2 / (2 sigma^2))`` for
  ``j = 0..k-1``, normalised to unit sum.
* ``N(0, v)`` takes ``v`` as the *variance* (the paper writes ``N(0, 0.01^2)``).
* A sparse ground truth has exactly ``floor(density * n)`` nonzeros at positions
  drawn without replacement.
* Lasso regularisation ``lambda = 0.1 * ||A^T b||_inf`` (Section V-B); the value
  ``||A^T b||_inf`` is the smallest lambda with an all-zero solution.
* Every draw uses ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "gaussian_kernel",
    "deconv_instance",
    "lasso_matrix",
    "lasso_instance",
    "serving_trace",
    "regls_instance",
    "conv_lasso_instance",
    "WORKLOADS",
    "workload",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_kernel(k: int, sigma: float) -> np.ndarray:
    """Unit-sum Gaussian of ``k`` taps centred at ``(k-1)/2`` (float64)."""
    if k < 1:
        raise ValueError("kernel length must be >= 1")
    j = np.arange(k, dtype=np.float64)
    c = np.exp(-((j - (k - 1) / 2.0) ** 2) / (2.0 * float(sigma) ** 2))
    return c / c.sum()


def _sparse_signal(rng: np.random.Generator, n: int, density: float, dist: str) -> np.ndarray:
    nnz = int(math.floor(density * n))
    x = np.zeros(n, dtype=np.float64)
    if nnz > 0:
        pos = rng.choice(n, size=nnz, replace=False)
        if dist == "uniform":
            x[pos] = rng.uniform(0.0, 1.0, size=nnz)
        elif dist == "normal":
            x[pos] = rng.standard_normal(nnz)
        else:
            raise ValueError(dist)
    return x


def deconv_instance(n: int, k: int, sigma: float, density: float, noise_var: float,
                    seed: int) -> Dict[str, np.ndarray]:
    """Nonnegative deconvolution data (Section V-C, eq. 6).

    Returns ``c`` (k taps), ``x_true`` (n, nonnegative, sparse) and
    ``b = c * x_true + v`` (full convolution, length ``n + k - 1``) with
    ``v ~ N(0, noise_var)``.
    """
    rng = _rng(seed)
    c = gaussian_kernel(k, sigma)
    x_true = _sparse_signal(rng, n, density, "uniform")
    clean = np.convolve(c, x_true)  # full convolution, n + k - 1 samples
    b = clean + rng.normal(0.0, math.sqrt(noise_var), size=clean.shape[0])
    return {"c": c, "x_true": x_true, "b": b}


def lasso_matrix(m: int, n: int, seed: int) -> np.ndarray:
    """Dense ``m x n`` matrix with i.i.d. ``N(0, 1/m)`` entries (float64, row-major)."""
    rng = _rng(seed)
    return rng.standard_normal((m, n)) * (1.0 / math.sqrt(m))


def lasso_instance(m: int, n: int, density: float, noise_var: float, seed: int,
                   A: Optional[np.ndarray] = None, matrix_seed: Optional[int] = None,
                   lam_factor: float = 0.1) -> Dict[str, np.ndarray]:
    """Lasso data (Section V-B, eq. 5).

    ``A`` is drawn from ``matrix_seed`` (default: ``seed``) unless given.  The
    ground truth has ``floor(density*n)`` ``N(0,1)`` nonzeros, ``b = A x_true + v``
    and ``lam = lam_factor * ||A^T b||_inf``.
    """
    if A is None:
        A = lasso_matrix(m, n, seed if matrix_seed is None else matrix_seed)
    # the signal/noise stream is the jumped PCG64 stream of ``seed``, so it never
    # repeats the matrix draws even when both use the same seed
    rng = np.random.Generator(np.random.PCG64(int(seed)).jumped())
    x_true = _sparse_signal(rng, n, density, "normal")
    b = A @ x_true + rng.normal(0.0, math.sqrt(noise_var), size=m)
    lam = lam_factor * float(np.max(np.abs(A.T @ b)))
    return {"A": A, "x_true": x_true, "b": b, "lam": np.float64(lam)}


def regls_instance(kind: str, n: int, seed: int, m: int = 0, k: int = 0, sigma: float = 0.0,
                   noise_var: float = 1e-4, lam: float = 1e-2) -> Dict[str, object]:
    """Regularized least-squares data (Section V-A, eq. 4).

    ``kind = "dense"``: ``A`` is ``m x n`` with i.i.d. ``N(0, 1)`` entries;
    ``kind = "conv"``: ``A x = c * x`` (full convolution, ``n + k - 1`` rows)
    with the unit-sum ``k``-tap Gaussian of standard deviation ``sigma``.
    ``x_hat ~ N(0, 1)`` (all ``n`` entries) and ``b = A x_hat + v`` with
    ``v ~ N(0, noise_var)``; ``lam`` is returned unchanged (the paper does not
    state its value).
    """
    rng = _rng(seed)
    out: Dict[str, object] = {"kind": kind, "lam": np.float64(lam)}
    if kind == "dense":
        A = rng.standard_normal((m, n))
        x_hat = rng.standard_normal(n)
        clean = A @ x_hat
        out["A"] = A
    elif kind == "conv":
        c = gaussian_kernel(k, sigma)
        x_hat = rng.standard_normal(n)
        clean = np.convolve(c, x_hat)
        out["c"] = c
    else:
        raise ValueError(kind)
    out["x_hat"] = x_hat
    out["b"] = clean + rng.normal(0.0, math.sqrt(noise_var), size=clean.shape[0])
    return out


def conv_lasso_instance(n: int, k: int, sigma: float, noise_var: float, seed: int,
                        lam_factor: float = 0.1) -> Dict[str, np.ndarray]:
    """Lasso with a convolution operator (Section V-B, the convolution column of
    Table II): ``A x = c * x`` as in :func:`regls_instance` (``kind = "conv"``),
    ``x_true ~ N(0, 1)``, ``b = A x_true + v`` and
    ``lam = lam_factor * ||A^T b||_inf`` (``A^T`` = valid correlation with ``c``).
    """
    rng = _rng(seed)
    c = gaussian_kernel(k, sigma)
    x_true = rng.standard_normal(n)
    clean = np.convolve(c, x_true)
    b = clean + rng.normal(0.0, math.sqrt(noise_var), size=clean.shape[0])
    lam = lam_factor * float(np.max(np.abs(np.correlate(b, c, mode="valid"))))
    return {"c": c, "x_true": x_true, "b": b, "lam": np.float64(lam)}


@dataclasses.dataclass
class Request:
    """One solve request of the serving workload."""
    rid: int
    arrival_s: float
    n: int
    k: int
    sigma: float
    seed: int


def serving_trace(count: int = 2000, rate: float = 200.0, seed: int = 1005,
                  n_lo: float = 1e3, n_hi: float = 1e5, k_half_lo: int = 5,
                  k_half_hi: int = 250) -> List[Request]:
    """Poisson arrival trace of deconvolution requests.

    Inter-arrival gaps are exponential with the given rate; ``n`` is log-uniform
    in ``[n_lo, n_hi]``; the kernel length is ``2*U{k_half_lo..k_half_hi}+1``
    (odd, 11..501 by default) with ``sigma = k/7``.  Request ``r`` draws its data
    with seed ``seed*1000 + r``.
    """
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(math.log(n_lo), math.log(n_hi), size=count)
    ns = np.rint(np.exp(logn)).astype(np.int64)
    ks = 2 * rng.integers(k_half_lo, k_half_hi + 1, size=count) + 1
    return [Request(r, float(arrivals[r]), int(ns[r]), int(ks[r]), float(ks[r]) / 7.0,
                    seed * 1000 + r) for r in range(count)]


def serving_request_data(req: Request, density: float = 0.05,
                         noise_var: float = 1e-4) -> Dict[str, np.ndarray]:
    return deconv_instance(req.n, req.k, req.sigma, density, noise_var, req.seed)


# Named workloads.  The "full" entries are the sizes quoted for the benchmark;
# the "small" variants keep the same structure at sizes the FP64 oracle solves in
# seconds (several kernel tiles plus a ragged tail).
WORKLOADS = {
    # Section V-C deconvolution, FP64, n = 1000, 101-tap Gaussian (sigma 15).
    # (block equilibration, normalize = 2: with data scaling alone the method
    # needs tens of thousands of iterations to reach 1e-6 here)
    "deconv_n1000_k101": dict(family="deconv", n=1000, k=101, sigma=15.0, density=0.10,
                              noise_var=1e-4, seed=1001, eps=1e-6, precision="fp64", normalize=2),
    # Large deconvolution: n = 2^20, 1025-tap Gaussian (sigma 150).
    "deconv_n1M_k1025": dict(family="deconv", n=1 << 20, k=1025, sigma=150.0, density=0.01,
                             noise_var=1e-6, seed=1002, eps=1e-4, precision="fp32"),
    # Dense lasso, A 5000 x 10000 (Section V-B).
    # stop_eps: the solvers stop at residuals of 1e-5 (<= the workload's 1e-4),
    # where the objective lands within 1e-4 of the optimum (a 1e-4 stop leaves
    # it up to ~3e-4 off on these instances)
    "lasso_5000x10000": dict(family="lasso", m=5000, n=10000, density=0.05, noise_var=1e-4,
                             seed=1003, eps=1e-4, stop_eps=1e-5, precision="fp32"),
    # Batched lasso: 64 instances sharing A 2000 x 8000.
    "lasso_batch64_2000x8000": dict(family="lasso_batch", m=2000, n=8000, batch=64,
                                    density=0.05, noise_var=1e-4, seed=1004, eps=1e-4,
                                    stop_eps=1e-5, precision="bf16"),
    # Regularized least squares by CG (Section V-A, Table I): dense 6000 x 3000
    # and a 3000-variable convolution whose 1365 taps give Table I's 4,095,000
    # nonzeros; stopped at ||(lam I + A^T A) x - A^T b|| <= 1e-8 ||A^T b||.
    "regls_dense_6000x3000": dict(family="regls", kind="dense", m=6000, n=3000, lam=1e-2,
                                  noise_var=1e-4, seed=1006, tol=1e-8, precision="fp64"),
    "regls_conv_3000_k1365": dict(family="regls", kind="conv", n=3000, k=1365, sigma=300.0,
                                  lam=1e-2, noise_var=1e-4, seed=1007, tol=1e-8, precision="fp64"),
    # Lasso with that convolution operator (Table II, convolution column).
    "lasso_conv_3000_k1365": dict(family="lasso_conv", n=3000, k=1365, sigma=300.0,
                                  noise_var=1e-4, seed=1008, eps=1e-4, precision="fp32"),
    # Serving stream of deconvolution requests.
    "serve_deconv_2000req": dict(family="serve", count=2000, rate=200.0, seed=1005,
                                 density=0.05, noise_var=1e-4, eps=1e-4, precision="fp32"),
}


def workload(name: str, **overrides) -> dict:
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    cfg["name"] = name
    return cfg


def make_deconv(cfg: dict) -> Dict[str, np.ndarray]:
    return deconv_instance(cfg["n"], cfg["k"], cfg["sigma"], cfg["density"],
                           cfg["noise_var"], cfg["seed"])


def make_lasso(cfg: dict) -> Dict[str, np.ndarray]:
    return lasso_instance(cfg["m"], cfg["n"], cfg["density"], cfg["noise_var"], cfg["seed"])


def make_regls(cfg: dict) -> Dict[str, object]:
    return regls_instance(cfg["kind"], cfg["n"], cfg["seed"], m=cfg.get("m", 0), k=cfg.get("k", 0),
                          sigma=cfg.get("sigma", 0.0), noise_var=cfg["noise_var"], lam=cfg["lam"])


def make_conv_lasso(cfg: dict) -> Dict[str, np.ndarray]:
    return conv_lasso_instance(cfg["n"], cfg["k"], cfg["sigma"], cfg["noise_var"], cfg["seed"])


def make_lasso_batch(cfg: dict) -> Dict[str, object]:
    """Shared ``A`` (seed ``cfg['seed']``) and per-instance ``b_i, lam_i``
    (instance ``i`` uses seed ``cfg['seed']*1000 + i``)."""
    A = lasso_matrix(cfg["m"], cfg["n"], cfg["seed"])
    insts = [lasso_instance(cfg["m"], cfg["n"], cfg["density"], cfg["noise_var"],
                            cfg["seed"] * 1000 + i, A=A, matrix_seed=cfg["seed"])
             for i in range(cfg["batch"])]
    return {"A": A, "b": [d["b"] for d in insts], "lam": [float(d["lam"]) for d in insts],
            "x_true": [d["x_true"] for d in insts]}
