"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
printed value (Tables II/III dimensions), a closed form, a characterisation
(Moreau decomposition, KKT conditions with an analytic dual), a library routine
for a special case (Lawson-Hanson NNLS, soft thresholding) or brute force on tiny
inputs (all supports, all LP vertices).
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.optimize import nnls

import oracle as o
import workloads as w
from oracle.program import conv_matrix
from oracle.scs import embedding_vector, hsde_subspace_step, residuals

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- cones

def test_soc_projection_hand_values():
    # inside: unchanged; in the polar cone: zero; otherwise ((t+|z|)/2)(1, z/|z|)
    np.testing.assert_allclose(o.proj_soc(np.array([2.0, 1.0, -1.0])), [2.0, 1.0, -1.0])
    np.testing.assert_allclose(o.proj_soc(np.array([-5.0, 3.0, 4.0])), [0.0, 0.0, 0.0])
    np.testing.assert_allclose(o.proj_soc(np.array([0.0, 3.0, 4.0])), [2.5, 1.5, 2.0])
    np.testing.assert_allclose(o.proj_soc(np.array([1.0, 3.0, 4.0])), [3.0, 1.8, 2.4])
    # size-1 cone is the half line
    assert o.proj_soc(np.array([-0.3]))[0] == 0.0
    assert o.proj_soc(np.array([0.7]))[0] == 0.7


@pytest.mark.parametrize("seed", range(5))
def test_projection_characterisation(seed):
    """p = Pi_K(v) iff p in K, p - v in K* (= K) and <p, p - v> = 0 (Moreau)."""
    rng = np.random.default_rng(seed)
    l, q = 7, [1, 2, 5, 9]
    v = rng.standard_normal(l + sum(q)) * 3
    p = o.proj_cone(v, l, q)
    assert o.in_cone(p, l, q, 1e-12)
    assert o.in_cone(p - v, l, q, 1e-12)
    assert abs(p @ (p - v)) < 1e-10
    # idempotent and Moreau: v = Pi(v) - Pi(-v)
    np.testing.assert_allclose(o.proj_cone(p, l, q), p, atol=1e-14)
    np.testing.assert_allclose(p - o.proj_cone(-v, l, q), v, atol=1e-12)


def test_projection_is_nearest_point_bruteforce():
    """Nearest point of a 3-dim SOC found by dense sampling of the cone."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        v = rng.standard_normal(3) * 2
        p = o.proj_soc(v)
        # sample cone points (t, r cos a, r sin a), r <= t
        t = np.linspace(0, 2 * np.linalg.norm(v) + 1, 241)[:, None, None]
        frac = np.linspace(0, 1, 41)[None, :, None]
        ang = np.linspace(0, 2 * np.pi, 181)[None, None, :]
        pts = np.stack(np.broadcast_arrays(t, t * frac * np.cos(ang), t * frac * np.sin(ang)), -1)
        d = np.linalg.norm(pts - v, axis=-1).min()
        assert np.linalg.norm(p - v) <= d + 1e-12
        assert np.linalg.norm(p - v) >= d - 0.1   # grid resolution


# ----------------------------------------------------------------- canonical forms

def test_deconv_dimensions_match_table3():
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))["deconv_table3"]
    for row in tab:
        n0 = row["n0"]
        c = np.ones(n0) / n0       # an n0-tap kernel, b in R^{2 n0 - 1}
        b = np.zeros(2 * n0 - 1)
        prog = o.deconv_program(c, b)
        assert prog.n == row["variables"] and prog.m == row["constraints"]


def test_lasso_dimensions_and_nnz_match_table2():
    row = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))["lasso_table2_dense"]
    A = w.lasso_matrix(row["m0"], row["n0"], 11)
    prog = o.lasso_program(A, np.ones(row["m0"]), 0.1)
    assert prog.n == row["variables"] and prog.m == row["constraints"]
    Ac = prog.explicit()
    assert int(np.count_nonzero(Ac)) == row["nonzeros"]


def test_conv_lasso_dimensions_and_nnz_match_table2():
    """The nonzero count of the conv-lasso cone form is 4 n0 + k n0 + 2 (checked
    on an explicit small instance), which at n0 = 3000, k = 1365 is the 4,107,002
    of Table II; Table I's convolution has k n0 = 4,095,000 nonzeros."""
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    for n0, k in ((40, 9), (25, 25)):
        prog = o.conv_lasso_program(w.gaussian_kernel(k, k / 4), np.ones(n0 + k - 1), 0.1)
        assert int(np.count_nonzero(prog.explicit())) == 4 * n0 + k * n0 + 2
        assert int(np.count_nonzero(conv_matrix(w.gaussian_kernel(k, k / 4), n0))) == k * n0
        assert prog.n == 2 * n0 + 1 and prog.m == 2 * n0 + (n0 + k - 1) + 2
    row = tab["lasso_table2_conv"]
    n0, k = row["n0"], row["k"]
    assert 2 * n0 + 1 == row["variables"]
    assert 4 * n0 + k * n0 + 2 == row["nonzeros"]
    t1 = tab["regls_table1"]
    assert t1["conv_k"] * t1["n"] == t1["conv_nonzeros"]
    assert t1["dense_rows"] * t1["n"] == t1["dense_nonzeros"]


def test_conv_lasso_canonical_form_kkt_with_polished_optimum():
    """The conv-lasso cone program solved by the oracle and polished: the
    polished point satisfies the lasso's subgradient optimality conditions (the
    definition of the optimum) and the analytic primal-dual pair of the cone
    form at it has zero residuals."""
    d = w.conv_lasso_instance(70, 11, 2.0, 1e-4, 9)
    prog = o.conv_lasso_program(d["c"], d["b"], d["lam"])
    res = o.scs_solve(prog, eps=1e-8, max_iters=200_000)
    assert res.status == "solved"
    C = conv_matrix(d["c"], 70)
    pol = o.polish_lasso(C, d["b"], d["lam"], res.x[:70])
    assert pol["kkt_ok"]
    g = C.T @ (d["b"] - C @ pol["x"])
    S = pol["x"] != 0
    assert np.all(np.abs(g[S] - d["lam"] * np.sign(pol["x"][S])) <= 1e-9 * d["lam"])
    assert np.all(np.abs(g[~S]) <= d["lam"] * (1 + 1e-9))
    z, y, s = _lasso_kkt_point(C, d["b"], d["lam"], pol["x"])
    rp, rd, gap, pobj, _ = residuals(prog, z, y, 1.0, s)
    assert rp < 1e-12 and rd < 1e-10 and gap < 1e-12
    assert abs(pobj - pol["obj"]) < 1e-10


@pytest.mark.parametrize("kind", ["dense", "conv"])
def test_regls_closed_form_against_stacked_least_squares(kind):
    """x* = (lam I + A^T A)^{-1} A^T b (eq. (5)) equals the least-squares solution
    of the stacked system [A; sqrt(lam) I] x = [b; 0] computed by an orthogonal
    factorisation (a different route to the same minimiser), and zeroes the
    gradient A^T (A x - b) + lam x."""
    if kind == "dense":
        d = w.regls_instance("dense", 30, 3, m=50, lam=0.05)
        A = d["A"]
    else:
        d = w.regls_instance("conv", 80, 4, k=21, sigma=5.0, lam=0.05)
        A = conv_matrix(d["c"], 80)
    lam = float(d["lam"])
    x = o.regls_solution(d)
    n = A.shape[1]
    M = np.vstack([A, np.sqrt(lam) * np.eye(n)])
    ref = np.linalg.lstsq(M, np.concatenate([d["b"], np.zeros(n)]), rcond=None)[0]
    np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12)
    grad = A.T @ (A @ x - d["b"]) + lam * x
    assert np.linalg.norm(grad) <= 1e-11 * np.linalg.norm(A.T @ d["b"])
    # the objective is minimal along random directions (convex quadratic)
    rng = np.random.default_rng(0)
    f0 = o.regls_objective(d, x)
    for _ in range(5):
        assert o.regls_objective(d, x + 1e-3 * rng.standard_normal(n)) > f0


def test_convolution_primitive_matches_bruteforce_sum():
    rng = np.random.default_rng(0)
    c, x = rng.standard_normal(7), rng.standard_normal(19)
    y = np.zeros(25)
    for i in range(25):
        for j in range(7):
            if 0 <= i - j < 19:
                y[i] += c[j] * x[i - j]
    prog = o.deconv_program(c, np.zeros(25))
    z = np.concatenate([x, [0.0]])
    np.testing.assert_allclose(-prog.A(z)[20:], y, atol=1e-13)
    np.testing.assert_allclose(conv_matrix(c, 19) @ x, y, atol=1e-13)


@pytest.mark.parametrize("family", ["deconv", "lasso", "lasso_conv"])
def test_apply_adjoint_and_factor_against_explicit(family):
    rng = np.random.default_rng(1)
    if family == "deconv":
        prog = o.deconv_program(w.gaussian_kernel(9, 2.0), rng.standard_normal(40 + 8))
    elif family == "lasso_conv":
        prog = o.conv_lasso_program(w.gaussian_kernel(9, 2.0), rng.standard_normal(40 + 8), 0.3)
    else:
        prog = o.lasso_program(rng.standard_normal((15, 11)), rng.standard_normal(15), 0.3)
    A = prog.explicit()
    x, y = rng.standard_normal(prog.n), rng.standard_normal(prog.m)
    np.testing.assert_allclose(prog.A(x), A @ x, atol=1e-12)
    np.testing.assert_allclose(prog.AT(y), A.T @ y, atol=1e-12)
    r = rng.standard_normal(prog.n)
    np.testing.assert_allclose(prog.factor().solve(r),
                               np.linalg.solve(np.eye(prog.n) + A.T @ A, r), atol=1e-11)


def _deconv_kkt_point(c, b, x):
    """Analytic primal-dual pair of the deconvolution cone program at the NNLS optimum.

    From A^T y + c = 0 and complementarity: y_t = 1, y_z = (b - Cx)/||b - Cx||,
    y_nonneg = C^T (Cx - b)/||Cx - b||;  s = (x, ||Cx - b||, Cx - b).
    """
    r = np.convolve(c, x) - b
    nr = np.linalg.norm(r)
    y = np.concatenate([np.correlate(r, c, "valid") / nr, [1.0], -r / nr])
    s = np.concatenate([x, [nr], r])
    z = np.concatenate([x, [nr]])
    return z, y, s


def _lasso_kkt_point(A, b, lam, x):
    """Analytic primal-dual pair of the lasso cone program at the optimum.

    y_q = (1/4)(u+1, -2r, -(u-1)) with r = Ax - b, u = ||r||^2; with
    g = A^T (b - Ax): y_1 = (lam + g)/2, y_2 = (lam - g)/2.
    """
    r = A @ x - b
    u = r @ r
    g = A.T @ (-r)
    y = np.concatenate([(lam + g) / 2, (lam - g) / 2, [(u + 1) / 4], -r / 2, [-(u - 1) / 4]])
    t = np.abs(x)
    s = np.concatenate([t - x, t + x, [u + 1], 2 * r, [u - 1]])
    z = np.concatenate([x, t, [u]])
    return z, y, s


def test_deconv_canonical_form_kkt_with_exact_nnls():
    d = w.deconv_instance(60, 11, 2.0, 0.1, 1e-4, 5)
    x = nnls(conv_matrix(d["c"], 60), d["b"])[0]
    prog = o.deconv_program(d["c"], d["b"])
    z, y, s = _deconv_kkt_point(d["c"], d["b"], x)
    rp, rd, gap, pobj, dobj = residuals(prog, z, y, 1.0, s)
    assert rp < 1e-12 and rd < 1e-9 and gap < 1e-12
    assert o.in_cone(s, prog.l, prog.q, 1e-12) and o.in_cone(y, prog.l, prog.q, 1e-9)
    assert abs(pobj - np.linalg.norm(np.convolve(d["c"], x) - d["b"])) < 1e-12


def test_lasso_canonical_form_kkt_with_polished_optimum():
    d = w.lasso_instance(40, 60, 0.1, 1e-4, 9)
    prog = o.lasso_program(d["A"], d["b"], d["lam"])
    res = o.scs_solve(prog, eps=1e-7)
    pol = o.polish_lasso(d["A"], d["b"], d["lam"], res.x[:60])
    assert pol["kkt_ok"]
    z, y, s = _lasso_kkt_point(d["A"], d["b"], d["lam"], pol["x"])
    rp, rd, gap, pobj, _ = residuals(prog, z, y, 1.0, s)
    assert rp < 1e-12 and rd < 1e-10 and gap < 1e-12
    assert o.in_cone(y, prog.l, prog.q, 1e-10)
    assert abs(pobj - pol["obj"]) < 1e-10


# ----------------------------------------------------------------- the embedding step

def _explicit_Q(prog):
    A = prog.explicit()
    n, m = prog.n, prog.m
    Q = np.zeros((n + m + 1, n + m + 1))
    Q[:n, n:n + m] = A.T
    Q[:n, -1] = prog.c
    Q[n:n + m, :n] = -A
    Q[n:n + m, -1] = prog.b
    Q[-1, :n] = -prog.c
    Q[-1, n:n + m] = -prog.b
    return Q


@pytest.mark.parametrize("family", ["deconv", "lasso", "lp"])
def test_subspace_step_solves_I_plus_Q(family):
    rng = np.random.default_rng(2)
    if family == "deconv":
        prog = o.deconv_program(w.gaussian_kernel(5, 1.0), rng.standard_normal(12 + 4))
    elif family == "lasso":
        prog = o.lasso_program(rng.standard_normal((9, 6)), rng.standard_normal(9), 0.2)
    else:
        prog = o.dense_program(rng.standard_normal((8, 4)), rng.standard_normal(8),
                               rng.standard_normal(4), 8)
    fac = prog.factor()
    gx, gy, eta = embedding_vector(prog, fac)
    assert eta > 1.0
    wv = rng.standard_normal(prog.n + prog.m + 1)
    ux, uy, ut = hsde_subspace_step(prog, fac, gx, gy, eta, wv[:prog.n], wv[prog.n:-1], wv[-1])
    ref = np.linalg.solve(np.eye(prog.n + prog.m + 1) + _explicit_Q(prog), wv)
    np.testing.assert_allclose(np.concatenate([ux, uy, [ut]]), ref, atol=1e-11)


def test_admm_invariants_every_iterate():
    d = w.deconv_instance(30, 7, 1.5, 0.2, 1e-4, 4)
    prog = o.deconv_program(d["c"], d["b"])
    seen = []

    def cb(it, ux, uy, tau, vs, kappa):
        assert o.in_cone(uy, prog.l, prog.q, 1e-12)
        assert o.in_cone(vs, prog.l, prog.q, 1e-12)
        assert abs(uy @ vs) <= 1e-10 * (1 + np.linalg.norm(uy) * np.linalg.norm(vs))
        assert tau >= 0 and kappa >= -1e-15 and abs(tau * kappa) < 1e-12
        seen.append(it)

    o.scs_solve(prog, eps=1e-6, max_iters=300, callback=cb)
    assert len(seen) > 10


# ----------------------------------------------------------------- whole solver

def _nnls_bruteforce(C, b):
    n = C.shape[1]
    best, xb = np.linalg.norm(b), np.zeros(n)
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            xs = np.linalg.lstsq(C[:, S], b, rcond=None)[0]
            if np.all(xs > 0):
                f = np.linalg.norm(C[:, S] @ xs - b)
                if f < best:
                    best = f
                    xb = np.zeros(n)
                    xb[list(S)] = xs
    return best, xb


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_deconv_matches_bruteforce_nnls(seed):
    rng = np.random.default_rng(seed)
    c = np.abs(rng.standard_normal(3)) + 0.2
    b = rng.standard_normal(10 + 2)
    fstar, xstar = _nnls_bruteforce(conv_matrix(c, 10), b)
    res = o.scs_solve(o.deconv_program(c, b), eps=1e-9, max_iters=200_000)
    assert res.status == "solved"
    f = o.deconv_objective(c, b, res.x[:10])
    assert abs(f - fstar) <= 1e-6 * max(1.0, fstar)
    np.testing.assert_allclose(res.x[:10], xstar, atol=1e-5)


def _lp_vertex_enum(G, h, c):
    """min c^T x s.t. G x <= h by enumerating all vertices (bounded LP)."""
    m, n = G.shape
    best, xb = np.inf, None
    for rows in itertools.combinations(range(m), n):
        Gs = G[list(rows)]
        if abs(np.linalg.det(Gs)) < 1e-12:
            continue
        x = np.linalg.solve(Gs, h[list(rows)])
        if np.all(G @ x <= h + 1e-9) and c @ x < best:
            best, xb = c @ x, x
    return best, xb


@pytest.mark.parametrize("seed", range(4))
def test_lp_matches_vertex_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 3, 9
    G = rng.standard_normal((m, n))
    G = np.vstack([G, np.eye(n), -np.eye(n)])   # box keeps it bounded
    h = np.concatenate([np.abs(rng.standard_normal(m)) + 0.5, 2 * np.ones(2 * n)])
    c = rng.standard_normal(n)
    fstar, xstar = _lp_vertex_enum(G, h, c)
    res = o.scs_solve(o.dense_program(G, h, c, G.shape[0]), eps=1e-9, max_iters=200_000)
    assert res.status == "solved"
    assert abs(res.pobj - fstar) <= 1e-6 * max(1.0, abs(fstar))
    np.testing.assert_allclose(res.x, xstar, atol=1e-5)


def test_infeasible_lp_certificate():
    # x >= 1 and x <= 0:  s1 = x - 1 >= 0 (A=-1, b=-1), s2 = -x >= 0 (A=1, b=0)
    prog = o.dense_program(np.array([[-1.0], [1.0]]), np.array([-1.0, 0.0]), np.array([0.0]), 2)
    res = o.scs_solve(prog, eps=1e-7, max_iters=50_000)
    assert res.status == "infeasible"
    y = res.y
    assert np.all(y >= -1e-9) and prog.b @ y < 0 and np.linalg.norm(prog.AT(y)) < 1e-6


def test_unbounded_lp_certificate():
    # minimise -x subject to x >= 0
    prog = o.dense_program(np.array([[-1.0]]), np.array([0.0]), np.array([-1.0]), 1)
    res = o.scs_solve(prog, eps=1e-7, max_iters=50_000)
    assert res.status == "unbounded"
    assert prog.c @ res.x < 0 and np.linalg.norm(prog.A(res.x) + res.s) < 1e-6


def test_identity_kernel_deconv_is_clipping():
    rng = np.random.default_rng(7)
    b = rng.standard_normal(25)
    res = o.scs_solve(o.deconv_program(np.array([1.0]), b), eps=1e-9)
    np.testing.assert_allclose(res.x[:25], np.maximum(b, 0), atol=1e-7)
    assert abs(res.pobj - np.linalg.norm(np.minimum(b, 0))) < 1e-7


def test_lasso_orthonormal_design_soft_threshold():
    rng = np.random.default_rng(8)
    Qm, _ = np.linalg.qr(rng.standard_normal((30, 12)))
    b = rng.standard_normal(30)
    lam = 0.4
    g = Qm.T @ b
    xstar = np.sign(g) * np.maximum(np.abs(g) - lam, 0)
    res = o.scs_solve(o.lasso_program(Qm, b, lam), eps=1e-9)
    np.testing.assert_allclose(res.x[:12], xstar, atol=1e-6)


def test_lasso_large_lambda_gives_zero():
    d = w.lasso_instance(20, 30, 0.2, 1e-4, 3, lam_factor=1.0)   # lam = ||A^T b||_inf
    res = o.scs_solve(o.lasso_program(d["A"], d["b"], d["lam"] * 1.01), eps=1e-9)
    assert np.max(np.abs(res.x[:30])) < 1e-6


@pytest.mark.parametrize("alpha", [1.0, 1.8])
def test_solution_independent_of_relaxation(alpha):
    d = w.lasso_instance(30, 40, 0.1, 1e-4, 12)
    prog = o.lasso_program(d["A"], d["b"], d["lam"])
    r1 = o.scs_solve(prog, eps=1e-9, alpha=1.5)
    r2 = o.scs_solve(prog, eps=1e-9, alpha=alpha)
    np.testing.assert_allclose(r1.x[:40], r2.x[:40], atol=1e-6)


def test_deconv_small_workload_against_nnls_and_noise_bound():
    cfg = w.workload("deconv_n1000_k101")
    d = w.make_deconv(cfg)
    ref = o.polish_deconv(d["c"], d["b"])
    assert ref["kkt_ok"]
    noise = d["b"] - np.convolve(d["c"], d["x_true"])
    assert ref["obj"] <= np.linalg.norm(noise)          # x_true is feasible
    res = o.scs_solve(o.deconv_program(d["c"], d["b"]), eps=1e-4)
    assert res.status == "solved"
    f = o.deconv_objective(d["c"], d["b"], res.x[:cfg["n"]])
    assert ref["obj"] <= f + 1e-12
    # a 1e-4 residual stop leaves the objective of this ill-conditioned blur
    # within a few 1e-3 of the optimum
    assert (f - ref["obj"]) / ref["obj"] < 5e-3


# ----------------------------------------------------------------- equilibration

def _small_programs():
    rng = np.random.default_rng(21)
    d = w.deconv_instance(40, 9, 2.0, 0.2, 1e-4, 5)
    yield o.deconv_program(d["c"], d["b"])
    d = w.lasso_instance(15, 11, 0.2, 1e-4, 6)
    yield o.lasso_program(d["A"], d["b"], d["lam"])
    G = rng.standard_normal((9, 4))
    yield o.dense_program(G, rng.random(9), rng.standard_normal(4), 4, [5])
    d = w.conv_lasso_instance(12, 5, 1.5, 1e-4, 7)
    yield o.conv_lasso_program(d["c"], d["b"], d["lam"])


def test_partition_merges_overlaps_and_keeps_gaps():
    from oracle.equil import partition
    g = partition(12, [(2, 5), (4, 7), (9, 10)])
    assert g.tolist() == [0, 0, 1, 1, 1, 1, 1, 2, 2, 3, 4, 4]
    assert partition(3, []).tolist() == [0, 0, 0]


def test_groups_of_the_canonical_forms():
    """Deconv: rows {x >= 0}, {the SOC}; columns {x}, {t}.  Lasso: the two
    nonnegative row blocks and the SOC; columns {x}, {t}, {u}.  One dense block:
    one group each way."""
    from oracle.equil import groups
    dec, las, den, _ = _small_programs()
    rg, cg = groups(dec)
    assert np.bincount(rg).tolist() == [40, 40 + 9] and np.bincount(cg).tolist() == [40, 1]
    rg, cg = groups(las)
    assert np.bincount(rg).tolist() == [11, 11, 17] and np.bincount(cg).tolist() == [11, 11, 1]
    rg, cg = groups(den)
    assert np.bincount(rg).tolist() == [9] and np.bincount(cg).tolist() == [4]


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_group_norms_and_squared_apply_against_explicit(which):
    from oracle.equil import groups, group_norms
    prog = list(_small_programs())[which]
    A = prog.explicit()
    rg, cg = groups(prog)
    F = group_norms(prog, rg, cg)
    for g in range(F.shape[0]):
        for h in range(F.shape[1]):
            assert np.isclose(F[g, h], (A[np.ix_(rg == g, cg == h)] ** 2).sum(), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_equilibrated_operator_properties(which):
    """The scaled matrix D A E: the cone is preserved (D constant on each SOC),
    its group RMS row norms agree across row groups and its column norms across
    column groups (the Ruiz fixed point), the
    structured factorisation solves I + (DAE)^T (DAE), and the scaled data are
    sigma_b D b, sigma_c E c.  (Rows and columns cannot both reach RMS 1
    when one group spans an m x n block: their ratio is sqrt(n / m).)"""
    prog = list(_small_programs())[which]
    s = o.equilibrate(prog)
    start = prog.l
    for qq in prog.q:
        assert np.all(s.D[start:start + qq] == s.D[start])
        start += qq
    As = s.D[:, None] * prog.explicit() * s.E[None, :]
    rn = np.linalg.norm(As, axis=1) ** 2
    cn = np.linalg.norm(As, axis=0) ** 2
    rms_r = np.sqrt(np.bincount(s.row_groups, rn) / np.bincount(s.row_groups))
    rms_c = np.sqrt(np.bincount(s.col_groups, cn) / np.bincount(s.col_groups))
    assert rms_r.max() / rms_r.min() < 1.05 and rms_c.max() / rms_c.min() < 1.05, (rms_r, rms_c)
    sp = o.scaled_program(prog, s)
    rng = np.random.default_rng(which)
    r = rng.standard_normal(prog.n)
    np.testing.assert_allclose(sp.factor().solve(r), np.linalg.solve(np.eye(prog.n) + As.T @ As, r),
                               rtol=1e-10, atol=1e-12)
    x = rng.standard_normal(prog.n)
    np.testing.assert_allclose(sp.A(x), As @ x, atol=1e-12)
    np.testing.assert_allclose(sp.b, s.sigma_b * s.D * prog.b)
    np.testing.assert_allclose(sp.c, s.sigma_c * s.E * prog.c)


@pytest.mark.parametrize("family", ["deconv", "lasso"])
def test_solution_independent_of_equilibration(family):
    """Same optimum with and without the scaling, and the reported residuals are
    those of the returned (unscaled) point on the original data."""
    if family == "deconv":
        d = w.deconv_instance(60, 11, 2.0, 0.2, 1e-4, 8)
        prog = o.deconv_program(d["c"], d["b"])
        C, b = conv_matrix(d["c"], 60), d["b"]
        xs, _ = nnls(C, b)
        ref = np.linalg.norm(C @ xs - b)
        f = lambda r: np.linalg.norm(C @ np.maximum(r.x[:60], 0) - b)
    else:
        d = w.lasso_instance(30, 40, 0.1, 1e-4, 12)
        prog = o.lasso_program(d["A"], d["b"], d["lam"])
        x0 = o.scs_solve(prog, eps=1e-8, normalize=0).x[:40]
        pol = o.polish_lasso(d["A"], d["b"], d["lam"], x0)
        assert pol["kkt_ok"]
        ref = pol["obj"]
        f = lambda r: o.lasso_objective(d["A"], d["b"], d["lam"], r.x[:40])
    for norm in (0, 1, 2):
        r = o.scs_solve(prog, eps=1e-9, normalize=norm, max_iters=200_000)
        assert r.status == "solved"
        assert abs(f(r) - ref) <= 1e-7 * (1 + ref), (norm, f(r), ref)
        rp, rd, gap, _, _ = residuals(prog, r.x, r.y, 1.0, r.s)
        assert np.isclose(rp, r.res_pri, rtol=1e-6, atol=1e-15)
        assert np.isclose(rd, r.res_dual, rtol=1e-6, atol=1e-15)
        assert max(rp, rd, gap) <= 1e-9


def test_jacobi_diagonal_is_block_constant():
    """Why the CG has no Jacobi preconditioner: diag(I + A^T A) of the
    canonical forms is constant on every block for convolution and identity
    blocks (each column of a full convolution holds the whole kernel), and for
    the dense lasso block its extreme ratio is close to 1 (the squared column
    norms of an m x n N(0, 1/m) matrix spread by sqrt(2/m))."""
    d = w.deconv_instance(50, 9, 2.0, 0.2, 1e-4, 5)
    for prog in (o.deconv_program(d["c"], d["b"]),
                 o.conv_lasso_program(d["c"], d["b"], 0.1)):
        A = prog.explicit()
        diag = 1.0 + (A * A).sum(axis=0)
        for _, _, c0, cols in prog.blocks:
            blk = diag[c0:c0 + cols]
            assert np.ptp(blk) <= 1e-12 * blk.max()
    A = w.lasso_matrix(5000, 10000, 1003)
    dx = 3.0 + 4.0 * (A * A).sum(axis=0)
    assert dx.max() / dx.min() < 1.15
