"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every test prints its case name before touching the GPU.  Sizes span several
tiles plus a ragged tail (vector tiles of 1024, convolution tiles of 1024/2048
outputs, tap chunks of 256/512, dense tiles of 4 rows).
"""
import numpy as np
import pytest

import oracle as o
import workloads as w

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1609_03488_amd")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _say(*a):
    print("[case]", *a, flush=True)


def _solver(pr, precision, batch=1, **kw):
    st = P.Settings.make(precision=precision, **kw)
    s = P.Solver(pr.op, pr.l, pr.q, st, batch=batch)
    return s


def _cases():
    out = []
    d = w.deconv_instance(3000, 101, 15.0, 0.1, 1e-4, 11)
    out.append(("deconv_n3000_k101", P.deconv_problem(d["c"], d["b"]),
                o.deconv_program(d["c"], d["b"])))
    d = w.deconv_instance(5000, 1025, 150.0, 0.01, 1e-6, 12)
    out.append(("deconv_n5000_k1025", P.deconv_problem(d["c"], d["b"]),
                o.deconv_program(d["c"], d["b"])))
    d = w.lasso_instance(300, 700, 0.05, 1e-4, 13)
    out.append(("lasso_300x700", P.lasso_problem(d["A"], d["b"], d["lam"]),
                o.lasso_program(d["A"], d["b"], d["lam"])))
    d = w.conv_lasso_instance(1500, 301, 60.0, 1e-4, 14)
    out.append(("lasso_conv_n1500_k301", P.conv_lasso_problem(d["c"], d["b"], d["lam"]),
                o.conv_lasso_program(d["c"], d["b"], d["lam"])))
    return out


CASES = _cases()


# ----------------------------------------------------------------- a2, a3: applies

def _abs_bound(prog, v, adj):
    """sum_j |a_ij| |v_j| per output (what floating-point error of the apply scales with)."""
    v = np.abs(v)
    if prog.family == "deconv":
        n, c = prog.data["n"], np.abs(prog.data["c"])
        if not adj:
            return np.concatenate([v[:n], [v[n]], np.convolve(c, v[:n])])
        return np.concatenate([v[:n] + np.correlate(v[n + 1:], c, "valid"), [v[n]]])
    if prog.family == "lasso_conv":
        n, m0, c = prog.data["n"], prog.data["m"], np.abs(prog.data["c"])
        if not adj:
            xt = v[:n] + v[n:2 * n]
            return np.concatenate([xt, xt, [v[2 * n]], 2 * np.convolve(c, v[:n]), [v[2 * n]]])
        y12 = v[:n] + v[n:2 * n]
        return np.concatenate([y12 + 2 * np.correlate(v[2 * n + 1:2 * n + 1 + m0], c, "valid"), y12,
                               [v[2 * n] + v[-1]]])
    n, m0, A = prog.data["n"], prog.data["m"], np.abs(prog.data["A"])
    if not adj:
        xt = v[:n] + v[n:2 * n]
        return np.concatenate([xt, xt, [v[2 * n]], 2 * (A @ v[:n]), [v[2 * n]]])
    y12 = v[:n] + v[n:2 * n]
    return np.concatenate([y12 + 2 * (A.T @ v[2 * n + 1:2 * n + 1 + m0]), y12,
                           [v[2 * n] + v[-1]]])


FFT_L = 2048


def _fft_term(prog, v, adj, D, E):
    """Normwise rounding term of the FFT convolution engine for every output:
    an FP32 transform of L points (forward and inverse, about 3 flops per
    stage and value) perturbs the circular correlation by at most
    ~ c log2(L) u ||W||_inf ||u_window||_2 with ||W||_inf <= ||w||_1; c = 12 is
    generous.  Two windows share one complex transform, so the window norm is
    that of both (sqrt 2 times the largest length-L window of the input)."""
    if prog.family not in ("deconv", "lasso_conv"):
        return 0.0
    n, c = prog.data["n"], prog.data["c"]
    k = c.shape[0]
    scale = 1.0 if prog.family == "deconv" else 2.0
    if not adj:
        src, dsc = (E * v)[:n], D[-(n + k - 1):].max() if prog.family == "deconv" else D[2 * n + 1:2 * n + 1 + n + k - 1].max()
        cin = src
    else:
        r0 = n + 1 if prog.family == "deconv" else 2 * n + 1
        cin = (D * v)[r0:r0 + n + k - 1]
        dsc = E[:n].max()
    sq = np.concatenate([[0.0], np.cumsum(cin * cin)])
    L = min(FFT_L, cin.shape[0])
    win = np.sqrt(np.max(sq[L:] - sq[:-L])) if cin.shape[0] >= L else np.sqrt(sq[-1])
    return 12 * np.log2(FFT_L) * 2.0 ** -24 * scale * dsc * np.abs(c).sum() * np.sqrt(2) * win


@pytest.mark.parametrize("norm", [0, 2], ids=["given", "equilibrated"])
@pytest.mark.parametrize("prec,mfma", [(P.FP64, 0), (P.FP32, 0), (P.FP32, 1), (P.FP32, 2)],
                         ids=["fp64", "fp32-valu", "fp32-mfma", "fp32-fft"])
@pytest.mark.parametrize("idx", range(len(CASES)))
def test_forward_and_adjoint_apply(idx, prec, mfma, norm):
    """Elementwise: |dev - ref| <= (K + 4) u sum_j |a_ij||v_j|, with u the unit
    roundoff of the working precision and K the number of terms accumulated in
    that precision (convolution taps; the dense block accumulates in FP64).
    FP32 convolutions run on the vector ALU or on the matrix cores; on the FFT
    engine the convolution's rounding is normwise per window and its bound is
    added (_fft_term).  With equilibration the device applies D A E, the
    oracle's scaled operator."""
    name, pr, prog = CASES[idx]
    _say("apply", name, prec, "mfma" if mfma else "valu", "norm" if norm else "given")
    s = _solver(pr, prec, conv_mfma=mfma, normalize=norm)
    rng = np.random.default_rng(idx)
    z = rng.standard_normal(prog.n)
    y = rng.standard_normal(prog.m)
    az = s.apply(z)
    aty = s.apply(y, transpose=True)
    # the library's scaling (it agrees with the oracle's to ~1e-14, checked on
    # the CPU; the FP64 bound here is tighter than that)
    if norm:
        D, E, _ = pr.op.equilibrate(pr.l, pr.q, level=norm)
    else:
        D, E = np.ones(prog.m), np.ones(prog.n)
    ref_az, ref_aty = D * prog.A(E * z), E * prog.AT(D * y)
    u = 2.0 ** -53 if prec == P.FP64 else 2.0 ** -24
    K = prog.data.get("k", 4) + 4
    # |D A E| |v| = D (|A| (E |v|))
    bf = D * _abs_bound(prog, E * z, False)
    ba = E * _abs_bound(prog, D * y, True)
    tf = _fft_term(prog, z, False, D, E) if mfma == 2 else 0.0
    ta = _fft_term(prog, y, True, D, E) if mfma == 2 else 0.0
    assert np.all(np.abs(az - ref_az) <= (K + 4) * u * bf + tf + 1e-300)
    assert np.all(np.abs(aty - ref_aty) <= (K + 4) * u * ba + ta + 1e-300)
    # adjoint identity on the device results
    assert abs(az @ y - z @ aty) <= (4 * (K + 4) * u * (bf @ np.abs(y) + ba @ np.abs(z)) +
                                     tf * np.abs(y).sum() + ta * np.abs(z).sum())


def test_identity_kernel_conv_is_exact():
    _say("conv k=1")
    b = np.linspace(-1, 1, 2500)
    pr = P.deconv_problem(np.array([1.0]), b)
    s = _solver(pr, P.FP64, normalize=0)
    z = np.concatenate([np.arange(2500.0), [3.0]])
    out = s.apply(z)
    np.testing.assert_array_equal(out[:2500], -np.arange(2500.0))
    np.testing.assert_array_equal(out[2501:], -np.arange(2500.0))


# ----------------------------------------------------------------- a4: CG

@pytest.mark.parametrize("prec,engine", [(P.FP64, 0), (P.FP32, 1), (P.FP32, 2)],
                         ids=["fp64", "fp32-mfma", "fp32-fft"])
@pytest.mark.parametrize("idx", range(len(CASES)))
def test_cg_matches_direct_solve(idx, prec, engine):
    name, pr, prog = CASES[idx]
    _say("cg", name, prec, engine)
    s = _solver(pr, prec, conv_mfma=engine)
    rng = np.random.default_rng(100 + idx)
    r = rng.standard_normal(prog.n)
    tol = 1e-12 if prec == P.FP64 else 1e-6
    z, it = s.normal_solve(r, tol=tol, max_iters=500)
    ref = o.prepare(prog)[0].factor().solve(r)   # I + (D A E)^T (D A E)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    assert err < (1e-10 if prec == P.FP64 else 2e-5), err
    assert 0 < it < 500
    # warm start at the solution: no iteration needed
    z2, it2 = s.normal_solve(r, z0=ref, tol=1e-6, max_iters=50)
    assert it2 <= 1


# ----------------------------------------------------------------- a5-a6: iterates

def _iter_cases():
    out = []
    d = w.deconv_instance(1200, 31, 4.0, 0.1, 1e-4, 21)
    out.append(("deconv_n1200_k31", P.deconv_problem(d["c"], d["b"]),
                o.deconv_program(d["c"], d["b"])))
    d = w.lasso_instance(120, 300, 0.05, 1e-4, 22)
    out.append(("lasso_120x300", P.lasso_problem(d["A"], d["b"], d["lam"]),
                o.lasso_program(d["A"], d["b"], d["lam"])))
    # a generic program with a nonnegative block and several second-order cones
    rng = np.random.default_rng(23)
    m, n, l, q = 1500, 40, 500, [1, 3, 996]
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x0 = rng.standard_normal(n)
    s0 = o.proj_cone(rng.standard_normal(m), l, q)
    b = A @ x0 + s0
    y0 = o.proj_cone(rng.standard_normal(m), l, q)
    c = -A.T @ y0
    op = P.Operator(m, n).add_dense(0, 0, A)
    from paper_1609_03488_amd.problems import ConeProblem
    out.append(("socp_1500x40", ConeProblem(op, l, q, b, c, n), o.dense_program(A, b, c, l, q)))
    d = w.conv_lasso_instance(700, 61, 12.0, 1e-4, 24)
    out.append(("lasso_conv_n700_k61", P.conv_lasso_problem(d["c"], d["b"], d["lam"]),
                o.conv_lasso_program(d["c"], d["b"], d["lam"])))
    return out


ITER_CASES = _iter_cases()


@pytest.mark.parametrize("fused", [0, 65536], ids=["multikernel", "fused"])
@pytest.mark.parametrize("idx", range(len(ITER_CASES)))
def test_admm_iterates_match_oracle(idx, fused):
    """FP64 with CG solved to 1e-13: after N steps the embedding state matches
    the oracle (exact subspace solve) element by element, on both execution
    paths (one launch per kernel, or whole steps in one workgroup)."""
    name, pr, prog = ITER_CASES[idx]
    _say("iterates", name, "fused" if fused else "multikernel")
    N = 25
    s = _solver(pr, P.FP64, cg_tol=0.0, cg_floor=1e-13, cg_max_iters=60, setup_tol=1e-14,
                setup_max_iters=2000, fused_max=fused)
    s.set_data(0, pr.b, pr.c)
    s.iterate(N)
    ux, uy, tau, vs, kap = s.state(0)
    ref = o.scs_solve(prog, eps=1e-300, max_iters=N)
    rux, ruy, rtau, rvs, rkap = ref.u
    scale = max(1.0, np.abs(rux).max(), np.abs(ruy).max(), np.abs(rvs).max())
    for a, b_ in ((ux, rux), (uy, ruy), (vs, rvs)):
        assert np.abs(a - b_).max() <= 1e-8 * scale
    assert abs(tau - rtau) <= 1e-8 * max(1, rtau) and abs(kap - rkap) <= 1e-8 * max(1, rkap)
    # cone membership and complementarity of the device iterate
    assert o.in_cone(uy, prog.l, prog.q, 1e-12 * scale)
    assert o.in_cone(vs, prog.l, prog.q, 1e-12 * scale)
    assert abs(uy @ vs) <= 1e-9 * scale ** 2


@pytest.mark.parametrize("idx", range(len(ITER_CASES)))
def test_residuals_match_oracle(idx):
    name, pr, prog = ITER_CASES[idx]
    _say("residuals", name)
    s = _solver(pr, P.FP64, cg_tol=0.0, cg_floor=1e-13, cg_max_iters=60, setup_tol=1e-14)
    s.set_data(0, pr.b, pr.c)
    s.iterate(15)
    ux, uy, tau, vs, kap = s.state(0)
    info = s.residuals()[0]
    for _ in range(20):   # the embedding can start with tau = 0; ratios are then undefined
        if tau > 0.0:
            break
        assert np.isinf(info["res_pri"]) and np.isinf(info["res_dual"])
        s.iterate(10)
        ux, uy, tau, vs, kap = s.state(0)
        info = s.residuals()[0]
    assert tau > 0.0
    # the state is that of the equilibrated problem; the residuals are the original's
    x, y, sl = o.prepare(prog, 1)[1].unscale(ux, uy, 1.0, vs)
    rp, rd, gap, pobj, dobj = o.scs.residuals(prog, x, y, tau, sl)
    np.testing.assert_allclose([info["res_pri"], info["res_dual"], info["gap"]], [rp, rd, gap],
                               rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose([info["pobj"], info["dobj"]], [pobj, dobj], rtol=1e-9, atol=1e-12)


# ----------------------------------------------------------------- whole solves

def _objective(prog, x):
    if prog.family == "deconv":
        return o.deconv_objective(prog.data["c"], prog.data["b_obs"], x[:prog.data["n"]])
    if prog.family == "lasso_conv":
        xs = x[:prog.data["n"]]
        r = np.convolve(prog.data["c"], xs) - prog.data["b_obs"]
        return float(0.5 * (r @ r) + prog.data["lam"] * np.sum(np.abs(xs)))
    return o.lasso_objective(prog.data["A"], prog.data["b_obs"], prog.data["lam"], x[:prog.data["n"]])


@pytest.mark.parametrize("fused", [0, 65536], ids=["multikernel", "fused"])
@pytest.mark.parametrize("idx,prec,eps,engine", [(0, P.FP64, 1e-4, 0), (0, P.FP32, 1e-4, 1),
                                                  (0, P.FP32, 1e-4, 2),
                                                  (1, P.FP64, 1e-6, 0), (1, P.FP32, 1e-5, 1),
                                                  (3, P.FP64, 1e-4, 0), (3, P.FP32, 1e-4, 1),
                                                  (3, P.FP32, 1e-4, 2)])
def test_solve_matches_oracle(idx, prec, eps, engine, fused):
    """Same method, same tolerance: the natural objective of the GPU solution is
    within 1e-4 (relative) of the oracle's, and the GPU point's residuals,
    recomputed in FP64, meet the tolerance.  At a 1e-4 stop the lasso's
    objective is itself only ~1e-4 accurate (a 1.3e-4 spread was measured
    between the FP32 and FP64 stopping points), so its FP32 case stops at 1e-5;
    the deconvolution's FP32 and FP64 trajectories stay together at 1e-4."""
    name, pr, prog = ITER_CASES[idx]
    _say("solve", name, prec, eps, engine, fused)
    s = _solver(pr, prec, eps=eps, check_every=10, fused_max=fused, conv_mfma=engine)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    # residuals of the returned point, recomputed in FP64 by the oracle
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * eps
    ref = o.scs_solve(prog, eps=eps, check_every=10)
    f, fr = _objective(prog, x), _objective(prog, ref.x)
    if prog.family == "lasso_conv":
        # the iteration converges slowly on a blur operator (no 1e-6 point in
        # 1e5 oracle iterations), and an eps = 1e-4 point's objective is only
        # ~1e-3 accurate: the GPU point is held to the oracle's own eps-solution
        # against the KKT-certified optimum
        from oracle.program import conv_matrix
        n0 = prog.data["n"]
        pol = o.polish_lasso(conv_matrix(prog.data["c"], n0), prog.data["b_obs"], prog.data["lam"],
                             ref.x[:n0])
        assert pol["kkt_ok"]
        opt = pol["obj"]
        assert f >= opt * (1 - 1e-12) and fr >= opt * (1 - 1e-12)
        assert f - opt <= 2 * (fr - opt) + 1e-4 * opt, (f, fr, opt)
        return
    assert abs(f - fr) / abs(fr) <= 1e-4, (f, fr)


def test_status_outcomes():
    _say("status")
    # infeasible: x >= 1 and x <= 0
    op = P.Operator(2, 1).add_dense(0, 0, np.array([[-1.0], [1.0]]))
    s = P.Solver(op, 2, [], P.Settings.make(precision=P.FP64, eps=1e-7, check_every=1, max_iters=50000))
    s.set_data(0, np.array([-1.0, 0.0]), np.array([0.0]))
    assert s.solve()[0]["status"] == P.INFEASIBLE
    _, y, _ = s.solution(0)
    assert np.all(y >= -1e-9) and -1.0 * y[0] + 0.0 * y[1] < 0
    # unbounded: minimise -x, x >= 0
    op = P.Operator(1, 1).add_dense(0, 0, np.array([[-1.0]]))
    s = P.Solver(op, 1, [], P.Settings.make(precision=P.FP64, eps=1e-7, check_every=1, max_iters=50000))
    s.set_data(0, np.array([0.0]), np.array([-1.0]))
    assert s.solve()[0]["status"] == P.UNBOUNDED
    x, _, _ = s.solution(0)
    assert x[0] > 0 and abs(-x[0] + 1.0) < 1e-6
    # iteration limit
    name, pr, prog = ITER_CASES[0]
    s = _solver(pr, P.FP32, max_iters=1, check_every=1)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.MAX_ITERS and info["iters"] == 1
    # non-finite data are rejected before any device work
    with pytest.raises(P.CgsError) as e:
        s.set_data(0, np.full(pr.op.m, np.nan), pr.c)
    assert e.value.code == -1


def test_warm_start_resumes():
    name, pr, prog = ITER_CASES[1]
    _say("warm start", name)
    s = _solver(pr, P.FP64, cg_tol=0.0, cg_floor=1e-13, cg_max_iters=60, setup_tol=1e-14)
    s.set_data(0, pr.b, pr.c)
    s.iterate(10)
    st = s.state(0)
    s.iterate(10)
    a = s.state(0)
    s2 = _solver(pr, P.FP64, cg_tol=0.0, cg_floor=1e-13, cg_max_iters=60, setup_tol=1e-14)
    s2.set_data(0, pr.b, pr.c)
    s2.set_state(0, st[0], st[1], st[2], st[3], st[4])
    s2.iterate(10)
    b_ = s2.state(0)
    np.testing.assert_allclose(a[0], b_[0], atol=1e-9)
    np.testing.assert_allclose(a[1], b_[1], atol=1e-9)


# ----------------------------------------------------------------- batch and server

def test_batch_instances_equal_single_solves():
    _say("batch")
    A = w.lasso_matrix(150, 400, 31)
    insts = [w.lasso_instance(150, 400, 0.05, 1e-4, 3100 + i, A=A, matrix_seed=31) for i in range(3)]
    prs = [P.lasso_problem(A, d["b"], d["lam"]) for d in insts]
    st = dict(eps=1e-5, check_every=10, cg_adaptive=0)
    sb = _solver(prs[0], P.FP32, batch=3, **st)
    for i, pr in enumerate(prs):
        sb.set_data(i, pr.b, pr.c)
    infos = sb.solve()
    for i, pr in enumerate(prs):
        s1 = _solver(pr, P.FP32, **st)
        s1.set_data(0, pr.b, pr.c)
        i1 = s1.solve()[0]
        assert infos[i]["status"] == P.SOLVED and i1["status"] == P.SOLVED
        assert infos[i]["iters"] == i1["iters"]
        np.testing.assert_array_equal(sb.solution(i)[0], s1.solution(0)[0])


def _spec_cases():
    d1 = w.deconv_instance(3000, 101, 15.0, 0.1, 1e-4, 11)
    d2 = w.deconv_instance(20000, 1025, 150.0, 0.01, 1e-6, 13)
    A = w.lasso_matrix(300, 900, 41)
    d3 = w.lasso_instance(300, 900, 0.05, 1e-4, 4100, A=A, matrix_seed=41)
    return [("deconv_n3000_k101", P.deconv_problem(d1["c"], d1["b"])),
            ("deconv_n20000_k1025", P.deconv_problem(d2["c"], d2["b"])),
            ("lasso_300x900", P.lasso_problem(A, d3["b"], d3["lam"]))]


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_predicted_cg_launches_equal_full_launches(prec, graph):
    """cg_adaptive = 1 runs each check interval with the previous interval's
    most CG iterations per step as launches and runs an interval again from
    its snapshot when a step needed more; the iterates must equal those of
    cg_adaptive = 0 (cg_max_iters launches every step) bit for bit.  A fast
    tightening CG tolerance (cg_rate 3) makes the per-step need grow, so some
    interval is run again.  With a stream the intervals are captured and
    replayed as graphs (snapshot, suspension and rerun included)."""
    import torch
    reruns = 0
    for name, pr in _spec_cases():
        for rate in (1.5, 3.0):
            _say("predicted cg launches", name, prec, rate, "graph" if graph else "direct")
            out = {}
            for ad in (0, 1):
                st = P.Settings.make(precision=prec, eps=1e-5, check_every=10, fused_max=0, cg_rate=rate,
                                     cg_floor=1e-9, max_iters=3000, cg_adaptive=ad)
                s = P.Solver(pr.op, pr.l, pr.q, st, stream=torch.cuda.Stream() if graph else None)
                s.set_data(0, pr.b, pr.c)
                info = s.solve()[0]
                out[ad] = (info, s.solution(0), s.rounds())
            i0, i1 = out[0][0], out[1][0]
            assert (i0["status"], i0["iters"], i0["cg_iters"]) == (i1["status"], i1["iters"], i1["cg_iters"])
            for a, b in zip(out[0][1], out[1][1]):
                np.testing.assert_array_equal(a, b)
            print("[case] rounds/reruns", name, rate, out[1][2], "iters", i1["iters"], "cg", i1["cg_iters"],
                  flush=True)
            reruns += out[1][2][1]
    assert reruns > 0


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
def test_predicted_cg_launches_batch_equal_full_launches(graph):
    """The same with three instances in one solver: an interval that one
    instance needs to run again is run again for all of them (each restored from
    its own copy), and every instance's iterates equal those of
    cg_adaptive = 0 bit for bit."""
    import torch
    A = w.lasso_matrix(300, 900, 41)
    insts = [w.lasso_instance(300, 900, 0.05, 1e-4, 4100 + i, A=A, matrix_seed=41) for i in range(3)]
    prs = [P.lasso_problem(A, d["b"], d["lam"]) for d in insts]
    reruns = 0
    for rate in (1.5, 2.0, 2.5):
        _say("predicted cg launches, batch", rate)
        out = {}
        for ad in (0, 1):
            st = P.Settings.make(precision=P.FP32, eps=1e-5, check_every=10, fused_max=0, cg_rate=rate,
                                 cg_floor=1e-9, max_iters=2000, cg_adaptive=ad)
            s = P.Solver(prs[0].op, prs[0].l, prs[0].q, st, batch=3,
                         stream=torch.cuda.Stream() if graph else None)
            for i, pr in enumerate(prs):
                s.set_data(i, pr.b, pr.c)
            infos = s.solve()
            out[ad] = (infos, [s.solution(i) for i in range(3)], s.rounds())
        print("[case] rounds/reruns batch", rate, out[1][2], flush=True)
        reruns += out[1][2][1]
        for i in range(3):
            a, b = out[0][0][i], out[1][0][i]
            assert (a["status"], a["iters"], a["cg_iters"]) == (b["status"], b["iters"], b["cg_iters"]), i
            for u, v in zip(out[0][1][i], out[1][1][i]):
                np.testing.assert_array_equal(u, v)
    assert reruns > 0


def test_server_result_same_alone_and_in_mix():
    _say("server alone vs mix")
    reqs = [w.deconv_instance(n, k, k / 7.0, 0.05, 1e-4, 4000 + n) for n, k in
            ((1500, 41), (3700, 101), (900, 11), (2600, 65))]
    prs = [P.deconv_problem(d["c"], d["b"]) for d in reqs]
    # fused_max 8000: the (3700, 101) request runs one launch per kernel, the
    # others whole steps in one workgroup; both paths share the rounds
    st = P.Settings.make(precision=P.FP32, eps=1e-4, check_every=10, fused_max=8000)
    alone = []
    for pr in prs:
        sv = P.Server(64 << 20, 8, st)
        t = sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c)
        while sv.step(50):
            pass
        alone.append(sv.fetch(t))
        sv.close()
    sv = P.Server(64 << 20, 8, st)
    tickets = {}
    tickets[0] = sv.submit(prs[0].op, prs[0].l, prs[0].q, prs[0].b, prs[0].c)
    sv.step(30)
    tickets[1] = sv.submit(prs[1].op, prs[1].l, prs[1].q, prs[1].b, prs[1].c)
    tickets[2] = sv.submit(prs[2].op, prs[2].l, prs[2].q, prs[2].b, prs[2].c)
    sv.step(20)
    tickets[3] = sv.submit(prs[3].op, prs[3].l, prs[3].q, prs[3].b, prs[3].c)
    mixed = {}
    while len(mixed) < 4:
        sv.step(10)
        for i, t in tickets.items():
            if i not in mixed and sv.poll(t) != P.RUNNING:
                mixed[i] = sv.fetch(t)
    for i in range(4):
        xa, _, _, ia = alone[i]
        xm, _, _, im = mixed[i]
        assert ia["status"] == P.SOLVED and im["status"] == P.SOLVED
        assert ia["iters"] == im["iters"]
        np.testing.assert_array_equal(xa, xm)


def test_fused_result_same_with_vectors_in_lds_or_memory():
    """The fused kernel keeps an instance's most used vectors in LDS while they
    fit next to the convolution's staging area, whose size is set by the
    longest kernel in the launch.  Alone, every such vector of the (2500, 101)
    request fits (with 160 KB of LDS per workgroup); next to a 1365-tap
    request the staging area grows and z_y stays in global memory.  Where the
    values sit must not change them."""
    _say("fused lds residency")
    reqs = [w.deconv_instance(n, k, k / 7.0, 0.05, 1e-4, 4100 + n) for n, k in ((2500, 101), (3000, 1365))]
    prs = [P.deconv_problem(d["c"], d["b"]) for d in reqs]
    st = P.Settings.make(precision=P.FP32, eps=1e-4, check_every=10, fused_max=16384)
    alone = []
    for pr in prs:
        sv = P.Server(64 << 20, 8, st)
        t = sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c)
        while sv.step(50):
            pass
        alone.append(sv.fetch(t))
        sv.close()
    sv = P.Server(64 << 20, 8, st)
    tickets = [sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c) for pr in prs]
    while sv.step(50):
        pass
    mixed = [sv.fetch(t) for t in tickets]
    sv.close()
    for (xa, _, _, ia), (xm, _, _, im) in zip(alone, mixed):
        assert ia["status"] == P.SOLVED and im["status"] == P.SOLVED
        assert ia["iters"] == im["iters"]
        np.testing.assert_array_equal(xa, xm)


def test_server_results_match_oracle():
    """Served results against the oracle: a seeded Poisson trace with the
    serving workload's recipe (Section V-C deconvolution; log-uniform n, odd
    Gaussian kernels of length k with sigma = k / 7, 5 % nonzeros, noise
    variance 1e-4) at sizes the oracle solves in seconds, replayed through the
    continuous-batching server with fused (one workgroup) and one-launch-per-
    kernel requests in the same rounds.  Every request is solved and its
    natural objective is within 1e-4 of the oracle's run of the same method to
    the same eps (FP64, exact subspace solves, data scaling)."""
    from paper_1609_03488_amd.serve import replay
    _say("server vs oracle")
    trace = w.serving_trace(count=10, rate=400.0, seed=2005, n_lo=600, n_hi=4000, k_half_lo=5,
                            k_half_hi=60)
    data = {r.rid: w.serving_request_data(r) for r in trace}
    probs = {rid: P.deconv_problem(d["c"], d["b"]) for rid, d in data.items()}
    st = P.Settings.make(precision=P.FP32, eps=1e-4, check_every=10, cg_max_iters=3, fused_max=4000)
    res = replay(trace, lambda r: probs[r.rid], settings=st, workspace_bytes=256 << 20,
                 steps_per_call=10, keep_x=True)
    assert res["completed"] == len(trace) and res["solved"] == len(trace), res["solved"]
    for c in res["completions"]:
        d = data[c.rid]
        n = d["x_true"].shape[0]
        ref = o.scs_solve(o.deconv_program(d["c"], d["b"]), eps=1e-4, check_every=10)
        assert ref.status == "solved"
        f = o.deconv_objective(d["c"], d["b"], c.x)
        fr = o.deconv_objective(d["c"], d["b"], ref.x[:n])
        assert abs(f - fr) / fr <= 1e-4, (c.rid, n, f, fr)


def test_server_admission_by_memory():
    _say("server admission")
    d = w.deconv_instance(20000, 101, 15.0, 0.05, 1e-4, 77)
    pr = P.deconv_problem(d["c"], d["b"])
    need = P.Server.request_bytes(pr.op, pr.l, pr.q, P.FP32)
    sv = P.Server(24 << 20, 64, P.Settings.make(precision=P.FP32))
    used, free = sv.usage()
    assert used == 0
    fits = free // need
    assert fits >= 1
    tickets = [sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c) for _ in range(fits)]
    assert all(t is not None for t in tickets)
    assert sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c) is None      # refused: no memory
    sv.cancel(tickets[0])
    assert sv.submit(pr.op, pr.l, pr.q, pr.b, pr.c) is not None  # memory came back
    # slot limit
    sv2 = P.Server(64 << 20, 1, P.Settings.make(precision=P.FP32))
    assert sv2.submit(pr.op, pr.l, pr.q, pr.b, pr.c) is not None
    assert sv2.submit(pr.op, pr.l, pr.q, pr.b, pr.c) is None


# ----------------------------------------------------------------- a10: BF16 MFMA batch

def _lasso_batch(m, n, B, seed):
    A = w.lasso_matrix(m, n, seed)
    insts = [w.lasso_instance(m, n, 0.05, 1e-4, seed * 1000 + i, A=A, matrix_seed=seed)
             for i in range(B)]
    prs = [P.lasso_problem(A, d["b"], d["lam"]) for d in insts]
    progs = [o.lasso_program(A, d["b"], d["lam"]) for d in insts]
    return A, prs, progs


@pytest.mark.parametrize("B", [1, 37, 70])
def test_bf16_gemm_apply(B):
    """BF16 operands (RNE) with FP32 accumulation: |dev - ref| <= (2^-8 + K 2^-24) sum |a||v|."""
    _say("bf16 gemm apply", B)
    A, prs, progs = _lasso_batch(300, 700, B, 41)
    s = _solver(prs[0], P.BF16, batch=B, normalize=0)
    prog = progs[0]
    rng = np.random.default_rng(B)
    z = rng.standard_normal(prog.n)
    y = rng.standard_normal(prog.m)
    az, aty = s.apply(z), s.apply(y, transpose=True)
    bf, ba = _abs_bound(prog, z, False), _abs_bound(prog, y, True)
    tol = 2.0 ** -8 + 700 * 2.0 ** -24
    assert np.all(np.abs(az - prog.A(z)) <= tol * bf + 1e-30)
    assert np.all(np.abs(aty - prog.AT(y)) <= tol * ba + 1e-30)
    # and it is a BF16 product, not an FP32 one: the error is visible
    assert np.abs(az - prog.A(z)).max() > 1e-6 * np.abs(prog.A(z)).max()


BF16_EPS = 1e-5   # two-phase BF16 solves stop at eps / 10 (objective bar: 1e-4)


def test_bf16_batch_solve_matches_oracle():
    """Each instance's residuals (recomputed in FP64) are <= 1e-4 and its
    objective is within 1e-4 of the optimum (the oracle at 1e-6).  The relative
    criteria scale with 1 + ||b|| while the objective can be much smaller (here
    ~2.5 against ||b|| ~ 25), and a point at a 2.5e-5 residual was measured
    1.06e-4 off in objective, so the batch stops at 1e-5."""
    _say("bf16 batch solve")
    B = 12
    A, prs, progs = _lasso_batch(250, 600, B, 43)
    s = _solver(prs[0], P.BF16, batch=B, eps=BF16_EPS, check_every=10)
    for i, pr in enumerate(prs):
        s.set_data(i, pr.b, pr.c)
    infos = s.solve()
    for i in range(B):
        assert infos[i]["status"] == P.SOLVED, infos[i]
        x, y, sl = s.solution(i)
        rp, rd, gap, _, _ = o.scs.residuals(progs[i], x, y, 1.0, sl)
        assert max(rp, rd, gap) <= 1e-4, (i, rp, rd, gap)
        ref = o.scs_solve(progs[i], eps=1e-6, check_every=10)
        f, fr = _objective(progs[i], x), _objective(progs[i], ref.x)
        assert abs(f - fr) / abs(fr) <= 1e-4, (i, f, fr)


@pytest.mark.parametrize("prec,tdtype", [(P.FP32, "float32"), (P.FP64, "float64"), (P.BF16, "float32")],
                         ids=["fp32", "fp64", "bf16"])
def test_borrowed_dense_block_equals_host_copy(prec, tdtype):
    """A dense block read in place from a torch tensor on the GPU (never copied
    to the host) gives the same solve, bit for bit, as the same values copied
    from host FP64 memory: the block's norm (the scaling) and its conversion to
    the working precision are formed in the same order.  The solution also
    meets the oracle's residual test."""
    import torch
    _say("borrowed dense block", prec, tdtype)
    B = 4 if prec == P.BF16 else 1
    A, prs, progs = _lasso_batch(250, 600, B, 47)
    if tdtype == "float32":
        A = A.astype(np.float32).astype(np.float64)   # values an FP32 tensor holds exactly
    At = torch.tensor(A, dtype=getattr(torch, tdtype), device="cuda")
    out = []
    for a in (A, At):
        ps = [P.lasso_problem(a, pr.b[2 * 600 + 1:-1] / -2.0, float(pr.c[600])) for pr in prs]
        s = _solver(ps[0], prec, batch=B, eps=BF16_EPS if prec == P.BF16 else 1e-5, check_every=10,
                    normalize=2)
        for i, p_ in enumerate(ps):
            s.set_data(i, p_.b, p_.c)
        infos = s.solve()
        out.append([(inf["iters"], s.solution(i)) for i, inf in enumerate(infos)])
        del s
    for i in range(B):
        (it_h, (xh, yh, sh)), (it_d, (xd, yd, sd)) = out[0][i], out[1][i]
        assert it_h == it_d
        assert np.array_equal(xh, xd) and np.array_equal(yh, yd) and np.array_equal(sh, sd)
        prog = o.lasso_program(A, prs[i].b[2 * 600 + 1:-1] / -2.0, float(prs[i].c[600]))
        rp, rd, gap, _, _ = o.scs.residuals(prog, xd, yd, 1.0, sd)
        assert max(rp, rd, gap) <= 1e-4, (i, rp, rd, gap)


def test_borrowed_dense_block_must_be_device_memory():
    """A host pointer (or a device pointer of another kind) is refused with
    CGS_EINVAL instead of being dereferenced on the device."""
    lib = P.lib()
    A = np.ones((4, 3), dtype=np.float32)
    op = P.Operator(4, 3)
    assert lib.cgs_op_add_dense_ex(op._h, 0, 0, 4, 3, A.ctypes.data, 3, P.DTYPE_F32,
                                   P.MEM_DEVICE_BORROW, 1.0) == -1


# ----------------------------------------------------------------- autotuner

def test_autotune_keeps_results_within_bounds():
    """The autotuner only picks how the same products are computed: after it,
    the FP32 convolution applies and the BF16 GEMM applies stay inside the
    error bounds of the apply tests above."""
    name, pr, prog = CASES[1]
    _say("autotune conv", name)
    s = _solver(pr, P.FP32, normalize=0)
    ch = s.autotune(reps=3)
    assert ch["conv_mfma"] in (0, 1, 2) and ch["gemm_target_wgs"] == -1
    rng = np.random.default_rng(5)
    z = rng.standard_normal(prog.n)
    u, K = 2.0 ** -24, prog.data["k"] + 4
    one_m, one_n = np.ones(prog.m), np.ones(prog.n)
    tf = _fft_term(prog, z, False, one_m, one_n) if ch["conv_mfma"] == 2 else 0.0
    assert np.all(np.abs(s.apply(z) - prog.A(z)) <= (K + 4) * u * _abs_bound(prog, z, False) + tf)
    _say("autotune gemm")
    A, prs, progs = _lasso_batch(300, 700, 37, 41)
    s = _solver(prs[0], P.BF16, batch=37, normalize=0)
    ch = s.autotune(reps=3)
    assert ch["conv_mfma"] == -1 and ch["gemm_target_wgs"] in (128, 256, 512, 1024)
    y = rng.standard_normal(progs[0].m)
    tol = 2.0 ** -8 + 700 * 2.0 ** -24
    assert np.all(np.abs(s.apply(y, transpose=True) - progs[0].AT(y))
                  <= tol * _abs_bound(progs[0], y, True) + 1e-30)


@pytest.mark.parametrize("vec_tile", [1024, 2048])
@pytest.mark.parametrize("idx,prec,eps", [(0, P.FP32, 1e-4), (1, P.FP64, 1e-6), (2, P.FP32, 1e-4)])
def test_vector_tiles_solve_matches_oracle(idx, prec, eps, vec_tile):
    """Either vector tile length the autotuner chooses from gives a solution
    whose objective is within 1e-4 of the oracle's at the same eps (the tiles
    change only how the vector kernels and reductions split the work)."""
    name, pr, prog = ITER_CASES[idx]
    _say("vector tiles", name, prec, vec_tile)
    s = _solver(pr, prec, eps=eps, check_every=10, fused_max=0, vec_tile=vec_tile)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * eps, (rp, rd, gap)
    ref = o.scs_solve(prog, eps=eps, check_every=10)
    if prog.family in ("deconv", "lasso", "lasso_conv"):
        f, fr = _objective(prog, x), _objective(prog, ref.x)
    else:   # a generic program: its conic objective c^T x
        f, fr = float(prog.c @ x), float(prog.c @ ref.x)
    assert abs(f - fr) <= 1e-4 * max(1.0, abs(fr)), (f, fr)


def test_autotune_on_steps_then_solve():
    """With data on the instance the autotuner times whole ADMM steps for each
    engine and tile length, then restarts the instance: the following solve
    starts from u = v = (0, 0, 1) and matches the oracle."""
    import torch
    name, pr, prog = CASES[1]
    _say("autotune on steps", name)
    s = P.Solver(pr.op, pr.l, pr.q, P.Settings.make(precision=P.FP32, eps=1e-4, fused_max=0),
                 stream=torch.cuda.Stream())
    s.set_data(0, pr.b, pr.c)
    ch = s.autotune(reps=3)
    assert ch["conv_mfma"] in (0, 1, 2) and ch["vec_tile"] in (1024, 2048) and ch["gemm_target_wgs"] == -1
    ux, uy, tau, vs, kappa = s.state(0)
    assert tau == 1.0 and kappa == 1.0 and not ux.any() and not uy.any() and not vs.any()
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, _, _ = s.solution(0)
    ref = o.scs_solve(prog, eps=1e-4, check_every=10)
    f, fr = _objective(prog, x), _objective(prog, ref.x)
    assert abs(f - fr) / abs(fr) <= 1e-4, (f, fr)


@pytest.mark.parametrize("fused", [0, 65536], ids=["multikernel", "fused"])
@pytest.mark.parametrize("idx,prec,eps", [(0, P.FP32, 1e-4), (1, P.FP64, 1e-6)])
def test_solve_with_block_equilibration_matches_oracle(idx, prec, eps, fused):
    """normalize = 2 (Ruiz-balanced blocks, then b and c) on both sides."""
    name, pr, prog = ITER_CASES[idx]
    _say("solve normalize=2", name, prec, eps, fused)
    s = _solver(pr, prec, eps=eps, check_every=10, fused_max=fused, normalize=2,
                cg_max_iters=40)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * eps
    ref = o.scs_solve(prog, eps=eps, check_every=10, normalize=2)
    f, fr = _objective(prog, x), _objective(prog, ref.x)
    assert abs(f - fr) / abs(fr) <= 1e-4, (f, fr)


@pytest.mark.parametrize("mfma", [0, 1], ids=["valu", "mfma"])
def test_conv_output_ownership_mixed(mfma):
    """Two convolutions writing the same rows (neither owns them in A x; each
    owns its columns in A^T y, shared with an identity block) and one that owns
    its rows: every apply against the explicit matrix."""
    _say("conv ownership", mfma)
    rng = np.random.default_rng(9)
    c1, c2, c3 = rng.standard_normal(33), rng.standard_normal(17), rng.standard_normal(9)
    n1, n2, n3 = 1500, 1516, 700
    m = n1 + 33 - 1 + (n3 + 9 - 1)
    n = n1 + n2 + n3
    op = (P.Operator(m, n).add_conv(0, 0, c1, n1, 0.5).add_conv(0, n1, c2, n2, -1.5)
          .add_identity(3, 10, 40, 2.0).add_conv(n1 + 32, n1 + n2, c3, n3, 1.0))
    from oracle.program import conv_matrix
    A = np.zeros((m, n))
    A[0:n1 + 32, 0:n1] += 0.5 * conv_matrix(c1, n1)
    A[0:n2 + 16, n1:n1 + n2] += -1.5 * conv_matrix(c2, n2)
    A[3:43, 10:50] += 2.0 * np.eye(40)
    A[n1 + 32:, n1 + n2:] += conv_matrix(c3, n3)
    s = P.Solver(op, m, [], P.Settings.make(precision=P.FP32, conv_mfma=mfma, normalize=0))
    x, y = rng.standard_normal(n), rng.standard_normal(m)
    u = 2.0 ** -24
    ax, aty = s.apply(x), s.apply(y, transpose=True)
    assert np.all(np.abs(ax - A @ x) <= 50 * u * (np.abs(A) @ np.abs(x)) + 1e-30)
    assert np.all(np.abs(aty - A.T @ y) <= 50 * u * (np.abs(A).T @ np.abs(y)) + 1e-30)


# ----------------------------------------------------------------- regularized least squares (CG)

def _regls_cases():
    return [("regls_dense_300x150", w.regls_instance("dense", 150, 31, m=300, lam=1e-2)),
            ("regls_conv_n700_k151", w.regls_instance("conv", 700, 32, k=151, sigma=70.0, lam=1e-2))]


REGLS_CASES = _regls_cases()


@pytest.mark.parametrize("prec,tol", [(P.FP64, 1e-10), (P.FP32, 1e-5)], ids=["fp64", "fp32"])
@pytest.mark.parametrize("idx", range(len(REGLS_CASES)))
def test_regls_matches_closed_form(idx, prec, tol):
    """CG through the library on (lam I + A^T A) x = A^T b stops at the paper's
    relative residual test, recomputed here in FP64 against the data as given;
    the iterate is within cond * tol of the closed form."""
    name, d = REGLS_CASES[idx]
    _say("regls", name, prec, tol)
    if d["kind"] == "dense":
        rs = P.RegLS(d["lam"], A=d["A"], precision=prec)
    else:
        rs = P.RegLS(d["lam"], taps=d["c"], n=d["x_hat"].shape[0], precision=prec)
    x, it = rs.solve(d["b"], tol=tol, max_iters=5000)
    ref = o.regls_solution(d)
    rhs = o.regls_rhs(d)
    res = np.linalg.norm(o.regls_apply_normal(d, x) - rhs) / np.linalg.norm(rhs)
    # the device's own test passed in its precision; FP64 recomputation adds
    # the rounding of the FP32 operator for the FP32 case
    assert res <= (1.01 * tol if prec == P.FP64 else 4 * tol), res
    lam = float(d["lam"])
    if d["kind"] == "dense":
        sv = np.linalg.svd(d["A"], compute_uv=False)
        cond = (lam + sv[0] ** 2) / (lam + sv[-1] ** 2)
    else:
        cond = (lam + 1.0) / lam     # unit-sum kernel: ||C|| <= 1
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert err <= 2 * cond * res + (1e-13 if prec == P.FP64 else 1e-6), (err, cond, res)
    assert 0 < it < 5000
    rs.close()
