"""GPU checks at the benchmark sizes, in the launch configuration bench.py uses.

Reference values come from tests/golden/reference_objectives.json (written by
tests/golden/make_reference.py from the FP64 oracle only): exact optima where
the oracle can certify one, and the oracle's run of the same method to the
same tolerance for the deconvolutions (at n = 2^20 the oracle's banded
factorisation takes about 17 GB and its 620 iterations some 20 minutes).  The
returned points are also checked through properties that hold at any size:
the KKT residuals recomputed in FP64 on the host, and for deconvolution the
objective bound ||noise|| (x_true is feasible).
"""
import json
import os

import numpy as np
import pytest

import oracle as o
import workloads as w

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1609_03488_amd")
REF = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_objectives.json")))


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("engine", [1, 2, "autotune"], ids=["mfma", "fft", "autotune"])
def test_deconv_n1M_k1025_fp32(engine):
    """The benchmark solve on each FP32 convolution engine (and the one the
    autotuner picks, as bench.py runs it)."""
    import torch
    cfg = w.workload("deconv_n1M_k1025")
    _say(cfg["name"], engine)
    d = w.make_deconv(cfg)
    pr = P.deconv_problem(d["c"], d["b"])
    st = P.Settings.make(precision=P.FP32, eps=cfg["eps"], check_every=10,
                         conv_mfma=1 if engine == "autotune" else engine)
    s = P.Solver(pr.op, pr.l, pr.q, st, stream=torch.cuda.Stream())
    s.set_data(0, pr.b, pr.c)
    if engine == "autotune":
        s.autotune(reps=5)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    prog = o.deconv_program(d["c"], d["b"])
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05e-4, (rp, rd, gap)
    f = o.deconv_objective(d["c"], d["b"], x[:cfg["n"]])
    noise = np.linalg.norm(d["b"] - np.convolve(d["c"], d["x_true"]))
    assert f <= noise * (1 + 1e-4), (f, noise)
    # the oracle's run of the same method to the same eps and scaling
    same = REF[cfg["name"] + "_scs"]
    assert (same["eps"], same["normalize"]) == (cfg["eps"], 1)
    assert abs(f - same["objective"]) / same["objective"] <= 1e-4, (f, same["objective"])
    # dual side: y in K (cone membership of the returned dual point)
    assert o.in_cone(y, prog.l, prog.q, 1e-6 * (1 + np.abs(y).max()))


def test_deconv_n1000_k101_fp64_at_its_tolerance():
    """The n = 1000 deconvolution at its own tolerance 1e-6 in FP64, with block
    equilibration (normalize = 2: data scaling alone needs tens of thousands of
    iterations here).  Residuals of the returned point recomputed in FP64 are
    within 1e-6; the natural objective is within 1e-4 of the oracle's run of
    the same method to the same tolerance and scaling, and within 1e-4 of the
    exact optimum (Lawson-Hanson), both stored by make_reference.py."""
    cfg = w.workload("deconv_n1000_k101")
    _say(cfg["name"], "eps", cfg["eps"])
    d = w.make_deconv(cfg)
    pr = P.deconv_problem(d["c"], d["b"])
    st = P.Settings.make(precision=P.FP64, eps=cfg["eps"], check_every=10, normalize=2)
    s = P.Solver(pr.op, pr.l, pr.q, st)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    prog = o.deconv_program(d["c"], d["b"])
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * cfg["eps"], (rp, rd, gap)
    f = o.deconv_objective(d["c"], d["b"], x[:cfg["n"]])
    same = REF["deconv_n1000_k101_scs"]
    assert (same["eps"], same["normalize"]) == (cfg["eps"], 2)
    assert abs(f - same["objective"]) / same["objective"] <= 1e-4, (f, same["objective"])
    exact = REF[cfg["name"]]["objective"]
    assert exact * (1 - 1e-12) <= f and (f - exact) / exact <= 1e-4, (f, exact)


@pytest.mark.parametrize("prec", [P.FP32, P.FP64], ids=["fp32", "fp64"])
def test_lasso_5000x10000_against_exact(prec):
    """The dense lasso at the settings bench.py runs (block equilibration,
    normalize = 2; stop at the workload's stop_eps = 1e-5), in FP32 and FP64:
    residuals of the returned point recomputed in FP64 within the stop, and the
    objective within 1e-4 of the KKT-certified optimum."""
    import torch
    cfg = w.workload("lasso_5000x10000")
    _say(cfg["name"], prec)
    d = w.make_lasso(cfg)
    pr = P.lasso_problem(d["A"], d["b"], d["lam"])
    st = P.Settings.make(precision=prec, eps=cfg["stop_eps"], check_every=10, normalize=2)
    s = P.Solver(pr.op, pr.l, pr.q, st, stream=torch.cuda.Stream())
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    prog = o.lasso_program(d["A"], d["b"], d["lam"])
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * cfg["stop_eps"], (rp, rd, gap)
    f = o.lasso_objective(d["A"], d["b"], float(d["lam"]), x[:cfg["n"]])
    exact = REF[cfg["name"]]["objective"]
    assert abs(f - exact) / exact <= 1e-4, (f, exact)


def test_lasso_batch64_bf16_against_exact():
    """The batch at the settings bench.py runs (BF16 products, block
    equilibration, stop_eps = 1e-5): every one of the 64 instances is solved,
    certified by the residual test on the FP32 operator, has FP64 residuals
    within the stop and an objective within 1e-4 of its KKT-certified optimum."""
    import torch
    cfg = w.workload("lasso_batch64_2000x8000")
    _say(cfg["name"])
    d = w.make_lasso_batch(cfg)
    B = cfg["batch"]
    prs = [P.lasso_problem(d["A"], d["b"][i], d["lam"][i]) for i in range(B)]
    st = P.Settings.make(precision=P.BF16, eps=cfg["stop_eps"], check_every=10, normalize=2)
    s = P.Solver(prs[0].op, prs[0].l, prs[0].q, st, batch=B, stream=torch.cuda.Stream())
    for i, pr in enumerate(prs):
        s.set_data(i, pr.b, pr.c)
    infos = s.solve()
    assert all(inf["status"] == P.SOLVED for inf in infos), [inf["status"] for inf in infos]
    assert all(inf["cert_precision"] == P.FP32 for inf in infos)
    refs = REF[cfg["name"]]
    assert len(refs) == B
    for i in range(B):
        x, y, sl = s.solution(i)
        prog = o.lasso_program(d["A"], d["b"][i], d["lam"][i])
        rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
        assert max(rp, rd, gap) <= 1.05 * cfg["stop_eps"], (i, rp, rd, gap)
        f = o.lasso_objective(d["A"], d["b"][i], d["lam"][i], x[:cfg["n"]])
        ref = refs[str(i)]["objective"]
        assert abs(f - ref) / ref <= 1e-4, (i, f, ref)


@pytest.mark.parametrize("name", ["regls_dense_6000x3000", "regls_conv_3000_k1365"])
def test_regls_paper_sizes_against_closed_form(name):
    """Table I sizes (Section V-A): CG in FP64 to the paper's stop test
    ||(lam I + A^T A) x - A^T b|| <= 1e-8 ||A^T b||, recomputed here in FP64;
    the iterate is within cond * 1e-8 of the closed form."""
    cfg = w.workload(name)
    _say(name)
    d = w.make_regls(cfg)
    if d["kind"] == "dense":
        rs = P.RegLS(d["lam"], A=d["A"], precision=P.FP64)
    else:
        rs = P.RegLS(d["lam"], taps=d["c"], n=cfg["n"], precision=P.FP64)
    x, it = rs.solve(d["b"], tol=cfg["tol"])
    rhs = o.regls_rhs(d)
    res = np.linalg.norm(o.regls_apply_normal(d, x) - rhs) / np.linalg.norm(rhs)
    assert res <= 1.01 * cfg["tol"], res
    ref = o.regls_solution(d)
    lam = float(d["lam"])
    if d["kind"] == "dense":
        sv = np.linalg.svd(d["A"], compute_uv=False)
        cond = (lam + sv[0] ** 2) / (lam + sv[-1] ** 2)
    else:
        cond = (lam + 1.0) / lam
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert err <= 2 * cond * res + 1e-13, (err, cond, res)
    assert 0 < it < 1000
    rs.close()


def test_lasso_conv_3000_fp32_against_exact():
    """Lasso with the Table I convolution (Table II, convolution column) at the
    workload's settings (FP32, eps = 1e-4, data scaling): solved, FP64 residuals
    of the returned point within eps, and its objective no farther from the
    KKT-certified optimum than twice the oracle's own eps = 1e-4 point (both
    stored by tests/golden/make_reference.py) plus 1e-4 relative."""
    cfg = w.workload("lasso_conv_3000_k1365")
    _say(cfg["name"])
    d = w.make_conv_lasso(cfg)
    pr = P.conv_lasso_problem(d["c"], d["b"], d["lam"])
    st = P.Settings.make(precision=P.FP32, eps=cfg["eps"], check_every=10, normalize=1)
    s = P.Solver(pr.op, pr.l, pr.q, st)
    s.set_data(0, pr.b, pr.c)
    info = s.solve()[0]
    assert info["status"] == P.SOLVED, info
    x, y, sl = s.solution(0)
    prog = o.conv_lasso_program(d["c"], d["b"], d["lam"])
    rp, rd, gap, _, _ = o.scs.residuals(prog, x, y, 1.0, sl)
    assert max(rp, rd, gap) <= 1.05 * cfg["eps"], (rp, rd, gap)
    refs = REF[cfg["name"]]
    opt, fr = refs["objective"], refs["scs_1e-4"]["objective"]
    xs = x[:cfg["n"]]
    r = np.convolve(d["c"], xs) - d["b"]
    f = float(0.5 * (r @ r) + d["lam"] * np.sum(np.abs(xs)))
    assert f >= opt * (1 - 1e-9)
    assert f - opt <= 2 * (fr - opt) + 1e-4 * opt, (f, fr, opt)
