"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
the host-side validation returns the documented error codes (no GPU calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgs.h")

P = pytest.importorskip("paper_1609_03488_amd")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = P.lib()
    names = _declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and nm agrees (extern "C", default visibility)
    syms = os.popen(f"nm -D --defined-only {P.library_path}").read()
    for n in names:
        assert re.search(rf"\bT {n}\b", syms), n


def test_binding_covers_every_declared_function():
    from paper_1609_03488_amd import _lib
    assert set(_declared_functions()) == set(_lib._SIGS)


def test_settings_defaults():
    s = P.Settings.make()
    assert s.eps == 1e-4 and s.alpha == 1.5 and s.precision == P.FP32
    assert s.cg_max_iters >= 1 and s.check_every >= 1 and s.use_graph == 1


def _ws(op, l, q, **kw):
    lib = P.lib()
    st = P.Settings.make(**kw)
    qa = np.asarray(q, dtype=np.int64)
    nb = C.c_size_t()
    rc = lib.cgs_workspace_bytes(op._h, l, qa.ctypes.data_as(C.POINTER(C.c_int64)), len(q),
                                 C.byref(st), 1, C.byref(nb))
    return rc, nb.value


def test_operator_validation_codes():
    with pytest.raises(P.CgsError) as e:
        P.Operator(0, 3)
    assert e.value.code == -2
    op = P.Operator(10, 4)
    with pytest.raises(P.CgsError) as e:
        op.add_identity(8, 0, 3)          # rows 8..10 exceed m
    assert e.value.code == -2
    with pytest.raises(P.CgsError) as e:
        op.add_conv(0, 0, [1.0, np.nan], 4)
    assert e.value.code == -1
    with pytest.raises(P.CgsError) as e:
        op.add_conv(0, 0, np.ones(8), 4)  # 11 rows > 10
    assert e.value.code == -2
    with pytest.raises(P.CgsError) as e:
        op.add_dense(0, 0, np.full((2, 2), np.inf))
    assert e.value.code == -1
    op.add_conv(0, 0, np.ones(7), 4)
    op.add_identity(0, 0, 4, -1.0)


def test_workspace_and_cone_validation():
    op = P.Operator(10, 4).add_conv(0, 0, np.ones(7), 4)
    rc, nb = _ws(op, 5, [5])
    assert rc == 0 and nb > 0
    assert _ws(op, 5, [4])[0] == -3                 # cones cover 9 of 10 rows
    assert _ws(op, 5, [0, 5])[0] == -3              # empty cone
    assert _ws(op, 5, [5], eps=0.0)[0] == -1
    assert _ws(op, 5, [5], alpha=2.0)[0] == -1
    assert _ws(op, 5, [5], precision=7)[0] == -1
    assert _ws(op, 5, [5], vec_tile=1024)[0] == 0
    assert _ws(op, 5, [5], vec_tile=512)[0] == -1    # tiles of 1024 or 2048 only
    # more batch instances need more memory
    rc1, nb1 = _ws(op, 10, [])
    assert rc1 == 0


def test_workspace_scales_with_precision_and_batch():
    lib = P.lib()
    op = P.Operator(1000, 400).add_dense(0, 0, np.ones((1000, 400)))
    q = np.array([1000], dtype=np.int64)
    out = {}
    for prec in (P.FP64, P.FP32):
        for batch in (1, 4):
            st = P.Settings.make(precision=prec)
            nb = C.c_size_t()
            assert lib.cgs_workspace_bytes(op._h, 0, q.ctypes.data_as(C.POINTER(C.c_int64)), 1,
                                           C.byref(st), batch, C.byref(nb)) == 0
            out[prec, batch] = nb.value
    assert out[P.FP64, 1] > out[P.FP32, 1]
    assert out[P.FP32, 4] > out[P.FP32, 1]
    # the shared dense block is stored once (plus its transpose), not per instance
    assert out[P.FP32, 4] - out[P.FP32, 1] < 2 * 1000 * 400 * 4


def test_canonical_forms_match_paper_dimensions():
    """Table III (deconvolution) and Table II (lasso) problem sizes."""
    for n0 in (100, 1000):
        pr = P.deconv_problem(np.ones(n0) / n0, np.zeros(2 * n0 - 1))
        assert (pr.op.n, pr.op.m) == (n0 + 1, 3 * n0)
        assert pr.l + sum(pr.q) == pr.op.m
    pr = P.lasso_problem(np.ones((60, 30)), np.zeros(60), 0.1)
    assert (pr.op.n, pr.op.m) == (61, 122)
    assert pr.op.kinds.count("dense") == 1


def test_request_bytes_and_server_precision_check():
    op = P.Operator(10, 4).add_conv(0, 0, np.ones(7), 4)
    nb = P.Server.request_bytes(op, 5, [5], P.FP32)
    assert nb >= 512
    with pytest.raises(P.CgsError):
        P.Server.request_bytes(op, 5, [5], P.BF16)


def _equil_cases():
    import workloads as w
    from paper_1609_03488_amd.problems import ConeProblem
    import oracle as o
    d = w.deconv_instance(300, 31, 4.0, 0.1, 1e-4, 3)
    yield P.deconv_problem(d["c"], d["b"]), o.deconv_program(d["c"], d["b"])
    d = w.lasso_instance(40, 70, 0.1, 1e-4, 4)
    yield P.lasso_problem(d["A"], d["b"], d["lam"]), o.lasso_program(d["A"], d["b"], d["lam"])
    d = w.conv_lasso_instance(90, 17, 3.0, 1e-4, 6)
    yield (P.conv_lasso_problem(d["c"], d["b"], d["lam"]),
           o.conv_lasso_program(d["c"], d["b"], d["lam"]))
    # two dense blocks in different row ranges, a row no block touches, cones
    rng = np.random.default_rng(5)
    A1, A2 = rng.standard_normal((6, 3)), 10.0 * rng.standard_normal((5, 2))
    op = P.Operator(12, 5).add_dense(0, 0, A1).add_dense(7, 3, A2, scale=0.5)
    A = np.zeros((12, 5))
    A[0:6, 0:3] = A1
    A[7:12, 3:5] = 0.5 * A2
    b, c = rng.standard_normal(12), rng.standard_normal(5)
    prog = o.dense_program(A, b, c, 7, [5])
    prog.blocks = [(0, 6, 0, 3), (7, 5, 3, 2)]      # the blocks the library sees
    yield ConeProblem(op, 7, [5], b, c, 5), prog


def test_library_equilibration_matches_oracle():
    """Host-side scaling of the library (block Frobenius norms) against the
    oracle's (squared-operator applies): same groups, D, E and data scales."""
    import oracle as o
    for pr, prog in _equil_cases():
        for level, passes in ((1, 0), (2, 20)):
            d, e, sig = pr.op.equilibrate(pr.l, pr.q, pr.b, pr.c, level=level)
            ref = o.equilibrate(prog, passes=passes)
            np.testing.assert_allclose(d, ref.D, rtol=1e-12)
            np.testing.assert_allclose(e, ref.E, rtol=1e-12)
            np.testing.assert_allclose(sig, (ref.sigma_b, ref.sigma_c), rtol=1e-12)
            if level == 1:
                assert np.all(d == 1.0) and np.all(e == 1.0)


def test_typed_dense_blocks():
    """cgs_op_add_dense_ex: unknown dtype or memory kind and non-finite entries
    are rejected; an FP32 host block is widened exactly, so the operator (its
    norms, hence its scaling) equals the FP64 copy of the same values."""
    lib = P.lib()
    rng = np.random.default_rng(3)
    A = rng.standard_normal((7, 5)).astype(np.float32)
    op = P.Operator(9, 6)
    assert lib.cgs_op_add_dense_ex(op._h, 0, 0, 2, 2, A.ctypes.data, 5, 7, P.MEM_HOST_COPY, 1.0) == -1
    assert lib.cgs_op_add_dense_ex(op._h, 0, 0, 2, 2, A.ctypes.data, 5, P.DTYPE_F32, 5, 1.0) == -1
    assert lib.cgs_op_add_dense_ex(op._h, 0, 0, 2, 2, None, 5, P.DTYPE_F32, P.MEM_HOST_COPY, 1.0) == -1
    assert lib.cgs_op_add_dense_ex(op._h, 0, 0, 2, 6, A.ctypes.data, 5, P.DTYPE_F32, P.MEM_HOST_COPY, 1.0) == -2
    bad = A.copy()
    bad[2, 3] = np.inf
    with pytest.raises(P.CgsError) as e:
        P.Operator(9, 6).add_dense(1, 0, bad)
    assert e.value.code == -1
    op64 = P.Operator(9, 6).add_dense(1, 0, A.astype(np.float64), scale=0.5)
    op32 = P.Operator(9, 6).add_dense(1, 0, A, scale=0.5)
    for level in (1, 2):
        d64, e64, _ = op64.equilibrate(9, [], level=level)
        d32, e32, _ = op32.equilibrate(9, [], level=level)
        assert np.array_equal(d64, d32) and np.array_equal(e64, e32)
