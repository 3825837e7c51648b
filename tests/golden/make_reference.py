#!/usr/bin/env python3
"""Write tests/golden/reference_objectives.json from the FP64 oracle only.

Entries (exact optima, each with its KKT certificate error):
  deconv_n1000_k101   Lawson-Hanson NNLS of eq. (6) on the seeded workload
  lasso_5000x10000    lasso (eq. 5): oracle HSDE iteration to 1e-6, then the
                      active-set polish accepted only with KKT error <= 1e-9
  lasso_batch64_2000x8000[i] for i in a sample of the 64 instances (same method)
  lasso_conv_3000_k1365   lasso with the convolution operator: oracle HSDE
                      iteration to 1e-4, then the polish on the explicit
                      convolution matrix (KKT error <= 1e-9); the 1e-4 point's
                      objective is stored beside the optimum

Run from the repository root:  python tests/golden/make_reference.py [name ...]
(names: recompute only those entries and keep the others).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as w  # noqa: E402


def main(only=None):
    path = os.path.join(HERE, "reference_objectives.json")
    out = {"_source": "written by tests/golden/make_reference.py from oracle/ (FP64) only"}
    if only and os.path.exists(path):
        out.update(json.load(open(path)))

    def want(name):
        return not only or name in only

    if want("deconv_n1000_k101"):
        t = time.time()
        cfg = w.workload("deconv_n1000_k101")
        d = w.make_deconv(cfg)
        ref = oracle.polish_deconv(d["c"], d["b"])
        assert ref["kkt_ok"], ref["kkt_err"]
        out[cfg["name"]] = {"objective": ref["obj"], "kkt_err": ref["kkt_err"], "support": ref["support"],
                            "method": "Lawson-Hanson NNLS"}
        print(cfg["name"], ref["obj"], f"{time.time() - t:.1f}s", flush=True)

    def lasso_ref(prog, A, b, lam, label, normalize=1):
        t0 = time.time()
        res = oracle.scs_solve(prog, eps=1e-6, check_every=10, normalize=normalize)
        n = A.shape[1]
        pol = oracle.polish_lasso(A, b, lam, res.x[:n])
        assert pol["kkt_ok"], (label, pol["kkt_err"])
        print(label, pol["obj"], res.iters, res.status, f"{time.time() - t0:.1f}s", flush=True)
        out = {"objective": pol["obj"], "kkt_err": pol["kkt_err"], "support": pol["support"],
               "scs_iters_1e-6": res.iters, "method": "HSDE to 1e-6 + active-set polish"}
        if normalize != 1:
            out["scs_normalize"] = normalize
        if res.status != "solved":
            out["scs_status"] = res.status
        return out

    if want("lasso_5000x10000"):
        cfg = w.workload("lasso_5000x10000")
        d = w.make_lasso(cfg)
        out[cfg["name"]] = lasso_ref(oracle.lasso_program(d["A"], d["b"], d["lam"]),
                                     d["A"], d["b"], float(d["lam"]), cfg["name"])

    if want("lasso_batch64_2000x8000"):
        cfg = w.workload("lasso_batch64_2000x8000")
        d = w.make_lasso_batch(cfg)
        out[cfg["name"]] = {str(i): lasso_ref(oracle.lasso_program(d["A"], d["b"][i], d["lam"][i]),
                                              d["A"], d["b"][i], d["lam"][i], f"{cfg['name']}[{i}]")
                            for i in (0, 21, 42, 63)}

    if want("lasso_conv_3000_k1365"):
        from oracle.program import conv_matrix
        cfg = w.workload("lasso_conv_3000_k1365")
        d = w.make_conv_lasso(cfg)
        C = conv_matrix(d["c"], cfg["n"])
        # block equilibration: the blur operator's flat group norms make it the
        # faster scaling here (the polish certifies the optimum either way)
        prog = oracle.conv_lasso_program(d["c"], d["b"], d["lam"])
        # the HSDE iteration converges slowly on this blur operator (it does not
        # reach 1e-6 in 1e5 iterations), so the polish starts from the eps = 1e-4
        # point, the workload's own tolerance (data scaling only); the KKT check
        # decides whether the polished point is the optimum
        t0 = time.time()
        res = oracle.scs_solve(prog, eps=1e-4, check_every=10, normalize=1)
        assert res.status == "solved", res.status
        n = cfg["n"]
        pol = oracle.polish_lasso(C, d["b"], float(d["lam"]), res.x[:n])
        assert pol["kkt_ok"], pol["kkt_err"]
        out[cfg["name"]] = {
            "objective": pol["obj"], "kkt_err": pol["kkt_err"], "support": pol["support"],
            "method": "HSDE to 1e-4 + active-set polish",
            "scs_1e-4": {"objective": oracle.lasso_objective(C, d["b"], float(d["lam"]), res.x[:n]),
                         "iters": res.iters, "normalize": 1}}
        print(cfg["name"], out[cfg["name"]], f"{time.time() - t0:.1f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
