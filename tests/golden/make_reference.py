#!/usr/bin/env python3
"""Write tests/golden/reference_objectives.json from the FP64 oracle only.

Entries (exact optima, each with its KKT certificate error):
  deconv_n1000_k101   Lawson-Hanson NNLS of eq. (6) on the seeded workload
  lasso_5000x10000    lasso (eq. 5): oracle HSDE iteration to 1e-6, then the
                      active-set polish accepted only with KKT error <= 1e-9
  lasso_batch64_2000x8000[i] for i in a sample of the 64 instances (same method)

Run from the repository root:  python tests/golden/make_reference.py
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


def main():
    out = {"_source": "written by tests/golden/make_reference.py from oracle/ (FP64) only"}
    t = time.time()
    cfg = w.workload("deconv_n1000_k101")
    d = w.make_deconv(cfg)
    ref = oracle.polish_deconv(d["c"], d["b"])
    assert ref["kkt_ok"], ref["kkt_err"]
    out[cfg["name"]] = {"objective": ref["obj"], "kkt_err": ref["kkt_err"], "support": ref["support"],
                        "method": "Lawson-Hanson NNLS"}
    print(cfg["name"], ref["obj"], f"{time.time() - t:.1f}s", flush=True)

    def lasso_ref(A, b, lam, label):
        t0 = time.time()
        prog = oracle.lasso_program(A, b, lam)
        res = oracle.scs_solve(prog, eps=1e-6, check_every=10)
        n = A.shape[1]
        pol = oracle.polish_lasso(A, b, lam, res.x[:n])
        assert pol["kkt_ok"], (label, pol["kkt_err"])
        print(label, pol["obj"], res.iters, f"{time.time() - t0:.1f}s", flush=True)
        return {"objective": pol["obj"], "kkt_err": pol["kkt_err"], "support": pol["support"],
                "scs_iters_1e-6": res.iters, "method": "HSDE to 1e-6 + active-set polish"}

    cfg = w.workload("lasso_5000x10000")
    d = w.make_lasso(cfg)
    out[cfg["name"]] = lasso_ref(d["A"], d["b"], float(d["lam"]), cfg["name"])

    cfg = w.workload("lasso_batch64_2000x8000")
    d = w.make_lasso_batch(cfg)
    out[cfg["name"]] = {str(i): lasso_ref(d["A"], d["b"][i], d["lam"][i], f"{cfg['name']}[{i}]")
                        for i in (0, 21, 42, 63)}
    with open(os.path.join(HERE, "reference_objectives.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
