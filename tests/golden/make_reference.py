#!/usr/bin/env python3
"""Write tests/golden/reference_objectives.json from the FP64 oracle only.

Entries (exact optima, each with its KKT certificate error):
  deconv_n1000_k101   Lawson-Hanson NNLS of eq. (6) on the seeded workload
  lasso_5000x10000    lasso (eq. 5): oracle HSDE iteration to 1e-6, then the
                      active-set polish accepted only with KKT error <= 1e-9
  lasso_batch64_2000x8000[i] for every one of the 64 instances (same method)
  lasso_conv_3000_k1365   lasso with the convolution operator: oracle HSDE
                      iteration to 1e-4, then the polish on the explicit
                      convolution matrix (KKT error <= 1e-9); the 1e-4 point's
                      objective is stored beside the optimum
  deconv_n1000_k101_scs   the same method (HSDE ADMM, exact subspace solves) on
                      the n = 1000 deconvolution to its own tolerance 1e-6 with
                      block equilibration (normalize = 2): objective, iterations
  deconv_n1M_k1025_scs    the same method on the n = 2^20 deconvolution to 1e-4
                      with data scaling (normalize = 1): objective, iterations
                      (banded factor of 2I + C^T C, about 17 GB and tens of
                      minutes on 8 cores)
  serve_deconv_2000req_sample   the same method (eps 1e-4, data scaling) on a
                      seeded 5 % subsample of the serving trace spread over its
                      size range (serve_sample_ids): objective, iterations

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


SERVE_SAMPLE = 100   # requests of the serving trace with a stored oracle result (5 %)


def serve_sample_ids(trace, count=SERVE_SAMPLE):
    """A seeded subsample spread over the trace's size range: the requests
    sorted by n, every len/count-th of them."""
    order = sorted(range(len(trace)), key=lambda i: (trace[i].n, trace[i].k, i))
    step = len(order) / count
    return sorted(order[int(j * step + step / 2)] for j in range(count))


def _serve_one(args):
    rid, eps = args
    cfg = w.workload("serve_deconv_2000req")
    req = w.serving_trace(cfg["count"], cfg["rate"], cfg["seed"])[rid]
    d = w.serving_request_data(req, cfg["density"], cfg["noise_var"])
    t0 = time.time()
    res = oracle.scs_solve(oracle.deconv_program(d["c"], d["b"]), eps=eps, check_every=10, normalize=1)
    return rid, {"n": req.n, "k": req.k, "status": res.status, "iters": res.iters,
                 "objective": oracle.deconv_objective(d["c"], d["b"], res.x[:req.n]),
                 "seconds": time.time() - t0}


def serve_sample():
    """The oracle (same method, eps = 1e-4, data scaling) on the serving
    trace's seeded subsample, in parallel worker processes."""
    import multiprocessing as mp
    cfg = w.workload("serve_deconv_2000req")
    trace = w.serving_trace(cfg["count"], cfg["rate"], cfg["seed"])
    ids = serve_sample_ids(trace)
    # largest first, so that the long solves do not end up last
    ids_by_cost = sorted(ids, key=lambda i: -trace[i].n * trace[i].k)
    t0 = time.time()
    with mp.get_context("spawn").Pool(int(os.environ.get("REF_WORKERS", "8"))) as pool:
        got = dict(pool.imap_unordered(_serve_one, [(i, cfg["eps"]) for i in ids_by_cost]))
    print("serve sample", len(got), f"{time.time() - t0:.1f}s", flush=True)
    return {"eps": cfg["eps"], "normalize": 1, "check_every": 10,
            "method": "HSDE ADMM with exact subspace solves (oracle.scs_solve)",
            "requests": {str(i): got[i] for i in ids}}


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

    def lasso_ref(prog, A, b, lam, label, normalize=1, fac=None):
        t0 = time.time()
        res = oracle.scs_solve(prog, eps=1e-6, check_every=10, normalize=normalize, fac=fac)
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
        # every instance; data scaling (normalize = 1) leaves A, and so the
        # factorisation of I + A^T A, the same for all of them
        prog0 = oracle.lasso_program(d["A"], d["b"][0], d["lam"][0])
        fac = oracle.prepare(prog0, 1)[0].factor()
        out[cfg["name"]] = {str(i): lasso_ref(oracle.lasso_program(d["A"], d["b"][i], d["lam"][i]),
                                              d["A"], d["b"][i], d["lam"][i], f"{cfg['name']}[{i}]",
                                              fac=fac)
                            for i in range(cfg["batch"])}

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
    def deconv_scs(name, eps, normalize):
        t0 = time.time()
        cfg = w.workload(name)
        d = w.make_deconv(cfg)
        prog = oracle.deconv_program(d["c"], d["b"])
        res = oracle.scs_solve(prog, eps=eps, check_every=10, normalize=normalize)
        assert res.status == "solved", res.status
        n = cfg["n"]
        rec = {"objective": oracle.deconv_objective(d["c"], d["b"], res.x[:n]),
               "iters": res.iters, "eps": eps, "normalize": normalize, "check_every": 10,
               "res_pri": res.res_pri, "res_dual": res.res_dual, "gap": res.gap,
               "method": "HSDE ADMM with exact subspace solves (oracle.scs_solve)"}
        print(name, rec, f"{time.time() - t0:.1f}s", flush=True)
        return rec

    if want("deconv_n1000_k101_scs"):
        out["deconv_n1000_k101_scs"] = deconv_scs("deconv_n1000_k101", 1e-6, 2)

    if want("deconv_n1M_k1025_scs"):
        out["deconv_n1M_k1025_scs"] = deconv_scs("deconv_n1M_k1025", 1e-4, 1)

    if want("serve_deconv_2000req_sample"):
        out["serve_deconv_2000req_sample"] = serve_sample()

    if only and os.path.exists(path):
        # another run may have written entries meanwhile: keep them
        cur = json.load(open(path))
        cur.update({k: v for k, v in out.items() if want(k)})
        out = cur
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
